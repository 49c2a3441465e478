// Small dense FP64 linear algebra kernels: one workgroup per matrix.
#include "linalg.h"

#include <cmath>

namespace ipeps {

// ----------------------------------------------------------------- Jacobi SVD
// Circle-method pairing: with ne (even) columns, round r pairs r with ne-1
// and (r+k, r-k) mod (ne-1) for k = 1..ne/2-1; every pair meets once per
// sweep and the pairs of one round are disjoint.
__device__ inline void circle_pair(int r, int k, int ne, int* p, int* q) {
    if (k == 0) {
        *p = r;
        *q = ne - 1;
    } else {
        // 0 <= r < m and 1 <= k < m: one conditional correction each
        const int m = ne - 1;
        *p = r + k >= m ? r + k - m : r + k;
        *q = r - k < 0 ? r - k + m : r - k;
    }
    if (*p > *q) {
        int t = *p;
        *p = *q;
        *q = t;
    }
}

// Ac: m x n column-major working copy of A, Vc: n x n column-major (or NULL),
// nrm: n squared column norms (recomputed exactly at the start of each sweep,
// updated in closed form after each rotation, so a pair needs only one inner
// product).  Each pair of a round is handled by a group of 16 lanes (4 groups
// per wave) holding its two columns in registers (EPL elements per lane);
// the inner product is summed with DPP moves inside the group.
// A sweep asks for another only if one of its rotations turned by more than
// kSweepAngle: rotations of angle <= theta leave inner products of order
// theta^2 |a_p||a_q|, far below the convergence test, so the sweep after
// would rotate nothing that matters (it only confirmed convergence).
constexpr double kSweepAngle = 1e-9;
// Tail sweeps: once a sweep rotates no pair that involves a column above
// kHeadRel |A|_F at all (every such pair passed the relative test), the
// sweeps that follow pair only the columns below it (the noise-level tail of
// a Rayleigh-Ritz matrix, whose clustered values converge linearly while the
// head converges quadratically).  Rotating two tail columns turns their inner
// products with a head column into combinations of two that already passed
// the test, the same drift a full last sweep leaves behind its own rotations.
constexpr double kHeadRel = 1e-6;

// One sweep over the columns list[0..nc) (list == nullptr: columns 0..nc):
// exact squared norms first, then the ne - 1 rounds of the circle method.
// Returns whether a rotation turned by more than kSweepAngle; *head is set
// when any pair with a column above head2 was rotated.
template <int EPL>
__device__ __forceinline__ bool jacobi_one_sweep(int m, int n, int nc, const short* list, double* Ac,
                                                 double* Vc, double* nrm, int* flag, int* head,
                                                 double tol2, double small2, double head2) {
    const int g16 = threadIdx.x & 15, group = threadIdx.x >> 4, ngroups = blockDim.x >> 4;
    const int ne = nc + (nc & 1);
    const int npair = ne / 2;
    for (int jj = group; jj < nc; jj += ngroups) {
        const int j = list ? list[jj] : jj;
        const double* aj = Ac + (long)j * m;
        double sq = 0.0;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int i = g16 + 16 * e;
            const double v = (i < m) ? aj[i] : 0.0;
            sq += v * v;
        }
        sq = group16_sum(sq);
        if (g16 == 0) nrm[j] = sq;
    }
    if (threadIdx.x == 0) {
        *flag = 0;
        *head = 0;
    }
    __syncthreads();
    for (int r = 0; r < ne - 1; ++r) {
        for (int kk = group; kk < npair; kk += ngroups) {
            int p, q;
            circle_pair(r, kk, ne, &p, &q);
            if (q >= nc) continue;
            if (list) {
                p = list[p];
                q = list[q];
            }
            double* ap = Ac + (long)p * m;
            double* aq = Ac + (long)q * m;
            double x[EPL], y[EPL];
            double ga = 0.0;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int i = g16 + 16 * e;
                x[e] = (i < m) ? ap[i] : 0.0;
                y[e] = (i < m) ? aq[i] : 0.0;
                ga += x[e] * y[e];
            }
            ga = group16_sum(ga);
            const double al = nrm[p], be = nrm[q];
            if (al <= small2 || be <= small2) continue;
            // converged pair: relative test, or an inner product below
            // skip_rel^2 |A|_F^2, which moves no singular value by more
            // than ~skip_rel |A|_F
            if (ga * ga <= tol2 * al * be || fabs(ga) <= small2) continue;
            const double zeta = 0.5 * (be - al) * fast_rcp(ga);
            const double az = fabs(zeta);
            const double den = (az > 1e150) ? 2.0 * az : az + (1.0 + az * az) * fast_rsq(1.0 + az * az);
            const double t = copysign(fast_rcp(den), zeta);
            const double c = fast_rsq(1.0 + t * t), s = c * t;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int i = g16 + 16 * e;
                if (i < m) {
                    ap[i] = c * x[e] - s * y[e];
                    aq[i] = s * x[e] + c * y[e];
                }
            }
            if (Vc) {
                double* vp = Vc + (long)p * n;
                double* vq = Vc + (long)q * n;
#pragma unroll
                for (int e = 0; e < EPL; ++e) {
                    const int i = g16 + 16 * e;
                    if (i < n) {
                        const double xv = vp[i], yv = vq[i];
                        vp[i] = c * xv - s * yv;
                        vq[i] = s * xv + c * yv;
                    }
                }
            }
            if (g16 == 0) {
                nrm[p] = al - t * ga;
                nrm[q] = be + t * ga;
                if (fabs(t) > kSweepAngle) *flag = 1;
                if (fmax(al, be) > head2) *head = 1;
            }
        }
        __syncthreads();
    }
    const bool any = *flag != 0;
    __syncthreads();
    return any;
}

template <int EPL>
__device__ __forceinline__ void jacobi_sweeps(int m, int n, double* Ac, double* Vc, double* nrm, int* flag,
                                              double* red, double skip_rel) {
    __shared__ int s_head, s_ntail;
    __shared__ short s_tail[256];
    const double tol = 4.0 * m * 1.11e-16, tol2 = tol * tol;
    // columns below skip_rel |A|_F are left alone: a rotation against a large
    // column re-pollutes them at their own size; pairs whose inner product is
    // below skip_rel^2 |A|_F^2 count as converged
    double fro = 0.0;
    for (long e = threadIdx.x; e < (long)m * n; e += blockDim.x) fro += Ac[e] * Ac[e];
    fro = block_sum(fro, red);
    const double small2 = skip_rel * skip_rel * fro;
    const double head2 = kHeadRel * kHeadRel * fro;
    int sweep = 0;
    for (; sweep < 40; ++sweep) {
        if (!jacobi_one_sweep<EPL>(m, n, n, nullptr, Ac, Vc, nrm, flag, &s_head, tol2, small2, head2))
            return;
        const int head = s_head;
        __syncthreads();
        if (!head) break;
    }
    if (++sweep >= 40) return;
    // the head has converged: the remaining sweeps pair the tail only
    if (threadIdx.x == 0) {
        int c = 0;
        for (int j = 0; j < n; ++j)
            if (nrm[j] <= head2) s_tail[c++] = (short)j;
        s_ntail = c;
    }
    __syncthreads();
    const int ntail = s_ntail;
    if (ntail < 2) return;
    for (; sweep < 40; ++sweep)
        if (!jacobi_one_sweep<EPL>(m, n, ntail, s_tail, Ac, Vc, nrm, flag, &s_head, tol2, small2, head2))
            return;
}

// Column norms, ranks (descending, ties by index) and sorted outputs.
__device__ void jacobi_finish(int m, int n, const double* Ac, const double* Vc, double* sig_s,
                              double* sigma, double* U, double* V) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double s = 0;
        for (int i = 0; i < m; ++i) s += Ac[(long)j * m + i] * Ac[(long)j * m + i];
        sig_s[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double sj = sig_s[j];
        int rank = 0;
        for (int l = 0; l < n; ++l) {
            const double sl = sig_s[l];
            rank += (sl > sj) || (sl == sj && l < j);
        }
        sigma[rank] = sj;
        if (U) {
            const double inv = sj > 0 ? 1.0 / sj : 0.0;
            for (int i = 0; i < m; ++i) U[(long)i * n + rank] = Ac[(long)j * m + i] * inv;
        }
        if (V)
            for (int i = 0; i < n; ++i) V[(long)i * n + rank] = Vc[(long)j * n + i];
    }
}

// Threads per workgroup: 1024 while the two register columns fit the
// 128-VGPR budget of a 16-wave group, 512 for longer columns.
template <int EPL>
constexpr int jacobi_threads() { return EPL <= 6 ? 1024 : 512; }

template <bool IN_LDS, int EPL>
__global__ __launch_bounds__(jacobi_threads<EPL>()) void k_jacobi_svd(int m, int n, const double* __restrict__ A,
                                                     long lda, long strideA, double* sigma,
                                                     double* U, double* V, double* work,
                                                     double skip_rel, JobMap jm) {
    extern __shared__ double smem[];
    __shared__ int flag;
    __shared__ double red[16];
    const int b = jlocal(jm, blockIdx.x);
    A = jptr(A, jm, blockIdx.x);
    sigma = jptr(sigma, jm, blockIdx.x);
    U = jptr(U, jm, blockIdx.x);
    V = jptr(V, jm, blockIdx.x);
    work = jptr(work, jm, blockIdx.x);
    const bool wantV = (V != nullptr);
    const long nv = wantV ? (long)n * n : 0;
    double *Ac, *Vc, *sig_s, *nrm;
    if (IN_LDS) {
        Ac = smem;
    } else {
        Ac = work + (long)b * ((long)m * n + nv + 2 * n);
    }
    Vc = Ac + (long)m * n;
    sig_s = Vc + nv;
    nrm = sig_s + n;
    const double* Ab = A + (long)b * strideA;
    for (long e = threadIdx.x; e < (long)m * n; e += blockDim.x) {
        const int j = (int)(e / m), i = (int)(e % m);
        Ac[e] = Ab[(long)i * lda + j];
    }
    for (long e = threadIdx.x; e < nv; e += blockDim.x) Vc[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
    __syncthreads();
    jacobi_sweeps<EPL>(m, n, Ac, wantV ? Vc : nullptr, nrm, &flag, red, skip_rel);
    __syncthreads();
    jacobi_finish(m, n, Ac, Vc, sig_s, sigma + (long)b * n, U ? U + (long)b * m * n : nullptr,
                  V ? V + (long)b * n * n : nullptr);
}

static size_t jacobi_lds_bytes(int m, int n, bool wantV) {
    return ((size_t)m * n + (wantV ? (size_t)n * n : 0) + 2 * (size_t)n) * sizeof(double);
}
static const size_t kMaxLds = 160 * 1024 - 1024;

size_t jacobi_svd_real_work(int batch, int m, int n) {
    if (jacobi_lds_bytes(m, n, true) <= kMaxLds) return 0;
    return (size_t)batch * ((size_t)m * n + (size_t)n * n + 2 * (size_t)n);
}

template <int EPL>
static void launch_jacobi(hipStream_t s, int batch, int m, int n, const double* A, long lda,
                          long strideA, double* sigma, double* U, double* V, double* work,
                          double skip_rel, JobMap jm) {
    const int blocks = batch * (jm.delta ? jm.njobs : 1);
    if (jm.delta) jm.per_job = batch;
    const size_t lds = jacobi_lds_bytes(m, n, V != nullptr);
    if (lds <= kMaxLds) {
        static bool attr_set = false;
        if (!attr_set) {
            HIP_CHECK(hipFuncSetAttribute((const void*)k_jacobi_svd<true, EPL>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)kMaxLds));
            attr_set = true;
        }
        hipLaunchKernelGGL((k_jacobi_svd<true, EPL>), dim3(blocks), dim3(jacobi_threads<EPL>()), lds, s, m, n, A, lda,
                           strideA, sigma, U, V, work, skip_rel, jm);
    } else {
        IPEPS_REQUIRE(work != nullptr, IPEPS_EINVAL, "jacobi_svd_real: work buffer needed");
        hipLaunchKernelGGL((k_jacobi_svd<false, EPL>), dim3(blocks), dim3(jacobi_threads<EPL>()), 0, s, m, n, A, lda,
                           strideA, sigma, U, V, work, skip_rel, jm);
    }
    HIP_CHECK(hipGetLastError());
}

void jacobi_svd_real(hipStream_t s, int batch, int m, int n, const double* A, long lda,
                     long strideA, double* sigma, double* U, double* V, double* work,
                     double skip_rel, JobMap jm) {
    if (batch <= 0 || n <= 0) return;
    IPEPS_REQUIRE(m >= n && m <= 256, IPEPS_EINVAL, "jacobi_svd_real: need n <= m <= 256");
    if (m <= 64)
        launch_jacobi<4>(s, batch, m, n, A, lda, strideA, sigma, U, V, work, skip_rel, jm);
    else if (m <= 96)
        launch_jacobi<6>(s, batch, m, n, A, lda, strideA, sigma, U, V, work, skip_rel, jm);
    else if (m <= 128)
        launch_jacobi<8>(s, batch, m, n, A, lda, strideA, sigma, U, V, work, skip_rel, jm);
    else if (m <= 176)
        launch_jacobi<11>(s, batch, m, n, A, lda, strideA, sigma, U, V, work, skip_rel, jm);
    else
        launch_jacobi<16>(s, batch, m, n, A, lda, strideA, sigma, U, V, work, skip_rel, jm);
}

// ----------------------------------------------------------------- Cholesky
// G = R^T R (R upper) with dropping, and X = R^{-1} built alongside, in
// place; one workgroup of 4 waves per matrix, blocked by NB = 16 columns.
// Per block J (three barriers):
//  (a) wave 0 factors the 16 x 16 diagonal block in registers (lane c holds
//      column c; rows are broadcast with readlane) and inverts it the same way
//      (lane i builds row i of X_JJ), writing X_JJ over R_JJ;
//  (b) the panel R[J, rest] = X_JJ^T G[J, rest] (independent dot products) and
//      T = X[:J, :J] R[:J, J] (4 x 4 register tiles);
//  (c) the trailing update G[rest, rest] -= R[J, rest]^T R[J, rest] (4 x 4
//      tiles) and X[:J, J] = -T X_JJ.
// A dropped pivot (Schur diagonal <= tol) zeroes its row of R and its row and
// column of X, so the matching column of Y X is zero.  R lives in LDS for
// k <= 128, else in the output buffer (L2-resident).
constexpr int kNb = 16;

__device__ inline double readlane_d(double v, int lane) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)x, lane);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <bool IN_LDS>
__global__ __launch_bounds__(256) void k_chol_inverse(int k, const double* __restrict__ G,
                                                      double* __restrict__ Rinv, double tol,
                                                      int* __restrict__ dead, double near_identity,
                                                      JobMap jm, int nbatch) {
    extern __shared__ double smem[];
    __shared__ int dead_s[256];
    __shared__ double dsc[256];  // 1/sqrt(G_ii): G is factored scaled to unit diagonal
    __shared__ double red[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int b = jlocal(jm, blockIdx.x);
    G = jptr(G, jm, blockIdx.x);
    Rinv = jptr(Rinv, jm, blockIdx.x);
    dead = jptr(dead, jm, blockIdx.x);
    const double* Gb = G + (long)b * k * k;
    double* out = Rinv + (long)b * k * k;
    double* R = IN_LDS ? smem : out;
    double* Tb = IN_LDS ? smem + (long)k * k : smem;  // k x NB
    for (int i = tid; i < k; i += 256) {
        const double gii = Gb[(long)i * k + i];
        dsc[i] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
    }
    __syncthreads();
    double off_max = 0.0;  // largest |G'_ij| off the diagonal; 1 if a diagonal is zero
    for (int e = tid; e < k * k; e += 256) {
        const int i = e / k, c = e - (e / k) * k;
        const double v = Gb[e] * dsc[i] * dsc[c];
        R[e] = v;
        if (i != c) off_max = fmax(off_max, fabs(v));
        else if (!(dsc[i] > 0.0)) off_max = 1.0;
    }
    if (near_identity > 0.0) {
        off_max = block_max(off_max, red);
        if (off_max <= near_identity) {  // R' = I: R^{-1} = D^{-1}, nothing dropped
            for (int e = tid; e < k * k; e += 256) {
                const int i = e / k, c = e - (e / k) * k;
                out[e] = (i == c) ? dsc[i] : 0.0;
            }
            if (dead) {
                for (int j = tid; j < k; j += 256) dead[(long)b * k + j] = 0;
                if (tid == 0) dead[(long)nbatch * k + b] = 0;
            }
            return;
        }
    }
    __syncthreads();

    for (int J0 = 0; J0 < k; J0 += kNb) {
        const int jb = min(kNb, k - J0), J1 = J0 + jb;
        // (a) diagonal block: factor, then invert, in the registers of wave 0
        if (tid < 64) {
            const int c = lane;
            double col[kNb];
#pragma unroll
            for (int r = 0; r < kNb; ++r)
                col[r] = (c < jb && r <= c) ? R[(long)(J0 + r) * k + J0 + c] : 0.0;
            unsigned int deadmask = 0;
            double ipc[kNb];  // 1 / R[j][j] (0 when dropped), the same in every lane
#pragma unroll
            for (int j = 0; j < kNb; ++j) {
                ipc[j] = 0.0;
                if (j < jb) {
                    const double d = readlane_d(col[j], j);
                    const bool dj = !(d > tol);
                    const double piv = dj ? 0.0 : sqrt(d);
                    const double ip = dj ? 0.0 : 1.0 / piv;
                    ipc[j] = ip;
                    if (c == j) col[j] = piv;
                    else if (c > j) col[j] *= ip;
                    deadmask |= dj ? (1u << j) : 0u;
#pragma unroll
                    for (int a = j + 1; a < kNb; ++a) {
                        const double rja = readlane_d(col[j], a);
                        if (c >= a) col[a] -= rja * col[j];
                    }
                }
            }
            // row i = lane of X_JJ: X[i][c] = (delta_ic - sum_{l<c} X[i][l] R[l][c]) / R[c][c]
            double x[kNb];
#pragma unroll
            for (int cc = 0; cc < kNb; ++cc) {
                double s0 = (lane == cc) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
                for (int l = 0; l < cc; ++l) {
                    const double rlc = readlane_d(col[l], cc);
                    if (l & 1) s1 -= x[l] * rlc;
                    else s0 -= x[l] * rlc;
                }
                x[cc] = (cc >= jb || lane > cc) ? 0.0 : (s0 + s1) * ipc[cc];
            }
            if (lane < jb) {
                dead_s[J0 + lane] = (deadmask >> lane) & 1u;
#pragma unroll
                for (int cc = 0; cc < kNb; ++cc)
                    if (cc >= lane && cc < jb) R[(long)(J0 + lane) * k + J0 + cc] = x[cc];
            }
        }
        __syncthreads();
        // (b) panel rows of R and T = X[:J0, :J0] R[:J0, J]
        const int npanel = k - J1;
        const int ntile = ((J0 + 3) / 4) * (kNb / 4);
        for (int t = tid; t < npanel + ntile; t += 256) {
            if (t < npanel) {
                const int c = J1 + t;
                double g[kNb];
#pragma unroll
                for (int i = 0; i < kNb; ++i) g[i] = (i < jb) ? R[(long)(J0 + i) * k + c] : 0.0;
#pragma unroll
                for (int j = 0; j < kNb; ++j) {
                    if (j < jb) {
                        double sacc = 0.0;
#pragma unroll
                        for (int i = 0; i <= j; ++i) sacc += R[(long)(J0 + i) * k + J0 + j] * g[i];
                        R[(long)(J0 + j) * k + c] = sacc;
                    }
                }
            } else {
                const int u = t - npanel;
                const int i0 = 4 * (u / (kNb / 4)), c0 = 4 * (u % (kNb / 4));
                double acc[4][4] = {};
                for (int L = i0; L < J0; ++L) {
                    double xv[4], rv[4];
#pragma unroll
                    for (int p = 0; p < 4; ++p)
                        xv[p] = (i0 + p <= L) ? R[(long)(i0 + p) * k + L] : 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        rv[q] = (c0 + q < jb) ? R[(long)L * k + J0 + c0 + q] : 0.0;
#pragma unroll
                    for (int p = 0; p < 4; ++p)
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[p][q] += xv[p] * rv[q];
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (i0 + p < J0) Tb[(i0 + p) * kNb + c0 + q] = acc[p][q];
            }
        }
        __syncthreads();
        // (c) trailing update (4 x 4 register tiles) and X[:J0, J] = -T X_JJ
        const int m = k - J1, T4 = (m + 3) / 4;
        const int nupd = T4 * T4, nx = J0 * jb;
        for (int t = tid; t < nupd + nx; t += 256) {
            if (t < nupd) {
                const int ta = t / T4, tc = t - (t / T4) * T4;
                if (ta > tc) continue;
                const int a0 = J1 + 4 * ta, c0 = J1 + 4 * tc;
                double acc[4][4] = {};
                for (int j = 0; j < jb; ++j) {
                    const double* rj = R + (long)(J0 + j) * k;
                    double ra[4], rc[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        ra[q] = (a0 + q < k) ? rj[a0 + q] : 0.0;
                        rc[q] = (c0 + q < k) ? rj[c0 + q] : 0.0;
                    }
#pragma unroll
                    for (int p = 0; p < 4; ++p)
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[p][q] += ra[p] * rc[q];
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (a0 + p < k && c0 + q < k) R[(long)(a0 + p) * k + c0 + q] -= acc[p][q];
            } else {
                const int u = t - nupd;
                const int i = u / jb, jj = u - (u / jb) * jb;
                double sacc = 0.0;
                for (int l = 0; l <= jj; ++l) sacc += Tb[i * kNb + l] * R[(long)(J0 + l) * k + J0 + jj];
                R[(long)i * k + J0 + jj] = -sacc;
            }
        }
        __syncthreads();
    }
    // X = D^{-1} R'^{-1}: G = D R'^T R' D with D = diag(sqrt(G_ii))
    for (int e = tid; e < k * k; e += 256) {
        const int i = e / k, c = e - (e / k) * k;
        out[e] = (c >= i && !dead_s[i]) ? R[e] * dsc[i] : 0.0;
    }
    if (dead) {
        for (int j = tid; j < k; j += 256) dead[(long)b * k + j] = dead_s[j];
        if (tid == 0) {
            int cnt = 0;
            for (int j = 0; j < k; ++j) cnt += dead_s[j];
            dead[(long)nbatch * k + b] = cnt;
        }
    }
}

// k <= 128: right-looking in registers, one barrier per pivot.  Thread
// (rb, cb) holds the 4 x 8 block at rows 4 rb.., columns 8 cb.. of the k x k
// working matrix W (column-block-major, so the waves whose columns are all
// factored drop out).  Row r of W holds the Schur complement S of the scaled
// Gram until pivot r is taken (both triangles, kept symmetric), then row r of
// the matrix V that becomes R'^{-1}: X R' = I is solved left to right, so at
// pivot j column j of X is final (X[i][j] = V[i][j] / R'[j][j], V[j][j] = 1)
// and its contribution V[i][c] -= X[i][j] R'[j][c] (i <= j < c) goes out at
// once from the row R'[j][.] = S[j][.] / R'[j][j] the trailing update uses.
// Every element (r, c > j) then takes one fused multiply-add with the
// coefficient W[r][j] (V[r][j] above the pivot, S[j][r] = S[r][j] below it;
// 1 + S[j][j] on the pivot row, which turns S[j][c] into V[j][c] =
// -S[j][c] / S[j][j]).  Pivot j's row (zero at and left of j) and column go
// through LDS, double-buffered; the pivot loop is unrolled by 8 so that the
// register holding them is known at compile time.  A dropped pivot has
// 1/R'[j][j] = 0: its row of R' and its row and column of X are zero.
constexpr int kCholThreads = 512, kCholRB = 4, kCholCB = 8;

template <int U>
struct CholStep {
    static constexpr int value = U;
};

__global__ __launch_bounds__(kCholThreads) void k_chol_inverse_reg(int k, const double* __restrict__ G,
                                                                 double* __restrict__ Rinv, double tol,
                                                                 int* __restrict__ dead, double near_identity,
                                                                 JobMap jm, int nbatch) {
    __shared__ double rowbuf[2][128];
    __shared__ double colbuf[2][128];
    __shared__ double dbuf[2];
    __shared__ int dead_s[128];
    __shared__ double dsc[128];  // 1/sqrt(G_ii)
    __shared__ double ipv[128];  // 1/R'[j][j], 0 for a dropped pivot
    __shared__ double red[kCholThreads / 64];
    const int tid = threadIdx.x;
    const int b = jlocal(jm, blockIdx.x);
    G = jptr(G, jm, blockIdx.x);
    Rinv = jptr(Rinv, jm, blockIdx.x);
    dead = jptr(dead, jm, blockIdx.x);
    const double* Gb = G + (long)b * k * k;
    double* out = Rinv + (long)b * k * k;
    const int RB = (k + kCholRB - 1) / kCholRB, CB = (k + kCholCB - 1) / kCholCB;
    const int cb = tid / RB, rb = tid - (tid / RB) * RB;
    const bool act = cb < CB;
    const int r0 = kCholRB * rb, c0 = kCholCB * cb;
    for (int i = tid; i < 128; i += kCholThreads) {
        const double gii = i < k ? Gb[(long)i * k + i] : 0.0;
        dsc[i] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
        colbuf[0][i] = colbuf[1][i] = 0.0;
        rowbuf[0][i] = rowbuf[1][i] = 0.0;
    }
    __syncthreads();
    double w[kCholRB][kCholCB];
    double off_max = 0.0;  // largest |G'_ij| off the diagonal; 1 if a diagonal is zero
#pragma unroll
    for (int p = 0; p < kCholRB; ++p)
#pragma unroll
        for (int q = 0; q < kCholCB; ++q) {
            const int r = r0 + p, c = c0 + q;
            const bool in = act && r < k && c < k;
            const double v = in ? Gb[(long)r * k + c] * dsc[r] * dsc[c] : 0.0;
            w[p][q] = v;
            if (in && r != c) off_max = fmax(off_max, fabs(v));
            else if (in && !(dsc[r] > 0.0)) off_max = 1.0;
        }
    if (near_identity > 0.0) {
        off_max = block_max(off_max, red);
        if (off_max <= near_identity) {  // R' = I: R^{-1} = D^{-1}, nothing dropped
            for (int e = tid; e < k * k; e += kCholThreads) {
                const int i = e / k, c = e - (e / k) * k;
                out[e] = (i == c) ? dsc[i] : 0.0;
            }
            if (dead) {
                for (int j = tid; j < k; j += kCholThreads) dead[(long)b * k + j] = 0;
                if (tid == 0) dead[(long)nbatch * k + b] = 0;
            }
            return;
        }
    }
    // pivot jn's row and column (jn % 8 == QN, so its row is w[QN % 4] of the
    // threads with r0 == jn - QN % 4 and its column w[.][QN] of those with
    // c0 == jn - QN) into buffer bf
    auto publish = [&](auto qn, int jn, int bf) {
        constexpr int QN = decltype(qn)::value, PN = QN % kCholRB;
        if (act && r0 + PN == jn) {
#pragma unroll
            for (int q = 0; q < kCholCB; ++q) rowbuf[bf][c0 + q] = c0 + q > jn ? w[PN][q] : 0.0;
            if (c0 + QN == jn) dbuf[bf] = w[PN][QN];
        }
        if (act && c0 + QN == jn)
#pragma unroll
            for (int p = 0; p < kCholRB; ++p) colbuf[bf][r0 + p] = r0 + p == jn ? 1.0 + w[p][QN] : w[p][QN];
    };
    // pivot j (j % 8 == U; bf = j & 1 = U & 1 since the blocks of 8 start even)
    auto step = [&](auto u, int j) {
        constexpr int U = decltype(u)::value, bf = U & 1;
        const double d = dbuf[bf];
        const bool dj = !(d > tol);
        const double ip = dj ? 0.0 : fast_rsq(d);
        const double ip2 = ip * ip;
        if (act && c0 + kCholCB - 1 > j) {
            double rc[kCholCB], cr[kCholRB];
#pragma unroll
            for (int q = 0; q < kCholCB; ++q) rc[q] = rowbuf[bf][c0 + q] * ip2;
#pragma unroll
            for (int p = 0; p < kCholRB; ++p) cr[p] = colbuf[bf][r0 + p];
#pragma unroll
            for (int p = 0; p < kCholRB; ++p)
#pragma unroll
                for (int q = 0; q < kCholCB; ++q) w[p][q] = fma(-cr[p], rc[q], w[p][q]);
        }
        if (j + 1 < k) publish(CholStep<(U + 1) % kCholCB>{}, j + 1, bf ^ 1);
        if (tid == 0) {
            ipv[j] = ip;
            dead_s[j] = dj ? 1 : 0;
        }
        __syncthreads();
    };
    publish(CholStep<0>{}, 0, 0);
    __syncthreads();
    for (int J = 0; J < k; J += kCholCB) {
        step(CholStep<0>{}, J);
        if (J + 1 < k) step(CholStep<1>{}, J + 1);
        if (J + 2 < k) step(CholStep<2>{}, J + 2);
        if (J + 3 < k) step(CholStep<3>{}, J + 3);
        if (J + 4 < k) step(CholStep<4>{}, J + 4);
        if (J + 5 < k) step(CholStep<5>{}, J + 5);
        if (J + 6 < k) step(CholStep<6>{}, J + 6);
        if (J + 7 < k) step(CholStep<7>{}, J + 7);
    }
    // R^{-1} = D^{-1} R'^{-1}, X[i][c] = V[i][c] / R'[c][c]
    if (act)
#pragma unroll
        for (int p = 0; p < kCholRB; ++p)
#pragma unroll
            for (int q = 0; q < kCholCB; ++q) {
                const int i = r0 + p, c = c0 + q;
                const double v = c == i ? 1.0 : w[p][q];  // V[i][i] = 1
                if (i < k && c < k) out[(long)i * k + c] = (c >= i && !dead_s[i]) ? v * ipv[c] * dsc[i] : 0.0;
            }
    if (dead) {
        for (int j = tid; j < k; j += kCholThreads) dead[(long)b * k + j] = dead_s[j];
        if (tid == 0) {
            int cnt = 0;
            for (int j = 0; j < k; ++j) cnt += dead_s[j];
            dead[(long)nbatch * k + b] = cnt;
        }
    }
}

static size_t chol_lds_bytes(int k, bool in_lds) {
    return ((in_lds ? (size_t)k * k : 0) + (size_t)k * kNb) * sizeof(double);
}

void chol_inverse(hipStream_t s, int batch, int k, const double* G, double* Rinv, double tol,
                  int* dead, double near_identity, JobMap jm) {
    if (batch <= 0) return;
    const int blocks = batch * (jm.delta ? jm.njobs : 1);
    if (jm.delta) jm.per_job = batch;
    IPEPS_REQUIRE(k >= 1 && k <= 256, IPEPS_EINVAL, "chol_inverse: k must be in 1..256");
    const bool in_lds = k <= 128;
    const size_t lds = chol_lds_bytes(k, in_lds);
    static bool attr_set = false;
    if (!attr_set) {
        HIP_CHECK(hipFuncSetAttribute((const void*)k_chol_inverse<true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)chol_lds_bytes(128, true)));
        HIP_CHECK(hipFuncSetAttribute((const void*)k_chol_inverse<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)chol_lds_bytes(256, false)));
        attr_set = true;
    }
    if (in_lds)
        hipLaunchKernelGGL(k_chol_inverse_reg, dim3(blocks), dim3(kCholThreads), 0, s, k, G, Rinv, tol, dead,
                           near_identity, jm, batch);
    else
        hipLaunchKernelGGL(k_chol_inverse<false>, dim3(blocks), dim3(256), lds, s, k, G, Rinv, tol, dead,
                           near_identity, jm, batch);
    HIP_CHECK(hipGetLastError());
}

// ----------------------------------------------------------------- columns
__global__ __launch_bounds__(256) void k_normalize_columns(int n, int k, double* X) {
    __shared__ double red[4];
    const int j = blockIdx.x, b = blockIdx.y;
    double* Xb = X + (long)b * n * k;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += Xb[(long)i * k + j] * Xb[(long)i * k + j];
    s = block_sum(s, red);
    const double inv = s > 0 ? 1.0 / sqrt(s) : 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) Xb[(long)i * k + j] *= inv;
}

void normalize_columns(hipStream_t s, int batch, int n, int k, double* X) {
    if (batch <= 0 || k <= 0) return;
    hipLaunchKernelGGL(k_normalize_columns, dim3(k, batch), dim3(256), 0, s, n, k, X);
    HIP_CHECK(hipGetLastError());
}

// The refill seed of a job: ctr = {config seed, calls so far}; every call
// hashes seed * C1 + C2 * (calls + 1), then k_count_up advances the count
// (device-resident, so a replayed graph draws new numbers each time).
__device__ inline uint64_t refill_seed(const uint64_t* ctr) {
    return ctr[0] * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull * (ctr[1] + 1);
}

__global__ __launch_bounds__(256) void k_dead_fill(int n, int k, const int* __restrict__ dead,
                                                   const uint64_t* __restrict__ ctr, double* __restrict__ R,
                                                   JobMap jm, int batch) {
    const long tot = (long)n * k;
    dead = jptr(dead, jm, blockIdx.y);
    ctr = jptr(ctr, jm, blockIdx.y);
    R = jptr(R, jm, blockIdx.y);
    const int b = jlocal(jm, blockIdx.y);
    if (dead[(long)batch * k + b] == 0) return;
    const uint64_t seed = refill_seed(ctr);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
         e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e % k);
        R[b * tot + e] = dead[(long)b * k + j] ? 2.0 * hash_uniform(seed, (uint64_t)(b * tot + e)) - 1.0
                                               : 0.0;
    }
}

__global__ void k_count_up(uint64_t* ctr, JobMap jm) {
    if (threadIdx.x == 0) jptr(ctr, jm, blockIdx.x)[1] += 1;
}

void dead_fill(hipStream_t s, int batch, int n, int k, const int* dead, uint64_t* ctr, double* R, JobMap jm) {
    if (batch <= 0 || k <= 0) return;
    const long tot = (long)n * k;
    const int grid = ceil_div(tot, 256) < 1024 ? (int)ceil_div(tot, 256) : 1024;
    const int nj = jm.delta ? jm.njobs : 1;
    jm.per_job = batch;
    hipLaunchKernelGGL(k_dead_fill, dim3(grid, batch * nj), dim3(256), 0, s, n, k, dead, ctr, R, jm, batch);
    jm.per_job = 1;
    hipLaunchKernelGGL(k_count_up, dim3(nj), dim3(64), 0, s, ctr, jm);
    HIP_CHECK(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_add_gated(long count, const int* __restrict__ gate,
                                                   const double* __restrict__ Y,
                                                   double* __restrict__ X, JobMap jm) {
    gate = jptr(gate, jm, blockIdx.y);
    Y = jptr(Y, jm, blockIdx.y);
    X = jptr(X, jm, blockIdx.y);
    const int b = jlocal(jm, blockIdx.y);
    if (gate[b] == 0) return;
    const double* Yb = Y + b * count;
    double* Xb = X + b * count;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
         e += (long)gridDim.x * blockDim.x)
        Xb[e] += Yb[e];
}

void add_gated(hipStream_t s, int batch, long count, const int* gate, const double* Y, double* X, JobMap jm) {
    if (batch <= 0 || count <= 0) return;
    const int grid = ceil_div(count, 256) < 1024 ? (int)ceil_div(count, 256) : 1024;
    const int nj = jm.delta ? jm.njobs : 1;
    jm.per_job = batch;
    hipLaunchKernelGGL(k_add_gated, dim3(grid, batch * nj), dim3(256), 0, s, count, gate, Y, X, jm);
    HIP_CHECK(hipGetLastError());
}

}  // namespace ipeps
