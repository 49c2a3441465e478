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
        const int m = ne - 1;
        *p = (r + k) % m;
        *q = (r - k + m) % m;
    }
    if (*p > *q) {
        int t = *p;
        *p = *q;
        *q = t;
    }
}

// Ac: m x n column-major working copy of A, Vc: n x n column-major (or NULL).
// Each pair of a round is handled by a group of 16 lanes (4 groups per wave);
// the three inner products are summed with DPP moves inside the group.
__device__ void jacobi_sweeps(int m, int n, double* Ac, double* Vc, int* flag, double* red) {
    const int g16 = threadIdx.x & 15, group = threadIdx.x >> 4, ngroups = blockDim.x >> 4;
    const int ne = n + (n & 1);
    const int npair = ne / 2;
    const double tol = 4.0 * m * 1.11e-16;
    // columns below 1e-14 |A|_F are rounding noise: a rotation against a large
    // column re-pollutes them at their own size, so they are left alone
    double fro = 0.0;
    for (long e = threadIdx.x; e < (long)m * n; e += blockDim.x) fro += Ac[e] * Ac[e];
    fro = block_sum(fro, red);
    const double small2 = 1e-28 * fro;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int r = 0; r < ne - 1; ++r) {
            for (int k = group; k < npair; k += ngroups) {
                int p, q;
                circle_pair(r, k, ne, &p, &q);
                if (q >= n) continue;
                double* ap = Ac + (long)p * m;
                double* aq = Ac + (long)q * m;
                double al = 0, be = 0, ga = 0;
                for (int i = g16; i < m; i += 16) {
                    const double x = ap[i], y = aq[i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = group16_sum(al);
                be = group16_sum(be);
                ga = group16_sum(ga);
                if (al <= small2 || be <= small2) continue;
                if (fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = g16; i < m; i += 16) {
                    const double x = ap[i], y = aq[i];
                    ap[i] = c * x - s * y;
                    aq[i] = s * x + c * y;
                }
                if (Vc) {
                    double* vp = Vc + (long)p * n;
                    double* vq = Vc + (long)q * n;
                    for (int i = g16; i < n; i += 16) {
                        const double x = vp[i], y = vq[i];
                        vp[i] = c * x - s * y;
                        vq[i] = s * x + c * y;
                    }
                }
                if (g16 == 0) *flag = 1;
            }
            __syncthreads();
        }
        const int any = *flag;
        __syncthreads();
        if (!any) break;
    }
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

template <bool IN_LDS>
__global__ __launch_bounds__(1024) void k_jacobi_svd(int m, int n, const double* __restrict__ A,
                                                     long lda, long strideA, double* sigma,
                                                     double* U, double* V, double* work) {
    extern __shared__ double smem[];
    __shared__ int flag;
    __shared__ double red[16];
    const int b = blockIdx.x;
    const bool wantV = (V != nullptr);
    const long nv = wantV ? (long)n * n : 0;
    double *Ac, *Vc, *sig_s;
    if (IN_LDS) {
        Ac = smem;
    } else {
        Ac = work + (long)b * ((long)m * n + nv + n);
    }
    Vc = Ac + (long)m * n;
    sig_s = Vc + nv;
    const double* Ab = A + (long)b * strideA;
    for (long e = threadIdx.x; e < (long)m * n; e += blockDim.x) {
        const int j = (int)(e / m), i = (int)(e % m);
        Ac[e] = Ab[(long)i * lda + j];
    }
    for (long e = threadIdx.x; e < nv; e += blockDim.x) Vc[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
    __syncthreads();
    jacobi_sweeps(m, n, Ac, wantV ? Vc : nullptr, &flag, red);
    __syncthreads();
    jacobi_finish(m, n, Ac, Vc, sig_s, sigma + (long)b * n, U ? U + (long)b * m * n : nullptr,
                  V ? V + (long)b * n * n : nullptr);
}

static size_t jacobi_lds_bytes(int m, int n, bool wantV) {
    return ((size_t)m * n + (wantV ? (size_t)n * n : 0) + n) * sizeof(double);
}
static const size_t kMaxLds = 160 * 1024 - 1024;

size_t jacobi_svd_real_work(int batch, int m, int n) {
    if (jacobi_lds_bytes(m, n, true) <= kMaxLds) return 0;
    return (size_t)batch * ((size_t)m * n + (size_t)n * n + n);
}

void jacobi_svd_real(hipStream_t s, int batch, int m, int n, const double* A, long lda,
                     long strideA, double* sigma, double* U, double* V, double* work) {
    if (batch <= 0 || n <= 0) return;
    const size_t lds = jacobi_lds_bytes(m, n, V != nullptr);
    if (lds <= kMaxLds) {
        static bool attr_set = false;
        if (!attr_set) {
            HIP_CHECK(hipFuncSetAttribute((const void*)k_jacobi_svd<true>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)kMaxLds));
            attr_set = true;
        }
        hipLaunchKernelGGL(k_jacobi_svd<true>, dim3(batch), dim3(1024), lds, s, m, n, A, lda,
                           strideA, sigma, U, V, work);
    } else {
        IPEPS_REQUIRE(work != nullptr, IPEPS_EINVAL, "jacobi_svd_real: work buffer needed");
        hipLaunchKernelGGL(k_jacobi_svd<false>, dim3(batch), dim3(1024), 0, s, m, n, A, lda,
                           strideA, sigma, U, V, work);
    }
    HIP_CHECK(hipGetLastError());
}

// ----------------------------------------------------------------- Cholesky
// G = R^T R (R upper) with dropping, then R^{-1} in place (column-oriented
// triangular inversion); both in LDS (k <= 128), one workgroup of 4 waves per
// matrix.  Each trailing-update row is split over 4 lanes.  A dropped pivot
// zeroes its row of R and its row and column of R^{-1}, so the matching
// column of X R^{-1} is zero; dead (if not null) receives 1 for such columns.
__global__ __launch_bounds__(256) void k_chol_inverse(int k, const double* __restrict__ G,
                                                      double* __restrict__ Rinv, double tol,
                                                      int* __restrict__ dead) {
    extern __shared__ double R[];  // k*k, row-major
    __shared__ double colj[128];
    __shared__ int dead_s[128];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int b = blockIdx.x;
    const double* Gb = G + (long)b * k * k;
    double* Xb = Rinv + (long)b * k * k;
    for (int e = tid; e < k * k; e += nt) R[e] = Gb[e];
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        const double dj = R[j * k + j];
        const bool dead = !(dj > tol);  // every thread decides alike
        const double piv = dead ? 0.0 : sqrt(dj);
        const double ipiv = dead ? 0.0 : 1.0 / piv;
        __syncthreads();
        for (int c = j + 1 + tid; c < k; c += nt) R[j * k + c] *= ipiv;
        if (tid == 0) {
            R[j * k + j] = piv;
            dead_s[j] = dead;
        }
        __syncthreads();
        // trailing update of the upper triangle: row a split over 4 threads
        for (int t = tid; t < 4 * (k - j - 1); t += nt) {
            const int a = j + 1 + (t >> 2), part = t & 3;
            const double rja = R[j * k + a];
            double* __restrict__ ra = R + a * k;
            const double* __restrict__ rj = R + j * k;
            if (rja != 0.0) {
#pragma unroll 4
                for (int c = a + part; c < k; c += 4) ra[c] -= rja * rj[c];
            }
        }
        __syncthreads();
    }
    // in-place inverse of the upper-triangular R
    for (int j = 0; j < k; ++j) {
        const bool dead = dead_s[j];
        for (int i = tid; i < j; i += nt) colj[i] = R[i * k + j];
        __syncthreads();
        if (dead) {
            for (int i = tid; i <= j; i += nt) R[i * k + j] = 0.0;
        } else {
            const double inv = 1.0 / R[j * k + j];
            for (int i = tid; i < j; i += nt) {
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                const double* __restrict__ ri = R + i * k;
                int l = i;
                for (; l + 3 < j; l += 4) {
                    s0 += ri[l] * colj[l];
                    s1 += ri[l + 1] * colj[l + 1];
                    s2 += ri[l + 2] * colj[l + 2];
                    s3 += ri[l + 3] * colj[l + 3];
                }
                for (; l < j; ++l) s0 += ri[l] * colj[l];
                R[i * k + j] = -inv * ((s0 + s1) + (s2 + s3));
            }
            if (tid == 0) R[j * k + j] = inv;
        }
        __syncthreads();
    }
    for (int e = tid; e < k * k; e += nt) {
        const int i = e / k, c = e % k;
        Xb[e] = (c >= i && !dead_s[i]) ? R[e] : 0.0;
    }
    if (dead) {
        for (int j = tid; j < k; j += nt) dead[(long)b * k + j] = dead_s[j];
        if (tid == 0) {
            int c = 0;
            for (int j = 0; j < k; ++j) c += dead_s[j];
            dead[(long)gridDim.x * k + b] = c;
        }
    }
}

void chol_inverse(hipStream_t s, int batch, int k, const double* G, double* Rinv, double tol,
                  int* dead) {
    if (batch <= 0) return;
    IPEPS_REQUIRE(k <= 128, IPEPS_EINVAL, "chol_inverse: k > 128");
    const size_t lds = (size_t)k * k * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
        HIP_CHECK(hipFuncSetAttribute((const void*)k_chol_inverse,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      128 * 128 * (int)sizeof(double)));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_chol_inverse, dim3(batch), dim3(256), lds, s, k, G, Rinv, tol, dead);
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

__global__ __launch_bounds__(256) void k_dead_fill(int n, int k, const int* __restrict__ dead,
                                                   uint64_t seed, double* __restrict__ R) {
    const long tot = (long)n * k;
    const int b = blockIdx.y;
    if (dead[(long)gridDim.y * k + b] == 0) return;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
         e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e % k);
        R[b * tot + e] = dead[(long)b * k + j] ? 2.0 * hash_uniform(seed, (uint64_t)(b * tot + e)) - 1.0
                                               : 0.0;
    }
}

void dead_fill(hipStream_t s, int batch, int n, int k, const int* dead, uint64_t seed, double* R) {
    if (batch <= 0 || k <= 0) return;
    const long tot = (long)n * k;
    const int grid = ceil_div(tot, 256) < 1024 ? (int)ceil_div(tot, 256) : 1024;
    hipLaunchKernelGGL(k_dead_fill, dim3(grid, batch), dim3(256), 0, s, n, k, dead, seed, R);
    HIP_CHECK(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_add_gated(long count, const int* __restrict__ gate,
                                                   const double* __restrict__ Y,
                                                   double* __restrict__ X) {
    const int b = blockIdx.y;
    if (gate[b] == 0) return;
    const double* Yb = Y + b * count;
    double* Xb = X + b * count;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
         e += (long)gridDim.x * blockDim.x)
        Xb[e] += Yb[e];
}

void add_gated(hipStream_t s, int batch, long count, const int* gate, const double* Y, double* X) {
    if (batch <= 0 || count <= 0) return;
    const int grid = ceil_div(count, 256) < 1024 ? (int)ceil_div(count, 256) : 1024;
    hipLaunchKernelGGL(k_add_gated, dim3(grid, batch), dim3(256), 0, s, count, gate, Y, X);
    HIP_CHECK(hipGetLastError());
}

}  // namespace ipeps
