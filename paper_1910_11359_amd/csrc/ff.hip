// Free-fermion Néel dynamics (non-interacting comparison workload).
//
// One workgroup per (realization r, filled orbital j): the orbital's L*L
// complex amplitudes stay in registers (a run of S consecutive sites per
// thread) for the whole run, and the hopping term is applied as a five-point
// stencil, neighbours inside a thread's run from registers and the others
// through a double-buffered LDS copy (one barrier per application).  Each observation
// interval is split into pieces whose Chebyshev argument a*dt is at most
// kMaxArg, and each piece applies
//     exp(-i h dt) = exp(-i b dt) sum_k (2 - [k = 0]) (-i)^k J_k(a dt) T_k((h - b) / a)
// (Chebyshev polynomials of the shifted, scaled Hamiltonian, whose spectrum
// lies in [-1, 1] by Gershgorin's bound a = (max eps - min eps)/2 + 4|tau|,
// b = (max eps + min eps)/2), truncated where |J_k| < 1e-18.  After each
// interval the orbital's weight on the two sublattices is written to a
// workspace; a second kernel sums the orbitals of each (r, t) in a fixed
// order, so results are deterministic.
#include "../../include/ff.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <vector>

#include "common.h"
#include "linalg.h"

namespace ipeps {
namespace {

constexpr int kFfThreads = 256;
constexpr int kFfMaxTerms = 160;    // coefficients kept per piece
constexpr double kFfMaxArg = 60.0;  // a * dt per piece
constexpr double kFfCut = 1e-18;    // |J_k| below which the series stops

// J_0(x) .. J_kmax(x), x >= 0.  x < 0.5: power series; otherwise the
// backward recurrence J_{k-1} = (2k/x) J_k - J_{k+1} started well above
// max(kmax, x) (Miller's method), normalised by J_0 + 2 sum_{m>=1} J_{2m} = 1
// and rescaled whenever it grows beyond 1e200.
__host__ __device__ inline void bessel_j_seq(double x, int kmax, double* J) {
    if (x == 0.0) {
        J[0] = 1.0;
        for (int k = 1; k <= kmax; ++k) J[k] = 0.0;
        return;
    }
    if (x < 0.5) {
        const double h = 0.5 * x, h2 = h * h;
        double lead = 1.0;  // (x/2)^k / k!
        for (int k = 0; k <= kmax; ++k) {
            if (k > 0) lead *= h / k;
            double term = lead, sum = lead;
            for (int m = 1; m <= 12; ++m) {
                term *= -h2 / ((double)m * (double)(m + k));
                sum += term;
            }
            J[k] = sum;
        }
        return;
    }
    const int base = kmax > (int)x ? kmax : (int)x;
    int top = base + 40 + (int)(4.0 * sqrt((double)base));
    top += top & 1;
    double jp = 0.0, jc = 1e-30, norm = 0.0;
    for (int k = top; k >= 1; --k) {
        const double jm = (2.0 * k / x) * jc - jp;  // J_{k-1} up to a common factor
        const int km = k - 1;
        if (km <= kmax) J[km] = jm;
        if (km == 0) norm += jm;
        else if ((km & 1) == 0) norm += 2.0 * jm;
        jp = jc;
        jc = jm;
        if (fabs(jc) > 1e200) {
            jc *= 1e-200;
            jp *= 1e-200;
            norm *= 1e-200;
            for (int q = km; q <= kmax; ++q) J[q] *= 1e-200;
        }
    }
    const double inv = 1.0 / norm;
    for (int k = 0; k <= kmax; ++k) J[k] *= inv;
}

// Thread t owns the contiguous run of sites t*S .. t*S + S - 1, so the
// neighbours along y (i +- 1) are mostly its own registers; the other
// neighbours are read from the LDS copy.
template <int S>
__global__ __launch_bounds__(kFfThreads) void k_ff_neel(int L, int pbc, double tau, double dt, int n_times,
                                                        const double* __restrict__ eps_all, int M,
                                                        double* __restrict__ part_e, double* __restrict__ part_o) {
    extern __shared__ double lds[];  // [2 buffers][re, im][L*L]
    __shared__ double cj[kFfMaxTerms];
    __shared__ double red[kFfThreads / 64];
    __shared__ int sh_K, sh_site;
    const int nsite = L * L, tid = threadIdx.x;
    const int j = blockIdx.x, r = blockIdx.y;
    const int i0 = tid * S;
    const double* eps = eps_all + (long)r * nsite;

    double ep[S];
    double lo = 1e300, hi = -1e300;
#pragma unroll
    for (int e = 0; e < S; ++e) {
        ep[e] = 0.0;
        if (i0 + e < nsite) {
            ep[e] = eps[i0 + e];
            lo = fmin(lo, ep[e]);
            hi = fmax(hi, ep[e]);
        }
    }
    hi = block_max(hi, red);
    lo = -block_max(-lo, red);
    const double b = 0.5 * (hi + lo);
    double a = 0.5 * (hi - lo) + 4.0 * fabs(tau);
    if (!(a > 0.0)) a = 1.0;  // h = b: any positive a is a valid bound
    const double ia = 1.0 / a, tia = tau * ia;
    const double xtot = a * dt;
    if (!(xtot <= kFfMaxArg * 1e5)) {
        // infinite fields, or more than 1e5 pieces per interval: NaN outputs
        if (tid == 0)
            for (int m = 0; m < n_times; ++m) {
                const long q = ((long)r * n_times + m) * M + j;
                part_e[q] = part_o[q] = __builtin_nan("");
            }
        return;
    }
    int nsub = (int)ceil(xtot / kFfMaxArg);
    nsub = nsub < 1 ? 1 : nsub;
    const double xs = xtot / nsub, dts = dt / nsub;
    if (tid == 0) {
        bessel_j_seq(xs, kFfMaxTerms - 1, cj);
        int K = kFfMaxTerms;
        while (K > 1 && fabs(cj[K - 1]) < kFfCut) --K;
        sh_K = K;
        // j-th filled site in increasing site order (row x holds (L - (x & 1) + 1) / 2)
        int rem = j, x = 0;
        while (rem >= (L - (x & 1) + 1) / 2) {
            rem -= (L - (x & 1) + 1) / 2;
            ++x;
        }
        sh_site = x * L + (x & 1) + 2 * rem;
    }
    __syncthreads();
    const int K = sh_K, site = sh_site;
    const double cph = cos(b * dts), sph = -sin(b * dts);  // exp(-i b dts)
    // diagonal of (h - b)/a, zero beyond the lattice
    double dg[S];
#pragma unroll
    for (int e = 0; e < S; ++e) dg[e] = (i0 + e < nsite) ? (ep[e] - b) * ia : 0.0;
    const int y0 = i0 % L;

    double t0r[S], t0i[S], t1r[S], t1i[S], ar[S], ai[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
        t0r[e] = (i0 + e == site) ? 1.0 : 0.0;
        t0i[e] = 0.0;
        t1r[e] = t1i[e] = ar[e] = ai[e] = 0.0;
    }
    int par = 0;
    // out <- H~ in (rec = false) or out <- 2 H~ in - out (rec = true), with
    // H~ = (h - b)/a, through LDS buffer par
    auto apply = [&](const double* inr, const double* ini, double* outr, double* outi, bool rec) {
        double* br = lds + (long)par * 2 * nsite;
        double* bi = br + nsite;
#pragma unroll
        for (int e = 0; e < S; ++e)
            if (i0 + e < nsite) {
                br[i0 + e] = inr[e];
                bi[i0 + e] = ini[e];
            }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int i = i0 + e;
            double sr = 0.0, si = 0.0;
            if (i < nsite) {
                int y = y0 + e;  // y of site i (run may cross rows)
                while (y >= L) y -= L;
                const int x = i / L;
                // along y
                if (y > 0) {
                    if (e > 0) {
                        sr += inr[e - 1];
                        si += ini[e - 1];
                    } else {
                        sr += br[i - 1];
                        si += bi[i - 1];
                    }
                } else if (pbc) {
                    sr += br[i + L - 1];
                    si += bi[i + L - 1];
                }
                if (y + 1 < L) {
                    if (e + 1 < S) {
                        sr += inr[e + 1];
                        si += ini[e + 1];
                    } else {
                        sr += br[i + 1];
                        si += bi[i + 1];
                    }
                } else if (pbc) {
                    sr += br[i - L + 1];
                    si += bi[i - L + 1];
                }
                // along x
                if (x > 0) {
                    sr += br[i - L];
                    si += bi[i - L];
                } else if (pbc) {
                    sr += br[i + nsite - L];
                    si += bi[i + nsite - L];
                }
                if (x + 1 < L) {
                    sr += br[i + L];
                    si += bi[i + L];
                } else if (pbc) {
                    sr += br[i - nsite + L];
                    si += bi[i - nsite + L];
                }
            }
            const double hr = dg[e] * inr[e] - tia * sr, hi2 = dg[e] * ini[e] - tia * si;
            outr[e] = rec ? 2.0 * hr - outr[e] : hr;
            outi[e] = rec ? 2.0 * hi2 - outi[e] : hi2;
        }
        par ^= 1;
    };
    // acc += (-i)^k w T_k
    auto accum = [&](int k, const double* tr, const double* ti) {
        const double w = 2.0 * cj[k];
        const int ph = k & 3;
#pragma unroll
        for (int e = 0; e < S; ++e) {
            if (ph == 0) {
                ar[e] += w * tr[e];
                ai[e] += w * ti[e];
            } else if (ph == 1) {
                ar[e] += w * ti[e];
                ai[e] -= w * tr[e];
            } else if (ph == 2) {
                ar[e] -= w * tr[e];
                ai[e] -= w * ti[e];
            } else {
                ar[e] -= w * ti[e];
                ai[e] += w * tr[e];
            }
        }
    };
    for (int m = 0; m < n_times; ++m) {
        for (int s = 0; s < nsub; ++s) {
            const double w0 = cj[0];
#pragma unroll
            for (int e = 0; e < S; ++e) {
                ar[e] = w0 * t0r[e];
                ai[e] = w0 * t0i[e];
            }
            if (K > 1) {
                apply(t0r, t0i, t1r, t1i, false);  // T_1
                accum(1, t1r, t1i);
            }
            // T_{k+1} = 2 H~ T_k - T_{k-1} overwrites T_{k-1}: t0 and t1 swap roles
            for (int k = 2; k < K; k += 2) {
                apply(t1r, t1i, t0r, t0i, true);  // T_k into t0
                accum(k, t0r, t0i);
                if (k + 1 < K) {
                    apply(t0r, t0i, t1r, t1i, true);  // T_{k+1} into t1
                    accum(k + 1, t1r, t1i);
                }
            }
#pragma unroll
            for (int e = 0; e < S; ++e) {
                t0r[e] = cph * ar[e] - sph * ai[e];
                t0i[e] = cph * ai[e] + sph * ar[e];
            }
        }
        double se = 0.0, so = 0.0;
#pragma unroll
        for (int e = 0; e < S; ++e) {
            const int i = i0 + e;
            if (i < nsite) {
                const double p = t0r[e] * t0r[e] + t0i[e] * t0i[e];
                if ((((i / L) + (i - (i / L) * L)) & 1) == 0) se += p;
                else so += p;
            }
        }
        se = block_sum(se, red);
        so = block_sum(so, red);
        if (tid == 0) {
            const long q = ((long)r * n_times + m) * M + j;
            part_e[q] = se;
            part_o[q] = so;
        }
    }
}

// n[q] = scale * sum_j part[q*M + j], fixed order (block tree over j)
__global__ __launch_bounds__(256) void k_ff_sum(int M, const double* __restrict__ part_e,
                                                const double* __restrict__ part_o, double se, double so,
                                                double* __restrict__ n_even, double* __restrict__ n_odd) {
    __shared__ double red[4];
    const long q = blockIdx.x;
    double ae = 0.0, ao = 0.0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        ae += part_e[q * M + j];
        ao += part_o[q * M + j];
    }
    ae = block_sum(ae, red);
    ao = block_sum(ao, red);
    if (threadIdx.x == 0) {
        n_even[q] = ae * se;
        n_odd[q] = ao * so;
    }
}

template <int S>
hipError_t launch_ff(hipStream_t s, int L, int pbc, double tau, double dt, int n_times, int n_real,
                     const double* eps, int M, double* pe, double* po) {
    const size_t lds = (size_t)4 * L * L * sizeof(double);
    static bool attr_set = false;  // L*L <= 2048: up to 64 KB of dynamic LDS
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_ff_neel<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 4 * 2048 * (int)sizeof(double));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_ff_neel<S>, dim3(M, n_real), dim3(kFfThreads), lds, s, L, pbc, tau, dt, n_times, eps, M,
                       pe, po);
    return hipGetLastError();
}

}  // namespace
// ------------------------------------------------------------ spectrum, IPR
// h + c I per realization (row-major n x n, n = L^2) with c = 2 G, G =
// max_i |eps_i| + 4 |tau| (a Gershgorin bound on |E|; c = 1 when G = 0): its
// spectrum lies in [G, 3G], so its singular vectors are eigenvectors of h
// and sigma - c are the energies.
__global__ __launch_bounds__(256) void k_ff_shifted_h(int L, int pbc, double tau, const double* eps,
                                                     double* H, double* shift) {
    __shared__ double red[4];
    const int b = blockIdx.x, n = L * L;
    const double* e = eps + (long)b * n;
    double g = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) g = fmax(g, fabs(e[i]));
    g = block_max(g, red) + 4.0 * fabs(tau);
    const double c = g > 0.0 ? 2.0 * g : 1.0;
    if (threadIdx.x == 0) shift[b] = c;
    double* Hb = H + (long)b * n * n;
    for (long idx = threadIdx.x; idx < (long)n * n; idx += blockDim.x) {
        const int i = (int)(idx / n), j = (int)(idx % n);
        double v = 0.0;
        if (i == j) {
            v = e[i] + c;
        } else {
            int dx = j / L - i / L, dy = j % L - i % L;
            bool adj;
            if (pbc) {  // L >= 3: +-1 modulo L are distinct neighbours
                dx = (dx + L) % L;
                dy = (dy + L) % L;
                adj = ((dx == 1 || dx == L - 1) && dy == 0) || (dx == 0 && (dy == 1 || dy == L - 1));
            } else {
                adj = (abs(dx) == 1 && dy == 0) || (dx == 0 && abs(dy) == 1);
            }
            if (adj) v = -tau;
        }
        Hb[idx] = v;
    }
}

// Energies ascending, IPR of every eigenvector (sum_i u_i^4), and per
// rescaled-energy bin (width 0.05, epsilon = 1 in the last one) the summed
// IPR and the number of states, one realization per workgroup; the bin sums
// run over the states in ascending order (deterministic).
constexpr int kIprBins = 20;
__global__ __launch_bounds__(256) void k_ff_ipr(int n, const double* sig, const double* U,
                                               const double* shift, double* E, double* ipr,
                                               double* bin_ipr, int* bin_cnt) {
    __shared__ double Es[256], Is[256];
    __shared__ int Bs[256];
    const int b = blockIdx.x;
    const double c = shift[b];
    const double* sb = sig + (long)b * n;
    const double* Ub = U + (long)b * n * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {  // k: descending singular value
        double s4 = 0.0;
        for (int i = 0; i < n; ++i) {
            const double u = Ub[(long)i * n + k];
            s4 += (u * u) * (u * u);
        }
        Es[n - 1 - k] = sb[k] - c;
        Is[n - 1 - k] = s4;
    }
    __syncthreads();
    const double lo = Es[0], hi = Es[n - 1];
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        int bin = 0;
        if (hi > lo) {
            bin = (int)floor((Es[a] - lo) / (hi - lo) / 0.05);
            bin = bin < kIprBins - 1 ? bin : kIprBins - 1;
        }
        Bs[a] = bin;
        E[(long)b * n + a] = Es[a];
        ipr[(long)b * n + a] = Is[a];
    }
    __syncthreads();
    if (threadIdx.x < kIprBins) {
        double sum = 0.0;
        int cnt = 0;
        for (int a = 0; a < n; ++a)
            if (Bs[a] == (int)threadIdx.x) {
                sum += Is[a];
                ++cnt;
            }
        bin_ipr[(long)b * kIprBins + threadIdx.x] = sum;
        bin_cnt[(long)b * kIprBins + threadIdx.x] = cnt;
    }
}


// ------------------------------------------------- block Jacobi (L > 16)
// The L^2 x L^2 eigenproblems beyond one workgroup's LDS: a two-sided block
// Jacobi on h (padded to np = 32 nb rows with decoupled diagonal entries 3G
// above the spectrum), blocks of 32 indices paired by the circle method
// (nb - 1 rounds a sweep, nb rounded up to even, so padding may fill a
// whole block).  Per round and pair (I, J): the 64 x 64 block
// S = h[IJ, IJ] is diagonalised exactly (one-sided Jacobi of S + 2G I, which
// is positive definite, so its right singular vectors Q are eigenvectors of
// S), then h <- Q^T h Q on the rows and columns IJ and V <- V Q, as 64 x 64
// MFMA products per 64-row (or 64-column) chunk.  Sweeps end once the
// squared off-diagonal part of h is below 1e-24 of its squared Frobenius
// norm, or below 1e-18 and no longer shrinking by 4x per sweep (the level
// the 64 x 64 solves can reach).
constexpr int kBjB = 32, kBjW = 2 * kBjB;

__device__ inline void bj_pair(int r, int kk, int nbp, int* p, int* q) {
    if (kk == 0) {
        *p = r;
        *q = nbp - 1;
    } else {
        const int m = nbp - 1;
        *p = r + kk >= m ? r + kk - m : r + kk;
        *q = r - kk < 0 ? r - kk + m : r - kk;
    }
    if (*p > *q) {
        const int t = *p;
        *p = *q;
        *q = t;
    }
}

// h padded to np (decoupled 3G on the padded diagonal), V = I, G per
// realization (max |eps| + 4 |tau|, 1 when that is 0)
__global__ __launch_bounds__(256) void k_bj_init(int L, int pbc, double tau, const double* eps, int np,
                                                 double* H, double* V, double* gmax) {
    __shared__ double red[4];
    const int b = blockIdx.y, n = L * L;
    const double* e = eps + (long)b * n;
    double g = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) g = fmax(g, fabs(e[i]));
    g = block_max(g, red) + 4.0 * fabs(tau);
    if (!(g > 0.0)) g = 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) gmax[b] = g;
    double* Hb = H + (long)b * np * np;
    double* Vb = V + (long)b * np * np;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (long)np * np;
         idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / np), j = (int)(idx % np);
        double v = 0.0;
        if (i >= n || j >= n) {
            v = i == j ? 3.0 * g : 0.0;
        } else if (i == j) {
            v = e[i];
        } else {
            int dx = j / L - i / L, dy = j % L - i % L;
            bool adj;
            if (pbc) {
                dx = (dx + L) % L;
                dy = (dy + L) % L;
                adj = ((dx == 1 || dx == L - 1) && dy == 0) || (dx == 0 && (dy == 1 || dy == L - 1));
            } else {
                adj = (abs(dx) == 1 && dy == 0) || (dx == 0 && abs(dy) == 1);
            }
            if (adj) v = -tau;
        }
        Hb[idx] = v;
        Vb[idx] = i == j ? 1.0 : 0.0;
    }
}

// global index of entry t (< 64) of pair (p, q)
__device__ inline int bj_index(int t, int p, int q) { return t < kBjB ? p * kBjB + t : q * kBjB + t - kBjB; }

// S = h[IJ, IJ] + 2G I for every pair of the round (pairs kk0 .. of the
// circle method), 64 x 64 row-major each
__global__ __launch_bounds__(256) void k_bj_gather(int np, int nbp, int round, int kk0, const double* H,
                                                   const double* gmax, double* S) {
    const int pi = blockIdx.x, npe = gridDim.x, b = blockIdx.y;
    int p, q;
    bj_pair(round, pi + kk0, nbp, &p, &q);
    const double* Hb = H + (long)b * np * np;
    double* Sb = S + ((long)b * npe + pi) * kBjW * kBjW;
    const double c = 2.0 * gmax[b];
    for (int e = threadIdx.x; e < kBjW * kBjW; e += blockDim.x) {
        const int i = e / kBjW, j = e % kBjW;
        Sb[e] = Hb[(long)bj_index(i, p, q) * np + bj_index(j, p, q)] + (i == j ? c : 0.0);
    }
}

// One 64 x 64 x 64 FP64 product per workgroup on v_mfma_f64_16x16x4f64,
// operands in LDS as unpadded 64 x 64 row-major tiles (64 KB for two):
// wave w computes rows 16 w .. 16 w + 15 of C = A B; result register r of
// lane l is row l / 16 + 4 r, column l % 16 of its 16 x 16 block.  An A
// tile read by rows (lane i of a 16-lane group takes row i, the group takes
// column k) stores element (i, j) at column j ^ 2 (i % 16); a tile read by
// columns (B, or A^T: a 16-lane group takes 16 consecutive columns of row
// k) stores it at column j ^ 16 (i % 2).  Either way the two 16-lane groups
// of a half-wave read 32 distinct bank pairs.
typedef double bj_d4 __attribute__((ext_vector_type(4)));
__device__ inline int bj_rsw(int i, int j) { return i * kBjW + (j ^ (2 * (i & 15))); }
__device__ inline int bj_csw(int i, int j) { return i * kBjW + (j ^ (16 * (i & 1))); }
template <bool TRANS_A>
__device__ inline void bj_mm(const double* As, const double* Bs, bj_d4 acc[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int f = 0; f < 4; ++f) acc[f] = bj_d4{0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < kBjW / 4; ++s) {
        const int k = 4 * s + kq;
        const double a = TRANS_A ? As[bj_csw(k, 16 * w + i)] : As[bj_rsw(16 * w + i, k)];
#pragma unroll
        for (int f = 0; f < 4; ++f)
            acc[f] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[bj_csw(k, 16 * f + i)], acc[f], 0, 0, 0);
    }
}

// columns IJ of h (z = 0) and of V (z = 1) times Q, one 64-row chunk
__global__ __launch_bounds__(256) void k_bj_cols(int np, int nbp, int round, int kk0, int npe, double* H,
                                                 double* V, const double* Q) {
    __shared__ double As[kBjW * kBjW], Qs[kBjW * kBjW];
    const int pi = blockIdx.x % npe, b = blockIdx.y;
    double* M = (blockIdx.z ? V : H) + (long)b * np * np;
    int p, q;
    bj_pair(round, pi + kk0, nbp, &p, &q);
    const double* Qb = Q + ((long)b * npe + pi) * kBjW * kBjW;
    const int row0 = (blockIdx.x / npe) * kBjW;
    // all loads in flight before the LDS stores (one wait, not one per element)
    constexpr int PER = kBjW * kBjW / 256;
    double va[PER], vq[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = threadIdx.x + 256 * t, i = e / kBjW, j = e % kBjW;
        va[t] = M[(long)(row0 + i) * np + bj_index(j, p, q)];
        vq[t] = Qb[e];
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = threadIdx.x + 256 * t, i = e / kBjW, j = e % kBjW;
        As[bj_rsw(i, j)] = va[t];
        Qs[bj_csw(i, j)] = vq[t];
    }
    __syncthreads();
    bj_d4 acc[4];
    bj_mm<false>(As, Qs, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + (lane >> 4) + 4 * r, j = 16 * f + (lane & 15);
            M[(long)(row0 + i) * np + bj_index(j, p, q)] = acc[f][r];
        }
}

// rows IJ of h: Q^T times them, one 64-column chunk
__global__ __launch_bounds__(256) void k_bj_rows(int np, int nbp, int round, int kk0, int npe, double* H,
                                                 const double* Q) {
    __shared__ double Bs[kBjW * kBjW], Qs[kBjW * kBjW];
    const int pi = blockIdx.x % npe, b = blockIdx.y;
    double* Hb = H + (long)b * np * np;
    int p, q;
    bj_pair(round, pi + kk0, nbp, &p, &q);
    const double* Qb = Q + ((long)b * npe + pi) * kBjW * kBjW;
    const int col0 = (blockIdx.x / npe) * kBjW;
    constexpr int PER = kBjW * kBjW / 256;
    double vb[PER], vq[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = threadIdx.x + 256 * t, i = e / kBjW, j = e % kBjW;
        vb[t] = Hb[(long)bj_index(i, p, q) * np + col0 + j];
        vq[t] = Qb[e];
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = threadIdx.x + 256 * t, i = e / kBjW, j = e % kBjW;
        Bs[bj_csw(i, j)] = vb[t];
        Qs[bj_csw(i, j)] = vq[t];
    }
    __syncthreads();
    bj_d4 acc[4];
    bj_mm<true>(Qs, Bs, acc);  // (Q^T)(i, k) = Q(k, i)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + (lane >> 4) + 4 * r, j = 16 * f + (lane & 15);
            Hb[(long)bj_index(i, p, q) * np + col0 + j] = acc[f][r];
        }
}

// off-diagonal over total squared Frobenius norm of h, per realization
__global__ __launch_bounds__(256) void k_bj_off(int np, const double* H, double* ratio) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const double* Hb = H + (long)b * np * np;
    double off = 0.0, tot = 0.0;
    for (long idx = threadIdx.x; idx < (long)np * np; idx += blockDim.x) {
        const double v = Hb[idx];
        tot += v * v;
        if (idx / np != idx % np) off += v * v;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (threadIdx.x == 0) ratio[b] = tot > 0.0 ? off / tot : 0.0;
}

// energies ascending (the diagonal of the converged h, the np - n padded
// entries 3G last and dropped), IPR of the matching columns of V, bins as
// k_ff_ipr; one realization per workgroup
constexpr int kBjMaxN = 1600;
__global__ __launch_bounds__(1024) void k_bj_ipr(int n, int np, const double* H, const double* V, double* E,
                                                 double* ipr, double* bin_ipr, int* bin_cnt) {
    __shared__ double d[kBjMaxN + kBjB], Es[kBjMaxN], Is[kBjMaxN];
    __shared__ int Bs[kBjMaxN];
    const int b = blockIdx.x;
    const double* Hb = H + (long)b * np * np;
    const double* Vb = V + (long)b * np * np;
    for (int k = threadIdx.x; k < np; k += blockDim.x) d[k] = Hb[(long)k * np + k];
    __syncthreads();
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
        const double dk = d[k];
        int rank = 0;
        for (int l = 0; l < np; ++l) rank += (d[l] < dk) || (d[l] == dk && l < k);
        if (rank < n) {
            double s4 = 0.0;
            for (int i = 0; i < n; ++i) {
                const double u = Vb[(long)i * np + k];
                s4 += (u * u) * (u * u);
            }
            Es[rank] = dk;
            Is[rank] = s4;
        }
    }
    __syncthreads();
    const double lo = Es[0], hi = Es[n - 1];
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        int bin = 0;
        if (hi > lo) {
            bin = (int)floor((Es[a] - lo) / (hi - lo) / 0.05);
            bin = bin < kIprBins - 1 ? bin : kIprBins - 1;
        }
        Bs[a] = bin;
        E[(long)b * n + a] = Es[a];
        ipr[(long)b * n + a] = Is[a];
    }
    __syncthreads();
    if (threadIdx.x < kIprBins) {
        double sum = 0.0;
        int cnt = 0;
        for (int a = 0; a < n; ++a)
            if (Bs[a] == (int)threadIdx.x) {
                sum += Is[a];
                ++cnt;
            }
        bin_ipr[(long)b * kIprBins + threadIdx.x] = sum;
        bin_cnt[(long)b * kIprBins + threadIdx.x] = cnt;
    }
}

// Enqueue the block Jacobi for n_real realizations on s; waits on the host
// once per sweep for the convergence test.  Returns IPEPS_OK, IPEPS_ENOMEM,
// IPEPS_ENOTCONV (60 sweeps) or IPEPS_EDEVICE.
int bj_spectrum_ipr(hipStream_t s, int L, int pbc, double tau, int n_real, const double* eps, double* energies,
                    double* ipr, double* bin_ipr, int* bin_count) {
    const int n = L * L;
    int nb = (n + kBjB - 1) / kBjB;
    nb += nb & 1;  // even: every block has a partner, and np is a multiple of 64
    const int np = nb * kBjB, nbp = nb, kk0 = 0, npe = nb / 2, nch = np / kBjW;
    const long nn = (long)np * np;
    const size_t doubles = 2 * (size_t)n_real * nn + 2 * (size_t)n_real * npe * kBjW * kBjW +
                           (size_t)n_real * npe * kBjW + 2 * (size_t)n_real;
    double* ws = nullptr;
    if (hipMallocAsync((void**)&ws, doubles * sizeof(double), s) != hipSuccess) {
        (void)hipGetLastError();
        return IPEPS_ENOMEM;
    }
    double* H = ws;
    double* V = H + (long)n_real * nn;
    double* S = V + (long)n_real * nn;
    double* Q = S + (long)n_real * npe * kBjW * kBjW;
    double* sig = Q + (long)n_real * npe * kBjW * kBjW;
    double* gmax = sig + (long)n_real * npe * kBjW;
    double* ratio = gmax + n_real;
    int rc = IPEPS_OK;
    std::vector<double> hr(n_real);
    try {
        const int gi = (int)std::min<long>(1024, (nn + 255) / 256);
        hipLaunchKernelGGL(k_bj_init, dim3(gi, n_real), dim3(256), 0, s, L, pbc, tau, eps, np, H, V, gmax);
        HIP_CHECK(hipGetLastError());
        bool conv = false;
        double prev = 1.0;
        for (int sweep = 0; sweep < 60 && !conv; ++sweep) {
            for (int round = 0; round < nbp - 1; ++round) {
                hipLaunchKernelGGL(k_bj_gather, dim3(npe, n_real), dim3(256), 0, s, np, nbp, round, kk0, H,
                                   gmax, S);
                jacobi_svd_real(s, n_real * npe, kBjW, kBjW, S, kBjW, (long)kBjW * kBjW, sig, nullptr, Q,
                                nullptr, 0.0);
                hipLaunchKernelGGL(k_bj_cols, dim3(nch * npe, n_real, 2), dim3(256), 0, s, np, nbp, round, kk0,
                                   npe, H, V, Q);
                hipLaunchKernelGGL(k_bj_rows, dim3(nch * npe, n_real), dim3(256), 0, s, np, nbp, round, kk0, npe,
                                   H, Q);
            }
            hipLaunchKernelGGL(k_bj_off, dim3(n_real), dim3(256), 0, s, np, H, ratio);
            HIP_CHECK(hipGetLastError());
            HIP_CHECK(hipMemcpyAsync(hr.data(), ratio, n_real * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            double worst = 0.0;
            bool nan = false;
            for (double v : hr) {
                nan = nan || std::isnan(v);
                worst = std::max(worst, v);
            }
            if (nan) break;  // NaN fields: the outputs carry them, IPEPS_ENOTCONV
            // converged: below 1e-24, or below 1e-18 and no longer shrinking
            // (the floor the 64 x 64 solves leave: they diagonalise S + 2G I
            // to 4 (2b) eps relative, i.e. leave entries ~1e-13 G of S)
            conv = worst < 1e-24 || (worst < 1e-18 && worst > 0.25 * prev);
            prev = worst;
        }
        if (!conv) rc = IPEPS_ENOTCONV;
        hipLaunchKernelGGL(k_bj_ipr, dim3(n_real), dim3(1024), 0, s, n, np, H, V, energies, ipr, bin_ipr,
                           bin_count);
        HIP_CHECK(hipGetLastError());
    } catch (...) {
        rc = IPEPS_EDEVICE;
    }
    if (hipFreeAsync(ws, s) != hipSuccess) rc = IPEPS_EDEVICE;
    return rc;
}
}  // namespace ipeps

extern "C" {

int ff_bessel_j(double x, int kmax, double* out) {
    if (!out || !(x >= 0.0) || !std::isfinite(x) || kmax < 0 || kmax > 200) return IPEPS_EINVAL;
    ipeps::bessel_j_seq(x, kmax, out);
    return IPEPS_OK;
}

}  // extern "C"

namespace ipeps {
namespace {

int neel_check(int L, int pbc, double tau, double dt, int n_times, int n_real) {
    if (L < 1 || L * L > 2048 || (pbc != 0 && pbc != 1) || (pbc && L < 3)) return IPEPS_EINVAL;
    if (!std::isfinite(tau) || !(dt > 0.0) || !std::isfinite(dt)) return IPEPS_EINVAL;
    if (n_times < 0 || n_real < 0 || n_real > 65535) return IPEPS_EINVAL;
    return IPEPS_OK;
}

// The dynamics kernel and the fixed-order sum into n_even / n_odd, with the
// per-orbital partial weights in ws (2 * n_real * n_times * ceil(L^2/2)
// doubles, each written once before it is read: nothing needs clearing).
hipError_t neel_enqueue(hipStream_t s, int L, int pbc, double tau, double dt, int n_times, int n_real,
                        const double* eps, double* n_even, double* n_odd, double* ws) {
    const int nsite = L * L, M = (nsite + 1) / 2, Mo = nsite - M;
    const long nq = (long)n_real * n_times;
    double* pe = ws;
    double* po = ws + nq * M;
    const int S = (nsite + kFfThreads - 1) / kFfThreads;
    hipError_t e;
    if (S <= 1) e = launch_ff<1>(s, L, pbc, tau, dt, n_times, n_real, eps, M, pe, po);
    else if (S <= 2) e = launch_ff<2>(s, L, pbc, tau, dt, n_times, n_real, eps, M, pe, po);
    else if (S <= 4) e = launch_ff<4>(s, L, pbc, tau, dt, n_times, n_real, eps, M, pe, po);
    else if (S <= 7) e = launch_ff<7>(s, L, pbc, tau, dt, n_times, n_real, eps, M, pe, po);
    else e = launch_ff<8>(s, L, pbc, tau, dt, n_times, n_real, eps, M, pe, po);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_ff_sum, dim3((unsigned)nq), dim3(256), 0, s, M, pe, po, 1.0 / M,
                           Mo > 0 ? 1.0 / Mo : 0.0, n_even, n_odd);
        e = hipGetLastError();
    }
    return e;
}

// Scratch of ff_neel_dynamics_noalloc: one copy per device, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device with that device current.
constexpr long kNeelScratchDoubles = FF_NOALLOC_SCRATCH_DOUBLES;
__device__ __align__(256) double scratch[kNeelScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (nullptr and a message on failure).
double* scratch_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fprintf(stderr, "ff_neel_dynamics_noalloc: hipGetSymbolAddress failed on device %d: %s\n", dev,
                    hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = (double*)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace ipeps

extern "C" {

int ff_neel_dynamics(int L, int pbc, double tau, double dt, int n_times, int n_real, const double* eps,
                     double* n_even, double* n_odd, void* hip_stream) {
    using namespace ipeps;
    const int rc = neel_check(L, pbc, tau, dt, n_times, n_real);
    if (rc != IPEPS_OK) return rc;
    if (n_times == 0 || n_real == 0) return IPEPS_OK;
    if (!eps || !n_even || !n_odd) return IPEPS_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const long nq = (long)n_real * n_times, M = (L * L + 1) / 2;
    double* ws = nullptr;
    if (hipMallocAsync((void**)&ws, (size_t)2 * nq * M * sizeof(double), s) != hipSuccess) {
        (void)hipGetLastError();
        return IPEPS_ENOMEM;
    }
    const hipError_t e = neel_enqueue(s, L, pbc, tau, dt, n_times, n_real, eps, n_even, n_odd, ws);
    const hipError_t f = hipFreeAsync(ws, s);
    if (e != hipSuccess || f != hipSuccess) {
        fprintf(stderr, "ff_neel_dynamics: %s\n", hipGetErrorString(e != hipSuccess ? e : f));
        return IPEPS_EDEVICE;
    }
    return IPEPS_OK;
}

int ff_neel_dynamics_noalloc(int L, int pbc, double tau, double dt, int n_times, int n_real,
                             const double* eps, double* n_even, double* n_odd, void* hip_stream) {
    using namespace ipeps;
    const int rc = neel_check(L, pbc, tau, dt, n_times, n_real);
    if (rc != IPEPS_OK) return rc;
    if (n_times == 0 || n_real == 0) return IPEPS_OK;
    if (!eps || !n_even || !n_odd) return IPEPS_EINVAL;
    const long need = 2L * n_real * n_times * ((L * L + 1) / 2);
    if (need > kNeelScratchDoubles) {
        fprintf(stderr,
                "ff_neel_dynamics_noalloc: 2 * n_real * n_times * ceil(L^2/2) = %ld doubles exceeds the "
                "fixed scratch of %ld doubles\n",
                need, kNeelScratchDoubles);
        return IPEPS_ETOOBIG;
    }
    double* ws = scratch_for_current_device();
    if (!ws) return IPEPS_EDEVICE;
    const hipError_t e =
        neel_enqueue((hipStream_t)hip_stream, L, pbc, tau, dt, n_times, n_real, eps, n_even, n_odd, ws);
    if (e != hipSuccess) {
        fprintf(stderr, "ff_neel_dynamics_noalloc: %s\n", hipGetErrorString(e));
        return IPEPS_EDEVICE;
    }
    return IPEPS_OK;
}

int ff_spectrum_ipr(int L, int pbc, double tau, int n_real, const double* eps, double* energies,
                    double* ipr, double* bin_ipr, int* bin_count, void* hip_stream) {
    using namespace ipeps;
    if (L < 1 || L > 40 || (pbc != 0 && pbc != 1) || (pbc && L < 3)) return IPEPS_EINVAL;
    if (!std::isfinite(tau) || n_real < 0 || n_real > 65535) return IPEPS_EINVAL;
    if (n_real == 0) return IPEPS_OK;
    if (!eps || !energies || !ipr || !bin_ipr || !bin_count) return IPEPS_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (L > 16) {
        const int rc = bj_spectrum_ipr(s, L, pbc, tau, n_real, eps, energies, ipr, bin_ipr, bin_count);
        if (rc == IPEPS_EDEVICE) fprintf(stderr, "ff_spectrum_ipr: HIP error in the block Jacobi\n");
        return rc;
    }
    const int n = L * L;
    const long nn = (long)n_real * n * n;
    const size_t jw = jacobi_svd_real_work(n_real, n, n);
    const size_t doubles = 2 * (size_t)nn + (size_t)n_real * n + (size_t)n_real + (jw > 0 ? jw : 1);
    double* ws = nullptr;
    if (hipMallocAsync((void**)&ws, doubles * sizeof(double), s) != hipSuccess) {
        (void)hipGetLastError();
        return IPEPS_ENOMEM;
    }
    double* H = ws;
    double* Uv = H + nn;
    double* sig = Uv + nn;
    double* shift = sig + (long)n_real * n;
    double* work = shift + n_real;
    hipError_t e = hipSuccess;
    try {
        hipLaunchKernelGGL(k_ff_shifted_h, dim3(n_real), dim3(256), 0, s, L, pbc, tau, eps, H, shift);
        e = hipGetLastError();
        if (e == hipSuccess) {
            // left singular vectors only (normalised columns): eigenvectors
            jacobi_svd_real(s, n_real, n, n, H, n, (long)n * n, sig, Uv, nullptr, work, 0.0);
            hipLaunchKernelGGL(k_ff_ipr, dim3(n_real), dim3(256), 0, s, n, sig, Uv, shift, energies, ipr,
                               bin_ipr, bin_count);
            e = hipGetLastError();
        }
    } catch (...) {
        e = hipErrorUnknown;
    }
    const hipError_t f = hipFreeAsync(ws, s);
    if (e != hipSuccess || f != hipSuccess) {
        fprintf(stderr, "ff_spectrum_ipr: %s\n", hipGetErrorString(e != hipSuccess ? e : f));
        return IPEPS_EDEVICE;
    }
    return IPEPS_OK;
}

}  // extern "C"
