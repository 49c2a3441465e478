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
__device__ void jacobi_sweeps(int m, int n, double* Ac, double* Vc, int* flag) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int ne = n + (n & 1);
    const int npair = ne / 2;
    const double tol = fmax(1e-15, sqrt((double)m) * 2.3e-16);
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int r = 0; r < ne - 1; ++r) {
            for (int k = wave; k < npair; k += nw) {
                int p, q;
                circle_pair(r, k, ne, &p, &q);
                if (q >= n) continue;
                double* ap = Ac + (long)p * m;
                double* aq = Ac + (long)q * m;
                double al = 0, be = 0, ga = 0;
                for (int i = lane; i < m; i += 64) {
                    const double x = ap[i], y = aq[i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (al == 0.0 || be == 0.0) continue;
                if (fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = lane; i < m; i += 64) {
                    const double x = ap[i], y = aq[i];
                    ap[i] = c * x - s * y;
                    aq[i] = s * x + c * y;
                }
                if (Vc) {
                    double* vp = Vc + (long)p * n;
                    double* vq = Vc + (long)q * n;
                    for (int i = lane; i < n; i += 64) {
                        const double x = vp[i], y = vq[i];
                        vp[i] = c * x - s * y;
                        vq[i] = s * x + c * y;
                    }
                }
                if (lane == 0) *flag = 1;
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
    jacobi_sweeps(m, n, Ac, wantV ? Vc : nullptr, &flag);
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
// G = R^T R (R upper) with dropping, then Rinv = R^{-1}.  G and Rinv are
// row-major k x k.  One workgroup of 256 threads per matrix; R lives in LDS
// (k <= 128), the inverse is written straight to global memory.
__global__ __launch_bounds__(256) void k_chol_inverse(int k, const double* __restrict__ G,
                                                      double* __restrict__ Rinv, double tol) {
    extern __shared__ double R[];  // k*k, row-major, upper part used
    __shared__ double piv;
    __shared__ int dead_s[256];
    const int b = blockIdx.x;
    const double* Gb = G + (long)b * k * k;
    double* Xb = Rinv + (long)b * k * k;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) R[e] = Gb[e];
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (threadIdx.x == 0) {
            // diagonal of a column-normalised Gram matrix is ~1; the original
            // diagonal is not kept, so the threshold is taken relative to 1
            // when the caller normalised the columns (tol * max(G_jj_orig,...))
            const double d = R[j * k + j];
            const int dead = !(d > tol);
            dead_s[j] = dead;
            piv = dead ? 0.0 : sqrt(d);
        }
        __syncthreads();
        const double pj = piv;
        for (int c = j + threadIdx.x; c < k; c += blockDim.x)
            R[j * k + c] = (pj > 0.0) ? R[j * k + c] / pj : 0.0;
        __syncthreads();
        // trailing update of the upper triangle: R[a][c] -= R[j][a] R[j][c]
        const int rem = k - j - 1;
        for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
            const int a = j + 1 + e / rem, c = j + 1 + e % rem;
            if (c >= a) R[a * k + c] -= R[j * k + a] * R[j * k + c];
        }
        __syncthreads();
    }
    // back substitution, one column of the inverse per thread
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        for (int i = k - 1; i >= 0; --i) {
            double v;
            if (i > c || dead_s[i]) {
                v = 0.0;
            } else {
                double s = (i == c) ? 1.0 : 0.0;
                for (int l = i + 1; l <= c; ++l) s -= R[i * k + l] * Xb[(long)l * k + c];
                v = s / R[i * k + i];
            }
            Xb[(long)i * k + c] = v;
        }
    }
}

void chol_inverse(hipStream_t s, int batch, int k, const double* G, double* Rinv, double tol) {
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
    hipLaunchKernelGGL(k_chol_inverse, dim3(batch), dim3(256), lds, s, k, G, Rinv, tol);
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

}  // namespace ipeps
