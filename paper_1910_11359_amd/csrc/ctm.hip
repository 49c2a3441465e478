// CTMRG support kernels (double layer, layouts, environment init, permutes,
// norms, projector factors, spectra, readout).
#include "ctm.h"

#include <cmath>

namespace ipeps {

__device__ inline int site_idx(int x, int y) { return ((x % 2 + 2) % 2) + 2 * ((y % 2 + 2) % 2); }

// ------------------------------------------------------------ A = Gamma sqrt(lambda)
__global__ void k_absorb(int D, int d, const cplx* __restrict__ gam, const double* __restrict__ lam,
                         cplx* __restrict__ A) {
    const int site = blockIdx.y;
    const int x = site % 2, y = site / 2;
    const long D4 = (long)D * D * D * D, sz = d * D4;
    const double* lu = lam + (4 + site_idx(x, y - 1)) * D;
    const double* ll = lam + site_idx(x - 1, y) * D;
    const double* ld = lam + (4 + site_idx(x, y)) * D;
    const double* lr = lam + site_idx(x, y) * D;
    for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < sz; e += (long)gridDim.x * blockDim.x) {
        const int r = e % D, dd = (e / D) % D, l = (e / (D * D)) % D, u = (e / (D * D * D)) % D;
        const double w = sqrt(lu[u] * ll[l] * ld[dd] * lr[r]);
        A[site * sz + e] = cscale(gam[site * sz + e], w);
    }
}

void absorb_sqrt_lambda(hipStream_t s, int D, int d, const cplx* gam, const double* lam, cplx* A) {
    const long sz = (long)d * D * D * D * D;
    hipLaunchKernelGGL(k_absorb, dim3(ceil_div(sz, 256), 4), dim3(256), 0, s, D, d, gam, lam, A);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ Hermitian basis
// Forward terms of one leg: a_H[m] = sum_t c_t a[(x_t, y_t)] for the basis of
// pair m = (k, k'); H^T legs read a at (y_t, x_t).
struct LegTerms {
    int n;
    int x[2], y[2];
    cplx c[2];
};
__device__ inline LegTerms fwd_terms(int m, int D, bool transposed) {
    const int k = m / D, kp = m % D;
    const double h = 0.70710678118654752440;
    LegTerms t;
    t.x[1] = t.y[1] = 0;
    t.c[1] = cmake(0, 0);
    if (k == kp) {
        t.n = 1;
        t.x[0] = k;
        t.y[0] = k;
        t.c[0] = cmake(1, 0);
    } else {
        t.n = 2;
        t.x[0] = k;
        t.y[0] = kp;
        t.x[1] = kp;
        t.y[1] = k;
        if (k < kp) {
            t.c[0] = cmake(h, 0);
            t.c[1] = cmake(h, 0);
        } else {
            t.c[0] = cmake(0, h);
            t.c[1] = cmake(0, -h);
        }
    }
    if (transposed) {  // constant indices: the terms stay in registers
        const int x0 = t.x[0], x1 = t.x[1];
        t.x[0] = t.y[0];
        t.x[1] = t.y[1];
        t.y[0] = x0;
        t.y[1] = x1;
    }
    return t;
}
// Term i (0 or 1) of a leg, read with constant indices (a run-time index into
// the term arrays would put them in scratch memory).
__device__ inline int term_x(const LegTerms& t, int i) { return i ? t.x[1] : t.x[0]; }
__device__ inline int term_y(const LegTerms& t, int i) { return i ? t.y[1] : t.y[0]; }
__device__ inline cplx term_c(const LegTerms& t, int i) { return i ? t.c[1] : t.c[0]; }

// Inverse terms: E_c[(k, k')] = sum_t c_t E_H[m_t] (H legs); H^T legs use the
// pair (k', k).
struct InvTerms {
    int n;
    int m[2];
    cplx c[2];
};
__device__ inline InvTerms inv_terms(int k, int kp, int D, bool transposed) {
    if (transposed) {
        int t = k;
        k = kp;
        kp = t;
    }
    const double h = 0.70710678118654752440;
    InvTerms t;
    t.m[1] = 0;
    t.c[1] = cmake(0, 0);
    if (k == kp) {
        t.n = 1;
        t.m[0] = k * D + k;
        t.c[0] = cmake(1, 0);
    } else if (k < kp) {
        t.n = 2;
        t.m[0] = k * D + kp;  // symmetric element
        t.c[0] = cmake(h, 0);
        t.m[1] = kp * D + k;  // antisymmetric element, H[k][k'] = -i/sqrt2
        t.c[1] = cmake(0, -h);
    } else {
        t.n = 2;
        t.m[0] = kp * D + k;
        t.c[0] = cmake(h, 0);
        t.m[1] = k * D + kp;  // H[k][k'] = +i/sqrt2
        t.c[1] = cmake(0, h);
    }
    return t;
}

// Double layer in the real basis: a[mu][ml][md][mr] = Re sum over the leg
// terms (at most two per leg) of c_u c_l c_d c_r sum_p A_p[x] conj(A_p[y]),
// x = (xu, xl, xd, xr) the ket and y the bra indices of the terms.  One
// workgroup per (site, mu, ml): the A_p[xu][xl][.][.] and A_p[yu][yl][.][.]
// slices of its (at most four) up/left term pairs go to LDS, then
// W[kx][ky] = sum over those pairs of c_u c_l sum_p A_p[xu xl kx]
// conj(A_p[yu yl ky]) (kx, ky the down/right index pairs), and each output
// is Re sum over its down/right terms of c_d c_r W[kx][ky].
__global__ __launch_bounds__(256) void k_double_layer(int D, int d, const cplx* __restrict__ A,
                                                      double* __restrict__ a) {
    extern __shared__ cplx sl[];  // [ket, bra][pair < 4][p < d][D^2], then W[D^2][D^2]
    const int site = blockIdx.y, mul = blockIdx.x;
    const int q = D * D;
    const long q4 = (long)q * q * q * q;
    const long D4 = (long)q * q;
    const int mu = mul / q, ml = mul - (mul / q) * q;
    const cplx* As = A + (long)site * d * D4;
    const LegTerms tu = fwd_terms(mu, D, false), tl = fwd_terms(ml, D, false);
    const int npair = tu.n * tl.n;
    const int slab = d * q;  // one slice: d x D^2
    for (int e = threadIdx.x; e < 2 * npair * slab; e += blockDim.x) {
        const int side = e / (npair * slab), rem = e - side * (npair * slab);
        const int pr = rem / slab, rem2 = rem - pr * slab;
        const int pp = rem2 / q, dr = rem2 - pp * q;
        const int iu = pr / tl.n, il = pr - (pr / tl.n) * tl.n;
        const int u = side ? term_y(tu, iu) : term_x(tu, iu), l = side ? term_y(tl, il) : term_x(tl, il);
        sl[e] = As[(long)pp * D4 + ((long)u * D + l) * q + dr];
    }
    __syncthreads();
    const cplx* kx_s = sl;
    const cplx* ky_s = sl + npair * slab;
    cplx* W = sl + 2 * 4 * slab;
    for (int e = threadIdx.x; e < q * q; e += blockDim.x) {
        const int kx = e / q, ky = e - (e / q) * q;
        cplx w = cmake(0, 0);
        for (int pr = 0; pr < npair; ++pr) {
            const int iu = pr / tl.n, il = pr - (pr / tl.n) * tl.n;
            cplx sum = cmake(0, 0);
            for (int p = 0; p < d; ++p)
                sum = cadd(sum, cmul(kx_s[(pr * d + p) * q + kx], cconj(ky_s[(pr * d + p) * q + ky])));
            w = cadd(w, cmul(cmul(term_c(tu, iu), term_c(tl, il)), sum));
        }
        W[e] = w;
    }
    __syncthreads();
    double* out = a + (long)site * q4 + (long)mul * q * q;
    for (int o = threadIdx.x; o < q * q; o += blockDim.x) {
        const int md = o / q, mr = o - (o / q) * q;
        const LegTerms td = fwd_terms(md, D, true), tr = fwd_terms(mr, D, true);
        double acc = 0.0;
#pragma unroll
        for (int id = 0; id < 2; ++id)
#pragma unroll
            for (int ir = 0; ir < 2; ++ir)
                if (id < td.n && ir < tr.n) {
                    const int kx = td.x[id] * D + tr.x[ir], ky = td.y[id] * D + tr.y[ir];
                    acc += cmul(cmul(td.c[id], tr.c[ir]), W[kx * q + ky]).re;
                }
        out[o] = acc;
    }
}

void double_layer_real(hipStream_t s, int D, int d, const cplx* A, double* a_base) {
    const long q = (long)D * D;
    const size_t lds = (2 * 4 * (size_t)d * q + (size_t)q * q) * sizeof(cplx);
    static bool attr_set = false;
    if (!attr_set) {
        HIP_CHECK(hipFuncSetAttribute((const void*)k_double_layer, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      160 * 1024 - 1024));
        attr_set = true;
    }
    IPEPS_REQUIRE(lds <= 160 * 1024 - 1024, IPEPS_EINVAL, "double layer: d D^2 too large for LDS");
    hipLaunchKernelGGL(k_double_layer, dim3(q * q, 4), dim3(256), lds, s, D, d, A, a_base);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ frame layouts
// Each site's double layer a[u][l][d][r] (FP64) in the leg orders the
// contractions read, for the 4 frame rotations g (frame leg F sits at source
// position (F - g) mod 4): kind 0 as [L][U][D][R], kind 1 as [D][L][R][U].
// One workgroup per output and pair of its outer legs: the output's fastest
// leg and the leg that is fastest in the source form a q x q tile, read along
// the source's fastest leg and written along the output's through LDS (one
// pass, no tile, when the two coincide).
template <typename T>
__global__ __launch_bounds__(256) void k_frame_layouts(int q, const double* __restrict__ a_base, T* const* out_lu,
                                                       T* const* out_dl) {
    extern __shared__ double tile[];  // q x (q + 1)
    const int which = blockIdx.y;     // site*8 + g*2 + kind
    const int site = which / 8, g = (which / 2) % 4, kind = which % 2;
    T* __restrict__ out = kind == 0 ? out_lu[site * 4 + g] : out_dl[site * 4 + g];
    const long q2 = (long)q * q, q3 = q2 * q;
    const double* __restrict__ a = a_base + site * q3 * q;
    // frame leg (U 0, L 1, D 2, R 3) at output positions 0..3, and the source
    // stride of each output position
    const int F0 = kind == 0 ? 1 : 2, F1 = kind == 0 ? 0 : 1, F2 = kind == 0 ? 2 : 3, F3 = kind == 0 ? 3 : 0;
    auto sstride = [&](int F) {
        const int pos = (F - g + 4) & 3;
        return pos == 3 ? 1L : pos == 2 ? (long)q : pos == 1 ? q2 : q3;
    };
    const long s0 = sstride(F0), s1 = sstride(F1), s2 = sstride(F2), s3 = sstride(F3);
    // ob: the output position fastest in the source (3: no transpose)
    const int ob = s3 == 1 ? 3 : s0 == 1 ? 0 : s1 == 1 ? 1 : 2;
    // outer output positions x < y: the two not in {3, ob} ({0, 1} when ob = 3)
    const int x = ob == 0 ? 1 : 0, y = ob == 2 || ob == 3 ? 1 : 2;
    const long sx = x == 0 ? s0 : s1, sy = y == 1 ? s1 : s2;
    const long ox = x == 0 ? q3 : q2, oy = y == 1 ? q2 : (long)q;
    const int ix = blockIdx.x / q, iy = blockIdx.x - (blockIdx.x / q) * q;
    const double* __restrict__ src = a + ix * sx + iy * sy;
    T* __restrict__ dst = out + ix * ox + iy * oy;
    const int n = q * q;
    if (ob == 3) {
        // i3 fastest on both sides; the other tile leg is output position 2
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int i3 = e % q, i2 = e / q;
            dst[(long)i2 * q + i3] = (T)src[i2 * s2 + i3];
        }
        return;
    }
    const long ob_out = ob == 0 ? q3 : ob == 1 ? q2 : (long)q;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int b = e % q, i3 = e / q;  // b: the index of output position ob
        tile[i3 * (q + 1) + b] = src[i3 * s3 + b];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int i3 = e % q, b = e / q;
        dst[b * ob_out + i3] = (T)tile[i3 * (q + 1) + b];
    }
}

void frame_layouts(hipStream_t s, int q, int dtype, const double* a_base, void* const* out_lu,
                   void* const* out_dl) {
    IPEPS_REQUIRE(q >= 1 && q <= 64, IPEPS_EINVAL, "frame layouts: q must be in 1..64");
    const dim3 grid(q * q, 32);
    const size_t lds = (size_t)q * (q + 1) * sizeof(double);
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_frame_layouts<double>, grid, dim3(256), lds, s, q, a_base,
                           (double* const*)out_lu, (double* const*)out_dl);
    else
        hipLaunchKernelGGL(k_frame_layouts<float>, grid, dim3(256), lds, s, q, a_base,
                           (float* const*)out_lu, (float* const*)out_dl);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ cold environment
template <typename T>
__global__ void k_init_env(int D, int chi, const double* __restrict__ a_base, T* C, T* T_) {
    const int site = blockIdx.y / 8, which = blockIdx.y % 8;  // 0..3 corners, 4..7 edges
    const int x = site % 2, y = site / 2;
    const int q = D * D;
    const long q2 = (long)q * q, q3 = q2 * q, q4 = q3 * q;
    auto A = [&](int xx, int yy) { return a_base + site_idx(xx, yy) * q4; };
    if (which < 4) {
        const int k = which;
        T* out = C + (long)(site * 4 + k) * chi * chi;
        for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < (long)chi * chi;
             e += (long)gridDim.x * blockDim.x) {
            const int i = e / chi, j = e % chi;
            double v = 0.0;
            if (i < q && j < q) {
                for (int t1 = 0; t1 < D; ++t1)
                    for (int t2 = 0; t2 < D; ++t2) {
                        const int m1 = t1 * (D + 1), m2 = t2 * (D + 1);
                        if (k == 0) v += A(x - 1, y - 1)[m1 * q3 + m2 * q2 + i * q + j];       // tr u,l -> [d][r]
                        else if (k == 1) v += A(x + 1, y - 1)[m1 * q3 + i * q2 + j * q + m2];  // tr u,r -> [l][d]
                        else if (k == 2) v += A(x + 1, y + 1)[i * q3 + j * q2 + m1 * q + m2];  // tr d,r -> [u][l]
                        else v += A(x - 1, y + 1)[j * q3 + m1 * q2 + m2 * q + i];              // tr l,d -> [r][u]
                    }
            }
            out[e] = (T)v;
        }
    } else {
        const int k = which - 4;
        T* out = T_ + (long)(site * 4 + k) * chi * q * chi;
        for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < (long)chi * q * chi;
             e += (long)gridDim.x * blockDim.x) {
            const int i = e / ((long)q * chi), mq = (e / chi) % q, j = e % chi;
            double v = 0.0;
            if (i < q && j < q) {
                for (int t1 = 0; t1 < D; ++t1) {
                    const int m1 = t1 * (D + 1);
                    if (k == 0) v += A(x, y - 1)[m1 * q3 + i * q2 + mq * q + j];       // tr u -> [l][d][r]
                    else if (k == 1) v += A(x + 1, y)[i * q3 + mq * q2 + j * q + m1];  // tr r -> [u][l][d]
                    else if (k == 2) v += A(x, y + 1)[mq * q3 + j * q2 + m1 * q + i];  // tr d -> [r][u][l]
                    else v += A(x - 1, y)[j * q3 + m1 * q2 + i * q + mq];              // tr l -> [d][r][u]
                }
            }
            out[e] = (T)v;
        }
    }
}

void init_environment(hipStream_t s, int D, int chi, int dtype, const double* a_base, void* C,
                      void* T) {
    const long big = (long)chi * D * D * chi;
    dim3 grid(ceil_div(big, 256) < 2048 ? ceil_div(big, 256) : 2048, 32);
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_init_env<double>, grid, dim3(256), 0, s, D, chi, a_base, (double*)C,
                           (double*)T);
    else
        hipLaunchKernelGGL(k_init_env<float>, grid, dim3(256), 0, s, D, chi, a_base, (float*)C,
                           (float*)T);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ permutations
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(int R, int Cc, const T* __restrict__ in,
                                                   T* __restrict__ out) {
    __shared__ T tile[32][33];
    const long b = blockIdx.z;
    const T* ib = in + b * (long)R * Cc;
    T* ob = out + b * (long)R * Cc;
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + tx;
        if (r < R && c < Cc) tile[k][tx] = ib[(long)r * Cc + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + tx;
        if (r < R && c < Cc) ob[(long)c * R + r] = tile[tx][k];
    }
}

void batched_transpose(hipStream_t s, int dtype, int batch, int R, int Cc, const void* in,
                       void* out) {
    dim3 grid(ceil_div(Cc, 32), ceil_div(R, 32), batch);
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, s, R, Cc, (const double*)in,
                           (double*)out);
    else
        hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, s, R, Cc, (const float*)in,
                           (float*)out);
    HIP_CHECK(hipGetLastError());
}

template <typename T>
__global__ void k_permute3(int mode, int A, int B, int C, const T* __restrict__ in, T* __restrict__ out,
                           JobMap jm) {
    in = jptr(in, jm, blockIdx.y);
    out = jptr(out, jm, blockIdx.y);
    const long tot = (long)A * B * C;
    for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int c = e % C, b = (e / C) % B, a = e / ((long)B * C);
        long o;
        if (mode == 0) o = ((long)b * A + a) * C + c;
        else if (mode == 1) o = ((long)a * C + c) * B + b;
        else o = ((long)c * A + a) * B + b;
        out[o] = in[e];
    }
}

void permute3(hipStream_t s, int dtype, int mode, int A, int B, int C, const void* in, void* out,
              JobMap jm) {
    const long tot = (long)A * B * C;
    const int grid = ceil_div(tot, 256) < 4096 ? ceil_div(tot, 256) : 4096;
    jm.per_job = 1;
    const dim3 g(grid, jm.delta ? jm.njobs : 1);
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_permute3<double>, g, dim3(256), 0, s, mode, A, B, C,
                           (const double*)in, (double*)out, jm);
    else
        hipLaunchKernelGGL(k_permute3<float>, g, dim3(256), 0, s, mode, A, B, C,
                           (const float*)in, (float*)out, jm);
    HIP_CHECK(hipGetLastError());
}

// Up to kPermuteBatch independent permute3 copies in one launch (blockIdx.z
// selects the copy; grid x sized for the largest).
template <typename T>
__global__ void k_permute3_batch(Permute3Batch pb, JobMap jm) {
    const int z = blockIdx.z;
    const int mode = pb.mode[z], A = pb.A[z], B = pb.B[z], C = pb.C[z];
    const T* __restrict__ in = jptr((const T*)pb.in[z], jm, blockIdx.y);
    T* __restrict__ out = jptr((T*)pb.out[z], jm, blockIdx.y);
    const long tot = (long)A * B * C;
    for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int c = e % C, b = (e / C) % B, a = e / ((long)B * C);
        long o;
        if (mode == 0) o = ((long)b * A + a) * C + c;
        else if (mode == 1) o = ((long)a * C + c) * B + b;
        else o = ((long)c * A + a) * B + b;
        out[o] = in[e];
    }
}

void permute3_batch(hipStream_t s, int dtype, const Permute3Batch& pb, JobMap jm) {
    IPEPS_REQUIRE(pb.n >= 1 && pb.n <= kPermuteBatch, IPEPS_EINVAL, "permute3_batch: 1..6 copies");
    long tot = 0;
    for (int i = 0; i < pb.n; ++i) tot = std::max(tot, (long)pb.A[i] * pb.B[i] * pb.C[i]);
    const int grid = ceil_div(tot, 256) < 4096 ? ceil_div(tot, 256) : 4096;
    jm.per_job = 1;
    const dim3 g(grid, jm.delta ? jm.njobs : 1, pb.n);
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_permute3_batch<double>, g, dim3(256), 0, s, pb, jm);
    else
        hipLaunchKernelGGL(k_permute3_batch<float>, g, dim3(256), 0, s, pb, jm);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ norms / conversion
// Deterministic two-pass Frobenius normalisation: kNormBlocks blocks per
// tensor write partial sums of squares (FP64) in a fixed partition, then every
// block of the tensor adds the partials in the same order and scales its slice.
constexpr int kNormBlocks = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_norm_partial(const NormItem* items, double* ws) {
    __shared__ double red[4];
    const NormItem it = items[blockIdx.y];
    const T* p = (const T*)it.ptr;
    double s = 0.0;
    for (long e = blockIdx.x * 256L + threadIdx.x; e < it.count; e += 256L * kNormBlocks) {
        const double v = (double)p[e];
        s += v * v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) ws[blockIdx.y * kNormBlocks + blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_norm_scale(const NormItem* items, const double* ws) {
    const NormItem it = items[blockIdx.y];
    T* p = (T*)it.ptr;
    double s = 0.0;
    for (int b = 0; b < kNormBlocks; ++b) s += ws[blockIdx.y * kNormBlocks + b];
    const double inv = s > 0 ? 1.0 / sqrt(s) : 0.0;
    for (long e = blockIdx.x * 256L + threadIdx.x; e < it.count; e += 256L * kNormBlocks)
        p[e] = (T)((double)p[e] * inv);
}

size_t normalize_ws_doubles(int max_items) { return (size_t)max_items * kNormBlocks; }

void normalize_tensors(hipStream_t s, int dtype, const NormItem* d_items, int n, double* ws) {
    if (n <= 0) return;
    const dim3 grid(kNormBlocks, n);
    if (dtype == IPEPS_DTYPE_FP64) {
        hipLaunchKernelGGL(k_norm_partial<double>, grid, dim3(256), 0, s, d_items, ws);
        hipLaunchKernelGGL(k_norm_scale<double>, grid, dim3(256), 0, s, d_items, ws);
    } else {
        hipLaunchKernelGGL(k_norm_partial<float>, grid, dim3(256), 0, s, d_items, ws);
        hipLaunchKernelGGL(k_norm_scale<float>, grid, dim3(256), 0, s, d_items, ws);
    }
    HIP_CHECK(hipGetLastError());
}

template <typename T>
__global__ void k_to64(const T* in, double* out, double* out2, long n, JobMap jm) {
    in = jptr(in, jm, blockIdx.y);
    out = jptr(out, jm, blockIdx.y);
    if (out2) {
        out2 = jptr(out2, jm, blockIdx.y);
        for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
            const double v = (double)in[e];
            out[e] = v;
            out2[e] = v;
        }
        return;
    }
    for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = (double)in[e];
}
template <typename T>
__global__ void k_from64(const double* in, T* out, long n) {
    for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = (T)in[e];
}

void to_fp64(hipStream_t s, int dtype, const void* in, double* out, long count, JobMap jm, double* out2) {
    const int grid = ceil_div(count, 256) < 8192 ? ceil_div(count, 256) : 8192;
    if (count <= 0) return;
    jm.per_job = 1;
    const dim3 g(grid, jm.delta ? jm.njobs : 1);
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_to64<double>, g, dim3(256), 0, s, (const double*)in, out, out2, count, jm);
    else
        hipLaunchKernelGGL(k_to64<float>, g, dim3(256), 0, s, (const float*)in, out, out2, count, jm);
    HIP_CHECK(hipGetLastError());
}

void from_fp64(hipStream_t s, int dtype, const double* in, void* out, long count) {
    const int grid = ceil_div(count, 256) < 8192 ? ceil_div(count, 256) : 8192;
    if (count <= 0) return;
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_from64<double>, dim3(grid), dim3(256), 0, s, in, (double*)out, count);
    else
        hipLaunchKernelGGL(k_from64<float>, dim3(grid), dim3(256), 0, s, in, (float*)out, count);
    HIP_CHECK(hipGetLastError());
}

// 32 x 32 tiles through LDS: reads along the rows of the input, writes along
// the rows of the output in both orientations.
template <typename T, bool TRANS>
__global__ __launch_bounds__(256) void k_from64_blocks(const double* __restrict__ in,
                                                       T* __restrict__ out, int rows, int cols,
                                                       JobMap jm) {
    __shared__ double tile[32][33];
    const long bs = (long)rows * cols;
    in = jptr(in, jm, blockIdx.z) + jlocal(jm, blockIdx.z) * bs;
    out = jptr(out, jm, blockIdx.z) + jlocal(jm, blockIdx.z) * bs;
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = in[(long)r * cols + c];
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        if (TRANS) {
            const int c = c0 + i, r = r0 + tx;
            if (c < cols && r < rows) out[(long)c * rows + r] = (T)tile[tx][i];
        } else {
            const int r = r0 + i, c = c0 + tx;
            if (r < rows && c < cols) out[(long)r * cols + c] = (T)tile[i][tx];
        }
    }
}

void from_fp64_blocks(hipStream_t s, int dtype, const double* in, void* out, int batch, int rows,
                      int cols, bool transpose, JobMap jm) {
    if (batch <= 0 || rows <= 0 || cols <= 0) return;
    jm.per_job = batch;
    const dim3 grid(ceil_div(cols, 32), ceil_div(rows, 32), batch * (jm.delta ? jm.njobs : 1));
    if (dtype == IPEPS_DTYPE_FP64) {
        if (transpose)
            hipLaunchKernelGGL((k_from64_blocks<double, true>), grid, dim3(256), 0, s, in, (double*)out,
                               rows, cols, jm);
        else
            hipLaunchKernelGGL((k_from64_blocks<double, false>), grid, dim3(256), 0, s, in,
                               (double*)out, rows, cols, jm);
    } else {
        if (transpose)
            hipLaunchKernelGGL((k_from64_blocks<float, true>), grid, dim3(256), 0, s, in, (float*)out,
                               rows, cols, jm);
        else
            hipLaunchKernelGGL((k_from64_blocks<float, false>), grid, dim3(256), 0, s, in, (float*)out,
                               rows, cols, jm);
    }
    HIP_CHECK(hipGetLastError());
}

// 16-byte words when both ends and the size allow it, else bytes
__global__ __launch_bounds__(256) void k_copy_jobs(char* dst, const char* src, size_t bytes, JobMap jm) {
    dst = jptr(dst, jm, blockIdx.y);
    src = jptr(src, jm, blockIdx.y);
    const bool wide = ((((uintptr_t)dst) | ((uintptr_t)src) | bytes) & 15) == 0;
    if (wide) {
        const size_t nw = bytes / 16;
        for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nw; e += (size_t)gridDim.x * blockDim.x)
            ((uint4*)dst)[e] = ((const uint4*)src)[e];
    } else {
        for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < bytes; e += (size_t)gridDim.x * blockDim.x)
            dst[e] = src[e];
    }
}

void copy_jobs(hipStream_t s, void* dst, const void* src, size_t bytes, JobMap jm) {
    if (bytes == 0) return;
    if (!jm.delta) {
        HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
        return;
    }
    jm.per_job = 1;
    const int grid = ceil_div((long)(bytes / 16 + 1), 256) < 1024 ? ceil_div((long)(bytes / 16 + 1), 256) : 1024;
    hipLaunchKernelGGL(k_copy_jobs, dim3(grid, jm.njobs), dim3(256), 0, s, (char*)dst, (const char*)src, bytes, jm);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ projector factors
// Keep g <= K values: zeros (<= tau s_1) are dropped, and a multiplet
// (neighbours whose gap is <= 1e-10 of the larger plus tau s_1) is never cut.
__device__ inline int trunc_rule_dev(const double* s, int n, int K, double tau) {
    if (n <= 0 || !(s[0] > 0.0)) return 0;
    int r = 0;
    for (int i = 0; i < n; ++i) r += s[i] > tau * s[0];
    int g = r < K ? r : K;
    if (g < r)
        while (g > 1 && s[g - 1] - s[g] <= 1e-10 * s[g - 1] + tau * s[0]) --g;
    return g;
}

template <typename T>
__device__ inline void proj_factors_body(int n, int k, int chi, double tau, const double* U, const double* V,
                                         const double* sigma, long strideUV, T* Us, T* Vs, long strideP,
                                         int* g_out, JobMap jm) {
    // every block of matrix b re-derives g (k <= 256 values) and the weights
    __shared__ int g_s;
    __shared__ double w[256];
    const int b = jlocal(jm, blockIdx.y);
    U = jptr(U, jm, blockIdx.y);
    V = jptr(V, jm, blockIdx.y);
    sigma = jptr(sigma, jm, blockIdx.y);
    if (Us) Us = jptr(Us, jm, blockIdx.y);
    Vs = jptr(Vs, jm, blockIdx.y);
    if (g_out) g_out = jptr(g_out, jm, blockIdx.y);
    const double* sg = sigma + (long)b * k;
    if (threadIdx.x == 0) {
        g_s = trunc_rule_dev(sg, k, chi, tau);
        if (blockIdx.x == 0 && g_out) g_out[b] = g_s;
    }
    __syncthreads();
    const int g = g_s;
    for (int c = threadIdx.x; c < chi; c += blockDim.x) w[c] = (c < g) ? 1.0 / sqrt(sg[c]) : 0.0;
    __syncthreads();
    const double* Ub = U + b * strideUV;
    const double* Vb = V + b * strideUV;
    T* vs = Vs + b * strideP;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * chi;
         e += (long)gridDim.x * blockDim.x) {
        const int i = e / chi, c = e % chi;
        const double wc = w[c];
        vs[e] = (T)(wc != 0.0 ? Vb[(long)i * k + c] * wc : 0.0);
    }
    if (!Us) return;
    // Us transposed (chi x n): P_up = Us^T G is then a plain product with a
    // k-contiguous left operand
    T* us = Us + b * strideP;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * chi;
         e += (long)gridDim.x * blockDim.x) {
        const int c = e / n, i = e % n;
        const double wc = w[c];
        us[e] = (T)(wc != 0.0 ? Ub[(long)i * k + c] * wc : 0.0);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_proj_factors(int n, int k, int chi, double tau,
                                                      const double* U, const double* V,
                                                      const double* sigma, long strideUV, T* Us,
                                                      T* Vs, long strideP, int* g_out, JobMap jm) {
    proj_factors_body<T>(n, k, chi, tau, U, V, sigma, strideUV, Us, Vs, strideP, g_out, jm);
}

// Two projector_factors calls on the same singular values in one launch
// (blockIdx.z selects the call).
template <typename T>
__global__ __launch_bounds__(256) void k_proj_factors_pair(ProjFactorsPair pp, int k, int chi, double tau,
                                                           const double* sigma, JobMap jm) {
    const int z = blockIdx.z;
    proj_factors_body<T>(pp.n[z], k, chi, tau, pp.U[z], pp.V[z], sigma, pp.strideUV[z], (T*)pp.Us[z],
                         (T*)pp.Vs[z], pp.strideP[z], pp.g_out[z], jm);
}

void projector_factors_pair(hipStream_t s, int dtype, int batch, int k, int chi, double tau,
                            const double* sigma, const ProjFactorsPair& pp, JobMap jm) {
    IPEPS_REQUIRE(chi <= 256 && k <= 256, IPEPS_EINVAL, "projector_factors: chi, k > 256");
    const long tot = (long)std::max(pp.n[0], pp.n[1]) * chi;
    jm.per_job = batch;
    const dim3 grid(ceil_div(tot, 256) < 512 ? ceil_div(tot, 256) : 512, batch * (jm.delta ? jm.njobs : 1), 2);
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_proj_factors_pair<double>, grid, dim3(256), 0, s, pp, k, chi, tau, sigma, jm);
    else
        hipLaunchKernelGGL(k_proj_factors_pair<float>, grid, dim3(256), 0, s, pp, k, chi, tau, sigma, jm);
    HIP_CHECK(hipGetLastError());
}

void projector_factors(hipStream_t s, int dtype, int batch, int n, int k, int chi, double tau,
                       const double* U, const double* V, const double* sigma, long strideUV,
                       void* Us, void* Vs, long strideP, int* g_out, JobMap jm) {
    IPEPS_REQUIRE(chi <= 256 && k <= 256, IPEPS_EINVAL, "projector_factors: chi, k > 256");
    const long tot = (long)n * chi;
    jm.per_job = batch;
    const dim3 grid(ceil_div(tot, 256) < 512 ? ceil_div(tot, 256) : 512, batch * (jm.delta ? jm.njobs : 1));
    if (dtype == IPEPS_DTYPE_FP64)
        hipLaunchKernelGGL(k_proj_factors<double>, grid, dim3(256), 0, s, n, k, chi, tau, U, V,
                           sigma, strideUV, (double*)Us, (double*)Vs, strideP, g_out, jm);
    else
        hipLaunchKernelGGL(k_proj_factors<float>, grid, dim3(256), 0, s, n, k, chi, tau, U, V,
                           sigma, strideUV, (float*)Us, (float*)Vs, strideP, g_out, jm);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ spectra
__global__ void k_spectra_delta(int nspec, int chi, const double* sig, double* spectra, double* prev,
                                double* delta_out, int first, JobMap jm) {
    __shared__ double dmax[64];
    sig = jptr(sig, jm, blockIdx.x);
    spectra = jptr(spectra, jm, blockIdx.x);
    prev = jptr(prev, jm, blockIdx.x);
    delta_out = jptr(delta_out, jm, blockIdx.x);
    const int c = threadIdx.x;
    double dl = 0.0;
    if (c < nspec) {
        const double* sc = sig + (long)c * chi;
        double n2 = 0;
        for (int i = 0; i < chi; ++i) n2 += sc[i] * sc[i];
        const double inv = n2 > 0 ? 1.0 / sqrt(n2) : 0.0;
        double d2 = 0;
        for (int i = 0; i < chi; ++i) {
            const double v = sc[i] * inv;
            spectra[(long)c * chi + i] = v;
            const double dv = v - prev[(long)c * chi + i];
            d2 += dv * dv;
            prev[(long)c * chi + i] = v;
        }
        dl = sqrt(d2);
    }
    dmax[c] = dl;
    __syncthreads();
    if (c == 0) {
        double m = 0;
        for (int i = 0; i < nspec; ++i) m = fmax(m, dmax[i]);
        *delta_out = first ? INFINITY : m;
    }
}

void spectra_delta(hipStream_t s, int nspec, int chi, const double* sig, double* spectra,
                   double* prev, double* delta_out, int first, JobMap jm) {
    jm.per_job = 1;
    hipLaunchKernelGGL(k_spectra_delta, dim3(jm.delta ? jm.njobs : 1), dim3(64), 0, s, nspec, chi, sig,
                       spectra, prev, delta_out, first, jm);
    HIP_CHECK(hipGetLastError());
}

__global__ void k_random_block(int n, int k, uint64_t seed, double* X) {
    const long tot = (long)n * k;
    const int b = blockIdx.y;
    for (long e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
        X[b * tot + e] = 2.0 * hash_uniform(seed, (uint64_t)(b * tot + e)) - 1.0;
}

void random_block(hipStream_t s, int batch, int n, int k, uint64_t seed, double* X) {
    const long tot = (long)n * k;
    hipLaunchKernelGGL(k_random_block, dim3(ceil_div(tot, 256) < 1024 ? ceil_div(tot, 256) : 1024, batch),
                       dim3(256), 0, s, n, k, seed, X);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ readout
// Rows of T = E_c A^H: one wave per (site, x), lanes over x'; E_c(x, x') is
// rebuilt on the fly from the real-basis E (at most 16 terms).
__global__ __launch_bounds__(256) void k_readout_rows(int D, int d, const double* __restrict__ E,
                                                      const cplx* __restrict__ A, cplx* __restrict__ T) {
    const int q = D * D;
    const long q4 = (long)q * q * q * q, D4 = (long)D * D * D * D;
    const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= 4 * D4) return;
    const int site = (int)(row / D4);
    const long x = row % D4;
    const double* Es = E + site * q4;
    const cplx* As = A + site * d * D4;
    const int r = x % D, dd = (x / D) % D, l = (x / (D * D)) % D, u = x / (D * D * D);
    // d <= 10; the loops over sp run to 10 with a guard so that tr, ti stay
    // in registers
    double tr[10], ti[10];
#pragma unroll
    for (int sp = 0; sp < 10; ++sp) tr[sp] = ti[sp] = 0.0;
    for (long xp = lane; xp < D4; xp += 64) {
        const int rp = xp % D, dp = (xp / D) % D, lp = (xp / (D * D)) % D, up = xp / (D * D * D);
        const InvTerms tl = inv_terms(l, lp, D, false), tu = inv_terms(u, up, D, false);
        const InvTerms tR = inv_terms(r, rp, D, true), tD = inv_terms(dd, dp, D, true);
        cplx ec = cmake(0, 0);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int e = 0; e < 2; ++e)
                        if (a < tl.n && b < tu.n && c < tR.n && e < tD.n) {
                            const double ev = Es[(((long)tl.m[a] * q + tu.m[b]) * q + tR.m[c]) * q + tD.m[e]];
                            ec = cadd(ec, cscale(cmul(cmul(tl.c[a], tu.c[b]), cmul(tR.c[c], tD.c[e])), ev));
                        }
#pragma unroll
        for (int sp = 0; sp < 10; ++sp)
            if (sp < d) {
                const cplx t = cmul(ec, cconj(As[sp * D4 + xp]));
                tr[sp] += t.re;
                ti[sp] += t.im;
            }
    }
#pragma unroll
    for (int sp = 0; sp < 10; ++sp) {
        tr[sp] = wave_sum(tr[sp]);
        ti[sp] = wave_sum(ti[sp]);
    }
    if (lane == 0)
#pragma unroll
        for (int sp = 0; sp < 10; ++sp)
            if (sp < d) T[row * d + sp] = cmake(tr[sp], ti[sp]);
}

// rho[s][s'] = sum_x A[s][x] T[x][s'], trace-normalised; occupations with the
// auxiliary level traced out, imbalance, their sum, largest |rho_p[up,dn]|.
__global__ __launch_bounds__(1024) void k_readout_finish(int D, int d, int dA, const cplx* __restrict__ A,
                                                         const cplx* __restrict__ T, cplx* rho, double* obs) {
    __shared__ double red[16];
    __shared__ cplx rs[100];
    __shared__ double nsite[4], offd[4], s1[4], shalf[4];
    const long D4 = (long)D * D * D * D;
    for (int site = 0; site < 4; ++site) {
        const cplx* As = A + site * d * D4;
        const cplx* Ts = T + site * D4 * d;
        for (int i = 0; i < d * d; ++i) {
            const int s = i / d, sp = i % d;
            double re = 0, im = 0;
            for (long x = threadIdx.x; x < D4; x += blockDim.x) {
                const cplx v = cmul(As[s * D4 + x], Ts[x * d + sp]);
                re += v.re;
                im += v.im;
            }
            re = block_sum(re, red);
            im = block_sum(im, red);
            if (threadIdx.x == 0) rs[i] = cmake(re, im);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            cplx tr = cmake(0, 0);
            for (int i = 0; i < d; ++i) tr = cadd(tr, rs[i * d + i]);
            const double tn = cabs2(tr);
            const cplx inv = cmake(tr.re / tn, -tr.im / tn);
            for (int i = 0; i < d * d; ++i) rho[site * d * d + i] = cmul(rs[i], inv);
            cplx p00 = cmake(0, 0), p01 = cmake(0, 0), p11 = cmake(0, 0);
            for (int a = 0; a < dA; ++a) {
                p00 = cadd(p00, cmul(rs[(0 * dA + a) * d + (0 * dA + a)], inv));
                p01 = cadd(p01, cmul(rs[(0 * dA + a) * d + (1 * dA + a)], inv));
                p11 = cadd(p11, cmul(rs[(1 * dA + a) * d + (1 * dA + a)], inv));
            }
            nsite[site] = p00.re;
            offd[site] = sqrt(cabs2(p01));
            // Renyi entropies of the physical one-site matrix rho_p (2 x 2,
            // Hermitian, unit trace): eigenvalues (t +- r) / 2
            const double tt = p00.re + p11.re, df = p00.re - p11.re;
            const double r = sqrt(df * df + 4.0 * cabs2(p01));
            double lam[2] = {0.5 * (tt + r), 0.5 * (tt - r)};
            double e1 = 0.0, sq = 0.0;
            for (int i = 0; i < 2; ++i) {
                const double l = lam[i] > 0.0 ? lam[i] : 0.0;
                if (l > 0.0) e1 -= l * log(l);
                sq += sqrt(l);
            }
            s1[site] = e1;
            shalf[site] = 2.0 * log(sq);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double sum = 0, mo = 0;
        for (int i = 0; i < 4; ++i) {
            obs[i] = nsite[i];
            sum += nsite[i];
            mo = fmax(mo, offd[i]);
        }
        obs[4] = 0.5 * (nsite[0] + nsite[3] - nsite[1] - nsite[2]);
        obs[5] = sum;
        obs[6] = mo;
        obs[7] = 0.0;
        for (int i = 0; i < 4; ++i) {
            obs[8 + i] = s1[i];
            obs[12 + i] = shalf[i];
        }
    }
}

void readout(hipStream_t s, int D, int d, int d_A, const double* E, const cplx* A, cplx* Twork,
             cplx* rho, double* obs) {
    IPEPS_REQUIRE(d <= 10, IPEPS_EINVAL, "readout supports d <= 10");
    const long rows = 4L * D * D * D * D;
    hipLaunchKernelGGL(k_readout_rows, dim3(ceil_div(rows, 4)), dim3(256), 0, s, D, d, E, A, Twork);
    hipLaunchKernelGGL(k_readout_finish, dim3(1), dim3(1024), 0, s, D, d, d_A, A, Twork, rho, obs);
    HIP_CHECK(hipGetLastError());
}

}  // namespace ipeps
