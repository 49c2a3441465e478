// Grouped MFMA GEMM for gfx950 (CDNA4), FP64, FP32 and BF16 with FP32
// accumulation (BF16 modes: FP32 operands in memory and LDS, rounded to BF16
// (nearest even) as the MFMA fragment is built, v_mfma_f32_16x16x32_bf16,
// FP32 results; split BF16 carries each operand as two BF16 terms).
//
// One workgroup computes a BM x BN tile of one problem; 4 waves in a 2x2
// arrangement each own a (BM/2) x (BN/2) block made of 16x16 MFMA blocks
// (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).  Operand tiles go
// global -> registers -> LDS (k-major, one element of padding per row so the
// MFMA operand reads of 16 consecutive rows/columns hit distinct banks); the
// next tile's global loads are issued before the current tile's MFMAs.
//
// MFMA lane layouts (checked on the device): operand A element (i, k) is held
// by lane i + 16 k, operand B element (k, j) by lane j + 16 k; the FP32
// result register r of lane l is row 4 (l / 16) + r, column l % 16; the FP64
// result register r of lane l is row l / 16 + 4 r, column l % 16.  The BF16
// 16x16x32 MFMA takes 8 values per lane: lane l holds row (A) / column (B)
// l % 16, and element e of lane group g = l / 16 is paired with element e of
// the same lane group of the other operand; the k order (g, e) -> k is a
// free choice as long as A and B use the same one (here k = 8 g + e inside a
// 32-wide k tile); the result layout is that of the FP32 16x16x4 MFMA.
#include "gemm.h"

#include <cstdint>

namespace ipeps {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// BF = 1: each operand value x is rounded to h = bf16(x) (nearest even);
// BF = 3 (split BF16): x is carried as h + l with l = bf16(x - h), and the
// product as h_a h_b + h_a l_b + l_a h_b (three MFMAs; the dropped l_a l_b
// is ~2^-16 of the product), about 16 bits of operand precision.
template <int BF>
struct BfOperand {
    bf8_t h, l;
    __device__ inline void set(int e, float x) {
        const __bf16 hx = (__bf16)x;
        h[e] = hx;
        if constexpr (BF == 3) l[e] = (__bf16)(x - (float)hx);
    }
};
template <int BF>
__device__ inline f4_t mfma_bf16(const BfOperand<BF>& a, const BfOperand<BF>& b, f4_t c) {
    if constexpr (BF == 3) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
}

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef d4_t acc_t;
    static __device__ inline acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef f4_t acc_t;
    static __device__ inline acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// TAG only gives launches of one role (the n^3 cut products) their own kernel
// symbol, so profilers report them separately; the code is identical.
template <typename T, int BM, int BN, int BK, int TAG, int BF = 0>
__global__ __launch_bounds__(256) void k_gemm_grouped(const GemmProb* __restrict__ probs,
                                                      int nprob) {
    static_assert(BF == 0 || BF == 1 || BF == 3, "BF: 0, 1 or 3 BF16 products");
    static_assert(!BF || (sizeof(T) == 4 && BK % 32 == 0), "BF16 modes: FP32 storage, k tiles of 32");
    constexpr int NT = 256;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int LA = BM * BK / NT;  // A elements per thread per tile
    constexpr int LB = BN * BK / NT;
    constexpr int PA = BM + 1, PB = BN + 1;
    __shared__ T As[BK * PA];
    __shared__ T Bs[BK * PB];

    // ---- which problem / tile
    int bid = blockIdx.x;
    int p = 0;
    while (p + 1 < nprob && probs[p + 1].tile_begin <= bid) ++p;
    const GemmProb& P = probs[p];
    if (P.gate && *P.gate == 0) return;  // uniform over the workgroup, before any barrier
    const int ks = P.ksplit > 1 ? P.ksplit : 1;
    const int tt = bid - P.tile_begin;
    const int split = tt % ks, t = tt / ks;
    const int tm = t / P.tiles_n, tn = t - (t / P.tiles_n) * P.tiles_n;
    const int M = P.M, N = P.N;
    // K range of this split, in whole BK tiles
    const int kchunk = ((P.K + ks - 1) / ks + BK - 1) / BK * BK;
    const int kbeg = split * kchunk;
    const int K = (kbeg + kchunk < P.K) ? kbeg + kchunk : P.K;
    const int m0 = tm * BM, n0 = tn * BN;
    const T* __restrict__ A = (const T*)P.A;
    const T* __restrict__ B = (const T*)P.B;

    const int tid = threadIdx.x;
    const bool a_kcontig = (P.a_ks == 1);
    const bool b_ncontig = (P.b_cs == 1);

    // per-thread element coordinates inside the tile (fixed across k tiles)
    int a_mi[LA], a_ki[LA];
    long a_row[LA];
#pragma unroll
    for (int r = 0; r < LA; ++r) {
        int e = tid + r * NT;
        if (a_kcontig) {
            a_ki[r] = e % BK;
            a_mi[r] = e / BK;
        } else {
            a_mi[r] = e % BM;
            a_ki[r] = e / BM;
        }
        int i = m0 + a_mi[r];
        a_row[r] = (i < M) ? (long)(i / P.a_rows0) * P.a_rs1 + (long)(i % P.a_rows0) * P.a_rs0
                           : -1;
    }
    int b_ni[LB], b_ki[LB];
#pragma unroll
    for (int r = 0; r < LB; ++r) {
        int e = tid + r * NT;
        if (b_ncontig) {
            b_ni[r] = e % BN;
            b_ki[r] = e / BN;
        } else {
            b_ki[r] = e % BK;
            b_ni[r] = e / BK;
        }
    }

    T ra[LA], rb[LB];
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            int k = k0 + a_ki[r];
            ra[r] = (a_row[r] >= 0 && k < K) ? A[a_row[r] + (long)k * P.a_ks] : T(0);
        }
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            int k = k0 + b_ki[r], j = n0 + b_ni[r];
            rb[r] = (j < N && k < K) ? B[(long)k * P.b_ks + (long)j * P.b_cs] : T(0);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int r = 0; r < LA; ++r) As[a_ki[r] * PA + a_mi[r]] = ra[r];
#pragma unroll
        for (int r = 0; r < LB; ++r) Bs[b_ki[r] * PB + b_ni[r]] = rb[r];
    };

    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int nk = K > kbeg ? (K - kbeg + BK - 1) / BK : 0;
    if (nk > 0) {
        load(kbeg);
        store();
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load(kbeg + (kt + 1) * BK);
        if constexpr (BF) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 32) {
                BfOperand<BF> fa[FM], fb[FN];
                const int kr = kk + 8 * (lane >> 4);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
#pragma unroll
                    for (int a = 0; a < FM; ++a) fa[a].set(e, As[(kr + e) * PA + wm0 + a * 16 + (lane & 15)]);
#pragma unroll
                    for (int b = 0; b < FN; ++b) fb[b].set(e, Bs[(kr + e) * PB + wn0 + b * 16 + (lane & 15)]);
                }
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(fa[a], fb[b], acc[a][b]);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                T fa[FM], fb[FN];
                const int kr = kk + (lane >> 4);
#pragma unroll
                for (int a = 0; a < FM; ++a) fa[a] = As[kr * PA + wm0 + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < FN; ++b) fb[b] = Bs[kr * PB + wn0 + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) acc[a][b] = Mfma<T>::step(fa[a], fb[b], acc[a][b]);
            }
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store();
            __syncthreads();
        }
    }

    // ---- epilogue
    const T alpha = (T)P.alpha, beta = (T)P.beta;
    if (ks > 1) {
        T* __restrict__ W = (T*)P.ws + (long)split * M * N;
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int j = n0 + wn0 + b * 16 + (lane & 15);
            if (j >= N) continue;
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm0 + a * 16 + Mfma<T>::row(lane, r);
                    if (i < M) W[(long)i * N + j] = alpha * acc[a][b][r];
                }
        }
        return;
    }
    T* __restrict__ C = (T*)P.C;
#pragma unroll
    for (int b = 0; b < FN; ++b) {
        const int j = n0 + wn0 + b * 16 + (lane & 15);
        if (j >= N) continue;
        const long cj = (long)(j / P.c_cols0) * P.c_cs1 + (long)(j % P.c_cols0) * P.c_cs0;
#pragma unroll
        for (int a = 0; a < FM; ++a) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm0 + a * 16 + Mfma<T>::row(lane, r);
                if (i >= M) continue;
                const long off =
                    (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 + cj;
                T v = alpha * acc[a][b][r];
                if (beta != T(0)) v += beta * C[off];
                C[off] = v;
            }
        }
    }
}

GemmProb gemm_general(const void* A, bool transA, long lda, const void* B, bool transB,
                      long ldb, void* C, long ldc, int M, int N, int K, double alpha,
                      double beta) {
    GemmProb p{};
    p.A = A;
    p.B = B;
    p.C = C;
    p.M = M;
    p.N = N;
    p.K = K;
    p.a_rows0 = M > 0 ? M : 1;
    p.a_rs1 = 0;
    p.a_rs0 = transA ? 1 : lda;
    p.a_ks = transA ? lda : 1;
    p.b_ks = transB ? 1 : ldb;
    p.b_cs = transB ? ldb : 1;
    p.c_rows0 = M > 0 ? M : 1;
    p.c_cols0 = N > 0 ? N : 1;
    p.c_rs1 = 0;
    p.c_rs0 = ldc;
    p.c_cs1 = 0;
    p.c_cs0 = 1;
    p.alpha = alpha;
    p.beta = beta;
    p.ksplit = 1;
    p.ws = nullptr;
    return p;
}

GemmProb gemm_nn(const void* A, long lda, const void* B, long ldb, void* C, long ldc, int M,
                 int N, int K, double alpha, double beta) {
    return gemm_general(A, false, lda, B, false, ldb, C, ldc, M, N, K, alpha, beta);
}

static void tile_dims(int dtype, GemmTile tile, int* bm, int* bn) {
    (void)dtype;
    if (is_panel(tile)) {
        const int np = 16 * ((tile - TILE_PANEL) % 16);
        const bool sm = (tile - TILE_PANEL) >= 16;
        *bm = sm ? np : 64;
        *bn = sm ? 64 : np;
    } else if (tile == TILE_LARGE || tile == TILE_DIRECT) {
        *bm = 128;
        *bn = 128;
    } else {
        *bm = 64;
        *bn = 64;
    }
}

static bool direct_ok(const GemmProb* probs, int n, int dtype) {
    const long vw = dtype == IPEPS_DTYPE_FP64 ? 2 : 4;
    for (int i = 0; i < n; ++i) {
        const GemmProb& p = probs[i];
        if (!(p.a_ks == 1 && p.a_rs0 % vw == 0 && p.a_rs1 % vw == 0 && p.K % vw == 0 &&
              p.K >= vw && ((uintptr_t)p.A & 15) == 0 && p.b_cs == 1 && p.b_ks % vw == 0 &&
              p.N % vw == 0 && p.N >= vw && ((uintptr_t)p.B & 15) == 0))
            return false;
    }
    return true;
}

int gemm_plan_with(GemmProb* probs, int n, int dtype, GemmTile tile) {
    int bm, bn;
    tile_dims(dtype, tile, &bm, &bn);
    int total = 0;
    for (int i = 0; i < n; ++i) {
        int tm = ceil_div(probs[i].M, bm), tnn = ceil_div(probs[i].N, bn);
        if (probs[i].M <= 0 || probs[i].N <= 0) tm = tnn = 0;
        if (probs[i].ksplit < 1) probs[i].ksplit = 1;
        probs[i].tiles_n = tnn > 0 ? tnn : 1;
        probs[i].tile_begin = total;
        total += tm * tnn * probs[i].ksplit;
    }
    return total;
}

int gemm_plan_tiles(GemmProb* probs, int n, int dtype, GemmTile* tile) {
    // large tiles when the launch still has >= 2 workgroups per CU with them
    // and few problems are thinner than a large tile
    long small_work = 0, all_work = 0, large_tiles = 0;
    for (int i = 0; i < n; ++i) {
        long w = (long)probs[i].M * probs[i].N;
        all_work += w;
        if (probs[i].M < 96 || probs[i].N < 96) small_work += w;
        const int ks = probs[i].ksplit > 1 ? probs[i].ksplit : 1;
        large_tiles += (long)ceil_div(probs[i].M, 128) * ceil_div(probs[i].N, 128) * ks;
    }
    *tile = (small_work * 4 > all_work || large_tiles < 512) ? TILE_SMALL : TILE_LARGE;
    if (direct_ok(probs, n, dtype)) *tile = (*tile == TILE_LARGE) ? TILE_DIRECT : TILE_DIRECT_SMALL;
    return gemm_plan_with(probs, n, dtype, *tile);
}

int gemm_panel_for(const GemmProb* probs, int n, int dtype) {
    if (n < 1 || !direct_ok(probs, n, dtype)) return -1;
    auto pad = [](int v) { return v <= 80 ? 80 : (v + 15) / 16 * 16; };
    for (int sm = 0; sm < 2; ++sm) {
        const int w0 = sm ? probs[0].M : probs[0].N;
        bool ok = w0 > 64 && w0 <= 128;
        for (int i = 0; i < n && ok; ++i) {
            const int w = sm ? probs[i].M : probs[i].N, other = sm ? probs[i].N : probs[i].M;
            ok = w > 64 && pad(w) == pad(w0) && other > 128;
        }
        if (ok) return (int)panel_tile(sm != 0, pad(w0));
    }
    return -1;
}

int gemm_tile_candidates(const GemmProb* probs, int n, int dtype, GemmTile* out) {
    int c = 0;
    const int pt = gemm_panel_for(probs, n, dtype);
    if (pt >= 0) out[c++] = (GemmTile)pt;
    if (direct_ok(probs, n, dtype)) {
        out[c++] = TILE_DIRECT;
        out[c++] = TILE_DIRECT_SMALL;
    }
    out[c++] = TILE_LARGE;
    out[c++] = TILE_SMALL;
    return c;
}

// ---------------------------------------------------------------------------
template <typename T>
struct Vec16;
template <>
struct Vec16<float> { typedef float v_t __attribute__((ext_vector_type(4))); };
template <>
struct Vec16<double> { typedef double v_t __attribute__((ext_vector_type(2))); };

// Epilogue through LDS: the workgroup writes its accumulators into `lds`
// (RING elements, at least BN rows' worth; 16-byte chunks XOR-swizzled by the
// row) in passes of RP tile rows, then stores the tile in row order, one
// 16-byte vector per lane where the output layout keeps VW consecutive
// columns contiguous (always for the split-K partials, row-major M x N).
// Every lane of the workgroup must call it (it holds barriers).
template <typename T, int BM, int BN, int WM, int FM, int FN, int RING, typename Acc>
__device__ inline void store_tile_staged(const GemmProb& P, T* lds, const Acc (&acc)[FM][FN], int ks,
                                         int split, int m0, int n0, int wm0, int wn0) {
    typedef typename Vec16<T>::v_t v_t;
    constexpr int VW = 16 / (int)sizeof(T);
    constexpr int RP = (RING / BN) < BM ? (RING / BN) : BM;  // tile rows per pass
    static_assert(BM % RP == 0 && RP % WM == 0, "whole wave tiles per pass");
    constexpr int CPR = BN / VW;  // 16-byte chunks per tile row
    static_assert(CPR % 8 == 0, "the swizzle permutes groups of 8 chunks");
    const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15;
    const int M = P.M, N = P.N;
    const T alpha = (T)P.alpha, beta = (T)P.beta;
    const bool partial = ks > 1;
    T* __restrict__ C = partial ? (T*)P.ws + (long)split * M * N : (T*)P.C;
    const bool vec = partial || (P.c_cs0 == 1 && P.c_cols0 % VW == 0 && P.c_cs1 % VW == 0 &&
                                 P.c_rs0 % VW == 0 && P.c_rs1 % VW == 0 && ((uintptr_t)P.C & 15) == 0);
    __syncthreads();  // every wave is done reading the operand tiles
#pragma unroll
    for (int h = 0; h < BM / RP; ++h) {
        if (wm0 / RP == h) {
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm0 - h * RP + a * 16 + Mfma<T>::row(lane, r);
                        const int col = wn0 + b * 16 + l16;
                        lds[row * BN + ((col / VW) ^ (row & 7)) * VW + col % VW] = alpha * acc[a][b][r];
                    }
        }
        __syncthreads();
        for (int e = tid; e < RP * CPR; e += blockDim.x) {
            const int row = e / CPR, ch = e - (e / CPR) * CPR;
            const int i = m0 + h * RP + row, j0 = n0 + ch * VW;
            if (i >= M || j0 >= N) continue;  // N is a multiple of VW
            v_t v = *(const v_t*)(lds + row * BN + (ch ^ (row & 7)) * VW);
            if (partial) {
                *(v_t*)(C + (long)i * N + j0) = v;
            } else if (vec) {
                const long off = (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 +
                                 (long)(j0 / P.c_cols0) * P.c_cs1 + (long)(j0 % P.c_cols0);
                if (beta != T(0)) v += beta * *(const v_t*)(C + off);
                *(v_t*)(C + off) = v;
            } else {
#pragma unroll
                for (int q = 0; q < VW; ++q) {
                    const int j = j0 + q;
                    const long off = (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 +
                                     (long)(j / P.c_cols0) * P.c_cs1 + (long)(j % P.c_cols0) * P.c_cs0;
                    T w = v[q];
                    if (beta != T(0)) w += beta * C[off];
                    C[off] = w;
                }
            }
        }
        if (h + 1 < BM / RP) __syncthreads();
    }
}

// Direct kernel: operand tiles copied global -> LDS by 16-byte LDS-DMA loads
// (no register staging) through an NS-stage ring, one barrier per k tile, and
// an XCD-aware tile order (workgroup b runs on XCD b % 8; each XCD gets a
// contiguous range of tiles so neighbouring tiles share its L2).
// A (k contiguous) is stored [m][k] with the 16-byte chunk index XOR-swizzled
// by the row, read as 16-byte vectors (k order inside a tile permuted alike
// for A and B); B (n contiguous) is stored [k][n] with chunks swizzled by the
// lane group that reads the row, read as scalars.
// s_waitcnt vmcnt(N) (gfx9 encoding: vmcnt[3:0] and [15:14]; expcnt and
// lgkmcnt left at their maxima so they impose no wait)
template <int N>
__device__ inline void wait_vm_n() {
    static_assert(N >= 0 && N <= 63, "vmcnt is 6 bits");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// vmcnt(s * STEP) for s in 0..3 (the immediate must be a constant)
template <int STEP>
__device__ inline void wait_vm(int s) {
    switch (s) {
        case 0: wait_vm_n<0>(); break;
        case 1: wait_vm_n<STEP>(); break;
        case 2: wait_vm_n<2 * STEP>(); break;
        default: wait_vm_n<3 * STEP>(); break;
    }
}

// At least two waves per SIMD: without the bound the FP64 128 x 128 variant
// takes 194 VGPRs + 128 AGPRs (one wave per SIMD) and ran 27 % slower.
template <typename T, int BM, int BN, int BK, int NS, int TAG, int BF = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_gemm_direct(const GemmProb* __restrict__ probs, int nprob) {
    static_assert(BF == 0 || BF == 1 || BF == 3, "BF: 0, 1 or 3 BF16 products");
    static_assert(!BF || (sizeof(T) == 4 && BK == 32), "BF16 modes: FP32 storage, k tiles of 32");
    constexpr int VW = 16 / (int)sizeof(T);
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int KPL = BK / 4;
    constexpr int NCH = KPL / VW;
    constexpr int ACH = BK / VW;              // 16-byte chunks per A row (8)
    constexpr int BCH = BN / VW;              // 16-byte chunks per B row
    constexpr int BSW = (BCH / 4) < 8 ? (BCH / 4) : 8;  // B swizzle step per lane group
    constexpr int ASZ = BM * BK, BSZ = BK * BN;
    constexpr int NLD = (BM * ACH) / 256;     // A loads per lane per tile (= B loads)
    static_assert(BM * ACH == BK * BCH, "A and B tiles must need the same number of loads");
    static_assert(NS >= 2 && NS <= 5, "wait_vm covers up to 3 tiles in flight behind the current one");
    typedef typename Vec16<T>::v_t v_t;
    __shared__ __attribute__((aligned(16))) T Sm[NS * (ASZ + BSZ)];

    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int per = G >> 3, rem = G & 7;
    const int bid = xcd * per + (xcd < rem ? xcd : rem) + idx;
    int p = 0;
    while (p + 1 < nprob && probs[p + 1].tile_begin <= bid) ++p;
    const GemmProb& P = probs[p];
    if (P.gate && *P.gate == 0) return;
    const int ks = P.ksplit > 1 ? P.ksplit : 1;
    const int tt = bid - P.tile_begin;
    const int split = tt % ks, t = tt / ks;
    const int tm = t / P.tiles_n, tn = t - (t / P.tiles_n) * P.tiles_n;
    const int M = P.M, N = P.N;
    const int kchunk = ((P.K + ks - 1) / ks + BK - 1) / BK * BK;
    const int kbeg = split * kchunk;
    const int K = (kbeg + kchunk < P.K) ? kbeg + kchunk : P.K;
    const int m0 = tm * BM, n0 = tn * BN;
    const T* __restrict__ A = (const T*)P.A;
    const T* __restrict__ B = (const T*)P.B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // per-lane source offsets (fixed across k tiles)
    long a_src[NLD];
    int a_lk[NLD];
#pragma unroll
    for (int r = 0; r < NLD; ++r) {
        const int row = (r * 4 + wave) * (64 / ACH) + lane / ACH;
        const int lchunk = (lane % ACH) ^ (row & 7);
        int i = m0 + row;
        i = i < M ? i : M - 1;
        a_src[r] = (long)(i / P.a_rows0) * P.a_rs1 + (long)(i % P.a_rows0) * P.a_rs0;
        a_lk[r] = lchunk * VW;
    }
    int b_k[NLD], b_n[NLD];
#pragma unroll
    for (int r = 0; r < NLD; ++r) {
        const int c = (r * 4 + wave) * 64 + lane;
        const int k = c / BCH, pch = c % BCH;
        const int lchunk = pch ^ (((k / KPL) & 3) * BSW);
        int n = n0 + lchunk * VW;
        n = n < N ? n : N - VW;
        b_k[r] = k;
        b_n[r] = n;
    }
    auto issue = [&](int kt, int stg) {
        const int k0 = kbeg + kt * BK;
        T* as = Sm + stg * (ASZ + BSZ);
        T* bs = as + ASZ;
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            int k = k0 + a_lk[r];
            k = k < K ? k : K - VW;
            __builtin_amdgcn_global_load_lds((const void*)(A + a_src[r] + k),
                                             (__attribute__((address_space(3))) void*)(as + (r * 4 + wave) * 64 * VW),
                                             16, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            int k = k0 + b_k[r];
            k = k < K ? k : K - 1;
            __builtin_amdgcn_global_load_lds((const void*)(B + (long)k * P.b_ks + b_n[r]),
                                             (__attribute__((address_space(3))) void*)(bs + (r * 4 + wave) * 64 * VW),
                                             16, 0, 0);
        }
    };

    const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
    const int lg = lane >> 4, l16 = lane & 15;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int nk = K > kbeg ? (K - kbeg + BK - 1) / BK : 0;
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nk) issue(s, s);
    for (int kt = 0; kt < nk; ++kt) {
        const int ahead = nk - 1 - kt;  // tiles issued after this one
        wait_vm<NLD * 2>(ahead < NS - 2 ? ahead : NS - 2);
        const int stg = kt % NS;
        T* as = Sm + stg * (ASZ + BSZ);
        const T* bs = as + ASZ;
        const int k0 = kbeg + kt * BK;
        if (k0 + BK > K) {
            // tail tile: zero the A chunks of this lane that lie beyond K
#pragma unroll
            for (int r = 0; r < NLD; ++r)
                if (k0 + a_lk[r] >= K) {
                    v_t z = {};
                    *(v_t*)(as + (r * 4 + wave) * 64 * VW + lane * VW) = z;
                }
        }
        // plain s_barrier: the LDS-DMA loads this lane waited for above are in
        // LDS; a full __syncthreads fence would also drain the loads of the
        // stages still in flight
        __builtin_amdgcn_s_waitcnt((15 & 15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
        if (kt + NS - 1 < nk) issue(kt + NS - 1, (kt + NS - 1) % NS);
        BfOperand<BF> ha[FM], hb[FN];  // BF16 modes: the lane's 8 k values of this tile
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            v_t fa[FM];
            T fb[FN][VW];
#pragma unroll
            for (int a = 0; a < FM; ++a) {
                const int row = wm0 + a * 16 + l16;
                const int pc = (lg * NCH + ch) ^ (row & 7);
                fa[a] = *(const v_t*)(as + row * BK + pc * VW);
            }
#pragma unroll
            for (int tq = 0; tq < VW; ++tq) {
                const int k = lg * KPL + ch * VW + tq;
                const int sw = ((k / KPL) & 3) * BSW;
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    const int n = wn0 + b * 16 + l16;
                    fb[b][tq] = bs[k * BN + (((n / VW) ^ sw) * VW) + (n % VW)];
                }
            }
            if constexpr (BF) {
                // k = lg KPL + ch VW + tq for both operands (element ch VW + tq)
#pragma unroll
                for (int tq = 0; tq < VW; ++tq) {
#pragma unroll
                    for (int a = 0; a < FM; ++a) ha[a].set(ch * VW + tq, fa[a][tq]);
#pragma unroll
                    for (int b = 0; b < FN; ++b) hb[b].set(ch * VW + tq, fb[b][tq]);
                }
            } else {
#pragma unroll
                for (int tq = 0; tq < VW; ++tq)
#pragma unroll
                    for (int a = 0; a < FM; ++a)
#pragma unroll
                        for (int b = 0; b < FN; ++b)
                            acc[a][b] = Mfma<T>::step(fa[a][tq], fb[b][tq], acc[a][b]);
            }
        }
        if constexpr (BF) {
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(ha[a], hb[b], acc[a][b]);
        }
    }

    // ---- epilogue
    if constexpr (sizeof(T) == 4) {
        // FP32: the tile goes through LDS (the operand ring, free now) and
        // leaves as 16-byte row-order stores
        store_tile_staged<T, BM, BN, WM, FM, FN, NS * (ASZ + BSZ)>(P, Sm, acc, ks, split, m0, n0, wm0, wn0);
        return;
    }
    const T alpha = (T)P.alpha, beta = (T)P.beta;
    if (ks > 1) {
        T* __restrict__ W = (T*)P.ws + (long)split * M * N;
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int j = n0 + wn0 + b * 16 + l16;
            if (j >= N) continue;
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm0 + a * 16 + Mfma<T>::row(lane, r);
                    if (i < M) W[(long)i * N + j] = alpha * acc[a][b][r];
                }
        }
        return;
    }
    T* __restrict__ C = (T*)P.C;
#pragma unroll
    for (int b = 0; b < FN; ++b) {
        const int j = n0 + wn0 + b * 16 + l16;
        if (j >= N) continue;
        const long cj = (long)(j / P.c_cols0) * P.c_cs1 + (long)(j % P.c_cols0) * P.c_cs0;
#pragma unroll
        for (int a = 0; a < FM; ++a) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm0 + a * 16 + Mfma<T>::row(lane, r);
                if (i >= M) continue;
                const long off =
                    (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 + cj;
                T v = alpha * acc[a][b][r];
                if (beta != T(0)) v += beta * C[off];
                C[off] = v;
            }
        }
    }
}


// Panel kernel: the direct kernel's LDS-DMA ring and A layout, for problems
// with one side held whole in one tile (a k-column block of a subspace
// iteration against an n x n enlarged corner).  WGM = 4: a 64 x BN tile with
// the 4 waves stacked along M (16 x BN each); WGM = 1: a BM x 64 tile with
// the waves side by side along N (BM x 16 each).  BM and BN need not be
// powers of two: B chunks are rotated by 16 columns per reading lane group
// (the rows those groups read are KPL apart), and a stage's loads are padded
// to whole wave loads per wave (the surplus lands in a scratch area of the
// stage), so every wave issues the same count and vmcnt stays exact.
template <typename T, int BM, int BN, int BK, int WGM, int NS, int TAG, int BF = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_gemm_panel(const GemmProb* __restrict__ probs, int nprob) {
    static_assert(BF == 0 || BF == 1 || BF == 3, "BF: 0, 1 or 3 BF16 products");
    static_assert(!BF || (sizeof(T) == 4 && BK == 32), "BF16 modes: FP32 storage, k tiles of 32");
    static_assert(WGM == 4 || WGM == 1, "waves stacked along M or along N");
    constexpr int VW = 16 / (int)sizeof(T);
    constexpr int WGN = 4 / WGM;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int FM = WM / 16, FN = WN / 16;
    static_assert(FM * 16 * WGM == BM && FN * 16 * WGN == BN, "tiles of whole 16 x 16 blocks");
    constexpr int KPL = BK / 4;
    constexpr int NCH = KPL / VW;
    constexpr int ACH = BK / VW;  // 16-byte chunks per A row (8)
    static_assert(ACH == 8, "the A swizzle takes 8 chunks per row");
    constexpr int BCH = BN / VW;  // 16-byte chunks per B row
    constexpr int ROT = 16 / VW;  // B chunk rotation per reading lane group
    constexpr int ACHK = BM * ACH, BCHK = BK * BCH;  // chunks per stage
    static_assert(ACHK % 64 == 0 && BCHK % 64 == 0, "whole wave loads");
    constexpr int NLA = (ACHK + 255) / 256, NLB = (BCHK + 255) / 256;  // loads per lane and stage
    constexpr int ASZ = NLA * 256 * VW, BSZ = NLB * 256 * VW;             // padded stage areas
    static_assert(NS >= 2 && NS <= 4, "wait_vm covers up to 3 tiles in flight behind the current one");
    typedef typename Vec16<T>::v_t v_t;
    __shared__ __attribute__((aligned(16))) T Sm[NS * (ASZ + BSZ)];

    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int per = G >> 3, rem = G & 7;
    const int bid = xcd * per + (xcd < rem ? xcd : rem) + idx;
    int p = 0;
    while (p + 1 < nprob && probs[p + 1].tile_begin <= bid) ++p;
    const GemmProb& P = probs[p];
    if (P.gate && *P.gate == 0) return;
    const int ks = P.ksplit > 1 ? P.ksplit : 1;
    const int tt = bid - P.tile_begin;
    const int split = tt % ks, t = tt / ks;
    const int tm = t / P.tiles_n, tn = t - (t / P.tiles_n) * P.tiles_n;
    const int M = P.M, N = P.N;
    const int kchunk = ((P.K + ks - 1) / ks + BK - 1) / BK * BK;
    const int kbeg = split * kchunk;
    const int K = (kbeg + kchunk < P.K) ? kbeg + kchunk : P.K;
    const int m0 = tm * BM, n0 = tn * BN;
    const T* __restrict__ A = (const T*)P.A;
    const T* __restrict__ B = (const T*)P.B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // per-lane sources (fixed across k tiles); surplus chunks re-read chunk 0
    long a_src[NLA];
    int a_lk[NLA];
#pragma unroll
    for (int r = 0; r < NLA; ++r) {
        int c = (r * 4 + wave) * 64 + lane;
        c = c < ACHK ? c : lane;
        const int row = c / ACH;
        const int lchunk = (c % ACH) ^ (row & 7);
        int i = m0 + row;
        i = i < M ? i : M - 1;
        a_src[r] = (long)(i / P.a_rows0) * P.a_rs1 + (long)(i % P.a_rows0) * P.a_rs0;
        a_lk[r] = lchunk * VW;
    }
    int b_k[NLB], b_n[NLB];
#pragma unroll
    for (int r = 0; r < NLB; ++r) {
        int c = (r * 4 + wave) * 64 + lane;
        c = c < BCHK ? c : lane;
        const int k = c / BCH, slot = c % BCH;
        int gch = slot - ROT * ((k / KPL) & 3);
        gch = gch < 0 ? gch + BCH : gch;
        gch = gch < 0 ? gch + BCH : gch;
        int n = n0 + gch * VW;
        n = n < N ? n : N - VW;
        b_k[r] = k;
        b_n[r] = n;
    }
    auto issue = [&](int kt, int stg) {
        const int k0 = kbeg + kt * BK;
        T* as = Sm + stg * (ASZ + BSZ);
        T* bs = as + ASZ;
#pragma unroll
        for (int r = 0; r < NLA; ++r) {
            int k = k0 + a_lk[r];
            k = k < K ? k : K - VW;
            __builtin_amdgcn_global_load_lds((const void*)(A + a_src[r] + k),
                                             (__attribute__((address_space(3))) void*)(as + (r * 4 + wave) * 64 * VW),
                                             16, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < NLB; ++r) {
            int k = k0 + b_k[r];
            k = k < K ? k : K - 1;
            __builtin_amdgcn_global_load_lds((const void*)(B + (long)k * P.b_ks + b_n[r]),
                                             (__attribute__((address_space(3))) void*)(bs + (r * 4 + wave) * 64 * VW),
                                             16, 0, 0);
        }
    };

    const int wm0 = WGM == 4 ? wave * WM : 0, wn0 = WGM == 4 ? 0 : wave * WN;
    const int lg = lane >> 4, l16 = lane & 15;
    // B read offsets of this lane's columns (the rotation depends on lg only)
    int b_off[FN];
#pragma unroll
    for (int b = 0; b < FN; ++b) {
        const int n = wn0 + b * 16 + l16;
        int slot = n / VW + ROT * lg;
        slot = slot < BCH ? slot : slot - BCH;
        slot = slot < BCH ? slot : slot - BCH;
        b_off[b] = slot * VW + n % VW;
    }
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int nk = K > kbeg ? (K - kbeg + BK - 1) / BK : 0;
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nk) issue(s, s);
    for (int kt = 0; kt < nk; ++kt) {
        const int ahead = nk - 1 - kt;  // tiles issued after this one
        wait_vm<NLA + NLB>(ahead < NS - 2 ? ahead : NS - 2);
        const int stg = kt % NS;
        T* as = Sm + stg * (ASZ + BSZ);
        const T* bs = as + ASZ;
        const int k0 = kbeg + kt * BK;
        if (k0 + BK > K) {
            // tail tile: zero the A chunks of this lane that lie beyond K
#pragma unroll
            for (int r = 0; r < NLA; ++r)
                if (k0 + a_lk[r] >= K) {
                    v_t z = {};
                    *(v_t*)(as + (r * 4 + wave) * 64 * VW + lane * VW) = z;
                }
        }
        __builtin_amdgcn_s_waitcnt((15 & 15) | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
        if (kt + NS - 1 < nk) issue(kt + NS - 1, (kt + NS - 1) % NS);
        BfOperand<BF> ha[FM], hb[FN];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            v_t fa[FM];
            T fb[FN][VW];
#pragma unroll
            for (int a = 0; a < FM; ++a) {
                const int row = wm0 + a * 16 + l16;
                const int pc = (lg * NCH + ch) ^ (row & 7);
                fa[a] = *(const v_t*)(as + row * BK + pc * VW);
            }
#pragma unroll
            for (int tq = 0; tq < VW; ++tq) {
                const int k = lg * KPL + ch * VW + tq;
#pragma unroll
                for (int b = 0; b < FN; ++b) fb[b][tq] = bs[k * BN + b_off[b]];
            }
            if constexpr (BF) {
#pragma unroll
                for (int tq = 0; tq < VW; ++tq) {
#pragma unroll
                    for (int a = 0; a < FM; ++a) ha[a].set(ch * VW + tq, fa[a][tq]);
#pragma unroll
                    for (int b = 0; b < FN; ++b) hb[b].set(ch * VW + tq, fb[b][tq]);
                }
            } else {
#pragma unroll
                for (int tq = 0; tq < VW; ++tq)
#pragma unroll
                    for (int a = 0; a < FM; ++a)
#pragma unroll
                        for (int b = 0; b < FN; ++b)
                            acc[a][b] = Mfma<T>::step(fa[a][tq], fb[b][tq], acc[a][b]);
            }
        }
        if constexpr (BF) {
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) acc[a][b] = mfma_bf16(ha[a], hb[b], acc[a][b]);
        }
    }

    // ---- epilogue (as the direct kernel)
    const T alpha = (T)P.alpha, beta = (T)P.beta;
    if (ks > 1) {
        T* __restrict__ W = (T*)P.ws + (long)split * M * N;
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int j = n0 + wn0 + b * 16 + l16;
            if (j >= N) continue;
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm0 + a * 16 + Mfma<T>::row(lane, r);
                    if (i < M) W[(long)i * N + j] = alpha * acc[a][b][r];
                }
        }
        return;
    }
    T* __restrict__ C = (T*)P.C;
#pragma unroll
    for (int b = 0; b < FN; ++b) {
        const int j = n0 + wn0 + b * 16 + l16;
        if (j >= N) continue;
        const long cj = (long)(j / P.c_cols0) * P.c_cs1 + (long)(j % P.c_cols0) * P.c_cs0;
#pragma unroll
        for (int a = 0; a < FM; ++a) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = m0 + wm0 + a * 16 + Mfma<T>::row(lane, r);
                if (i >= M) continue;
                const long off =
                    (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 + cj;
                T v = alpha * acc[a][b][r];
                if (beta != T(0)) v += beta * C[off];
                C[off] = v;
            }
        }
    }
}

// C = sum over splits (fixed order) + beta C, with C's two-level indexing.
template <typename T>
__global__ __launch_bounds__(256) void k_splitk_reduce(const GemmProb* __restrict__ probs) {
    const GemmProb& P = probs[blockIdx.y];
    if (P.ksplit <= 1 || (P.gate && *P.gate == 0)) return;
    const long MN = (long)P.M * P.N;
    const T* W = (const T*)P.ws;
    T* C = (T*)P.C;
    const T beta = (T)P.beta;
    const int ks = P.ksplit;
    typedef typename Vec16<T>::v_t v_t;
    constexpr int VW = 16 / (int)sizeof(T);
    if (MN >= 65536 && P.N % VW == 0 && ((uintptr_t)W & 15) == 0) {
        // one 16-byte vector of a row per thread (MN is a multiple of VW, so
        // every split's partial stays aligned); the same additions per
        // element.  Small sums (the k x k Grams) keep one element per thread:
        // more loads in flight
        const bool vec = P.c_cs0 == 1 && P.c_cols0 % VW == 0 && P.c_cs1 % VW == 0 && P.c_rs0 % VW == 0 &&
                         P.c_rs1 % VW == 0 && ((uintptr_t)C & 15) == 0;
        for (long e = ((long)blockIdx.x * blockDim.x + threadIdx.x) * VW; e < MN;
             e += (long)gridDim.x * blockDim.x * VW) {
            const T* __restrict__ w = W + e;
            v_t v = *(const v_t*)w;
            for (int sp = 1; sp < ks; sp += 8) {
                v_t x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = sp + u < ks ? *(const v_t*)(w + (long)(sp + u) * MN) : v_t{};
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (sp + u < ks) v += x[u];
            }
            const int i = (int)(e / P.N), j0 = (int)(e % P.N);
            if (vec) {
                const long off = (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 +
                                 (long)(j0 / P.c_cols0) * P.c_cs1 + (long)(j0 % P.c_cols0);
                if (beta != T(0)) v += beta * *(const v_t*)(C + off);
                *(v_t*)(C + off) = v;
            } else {
#pragma unroll
                for (int q = 0; q < VW; ++q) {
                    const int j = j0 + q;
                    const long off = (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 +
                                     (long)(j / P.c_cols0) * P.c_cs1 + (long)(j % P.c_cols0) * P.c_cs0;
                    T y = v[q];
                    if (beta != T(0)) y += beta * C[off];
                    C[off] = y;
                }
            }
        }
        return;
    }
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < MN; e += (long)gridDim.x * blockDim.x) {
        // the partials are loaded eight at a time, then added in split order
        const T* __restrict__ w = W + e;
        T v = w[0];
        for (int sp = 1; sp < ks; sp += 8) {
            T x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = sp + u < ks ? w[(long)(sp + u) * MN] : T(0);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (sp + u < ks) v += x[u];
        }
        const int i = (int)(e / P.N), j = (int)(e % P.N);
        const long off = (long)(i / P.c_rows0) * P.c_rs1 + (long)(i % P.c_rows0) * P.c_rs0 +
                         (long)(j / P.c_cols0) * P.c_cs1 + (long)(j % P.c_cols0) * P.c_cs0;
        if (beta != T(0)) v += beta * C[off];
        C[off] = v;
    }
}

// panel tiles: np in 80..128, skinny M or N
template <typename T, int BK, int TAG, int BF>
static void launch_panel(hipStream_t stream, GemmTile tile, const GemmProb* d_probs, int nprob, dim3 grid) {
    dim3 block(256);
    const int np = 16 * ((tile - TILE_PANEL) % 16);
    const bool sm = (tile - TILE_PANEL) >= 16;
#define IPEPS_PANEL(NP)                                                                                   \
    if (np == NP) {                                                                                       \
        if (sm)                                                                                           \
            hipLaunchKernelGGL((k_gemm_panel<T, NP, 64, BK, 1, 2, TAG, BF>), grid, block, 0, stream, d_probs, \
                               nprob);                                                                    \
        else                                                                                              \
            hipLaunchKernelGGL((k_gemm_panel<T, 64, NP, BK, 4, 2, TAG, BF>), grid, block, 0, stream, d_probs, \
                               nprob);                                                                    \
        return;                                                                                           \
    }
    IPEPS_PANEL(80)
    IPEPS_PANEL(96)
    IPEPS_PANEL(112)
    IPEPS_PANEL(128)
#undef IPEPS_PANEL
    IPEPS_REQUIRE(false, IPEPS_EINVAL, "gemm: no panel kernel of this width");
}

template <int TAG, int BF>
static void launch_f32(hipStream_t stream, GemmTile tile, const GemmProb* d_probs, int nprob, dim3 grid) {
    dim3 block(256);
    if constexpr (TAG == 0)  // (panel tiles never carry the cut products)
        if (is_panel(tile)) return launch_panel<float, 32, TAG, BF>(stream, tile, d_probs, nprob, grid);
    if (tile == TILE_DIRECT)
        hipLaunchKernelGGL((k_gemm_direct<float, 128, 128, 32, 2, TAG, BF>), grid, block, 0, stream, d_probs,
                           nprob);
    else if (tile == TILE_DIRECT_SMALL)
        hipLaunchKernelGGL((k_gemm_direct<float, 64, 64, 32, 2, TAG, BF>), grid, block, 0, stream, d_probs,
                           nprob);
    else if (tile == TILE_LARGE)
        hipLaunchKernelGGL((k_gemm_grouped<float, 128, 128, 32, TAG, BF>), grid, block, 0, stream, d_probs,
                           nprob);
    else
        hipLaunchKernelGGL((k_gemm_grouped<float, 64, 64, 32, TAG, BF>), grid, block, 0, stream, d_probs,
                           nprob);
}

template <int TAG>
static void launch_tagged(hipStream_t stream, int dtype, GemmTile tile, const GemmProb* d_probs,
                          int nprob, dim3 grid) {
    dim3 block(256);
    if (dtype == IPEPS_DTYPE_BF16) return launch_f32<TAG, 1>(stream, tile, d_probs, nprob, grid);
    if (dtype == IPEPS_DTYPE_BF16X3) return launch_f32<TAG, 3>(stream, tile, d_probs, nprob, grid);
    if (dtype != IPEPS_DTYPE_FP64) return launch_f32<TAG, 0>(stream, tile, d_probs, nprob, grid);
    if constexpr (TAG == 0)
        if (is_panel(tile)) return launch_panel<double, 16, TAG, 0>(stream, tile, d_probs, nprob, grid);
    if (tile == TILE_DIRECT)
        hipLaunchKernelGGL((k_gemm_direct<double, 128, 128, 16, 2, TAG>), grid, block, 0, stream, d_probs,
                           nprob);
    else if (tile == TILE_DIRECT_SMALL)
        hipLaunchKernelGGL((k_gemm_direct<double, 64, 64, 16, 2, TAG>), grid, block, 0, stream, d_probs,
                           nprob);
    else if (tile == TILE_LARGE)
        hipLaunchKernelGGL((k_gemm_grouped<double, 128, 128, 16, TAG>), grid, block, 0, stream, d_probs,
                           nprob);
    else
        hipLaunchKernelGGL((k_gemm_grouped<double, 64, 64, 16, TAG>), grid, block, 0, stream, d_probs,
                           nprob);
}

void gemm_launch(hipStream_t stream, int dtype, GemmTile tile, const GemmProb* d_probs,
                 int nprob, int total_tiles, int tag, long reduce_elems) {
    if (total_tiles <= 0) return;
    dim3 grid(total_tiles);
    if (tag == 1)
        launch_tagged<1>(stream, dtype, tile, d_probs, nprob, grid);
    else
        launch_tagged<0>(stream, dtype, tile, d_probs, nprob, grid);
    if (reduce_elems > 0) {
        const int gx = ceil_div(reduce_elems, 256) < 1024 ? ceil_div(reduce_elems, 256) : 1024;
        if (dtype == IPEPS_DTYPE_FP64)
            hipLaunchKernelGGL(k_splitk_reduce<double>, dim3(gx, nprob), dim3(256), 0, stream, d_probs);
        else
            hipLaunchKernelGGL(k_splitk_reduce<float>, dim3(gx, nprob), dim3(256), 0, stream, d_probs);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace ipeps
