// CTMRG support kernels: double layer in the Hermitian (real) basis, frame
// layouts, cold environment, permutations, norms, spectra and readout.
#pragma once

#include "common.h"

namespace ipeps {

// A = Gamma with sqrt(lambda) on its four legs, for the 4 sites.
void absorb_sqrt_lambda(hipStream_t s, int D, int d, const cplx* gam, const double* lam,
                        cplx* A);

// Double layer of each site in the real basis: a[m_u][m_l][m_d][m_r] (FP64),
// up/left legs in the basis {H_m}, down/right legs in {H_m^T}, where for the
// pair (k, k') of a leg, m = k*D + k' and H_m = E_kk (k = k'),
// (E_kk' + E_k'k)/sqrt2 (k < k'), i(E_kk' - E_k'k)/sqrt2 (k > k').
void double_layer_real(hipStream_t s, int D, int d, const cplx* A, double* a_base);

// Frame copies: for site s and rotation g, out_lu[s][g] = rot^g(a) stored as
// [L][U][D][R] and out_dl[s][g] stored as [D][L][R][U] (frame legs), in the
// CTMRG dtype.  rot^g maps frame leg F to physical leg (F - g) mod 4.
void frame_layouts(hipStream_t s, int q, int dtype, const double* a_base, void* const* out_lu,
                   void* const* out_dl);

// Cold environment: every C/T of every site is its neighbour's double layer
// with the outward legs closed by the identity (diagonal basis elements),
// embedded in chi.  C[(site*4 + k) * chi^2], T[(site*4 + k) * chi*q*chi].
void init_environment(hipStream_t s, int D, int chi, int dtype, const double* a_base, void* C,
                      void* T);

// out[b][c][r] = in[b][r][c] for b < batch (rows R, cols Cc), dtype elements.
void batched_transpose(hipStream_t s, int dtype, int batch, int R, int Cc, const void* in,
                       void* out);

// Rank-3 permutations of small tensors (dtype elements):
//   mode 0: out[b][a][c] = in[a][b][c];  mode 1: out[a][c][b] = in[a][b][c];
//   mode 2: out[c][a][b] = in[a][b][c]
// With a JobMap (njobs > 1): the same permutation for every job (grid rows).
// Independent permute3 copies (same modes and index meaning) in one launch.
constexpr int kPermuteBatch = 6;
struct Permute3Batch {
    int n;
    int mode[kPermuteBatch], A[kPermuteBatch], B[kPermuteBatch], C[kPermuteBatch];
    const void* in[kPermuteBatch];
    void* out[kPermuteBatch];
};
void permute3_batch(hipStream_t s, int dtype, const Permute3Batch& pb, JobMap jm);
void permute3(hipStream_t s, int dtype, int mode, int A, int B, int C, const void* in, void* out,
              JobMap jm = JobMap());

// Divide each of the n tensors of d_items by its Frobenius norm (accumulated
// in FP64, deterministic order); ws holds normalize_ws_doubles(n) doubles.
struct NormItem {
    void* ptr;
    long count;
};
size_t normalize_ws_doubles(int max_items);
void normalize_tensors(hipStream_t s, int dtype, const NormItem* d_items, int n, double* ws);

// Convert between dtype and FP64 (to_fp64: for every job of jm; out2, if
// not NULL, receives a second copy).
void to_fp64(hipStream_t s, int dtype, const void* in, double* out, long count, JobMap jm = JobMap(),
             double* out2 = nullptr);
void from_fp64(hipStream_t s, int dtype, const double* in, void* out, long count);
// FP64 rows x cols blocks (row-major, batch of them back to back) into dtype,
// as they are (rows x cols) or transposed (cols x rows); LDS-tiled.
void from_fp64_blocks(hipStream_t s, int dtype, const double* in, void* out, int batch, int rows,
                      int cols, bool transpose, JobMap jm = JobMap());

// Device-to-device copy of `bytes` for every job of jm (one launch).
void copy_jobs(hipStream_t s, void* dst, const void* src, size_t bytes, JobMap jm);

// Projector factors from an SVD of the cut matrix: the truncation rule on
// sigma (k values, descending; values <= tau * s_1 count as zero, multiplets
// within 1e-10 of the larger plus tau s_1 are kept whole) picks g <= chi;
// Vs[i][c] = V[i][c]/sqrt(s_c) (n x chi) and, transposed, Us[c][i] =
// U[i][c]/sqrt(s_c) (chi x n) for c < g, zero for g <= c < chi (dtype).
// U and V are n x k row-major (ld k).  g_out[b] receives g.
void projector_factors(hipStream_t s, int dtype, int batch, int n, int k, int chi, double tau,
                       const double* U, const double* V, const double* sigma, long strideUV,
                       void* Us, void* Vs, long strideP, int* g_out, JobMap jm = JobMap());
// Two projector_factors calls with the same k, chi, tau and singular values
// in one launch; Us[i] and g_out[i] may be NULL (not written).
struct ProjFactorsPair {
    int n[2];
    const double* U[2];
    const double* V[2];
    long strideUV[2];
    void* Us[2];
    void* Vs[2];
    long strideP[2];
    int* g_out[2];
};
void projector_factors_pair(hipStream_t s, int dtype, int batch, int k, int chi, double tau,
                            const double* sigma, const ProjFactorsPair& pp, JobMap jm = JobMap());

// Normalised corner spectra (16 x chi) from raw singular values; delta_out =
// max over corners of |s - s_prev|_2; prev <- current.
void spectra_delta(hipStream_t s, int nspec, int chi, const double* sig, double* spectra,
                   double* prev, double* delta_out, int first, JobMap jm = JobMap());

// Random n x k starting block (seeded counter-based uniforms in [-1, 1)).
void random_block(hipStream_t s, int batch, int n, int k, uint64_t seed, double* X);

// One-site reduced density matrices from the site environments E (real
// basis, [L][U][R][D] each q^4, FP64) and A; writes rho (4 x d x d complex,
// trace-normalised) and obs[0..15] = n[4], imbalance, sum_n, max_offdiag, 0,
// Renyi S_1[4], S_1/2[4] of the physical one-site matrix (natural log).
// Twork: 4 * D^4 * d complex scratch.
void readout(hipStream_t s, int D, int d, int d_A, const double* E, const cplx* A, cplx* Twork,
             cplx* rho, double* obs);

}  // namespace ipeps
