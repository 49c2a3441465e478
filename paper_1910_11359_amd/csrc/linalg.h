// Small dense FP64 linear algebra on the device: one workgroup per matrix.
// The batched routines also take a JobMap: `batch` matrices for each of
// jm.njobs jobs of one buffer layout (common.h), in one launch.
#pragma once

#include "common.h"

namespace ipeps {

// Batched one-sided (Hestenes) Jacobi SVD of real m x n matrices, n <= m <= 256.
// Matrix b is read from A + b*strideA with element (i, j) at [i*lda + j]
// (row-major).  Outputs, sorted by descending singular value:
//   sigma[b*n + j], U (m x n, row-major ld n, b*m*n) with unit columns (zero
//   for zero singular values), V (n x n row-major, b*n*n) with A = U S V^T.
// U and V may be NULL.  Columns whose norm falls below skip_rel * |A|_F are
// not rotated (their singular values are then known to that absolute
// level).  Works in LDS when m*n + n*n + 2n doubles fit, else in `work`
// (device scratch of jacobi_svd_real_work doubles).
void jacobi_svd_real(hipStream_t s, int batch, int m, int n, const double* A, long lda,
                     long strideA, double* sigma, double* U, double* V, double* work,
                     double skip_rel = 1e-14, JobMap jm = JobMap());
size_t jacobi_svd_real_work(int batch, int m, int n);

// Batched Cholesky of k x k SPD Gram matrices G (row-major, stride k*k, k <= 256) with
// dependency dropping, followed by the inverse of the factor: on exit
// Rinv[b] holds R^{-1} (upper triangular, G = R^T R) with the rows/columns of
// dropped pivots set to zero.  The factorisation runs on G scaled to unit
// diagonal, G' = D^{-1} G D^{-1} = R'^T R' with D = diag(sqrt(G_ii)) (rows
// with G_ii <= 0 are zero), so a pivot is dropped when the Schur diagonal of
// G' is <= tol; R^{-1} = D^{-1} R'^{-1}.  X Rinv thus equals normalising the
// columns of X before taking the Gram.  If dead is not null
// (batch*k + batch ints), dead[b*k + j] is set to 1 for a dropped column j
// and 0 otherwise, and dead[batch*k + b] to the number of dropped columns.
// near_identity > 0: a matrix whose scaled Gram G' has every off-diagonal
// |G'_ij| <= near_identity and no zero diagonal skips the factorisation and
// gets R^{-1} = D^{-1} (the second pass of a Cholesky QR, whose first pass
// already left the columns orthonormal to that level).
void chol_inverse(hipStream_t s, int batch, int k, const double* G, double* Rinv, double tol,
                  int* dead = nullptr, double near_identity = 0.0, JobMap jm = JobMap());

// Scale the columns of batched n x k row-major matrices (stride n*k) to unit
// 2-norm; zero columns stay zero.
void normalize_columns(hipStream_t s, int batch, int n, int k, double* X);

// R (batched n x k row-major, flags as written by chol_inverse): column j
// uniform in [-1, 1) from a counter hash of (seed, element) where
// dead[b*k + j] != 0, zero elsewhere; matrices with no dropped column are
// left untouched.  The seed comes from ctr = {config seed, calls} on the
// device (seed * C1 + C2 * (calls + 1)), and the call count is advanced
// afterwards (once per call, for every job of jm).
void dead_fill(hipStream_t s, int batch, int n, int k, const int* dead, uint64_t* ctr, double* R,
               JobMap jm = JobMap());

// X_b[e] += Y_b[e] for e < count, for the batches b with gate[b] != 0
// (matrix b at offset b*count), for every job of jm.
void add_gated(hipStream_t s, int batch, long count, const int* gate, const double* Y, double* X,
               JobMap jm = JobMap());

}  // namespace ipeps
