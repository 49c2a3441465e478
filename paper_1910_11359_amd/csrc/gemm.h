// Grouped MFMA GEMM: C = alpha * A B + beta * C for a list of problems of
// one dtype, all tiles of all problems in one launch.
#pragma once

#include "common.h"

namespace ipeps {

// Element (i, k) of A lives at A[(i / a_rows0) * a_rs1 + (i % a_rows0) * a_rs0 + k * a_ks]
// (a two-level row index lets a tensor with two free legs on either side of
// the contracted ones be read in place); B(k, j) at B[k * b_ks + j * b_cs];
// C(i, j) at C[(i / c_rows0) * c_rs1 + (i % c_rows0) * c_rs0
//            + (j / c_cols0) * c_cs1 + (j % c_cols0) * c_cs0].
// beta == 0 never reads C.
struct GemmProb {
    const void* A;
    const void* B;
    void* C;
    int M, N, K;
    int a_rows0;
    long a_rs1, a_rs0, a_ks;
    long b_ks, b_cs;
    int c_rows0, c_cols0;
    long c_rs1, c_rs0, c_cs1, c_cs0;
    double alpha, beta;
    int ksplit;      // > 1: K is split over this many workgroups per tile, whose
    void* ws;        //   partial products go to ws[split][M][N] (row-major, dtype)
                     //   and are summed in a fixed order by a second kernel
    int tiles_n;     // filled by gemm_plan_tiles
    int tile_begin;  // first tile of this problem within its launch
    const int* gate; // not null: the problem is skipped while *gate == 0
};

// Plain row-major helpers: op(X) = X (lda = row stride) or X^T.
GemmProb gemm_nn(const void* A, long lda, const void* B, long ldb, void* C, long ldc, int M,
                 int N, int K, double alpha = 1.0, double beta = 0.0);
GemmProb gemm_general(const void* A, bool transA, long lda, const void* B, bool transB,
                      long ldb, void* C, long ldc, int M, int N, int K, double alpha = 1.0,
                      double beta = 0.0);

// TILE_DIRECT / TILE_DIRECT_SMALL: 128 x 128 / 64 x 64 tiles loaded straight
// into LDS (16-byte LDS-DMA); chosen instead of TILE_LARGE / TILE_SMALL when
// every problem of the group has A with k contiguous and B with n contiguous,
// 16-byte aligned, with K and N (and the A row strides, B k stride) multiples
// of the 16-byte vector.
//
// Panel tiles (TILE_PANEL + 16 m + np / 16): every problem of the group has
// one side of at most 128 (the columns of a subspace block), padded to
// np = 80, 96, 112 or 128 and held whole in one tile: m = 0, N <= np, tiles
// of 64 x np (4 waves stacked along M); m = 1, M <= np, tiles of np x 64
// (4 waves side by side along N).  Same operand layouts as the direct tiles.
enum GemmTile {
    TILE_LARGE = 0,
    TILE_SMALL = 1,
    TILE_DIRECT = 2,
    TILE_DIRECT_SMALL = 3,
    TILE_PANEL = 64,
    TILE_PANEL_LAST = TILE_PANEL + 16 + 8
};
inline GemmTile panel_tile(bool skinny_m, int np) { return (GemmTile)(TILE_PANEL + (skinny_m ? 16 : 0) + np / 16); }
inline bool is_panel(GemmTile t) { return t >= TILE_PANEL; }

// The panel tile for a group (all problems thin on the same side, with the
// same padded width in 80..128, operands as the direct tiles need them), or
// -1.
int gemm_panel_for(const GemmProb* probs, int n, int dtype);

// Chooses the tile shape for a group by a size heuristic and fills tiles_n /
// tile_begin; returns the total number of tiles (the grid size).
int gemm_plan_tiles(GemmProb* probs, int n, int dtype, GemmTile* tile);

// Tile kinds that can run the group (at most 5; the direct and panel ones
// only where the operand layout allows them); returns their number.
int gemm_tile_candidates(const GemmProb* probs, int n, int dtype, GemmTile* out);

// Fills tiles_n / tile_begin for a given tile kind; returns the total tiles.
int gemm_plan_with(GemmProb* probs, int n, int dtype, GemmTile tile);

// Launch on `stream`; d_probs is a device copy of the planned descriptors.
// tag 1 selects a separate kernel symbol for the cut products (profiling).
// reduce_elems > 0 (largest M*N of a split problem) adds the split-K sum.
void gemm_launch(hipStream_t stream, int dtype, GemmTile tile, const GemmProb* d_probs,
                 int nprob, int total_tiles, int tag = 0, long reduce_elems = 0);

}  // namespace ipeps
