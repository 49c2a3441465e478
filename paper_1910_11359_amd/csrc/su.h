// Simple-update kernels: Trotter gates and per-layer bond updates (FP64).
#pragma once

#include "common.h"

namespace ipeps {

// One bond of a layer.  Sites are numbered x + 2y; lambda vectors are
// numbered h(x,y) = x + 2y and v(x,y) = 4 + x + 2y.  Leg positions inside a
// site tensor [s][up][left][down][right] are 1..4.
struct BondDesc {
    int site_i, site_j;
    int leg_i, leg_j;    // bond leg of i (right or down) and of j (left or up)
    int lam_b;           // the bond's lambda
    int outer_i[3];      // lambda index of i's other legs, in leg order
    int outer_j[3];
};

struct LayerDesc {
    BondDesc bond[2];
    int gate;  // index into the gate table (layer * 2 + (tau == dt ? 1 : 0))
};

// Build h_bond for each of the 4 layers and G = exp(-i tau h) for tau in
// {dt/2, dt}: gates[(layer*2 + t) * d^4] complex, row (s_i*d + s_j).
void build_gates(hipStream_t s, const ipeps_config& cfg, cplx* gates);

// Scratch (bytes) one bond update needs.
size_t su_scratch_bytes(int D, int d);

// Apply one layer: both bonds in parallel (one workgroup each), for every
// job of jm (a row of workgroups per job).
//   gam: 4 * d * D^4 complex; lam: 8 * D; eps: 4.
void su_layer(hipStream_t s, int D, int d, const LayerDesc& L, cplx* gam, double* lam,
              double* eps, const cplx* gates, void* scratch, JobMap jm = JobMap());

}  // namespace ipeps
