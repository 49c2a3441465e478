// Internal state of one iPEPS job and its device-side execution plan.
#pragma once

#include <vector>

#include "common.h"
#include "gemm.h"
#include "su.h"
#include "ctm.h"

namespace ipeps {

// Device allocations of one state, through the caller's hooks or hipMalloc.
// In dry mode nothing is allocated and only the byte count is summed (the
// footprint used for admission is exactly what a real state allocates).
struct DevMem {
    ipeps_alloc_fn alloc = nullptr;
    ipeps_free_fn free_fn = nullptr;
    void* ctx = nullptr;
    hipStream_t stream = nullptr;
    bool dry = false;
    size_t total = 0;
    std::vector<void*> ptrs;
    void* get(size_t bytes);
    void release();
};

// A group of GEMM problems launched together (a slice of the plan table).
struct GemmGroup {
    int first = 0, count = 0, dtype = 0, tiles = 0;
    GemmTile tile = TILE_LARGE;
    int tag = 0;       // 1: the n^3 half-system products (own kernel symbol)
    long reduce_elems = 0;  // largest M*N of a split-K problem (0: none)
    double flops = 0;  // algorithmic flops of the whole launch
    double bytes = 0;  // algorithmic bytes: every operand read once, the result written once
};

struct ColumnStep {
    // half, nprod: the cut matrix formed explicitly (ipeps_state::factored
    // false); otherwise it is applied in factored form and proj2 finishes
    // the projectors (P_low = E0 (E1 Vs), P_up = (Us^T E2) E3)
    GemmGroup s1, s2, s3, half, nprod, proj, proj2, w1, w2, fin;
    // second column of a move (X = 1): its UR and DR enlarged corners read
    // only tensors the move leaves alone; the first column step enqueues
    // them on the aux stream (into X1p_aux, X2p_aux, their E slots) to fill the idle
    // phases of its projector SVD
    GemmGroup aux_s1, aux_s2, aux_s3;
    // left move, first column: the variant for later iterations of one call,
    // which reuses the corners of types 0 and 1 the down move left valid
    GemmGroup s1w, s2w, s3w;
    // buffers the step touches
    int site_x[2], site_x1[2];  // physical site of frame (X, Y) and (X+1, Y)
    void* t4[2];                 // T4(X, Y), [chi][q][chi], permuted into T4p[Y] before w1
    int slot;                    // warm-subspace slot (frame * 2 + X)
    long norm_first;             // index of the 6 NormItems in the table
};

struct SvdPlan {
    // N V and N^T Q through the four enlarged corners of each cut
    // (N = E2 E3 E0 E1), one product per group, in dtype; orth passes on Y
    // and Z and the Rayleigh-Ritz products, batch 2 (FP64)
    GemmGroup NV[8][4], NtQ[8][4];  // [column step][factor]
    GemmGroup NVf, NtQf;  // the same with the formed N64
    GemmGroup PlowT2;     // factored path: P_low = (E0 E1 Qz) (Uc S^-1/2)
    GemmGroup gramY, gramZ, gramQ, gramQz, QfromY, QfromZ, YfromQ, ZfromQz, Cs;
    GemmGroup UoVo[8];  // [column step]: Vo goes to that step's warm-start slot
    // restart of dropped left columns: Gm = Qw^T Rb, Rb -= Qw Gm
    GemmGroup projQw1, projQw2;

};

}  // namespace ipeps

struct ipeps_state {
    ipeps_config cfg;
    int D, d, q, chi, n, k, dtype;
    int mma;  // arithmetic of the environment contractions (dtype, or BF16 on FP32 tensors)
    bool factored;  // cut matrices applied through their factors (else formed)
    size_t esz;
    hipStream_t stream;
    // The simple update runs on its own stream so that the Trotter step t+1
    // overlaps the CTMRG of step t: su_stream waits for ev_gamma_free (the
    // double layer of the last CTMRG has read Gamma), the main stream waits
    // for ev_su_done before it reads Gamma again.
    hipStream_t su_stream;
    hipEvent_t ev_gamma_free, ev_su_done;
    // corner spectra run on their own stream, overlapping the next iteration
    hipStream_t spec_stream;
    hipEvent_t ev_c64_ready, ev_spec_done;
    // enlarged corners of the second column step of a move, computed ahead
    hipStream_t aux_stream;
    hipEvent_t ev_aux_go, ev_aux_done;
    int aux_defer = -1;  // >= 0: column step whose corners-ahead launch waits for its Rayleigh-Ritz SVD
    hipEvent_t ev_side_go;  // main stream at the second column step's Rayleigh-Ritz SVD: spectra and readout start
    // asynchronous readout (ipeps_observe_async): C, T, A and the truncation
    // errors are copied on the main stream, then read out on ro_stream with
    // scratch of its own while the main stream goes on
    hipStream_t ro_stream;
    hipEvent_t ev_ro_snap, ev_ro_done;
    bool ro_pending;
    bool ro_deferred;  // snapshot taken, readout kernels not yet enqueued
    bool corners_warm;  // corner slots valid from the previous iteration of this call
    bool spec_deferred, spec_first;  // corner spectra waiting to be enqueued
    // the main stream is being captured into a graph: waits on events
    // recorded before the capture are made before the graph's launch instead
    bool capturing;
    double ro_t;
    int ro_iters;
    double* jwork_c;
    double* eps_snap;  // truncation errors as of the last double-layer build
    double* eps_snap_pre;  // the same for the layers built ahead on the SU stream
    long ctm_step;     // Trotter steps contained in the current environment
    ipeps::DevMem mem;

    // simple update
    ipeps::cplx* gam;
    double* lam;
    double* eps;
    ipeps::cplx* gates;
    void* su_scratch;
    ipeps::LayerDesc layers[7];

    // double layers
    ipeps::cplx* A;
    double* a_base;
    // A and a_base of the state after the last Trotter step, built at the tail
    // of the simple update (SU stream); swapped with A, a_base by the next
    // CTMRG when pre_step == step_count
    ipeps::cplx* A_pre;
    double* a_base_pre;
    bool pre_valid;
    long pre_step;
    void* a_lu[16];
    void* a_dl[16];
    void** d_a_lu;
    void** d_a_dl;
    // the same 32 frame copies as two contiguous blocks: the live one the
    // plan reads and the one the simple update fills for the next CTMRG
    void* frames;
    void* frames_pre;
    void* a_lu_pre[16];
    void* a_dl_pre[16];
    void** d_a_lu_pre;
    void** d_a_dl_pre;

    // environment: C[(site*4 + k)], T[(site*4 + k)] contiguous
    void* Cenv;
    void* Tenv;

    // snapshot and scratch of the asynchronous readout
    void *Csnap, *Tsnap, *X1r, *X2r, *X2pr, *Er, *Eout_r;
    ipeps::cplx *Asnap, *rho_T_r, *rho_r;
    double *eps_r, *E64_r, *obs_r;
    ipeps::GemmGroup read1r, read2r, read3r, read4r;

    // column-step workspace
    void* X1;   // 8 blocks of chi * q * chi
    void* X1p;  // the same with columns (c, v) for v in q: [chi][chi][q]
    void* T4p;  // 2 blocks of chi * chi * q
    void* X2;   // 8 blocks of n^2
    void* X2p;  // 8 blocks of n^2
    // enlarged corners, one n^2 slot per (site, corner index g), kept across
    // the moves of an iteration (blocks 0..7 are readout scratch)
    void* E;
    // UR, DR corners of the second column step: 4 blocks each ([Y][j - 1])
    void* X1p_aux;
    void* X2p_aux;
    // cut matrices formed (not factored) only:
    void* Fh;   // 2 blocks of n^2
    void* Gh;   // 2 blocks of n^2
    void* Nd;   // 2 blocks of n^2 (dtype; aliases N64 in FP64 mode)
    double* N64;
    void* Z;    // 2 blocks of chi*q*chi
    void* Us;   // 2 blocks of n*chi
    void* Vs;
    void* Plow;
    void* Pup;
    void* PlowP;
    void* PupP;
    void* W1p;
    void* W2;
    int* g_dev;

    // projector SVD (FP64)
    double* warm;  // 16 slots of n*k
    bool warm_valid[16];
    double *Yw, *Zw, *Qw, *Qz, *Gm, *Ri, *Cs, *Uc, *Vc, *sig, *Uo, *Vo, *jwork;
    double* Rb;          // 2 blocks of n*k: refill directions for dropped columns
    // the cut matrix applied through its factors (n > 96), in dtype: Qt holds
    // Q^T (k x n); Ch[0..2] the blocks of the product chains (FP32 mode)
    void* Qt;
    void* Ch[3];
    // E0 E1 V of the last forward chain (n x k, dtype) and the k x chi factor
    // that turns it into P_low (factored path)
    void* T2;
    void* VsK;
    int* dead_dev;       // 2*k flags of dropped columns, then 2 counts
    uint64_t* refill_ctr; // device: {config seed, refill calls}, feeding the refill hash
    int extra_warm_iters; // added warm subspace iterations (converging to a tolerance)
    double* norm_ws;     // partial sums of the tensor normalisation (32 tensors)
    double* norm_ws_su;  // the same for normalisations on the SU stream
    double *Nfull_U, *Nfull_V;  // direct path (n <= 96)
    int ks_gram, ks_nv, ks_c, ks_p, ks_chain;  // split-K factors
    void* ws_p;                      // split-K partials of the n x chi products (dtype)
    double *ws_gram, *ws_nv;    // split-K partials (FP64)
    void* ws_c;                 // split-K partials of the corner renormalisations (dtype)

    // spectra / readout
    double* C64;
    double* csig;
    double* spectra;
    double* spec_prev;
    double* dev_scalars;  // [0] delta
    void* Eout;           // 4 blocks of q^4 (dtype)
    double* E64;
    ipeps::cplx* rho;
    ipeps::cplx* rho_T;
    double* obs_dev;
    double* host_buf;  // pinned

    // plan
    std::vector<ipeps::GemmProb> probs;
    std::vector<ipeps::GemmGroup> groups;  // every non-empty group, in plan order
    ipeps::GemmProb* d_probs;
    std::vector<ipeps::NormItem> norms;
    ipeps::NormItem* d_norms;
    bool autotune;              // IPEPS_FLAG_AUTOTUNE
    void* tune_dev;             // device copy of a group being timed
    int tune_cap;
    hipEvent_t tune_ev[2];
    long norm_a_first;    // 4 FP64 items: the double-layer tensors
    long norm_a_pre_first;  // 4 FP64 items: a_base_pre
    long norm_env_first;  // 32 dtype items: the 16 corners and 16 edges
    ipeps::ColumnStep steps[8];  // frame f (in move order) * 2 + X
    ipeps::SvdPlan svd;
    ipeps::GemmGroup read1, read2, read3, read4;

    // timing of the half-system product launches (HIP events on the stream)
    bool prof_on;
    int prof_mode;  // 1: the TAG 1 launches only; 2: every GEMM launch on the main stream
    std::vector<hipEvent_t> prof_ev;
    int prof_used;
    double prof_flops;
    struct ProfLaunch {
        double flops, bytes;
        int dtype, tag;
    };
    std::vector<ProfLaunch> prof_meta;  // one per recorded event pair

    long step_count;
    bool have_env;
    bool spectra_valid;
    bool poisoned;
    int last_iters;
    double last_delta;
};
