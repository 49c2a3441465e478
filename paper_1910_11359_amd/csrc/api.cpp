// C ABI of the iPEPS library: state lifetime, the simple-update Trotter step,
// the CTMRG driver with half-system projectors, and the readout.  Every step
// of the method runs in device kernels; this file only plans and enqueues.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>
#include <mutex>
#include <new>
#include <string>

#include "ctm.h"
#include "gemm.h"
#include "linalg.h"
#include "state.h"
#include "su.h"

using namespace ipeps;

// ---------------------------------------------------------------- memory
void* ipeps::DevMem::get(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    total += bytes;
    if (dry) return nullptr;
    void* p = nullptr;
    if (alloc) {
        p = alloc(bytes, (void*)stream, ctx);
        if (!p) throw status_error(IPEPS_ENOMEM, "allocation hook failed");
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) throw status_error(IPEPS_ENOMEM, "hipMalloc failed");
    }
    ptrs.push_back(p);
    return p;
}

void ipeps::DevMem::release() {
    for (void* p : ptrs) {
        if (free_fn)
            free_fn(p, (void*)stream, ctx);
        else
            (void)hipFree(p);
    }
    ptrs.clear();
}

namespace {

constexpr int kDirectMax = 96;  // projector SVD by direct Jacobi when n <= this
// cut matrices applied through their factors (no n^3 product) when n > this
// (below, forming them takes fewer launches and less time)
constexpr int kFactoredMin = 1024;
// tile kind of the factored chain products: a panel tile holding the k
// columns whole when k is in 65..128 (see chain_splits), else 64 x 64 tiles
constexpr int kChainTile = -2;
constexpr int kColdIters = 8;   // subspace iterations for a fresh random block
constexpr int kWarmIters = 2;   // ... when warm-started from the last iteration (FP64)
// With FP32 cut products the matrix itself carries ~1e-7 relative rounding;
// one warm iteration per CTMRG iteration is enough there (the FP32 path is
// checked against the FP64 path to its 1e-3 imbalance bound).
constexpr int kWarmItersLow = 1;
constexpr double kCholDrop = 1e-12;

int idx(int x, int y) { return ((x % 2 + 2) % 2) + 2 * ((y % 2 + 2) % 2); }
int hl(int x, int y) { return idx(x, y); }
int vl(int x, int y) { return 4 + idx(x, y); }

// physical site of frame coordinates (X, Y) in frame f: frames 0 and 2 keep
// the 2x2 cell, frames 1 and 3 transpose it (coordinates mod 2).
int frame_site(int f, int X, int Y) { return (f % 2 == 0) ? idx(X, Y) : idx(Y, X); }

// move order of one iteration: left, right, up, down = frames 0, 2, 1, 3
const int kMoveFrames[4] = {0, 2, 1, 3};

// Subspace size of the projector SVD: chi plus an oversampling of
// max(16, chi/3) columns with FP64 products.  With FP32 products, 8 columns
// from chi = 64 on (at D=6, chi=72 the FP32-vs-FP64 imbalance difference
// stays ~1e-5 for 8, 16 or 24 oversampling columns: FP32 rounding, not the
// subspace, sets it) and 16 below (with 8, jobs at D <= 4, chi <= 48 moved
// from 1.5e-5 to 1e-4 against FP64).
int choose_k(int n, int chi, int dtype) {
    const int p = dtype == IPEPS_DTYPE_FP64 ? std::max(16, chi / 3) : (chi >= 64 ? 8 : 16);
    return std::min(n, chi + p);
}

void validate(const ipeps_config* c) {
    IPEPS_REQUIRE(c != nullptr, IPEPS_EINVAL, "config is NULL");
    IPEPS_REQUIRE(c->D >= 1 && c->D <= 8, IPEPS_EINVAL, "D must be in 1..8");
    IPEPS_REQUIRE(c->d_A >= 1 && c->d_A <= 5, IPEPS_EINVAL, "d_A must be in 1..5");
    {
        const int d = 2 * c->d_A, Dc = c->D * c->D * c->D, nb = d * c->D;
        IPEPS_REQUIRE(d * (Dc < nb ? Dc : nb) <= 512, IPEPS_EINVAL,
                      "simple update: d * min(D^3, d D) must be <= 512");
    }
    IPEPS_REQUIRE(c->chi >= c->D * c->D && c->chi <= 160, IPEPS_EINVAL, "chi must be in D^2..160");
    IPEPS_REQUIRE(c->dt > 0 && std::isfinite(c->dt), IPEPS_EINVAL, "dt must be > 0");
    IPEPS_REQUIRE(c->trotter_order == 2, IPEPS_EINVAL, "trotter_order must be 2");
    IPEPS_REQUIRE(c->dtype == IPEPS_DTYPE_FP64 || c->dtype == IPEPS_DTYPE_FP32 || c->dtype == IPEPS_DTYPE_BF16 ||
                      c->dtype == IPEPS_DTYPE_BF16X3,
                  IPEPS_EINVAL, "dtype must be FP64, FP32, BF16 or BF16X3");
    IPEPS_REQUIRE(std::isfinite(c->J) && std::isfinite(c->V) && std::isfinite(c->W), IPEPS_EINVAL,
                  "non-finite model parameter");
    const uint32_t known = IPEPS_FLAG_AUTOTUNE | IPEPS_FLAG_FACTORED_CUTS | IPEPS_FLAG_FORMED_CUTS;
    IPEPS_REQUIRE((c->flags & ~known) == 0, IPEPS_EINVAL, "unknown flag");
    IPEPS_REQUIRE((c->flags & IPEPS_FLAG_FACTORED_CUTS) == 0 || (c->flags & IPEPS_FLAG_FORMED_CUTS) == 0,
                  IPEPS_EINVAL, "FACTORED_CUTS and FORMED_CUTS exclude each other");
}

// Opt-in autotuner (IPEPS_FLAG_AUTOTUNE): every candidate tile kind of a group
// is timed on the state's own buffers (one warm-up and two timed launches)
// and the fastest kept; choices are cached per process by problem shape.
// Different tile kinds sum in different orders, so results can differ from
// the default (heuristic) choice at rounding level.
std::mutex g_tune_mu;
std::map<std::string, GemmTile> g_tune_cache;

std::string group_signature(const std::vector<GemmProb>& probs, int dtype) {
    std::string k = std::to_string(dtype);
    for (const auto& p : probs) {
        k += "|" + std::to_string(p.M) + "," + std::to_string(p.N) + "," + std::to_string(p.K) + "," +
             std::to_string(p.ksplit) + "," + std::to_string(p.a_ks == 1) +
             std::to_string(p.b_cs == 1) + std::to_string(p.a_rows0 == p.M) +
             std::to_string(p.c_rows0 == p.M) + std::to_string(p.beta != 0.0);
    }
    return k;
}

GemmTile autotune_tile(ipeps_state* st, std::vector<GemmProb> probs, int dtype, long reduce_elems,
                       GemmTile fallback) {
    for (const auto& p : probs)
        if (p.gate) return fallback;  // a gated group may skip its work while timed
    const std::string key = group_signature(probs, dtype);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    const int n = (int)probs.size();
    if ((int)st->tune_cap < n) {
        if (st->tune_dev) HIP_CHECK(hipFree(st->tune_dev));
        HIP_CHECK(hipMalloc(&st->tune_dev, n * sizeof(GemmProb)));
        st->tune_cap = n;
    }
    GemmTile cand[5];
    const int nc = gemm_tile_candidates(probs.data(), n, dtype, cand);
    GemmTile best = fallback;
    float best_ms = 1e30f;
    for (int c = 0; c < nc; ++c) {
        std::vector<GemmProb> q = probs;
        const int tiles = gemm_plan_with(q.data(), n, dtype, cand[c]);
        HIP_CHECK(hipMemcpy(st->tune_dev, q.data(), n * sizeof(GemmProb), hipMemcpyHostToDevice));
        gemm_launch(st->stream, dtype, cand[c], (const GemmProb*)st->tune_dev, n, tiles, 0, reduce_elems);
        HIP_CHECK(hipEventRecord(st->tune_ev[0], st->stream));
        for (int r = 0; r < 2; ++r)
            gemm_launch(st->stream, dtype, cand[c], (const GemmProb*)st->tune_dev, n, tiles, 0, reduce_elems);
        HIP_CHECK(hipEventRecord(st->tune_ev[1], st->stream));
        HIP_CHECK(hipEventSynchronize(st->tune_ev[1]));
        float ms = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&ms, st->tune_ev[0], st->tune_ev[1]));
        if (ms < best_ms) {
            best_ms = ms;
            best = cand[c];
        }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return best;
}

// force >= 0: that tile kind (if the operands allow it) instead of the
// heuristic or the autotuner
GemmGroup add_group(ipeps_state* st, std::vector<GemmProb> probs, int dtype, int force = -1) {
    GemmGroup g;
    g.first = (int)st->probs.size();
    g.count = (int)probs.size();
    g.dtype = dtype;
    g.tiles = gemm_plan_tiles(probs.data(), g.count, dtype, &g.tile);
    for (const auto& p : probs)
        if (p.ksplit > 1) g.reduce_elems = std::max(g.reduce_elems, (long)p.M * p.N);
    bool forced = false;
    if (force == kChainTile) {
        const int pt = gemm_panel_for(probs.data(), g.count, dtype);
        force = pt >= 0 ? pt : (int)TILE_DIRECT_SMALL;
    }
    if (force >= 0 && g.count > 0) {
        GemmTile cand[5];
        const int nc = gemm_tile_candidates(probs.data(), g.count, dtype, cand);
        for (int i = 0; i < nc; ++i)
            if (cand[i] == (GemmTile)force) {
                g.tile = (GemmTile)force;
                g.tiles = gemm_plan_with(probs.data(), g.count, dtype, g.tile);
                forced = true;
            }
    }
    if (st->autotune && g.count > 0 && !forced) {
        const GemmTile t = autotune_tile(st, probs, dtype, g.reduce_elems, g.tile);
        if (t != g.tile) {
            g.tile = t;
            g.tiles = gemm_plan_with(probs.data(), g.count, dtype, t);
        }
    }
    const double esz = dtype == IPEPS_DTYPE_FP64 ? 8.0 : 4.0;  // BF16 modes keep FP32 operands
    for (auto& p : probs) {
        g.flops += 2.0 * p.M * (double)p.N * p.K;
        g.bytes += esz * ((double)p.M * p.K + (double)p.K * p.N + (double)p.M * p.N);
        st->probs.push_back(p);
    }
    if (g.count > 0) st->groups.push_back(g);
    return g;
}

// ---------------------------------------------------------------- execution
// The CTMRG and the simple update run on one state, or on several states of
// one buffer layout in lockstep (a batch; every state then holds the same
// buffers at the same offsets from its first allocation, and its buffers sit
// jm.delta[j] bytes from the lead's): every launch carries all the jobs.
// GEMM groups are replayed from a merged problem table (each problem of the
// lead's group once per job, its pointers moved by the job's offset, with the
// lead's tile kind, so every job's arithmetic is the one it has alone); the
// other kernels take the JobMap.  All work goes to the lead's streams.
struct Ex {
    ipeps_state* st = nullptr;       // lead: dimensions, plan, streams, control flags
    std::vector<ipeps_state*> jobs;  // every job, jobs[0] == st
    JobMap jm;                       // delta == nullptr: one job
    GemmProb* d_probs = nullptr;     // merged problem table (batch)
    std::unordered_map<int, GemmGroup> merged;  // lead group .first -> merged group
    NormItem* d_norms = nullptr;     // merged normalisation items (batch)
    std::unordered_map<long, long> norm_first;  // lead item range .first -> merged first
    double* norm_ws = nullptr;       // workspace of the merged normalisations
    std::vector<long> hdelta;        // host copy of jm.delta
    bool batched() const { return jm.delta != nullptr; }
    int nj() const { return (int)jobs.size(); }
    // a buffer pointer of the lead moved to job j's copy
    template <typename T>
    T* at(T* p, int j) const {
        return batched() ? (T*)((char*)p + hdelta[j]) : p;
    }
};

Ex solo(ipeps_state* st) {
    Ex x;
    x.st = st;
    x.jobs.push_back(st);
    return x;
}

void launch_group(const Ex& x, hipStream_t stream, const GemmGroup& g) {
    if (!x.batched()) {
        gemm_launch(stream, g.dtype, g.tile, x.st->d_probs + g.first, g.count, g.tiles, g.tag,
                    g.reduce_elems);
        return;
    }
    const GemmGroup& m = x.merged.at(g.first);
    gemm_launch(stream, m.dtype, m.tile, x.d_probs + m.first, m.count, m.tiles, g.tag, m.reduce_elems);
}

void run(const Ex& x, const GemmGroup& g) {
    if (g.count == 0) return;
    ipeps_state* st = x.st;
    const bool timed = !x.batched() && st->prof_on && (g.tag == 1 || st->prof_mode == 2) &&
                       st->prof_used + 2 <= (int)st->prof_ev.size();
    if (timed) HIP_CHECK(hipEventRecord(st->prof_ev[st->prof_used], st->stream));
    launch_group(x, st->stream, g);
    if (timed) {
        HIP_CHECK(hipEventRecord(st->prof_ev[st->prof_used + 1], st->stream));
        st->prof_used += 2;
        st->prof_meta.push_back({g.flops, g.bytes, g.dtype, g.tag});
        if (g.tag == 1) st->prof_flops = g.flops;
    }
}

char* off(void* base, long elems, size_t esz) { return (char*)base + elems * (long)esz; }

void run_on(const Ex& x, hipStream_t stream, const GemmGroup& g) {
    if (g.count == 0) return;
    launch_group(x, stream, g);
}

// Frobenius normalisation of `count` items of the lead's table from `first`
// (all jobs in a batch)
void normalize_items(const Ex& x, hipStream_t s, int dtype, long first, int count, double* ws) {
    if (!x.batched()) return normalize_tensors(s, dtype, x.st->d_norms + first, count, ws);
    normalize_tensors(s, dtype, x.d_norms + x.norm_first.at(first), count * x.nj(), x.norm_ws);
}

GemmProb split(GemmProb p, int ks, void* ws) {
    if (ks > 1) {
        p.ksplit = ks;
        p.ws = ws;
    }
    return p;
}

int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// K splits of the chain products (two n x n corners against n x k blocks per
// launch): with panel tiles (k in 65..128; 2 ceil(n / 64) tiles) enough for
// about two workgroups per CU (measured at n = 2592: 6 splits, FP32 k = 80
// 36 us and FP64 k = 96 66 us per launch, against 46 and 84 us with 64 x 64
// tiles); with 64 x 64 tiles one per 512 rows of K.
int chain_splits(int n, int k) {
    if (k > 64 && k <= 128) return clampi((512 + n / 64) / (2 * ceil_div(n, 64)), 1, 16);
    return clampi(n / 512, 1, 16);
}

// ---------------------------------------------------------------- allocation
void allocate(ipeps_state* st) {
    DevMem& M = st->mem;
    const int D = st->D, d = st->d, q = st->q, chi = st->chi, n = st->n, k = st->k;
    const size_t e = st->esz;
    const long D4 = (long)D * D * D * D, q4 = (long)q * q * q * q, n2 = (long)n * n;
    const long cqc = (long)chi * q * chi;
    st->gam = (cplx*)M.get(4 * d * D4 * sizeof(cplx));
    st->lam = (double*)M.get(8 * D * sizeof(double));
    st->eps = (double*)M.get(4 * sizeof(double));
    st->eps_snap = (double*)M.get(4 * sizeof(double));
    st->eps_snap_pre = (double*)M.get(4 * sizeof(double));
    st->gates = (cplx*)M.get(8 * (long)d * d * d * d * sizeof(cplx));
    st->su_scratch = M.get(su_scratch_bytes(D, d));
    st->A = (cplx*)M.get(4 * d * D4 * sizeof(cplx));
    st->a_base = (double*)M.get(4 * q4 * sizeof(double));
    st->A_pre = (cplx*)M.get(4 * d * D4 * sizeof(cplx));
    st->a_base_pre = (double*)M.get(4 * q4 * sizeof(double));
    // the 32 frame copies in one block (copied whole when the next step's
    // were built ahead), and the block the simple update builds them into
    st->frames = M.get(32 * q4 * e);
    st->frames_pre = M.get(32 * q4 * e);
    for (int i = 0; i < 16; ++i) {
        st->a_lu[i] = off(st->frames, i * q4, e);
        st->a_dl[i] = off(st->frames, (16 + i) * q4, e);
        st->a_lu_pre[i] = off(st->frames_pre, i * q4, e);
        st->a_dl_pre[i] = off(st->frames_pre, (16 + i) * q4, e);
    }
    st->d_a_lu = (void**)M.get(16 * sizeof(void*));
    st->d_a_dl = (void**)M.get(16 * sizeof(void*));
    st->d_a_lu_pre = (void**)M.get(16 * sizeof(void*));
    st->d_a_dl_pre = (void**)M.get(16 * sizeof(void*));
    st->Cenv = M.get(16L * chi * chi * e);
    st->Tenv = M.get(16L * cqc * e);
    st->X1 = M.get(8 * cqc * e);
    st->X1p = M.get(8 * cqc * e);
    st->T4p = M.get(2 * cqc * e);
    st->X2 = M.get(8 * n2 * e);
    st->X2p = M.get(8 * n2 * e);
    st->E = M.get(16 * n2 * e);
    st->X1p_aux = M.get(4 * cqc * e);
    st->X2p_aux = M.get(4 * n2 * e);
    if (!st->factored) {  // the cut matrix is formed
        st->Fh = M.get(2 * n2 * e);
        st->Gh = M.get(2 * n2 * e);
        st->N64 = (double*)M.get(2 * n2 * sizeof(double));
        st->Nd = (st->dtype == IPEPS_DTYPE_FP64) ? (void*)st->N64 : M.get(2 * n2 * e);
    } else {  // ... else applied through its factors
        st->Fh = st->Gh = st->Nd = nullptr;
        st->N64 = nullptr;
    }
    st->Z = M.get(2 * cqc * e);
    st->Us = M.get(2L * n * chi * e);
    st->Vs = M.get(2L * n * chi * e);
    st->Plow = M.get(2L * n * chi * e);
    st->Pup = M.get(2L * n * chi * e);
    st->PlowP = M.get(2L * n * chi * e);
    st->PupP = M.get(2L * n * chi * e);
    st->W1p = M.get(2 * n2 * e);
    st->W2 = M.get(2 * n2 * e);
    st->g_dev = (int*)M.get(2 * sizeof(int));
    const long nk = (long)n * k;
    st->ks_gram = clampi(n / 64, 1, 48);
    st->ks_nv = clampi(n / 512, 1, 8);
    st->ks_c = clampi(n / 256, 1, 32);
    st->ws_gram = (double*)M.get(2L * st->ks_gram * k * k * sizeof(double));
    st->ks_chain = chain_splits(n, k);
    st->ws_nv = (double*)M.get(2L * std::max((size_t)st->ks_nv * sizeof(double), (size_t)st->ks_chain * e) * nk);
    st->ws_c = M.get(4L * st->ks_c * chi * chi * e);
    st->ks_p = clampi(n / 512, 1, 8);
    st->ws_p = M.get(4L * st->ks_p * n * chi * e);
    st->warm = (double*)M.get(16 * nk * sizeof(double));
    st->Yw = (double*)M.get(2 * nk * sizeof(double));
    st->Zw = (double*)M.get(2 * nk * sizeof(double));
    st->Qw = (double*)M.get(2 * nk * sizeof(double));
    st->Qz = (double*)M.get(2 * nk * sizeof(double));
    st->Gm = (double*)M.get(2L * k * k * sizeof(double));
    st->Ri = (double*)M.get(2L * k * k * sizeof(double));
    st->Rb = (double*)M.get(2 * nk * sizeof(double));
    st->Qt = st->Ch[0] = st->Ch[1] = st->Ch[2] = st->T2 = st->VsK = nullptr;
    if (st->factored) {
        st->Qt = M.get(2 * nk * e);
        st->T2 = M.get(2 * nk * e);
        st->VsK = M.get(2L * k * chi * e);
        if (st->dtype != IPEPS_DTYPE_FP64)
            for (int i = 0; i < 3; ++i) st->Ch[i] = M.get(2 * nk * e);
    }
    st->dead_dev = (int*)M.get((2L * k + 2) * sizeof(int));
    st->refill_ctr = (uint64_t*)M.get(2 * sizeof(uint64_t));
    st->norm_ws = (double*)M.get(normalize_ws_doubles(32) * sizeof(double));
    st->norm_ws_su = (double*)M.get(normalize_ws_doubles(4) * sizeof(double));
    st->Cs = (double*)M.get(2L * k * k * sizeof(double));
    st->Uc = (double*)M.get(2L * k * k * sizeof(double));
    st->Vc = (double*)M.get(2L * k * k * sizeof(double));
    st->sig = (double*)M.get(2L * std::max(k, n) * sizeof(double));
    st->Uo = (double*)M.get(2 * std::max(nk, n2 <= 96L * 96 ? n2 : 0L) * sizeof(double));
    st->Vo = (double*)M.get(2 * std::max(nk, n2 <= 96L * 96 ? n2 : 0L) * sizeof(double));
    size_t jw = std::max({jacobi_svd_real_work(2, k, k), jacobi_svd_real_work(16, chi, chi),
                          n <= kDirectMax ? jacobi_svd_real_work(2, n, n) : (size_t)0});
    st->jwork = (double*)M.get(std::max(jw, (size_t)1) * sizeof(double));
    st->jwork_c = (double*)M.get(std::max(jacobi_svd_real_work(16, chi, chi), (size_t)1) * sizeof(double));
    st->C64 = (double*)M.get(16L * chi * chi * sizeof(double));
    st->csig = (double*)M.get(16L * chi * sizeof(double));
    st->spectra = (double*)M.get(16L * chi * sizeof(double));
    st->spec_prev = (double*)M.get(16L * chi * sizeof(double));
    st->dev_scalars = (double*)M.get(8 * sizeof(double));
    // asynchronous readout: snapshot of C, T, A, eps and its own scratch
    st->Csnap = M.get(16L * chi * chi * e);
    st->Tsnap = M.get(16L * cqc * e);
    st->Asnap = (cplx*)M.get(4 * d * D4 * sizeof(cplx));
    st->eps_r = (double*)M.get(8 * sizeof(double));
    st->X1r = M.get(8 * cqc * e);
    st->X2r = M.get(8 * n2 * e);
    st->X2pr = M.get(8 * n2 * e);
    st->Er = M.get(8 * n2 * e);
    st->Eout_r = M.get(4 * q4 * e);
    st->E64_r = (double*)M.get(4 * q4 * sizeof(double));
    st->rho_r = (cplx*)M.get(4 * (long)d * d * sizeof(cplx));
    st->rho_T_r = (cplx*)M.get(4 * D4 * d * sizeof(cplx));
    st->obs_r = (double*)M.get(16 * sizeof(double));
    st->Eout = M.get(4 * q4 * e);
    st->E64 = (double*)M.get(4 * q4 * sizeof(double));
    st->rho = (cplx*)M.get(4 * (long)d * d * sizeof(cplx));
    st->rho_T = (cplx*)M.get(4 * D4 * d * sizeof(cplx));
    st->obs_dev = (double*)M.get(16 * sizeof(double));
}

// ---------------------------------------------------------------- plan
// Output of a (chi q) x (chi q) product with rows (t, u) and columns (c, v)
// (t, c < chi; u, v < q) stored as [t][c][u][v]: runs of q contiguous
// elements, and directly the chi^2 x q^2 operand of the next product.
GemmProb permuted_rows_cols(GemmProb p, int chi, int q) {
    const long q2 = (long)q * q;
    p.c_rows0 = q;  // i = t q + u -> t chi q^2 + u q
    p.c_rs1 = chi * q2;
    p.c_rs0 = q;
    p.c_cols0 = q;  // j = c q + v -> c q^2 + v
    p.c_cs1 = q2;
    p.c_cs0 = 1;
    return p;
}

// Enlarged corner j (0 UL, 1 UR, 2 DR, 3 DL in the move's frame) of cut Y in
// column step si.  The matrix of an enlarged corner depends only on its site
// s and corner index g (it contracts C_g, T_g, T_{g-1} and the double layer
// of s, rows on the T_{g-1} side, columns on the T_g side), not on the frame,
// so each (s, g) has one slot in E and a slot stays valid while its inputs do.
char* cut_corner(const ipeps_state* st, int si, int Y, int j) {
    const int f = kMoveFrames[si / 2], X = si % 2;
    const int fx[4] = {X, X + 1, X + 1, X}, fy[4] = {Y, Y, Y + 1, Y + 1};
    const int site = frame_site(f, fx[j], fy[j]), g = (f + j) % 4;
    return off(st->E, (site * 4 + g) * (long)st->n * st->n, st->esz);
}

void build_plan(ipeps_state* st) {
    // dt: arithmetic of the environment contractions (BF16 mode: FP32 tensors,
    // BF16 MFMA operands); the readout products run in the storage precision
    const int q = st->q, chi = st->chi, n = st->n, k = st->k, dt = st->mma, dst = st->dtype;
    const size_t e = st->esz;
    const long n2 = (long)n * n, cqc = (long)chi * q * chi, cc = (long)chi * chi;
    auto Cp = [&](int site, int kk) { return off(st->Cenv, (site * 4 + kk) * cc, e); };
    auto Tp = [&](int site, int kk) { return off(st->Tenv, (site * 4 + kk) * cqc, e); };

    for (int mi = 0; mi < 4; ++mi) {
        const int f = kMoveFrames[mi];
        for (int X = 0; X < 2; ++X) {
            ColumnStep& cs = st->steps[mi * 2 + X];
            cs.slot = mi * 2 + X;
            std::vector<GemmProb> s1, s2, s3, half, np, pr, pr2, w1, w2, fin, a1, a2, a3, s1w, s2w, s3w;
            const int si = mi * 2 + X;
            // A move with frame f' rewrites C_f', C_{f'+3} and T_{f'+3}, i.e. the
            // enlarged corners with g = f' and g = f' + 3; those with g = f' + 1
            // and f' + 2 it computed for every site and left valid.  The first
            // column step of the next move reuses them (within one iteration:
            // each iteration starts on new double layers).
            const int fprev = mi > 0 ? kMoveFrames[mi - 1] : -1;
            for (int Y = 0; Y < 2; ++Y) {
                const int fx[4] = {X, X + 1, X + 1, X}, fy[4] = {Y, Y, Y + 1, Y + 1};
                for (int j = 0; j < 4; ++j) {
                    const int s = frame_site(f, fx[j], fy[j]);
                    const int g = (f + j) % 4;
                    const int blk = Y * 4 + j;
                    const bool reuse = X == 0 && mi > 0 && (g == (fprev + 1) % 4 || g == (fprev + 2) % 4);
                    // warm variant of the left move's first column step (later
                    // iterations of one call, double layers unchanged): the
                    // last move (down) left the types f_down + 1, + 2 valid
                    const bool warmv = mi == 0 && X == 0;
                    const bool reuse_w = warmv && (g == (kMoveFrames[3] + 1) % 4 || g == (kMoveFrames[3] + 2) % 4);
                    // UR and DR of the second column: computed ahead (aux stream)
                    const bool ahead = X == 1 && (j == 1 || j == 2);
                    const int ab = Y * 2 + (j - 1);
                    char* x1 = off(st->X1, blk * cqc, e);
                    char* x1p = ahead ? off(st->X1p_aux, ab * cqc, e) : off(st->X1p, blk * cqc, e);
                    char* x2p = ahead ? off(st->X2p_aux, ab * n2, e) : off(st->X2p, blk * n2, e);
                    char* E = cut_corner(st, si, Y, j);
                    // S1: C (chi x chi) . Tnext (chi x q chi), columns (v, c), where
                    // the C renormalisation reads it (UL); and with the columns
                    // written in (c, v) order (X1p) for the corner itself
                    if (j == 0) {
                        s1.push_back(gemm_nn(Cp(s, g), chi, Tp(s, g), (long)q * chi, x1, (long)q * chi,
                                             chi, q * chi, chi));
                        if (warmv) s1w.push_back(s1.back());
                    }
                    if (reuse) continue;
                    GemmProb p1 = gemm_nn(Cp(s, g), chi, Tp(s, g), (long)q * chi, x1p, (long)q * chi,
                                          chi, q * chi, chi);
                    p1.c_cols0 = chi;  // column j = v chi + c -> c q + v
                    p1.c_cs1 = 1;
                    p1.c_cs0 = q;
                    (ahead ? a1 : s1).push_back(p1);
                    if (warmv && !reuse_w) s1w.push_back(p1);
                    // S2: Tprev (chi q x chi) . X1p (chi x chi q): row (t, u), column
                    // (c, v), written as X2p[t][c][u][v] (the chi^2 x q^2 layout S3 reads)
                    (ahead ? a2 : s2)
                        .push_back(permuted_rows_cols(gemm_nn(Tp(s, (g + 3) % 4), chi, x1p, (long)q * chi,
                                                              x2p, 0, chi * q, q * chi, chi),
                                                      chi, q));
                    if (warmv && !reuse_w) s2w.push_back((ahead ? a2 : s2).back());
                    // S3: X2p (chi^2 x q^2) . a[L U][D R]; result as the n x n
                    // matrix [prev = (t, D)][next = (c, R)]
                    GemmProb p3 = gemm_nn(x2p, (long)q * q, st->a_lu[s * 4 + g], (long)q * q, E, n,
                                          chi * chi, q * q, q * q);
                    p3.c_rows0 = chi;
                    p3.c_rs1 = (long)q * n;
                    p3.c_rs0 = q;
                    p3.c_cols0 = q;
                    p3.c_cs1 = n;
                    p3.c_cs0 = 1;
                    (ahead ? a3 : s3).push_back(p3);
                    if (warmv && !reuse_w) s3w.push_back(p3);
                }
                char* E0 = cut_corner(st, si, Y, 0);
                char* E1 = cut_corner(st, si, Y, 1);
                char* E2 = cut_corner(st, si, Y, 2);
                char* E3 = cut_corner(st, si, Y, 3);
                // projectors: P_low = F Vs (n x chi), P_up = Us^T G (chi x n; Us is
                // stored transposed, chi x n), with the half systems F = E0 E1,
                // G = E2 E3
                char* us = off(st->Us, Y * (long)n * chi, e);
                char* vs = off(st->Vs, Y * (long)n * chi, e);
                char* plow = off(st->Plow, Y * (long)n * chi, e);
                char* pup = off(st->Pup, Y * (long)n * chi, e);
                // the n x n by n x chi products are split over K (a launch of a
                // few hundred workgroups would otherwise walk K = n serially)
                const int ksp = st->ks_p;
                auto wsp = [&](int r) { return off(st->ws_p, r * (long)ksp * n * chi, e); };
                if (!st->factored) {
                    char* F = off(st->Fh, Y * n2, e);
                    char* G = off(st->Gh, Y * n2, e);
                    half.push_back(gemm_nn(E0, n, E1, n, F, n, n, n, n));
                    half.push_back(gemm_nn(E2, n, E3, n, G, n, n, n, n));
                    np.push_back(gemm_nn(G, n, F, n, off(st->Nd, Y * n2, e), n, n, n, n));
                    pr.push_back(split(gemm_nn(F, n, vs, chi, plow, chi, n, chi, n), ksp, wsp(Y * 2)));
                    pr.push_back(split(gemm_nn(us, n, G, n, pup, n, chi, n, n), ksp, wsp(Y * 2 + 1)));
                } else {
                    // F and G are never formed: Us^T E2 first (into the PupP
                    // buffer, rewritten by the permute after), then (Us^T E2) E3;
                    // P_low comes from the last forward chain (SvdPlan::PlowT2)
                    (void)vs;
                    (void)plow;
                    char* pu1 = off(st->PupP, Y * (long)n * chi, e);
                    pr.push_back(split(gemm_nn(us, n, E2, n, pu1, n, chi, n, n), ksp, wsp(Y)));
                    pr2.push_back(split(gemm_nn(pu1, n, E3, n, pup, n, chi, n, n), ksp, wsp(Y)));
                }
                // renormalisation inputs of column X
                const int sxy = frame_site(f, X, Y);
                cs.site_x[Y] = sxy;
                cs.site_x1[Y] = frame_site(f, X + 1, Y);
                // Z = T3(X,Y) (chi q x chi) . C4(X,Y)  -> [t3p][q3][c4n]
                s1.push_back(gemm_nn(Tp(sxy, (2 + f) % 4), chi, Cp(sxy, (3 + f) % 4), chi,
                                     off(st->Z, Y * cqc, e), chi, chi * q, chi, chi));
                if (mi == 0 && X == 0) s1w.push_back(s1.back());
                // W1 = PupP (chi q x chi) . T4p(X,Y) (chi x chi q, columns (c, v)),
                // written as W1p[t][c][u][v] (the chi^2 x q^2 layout w2 reads)
                cs.t4[Y] = Tp(sxy, (3 + f) % 4);
                w1.push_back(permuted_rows_cols(gemm_nn(off(st->PupP, Y * (long)n * chi, e), chi,
                                                        off(st->T4p, Y * cqc, e), (long)q * chi,
                                                        off(st->W1p, Y * n2, e), 0, chi * q, q * chi, chi),
                                                chi, q));
                // W2 = W1p (chi^2 x q^2) . a[D L][R U] in frame f: row (c', t4n),
                // column (R, U), written as W2[c'][R][t4n][U], i.e. the
                // (chi q) x n matrix [(c', R)][(t4n, U)] the T4 update reads
                GemmProb pw2 = gemm_nn(off(st->W1p, Y * n2, e), (long)q * q, st->a_dl[sxy * 4 + f],
                                       (long)q * q, off(st->W2, Y * n2, e), 0, chi * chi, q * q, q * q);
                pw2.c_rows0 = chi;  // i = c' chi + t4n -> c' q n + t4n q
                pw2.c_rs1 = (long)q * n;
                pw2.c_rs0 = q;
                pw2.c_cols0 = q;  // j = R q + U -> R n + U
                pw2.c_cs1 = n;
                pw2.c_cs0 = 1;
                w2.push_back(pw2);
            }
            for (int Y = 0; Y < 2; ++Y) {
                const int Yn = (Y + 1) % 2, Yp = (Y + 1) % 2;  // Y+1 and Y-1 coincide mod 2
                // C1(X+1, Y+1) = P_up(Y) (chi x n) . X1 of UL at (X, Y+1) (n x chi)
                const int ksc = st->ks_c;
                fin.push_back(split(gemm_nn(off(st->Pup, Y * (long)n * chi, e), n,
                                            off(st->X1, (Yn * 4 + 0) * cqc, e), chi,
                                            Cp(frame_site(f, X + 1, Y + 1), f % 4), chi, chi, chi, n),
                                    ksc, off(st->ws_c, (2 * Y + 0) * (long)ksc * chi * chi, e)));
                // C4(X+1, Y) = Z(Y) (chi x q chi, k = (q3, c4n)) . PlowP(Y)
                fin.push_back(split(gemm_nn(off(st->Z, Y * cqc, e), (long)q * chi,
                                            off(st->PlowP, Y * (long)n * chi, e), chi,
                                            Cp(frame_site(f, X + 1, Y), (3 + f) % 4), chi, chi, chi, n),
                                    ksc, off(st->ws_c, (2 * Y + 1) * (long)ksc * chi * chi, e)));
                // T4(X+1, Y) = W2(Y) [rows (c', R), k = (t4n, U)] . P_low(Y-1)
                fin.push_back(split(gemm_nn(off(st->W2, Y * n2, e), n, off(st->Plow, Yp * (long)n * chi, e),
                                            chi, Tp(frame_site(f, X + 1, Y), (3 + f) % 4), chi, chi * q,
                                            chi, n),
                                    st->ks_p, off(st->ws_p, Y * (long)st->ks_p * n * chi, e)));
            }
            cs.s1 = add_group(st, s1, dt);
            cs.s2 = add_group(st, s2, dt);
            cs.s3 = add_group(st, s3, dt);
            if (mi == 0 && X == 0) cs.s3.tag = 1;  // all 8 corners: the roofline launch
            cs.s1w = add_group(st, s1w, dt);
            cs.s2w = add_group(st, s2w, dt);
            cs.s3w = add_group(st, s3w, dt);
            cs.aux_s1 = add_group(st, a1, dt);
            cs.aux_s2 = add_group(st, a2, dt);
            cs.aux_s3 = add_group(st, a3, dt);
            cs.half = add_group(st, half, dt);
            cs.nprod = add_group(st, np, dt);
            // P_up's chi rows against n x n factors: panel tiles when chi is in
            // 65..128 (64 x 64 tiles otherwise)
            cs.proj = add_group(st, pr, dt, st->factored ? kChainTile : -1);
            cs.proj2 = add_group(st, pr2, dt, st->factored ? kChainTile : -1);
            cs.w1 = add_group(st, w1, dt);
            cs.w2 = add_group(st, w2, dt);
            cs.fin = add_group(st, fin, dt);
            cs.norm_first = (long)st->norms.size();
            for (int Y = 0; Y < 2; ++Y) {
                st->norms.push_back({Cp(frame_site(f, X + 1, Y + 1), f % 4), cc});
                st->norms.push_back({Cp(frame_site(f, X + 1, Y), (3 + f) % 4), cc});
                st->norms.push_back({Tp(frame_site(f, X + 1, Y), (3 + f) % 4), cqc});
            }
        }
    }

    // projector SVD, FP64, batch of the two cuts
    if (n > kDirectMax) {
        const long nk = (long)n * k, kk = (long)k * k;
        std::vector<GemmProb> v;
        auto batch2 = [&](auto make) {
            std::vector<GemmProb> out;
            for (int b = 0; b < 2; ++b) out.push_back(make(b));
            return add_group(st, out, IPEPS_DTYPE_FP64);
        };
        SvdPlan& P = st->svd;
        const int kg = st->ks_gram, kv = st->ks_nv;
        double* wg = st->ws_gram;
        double* wv = st->ws_nv;
        // The cut matrix of cut b is N = G F = E2 E3 E0 E1 (n x n each),
        // applied factor by factor in dtype (4 n^2 k products instead of 3
        // n^3 to form it).  Y = N V with column blocks: V -> E1 V -> E0 . ->
        // E3 . -> E2 . (n x k each).  Z = N^T Q as Z^T = Q^T E2 E3 E0 E1 with
        // row blocks from Qt = Q^T (k x n), the last product written
        // transposed (n x k).  FP64 mode reads V from Qz, writes Y to Yw and Z
        // to Zw and uses as scratch the blocks the subspace iteration
        // overwrites next; FP32 mode goes through Ch[0..2] (converted at
        // both ends).
        if (!st->factored) {
            P.NVf = batch2([&](int b) {
                return split(gemm_nn(st->N64 + b * n2, n, st->Qz + b * nk, k, st->Yw + b * nk, k, n,
                                     k, n),
                             kv, wv + b * kv * nk);
            });
            P.NtQf = batch2([&](int b) {
                return split(gemm_general(st->N64 + b * n2, true, n, st->Qw + b * nk, false, k,
                                          st->Zw + b * nk, k, n, k, n),
                             kv, wv + b * kv * nk);
            });
        } else {
            const bool f64 = dt == IPEPS_DTYPE_FP64;
            // the chain products (n x n corner against a k-column block): panel
            // tiles that hold the k columns whole, so each corner is streamed
            // once (64 x 64 tiles streamed it twice at k = 80 and computed 128
            // columns), K split per chain_splits
            auto batch2d = [&](auto make) {
                std::vector<GemmProb> out;
                for (int b = 0; b < 2; ++b) out.push_back(make(b));
                return add_group(st, out, dt, k <= 128 ? kChainTile : -1);
            };
            const int kv = st->ks_chain;
            // the forward chain keeps E0 E1 V in T2: after the Rayleigh-Ritz
            // step (V = Qz, Vo = Qz Uc) P_low = F Vo S^-1/2 = T2 (Uc S^-1/2)
            void* fwd_buf[5] = {st->Qz, st->Zw, st->T2, st->Zw, st->Yw};
            void* bwd_buf[5] = {st->Qt, st->Yw, st->Qz, st->Yw, st->Zw};
            if (!f64) {
                void* const f[5] = {st->Ch[2], st->Ch[0], st->T2, st->Ch[0], st->Ch[1]};
                void* const g[5] = {st->Qt, st->Ch[0], st->Ch[1], st->Ch[0], st->Ch[2]};
                for (int t = 0; t < 5; ++t) fwd_buf[t] = f[t], bwd_buf[t] = g[t];
            }
            const int fwd_j[4] = {1, 0, 3, 2}, bwd_j[4] = {2, 3, 0, 1};
            for (int si = 0; si < 8; ++si)  // the corners' slots depend on the column step
            for (int t = 0; t < 4; ++t) {
                P.NV[si][t] = batch2d([&](int b) {
                    return split(gemm_nn(cut_corner(st, si, b, fwd_j[t]), n, off(fwd_buf[t], b * nk, e),
                                         k, off(fwd_buf[t + 1], b * nk, e), k, n, k, n),
                                 kv, off(wv, b * kv * nk, e));
                });
                P.NtQ[si][t] = batch2d([&](int b) {
                    GemmProb p = gemm_nn(off(bwd_buf[t], b * nk, e), n, cut_corner(st, si, b, bwd_j[t]),
                                         n, off(bwd_buf[t + 1], b * nk, e), n, k, n, n);
                    if (t == 3) {  // C(i, j) -> [j][i]
                        p.c_rows0 = k;
                        p.c_rs1 = 0;
                        p.c_rs0 = 1;
                        p.c_cols0 = n;
                        p.c_cs1 = 0;
                        p.c_cs0 = k;
                    }
                    return split(p, kv, off(wv, b * kv * nk, e));
                });
            }
            P.PlowT2 = batch2d([&](int b) {
                return gemm_nn(off(st->T2, b * nk, e), k, off(st->VsK, b * (long)k * chi, e), chi,
                               off(st->Plow, b * (long)n * chi, e), chi, n, chi, k);
            });
        }
        auto gram = [&](double* X) {
            return batch2([&](int b) {
                return split(gemm_general(X + b * nk, true, k, X + b * nk, false, k, st->Gm + b * kk,
                                          k, k, k, n),
                             kg, wg + b * kg * kk);
            });
        };
        auto mulR = [&](double* X, double* out) {
            return batch2([&](int b) {
                return gemm_nn(X + b * nk, k, st->Ri + b * kk, k, out + b * nk, k, n, k, k);
            });
        };
        P.gramY = gram(st->Yw);
        P.QfromY = mulR(st->Yw, st->Qw);
        P.gramQ = gram(st->Qw);
        P.YfromQ = mulR(st->Qw, st->Yw);
        P.gramZ = gram(st->Zw);
        P.QfromZ = mulR(st->Zw, st->Qz);
        P.gramQz = gram(st->Qz);
        P.ZfromQz = mulR(st->Qz, st->Zw);
        // final: Zw = N V (a copy of Yw before its orthonormalisation, V in
        // Qz), Cs = Yw^T Zw, Uo = Yw Uc, Vo = Qz Vc
        // Cs = Yw^T Zw = Q^T N V is the upper-triangular R of the two-pass
        // Cholesky QR of N V, its rows graded like the singular values.  It
        // is stored transposed: the one-sided Jacobi then rotates the rows of
        // R, whose cosines start at R_pq / R_pp instead of R_pq / R_qq
        // (QR-preconditioned Jacobi), and needs fewer sweeps.  The Jacobi
        // returns Cs^T = Uc S Vc^T, so N ~ (Yw Vc) S (Qz Uc)^T.
        P.Cs = batch2([&](int b) {
            GemmProb p = gemm_general(st->Yw + b * nk, true, k, st->Zw + b * nk, false, k,
                                      st->Cs + b * kk, k, k, k, n);
            p.c_rs0 = 1;  // C(i, j) -> Cs[j][i]
            p.c_cs0 = k;
            return split(p, kg, wg + b * kg * kk);
        });
        // Uo and Vo of both cuts in one launch (independent products); Vo is
        // written straight into the column step's warm-start slot, the next
        // iteration's starting block
        for (int si = 0; si < 8; ++si) {
            std::vector<GemmProb> uv;
            double* vo = st->warm + 2 * si * nk;
            for (int b = 0; b < 2; ++b)
                uv.push_back(gemm_nn(st->Yw + b * nk, k, st->Vc + b * kk, k, st->Uo + b * nk, k, n, k, k));
            for (int b = 0; b < 2; ++b)
                uv.push_back(gemm_nn(st->Qz + b * nk, k, st->Uc + b * kk, k, vo + b * nk, k, n, k, k));
            P.UoVo[si] = add_group(st, uv, IPEPS_DTYPE_FP64);
        }

        // gated on the number of dropped columns of matrix b
        auto proj1 = [&](double* Q) {
            return batch2([&](int b) {
                GemmProb p = split(gemm_general(Q + b * nk, true, k, st->Rb + b * nk, false, k,
                                                st->Gm + b * kk, k, k, k, n),
                                   kg, wg + b * kg * kk);
                p.gate = st->dead_dev + 2 * k + b;
                return p;
            });
        };
        auto proj2 = [&](double* Q) {
            return batch2([&](int b) {
                GemmProb p = gemm_nn(Q + b * nk, k, st->Gm + b * kk, k, st->Rb + b * nk, k, n, k, k,
                                     -1.0, 1.0);
                p.gate = st->dead_dev + 2 * k + b;
                return p;
            });
        };
        P.projQw1 = proj1(st->Qw);
        P.projQw2 = proj2(st->Qw);
    }

    // Frobenius normalisation of the double layers and of a fresh environment
    st->norm_a_first = (long)st->norms.size();
    const long qa = (long)q * q * q * q;
    for (int i = 0; i < 4; ++i) st->norms.push_back({st->a_base + i * qa, qa});
    st->norm_a_pre_first = (long)st->norms.size();
    for (int i = 0; i < 4; ++i) st->norms.push_back({st->a_base_pre + i * qa, qa});
    st->norm_env_first = (long)st->norms.size();
    for (int i = 0; i < 16; ++i) st->norms.push_back({off(st->Cenv, i * cc, e), cc});
    for (int i = 0; i < 16; ++i) st->norms.push_back({off(st->Tenv, i * cqc, e), cqc});

    // readout: per site, L' = (T4 (C1 T1)) C2 and R' = (T2 (C3 T3)) C4; once
    // on the live tensors and scratch, once on the snapshot of the
    // asynchronous readout
    auto build_read = [&](void* Cb, void* Tb, void* X1b, void* X2b, void* X2pb, void* Eb, void* Eoutb,
                          GemmGroup* g) {
        auto Cq = [&](int site, int kk) { return off(Cb, (site * 4 + kk) * cc, e); };
        auto Tq = [&](int site, int kk) { return off(Tb, (site * 4 + kk) * cqc, e); };
        std::vector<GemmProb> r1, r2, r3, r4;
        const long q4 = (long)q * q * q * q;
        for (int s = 0; s < 4; ++s) {
            for (int side = 0; side < 2; ++side) {
                const int g0 = side ? 2 : 0;
                const int blk = side * 4 + s;
                char* x1 = off(X1b, blk * cqc, e);
                char* x2 = off(X2b, blk * n2, e);
                r1.push_back(gemm_nn(Cq(s, g0), chi, Tq(s, g0), (long)q * chi, x1, (long)q * chi, chi,
                                     q * chi, chi));
                r2.push_back(gemm_nn(Tq(s, (g0 + 3) % 4), chi, x1, (long)q * chi, x2, (long)q * chi,
                                     chi * q, q * chi, chi));
                // contract the open chi leg with the next corner (C2 resp. C4)
                r3.push_back(gemm_nn(x2, chi, Cq(s, g0 + 1), chi, off(X2pb, blk * n2, e), chi,
                                     chi * q * q, chi, chi));
            }
            // E[s] = Lp (q^2 x chi^2) . Rp (chi^2 x q^2)
            r4.push_back(gemm_nn(off(Eb, s * n2, e), (long)chi * chi, off(Eb, (4 + s) * n2, e),
                                 (long)q * q, off(Eoutb, s * q4, e), (long)q * q, q * q, q * q,
                                 chi * chi));
        }
        g[0] = add_group(st, r1, dst);
        g[1] = add_group(st, r2, dst);
        g[2] = add_group(st, r3, dst);
        g[3] = add_group(st, r4, dst);
    };
    {
        GemmGroup g[4];
        build_read(st->Cenv, st->Tenv, st->X1, st->X2, st->X2p, st->E, st->Eout, g);
        st->read1 = g[0], st->read2 = g[1], st->read3 = g[2], st->read4 = g[3];
        build_read(st->Csnap, st->Tsnap, st->X1r, st->X2r, st->X2pr, st->Er, st->Eout_r, g);
        st->read1r = g[0], st->read2r = g[1], st->read3r = g[2], st->read4r = g[3];
    }

    // upload
    HIP_CHECK(hipMalloc(&st->d_probs, st->probs.size() * sizeof(GemmProb)));
    HIP_CHECK(hipMemcpy(st->d_probs, st->probs.data(), st->probs.size() * sizeof(GemmProb),
                        hipMemcpyHostToDevice));
    HIP_CHECK(hipMalloc(&st->d_norms, st->norms.size() * sizeof(NormItem)));
    HIP_CHECK(hipMemcpy(st->d_norms, st->norms.data(), st->norms.size() * sizeof(NormItem),
                        hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(st->d_a_lu, st->a_lu, 16 * sizeof(void*), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(st->d_a_dl, st->a_dl, 16 * sizeof(void*), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(st->d_a_lu_pre, st->a_lu_pre, 16 * sizeof(void*), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(st->d_a_dl_pre, st->a_dl_pre, 16 * sizeof(void*), hipMemcpyHostToDevice));
}

void build_layers(ipeps_state* st) {
    // H_A, H_B, V_A, V_B: bonds named by their left / upper site
    const int bonds[4][2][2] = {{{0, 0}, {1, 1}}, {{1, 0}, {0, 1}}, {{0, 0}, {1, 1}}, {{1, 0}, {0, 1}}};
    const int seq_layer[7] = {0, 1, 2, 3, 2, 1, 0};
    const int seq_full[7] = {0, 0, 0, 1, 0, 0, 0};
    for (int i = 0; i < 7; ++i) {
        const int L = seq_layer[i];
        LayerDesc& ld = st->layers[i];
        ld.gate = L * 2 + seq_full[i];
        for (int b = 0; b < 2; ++b) {
            const int x = bonds[L][b][0], y = bonds[L][b][1];
            BondDesc& bd = ld.bond[b];
            if (L < 2) {  // horizontal (x,y).right -- (x+1,y).left
                bd.site_i = idx(x, y);
                bd.site_j = idx(x + 1, y);
                bd.leg_i = 4;
                bd.leg_j = 2;
                bd.lam_b = hl(x, y);
                bd.outer_i[0] = vl(x, y - 1);
                bd.outer_i[1] = hl(x - 1, y);
                bd.outer_i[2] = vl(x, y);
                bd.outer_j[0] = vl(x + 1, y - 1);
                bd.outer_j[1] = vl(x + 1, y);
                bd.outer_j[2] = hl(x + 1, y);
            } else {  // vertical (x,y).down -- (x,y+1).up
                bd.site_i = idx(x, y);
                bd.site_j = idx(x, y + 1);
                bd.leg_i = 3;
                bd.leg_j = 1;
                bd.lam_b = vl(x, y);
                bd.outer_i[0] = vl(x, y - 1);
                bd.outer_i[1] = hl(x - 1, y);
                bd.outer_i[2] = hl(x, y);
                bd.outer_j[0] = hl(x - 1, y + 1);
                bd.outer_j[1] = vl(x, y + 1);
                bd.outer_j[2] = hl(x, y + 1);
            }
        }
    }
}

void set_neel(ipeps_state* st) {
    const int D = st->D, d = st->d, dA = st->cfg.d_A;
    const long D4 = (long)D * D * D * D;
    std::vector<cplx> g(4 * d * D4, cmake(0, 0));
    for (int s = 0; s < 4; ++s) {
        const int x = s % 2, y = s / 2;
        const int p = ((x + y) % 2 == 0) ? 0 : 1;
        for (int a = 0; a < dA; ++a) g[s * d * D4 + (p * dA + a) * D4] = cmake(1.0 / std::sqrt((double)dA), 0);
    }
    std::vector<double> lam(8 * D, 0.0);
    for (int b = 0; b < 8; ++b) lam[b * D] = 1.0;
    HIP_CHECK(hipMemcpyAsync(st->gam, g.data(), g.size() * sizeof(cplx), hipMemcpyHostToDevice, st->stream));
    HIP_CHECK(hipMemcpyAsync(st->lam, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice, st->stream));
    HIP_CHECK(hipMemsetAsync(st->eps, 0, 4 * sizeof(double), st->stream));
    const uint64_t ctr[2] = {st->cfg.seed, 0};  // refill seed and call count
    HIP_CHECK(hipMemcpyAsync(st->refill_ctr, ctr, sizeof(ctr), hipMemcpyHostToDevice, st->stream));
    HIP_CHECK(hipEventRecord(st->ev_gamma_free, st->stream));
    HIP_CHECK(hipStreamSynchronize(st->stream));
}

// ---------------------------------------------------------------- CTMRG pieces
// A = Gamma sqrt(lambda), the truncation-error snapshot and the normalised
// double layer of the current state into (A, a_base, eps) on stream s; a
// scale per site changes no projector, spectrum or expectation value, and
// unit norm keeps the cut products far from the FP32 underflow range.
void build_double_layers(ipeps_state* st, hipStream_t s, cplx* A, double* a_base, double* eps_snap,
                         long norm_first, double* ws) {
    absorb_sqrt_lambda(s, st->D, st->d, st->gam, st->lam, A);
    HIP_CHECK(hipMemcpyAsync(eps_snap, st->eps, 4 * sizeof(double), hipMemcpyDeviceToDevice, s));
    double_layer_real(s, st->D, st->d, A, a_base);
    normalize_tensors(s, IPEPS_DTYPE_FP64, st->d_norms + norm_first, 4, ws);
}

// Double layers of every job for the CTMRG about to run on the lead's main
// stream: the ones the simple update built ahead (swapped in, frame copies
// copied whole), or built here.
void prepare_double_layers(const Ex& x) {
    ipeps_state* L = x.st;
    hipStream_t s = L->stream;
    HIP_CHECK(hipStreamWaitEvent(s, L->ev_su_done, 0));
    const long q4 = (long)L->q * L->q * L->q * L->q;
    bool all_pre = true;
    for (ipeps_state* st : x.jobs) all_pre = all_pre && st->pre_valid && st->pre_step == st->step_count;
    if (all_pre) {
        // built at the tail of the simple update (ordered by ev_su_done),
        // frame copies included: one device copy into the plan's buffers
        for (ipeps_state* st : x.jobs) {
            std::swap(st->A, st->A_pre);
            std::swap(st->a_base, st->a_base_pre);
            std::swap(st->eps_snap, st->eps_snap_pre);
            std::swap(st->norm_a_first, st->norm_a_pre_first);
            st->pre_valid = false;
            st->ctm_step = st->step_count;
        }
        copy_jobs(s, L->frames, L->frames_pre, 32 * q4 * L->esz, x.jm);
        // the next simple update may rebuild the *_pre buffers (frames_pre
        // included) once this point is passed
        HIP_CHECK(hipEventRecord(L->ev_gamma_free, s));
        return;
    }
    for (ipeps_state* st : x.jobs) {
        absorb_sqrt_lambda(s, st->D, st->d, st->gam, st->lam, st->A);
        HIP_CHECK(hipMemcpyAsync(st->eps_snap, st->eps, 4 * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    HIP_CHECK(hipEventRecord(L->ev_gamma_free, s));
    for (ipeps_state* st : x.jobs) {
        double_layer_real(s, st->D, st->d, st->A, st->a_base);
        normalize_tensors(s, IPEPS_DTYPE_FP64, st->d_norms + st->norm_a_first, 4, st->norm_ws);
        frame_layouts(s, st->q, st->dtype, st->a_base, st->d_a_lu, st->d_a_dl);
        st->pre_valid = false;
        st->ctm_step = st->step_count;
    }
}

// Order the main stream after all enqueued simple-update work.
void join_su(ipeps_state* st) { HIP_CHECK(hipStreamWaitEvent(st->stream, st->ev_su_done, 0)); }

// Column-normalised Cholesky QR of X (n x k, batch 2) into Q.  Columns that
// the Cholesky drops as dependent (their directions sit below the rounding
// level of the dominant ones) are, with refill, restarted as random vectors
// made orthogonal to the kept columns by two projections: the block keeps k
// independent directions, and the next power step with N pulls out the
// directions the dominant ones were hiding.  two_pass re-orthonormalises Q
// back into X (CholQR2).
void orth(const Ex& x, double* X, double* Q, const GemmGroup& gram1, const GemmGroup& mul1,
          const GemmGroup& gram2, const GemmGroup& mul2, bool two_pass,
          const GemmGroup* proj1 = nullptr, const GemmGroup* proj2 = nullptr) {
    ipeps_state* st = x.st;
    const bool refill = proj1 && proj2;
    const int n = st->n, k = st->k;
    hipStream_t s = st->stream;
    // chol_inverse scales the Gram to unit diagonal itself (equivalent to
    // normalising the columns first)
    run(x, gram1);
    chol_inverse(s, 2, k, st->Gm, st->Ri, kCholDrop, refill ? st->dead_dev : nullptr, 0.0, x.jm);
    run(x, mul1);
    if (refill) {
        // each job's own random stream (its seed, its device-side call
        // counter); the blocks of a job that dropped nothing return at once
        dead_fill(s, 2, n, k, st->dead_dev, st->refill_ctr, st->Rb, x.jm);
        for (int pass = 0; pass < 2; ++pass) {
            run(x, *proj1);  // Gm = Q^T Rb
            run(x, *proj2);  // Rb -= Q Gm
        }
        add_gated(s, 2, (long)n * k, st->dead_dev + 2 * k, st->Rb, Q, x.jm);
    }
    if (!two_pass) return;
    run(x, gram2);
    // second pass: when the first left the columns orthonormal to 1e-13 the
    // factorisation would change them by no more than that; it is skipped
    chol_inverse(s, 2, k, st->Gm, st->Ri, kCholDrop, nullptr, 1e-13, x.jm);
    run(x, mul2);
}

// Relative cutoff below which singular values of a cut matrix count as zero:
// 1e-12 with FP64 products.  With FP32 products the tail below ~1e-6 is
// rounding noise, but such directions enter the renormalised tensors with
// weight sqrt(sigma): cutting at 1e-6 moved the D=6, chi=72 imbalance by 1e-4,
// at 1e-9 or 1e-12 by ~5e-6; 1e-9 is used.
double proj_cutoff(const ipeps_state* st) { return st->dtype == IPEPS_DTYPE_FP64 ? 1e-12 : 1e-9; }

// Yw = N Qz and Zw = N^T Qw for the two cuts: with the formed N64 (FP64), or
// through the enlarged corners (products in dtype; FP64 blocks converted at
// both ends in FP32 mode).
// Yw = N V; with copy, also Zw = Yw (returns whether that copy was made:
// the FP64 conversion at the end of a chain in FP32 or BF16 writes both).
bool apply_n(const Ex& x, int si, bool copy = false) {
    ipeps_state* st = x.st;
    if (!st->factored) {
        run(x, st->svd.NVf);
        return false;
    }
    const long nk = (long)st->n * st->k;
    const bool f64 = st->dtype == IPEPS_DTYPE_FP64;
    if (!f64) from_fp64_blocks(st->stream, st->dtype, st->Qz, st->Ch[2], 2, st->n, st->k, false, x.jm);
    for (const GemmGroup& g : st->svd.NV[si]) run(x, g);
    if (!f64) to_fp64(st->stream, st->dtype, st->Ch[1], st->Yw, 2 * nk, x.jm, copy ? st->Zw : nullptr);
    return copy && !f64;
}

void apply_nt(const Ex& x, int si) {
    ipeps_state* st = x.st;
    if (!st->factored) return run(x, st->svd.NtQf);
    const long nk = (long)st->n * st->k;
    from_fp64_blocks(st->stream, st->dtype, st->Qw, st->Qt, 2, st->n, st->k, true, x.jm);
    for (const GemmGroup& g : st->svd.NtQ[si]) run(x, g);
    if (st->dtype != IPEPS_DTYPE_FP64) to_fp64(st->stream, st->dtype, st->Ch[2], st->Zw, 2 * nk, x.jm);
}

// Columns of a projector SVD's matrix A left unrotated by the Jacobi: below
// skip |A|_F, i.e. below skip sqrt(k) sigma_1, far under the projector
// cutoff (a kept direction never rotated against the dominant ones would
// break P_up P_low = 1): 1e-14 with FP64 products (cutoff 1e-12), 5e-11 with
// FP32 or BF16 products (cutoff 1e-9; 5e-11 sqrt(k) < 1e-9 up to k = 400).
// The rotations among the columns between 1e-14 and 5e-11 of |A|_F cost the
// Rayleigh-Ritz Jacobi about one of its seven sweeps at D=6, chi=72, k=80.
double svd_skip(const ipeps_state* st) { return st->dtype == IPEPS_DTYPE_FP64 ? 1e-14 : 5e-11; }

// Truncated SVD of the two cut matrices (formed in N64, or applied through
// the enlarged corners in E); fills Us, Vs and g_dev.
void launch_aux_ahead(const Ex& x, int si);
void launch_side_spectra(const Ex& x);
void launch_side_readout(const Ex& x);
void projector_svd(const Ex& x, int slot) {
    ipeps_state* st = x.st;
    const int n = st->n, k = st->k, chi = st->chi;
    hipStream_t s = st->stream;
    const JobMap& jm = x.jm;
    if (n <= kDirectMax) {
        jacobi_svd_real(s, 2, n, n, st->N64, n, (long)n * n, st->sig, st->Uo, st->Vo, st->jwork, svd_skip(st),
                        jm);
        projector_factors(s, st->dtype, 2, n, n, chi, proj_cutoff(st), st->Uo, st->Vo, st->sig,
                          (long)n * n, st->Us, st->Vs, (long)n * chi, st->g_dev, jm);
        return;
    }
    const long nk = (long)n * k;
    SvdPlan& P = st->svd;
    const bool warm = st->warm_valid[2 * slot];
    // the current right block V lives in Qz (orthonormal after orth)
    if (warm) {
        copy_jobs(s, st->Qz, st->warm + 2 * slot * nk, 2 * nk * sizeof(double), jm);
    } else {
        for (ipeps_state* j : x.jobs)
            random_block(s, 2, n, k, j->cfg.seed * 1315423911ull + (uint64_t)slot + 1, j->Zw);
        orth(x, st->Zw, st->Qz, P.gramZ, P.QfromZ, P.gramQz, P.ZfromQz, true);
        copy_jobs(s, st->Qz, st->Zw, 2 * nk * sizeof(double), jm);
    }
    int iters = warm ? (st->dtype == IPEPS_DTYPE_FP64 ? kWarmIters : kWarmItersLow) : kColdIters;
    if (warm) iters += st->extra_warm_iters;
    for (int it = 0; it < iters; ++it) {
        // power step with one Cholesky-QR pass per side (only the span
        // matters).  Dropped left columns are restarted; a right column
        // dropped here is zero in V, hence dead in the next left block and
        // restarted there.  Zero columns of the final V only add zero Ritz
        // values.
        apply_n(x, slot);  // Yw = N V
        orth(x, st->Yw, st->Qw, P.gramY, P.QfromY, P.gramQ, P.YfromQ, false, &P.projQw1, &P.projQw2);
        apply_nt(x, slot);  // Zw = N^T Qw
        orth(x, st->Zw, st->Qz, P.gramZ, P.QfromZ, P.gramQz, P.ZfromQz, false);
    }
    // Rayleigh-Ritz on span(N V) x span(V)
    if (!apply_n(x, slot, true)) copy_jobs(s, st->Zw, st->Yw, 2 * nk * sizeof(double), jm);
    orth(x, st->Yw, st->Qw, P.gramY, P.QfromY, P.gramQ, P.YfromQ, true);
    run(x, P.Cs);  // Cs = (Q^T N V)^T
    if (st->aux_defer >= 0) {
        const int sd = st->aux_defer;
        st->aux_defer = -1;
        launch_aux_ahead(x, sd);
    }
    if (slot == 1) launch_side_spectra(x);
    if (slot == (st->dtype == IPEPS_DTYPE_FP64 ? 1 : 5)) launch_side_readout(x);
    // Rayleigh-Ritz SVD (columns below svd_skip |Cs|_F left unrotated).
    // (Taking the right vectors as Cs^T U S^-1 instead of accumulating them
    // halves the Jacobi traffic but moved the FP32 imbalance by 2e-4 at D=6,
    // chi=72; not used.)
    jacobi_svd_real(s, 2, k, k, st->Cs, k, (long)k * k, st->sig, st->Uc, st->Vc, st->jwork, svd_skip(st), jm);
    run(x, P.UoVo[slot]);
    double* Vo = st->warm + 2 * slot * nk;  // V_o of both cuts (and the next warm start)
    for (ipeps_state* j : x.jobs) j->warm_valid[2 * slot] = j->warm_valid[2 * slot + 1] = true;
    if (st->factored) {
        // one launch: Uc S^-1/2 truncated (k x chi, into VsK) and the
        // projector factors Us, Vs from Uo, Vo; then P_low = T2 (Uc S^-1/2)
        ProjFactorsPair pp{};
        pp.n[0] = k;
        pp.U[0] = st->Uc;
        pp.V[0] = st->Uc;
        pp.strideUV[0] = (long)k * k;
        pp.Us[0] = nullptr;
        pp.Vs[0] = st->VsK;
        pp.strideP[0] = (long)k * chi;
        pp.g_out[0] = nullptr;
        pp.n[1] = n;
        pp.U[1] = st->Uo;
        pp.V[1] = Vo;
        pp.strideUV[1] = nk;
        pp.Us[1] = st->Us;
        pp.Vs[1] = st->Vs;
        pp.strideP[1] = (long)n * chi;
        pp.g_out[1] = st->g_dev;
        projector_factors_pair(s, st->dtype, 2, k, chi, proj_cutoff(st), st->sig, pp, jm);
        run(x, P.PlowT2);
        return;
    }
    projector_factors(s, st->dtype, 2, n, k, chi, proj_cutoff(st), st->Uo, Vo, st->sig, nk, st->Us,
                      st->Vs, (long)n * chi, st->g_dev, jm);
}

void readout_enqueue(ipeps_state* st, hipStream_t s, bool snap);

// pinned host slots of the asynchronous readout (host_buf holds 65536)
constexpr int kAsyncHost = 1024;

// Enqueue the deferred corner spectra (of every job) on the lead's spectra
// stream, after the FP64 snapshot of the corners and, if given, after event
// `after` of the main stream.
void launch_deferred_spectra(const Ex& x, hipEvent_t after) {
    ipeps_state* st = x.st;
    if (!st->spec_deferred) return;
    const int chi = st->chi;
    hipStream_t ss = st->spec_stream;
    // under capture the spectra stream forks from the main stream at `after`,
    // which the snapshot precedes
    if (!st->capturing) HIP_CHECK(hipStreamWaitEvent(ss, st->ev_c64_ready, 0));
    if (after) HIP_CHECK(hipStreamWaitEvent(ss, after, 0));
    // spectra are reported to 1e-8 sigma_1 (FP64 corners) and carry the
    // ~1e-7 rounding of FP32 corners: columns below 1e-10 (FP64) or 1e-8
    // (FP32) of |C|_F need no rotation
    jacobi_svd_real(ss, 16, chi, chi, st->C64, chi, (long)chi * chi, st->csig, nullptr, nullptr,
                    st->jwork_c, st->dtype == IPEPS_DTYPE_FP64 ? 1e-10 : 1e-8, x.jm);
    // an asynchronous readout may still have to copy the previous Delta
    // (under capture the main stream waits for it before the graph's launch)
    if (!st->capturing) HIP_CHECK(hipStreamWaitEvent(ss, st->ev_ro_done, 0));
    spectra_delta(ss, 16, chi, st->csig, st->spectra, st->spec_prev, st->dev_scalars,
                  st->spec_first ? 1 : 0, x.jm);
    HIP_CHECK(hipEventRecord(st->ev_spec_done, ss));
    for (ipeps_state* j : x.jobs) j->spec_deferred = false;
}

// Enqueue a deferred asynchronous readout on ro_stream, after the snapshot
// and, if given, after event `after` of the main stream (the spectra of its
// environment first: the readout reports their Delta).  One job only.
void launch_deferred_readout(ipeps_state* st, hipEvent_t after) {
    if (!st->ro_deferred) return;
    launch_deferred_spectra(solo(st), after);
    hipStream_t rs = st->ro_stream;
    HIP_CHECK(hipStreamWaitEvent(rs, st->ev_ro_snap, 0));
    if (after) HIP_CHECK(hipStreamWaitEvent(rs, after, 0));
    readout_enqueue(st, rs, true);
    double* h = st->host_buf + kAsyncHost;
    HIP_CHECK(hipMemcpyAsync(h, st->obs_r, 16 * sizeof(double), hipMemcpyDeviceToHost, rs));
    HIP_CHECK(hipMemcpyAsync(h + 16, st->eps_r, 4 * sizeof(double), hipMemcpyDeviceToHost, rs));
    // Delta of the snapshot's environment (its CTMRG recorded ev_spec_done last:
    // a later CTMRG records it only after its spectra, which wait for
    // ev_ro_done before they overwrite Delta)
    HIP_CHECK(hipStreamWaitEvent(rs, st->ev_spec_done, 0));
    HIP_CHECK(hipMemcpyAsync(h + 20, st->dev_scalars, sizeof(double), hipMemcpyDeviceToHost, rs));
    HIP_CHECK(hipEventRecord(st->ev_ro_done, rs));
    st->ro_deferred = false;
}

// The UR / DR corners of column step si + 1 on the aux stream, once the
// main stream has passed everything that wrote the tensors they read (they
// read only tensors the move leaves alone).
void launch_aux_ahead(const Ex& x, int si) {
    ipeps_state* st = x.st;
    const ColumnStep& nx = st->steps[si + 1];
    HIP_CHECK(hipEventRecord(st->ev_aux_go, st->stream));
    HIP_CHECK(hipStreamWaitEvent(st->aux_stream, st->ev_aux_go, 0));
    run_on(x, st->aux_stream, nx.aux_s1);
    run_on(x, st->aux_stream, nx.aux_s2);
    run_on(x, st->aux_stream, nx.aux_s3);
    HIP_CHECK(hipEventRecord(st->ev_aux_done, st->aux_stream));
}

// The spectra of the previous environment (spectra stream) and a readout
// started after the previous CTMRG run (readout stream), each from the point
// of the main stream where it is called on.  With the subspace-iteration SVD
// the spectra start with the second column step's Rayleigh-Ritz Jacobi (a
// Jacobi phase whose idle CUs the corners ahead do not fill), and so does
// the readout in FP64; with FP32 or BF16 contractions the readout starts
// with the sixth column step's (after the second, its products slowed the
// T update that follows; FP64 steps lost 5 ms with it there).  With the
// direct SVD both start with the first column step's SVD.
void launch_side_spectra(const Ex& x) {
    ipeps_state* st = x.st;
    HIP_CHECK(hipEventRecord(st->ev_side_go, st->stream));
    launch_deferred_spectra(x, st->ev_side_go);
}
void launch_side_readout(const Ex& x) {
    ipeps_state* st = x.st;
    if (x.batched()) return;
    HIP_CHECK(hipEventRecord(st->ev_side_go, st->stream));
    launch_deferred_readout(st, st->ev_side_go);
}

void column_step(const Ex& x, int si) {
    ipeps_state* st = x.st;
    const ColumnStep& cs = st->steps[si];
    const int q = st->q, chi = st->chi, n = st->n;
    const long n2 = (long)n * n;
    hipStream_t s = st->stream;
    const bool warm = si == 0 && st->corners_warm;
    run(x, warm ? cs.s1w : cs.s1);
    run(x, warm ? cs.s2w : cs.s2);
    run(x, warm ? cs.s3w : cs.s3);
    if (si % 2 == 0) {
        // the next column step's UR / DR corners go to the aux stream; with
        // the subspace-iteration SVD they start with its Rayleigh-Ritz
        // Jacobi (launch_aux_ahead from projector_svd), whose one workgroup
        // per cut leaves the GPU to them, instead of sharing it with the
        // chain products before it
        if (n > kDirectMax) {
            st->aux_defer = si;
        } else {
            launch_aux_ahead(x, si);
            if (si == 0) {
                launch_side_spectra(x);
                launch_side_readout(x);
            }
        }
    } else {
        HIP_CHECK(hipStreamWaitEvent(s, st->ev_aux_done, 0));
    }
    if (!st->factored) {
        run(x, cs.half);
        run(x, cs.nprod);
        if (st->dtype != IPEPS_DTYPE_FP64) to_fp64(s, st->dtype, st->Nd, st->N64, 2 * n2, x.jm);
    }
    projector_svd(x, si);
    run(x, cs.proj);
    run(x, cs.proj2);
    const size_t e = st->esz;
    // PupP[c'][D][t4p] <- Pup[c'][t4p][D];  PlowP[q3][c4n][c'] <- Plow[c4n][q3][c'];
    // T4p[Y][t][c][v] <- T4[t][v][c]: six independent copies, one launch
    Permute3Batch pb{};
    auto add = [&](int mode, int A, int B, int C, const void* in, void* out) {
        const int i = pb.n++;
        pb.mode[i] = mode;
        pb.A[i] = A;
        pb.B[i] = B;
        pb.C[i] = C;
        pb.in[i] = in;
        pb.out[i] = out;
    };
    for (int Y = 0; Y < 2; ++Y) {
        add(1, chi, chi, q, off(st->Pup, Y * (long)n * chi, e), off(st->PupP, Y * (long)n * chi, e));
        add(0, chi, q, chi, off(st->Plow, Y * (long)n * chi, e), off(st->PlowP, Y * (long)n * chi, e));
    }
    for (int Y = 0; Y < 2; ++Y) add(1, chi, q, chi, cs.t4[Y], off(st->T4p, Y * (long)chi * q * chi, e));
    permute3_batch(s, st->dtype, pb, x.jm);
    run(x, cs.w1);
    run(x, cs.w2);
    run(x, cs.fin);
    normalize_items(x, s, st->dtype, cs.norm_first, 6, st->norm_ws);
}

// Snapshot the 16 corners (FP64) on the main stream; their spectra and the
// change Delta follow on the spectra stream, deferred like an asynchronous
// readout: the next CTMRG iteration enqueues them part way through
// (launch_side_spectra), where they fill CUs its SVD leaves idle, or any
// reader of spectra / Delta does (wait_spectra).
void corner_spectra_update(const Ex& x, bool first) {
    ipeps_state* st = x.st;
    const int chi = st->chi;
    hipStream_t s = st->stream;
    launch_deferred_spectra(x, nullptr);  // an earlier update nobody launched yet
    HIP_CHECK(hipStreamWaitEvent(s, st->ev_spec_done, 0));  // C64 free again
    to_fp64(s, st->dtype, st->Cenv, st->C64, 16L * chi * chi, x.jm);
    HIP_CHECK(hipEventRecord(st->ev_c64_ready, s));
    for (ipeps_state* j : x.jobs) {
        j->spec_deferred = true;
        j->spec_first = first;
        j->spectra_valid = true;
    }
}

void wait_spectra(const Ex& x) {
    launch_deferred_spectra(x, nullptr);
    HIP_CHECK(hipStreamWaitEvent(x.st->stream, x.st->ev_spec_done, 0));
}

// n_steps Trotter steps of every job on the lead's simple-update stream (one
// launch per layer for all jobs), then each job's double layers for the next
// CTMRG, built there ahead of it.
void trotter_steps(const Ex& x, int n_steps) {
    ipeps_state* L = x.st;
    hipStream_t ss = L->su_stream;
    HIP_CHECK(hipStreamWaitEvent(ss, L->ev_gamma_free, 0));
    for (int t = 0; t < n_steps; ++t) {
        for (int l = 0; l < 7; ++l)
            su_layer(ss, L->D, L->d, L->layers[l], L->gam, L->lam, L->eps, L->gates, L->su_scratch, x.jm);
        for (ipeps_state* j : x.jobs) j->step_count++;
    }
    if (n_steps > 0) {
        // build the next CTMRG's double layers here, hidden behind the
        // current CTMRG; the *_pre buffers were last read by main-stream
        // work that precedes ev_gamma_free
        for (ipeps_state* j : x.jobs) {
            build_double_layers(j, ss, j->A_pre, j->a_base_pre, j->eps_snap_pre, j->norm_a_pre_first,
                                j->norm_ws_su);
            frame_layouts(ss, j->q, j->dtype, j->a_base_pre, j->d_a_lu_pre, j->d_a_dl_pre);
            j->pre_valid = true;
            j->pre_step = j->step_count;
        }
    }
    HIP_CHECK(hipEventRecord(L->ev_su_done, ss));
}

// One warm CTMRG iteration captured from the lead's main stream into an
// executable graph (nothing runs).  Valid for the iterations after the first
// of a call with a fixed count: every projector subspace warm, the left move
// reusing the down move's corners, the previous iteration's spectra deferred,
// no added warm iterations.  The plan's buffers and tables are fixed for the
// life of the jobs (a batch's merged tables for the life of the batch), and
// the refill seeds count up on the device, so a replay does exactly what
// the same iteration enqueued eagerly does.
// The capture runs on `cap`, a stream of the caller's that stands in for the
// lead's main stream (which may be the null stream, where no capture is
// possible); the graph is launched on the main stream.
hipGraphExec_t capture_warm_iteration(const Ex& x, hipStream_t cap) {
    ipeps_state* L = x.st;
    hipGraph_t g = nullptr;
    hipStream_t main_stream = L->stream;
    HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    L->stream = cap;
    L->capturing = true;
    try {
        for (int si = 0; si < 8; ++si) column_step(x, si);
        corner_spectra_update(x, false);
    } catch (...) {
        L->capturing = false;
        L->stream = main_stream;
        (void)hipStreamEndCapture(cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    L->capturing = false;
    L->stream = main_stream;
    HIP_CHECK(hipStreamEndCapture(cap, &g));
    hipGraphExec_t ge = nullptr;
    const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_CHECK(e);
    return ge;
}

// CTMRG iterations of every job (section Readout; appendix).  tol <= 0:
// exactly max_iter; else until the lead's Delta < tol (one job only).
// want_delta: the lead's last Delta is read back.  graph (tol <= 0 only):
// the iterations after the first replay the warm-iteration graph held
// there, captured on stream cap on first use.
void ctmrg_iterations(const Ex& x, double tol, int max_iter, bool cold_start, bool want_delta, int* it_done,
                      double* dl, hipGraphExec_t* graph = nullptr, hipStream_t cap = nullptr) {
    ipeps_state* L = x.st;
    prepare_double_layers(x);
    if (cold_start || !L->have_env) {
        for (ipeps_state* j : x.jobs)
            init_environment(L->stream, j->D, j->chi, j->dtype, j->a_base, j->Cenv, j->Tenv);
        normalize_items(x, L->stream, L->dtype, L->norm_env_first, 32, L->norm_ws);
        for (ipeps_state* j : x.jobs) {
            for (bool& w : j->warm_valid) w = false;
            j->have_env = true;
        }
        corner_spectra_update(x, true);
    } else if (!L->spectra_valid) {
        corner_spectra_update(x, true);
    }
    // Converging to tol: once the spectra move by less than 1e-5 (1e-7) per
    // iteration, the warm-started projector subspaces get two (four) more
    // power iterations, so that their error (which decays like
    // (s_{k+1}/s_chi)^(2q) per iteration) stays below the change being
    // resolved; a fixed iteration count (tol <= 0) keeps the plain schedule.
    L->extra_warm_iters = 0;
    L->corners_warm = false;
    const bool replay = graph && tol <= 0 && L->extra_warm_iters == 0 && !L->prof_on;
    for (int it = 0; it < max_iter; ++it) {
        if (replay && it > 0) {
            if (!*graph) *graph = capture_warm_iteration(x, cap);
            HIP_CHECK(hipStreamWaitEvent(L->stream, L->ev_ro_done, 0));
            HIP_CHECK(hipGraphLaunch(*graph, L->stream));
            // the graph ends with this iteration's corner snapshot, its
            // spectra (of the previous one) already joined
            HIP_CHECK(hipEventRecord(L->ev_spec_done, L->stream));
            HIP_CHECK(hipEventRecord(L->ev_c64_ready, L->stream));
            for (ipeps_state* j : x.jobs) {
                j->spec_deferred = true;
                j->spec_first = false;
                j->spectra_valid = true;
            }
        } else {
            for (int si = 0; si < 8; ++si) column_step(x, si);
            L->corners_warm = true;  // the next left move may reuse the down move's corners
            corner_spectra_update(x, false);
        }
        *it_done = it + 1;
        if (tol > 0 || (want_delta && it + 1 == max_iter)) {
            wait_spectra(x);
            HIP_CHECK(hipMemcpyAsync(L->host_buf, L->dev_scalars, sizeof(double), hipMemcpyDeviceToHost, L->stream));
            HIP_CHECK(hipStreamSynchronize(L->stream));
            *dl = L->host_buf[0];
            IPEPS_REQUIRE(!std::isnan(*dl), IPEPS_ENUMERIC, "NaN in the environment");
            if (tol > 0 && *dl < tol) break;
            if (tol > 0) L->extra_warm_iters = *dl < 1e-7 ? 4 : (*dl < 1e-5 ? 2 : 0);
        }
    }
    for (ipeps_state* j : x.jobs) {
        j->extra_warm_iters = 0;
        j->corners_warm = false;
        j->last_iters = *it_done;
        j->last_delta = *dl;
    }
}

void check_poison(ipeps_state* st) {
    IPEPS_REQUIRE(!st->poisoned, IPEPS_ENUMERIC, "state poisoned by an earlier NaN/Inf");
}

int guard(ipeps_state* st, int code) {
    if (code == IPEPS_ENUMERIC && st) st->poisoned = true;
    return code;
}

template <typename F>
int wrap(ipeps_state* st, F&& fn) {
    try {
        fn();
        return IPEPS_OK;
    } catch (const status_error& e) {
        return guard(st, e.code);
    } catch (const hip_error& e) {
        fprintf(stderr, "ipeps: %s\n", e.what());
        return IPEPS_EDEVICE;
    } catch (const std::bad_alloc&) {
        return IPEPS_ENOMEM;
    }
}

}  // namespace

// ==================================================================== C ABI
extern "C" {

void ipeps_config_default(ipeps_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->D = 2;
    c->chi = 8;
    c->d_A = 2;
    c->J = 1.0;
    c->V = 1.0;
    c->W = 5.0;
    c->dt = 0.05;
    c->trotter_order = 2;
    c->dtype = IPEPS_DTYPE_FP64;
    for (int l = 0; l < 4; ++l) {
        c->layer_J[l] = 1.0;
        c->layer_V[l] = 1.0;
        c->layer_w[l] = 0.25;
    }
    c->seed = 1;
}

static void fill_dims_internal(ipeps_state* st, const ipeps_config* cfg) {
    st->cfg = *cfg;
    st->D = cfg->D;
    st->d = 2 * cfg->d_A;
    st->q = cfg->D * cfg->D;
    st->chi = cfg->chi;
    st->n = cfg->chi * st->q;
    st->k = choose_k(st->n, cfg->chi, cfg->dtype);
    // the BF16 modes keep the tensors in FP32 and round the MFMA operands
    st->dtype = cfg->dtype == IPEPS_DTYPE_FP64 ? IPEPS_DTYPE_FP64 : IPEPS_DTYPE_FP32;
    st->mma = cfg->dtype;
    st->esz = st->dtype == IPEPS_DTYPE_FP64 ? sizeof(double) : sizeof(float);
    const bool force_f = (cfg->flags & IPEPS_FLAG_FACTORED_CUTS) != 0;
    const bool force_n = (cfg->flags & IPEPS_FLAG_FORMED_CUTS) != 0;
    st->factored = st->n > kDirectMax && (force_f || (!force_n && st->n > kFactoredMin));
}

size_t ipeps_footprint_bytes(const ipeps_config* cfg) {
    try {
        validate(cfg);
        ipeps_state* st = new ipeps_state();
        fill_dims_internal(st, cfg);
        st->mem.dry = true;
        allocate(st);
        size_t tot = st->mem.total;
        delete st;
        return tot + (1 << 20);  // plan tables
    } catch (...) {
        return 0;
    }
}

int ipeps_init(const ipeps_config* cfg, void* hip_stream, ipeps_alloc_fn alloc, ipeps_free_fn free_fn,
               void* alloc_ctx, ipeps_state** out) {
    if (!out) return IPEPS_EINVAL;
    *out = nullptr;
    ipeps_state* st = nullptr;
    int rc = wrap(nullptr, [&] {
        validate(cfg);
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
            throw status_error(IPEPS_EDEVICE, "no HIP device");
        st = new ipeps_state();
        fill_dims_internal(st, cfg);
        st->stream = (hipStream_t)hip_stream;
        st->mem.alloc = alloc;
        st->mem.free_fn = free_fn;
        st->mem.ctx = alloc_ctx;
        st->mem.stream = st->stream;
        allocate(st);
        HIP_CHECK(hipStreamCreateWithFlags(&st->su_stream, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_gamma_free, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_su_done, hipEventDisableTiming));
        HIP_CHECK(hipStreamCreateWithFlags(&st->spec_stream, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_c64_ready, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_spec_done, hipEventDisableTiming));
        HIP_CHECK(hipStreamCreateWithFlags(&st->aux_stream, hipStreamNonBlocking));
        HIP_CHECK(hipStreamCreateWithFlags(&st->ro_stream, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_ro_snap, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_ro_done, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(st->ev_ro_done, st->ro_stream));  // complete: nothing pending
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_aux_go, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_side_go, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&st->ev_aux_done, hipEventDisableTiming));
        HIP_CHECK(hipHostMalloc((void**)&st->host_buf, 65536 * sizeof(double), hipHostMallocDefault));
        st->autotune = (cfg->flags & IPEPS_FLAG_AUTOTUNE) != 0;
        if (st->autotune) {
            HIP_CHECK(hipEventCreate(&st->tune_ev[0]));
            HIP_CHECK(hipEventCreate(&st->tune_ev[1]));
        }
        build_layers(st);
        build_plan(st);
        build_gates(st->stream, st->cfg, st->gates);
        set_neel(st);
    });
    if (rc != IPEPS_OK) {
        if (st) ipeps_destroy(st);
        return rc;
    }
    *out = st;
    return IPEPS_OK;
}

void ipeps_destroy(ipeps_state* st) {
    if (!st) return;
    (void)hipStreamSynchronize(st->stream);
    if (st->su_stream) (void)hipStreamSynchronize(st->su_stream);
    if (st->spec_stream) (void)hipStreamSynchronize(st->spec_stream);
    if (st->aux_stream) (void)hipStreamSynchronize(st->aux_stream);
    if (st->ro_stream) (void)hipStreamSynchronize(st->ro_stream);
    st->mem.release();
    if (st->su_stream) (void)hipStreamDestroy(st->su_stream);
    if (st->spec_stream) (void)hipStreamDestroy(st->spec_stream);
    if (st->aux_stream) (void)hipStreamDestroy(st->aux_stream);
    if (st->ev_aux_go) (void)hipEventDestroy(st->ev_aux_go);
    if (st->ev_side_go) (void)hipEventDestroy(st->ev_side_go);
    if (st->ev_aux_done) (void)hipEventDestroy(st->ev_aux_done);
    if (st->ro_stream) (void)hipStreamDestroy(st->ro_stream);
    if (st->ev_ro_snap) (void)hipEventDestroy(st->ev_ro_snap);
    if (st->ev_ro_done) (void)hipEventDestroy(st->ev_ro_done);
    if (st->ev_c64_ready) (void)hipEventDestroy(st->ev_c64_ready);
    if (st->ev_spec_done) (void)hipEventDestroy(st->ev_spec_done);
    if (st->ev_gamma_free) (void)hipEventDestroy(st->ev_gamma_free);
    if (st->ev_su_done) (void)hipEventDestroy(st->ev_su_done);
    if (st->d_probs) (void)hipFree(st->d_probs);
    if (st->d_norms) (void)hipFree(st->d_norms);
    if (st->tune_dev) (void)hipFree(st->tune_dev);
    for (auto& e : st->tune_ev)
        if (e) (void)hipEventDestroy(e);
    if (st->host_buf) (void)hipHostFree(st->host_buf);
    for (auto& e : st->prof_ev) (void)hipEventDestroy(e);
    delete st;
}

int ipeps_set_state(ipeps_state* st, const double* gamma, const double* lambda) {
    if (!st || !gamma || !lambda) return IPEPS_EINVAL;
    return wrap(st, [&] {
        const long D4 = (long)st->D * st->D * st->D * st->D;
        for (long i = 0; i < 8L * st->D; ++i)
            IPEPS_REQUIRE(std::isfinite(lambda[i]) && lambda[i] >= 0, IPEPS_EINVAL, "bad lambda");
        join_su(st);
        HIP_CHECK(hipMemcpyAsync(st->gam, gamma, 4 * st->d * D4 * sizeof(cplx), hipMemcpyHostToDevice, st->stream));
        HIP_CHECK(hipMemcpyAsync(st->lam, lambda, 8 * st->D * sizeof(double), hipMemcpyHostToDevice, st->stream));
        HIP_CHECK(hipMemsetAsync(st->eps, 0, 4 * sizeof(double), st->stream));
        HIP_CHECK(hipEventRecord(st->ev_gamma_free, st->stream));
        HIP_CHECK(hipStreamSynchronize(st->stream));
        st->have_env = false;
        st->poisoned = false;
        st->spectra_valid = false;
        st->pre_valid = false;
        for (bool& w : st->warm_valid) w = false;
    });
}

int ipeps_get_state(ipeps_state* st, double* gamma, double* lambda) {
    if (!st) return IPEPS_EINVAL;
    return wrap(st, [&] {
        const long D4 = (long)st->D * st->D * st->D * st->D;
        join_su(st);
        if (gamma) HIP_CHECK(hipMemcpyAsync(gamma, st->gam, 4 * st->d * D4 * sizeof(cplx), hipMemcpyDeviceToHost, st->stream));
        if (lambda) HIP_CHECK(hipMemcpyAsync(lambda, st->lam, 8 * st->D * sizeof(double), hipMemcpyDeviceToHost, st->stream));
        HIP_CHECK(hipStreamSynchronize(st->stream));
    });
}

int ipeps_trotter_step(ipeps_state* st, int n_steps, double* trunc_err_out) {
    if (!st || n_steps < 0) return IPEPS_EINVAL;
    return wrap(st, [&] {
        check_poison(st);
        trotter_steps(solo(st), n_steps);
        if (trunc_err_out) {
            hipStream_t ss = st->su_stream;
            HIP_CHECK(hipMemcpyAsync(st->host_buf, st->eps, 4 * sizeof(double), hipMemcpyDeviceToHost, ss));
            HIP_CHECK(hipMemcpyAsync(st->host_buf + 4, st->lam, 8 * st->D * sizeof(double), hipMemcpyDeviceToHost, ss));
            HIP_CHECK(hipStreamSynchronize(ss));
            for (int i = 0; i < 4; ++i) trunc_err_out[i] = st->host_buf[i];
            for (int i = 0; i < 8 * st->D; ++i)
                IPEPS_REQUIRE(std::isfinite(st->host_buf[4 + i]), IPEPS_ENUMERIC, "NaN in bond weights");
        }
    });
}

int ctmrg_converge(ipeps_state* st, double tol, int max_iter, int cold_start, int* iters, double* delta) {
    if (!st || max_iter < 1) return IPEPS_EINVAL;
    int it_done = 0;
    double dl = INFINITY;
    int rc = wrap(st, [&] {
        check_poison(st);
        ctmrg_iterations(solo(st), tol, max_iter, cold_start != 0, delta != nullptr, &it_done, &dl);
        if (tol > 0 && !(dl < tol)) throw status_error(IPEPS_ENOTCONV, "CTMRG not converged");
    });
    if (iters) *iters = it_done;
    if (delta) *delta = dl;
    return rc;
}

}  // extern "C"

namespace {
// The readout of one environment on stream s: the live tensors and scratch,
// or (snap) the snapshot taken by ipeps_observe_async and its own scratch.
void readout_enqueue(ipeps_state* st, hipStream_t s, bool snap) {
    const int q = st->q, chi = st->chi, n = st->n;
    const long n2 = (long)n * n, q4 = (long)q * q * q * q;
    const size_t e = st->esz;
    void* X2p = snap ? st->X2pr : st->X2p;
    void* E = snap ? st->Er : st->E;
    const Ex x = solo(st);
    run_on(x, s, snap ? st->read1r : st->read1);
    run_on(x, s, snap ? st->read2r : st->read2);
    run_on(x, s, snap ? st->read3r : st->read3);
    for (int site = 0; site < 4; ++site) {
        // Lp[q^2][t4p][t2p] <- L'[t4p][q^2][t2p];  Rp[t4p][t2p][q^2] <- R'[t2p][q^2][t4p]
        permute3(s, st->dtype, 0, chi, q * q, chi, off(X2p, site * n2, e), off(E, site * n2, e));
        permute3(s, st->dtype, 2, chi, q * q, chi, off(X2p, (4 + site) * n2, e), off(E, (4 + site) * n2, e));
    }
    run_on(x, s, snap ? st->read4r : st->read4);
    double* E64 = snap ? st->E64_r : st->E64;
    to_fp64(s, st->dtype, snap ? st->Eout_r : st->Eout, E64, 4 * q4);
    readout(s, st->D, st->d, st->cfg.d_A, E64, snap ? st->Asnap : st->A, snap ? st->rho_T_r : st->rho_T,
            snap ? st->rho_r : st->rho, snap ? st->obs_r : st->obs_dev);
}

// h: 16 readout values, 4 truncation errors, Delta (host layout of both paths)
void decode_obs(const double* h, double t, int iters, ipeps_obs* out) {
    for (int i = 0; i < 16; ++i) IPEPS_REQUIRE(std::isfinite(h[i]), IPEPS_ENUMERIC, "NaN in readout");
    out->t = t;
    for (int i = 0; i < 4; ++i) out->n[i] = h[i];
    out->imbalance = h[4];
    out->sum_n = h[5];
    out->max_offdiag = h[6];
    for (int i = 0; i < 4; ++i) out->trunc_err[i] = h[16 + i];
    out->ctm_iters = iters;
    out->ctm_delta = h[20];
    for (int i = 0; i < 4; ++i) {
        out->renyi1[i] = h[8 + i];
        out->renyi_half[i] = h[12 + i];
    }
}

}  // namespace

extern "C" {

int ipeps_observe(ipeps_state* st, ipeps_obs* out) {
    if (!st || !out) return IPEPS_EINVAL;
    return wrap(st, [&] {
        check_poison(st);
        IPEPS_REQUIRE(st->have_env, IPEPS_EINVAL, "no environment: call ctmrg_converge first");
        hipStream_t s = st->stream;
        readout_enqueue(st, s, false);
        HIP_CHECK(hipMemcpyAsync(st->host_buf, st->obs_dev, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(st->host_buf + 16, st->eps_snap, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        wait_spectra(solo(st));
        HIP_CHECK(hipMemcpyAsync(st->host_buf + 20, st->dev_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        decode_obs(st->host_buf, st->ctm_step * st->cfg.dt, st->last_iters, out);
    });
}

int ipeps_observe_async(ipeps_state* st) {
    if (!st) return IPEPS_EINVAL;
    return wrap(st, [&] {
        check_poison(st);
        IPEPS_REQUIRE(st->have_env, IPEPS_EINVAL, "no environment: call ctmrg_converge first");
        IPEPS_REQUIRE(!st->ro_pending, IPEPS_EINVAL, "an asynchronous readout is pending: call ipeps_observe_result");
        hipStream_t s = st->stream, rs = st->ro_stream;
        const int chi = st->chi, q = st->q;
        const long cc = (long)chi * chi, cqc = (long)chi * q * chi;
        const long D4 = (long)st->D * st->D * st->D * st->D;
        // snapshot on the main stream (after the CTMRG that made the environment)
        HIP_CHECK(hipMemcpyAsync(st->Csnap, st->Cenv, 16 * cc * st->esz, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(st->Tsnap, st->Tenv, 16 * cqc * st->esz, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(st->Asnap, st->A, 4 * st->d * D4 * sizeof(cplx), hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(st->eps_r, st->eps_snap, 4 * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipEventRecord(st->ev_ro_snap, s));
        // the readout kernels are enqueued by the next CTMRG once its first
        // enlarged corners are launched (they then fill the idle phases of its
        // first projector SVD), or by ipeps_observe_result
        st->ro_deferred = true;
        st->ro_pending = true;
        st->ro_t = st->ctm_step * st->cfg.dt;
        st->ro_iters = st->last_iters;
    });
}

int ipeps_observe_result(ipeps_state* st, ipeps_obs* out) {
    if (!st || !out) return IPEPS_EINVAL;
    return wrap(st, [&] {
        IPEPS_REQUIRE(st->ro_pending, IPEPS_EINVAL, "no asynchronous readout pending");
        launch_deferred_readout(st, nullptr);
        HIP_CHECK(hipEventSynchronize(st->ev_ro_done));
        st->ro_pending = false;
        decode_obs(st->host_buf + kAsyncHost, st->ro_t, st->ro_iters, out);
    });
}

int ipeps_corner_spectra(ipeps_state* st, double* out) {
    if (!st || !out) return IPEPS_EINVAL;
    return wrap(st, [&] {
        IPEPS_REQUIRE(st->have_env, IPEPS_EINVAL, "no environment");
        if (!st->spectra_valid) corner_spectra_update(solo(st), true);
        wait_spectra(solo(st));
        HIP_CHECK(hipMemcpyAsync(out, st->spectra, 16L * st->chi * sizeof(double), hipMemcpyDeviceToHost, st->stream));
        HIP_CHECK(hipStreamSynchronize(st->stream));
    });
}

int ipeps_bond_spectra(ipeps_state* st, double* out) {
    if (!st || !out) return IPEPS_EINVAL;
    return wrap(st, [&] {
        join_su(st);
        HIP_CHECK(hipMemcpyAsync(out, st->lam, 8L * st->D * sizeof(double), hipMemcpyDeviceToHost, st->stream));
        HIP_CHECK(hipStreamSynchronize(st->stream));
    });
}

int ipeps_profile(ipeps_state* st, int enable) {
    if (!st || enable < 0 || enable > 2) return IPEPS_EINVAL;
    return wrap(st, [&] {
        if (enable && st->prof_ev.empty()) {
            st->prof_ev.resize(2 * 16384);
            for (auto& e : st->prof_ev) HIP_CHECK(hipEventCreate(&e));
        }
        st->prof_on = enable != 0;
        st->prof_mode = enable;
        st->prof_used = 0;
        st->prof_meta.clear();
    });
}

int ipeps_profile_read(ipeps_state* st, double* total_ms, int* launches, double* flops_per_launch) {
    if (!st) return IPEPS_EINVAL;
    return wrap(st, [&] {
        HIP_CHECK(hipStreamSynchronize(st->stream));
        double tot = 0;
        int cnt = 0;
        for (int i = 0; i + 1 < st->prof_used; i += 2) {
            if (st->prof_meta[i / 2].tag != 1) continue;
            float ms = 0;
            HIP_CHECK(hipEventElapsedTime(&ms, st->prof_ev[i], st->prof_ev[i + 1]));
            tot += ms;
            ++cnt;
        }
        if (total_ms) *total_ms = tot;
        if (launches) *launches = cnt;
        if (flops_per_launch) *flops_per_launch = st->prof_flops;
        st->prof_used = 0;
        st->prof_meta.clear();
    });
}

int ipeps_profile_read_gemms(ipeps_state* st, int dtype, double* total_ms, double* flops, double* bytes,
                             int* launches) {
    if (!st) return IPEPS_EINVAL;
    return wrap(st, [&] {
        HIP_CHECK(hipStreamSynchronize(st->stream));
        double tot = 0, fl = 0, by = 0;
        int cnt = 0;
        for (int i = 0; i + 1 < st->prof_used; i += 2) {
            const auto& m = st->prof_meta[i / 2];
            if (m.dtype != dtype) continue;
            float ms = 0;
            HIP_CHECK(hipEventElapsedTime(&ms, st->prof_ev[i], st->prof_ev[i + 1]));
            tot += ms;
            fl += m.flops;
            by += m.bytes;
            ++cnt;
        }
        if (total_ms) *total_ms = tot;
        if (flops) *flops = fl;
        if (bytes) *bytes = by;
        if (launches) *launches = cnt;
    });
}

const char* ipeps_strerror(int code) {
    switch (code) {
        case IPEPS_OK: return "ok";
        case IPEPS_EINVAL: return "invalid argument";
        case IPEPS_ENOMEM: return "out of device memory";
        case IPEPS_EDEVICE: return "HIP device error";
        case IPEPS_ENUMERIC: return "NaN/Inf in the state";
        case IPEPS_ENOTCONV: return "CTMRG did not converge";
        case IPEPS_EAGAIN: return "not finished";
        case IPEPS_ENOTFOUND: return "unknown job";
        case IPEPS_ETOOBIG: return "request exceeds the fixed scratch of a no-allocation entry point";
        default: return "unknown error";
    }
}

}  // extern "C"

// ==================================================================== slabs and batches
namespace {

bool same_layout(const ipeps_config& a, const ipeps_config& b) {
    return a.D == b.D && a.chi == b.chi && a.d_A == b.d_A && a.dtype == b.dtype && a.flags == b.flags;
}

// Bytes one state of this layout draws from its allocator (every request
// rounded to 256 bytes, as DevMem::get does).
size_t layout_bytes(const ipeps_config* cfg) {
    ipeps_state* st = new ipeps_state();
    fill_dims_internal(st, cfg);
    st->mem.dry = true;
    allocate(st);
    const size_t tot = st->mem.total;
    delete st;
    return tot;
}

}  // namespace

struct ipeps_slab {
    std::mutex mu;
    ipeps_config layout;
    char* base = nullptr;
    size_t region = 0;
    int slots = 0;
    struct Cursor {
        ipeps_slab* slab;
        int slot;
        size_t used;
    };
    std::vector<Cursor> cur;
    std::vector<char> busy;
};

namespace {
void* slab_alloc(size_t bytes, void* stream, void* ctx) {
    (void)stream;
    auto* c = (ipeps_slab::Cursor*)ctx;
    ipeps_slab* sl = c->slab;
    if (c->used + bytes > sl->region) return nullptr;
    void* p = sl->base + (size_t)c->slot * sl->region + c->used;
    c->used += bytes;
    return p;
}
void slab_free(void* p, void* stream, void* ctx) {
    (void)stream;
    auto* c = (ipeps_slab::Cursor*)ctx;
    ipeps_slab* sl = c->slab;
    if (p == sl->base + (size_t)c->slot * sl->region) {  // the state's first allocation
        std::lock_guard<std::mutex> lk(sl->mu);
        sl->busy[c->slot] = 0;
        c->used = 0;
    }
}
}  // namespace

struct ipeps_batch {
    Ex x;
    std::vector<hipEvent_t> ev;  // cross-stream ordering with the jobs' own streams
    hipEvent_t ev_obs = nullptr;  // the pending readout's completion
    bool obs_pending = false;
    bool use_graph = false;         // replay warm iterations from a captured graph
    hipGraphExec_t graph = nullptr;  // captured on first use, kept for the batch's life
    hipStream_t cap = nullptr;       // the stream the capture runs on
};

namespace {
// jobs' own streams -> lead's streams (at batch creation), or back (at destruction)
void order_streams(ipeps_batch* b, bool into_lead) {
    ipeps_state* L = b->x.st;
    hipStream_t lead[3] = {L->stream, L->su_stream, L->spec_stream};
    int e = 0;
    for (ipeps_state* j : b->x.jobs) {
        if (j == L) continue;
        hipStream_t own[3] = {j->stream, j->su_stream, j->spec_stream};
        for (int a = 0; a < 3; ++a) {
            hipEvent_t ev = b->ev[e++];
            if (into_lead) {
                HIP_CHECK(hipEventRecord(ev, own[a]));
                for (hipStream_t t : lead) HIP_CHECK(hipStreamWaitEvent(t, ev, 0));
            } else {
                HIP_CHECK(hipEventRecord(ev, lead[a]));
                for (hipStream_t t : own) HIP_CHECK(hipStreamWaitEvent(t, ev, 0));
            }
        }
    }
}
}  // namespace

extern "C" {

int ipeps_slab_create(const ipeps_config* cfg, int slots, ipeps_slab** out) {
    if (!out || slots < 1) return IPEPS_EINVAL;
    *out = nullptr;
    ipeps_slab* sl = nullptr;
    int rc = wrap(nullptr, [&] {
        validate(cfg);
        sl = new ipeps_slab();
        sl->layout = *cfg;
        sl->region = (layout_bytes(cfg) + 4095) & ~(size_t)4095;
        sl->slots = slots;
        if (hipMalloc((void**)&sl->base, sl->region * slots) != hipSuccess) {
            (void)hipGetLastError();
            sl->base = nullptr;
            throw status_error(IPEPS_ENOMEM, "slab allocation failed");
        }
        sl->cur.resize(slots);
        sl->busy.assign(slots, 0);
        for (int i = 0; i < slots; ++i) sl->cur[i] = {sl, i, 0};
    });
    if (rc != IPEPS_OK) {
        delete sl;
        return rc;
    }
    *out = sl;
    return IPEPS_OK;
}

size_t ipeps_slab_region_bytes(const ipeps_config* cfg) {
    try {
        validate(cfg);
        return (layout_bytes(cfg) + 4095) & ~(size_t)4095;
    } catch (...) {
        return 0;
    }
}

int ipeps_slab_init(ipeps_slab* sl, int slot, const ipeps_config* cfg, void* hip_stream, ipeps_state** out) {
    if (!sl || !cfg || !out || slot < 0 || slot >= sl->slots) return IPEPS_EINVAL;
    if (!same_layout(*cfg, sl->layout)) return IPEPS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sl->mu);
        if (sl->busy[slot]) return IPEPS_EINVAL;
        sl->busy[slot] = 1;
        sl->cur[slot].used = 0;
    }
    const int rc = ipeps_init(cfg, hip_stream, slab_alloc, slab_free, &sl->cur[slot], out);
    if (rc != IPEPS_OK) {
        std::lock_guard<std::mutex> lk(sl->mu);
        sl->busy[slot] = 0;
    }
    return rc;
}

void ipeps_slab_destroy(ipeps_slab* sl) {
    if (!sl) return;
    if (sl->base) (void)hipFree(sl->base);
    delete sl;
}

int ipeps_batch_create(ipeps_state* const* states, int n, ipeps_batch** out) {
    if (!states || !out || n < 1) return IPEPS_EINVAL;
    *out = nullptr;
    ipeps_batch* b = nullptr;
    int rc = wrap(nullptr, [&] {
        ipeps_state* L = states[0];
        IPEPS_REQUIRE(L != nullptr, IPEPS_EINVAL, "NULL state");
        for (int j = 0; j < n; ++j) {
            ipeps_state* s = states[j];
            IPEPS_REQUIRE(s != nullptr && !s->poisoned, IPEPS_EINVAL, "NULL or poisoned state");
            IPEPS_REQUIRE(same_layout(s->cfg, L->cfg), IPEPS_EINVAL, "batch: states of different layouts");
            IPEPS_REQUIRE(s->mem.ptrs.size() == L->mem.ptrs.size(), IPEPS_EINVAL, "batch: allocation mismatch");
            const char* b0 = (const char*)s->mem.ptrs[0];
            const char* l0 = (const char*)L->mem.ptrs[0];
            for (size_t i = 0; i < s->mem.ptrs.size(); ++i)
                IPEPS_REQUIRE((const char*)s->mem.ptrs[i] - b0 == (const char*)L->mem.ptrs[i] - l0, IPEPS_EINVAL,
                              "batch: states not allocated in one layout (use one slab)");
            IPEPS_REQUIRE(s->have_env == L->have_env && s->spectra_valid == L->spectra_valid &&
                              !s->ro_pending && !s->spec_deferred == !L->spec_deferred &&
                              std::equal(s->warm_valid, s->warm_valid + 16, L->warm_valid),
                          IPEPS_EINVAL, "batch: states at different phases of their schedule");
            for (int k = 0; k < j; ++k) IPEPS_REQUIRE(states[k] != s, IPEPS_EINVAL, "batch: repeated state");
        }
        b = new ipeps_batch();
        Ex& x = b->x;
        x.st = L;
        for (int j = 0; j < n; ++j) {
            x.jobs.push_back(states[j]);
            x.hdelta.push_back((long)((const char*)states[j]->mem.ptrs[0] - (const char*)L->mem.ptrs[0]));
        }
        if (n > 1) {
            auto shift = [](const void* p, long d) -> void* { return p ? (void*)((const char*)p + d) : nullptr; };
            // merged GEMM table: every group of the lead's plan, once per job
            std::vector<GemmProb> mp;
            for (const GemmGroup& g : L->groups) {
                GemmGroup m = g;
                m.first = (int)mp.size();
                m.count = g.count * n;
                m.flops = g.flops * n;
                for (int j = 0; j < n; ++j)
                    for (int i = g.first; i < g.first + g.count; ++i) {
                        GemmProb p = L->probs[i];
                        p.A = shift(p.A, x.hdelta[j]);
                        p.B = shift(p.B, x.hdelta[j]);
                        p.C = shift(p.C, x.hdelta[j]);
                        p.ws = shift(p.ws, x.hdelta[j]);
                        p.gate = (const int*)shift(p.gate, x.hdelta[j]);
                        mp.push_back(p);
                    }
                m.tiles = gemm_plan_with(mp.data() + m.first, m.count, g.dtype, g.tile);
                x.merged[g.first] = m;
            }
            // merged normalisations: the environment and every column step
            std::vector<NormItem> mn;
            std::vector<std::pair<long, int>> ranges = {{L->norm_env_first, 32}};
            for (const ColumnStep& cs : L->steps) ranges.push_back({cs.norm_first, 6});
            for (auto& r : ranges) {
                x.norm_first[r.first] = (long)mn.size();
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < r.second; ++i) {
                        NormItem it = L->norms[r.first + i];
                        it.ptr = shift(it.ptr, x.hdelta[j]);
                        mn.push_back(it);
                    }
            }
            HIP_CHECK(hipMalloc(&x.d_probs, mp.size() * sizeof(GemmProb)));
            HIP_CHECK(hipMemcpy(x.d_probs, mp.data(), mp.size() * sizeof(GemmProb), hipMemcpyHostToDevice));
            HIP_CHECK(hipMalloc(&x.d_norms, mn.size() * sizeof(NormItem)));
            HIP_CHECK(hipMemcpy(x.d_norms, mn.data(), mn.size() * sizeof(NormItem), hipMemcpyHostToDevice));
            long* dd = nullptr;
            HIP_CHECK(hipMalloc(&dd, n * sizeof(long)));
            HIP_CHECK(hipMemcpy(dd, x.hdelta.data(), n * sizeof(long), hipMemcpyHostToDevice));
            x.jm.delta = dd;
            x.jm.njobs = n;
            HIP_CHECK(hipMalloc(&x.norm_ws, normalize_ws_doubles(32 * n) * sizeof(double)));
        }
        b->ev.resize(3 * (n - 1));
        for (auto& e : b->ev) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        order_streams(b, true);
    });
    if (rc != IPEPS_OK) {
        ipeps_batch_destroy(b);
        return rc;
    }
    *out = b;
    return IPEPS_OK;
}

void ipeps_batch_destroy(ipeps_batch* b) {
    if (!b) return;
    try {
        if (b->x.st && b->ev.size() == 3 * (b->x.jobs.size() - 1)) order_streams(b, false);
    } catch (...) {
    }
    if (b->x.st) {
        (void)hipStreamSynchronize(b->x.st->stream);
        (void)hipStreamSynchronize(b->x.st->su_stream);
        (void)hipStreamSynchronize(b->x.st->spec_stream);
    }
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->x.d_probs) (void)hipFree(b->x.d_probs);
    if (b->x.d_norms) (void)hipFree(b->x.d_norms);
    if (b->x.jm.delta) (void)hipFree((void*)b->x.jm.delta);
    if (b->x.norm_ws) (void)hipFree(b->x.norm_ws);
    for (auto& e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->ev_obs) (void)hipEventDestroy(b->ev_obs);
    delete b;
}

int ipeps_batch_trotter_step(ipeps_batch* b, int n_steps) {
    if (!b || n_steps < 0) return IPEPS_EINVAL;
    return wrap(b->x.st, [&] {
        for (ipeps_state* j : b->x.jobs) check_poison(j);
        trotter_steps(b->x, n_steps);
    });
}

int ipeps_batch_ctmrg(ipeps_batch* b, int iters, int cold_start) {
    if (!b || iters < 1) return IPEPS_EINVAL;
    return wrap(b->x.st, [&] {
        for (ipeps_state* j : b->x.jobs) check_poison(j);
        int it = 0;
        double dl = INFINITY;
        ctmrg_iterations(b->x, 0.0, iters, cold_start != 0, false, &it, &dl,
                         b->use_graph ? &b->graph : nullptr, b->cap);
    });
}

int ipeps_batch_set_graph(ipeps_batch* b, int enable) {
    if (!b) return IPEPS_EINVAL;
    return wrap(b->x.st, [&] {
        if (enable && !b->cap) HIP_CHECK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        b->use_graph = enable != 0;
    });
}

int ipeps_batch_observe_async(ipeps_batch* b) {
    if (!b) return IPEPS_EINVAL;
    ipeps_state* L = b->x.st;
    return wrap(L, [&] {
        IPEPS_REQUIRE(!b->obs_pending, IPEPS_EINVAL, "batch: a readout is pending");
        for (ipeps_state* j : b->x.jobs) {
            check_poison(j);
            IPEPS_REQUIRE(j->have_env, IPEPS_EINVAL, "no environment: run the CTMRG first");
        }
        hipStream_t s = L->stream;
        wait_spectra(b->x);
        for (ipeps_state* j : b->x.jobs) {
            readout_enqueue(j, s, false);
            HIP_CHECK(hipMemcpyAsync(j->host_buf, j->obs_dev, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipMemcpyAsync(j->host_buf + 16, j->eps_snap, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipMemcpyAsync(j->host_buf + 20, j->dev_scalars, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        if (!b->ev_obs) HIP_CHECK(hipEventCreateWithFlags(&b->ev_obs, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(b->ev_obs, s));
        b->obs_pending = true;
    });
}

int ipeps_batch_query(ipeps_batch* b) {
    if (!b) return IPEPS_EINVAL;
    if (!b->obs_pending) return IPEPS_EINVAL;
    const hipError_t e = hipEventQuery(b->ev_obs);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    (void)hipGetLastError();
    return IPEPS_EDEVICE;
}

int ipeps_batch_observe_result(ipeps_batch* b, ipeps_obs* out, int* status) {
    if (!b || !out) return IPEPS_EINVAL;
    ipeps_state* L = b->x.st;
    return wrap(L, [&] {
        IPEPS_REQUIRE(b->obs_pending, IPEPS_EINVAL, "batch: no readout pending");
        HIP_CHECK(hipEventSynchronize(b->ev_obs));
        b->obs_pending = false;
        int bad = IPEPS_OK;
        for (size_t i = 0; i < b->x.jobs.size(); ++i) {
            ipeps_state* j = b->x.jobs[i];
            if (status) status[i] = IPEPS_OK;
            try {
                decode_obs(j->host_buf, j->ctm_step * j->cfg.dt, j->last_iters, &out[i]);
            } catch (const status_error& e) {
                j->poisoned = true;  // the others' results stand
                std::memset(&out[i], 0, sizeof(ipeps_obs));
                if (status) status[i] = e.code;
                bad = e.code;
            }
        }
        if (bad != IPEPS_OK) throw status_error(bad, "NaN in the readout of a job of the batch");
    });
}

int ipeps_batch_observe(ipeps_batch* b, ipeps_obs* out) {
    const int rc = ipeps_batch_observe_async(b);
    if (rc != IPEPS_OK) return rc;
    return ipeps_batch_observe_result(b, out, nullptr);
}

}  // extern "C"
