/*
 * ipeps.h — C ABI of the MI355X iPEPS time-evolution library.
 *
 * The library evolves the disorder-dilated 2D XXZ model of arXiv:1910.11359
 * (Eq. Hanc: physical spin-1/2 ⊗ auxiliary spin per site, local dimension
 * d = 2 d_A) from the Néel ⊗ |+> product state (section "Set up for iPEPS",
 * Initialization) with the simple update and a symmetric second-order Trotter
 * step (Quench), and reads out the site occupations with the auxiliary spin
 * traced out and the sublattice imbalance from a CTMRG environment (Readout;
 * appendix: chi >= D^2, converged).  One state = one 2x2 unit cell
 * (checkerboard A = (0,0),(1,1), B = (1,0),(0,1)); all work runs in HIP
 * kernels on one gfx950 device, ordered on the stream given at init.
 *
 * Conventions shared by every call
 *   sites        order (0,0), (1,0), (0,1), (1,1); y grows downwards
 *   local index  s = p*d_A + a; p = 0 is the occupied spin-up state; the
 *                auxiliary level a carries the field value z(a) W with
 *                z(a) = 1 - 2a/(d_A-1) (equally spaced in [-1, 1])
 *   bonds        order h(0,0) h(1,0) h(0,1) h(1,1) v(0,0) v(1,0) v(0,1) v(1,1);
 *                h(x,y) joins (x,y).right to (x+1,y).left, v(x,y) joins
 *                (x,y).down to (x,y+1).up (coordinates mod 2)
 *   host Gamma   4 sites x [s][up][left][down][right], complex as interleaved
 *                (re, im) doubles: 4 * d * D^4 * 2 doubles
 *   host lambda  8 bonds x D doubles
 *   errors       every int-returning call returns 0 on success or a negative
 *                IPEPS_E* code; ipeps_strerror() names it.  A call that fails
 *                leaves no work queued on the stream, except IPEPS_ENUMERIC
 *                (NaN/Inf found), which poisons the state: every later call on
 *                it returns IPEPS_ENUMERIC.
 *   ownership    the caller owns configs, output buffers and the stream; the
 *                library owns states, servers and all device memory they use.
 *   threads      one ipeps_state must not be used from two threads at once;
 *                the solve_* server calls are thread-safe.
 */
#ifndef IPEPS_H
#define IPEPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPEPS_OK 0
#define IPEPS_EINVAL (-1)    /* bad argument or configuration */
#define IPEPS_ENOMEM (-2)    /* device allocation failed */
#define IPEPS_EDEVICE (-3)   /* HIP runtime error, or no gfx950 device */
#define IPEPS_ENUMERIC (-4)  /* NaN/Inf in the state; the state is poisoned */
#define IPEPS_ENOTCONV (-5)  /* CTMRG reached max_iter above tol (result still written) */
#define IPEPS_EAGAIN (-6)    /* job not finished yet */
#define IPEPS_ENOTFOUND (-7) /* unknown job id */
#define IPEPS_ETOOBIG (-8)   /* request larger than a no-allocation entry point's fixed scratch */

/* arithmetic of the CTMRG contractions; simple-update SVDs, projector
 * SVDs and environment norms are FP64 in every mode.  FP64 and FP32 store
 * the environment tensors in that precision and multiply on FP64 / FP32
 * MFMA.  BF16 stores them in FP32 and rounds every operand of the
 * environment contractions (enlarged corners, cut-matrix products,
 * projectors, renormalisation) to BF16 (nearest even) at the MFMA, with FP32
 * accumulation and FP32 results; the readout contraction stays in FP32.
 * BF16X3 (split BF16) is BF16 with each operand carried as two BF16 terms
 * x = h + l, l = bf16(x - h), and each product as h h' + h l' + l h' (three
 * BF16 MFMAs, about 16 bits of operand precision). */
enum { IPEPS_DTYPE_FP64 = 0, IPEPS_DTYPE_FP32 = 1, IPEPS_DTYPE_BF16 = 2, IPEPS_DTYPE_BF16X3 = 3 };

/* Job parameters (Eq. Hanc with S = sigma/2):
 *   h_bond = J (Sx Sx + Sy Sy) + V Sz Sz + w W (Sz Za (x) 1 + 1 (x) Sz Za)
 * on every nearest-neighbour bond, w = 1/4 (four bonds per site).
 * D: PEPS bond dimension (1..8); chi: environment dimension (D^2..160);
 * d_A: auxiliary levels, 1..5 (d = 2 d_A <= 10; d_A = 1 is the clean model;
 *      the simple update needs d min(D^3, d D) <= 512); dt: Trotter step (> 0);
 * trotter_order: must be 2.  layer_J / layer_V multiply J and V on the bonds
 * of the layers H_A, H_B, V_A, V_B, and layer_w sets their field weight w:
 * hooks for exactly solvable limits (a dimer lattice, decoupled chains);
 * ipeps_config_default() sets 1, 1, 1/4.  flags: IPEPS_FLAG_AUTOTUNE picks
 * every GEMM group's tile kind by timing the candidates once at ipeps_init
 * (cached per process by shape; results may then differ from the default
 * heuristic choice at rounding level).  The projector SVD of a cut matrix
 * N = G F (n x n, n = chi D^2) runs by subspace iteration when n > 96; by
 * default N is formed (two n^3 products) when n <= 1024 and applied through
 * its four enlarged-corner factors above (no n^3 product; more, narrower
 * launches).  IPEPS_FLAG_FACTORED_CUTS / IPEPS_FLAG_FORMED_CUTS force one of
 * the two for every n > 96 (both set: IPEPS_EINVAL).  Default 0. */
#define IPEPS_FLAG_AUTOTUNE 1u
#define IPEPS_FLAG_FACTORED_CUTS 2u
#define IPEPS_FLAG_FORMED_CUTS 4u

typedef struct {
    int D, chi, d_A;
    double J, V, W, dt;
    int trotter_order;
    int dtype;
    double layer_J[4], layer_V[4], layer_w[4];
    uint32_t flags;
    uint64_t seed; /* seeds the random start of the projector subspace iteration */
} ipeps_config;

/* One readout (section Results, interacting case): occupation n of each
 * site with the auxiliary spin traced out, imbalance
 * (n(0,0)+n(1,1)-n(1,0)-n(0,1))/2, the sum of the four n (2 at half
 * filling), the largest |rho_p[up,down]| (0 by particle-number
 * conservation), the accumulated local truncation error of each site (sum
 * over its bond updates of discarded squared weights / total squared
 * weights), the CTMRG iterations / last corner-spectrum change, and the
 * Renyi entropies S_1 = -Tr r ln r and S_1/2 = 2 ln Tr sqrt(r) of each
 * site's physical one-site matrix r (auxiliary spin traced; maximum ln 2),
 * the paper's monitor of how far the state is from saturation (section
 * Results). */
typedef struct {
    double t;
    double n[4];
    double imbalance;
    double sum_n;
    double max_offdiag;
    double trunc_err[4];
    int ctm_iters;
    double ctm_delta;
    double renyi1[4];
    double renyi_half[4];
} ipeps_obs;

typedef struct ipeps_state ipeps_state;

/* Optional device-memory hooks (e.g. a framework's caching allocator).
 * alloc returns device memory of at least `bytes` usable on `stream`, or
 * NULL; free releases it.  Both NULL: the library uses hipMalloc/hipFree. */
typedef void* (*ipeps_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*ipeps_free_fn)(void* ptr, void* stream, void* ctx);

void ipeps_config_default(ipeps_config* cfg);

/* Device memory (bytes) one state of this configuration allocates; used for
 * admission by HBM footprint.  Returns 0 for an invalid configuration. */
size_t ipeps_footprint_bytes(const ipeps_config* cfg);

/* Create a state holding Néel ⊗ |+> (a D = 1 iPEPS embedded in D, every
 * lambda = (1, 0, ...)) and the Trotter gates e^{-i tau h_bond}, tau in
 * {dt/2, dt}, built on the device in FP64 (Initialization; Eq. Hanc).
 * hip_stream: a hipStream_t (NULL = the default stream).  *out receives the
 * handle.  Errors: EINVAL (bad config), ENOMEM, EDEVICE. */
int ipeps_init(const ipeps_config* cfg, void* hip_stream, ipeps_alloc_fn alloc,
               ipeps_free_fn free_fn, void* alloc_ctx, ipeps_state** out);

/* Replace the site tensors and bond weights (host layouts above) and reset
 * the truncation errors and the environment; for tests that start from
 * arbitrary states.  Synchronises the stream. */
int ipeps_set_state(ipeps_state* st, const double* gamma, const double* lambda);

/* Copy the site tensors and bond weights to host buffers (layouts above);
 * either pointer may be NULL.  Synchronises the stream. */
int ipeps_get_state(ipeps_state* st, double* gamma, double* lambda);

/* Advance n_steps symmetric second-order Trotter steps (Quench: simple
 * update) on an internal stream of the state, ordered after the last
 * double-layer build (so it overlaps the rest of a pending CTMRG) and before
 * the next one.  Each step is the layers H_A/2 H_B/2 V_A/2 V_B V_A/2 H_B/2
 * H_A/2, two disjoint bonds per layer.  Each bond update: absorb the outer bond weights,
 * reduce both tensors by QR, apply the gate, SVD in FP64, keep at most D
 * values without splitting multiplets (relative gap <= 1e-10) or keeping
 * values <= 1e-12 s_1, normalise the new weights to unit 2-norm, divide the
 * outer weights back out (pseudo-inverse, cutoff 1e-14 relative), scale the
 * site tensors to max |.| = 1.  trunc_err_out (4 doubles, nullable) receives
 * the accumulated truncation error of each site (waits for the steps;
 * otherwise the call only enqueues work).  Errors: EINVAL, ENUMERIC. */
int ipeps_trotter_step(ipeps_state* st, int n_steps, double* trunc_err_out);

/* CTMRG environment of the current state (Readout; appendix).  Directional
 * CTMRG on the 2x2 cell: one iteration is a left, right, up and down move;
 * each move absorbs column 0 then column 1; the projectors of every cut come
 * from the truncated (FP64) SVD of the product of the four enlarged corners
 * of its 2x2 block (half-system projectors); every new C and T is
 * normalised in FP64.  cold_start != 0 rebuilds the environment from the
 * double-layer tensors (outward legs closed with the identity); 0 continues
 * from the last one (warm).  Stops after the first iteration whose largest
 * change of a normalised corner spectrum is < tol, or after max_iter
 * iterations; tol <= 0 runs exactly max_iter.  *iters and *delta (nullable)
 * receive the count and last change.  Synchronises the stream once per
 * iteration when tol > 0, and once at the end when delta is not NULL;
 * with tol <= 0 and delta NULL the call only enqueues work (the change is
 * reported by the next ipeps_observe).  Errors: EINVAL, ENUMERIC, ENOTCONV (tol > 0 not
 * reached; the environment is still usable). */
int ctmrg_converge(ipeps_state* st, double tol, int max_iter, int cold_start, int* iters,
                   double* delta);

/* Readout from the current environment (Readout; Results): one-site reduced
 * density matrices, auxiliary spin traced out.  out->t is the evolved time
 * (steps * dt).  Synchronises the stream.  Errors: EINVAL (no environment
 * yet), ENUMERIC. */
int ipeps_observe(ipeps_state* st, ipeps_obs* out);

/* The same readout, asynchronous (Readout; Results): copies the current
 * environment, site tensors and truncation errors on the state's stream
 * (about 12 MB at D=6, chi=72 FP32) and reads the copy out on a stream of its
 * own, so the caller can enqueue the next Trotter step and CTMRG before the
 * result is needed.  One readout may be pending per state: a second call
 * before ipeps_observe_result returns EINVAL.  The result equals what
 * ipeps_observe returns for the same environment (same kernels, same
 * inputs).  Errors: EINVAL (no environment yet, or a readout pending). */
int ipeps_observe_async(ipeps_state* st);

/* Waits for the pending asynchronous readout and fills out (fields as for
 * ipeps_observe, of the environment at the time of ipeps_observe_async).
 * Errors: EINVAL (nothing pending), ENUMERIC. */
int ipeps_observe_result(ipeps_state* st, ipeps_obs* out);

/* Singular values of the 16 corners (sites in order, C1..C4 each),
 * normalised to unit 2-norm, zero-padded: out holds 16 * chi doubles.
 * Synchronises the stream. */
int ipeps_corner_spectra(ipeps_state* st, double* out);

/* The 8 bond weight vectors (bond order above): out holds 8 * D doubles. */
int ipeps_bond_spectra(ipeps_state* st, double* out);

/* Release the state and its device memory (synchronises its stream). */
void ipeps_destroy(ipeps_state* st);

/* ------------------------------------------------------------------ serving
 * A request loop that owns an HBM budget and up to max_slots concurrently
 * resident jobs.  Each submitted job runs Néel ⊗ |+> for n_steps Trotter
 * steps, and after every observe_every steps (and after the last one) runs
 * ctm_iters CTMRG iterations (cold at the first observation, warm later) and
 * one readout.  A job is admitted when a slot is free and its footprint fits
 * the remaining budget; admitted jobs keep their tensors on the device and
 * run concurrently on their own streams; finished jobs release their slot
 * and memory at once so queued jobs can start. */
typedef struct {
    ipeps_config cfg;
    int n_steps;
    int observe_every;
    int ctm_iters;
    uint64_t tag;
} ipeps_job;

enum { IPEPS_JOB_QUEUED = 0, IPEPS_JOB_RUNNING = 1, IPEPS_JOB_DONE = 2 };

typedef struct ipeps_server ipeps_server;

/* hbm_budget: bytes of device memory the admitted jobs may hold together
 * (0 = 90% of the free memory at creation); max_slots >= 1.  Errors: EINVAL,
 * EDEVICE. */
int solve_server_create(size_t hbm_budget, int max_slots, ipeps_server** out);

/* Enqueue a job (non-blocking, thread-safe); *job_id receives its id.
 * Errors: EINVAL (bad job, or a footprint above the whole budget). */
int solve_submit(ipeps_server* srv, const ipeps_job* job, uint64_t* job_id);

/* Non-blocking status: *status = IPEPS_JOB_QUEUED / RUNNING / DONE, or a
 * negative error code of the failed job.  When done, copies up to cap
 * observations into series and sets *n_out to the number available; the
 * job's record is kept until the server is destroyed.  Returns 0 when done,
 * IPEPS_EAGAIN while queued or running, ENOTFOUND for an unknown id, or the
 * job's error code. */
int solve_poll(ipeps_server* srv, uint64_t job_id, int* status, ipeps_obs* series, int cap,
               int* n_out);

/* Wall-clock seconds (host monotonic clock) at which the job was submitted,
 * admitted and finished; for latency statistics.  Returns ENOTFOUND/EAGAIN
 * like solve_poll. */
int solve_job_times(ipeps_server* srv, uint64_t job_id, double* t_submit, double* t_admit,
                    double* t_done);

/* enable != 0: the batches the loop launches replay their warm CTMRG
 * iterations from captured graphs (ipeps_batch_set_graph); a group whose
 * jobs all go on keeps its batch, and its graph, for its next chunk.
 * Applies to batches created afterwards.  Errors: EINVAL (NULL). */
int solve_server_set_graphs(ipeps_server* srv, int enable);

/* Wait for all jobs, stop the loop and release everything. */
void solve_server_destroy(ipeps_server* srv);

/* ------------------------------------------------------------ batches
 * Many jobs of one layout advanced in lockstep, every launch carrying all of
 * them (the simple-update layers, the enlarged-corner, cut-matrix, projector
 * and renormalisation GEMMs, the Cholesky, Jacobi and projector kernels of
 * the projector SVDs, the spectra): the parameter points of a sweep, or the
 * resident requests of one shape in the request loop.  Each job keeps its own
 * state and its results are those it gets alone (every GEMM problem keeps the
 * tile kind and summation order of the job's own plan; FP64 results are
 * bitwise the same).
 *
 * Layout: D, chi, d_A, dtype and flags; jobs of one layout may differ in J, V,
 * W, dt, the layer hooks and the seed.  A slab is one device allocation with
 * `slots` regions of ipeps_slab_region_bytes(cfg) each; ipeps_slab_init
 * creates a state (as ipeps_init, Néel ⊗ |+>) inside region `slot`, and
 * ipeps_destroy of that state frees the region again.  Batches need their
 * states to come from one slab (their buffers then sit at one fixed offset
 * from each other). */
typedef struct ipeps_slab ipeps_slab;
typedef struct ipeps_batch ipeps_batch;

/* Bytes of one slab region for this layout; 0 for an invalid config. */
size_t ipeps_slab_region_bytes(const ipeps_config* cfg);
/* Errors: EINVAL (bad config, slots < 1), ENOMEM. */
int ipeps_slab_create(const ipeps_config* layout, int slots, ipeps_slab** out);
/* cfg must have the slab's layout; the slot must be free.  The state's own
 * stream is hip_stream.  Errors: EINVAL, ENOMEM, EDEVICE. */
int ipeps_slab_init(ipeps_slab* slab, int slot, const ipeps_config* cfg, void* hip_stream,
                    ipeps_state** out);
/* Releases the slab; its states must have been destroyed (ipeps_destroy
 * waits for each state's work) and no batch of them may exist. */
void ipeps_slab_destroy(ipeps_slab* slab);

/* A lockstep batch of n >= 1 states of one slab, at the same phase of their
 * schedules (all with or all without an environment, the same warm projector
 * subspaces, no pending asynchronous readout); states[0] leads: its streams
 * carry all the work, ordered after everything already enqueued on any
 * job's streams.  While the batch exists its states must not be used
 * otherwise.  Errors: EINVAL (NULL, repeated or poisoned states, different
 * layouts, not one slab, different phases), EDEVICE. */
int ipeps_batch_create(ipeps_state* const* states, int n, ipeps_batch** out);
/* ipeps_trotter_step for every job (no truncation errors returned). */
int ipeps_batch_trotter_step(ipeps_batch* b, int n_steps);
/* ctmrg_converge with tol <= 0 for every job: exactly iters iterations,
 * cold (cold_start != 0) or warm. */
int ipeps_batch_ctmrg(ipeps_batch* b, int iters, int cold_start);
/* enable != 0: from the second iteration of each ipeps_batch_ctmrg call on,
 * replay one warm iteration (the eight column steps of section Readout, the
 * corner snapshot and the previous iteration's spectra) from a HIP graph
 * captured from the lead's main stream on first use and kept until
 * ipeps_batch_destroy; results equal the eager launches bit for bit (the
 * random restarts of dropped subspace columns draw from counters kept on
 * the device).  Capture and instantiation happen on the calling thread and
 * cost about one iteration's launch time; the replays save the per-launch
 * host work, which dominates at small D and chi.  The capture runs on a
 * stream of the batch's own (the lead's stream may be the null stream), the
 * replays on the lead's stream.  Default: off.  Errors: EINVAL (NULL),
 * EDEVICE. */
int ipeps_batch_set_graph(ipeps_batch* b, int enable);
/* ipeps_observe for every job: out[i] for states[i].  Synchronises.
 * Errors: EINVAL, ENUMERIC (a job's readout is not finite: that job is
 * poisoned and its out[i] zeroed, the other jobs' results are valid). */
int ipeps_batch_observe(ipeps_batch* b, ipeps_obs* out);
/* The same in two halves: _async enqueues the readouts (one may be pending
 * per batch), _query returns 1 once they are complete (0 before; no
 * synchronisation), _result waits for them and fills out as above, and
 * status[i] (nullable) with job i's own code. */
int ipeps_batch_observe_async(ipeps_batch* b);
int ipeps_batch_query(ipeps_batch* b);
int ipeps_batch_observe_result(ipeps_batch* b, ipeps_obs* out, int* status);
/* Orders every job's streams after the batch's work, waits for it and
 * releases the batch (not the states). */
void ipeps_batch_destroy(ipeps_batch* b);

/* ------------------------------------------------------------ instrumentation
 * HIP-event timing of the GEMM launches on the state's stream.
 * ipeps_profile(st, 1) starts (and clears) recording of the launches of the
 * largest enlarged-corner GEMM launch of an iteration (the 8 corner products
 * of the left move's first column step, a kernel symbol of its own);
 * ipeps_profile(st, 2) records every GEMM launch on the state's stream (the
 * environment contractions, and the FP64 products of the projector SVDs);
 * ipeps_profile(st, 0) stops.  At most 16384 launches are recorded.
 * ipeps_profile_read synchronises the stream and returns the summed time in
 * ms of the recorded enlarged-corner launches, their number and the
 * algorithmic flops of one of them (2 M N K summed over its products), then
 * clears the record.  ipeps_profile_read_gemms synchronises and returns, for
 * the recorded launches whose arithmetic is `dtype` (IPEPS_DTYPE_*), their
 * summed time, summed algorithmic flops, summed algorithmic bytes (each
 * operand read once and each result written once, in the storage
 * precision) and number, without clearing.
 * Errors: EINVAL. */
int ipeps_profile(ipeps_state* st, int enable);
int ipeps_profile_read(ipeps_state* st, double* total_ms, int* launches,
                       double* flops_per_launch);
int ipeps_profile_read_gemms(ipeps_state* st, int dtype, double* total_ms, double* flops,
                             double* bytes, int* launches);

const char* ipeps_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* IPEPS_H */
