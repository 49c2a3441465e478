"""Throughput of the iPEPS hot path on one MI355X.

One step = one second-order Trotter step (14 simple-update bond updates) +
one CTMRG iteration (left, right, up and down moves: 64 enlarged corners, 52
of them computed, 16 half-system projector pairs, 16 T and 32 C
renormalisations, 16 corner spectra) continuing from the previous
environment + one readout of the four site occupations and the imbalance
(the readout of step t runs on its own stream while step t + 1 is enqueued;
every timed step's readout completes inside the timed region).
Workload: D=6, chi=72, d=4 (binary
disorder), J=1, V=1, W=8, dt=0.05, synthetic Néel ⊗ |+> start; the state is
first evolved (untimed) to t = 1 so that every bond carries D singular values.

Default precision: CTMRG contractions in FP32 on MFMA, the simple update,
projector SVDs and normalisations in FP64 (--dtype fp64 runs everything in
FP64; with FP32 the FP64 path is also timed and reported as fp64_path).

Prints one JSON line.  The roofline entry is for the dominant kernel family,
the environment-contraction GEMMs (k_gemm_direct / k_gemm_panel /
k_gemm_grouped in the contraction precision: enlarged corners, cut-matrix chains, projectors, C
and T renormalisation), every launch of the timed steps on the library's
stream: their algorithmic flops / their summed HIP-event time.  corner_launch
is the single largest launch (8 enlarged corners).  step_mfma_frac is the
time the step's algorithmic flops need at the MFMA peak of the contraction
precision over the measured step time; fp64_gemms covers the FP64 products
of the projector SVDs.  With a precision other than FP64 the same schedule
also runs in FP64 and in the other contraction precisions (fp32, bf16x3 =
split BF16, bf16); precision_vs_fp64 compares their imbalance with FP64 at
t = 1 after 10 cold CTMRG iterations.

sweep: batched jobs/s of the 64-job parameter sweep through the request loop
(jobs of one D advance as one lockstep batch) in the contraction precision,
split BF16 and FP64, with the largest imbalance difference from FP64 over
all observations.  serving: the first requests of the serving stream at
their own shapes (D up to 8, chi up to 128), Poisson arrivals at 0.8 x the
sweep's capacity, p50/p99 latency and jobs/s in the contraction precision
and in FP64.
cpu_baseline is the oracle (complex128 NumPy) timed on a bounded sample of
the same step and scaled to steps/s.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
# The largest single GEMM launch, reported beside the roofline: the 8
# enlarged-corner products of the left move's first column step (chi^2 x q^2
# by q^2 x q^2 each), a kernel symbol of its own (TAG=1).
ROOF_KERNEL = "k_gemm_direct<...,TAG=1> (8 enlarged-corner products)"
# HBM bytes per launch of the roofline kernel family (every environment-
# contraction GEMM launch of a step: FETCH_SIZE + WRITE_SIZE summed over its
# dispatches, scaled by a 256 MiB copy, divided by the launches), from the
# traffic profile in profiles/; valid only for the tile planning, kernels
# and launches they were measured on (the part of gemm.hip from tile_dims
# on, see gemm_kernel_digest).  Keyed by contraction precision.
TRAFFIC = {"fp32": {"kernel": "gemm_family", "gemm_kernel_sha256_16": "fb039deec08e37cb",
                    "bytes_per_launch": 1.1457e8,
                    "note": "FETCH_SIZE + WRITE_SIZE per GEMM launch (with its split-K sum), steady "
                            "steps, profiles/traffic_contraction_gemms_D6_chi72_fp32.md"}}


def gemm_kernel_digest():
    """sha256 (16 hex digits) of gemm.hip from its tile planning to the end:
    the tile choice, the kernels and their launch shapes."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1910_11359_amd", "csrc", "gemm.hip"), "rb") as f:
        src = f.read()
    return hashlib.sha256(src[src.index(b"static void tile_dims("):]).hexdigest()[:16]
DTYPE_NAME = {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3"}
METRIC = "Trotter+CTMRG steps/s at D=6,χ=72 (MFMA % peak); batched jobs/s, p50/p99 latency"


def step_flops(D, chi, dtype):
    """Algorithmic real flops of one CTMRG iteration in the real basis, all in
    the contraction precision.  52 enlarged corners per iteration (64 used;
    the first column step of the right, up and down moves reuses 4 that the
    previous move computed and left valid; later iterations of one CTMRG
    call compute 48, the left move reusing 4 of the down move's, but the
    headline step runs one iteration per call).  16 cuts per iteration (4 moves x
    2 columns x 2 cuts); the cut matrix N = E2 E3 E0 E1 is applied to blocks of k = chi + p
    columns through its four n x n factors (n = chi D^2), 2 w + 1 times (w
    warm subspace iterations: 1 with FP32 contractions, 2 with FP64; p = 8
    resp. max(16, chi/3)).  The FP64 orthogonalisations (O(n k^2)) are not
    counted."""
    q = D * D
    n = chi * q
    if dtype == "fp64":
        k, w = chi + max(16, chi // 3), 2
    else:
        k, w = chi + (8 if chi >= 64 else 16), 1
    k = min(k, n)
    return 2.0 * (52 * (chi ** 3 * q + chi ** 3 * q ** 2 + chi ** 2 * q ** 4)
                  + 16 * ((2 * w + 1) * 4 * n ** 2 * k + 4 * n ** 2 * chi)
                  + 16 * (chi ** 2 * q ** 4 + 2 * chi ** 3 * q ** 2)
                  + 32 * 2 * chi ** 3 * q)


def step_mfma_frac(D, chi, dtype, ms_per_step):
    """Time the step's algorithmic flops need at the MFMA peak of the
    contraction precision, as a fraction of the measured step time."""
    return step_flops(D, chi, dtype) / (PEAK_TFLOPS[dtype] * 1e12) / (ms_per_step * 1e-3)


def cpu_baseline(D, chi, W, V):
    """Oracle on a bounded sample: 1 bond update, 1 enlarged corner, 1 cut
    (3 n^3 products + full SVD), scaled to one step (14 bond updates, 64
    enlarged corners + 16 T renormalisations of the same cost, 16 cuts)."""
    import numpy as np

    import synthetic
    from oracle import ctmrg as ct
    from oracle import peps
    from oracle.model import Params

    par = Params(D=D, chi=chi, J=1.0, V=V, W=W, dt=0.05)
    gam, lam = synthetic.random_state(7, D)
    st = peps.new_state(par)
    for i, s in enumerate(peps.SITES):
        st["gam"][s], st["lam_h"][s], st["lam_v"][s] = gam[i], lam[i], lam[4 + i]
    G = par.layer_gate(0, 0.5 * par.dt)
    t0 = time.perf_counter()
    peps.update_horizontal(st, (0, 0), G, D)
    t_bond = time.perf_counter() - t0
    a = ct.double_layers(st)
    rng = np.random.default_rng(0)
    q = D * D
    C = rng.normal(size=(chi, chi)).astype(complex)
    T = rng.normal(size=(chi, q, chi)).astype(complex)
    t0 = time.perf_counter()
    E = ct.enlarged_corner(C, T, T, a[(0, 0)])
    t_corner = time.perf_counter() - t0
    t0 = time.perf_counter()
    ct.projectors(E, E, E, E, chi)
    t_cut = time.perf_counter() - t0
    t_step = 14 * t_bond + 80 * t_corner + 16 * t_cut
    cores = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(i.get("num_threads", 0)) for i in threadpool_info()) or cores
    except Exception:
        pass
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": (f"D={D} chi={chi}: 1 bond update {t_bond:.2f}s, 1 enlarged corner "
                       f"{t_corner:.2f}s, 1 cut (3 n^3 products + full SVD) {t_cut:.2f}s; "
                       f"step = 14 bonds + 80 corner-size contractions + 16 cuts "
                       f"= {t_step:.1f}s")}


FF_FLOP_PER_SITE = 28  # per application of (h - b)/a to a complex orbital: 5-point stencil
                       # (2 x 5 MACs) + Chebyshev recurrence (4) + series accumulation (4)


def spectrum_ipr_record(P, torch, synthetic, tau, with_cpu, n_real=100, h=100.0, reps=3):
    """Single-particle spectra and IPRs (the spectrum figure's h = 100, 100
    realizations) at L = 10, 16 (one-sided Jacobi, one workgroup per
    realization) and L = 20, 40 (block Jacobi), inputs resident on the device;
    the oracle (numpy eigh per realization) timed on the host for the same
    batch (L = 40: on 3 of the realizations, scaled)."""
    import numpy as np
    rec = {}
    for L in (10, 16, 20, 40):
        reps_l = reps if L <= 16 else 1
        n = L * L
        eps_h = synthetic.ff_fields(L, n_real, h, "continuous", 20191025)
        eps = torch.from_numpy(eps_h).cuda()
        E = torch.empty(n_real * n, dtype=torch.float64, device="cuda")
        I = torch.empty_like(E)
        B = torch.empty(n_real * 20, dtype=torch.float64, device="cuda")
        K = torch.empty(n_real * 20, dtype=torch.int32, device="cuda")
        stream = torch.cuda.Stream()
        run = lambda: P.ff_spectrum_ipr_device(L, eps.data_ptr(), n_real, E.data_ptr(), I.data_ptr(),
                                               B.data_ptr(), K.data_ptr(), tau, False, stream)
        run()
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps_l):
            run()
        e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / reps_l
        how = ("one-sided Jacobi SVD of h + 2G I per realization" if L <= 16 else
               "block Jacobi, 32-index blocks, 64 x 64 MFMA rotations")
        r = {"workload": f"spectrum + IPR + cumulative IPR: L={L}, open, continuous h={h:g}, tau={tau}, "
                         f"{n_real} realizations ({how})",
             "value": n_real / (ms * 1e-3), "unit": "realizations/s", "ms_per_batch": ms,
             "mean_ipr": float(I.mean().item())}
        if with_cpu:
            from oracle import freefermion as off
            ns = n_real if L <= 20 else 3
            t0 = time.perf_counter()
            for k in range(ns):
                off.spectrum_ipr(L, False, tau, eps_h[k])
            r["cpu_baseline"] = {"value": ns / (time.perf_counter() - t0), "unit": "realizations/s",
                                 "kind": "oracle",
                                 "sample": f"the same {n_real} realizations" if ns == n_real else
                                           f"{ns} of the {n_real} realizations"}
        rec[f"L{L}"] = r
    return rec


def free_fermion(P, torch, synthetic, reps=3, with_cpu=True):
    """The free-fermion Néel workload (L = 40, 100 realizations, t = 5 in 50
    intervals), inputs resident on the device; roofline against the FP64
    vector peak (the kernel is FP64 VALU + LDS, no MFMA)."""
    import numpy as np
    cfg = synthetic.ff_headline()
    L, nr, nt, dt, tau = cfg["L"], cfg["n_real"], cfg["n_times"], cfg["dt"], cfg["tau"]
    eps_h = synthetic.ff_fields(L, nr, cfg["h"], cfg["kind"], 20191025)
    eps = torch.from_numpy(eps_h).cuda()
    ne = torch.empty(nr * nt, dtype=torch.float64, device="cuda")
    no = torch.empty_like(ne)
    stream = torch.cuda.Stream()
    run = lambda: P.ff_neel_dynamics_device(L, eps.data_ptr(), nr, ne.data_ptr(), no.data_ptr(), nt, dt, tau,
                                            cfg["pbc"], stream)
    run()
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    stream.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # algorithmic work: per realization, pieces x (K - 1) stencil applications
    # on each of the ceil(L^2/2) orbitals, K from the library's own coefficient routine
    M = (L * L + 1) // 2
    apps = 0
    for r in range(nr):
        a = 0.5 * (eps_h[r].max() - eps_h[r].min()) + 4 * abs(tau)
        nsub = max(1, int(np.ceil(a * dt / 60.0)))
        J = P.ff_bessel_j(a * dt / nsub, 159)
        K = 160
        while K > 1 and abs(J[K - 1]) < 1e-18:
            K -= 1
        apps += nsub * (K - 1)
    flops = float(apps) * nt * M * L * L * FF_FLOP_PER_SITE
    ach = flops / (ms * 1e-3) / 1e12
    imb = (ne - no).view(nr, nt).mean(dim=0).cpu().numpy()
    out = {"workload": f"free-fermion Néel dynamics: L={L}, open, continuous fields h={cfg['h']}, tau={tau}, "
                       f"{nr} realizations, {nt} intervals of {dt} (t = {nt * dt:g})",
           "value": nr / (ms * 1e-3), "unit": "realizations/s", "ms_per_run": ms,
           "imbalance_t_end_mean": float(imb[-1]),
           "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                        "frac": ach / PEAK_TFLOPS["fp64"], "traffic": None, "kernel": "k_ff_neel<7>",
                        "flops_per_launch": flops}}
    out["spectrum_ipr"] = spectrum_ipr_record(P, torch, synthetic, tau, with_cpu)
    if with_cpu:
        from oracle import freefermion as off
        t0 = time.perf_counter()
        off.neel_dynamics(L, cfg["pbc"], tau, eps_h[0], dt * np.arange(1, 6))
        t5 = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / (t5 * nt / 5), "unit": "realizations/s", "kind": "oracle",
                               "cores": os.cpu_count(),
                               "sample": f"1 realization, 5 of {nt} observation times ({t5:.2f} s incl. the "
                                         f"dense eigh), scaled x{nt // 5}"}
    return out


def serving_sample(P, synthetic, dtype, rate, n_req=12, steps_max=10, slots=64):
    """Request loop on a bounded sample of the serving stream: the first n_req
    requests of default_rng(20191025) at their own shapes (D in 3..8, chi =
    min(128, c D^2), W, V), Trotter steps capped at steps_max, observed every
    10 steps with 10 CTMRG iterations, submitted at their Poisson arrival
    times (rate per second); latency = completion - arrival."""
    reqs = synthetic.serving_stream(n=n_req, rate=rate)
    srv = P.Server(hbm_budget=0, max_slots=slots)
    t0 = time.perf_counter()
    ids = []
    for k, r in enumerate(reqs):
        cfg = P.make_config(r["D"], r["chi"], J=r["J"], V=r["V"], W=r["W"], dt=r["dt"], dtype=dtype)
        while time.perf_counter() - t0 < r["arrival"]:
            time.sleep(0.001)
        if (k + 1) % 32 == 0:
            print(f"serving {dtype}: {k + 1}/{len(reqs)} requests submitted ({time.perf_counter() - t0:.0f} s)",
                  file=sys.stderr, flush=True)
        ids.append(srv.submit(cfg, n_steps=min(r["n_steps"], steps_max), observe_every=r["observe_every"],
                              ctm_iters=r["ctm_iters"]))
    lat, t_last, series = [], 0.0, []
    for k, jid in enumerate(ids):
        while True:
            res = srv.poll(jid)[1]
            if res is not None:
                break
            time.sleep(0.002)
        series.append([o["imbalance"] for o in res])
        if (k + 1) % 16 == 0:
            print(f"serving {dtype}: {k + 1}/{len(ids)} requests done ({time.perf_counter() - t0:.0f} s)",
                  file=sys.stderr, flush=True)
        rc, (ts, ta, td) = srv.times(jid)
        lat.append(td - ts)
        t_last = max(t_last, td)
    t_first = min(srv.times(j)[1][0] for j in ids)
    srv.close()
    lat = sorted(lat)
    pct = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]
    shapes = sorted({(r["D"], r["chi"]) for r in reqs})
    return {"jobs_per_s": len(ids) / (t_last - t_first), "p50_s": pct(0.5), "p99_s": pct(0.99),
            "requests": len(ids), "rate_per_s": rate, "dtype": dtype,
            "sample": f"first {n_req} requests of the serving stream at their shapes (D, chi) = {shapes}, "
                      f"Trotter steps capped at {steps_max}, observe every 10 with 10 CTMRG iterations"}, series


def sweep(P, synthetic, dtype, slots=64):
    """The batched parameter sweep: 64 jobs (D in 3..6 with chi = 2 D^2, V in
    {0, 1}, 8 seeded W in [1, 20]), 50 Trotter steps each, 10 CTMRG
    iterations every 10 steps, all submitted at once to the request loop
    (jobs of one D run as one lockstep batch).  Returns jobs/s, the duration
    and the imbalance series."""
    jobs = synthetic.sweep_jobs()
    srv = P.Server(hbm_budget=0, max_slots=slots)
    t0 = time.perf_counter()
    ids = [srv.submit(P.make_config(j["D"], j["chi"], J=j["J"], V=j["V"], W=j["W"], dt=j["dt"],
                                    dtype=dtype),
                      n_steps=j["n_steps"], observe_every=j["observe_every"],
                      ctm_iters=j["ctm_iters"]) for j in jobs]
    series = []
    for jid in ids:
        while True:
            res = srv.poll(jid)[1]
            if res is not None:
                break
            time.sleep(0.005)
        series.append([o["imbalance"] for o in res])
    dt = time.perf_counter() - t0
    print(f"sweep {dtype}: {len(ids)} jobs in {dt:.1f} s", file=sys.stderr, flush=True)
    srv.close()
    return {"jobs": len(ids), "seconds": dt, "jobs_per_s": len(ids) / dt, "dtype": dtype,
            "workload": "64 jobs: D in {3,4,5,6}, chi = 2D^2, V in {0,1}, W = 8 seeded values "
                        "in [1,20]; 50 steps, 10 CTMRG iterations every 10 steps"}, series


def max_err(a, b):
    return max(abs(x - y) for sa, sb in zip(a, b) for x, y in zip(sa, sb))


def headline(P, torch, wl, dtype, steps, warmup, prelude, flags=0, prof_steps=3):
    """Time `steps` steps (after `warmup`) of the headline workload; the state
    is first evolved for `prelude` Trotter steps and 10 cold CTMRG iterations.
    The 8-corner launch is timed with HIP events during the timed steps;
    every GEMM launch on the library's stream is timed during prof_steps
    further steps of the same schedule.  Returns the step rate and the
    launch statistics."""
    stream = torch.cuda.Stream()
    cfg = P.make_config(wl["D"], wl["chi"], J=wl["J"], V=wl["V"], W=wl["W"], dt=wl["dt"], dtype=dtype,
                        flags=flags)
    st = P.State(cfg, stream=stream)
    st.trotter_step(prelude)
    st.ctmrg(0.0, 10, True)

    pending = [False]

    def one_step():
        # CTMRG of the current state and the next Trotter step are enqueued
        # back to back: the simple update (its own stream) overlaps the CTMRG.
        # The readout of this environment runs on its own stream
        # (observe_async) while the next step is enqueued; its result is
        # collected one step later.
        st.ctmrg(0.0, 1, False, want_delta=False)
        st.trotter_step(1)
        if pending[0]:
            st.observe_result()
        st.observe_async()
        pending[0] = True

    def drain():
        if pending[0]:
            st.observe_result()
            pending[0] = False

    for _ in range(warmup):
        one_step()
    drain()
    stream.synchronize()
    torch.cuda.synchronize()
    st.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    drain()  # the last step's readout, inside the timed region
    stream.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_tot, launches, fl = st.profile_read()
    # every GEMM launch timed on its own (two events each add ~3 ms per step,
    # so this runs on prof_steps further steps of the same schedule, after
    # the timed ones)
    st.profile(True, every_gemm=True)
    for _ in range(prof_steps):
        one_step()
    drain()
    gemm = {k: st.profile_read_gemms(k) for k in ("fp64", dtype)}
    st.profile(False)
    st.close()
    launch_ms = ms_tot / max(1, launches)
    return {"value": steps / dt, "ms_per_step": 1e3 * dt / steps,
            "corner_achieved": fl / (launch_ms * 1e-3) / 1e12 if launches else 0.0,
            "corner_launch_ms": launch_ms, "corner_flops": fl, "gemm": gemm, "prof_steps": prof_steps}


def precision_point(P, wl, dtype, n_steps=20, iters=10):
    """Imbalance after n_steps Trotter steps from Néel and `iters` cold CTMRG
    iterations (the precision test's t = 1 observation)."""
    st = P.State(P.make_config(wl["D"], wl["chi"], J=wl["J"], V=wl["V"], W=wl["W"], dt=wl["dt"],
                               dtype=dtype))
    st.trotter_step(n_steps)
    st.ctmrg(0.0, iters, True)
    o = st.observe()
    st.close()
    return o["imbalance"], o["n"]


def gemm_roofline(rec, dtype):
    """Every environment-contraction GEMM launch of the timed steps (the
    enlarged corners, the cut-matrix chains, the projectors and the C / T
    renormalisation; main stream), as one kernel family: algorithmic flops
    per launch over the mean HIP-event launch time."""
    ms, fl, by, n = rec["gemm"][dtype]
    ach = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
            "frac": ach / PEAK_TFLOPS[dtype], "traffic": None,
            "kernel": f"k_gemm_direct / k_gemm_panel / k_gemm_grouped in {dtype}: every environment-contraction GEMM "
                      f"launch of the timed steps (main stream)",
            "launches_per_step": n / rec["prof_steps"], "launch_ms": ms / max(1, n),
            "flops_per_launch": fl / max(1, n), "algorithmic_bytes_per_launch": by / max(1, n),
            "ms_per_step": ms / rec["prof_steps"],
            "timing": f"HIP events around every such launch during {rec['prof_steps']} profiled steps "
                      f"after the timed ones"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="fp32", choices=["fp64", "fp32", "bf16", "bf16x3"],
                    help="CTMRG contraction precision (SVDs, simple update and norms stay FP64)")
    ap.add_argument("--no-fp64-ref", action="store_true",
                    help="skip the FP64 comparison run (headline and serving)")
    ap.add_argument("--no-other-dtypes", action="store_true",
                    help="skip the headline runs in the other contraction precisions")
    ap.add_argument("--autotune", action="store_true",
                    help="time every GEMM group's candidate tile kinds at init and keep the fastest")
    ap.add_argument("--prelude", type=int, default=20, help="untimed Trotter steps first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=12,
                    help="requests of the serving stream in the serving sample (the stream has 256)")
    ap.add_argument("--serving-rate", type=float, default=0.0,
                    help="arrivals per second for the serving sample, in --dtype only (default: 0.8 x the "
                         "sweep's jobs/s, in --dtype and FP64)")
    ap.add_argument("--no-free-fermion", action="store_true",
                    help="skip the free-fermion Néel workload (L=40, 100 realizations)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the 64-job batched sweep through the request loop")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also copy MIB MiB device to device once (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs one GPU only (the path has no multi-GPU mode); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1910_11359_amd as P
    import synthetic

    wl = synthetic.headline_config()
    D, chi = wl["D"], wl["chi"]
    torch.cuda.init()
    flags = P.FLAG_AUTOTUNE if args.autotune else 0
    rec = headline(P, torch, wl, args.dtype, args.steps, args.warmup, args.prelude, flags)
    peak = PEAK_TFLOPS[args.dtype]
    roof = gemm_roofline(rec, args.dtype)
    tr = TRAFFIC.get(args.dtype)
    if (tr and tr["bytes_per_launch"] and tr["kernel"] == "gemm_family"
            and gemm_kernel_digest() == tr["gemm_kernel_sha256_16"]):
        roof["traffic"] = tr["bytes_per_launch"]
        roof["traffic_note"] = tr["note"]
    ms64, fl64, _, n64 = rec["gemm"]["fp64"]
    out = {
        "metric": METRIC, "value": rec["value"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_NAME[args.dtype],
        "data": "synthetic",
        "config": {"workload": f"headline iPEPS step: D={D}, chi={chi}, d=4, J=1, V={wl['V']}, "
                               f"W={wl['W']}, dt={wl['dt']}, after {args.prelude} prelude steps",
                   "D": D, "chi": chi, "d": 4, "contractions": args.dtype, "svd_su_norms": "fp64",
                   "gemm_tiles": "autotuned" if args.autotune else "heuristic"},
        "roofline": roof,
        "step_mfma_frac": step_mfma_frac(D, chi, args.dtype, rec["ms_per_step"]),
        "corner_launch": {"kernel": ROOF_KERNEL, "achieved": rec["corner_achieved"],
                          "frac": rec["corner_achieved"] / peak, "launch_ms": rec["corner_launch_ms"],
                          "flops_per_launch": rec["corner_flops"]},
        "fp64_gemms": {"achieved": fl64 / (ms64 * 1e-3) / 1e12 if ms64 > 0 else 0.0,
                       "frac": (fl64 / (ms64 * 1e-3) / 1e12 if ms64 > 0 else 0.0) / PEAK_TFLOPS["fp64"],
                       "ms_per_step": ms64 / rec["prof_steps"], "launches_per_step": n64 / rec["prof_steps"],
                       "what": "FP64 products of the projector SVDs (Grams, orthogonalisation)"},
    }
    if args.dtype != "fp64" and not args.no_fp64_ref:
        r64 = headline(P, torch, wl, "fp64", args.steps, args.warmup, args.prelude, flags)
        out["fp64_path"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                            "roofline_frac": gemm_roofline(r64, "fp64")["frac"],
                            "step_mfma_frac": step_mfma_frac(D, chi, "fp64", r64["ms_per_step"])}
        i64, n64_ = precision_point(P, wl, "fp64")
        prec = {}
        compared = [args.dtype] + ([] if args.no_other_dtypes else
                                   [d for d in ("fp32", "bf16x3", "bf16") if d != args.dtype])
        for other in compared:
            io, no = precision_point(P, wl, other)
            prec[other] = {"imbalance_err": abs(io - i64), "max_n_err": float(max(abs(a - b) for a, b in zip(no, n64_)))}
        out["precision_vs_fp64"] = dict(prec, schedule="Néel, 20 Trotter steps (t = 1), 10 cold CTMRG "
                                                        "iterations, readout; the same in FP64")
        for other in [d for d in ("fp32", "bf16x3", "bf16") if d != args.dtype and not args.no_other_dtypes]:
            ro = headline(P, torch, wl, other, args.steps, args.warmup, args.prelude, flags)
            out[f"{other}_path"] = {"value": ro["value"], "ms_per_step": ro["ms_per_step"],
                                    "gemm_frac": gemm_roofline(ro, other)["frac"],
                                    "imbalance_err_vs_fp64": prec[other]["imbalance_err"]}
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if not args.no_sweep:
        # batched jobs/s: the 64-job sweep in the contraction precision, split
        # BF16 and FP64, each with its largest imbalance difference from FP64
        sw, ser = sweep(P, synthetic, args.dtype)
        sw64, ser64 = sweep(P, synthetic, "fp64")
        sw["fp64_jobs_per_s"] = sw64["jobs_per_s"]
        sw["max_imbalance_err_vs_fp64"] = max_err(ser, ser64)
        if args.dtype != "bf16x3":
            swb, serb = sweep(P, synthetic, "bf16x3")
            sw["bf16x3_jobs_per_s"] = swb["jobs_per_s"]
            sw["bf16x3_max_imbalance_err_vs_fp64"] = max_err(serb, ser64)
        out["sweep"] = sw
    if not args.no_serving:
        nreq = args.serving_requests
        if args.serving_rate > 0:  # a given arrival rate, one precision
            srv, _ = serving_sample(P, synthetic, args.dtype, rate=args.serving_rate, n_req=nreq)
            srv["rate_note"] = "--serving-rate"
            out["serving"] = srv
        else:
            # requests arrive at 0.8 x the measured capacity of the sweep mix
            cap = out["sweep"]["jobs_per_s"] if "sweep" in out else 1.0
            srv, ser = serving_sample(P, synthetic, args.dtype, rate=0.8 * cap, n_req=nreq)
            srv64, ser64 = serving_sample(P, synthetic, "fp64", rate=0.8 * cap, n_req=nreq)
            srv["fp64_jobs_per_s"] = srv64["jobs_per_s"]
            srv["fp64_p50_s"], srv["fp64_p99_s"] = srv64["p50_s"], srv64["p99_s"]
            srv["max_imbalance_err_vs_fp64"] = max_err(ser, ser64)
            srv["rate_note"] = "0.8 x the sweep's jobs/s in the contraction precision"
            out["serving"] = srv
    if not args.no_free_fermion:
        out["free_fermion"] = free_fermion(P, torch, synthetic, with_cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(D, chi, wl["W"], wl["V"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
