"""Lockstep batches of jobs (one launch per kernel for all of them) against
the same jobs run alone, through the C ABI (needs an MI355X).

A batch merges each GEMM group of the jobs' plans into one launch (every
problem keeps its own tile kind and summation order) and runs the simple
update, the Cholesky, Jacobi and projector kernels with one row of
workgroups per job, so each job's arithmetic is the one it has alone:
FP64 and FP32 results must be bitwise equal to the solo runs.  The jobs of a
batch differ in W, V, dt and seed; they share D, chi and the precision."""
import numpy as np
import pytest

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu

PARAMS = [dict(W=3.0, V=1.0, dt=0.05, seed=1), dict(W=8.0, V=0.0, dt=0.05, seed=2),
          dict(W=1.5, V=2.0, dt=0.04, seed=3)]


def _cfg(D, chi, dtype, flags, p):
    return P.make_config(D, chi, J=1.0, V=p["V"], W=p["W"], dt=p["dt"], dtype=dtype, seed=p["seed"],
                         flags=flags)


def _schedule_solo(st):
    out = []
    st.trotter_step(3)
    st.ctmrg(0.0, 4, True)
    out.append((st.observe(), st.corner_spectra(), st.bond_spectra()))
    st.trotter_step(2)
    st.ctmrg(0.0, 3, False)
    out.append((st.observe(), st.corner_spectra(), st.bond_spectra()))
    return out


@pytest.mark.parametrize("D,chi,dtype,flags", [(2, 8, "fp64", 0), (3, 12, "fp64", 0), (4, 16, "fp32", 0),
                                               (3, 18, "fp64", 2), (4, 32, "bf16x3", 2)])
def test_batch_equals_alone(D, chi, dtype, flags):
    print(f"batch D={D} chi={chi} {dtype} flags={flags}", flush=True)
    solo = []
    for p in PARAMS:
        st = P.State(_cfg(D, chi, dtype, flags, p))
        solo.append(_schedule_solo(st))
        st.close()
    slab = P.Slab(_cfg(D, chi, dtype, flags, PARAMS[0]), 4)
    # slots 3, 0, 2: a batch need not use contiguous or ordered slots
    sts = [slab.state(sl, _cfg(D, chi, dtype, flags, p)) for sl, p in zip((3, 0, 2), PARAMS)]
    got = [[] for _ in sts]
    b = P.Batch(sts)
    b.trotter_step(3)
    b.ctmrg(4, True)
    for i, o in enumerate(b.observe()):
        got[i].append(o)
    b.close()
    for i, st in enumerate(sts):  # spectra through the solo calls, after the batch
        got[i][0] = (got[i][0], st.corner_spectra(), st.bond_spectra())
    b = P.Batch(sts)
    b.trotter_step(2)
    b.ctmrg(3, False)
    for i, o in enumerate(b.observe()):
        got[i].append(o)
    b.close()
    for i, st in enumerate(sts):
        got[i][1] = (got[i][1], st.corner_spectra(), st.bond_spectra())
    for i in range(len(PARAMS)):
        for (a, ca, ba), (g, cg, bg) in zip(solo[i], got[i]):
            assert a["imbalance"] == g["imbalance"], (i, a["imbalance"], g["imbalance"])
            assert np.array_equal(a["n"], g["n"]) and np.array_equal(a["eps"], g["eps"])
            assert a["t"] == g["t"] and a["ctm_delta"] == g["ctm_delta"]
            assert np.array_equal(ca, cg) and np.array_equal(ba, bg)
    for st in sts:
        st.close()
    slab.close()


@pytest.mark.parametrize("D,chi,dtype,flags,njobs", [(2, 8, "fp64", 0, 3), (3, 18, "fp64", 2, 3),
                                                      (4, 16, "fp32", 0, 3), (4, 32, "bf16x3", 2, 3),
                                                      (3, 12, "fp64", 0, 1)])
def test_graph_replays_equal_eager(D, chi, dtype, flags, njobs):
    """Warm iterations replayed from the batch's captured graph: every
    observation of three chunks (the graph captured in the first, replayed in
    all) equals the jobs' solo eager runs bit for bit, with eager work of
    another state and host synchronisations between the chunks."""
    print(f"graph batch D={D} chi={chi} {dtype} flags={flags} jobs={njobs}", flush=True)
    params = PARAMS[:njobs]
    sched = [(3, 4, True), (2, 5, False), (1, 3, False)]  # (Trotter steps, iterations, cold)

    def solo_run(p):
        st = P.State(_cfg(D, chi, dtype, flags, p))
        out = []
        for n, it, cold in sched:
            st.trotter_step(n)
            st.ctmrg(0.0, it, cold)
            out.append((st.observe(), st.corner_spectra()))
        st.close()
        return out

    solo = [solo_run(p) for p in params]
    other = P.State(_cfg(D, chi, dtype, flags, PARAMS[-1]))
    slab = P.Slab(_cfg(D, chi, dtype, flags, params[0]), 4)
    sts = [slab.state(sl, _cfg(D, chi, dtype, flags, p)) for sl, p in zip((1, 3, 0), params)]
    b = P.Batch(sts, graph=True)
    got = []
    for n, it, cold in sched:
        b.trotter_step(n)
        b.ctmrg(it, cold)
        got.append(b.observe())
        # eager work on another state between the replays
        other.trotter_step(1)
        other.ctmrg(0.0, 2, True)
        other.observe()
    b.close()
    spectra = [st.corner_spectra() for st in sts]  # after the last chunk
    for i in range(njobs):
        for c, (ref, ref_spec) in enumerate(solo[i]):
            g = got[c][i]
            assert g["imbalance"] == ref["imbalance"], (i, c, g["imbalance"], ref["imbalance"])
            assert np.array_equal(g["n"], ref["n"]) and np.array_equal(g["eps"], ref["eps"])
            assert g["t"] == ref["t"] and g["ctm_delta"] == ref["ctm_delta"], (i, c)
        assert np.array_equal(spectra[i], solo[i][-1][1])
    other.close()
    for st in sts:
        st.close()
    slab.close()


def test_batch_rejects_mixed_layouts_and_foreign_states():
    a = P.State(P.make_config(2, 8))
    b = P.State(P.make_config(2, 8, W=2.0))
    with pytest.raises(P.IpepsError):  # not one slab: no common layout offset
        P.Batch([a, b])
    slab = P.Slab(P.make_config(2, 8), 2)
    with pytest.raises(P.IpepsError):  # a different layout in the slab
        slab.state(0, P.make_config(2, 12))
    s0 = slab.state(0, P.make_config(2, 8))
    with pytest.raises(P.IpepsError):  # slot taken
        slab.state(0, P.make_config(2, 8))
    s1 = slab.state(1, P.make_config(2, 8, W=3.0))
    s1.trotter_step(1)
    s1.ctmrg(0.0, 2, True)
    with pytest.raises(P.IpepsError):  # different phases (one has an environment)
        P.Batch([s0, s1])
    s0.close()
    s0 = slab.state(0, P.make_config(2, 8))  # the freed slot is reusable
    s0.close()
    for s in (a, b, s1):
        s.close()
    slab.close()


def test_nan_in_one_job_leaves_the_others():
    """Job 1 of a batch of three starts from a state with a NaN: its readout
    reports IPEPS_ENUMERIC and it is poisoned; jobs 0 and 2 give what they
    give alone."""
    import synthetic
    cfgs = [_cfg(3, 12, "fp64", 0, p) for p in PARAMS]
    gam, lam = synthetic.random_state(11, 3)
    bad = gam.copy()
    bad[0, 0, 0, 0, 0, 0] = np.nan
    ref = []
    for i in (0, 2):
        st = P.State(cfgs[i])
        st.set_state(gam, lam)
        st.trotter_step(1)
        st.ctmrg(0.0, 3, True)
        ref.append(st.observe())
        st.close()
    slab = P.Slab(cfgs[0], 3)
    sts = [slab.state(i, cfgs[i]) for i in range(3)]
    for i, st in enumerate(sts):
        st.set_state(bad if i == 1 else gam, lam)
    b = P.Batch(sts)
    b.trotter_step(1)
    b.ctmrg(3, True)
    obs, status = b.observe_status()
    b.close()
    assert status == [0, -4, 0], status
    for o, r in zip((obs[0], obs[2]), ref):
        assert o["imbalance"] == r["imbalance"] and np.array_equal(o["n"], r["n"])
    with pytest.raises(P.IpepsError) as e:
        sts[1].ctmrg(0.0, 1, True)
    assert e.value.code == -4
    for st in sts:
        st.close()
    slab.close()
