"""Request loop (solve_submit / solve_poll) on the device.

* every job's time series equals the same job run alone through the state
  API (same kernels, same order: bitwise in FP64);
* several jobs are resident and run at the same time when the HBM budget
  allows it, and are serialised when the budget holds one job;
* invalid jobs are refused at submission; unknown ids are reported.
"""
import time

import numpy as np
import pytest

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu


def _alone(cfg, n_steps, every, iters):
    st = P.State(cfg)
    out, done, first = [], 0, True
    while done < n_steps:
        chunk = min(every, n_steps - done)
        st.trotter_step(chunk)
        done += chunk
        st.ctmrg(0.0, iters, first)
        first = False
        out.append(st.observe())
    st.close()
    return out


def _wait(srv, ids, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(ids):
        for j in ids:
            if j in res:
                continue
            status, series = srv.poll(j)
            if series is not None:
                res[j] = series
        assert time.time() - t0 < timeout, "jobs did not finish"
        time.sleep(0.01)
    return res


JOBS = [dict(D=2, chi=8, W=5.0, V=1.0), dict(D=3, chi=18, W=3.0, V=0.0),
        dict(D=2, chi=8, W=12.0, V=1.0), dict(D=3, chi=9, W=7.0, V=1.0),
        dict(D=4, chi=16, W=2.0, V=1.0), dict(D=2, chi=12, W=1.5, V=0.5)]


@pytest.mark.parametrize("graphs", [False, True])
def test_mix_equals_alone(graphs):
    """graphs: the loop's batches replay captured warm iterations and a group
    whose jobs all go on keeps its batch (and graph) for the next chunk."""
    print(f"server mix graphs={graphs}", flush=True)
    srv = P.Server(hbm_budget=0, max_slots=4, graphs=graphs)
    ids, cfgs = [], []
    for j in JOBS:
        cfg = P.make_config(j["D"], j["chi"], W=j["W"], V=j["V"], dt=0.05)
        cfgs.append(cfg)
        ids.append(srv.submit(cfg, n_steps=9, observe_every=3, ctm_iters=4))
    res = _wait(srv, ids)
    times = [srv.times(j)[1] for j in ids]
    srv.close()
    for jid, cfg in zip(ids, cfgs):
        ref = _alone(cfg, 9, 3, 4)
        got = res[jid]
        assert len(got) == len(ref) == 3
        for g, r in zip(got, ref):
            assert g["t"] == r["t"]
            assert g["imbalance"] == r["imbalance"]
            assert np.array_equal(g["n"], r["n"]) and np.array_equal(g["eps"], r["eps"])
    # at least two jobs were resident at once
    spans = [(a, d) for (_, a, d) in times]
    overlap = any(a2 < d1 and a1 < d2 for i, (a1, d1) in enumerate(spans)
                  for (a2, d2) in spans[i + 1:])
    assert overlap


def test_budget_of_one_job_serialises():
    cfg = P.make_config(3, 9, W=4.0, V=1.0)
    fp = P.footprint_bytes(cfg)
    srv = P.Server(hbm_budget=fp, max_slots=4)
    ids = [srv.submit(cfg, n_steps=2, observe_every=2, ctm_iters=2) for _ in range(3)]
    _wait(srv, ids)
    spans = sorted(srv.times(j)[1][1:] for j in ids)
    srv.close()
    for (a1, d1), (a2, d2) in zip(spans, spans[1:]):
        assert a2 >= d1


def test_rejections():
    srv = P.Server(hbm_budget=1 << 30, max_slots=2)
    with pytest.raises(P.IpepsError):
        srv.submit(P.make_config(3, 4), n_steps=2)          # chi < D^2
    with pytest.raises(P.IpepsError):
        srv.submit(P.make_config(8, 128), n_steps=2)        # above the whole budget
    with pytest.raises(P.IpepsError):
        srv.poll(987654)
    srv.close()


def test_bond_dimension_stopping_rule():
    """D=2 and D=3 evolved together through the request loop: each series
    equals its job run alone, t_stop is the first time their imbalances
    differ by more than tol, and the entropies stay in [0, ln 2]."""
    from paper_1910_11359_amd import validity

    kw = dict(J=1.0, V=1.0, W=3.0, dt=0.05)
    out = validity.compare_bond_dimensions(2, lambda D: 2 * D * D, n_steps=20, observe_every=5,
                                           ctm_iters=6, tol=1e-3, **kw)
    s2, s3 = out["series"][2], out["series"][3]
    assert len(s2) == len(s3) == 4
    ref = _alone(P.make_config(3, 18, **kw), 20, 5, 6)
    assert all(a["imbalance"] == b["imbalance"] for a, b in zip(s3, ref))
    diffs = [abs(a["imbalance"] - b["imbalance"]) for a, b in zip(s2, s3)]
    expect = next((a["t"] for a, d in zip(s2, diffs) if d > 1e-3), None)
    assert out["t_stop"] == expect
    for s in (s2, s3):
        for o in s:
            assert np.all(o["renyi1"] >= -1e-12) and np.all(o["renyi1"] <= np.log(2) + 1e-12)
            assert np.all(o["renyi_half"] >= o["renyi1"] - 1e-12)
