"""Serving (continuous batching) on the GPU: every request's result is the same
whether it ran alone or in the mix with runs that arrived before and after it
(fields to FP32 summation-order noise, identical ionization events), and the
server admits by footprint and retires every request."""

import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2502_13695_amd import pic
    pic.lib()
    return pic


def _requests():
    c1 = W.config_1d(hi=True, ppc=4, nsteps=300, n=256)
    c2 = W.config_2d(nx=128, ny=32, nsteps=240, ppc=2, peak=3e14, slab_cells=10, waist=0.6e-6, seed=5)
    c3 = W.config_3d(nx=64, ny=8, nz=8, nsteps=200, ppc=4, fluence=1.5, front=16)
    c4 = W.config_2d(nx=96, ny=48, nsteps=260, ppc=2, peak=3e14, slab_cells=8, waist=0.6e-6, seed=9)
    # staggered arrivals: later requests join while earlier ones are running
    return [dict(cfg=c1, arrival_s=0.0), dict(cfg=c2, arrival_s=0.0),
            dict(cfg=c3, arrival_s=0.05), dict(cfg=c4, arrival_s=0.1)]


def _l2(fa, fb):
    num = sum(np.sum((a - b) ** 2) for a, b in zip(fa[0] + fa[1], fb[0] + fb[1]))
    den = sum(np.sum(b ** 2) for b in fb[0] + fb[1])
    return math.sqrt(num / den)


def test_served_results_match_runs_alone(P):
    from paper_2502_13695_amd import serve as S
    reqs = _requests()
    srv = S.Server(chunk=20, max_members=8)
    res = srv.run(reqs, keep_fields=True)
    assert srv.stats["completed"] == len(reqs)
    assert srv.stats["max_resident"] >= 2          # runs overlapped on the device
    for r, q in zip(res, reqs):
        x = P.Context(q["cfg"])
        x.step(q["cfg"]["nsteps"])
        f_alone = x.fields()
        ev_alone = set(map(tuple, x.events().tolist()))
        sc_alone = x.scalars()
        x.close()
        assert r["steps"] == q["cfg"]["nsteps"]
        assert r["scalars"]["step"] == q["cfg"]["nsteps"]
        assert _l2(r["fields"], f_alone) < 1e-5
        ev = set(map(tuple, r["events"].tolist()))
        assert len(ev ^ ev_alone) <= max(1, int(1e-4 * len(ev | ev_alone)))
        assert abs(r["scalars"]["n_e"] - sc_alone["n_e"]) <= max(1.0, 5e-3 * sc_alone["n_e"])
        assert r["latency_s"] >= 0.0


def test_server_waits_for_memory(P):
    """With a budget that holds one run at a time, runs are served one after the
    other and all of them complete."""
    from paper_2502_13695_amd import serve as S
    reqs = _requests()[:2]
    need = max(P.footprint(q["cfg"]) for q in reqs)
    srv = S.Server(hbm_budget=need, chunk=50)
    res = srv.run(reqs)
    assert srv.stats["completed"] == 2 and srv.stats["max_resident"] == 1
    assert res[1]["admit_s"] >= res[0]["done_s"] - 1e-3 or res[0]["admit_s"] >= res[1]["done_s"] - 1e-3
