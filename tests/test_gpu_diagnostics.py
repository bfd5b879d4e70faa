"""GPU parity of the paper-style diagnostics (Sec. 5) through the C ABI.

* Energy histogram: from the same seeded particle state (set through
  pic_set_state, FP32 u) the device counts must equal the oracle's exactly,
  per kind and bin, with and without an x range, for log and linear edges, in
  the per-block LDS path and the direct HBM path, at small sizes in 1D/2D/3D
  and at the 2D benchmark grid with 1.2e6 particles.
* Maximum accumulated intensity: from a seeded random field state, sampled
  every other step, against the oracle's running maximum (FP32 fields after a
  few steps: 5e-6 of the largest value); through a whole 1D slab run with
  ionization, sampled at 0.5 fs intervals (relative L2 2e-5, twice the field
  tolerance since the quantity is squared); stopping keeps the maximum; a batch
  refuses a member that samples.
* Trajectory sampling: from a seeded state through sorts and through a slab
  run with births, the same (id, kind, step) records as the oracle, positions
  to FP32 accuracy; a record budget keeps that many and counts the rest.
* Edge cases: no charged particles, a zero record budget, sampling that never
  reaches its step, the largest edge count.
"""

import numpy as np
import pytest

import workloads as W
from oracle import pic as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2502_13695_amd import pic
    pic.lib()
    return pic


def _cfg(ndim, n, nsteps=20):
    dx = W.LAMBDA / 30
    return dict(ndim=ndim, n=n, dx=[dx] * ndim, cfl=0.95, nsteps=nsteps, transverse_bc="outflow",
                materials=[W.silica_like(), dict(W.high_index(), gap_eV=9.0)],
                layers=[(0, 0.3 * n[0] * dx, 0.5 * n[0] * dx), (1, 0.5 * n[0] * dx, 0.62 * n[0] * dx)],
                ppc=2, T_K=300.0, shape_order=2, keldysh_terms=500, seed=11,
                laser=dict(lambda_m=W.LAMBDA, fwhm_s=W.cycles(2), peak_Wcm2=1e12, envelope="gauss",
                           pol_axis=1), particle_capacity=0, preionize_eV=0.0)


def _records(P, st, ndim):
    rec = np.zeros(len(st["kind"]), dtype=P.PARTICLE_DTYPE)
    rec["cell"][:, :ndim] = st["cell"][:, :ndim]
    rec["off"] = st["off"]
    rec["u"] = st["u"].astype(np.float32)
    rec["kind"] = st["kind"]
    return rec


def _oracle_with(cfg, st, load_neutrals=False):
    sim = OP.Sim(cfg, load_neutrals=load_neutrals)
    for c in range(3):
        sim.E[c][sim._domain_slices(sim.stE[c])] = np.asarray(st["E"][c], dtype=np.float32)
        sim.b[c][sim._domain_slices(sim.stB[c])] = np.asarray(st["b"][c], dtype=np.float32)
    sim.px = st["cell"].astype(np.float64) + st["off"].astype(np.float64)
    sim.pu = st["u"].astype(np.float32).astype(np.float64)
    sim.pk = st["kind"].astype(np.int64)
    return sim


def _u_wide(st, seed):
    """Momenta spanning meV to MeV electrons: |u| log-uniform over 1e-4 .. 3."""
    rng = np.random.default_rng(seed)
    d = st["u"] / np.linalg.norm(st["u"], axis=1, keepdims=True)
    mag = 10.0 ** rng.uniform(-4.0, 0.5, len(d))
    st["u"] = (d * mag[:, None]).astype(np.float32)
    return st


EDGE_SETS = {
    "log200": np.geomspace(1e-4, 3e6, 201),                 # 4 kinds x 202 columns: LDS counts
    "linear": np.linspace(0.0, 500.0, 51),
    "log3000": np.geomspace(1e-3, 1e6, 3001),               # 4 x 3002 > LDS budget: HBM atomics
}


@pytest.mark.parametrize("edges", sorted(EDGE_SETS))
@pytest.mark.parametrize("ndim,n", [(1, [300]), (2, [60, 24]), (3, [20, 12, 10])])
def test_spectrum_bit_exact(P, ndim, n, edges):
    cfg = _cfg(ndim, n)
    st = _u_wide(W.random_state(cfg, 4000, seed=300 + ndim, e_scale=1e8), seed=ndim)
    ctx = P.Context(cfg)
    ctx.set_state(0, st["E"], st["b"], _records(P, st, ndim))
    sim = _oracle_with(cfg, st)
    e = EDGE_SETS[edges]
    for lo, hi in ((0, 0), (n[0] // 4, n[0] // 2), (n[0] - 5, n[0] + 10)):
        got = ctx.spectrum(e, lo, hi).astype(np.int64)
        want = sim.energy_spectrum(e, lo, hi)
        assert got.shape == want.shape
        assert np.array_equal(got, want), (lo, hi, np.argwhere(got != want)[:5])
    ctx.close()


def test_spectrum_at_benchmark_size(P):
    """The 2D slab grid (2048 x 512) with 1.2e6 charged particles."""
    cfg = W.config_2d()
    st = _u_wide(W.random_state(cfg, 1_200_000, seed=77, e_scale=1e8), seed=78)
    ctx = P.Context(cfg)
    ctx.set_state(0, st["E"], st["b"], _records(P, st, 2))
    sim = _oracle_with(cfg, st)
    for name in ("log200", "log3000"):
        e = EDGE_SETS[name]
        for lo, hi in ((0, 0), (512, 592)):
            got = ctx.spectrum(e, lo, hi).astype(np.int64)
            assert np.array_equal(got, sim.energy_spectrum(e, lo, hi)), (name, lo, hi)
    ctx.close()


def test_spectrum_rejects_bad_edges(P):
    cfg = _cfg(1, [100])
    ctx = P.Context(cfg)
    for bad in ([1.0], [1.0, 1.0], [2.0, 1.0], [0.0, np.inf], np.linspace(0, 1, 4099)):
        with pytest.raises(P.PicError):
            ctx.spectrum(np.asarray(bad, dtype=np.float64))
    ctx.close()


@pytest.mark.parametrize("ndim,n,bc", [(1, [200], "outflow"), (2, [40, 24], "outflow"),
                                       (2, [40, 24], "periodic"), (3, [20, 12, 10], "periodic")])
def test_imax_from_random_fields(P, ndim, n, bc):
    cfg = dict(_cfg(ndim, n), transverse_bc=bc)
    st = W.random_state(cfg, 0, seed=500 + ndim, e_scale=1e8)
    ctx = P.Context(cfg)
    ctx.set_state(0, st["E"], st["b"], None)
    ctx.set_imax(2)
    sim = _oracle_with(cfg, st, load_neutrals=True)
    sim.set_imax(2)
    for _ in range(7):
        sim.step()
    ctx.step(7)
    got, want = ctx.imax(), sim.imax_nodes()
    assert got.shape == want.shape
    assert np.max(want) > 0
    assert np.max(np.abs(got - want)) < 5e-6 * np.max(want)
    # stopping keeps the maximum
    ctx.set_imax(0)
    ctx.step(3)
    assert np.array_equal(ctx.imax(), got)
    ctx.close()


def test_imax_through_slab_run(P):
    nsteps = 900
    cfg = W.config_1d(hi=True, ppc=10, nsteps=nsteps)
    ctx = P.Context(cfg)
    dt = ctx.params().dt
    every = max(1, int(round(0.5e-15 / dt)))     # the paper's 0.5 fs sampling
    ctx.set_imax(every)
    ctx.step(nsteps)
    sim = OP.Sim(cfg)
    sim.set_imax(every)
    sim.run(nsteps)
    got, want = ctx.imax().astype(np.float64), sim.imax_nodes()
    l2 = np.sqrt(np.sum((got - want) ** 2) / np.sum(want ** 2))
    assert l2 < 2e-5, l2
    ctx.close()


def test_batch_refuses_sampling_member(P):
    cfg = _cfg(1, [100])
    a, b = P.Context(cfg), P.Context(cfg)
    a.set_imax(4)
    bt = P.Batch([a, b])
    with pytest.raises(P.PicError):
        bt.step(1)
    a.set_imax(0)
    bt.step(1)
    bt.close()
    a.close()
    b.close()


def _tracks_oracle(sim):
    return {(i, k, s): np.array([x, y, z]) for i, k, s, x, y, z in sim.tracks}


def _tracks_gpu(recs, ndim):
    pos = recs["cell"].astype(np.float64) + recs["off"].astype(np.float64)
    return {(int(r["id"]), int(r["kind"]), int(r["step"])): pos[q] for q, r in enumerate(recs)}


@pytest.mark.parametrize("ndim,n,bc", [(1, [300], "outflow"), (2, [60, 24], "periodic"),
                                       (3, [20, 12, 10], "periodic")])
def test_tracks_from_seeded_state(P, ndim, n, bc):
    """Placed particles (ids cells x ppc + index) sampled at 1/4, recorded every
    other step for 10 steps, then the tile sort reorders the slots: the same
    (id, kind, step) records as the oracle, positions to FP32 accuracy."""
    cfg = dict(_cfg(ndim, n), transverse_bc=bc)
    st = W.random_state(cfg, 3000, seed=700 + ndim, e_scale=3e8, u_scale=0.05)
    ctx = P.Context(cfg)
    ctx.set_resort(1)
    ctx.set_state(0, st["E"], st["b"], _records(P, st, ndim))
    ctx.set_tracks(0.25, 2)
    sim = _oracle_with(cfg, st, load_neutrals=True)
    sim.set_tracks(0.25, 2)
    for _ in range(10):
        sim.step()
    ctx.step(10)
    g, o = _tracks_gpu(ctx.tracks(), ndim), _tracks_oracle(sim)
    assert len(o) > 500
    assert set(g) == set(o)
    err = max(np.max(np.abs(g[k][:ndim] - o[k][:ndim])) for k in o)
    assert err < 2e-4, err
    assert ctx.scalars()["tracks_dropped"] == 0
    ctx.close()


def test_tracks_through_slab_run(P):
    """A 1D slab run with ionization: births sampled by their neutral's id; the
    same records as the oracle (electron and positive carrier together)."""
    nsteps = 1400
    cfg = W.config_1d(hi=True, ppc=10, nsteps=nsteps)
    ctx = P.Context(cfg)
    ctx.set_tracks(0.5, 5)
    ctx.step(nsteps)
    sim = OP.Sim(cfg)
    sim.set_tracks(0.5, 5)
    sim.run(nsteps)
    g, o = _tracks_gpu(ctx.tracks(), 1), _tracks_oracle(sim)
    assert len(o) > 100
    assert set(g) == set(o)
    err = max(abs(g[k][0] - o[k][0]) for k in o)
    assert err < 1e-3, err
    ids = {k[0] for k in g}
    kinds = {(k[0], k[1]) for k in g}
    assert len(kinds) == 2 * len(ids)           # both carriers of every sampled birth
    # a small record budget keeps that many and counts the rest
    ctx2 = P.Context(cfg)
    ctx2.set_tracks(0.5, 5, max_records=50)
    ctx2.step(nsteps)
    kept = _tracks_gpu(ctx2.tracks(), 1)
    assert len(kept) == 50 and set(kept) <= set(o)
    assert ctx2.scalars()["tracks_dropped"] == len(o) - 50
    ctx.close()
    ctx2.close()


def test_batch_refuses_recording_member(P):
    cfg = _cfg(1, [100])
    a, b = P.Context(cfg), P.Context(cfg)
    a.set_tracks(0.5, 3)
    bt = P.Batch([a, b])
    with pytest.raises(P.PicError):
        bt.step(1)
    a.set_tracks(0.5, 0)
    bt.step(1)
    bt.close()
    a.close()
    b.close()


def test_diagnostics_edge_cases(P):
    """Empty and degenerate inputs: no charged particles, a zero record budget,
    sampling that never reaches its step, the largest edge count."""
    cfg = _cfg(1, [200])
    ctx = P.Context(cfg)
    edges = np.geomspace(1e-3, 1e3, 4097)                 # the largest edge count
    h = ctx.spectrum(edges)
    assert h.shape == (4, 4098) and not h.any()           # no charged particles yet
    assert not ctx.imax().any()                           # never enabled
    ctx.set_imax(1000)
    ctx.step(5)
    assert not ctx.imax().any()                           # no sampled step yet
    ctx.set_tracks(1.0, 1, max_records=0)
    ctx.step(2)
    assert len(ctx.tracks()) == 0 and ctx.scalars()["tracks_dropped"] == 0
    # particles placed, every one sampled, none kept: all counted as dropped
    st = W.random_state(cfg, 500, seed=9, e_scale=1e7, u_scale=0.01)
    ctx.set_state(ctx.scalars()["step"], st["E"], st["b"], _records(P, st, 1))
    ctx.set_tracks(1.0, 1, max_records=0)
    ctx.step(1)
    n_live = int(ctx.scalars()["n_e"] + ctx.scalars()["n_pos"])
    assert len(ctx.tracks()) == 0 and ctx.scalars()["tracks_dropped"] == n_live > 0
    # the largest edge count, against the oracle, from the placed state
    sim = _oracle_with(cfg, st)
    ctx2 = P.Context(cfg)
    ctx2.set_state(0, st["E"], st["b"], _records(P, st, 1))
    assert np.array_equal(ctx2.spectrum(edges).astype(np.int64), sim.energy_spectrum(edges))
    ctx.close()
    ctx2.close()
