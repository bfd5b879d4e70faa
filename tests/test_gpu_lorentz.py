"""GPU parity of the Lorentz media (the dispersive extension of the linear
response of Sec. 2.3): the field update's oscillators through the C ABI
against the FP64 oracle.

* random fields evolving for 40 steps in boxes with a Lorentz layer beside a
  static one, 1D / 2D / 3D, outflow and periodic transverse boundaries, the
  tiled and the z-marching 3D update: E, b, the polarisation Q and its current
  K element by element;
* the z-marching update against the tiled one bit for bit;
* whole runs (laser through dispersive slabs and the dispersive mirror share,
  ionization births): fields, events, energies and the Gauss law with the
  bound charge, as for the static media.

Tolerances: FP32 against FP64 over 40 steps, 1e-5 of the largest field
(the error grows like the square root of the steps from ~1e-7 per step);
whole runs as for the static media (relative L2 <= 1e-5, identical events).
"""

import numpy as np
import pytest

import workloads as W
from oracle import pic as OP

from test_gpu_parity import P, _compare_run, _run_both  # noqa: F401  (fixture and helpers)

pytestmark = pytest.mark.gpu

SIL = W.silica_dispersive()


def _box_cfg(ndim, n, bc, dxfrac=30, kerr=0.0):
    dx = W.LAMBDA / dxfrac
    m0, m1 = SIL, dict(W.high_index(), gap_eV=9.0)
    if kerr:
        # Kerr terms in both layers (n2 large enough that chi3 E^2 ~ 1e-2 at the
        # test's 1e6 V/m fields)
        m0, m1 = dict(m0, kerr_n2_m2W=kerr), dict(m1, kerr_n2_m2W=0.5 * kerr)
    return dict(ndim=ndim, n=n, dx=[dx] * ndim, cfl=0.95, nsteps=100, transverse_bc=bc,
                # a Lorentz layer beside a static one (9 eV gaps: nothing ionizes)
                materials=[m0, m1],
                layers=[(0, 0.25 * n[0] * dx, 0.55 * n[0] * dx), (1, 0.55 * n[0] * dx, 0.7 * n[0] * dx)],
                ppc=1, T_K=300.0, shape_order=2, keldysh_terms=500, seed=5,
                laser=dict(lambda_m=W.LAMBDA, fwhm_s=W.cycles(2), peak_Wcm2=1e12, envelope="gauss",
                           pol_axis=1), particle_capacity=0, preionize_eV=0.0)


def _random_fields(cfg, seed, scale=1e6):
    rng = np.random.default_rng(seed)
    E = [rng.uniform(-scale, scale, W.domain_shape(cfg, "E", c)).astype(np.float32) for c in range(3)]
    b = [rng.uniform(-scale, scale, W.domain_shape(cfg, "b", c)).astype(np.float32) for c in range(3)]
    return E, b


def _oracle_fields(sim):
    E = [sim.interior_field("E", c) for c in range(3)]
    b = [sim.interior_field("b", c) for c in range(3)]
    Q = [sim.Q[c][sim._domain_slices(sim.stE[c])] for c in range(3)]
    K = [sim.K[c][sim._domain_slices(sim.stE[c])] for c in range(3)]
    return E, b, Q, K


KERR_N2 = 2.7e-12


@pytest.mark.parametrize("ndim,n,bc,tile,kerr", [
    (1, [300], "outflow", None, 0.0), (2, [40, 24], "outflow", None, 0.0), (2, [40, 24], "periodic", None, 0.0),
    (3, [20, 12, 10], "outflow", None, 0.0), (3, [40, 20, 36], "periodic", "5", 0.0),
    (3, [40, 20, 36], "periodic", "7", 0.0),
    (1, [300], "outflow", None, KERR_N2), (2, [40, 24], "periodic", None, KERR_N2),
    (3, [40, 20, 36], "periodic", "5", KERR_N2), (3, [40, 20, 36], "periodic", "7", KERR_N2)])
def test_lorentz_random_fields_match_oracle(P, ndim, n, bc, tile, kerr, monkeypatch):
    """Lorentz layer beside a static one; with kerr, both layers add a Kerr term."""
    if tile:
        monkeypatch.setenv("PIC_FIELD_TILE", tile)
    cfg = _box_cfg(ndim, n, bc, kerr=kerr)
    E, b = _random_fields(cfg, 40 + ndim)
    ctx = P.Context(cfg)
    if tile:
        assert int(ctx.timers()[23]) == int(tile)
    ctx.set_state(0, E, b, None)
    sim = OP.Sim(cfg)
    for c in range(3):
        sim.E[c][sim._domain_slices(sim.stE[c])] = E[c]
        sim.b[c][sim._domain_slices(sim.stB[c])] = b[c]
    nsteps = 40
    ctx.step(nsteps)
    sim.run(nsteps)
    Eg, bg = ctx.fields()
    Qg, Kg = ctx.polarisation()
    Eo, bo, Qo, Ko = _oracle_fields(sim)
    scale = max(np.max(np.abs(a)) for a in Eo + bo)
    assert max(np.max(np.abs(q)) for q in Qo) > 0.05 * scale   # the oscillators are excited
    for name, g_, o_ in (("E", Eg, Eo), ("b", bg, bo), ("Q", Qg, Qo), ("K", Kg, Ko)):
        for c in range(3):
            assert g_[c].shape == o_[c].shape, (name, c)
            err = np.max(np.abs(g_[c] - o_[c]))
            assert err < 1e-5 * scale, (name, c, err / scale)
    if kerr:
        sim_lin = OP.Sim(_box_cfg(ndim, n, bc))
        for c in range(3):
            sim_lin.E[c][sim_lin._domain_slices(sim_lin.stE[c])] = E[c]
            sim_lin.b[c][sim_lin._domain_slices(sim_lin.stB[c])] = b[c]
        sim_lin.run(nsteps)
        # the Kerr term changed the fields far beyond the tolerance
        assert max(np.max(np.abs(sim_lin.interior_field("E", c) - Eo[c])) for c in range(3)) > 1e-3 * scale
    # outside the Lorentz layer the polarisation stays exactly zero
    mat_node = sim.P.mat_node
    static_nodes = np.nonzero(mat_node != 0)[0]
    assert np.all(Qg[1][static_nodes] == 0) and np.all(Kg[2][static_nodes] == 0)
    ctx.close()


def test_lorentz_marching_update_matches_tiled_bitwise(P, monkeypatch):
    """Dispersive mirror layers, random fields: the z-marching update equals
    the tiled one bit for bit in E, b, Q and K after each of 10 steps."""
    cfg = W.config_3d(nx=128, ny=20, nz=36, nsteps=200, ppc=2, fluence=1.0, front=24, dispersive=True)
    E, b = _random_fields(cfg, 78)
    out = {}
    for tile in ("5", "7"):
        monkeypatch.setenv("PIC_FIELD_TILE", tile)
        ctx = P.Context(cfg)
        assert int(ctx.timers()[23]) == int(tile)
        ctx.set_state(0, E, b, None)
        runs = []
        for _ in range(10):
            ctx.step(1)
            Eg, bg = ctx.fields()
            Qg, Kg = ctx.polarisation()
            runs.append(Eg + bg + Qg + Kg)
        out[tile] = runs
        ctx.close()
    for ra, rb in zip(out["5"], out["7"]):
        for a, c in zip(ra, rb):
            assert np.array_equal(a, c)
    assert max(np.max(np.abs(q)) for q in out["7"][-1][6:9]) > 0


def test_kerr_run_1d_slab(P):
    """The 1D slab at 1e14 W/cm^2 with fused silica's Kerr index (2.5e-20 m^2/W)
    on top of its Lorentz response."""
    cfg = W.config_1d(hi=True, ppc=10, nsteps=1400, dispersive=True)
    cfg["materials"] = [dict(cfg["materials"][0], kerr_n2_m2W=2.5e-20)]
    ctx, sim = _run_both(P, cfg, 1400)
    _compare_run(P, ctx, sim, min_events=20, name="run_1d_kerr")
    ctx.close()


def test_lorentz_run_1d_slab(P):
    cfg = W.config_1d(hi=True, ppc=10, nsteps=1400, dispersive=True)
    ctx, sim = _run_both(P, cfg, 1400)
    _compare_run(P, ctx, sim, min_events=20, name="run_1d_lorentz")
    Qg, _ = ctx.polarisation()
    Qo = sim.Q[1][sim._domain_slices(sim.stE[1])]
    assert np.max(np.abs(Qg[1] - Qo)) <= 1e-4 * np.max(np.abs(Qo))
    ctx.close()


def test_lorentz_run_2d_slab_gaussian_beam(P):
    cfg = W.config_2d(nx=192, ny=48, nsteps=520, ppc=2, peak=3e14, slab_cells=12, waist=0.6e-6,
                      dispersive=True)
    ctx, sim = _run_both(P, cfg, 520)
    _compare_run(P, ctx, sim, min_events=20, name="run_2d_lorentz")
    ctx.close()


@pytest.mark.parametrize("field_tile", ["tiled", "march"])
def test_lorentz_run_3d_mirror_periodic(P, field_tile, monkeypatch):
    if field_tile == "march":
        monkeypatch.setenv("PIC_FIELD_TILE", "7")
    cfg = W.config_3d(nx=96, ny=8, nz=8, nsteps=380, ppc=8, fluence=1.0, front=24, dispersive=True)
    ctx, sim = _run_both(P, cfg, 380)
    _compare_run(P, ctx, sim, min_events=20, name="run_3d_lorentz" + ("_march" if field_tile == "march" else ""))
    ctx.close()
