"""GPU parity of impact ionization (Keldysh's impact rate, the paper's future
work, Sec. 2.2) through the C ABI against the FP64 oracle.

* one step from a seeded state of hot electrons in a material with neutrals
  (1D and 2D): identical events (neutral ids), the impacting electrons'
  momenta element by element, the births matched by kind and position;
* a whole 1D slab run at 3e14 W/cm^2 where impacts add to photoionization:
  fields, identical events, counts and energies as for every run.
"""

import numpy as np
import pytest

import workloads as W
from oracle import pic as OP
from oracle import impact as IM
from oracle.constants import C, QE

from test_gpu_parity import P, _compare_run, _records, _run_both, _state_f32, _to_oracle_state  # noqa: F401

pytestmark = pytest.mark.gpu


def _hot_state(cfg, n, seed, eps_eV):
    """Electrons of material 0 at kinetic energy eps_eV, random directions,
    in the material's cells; weak random fields."""
    rng = np.random.default_rng(seed)
    st = W.random_state(cfg, n, seed=seed, e_scale=1e5, u_scale=0.0, margin=2)
    me = 0.6 * 9.1093837015e-31
    g = 1.0 + eps_eV * QE / (me * C * C)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    st["u"] = d * np.sqrt(g * g - 1.0)
    st["kind"] = np.zeros(n, dtype=np.int64)
    nx = cfg["n"][0]
    st["cell"][:, 0] = rng.integers(2, int(0.7 * nx) - 1, n)
    return _state_f32(st)


@pytest.mark.parametrize("ndim,n", [(1, [96]), (2, [32, 8])])
def test_impact_one_step_matches_oracle(P, ndim, n):
    dx = W.LAMBDA / 30
    probe = OP.Sim(dict(W.config_1d(n=32, ppc=1, nsteps=10)), load_neutrals=False)
    eth = IM.threshold_eV(probe.P.mats[0])
    cfg = dict(ndim=ndim, n=n, dx=[dx] * ndim, cfl=0.95, nsteps=10, transverse_bc="periodic",
               materials=[W.with_impact(W.silica_like(), 0.0)],
               layers=[(0, 0.0, 0.7 * n[0] * dx)], ppc=4, T_K=300.0, shape_order=2, keldysh_terms=500,
               seed=41, laser=dict(lambda_m=W.LAMBDA, fwhm_s=W.cycles(2), peak_Wcm2=1e10, envelope="gauss",
                                   pol_axis=1), particle_capacity=0, preionize_eV=0.0)
    dt = OP.Sim(cfg, load_neutrals=False).P.dt
    # rate constant giving p = 0.3 at 2 E_th
    cfg["materials"] = [W.with_impact(W.silica_like(), -np.log(0.7) / dt)]
    st = _hot_state(cfg, 400 if ndim == 1 else 800, 500 + ndim, 2.0 * eth)
    ctx = P.Context(cfg)
    ctx.set_resort(0)
    ctx.set_state(0, st["E"], st["b"], _records(P, st, ndim))
    ctx.step(1)
    parts = ctx.particles()
    sim = OP.Sim(cfg)
    _to_oracle_state(sim, st)
    sim.step()
    ev_g = set(map(tuple, ctx.events().tolist()))
    ev_o = sim.event_set()
    assert len(ev_o) > 40
    assert ev_g == ev_o
    assert len(parts) == len(sim.px)
    npre = len(st["kind"])
    umax = np.max(np.abs(sim.pu[:npre]))
    assert np.max(np.abs(parts["u"][:npre] - sim.pu[:npre])) < 1e-5 * umax
    pos_g = parts["cell"][:, :ndim] + parts["off"][:, :ndim].astype(np.float64)
    kg = parts["kind"][npre:].astype(np.int64)
    og = np.lexsort(tuple(pos_g[npre:, d] for d in range(ndim)) + (kg,))
    oo = np.lexsort(tuple(sim.px[npre:, d] for d in range(ndim)) + (sim.pk[npre:],))
    assert np.array_equal(kg[og], sim.pk[npre:][oo])
    assert np.max(np.abs(pos_g[npre:][og] - sim.px[npre:, :ndim][oo])) < 1e-6
    assert np.max(np.abs(parts["u"][npre:][og] - sim.pu[npre:][oo])) < 1e-5 * max(umax, 1e-4)
    sc = ctx.scalars()
    assert sc["events"] == len(ev_o)
    assert abs(sc["e_gap"] - sim.energy_gap) <= 1e-10 * sim.energy_gap
    ctx.close()


def test_impact_run_1d_slab(P):
    cfg = W.config_1d(hi=True, ppc=4, n=512, nsteps=1100, peak=3e14)
    cfg["materials"] = [W.with_impact(cfg["materials"][0], 1e16)]
    ctx, sim = _run_both(P, cfg, 1100)
    _compare_run(P, ctx, sim, min_events=20, name="run_1d_impact")
    ctx.close()
