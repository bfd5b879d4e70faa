"""GPU parity of the binary collisions (Sec. 2.2, Eq. 4) through the C ABI
against the FP64 oracle.

* one step from a seeded random state with many particles per cell (two
  materials, all four kinds, weak fields so nothing ionizes), 1D / 2D / 3D,
  and three materials in 2D (six kinds, most cells holding five or six):
  every particle's position and momentum element by element;
* the tile sort on against off: the same momenta bit for bit (the pairing
  order is keyed by id and kind, not by the slot);
* a whole 1D run with ionization births and collisions: fields, events,
  counts and energies as for the runs without collisions.

Tolerances: the collisions run in FP64 on momenta stored as FP32 between the
collisions of a step, against FP64 throughout: 1e-5 of the largest |u|.
"""

import numpy as np
import pytest

import workloads as W
from oracle import pic as OP

from test_gpu_parity import P, _compare_run, _records, _run_both, _state_f32, _to_oracle_state  # noqa: F401

pytestmark = pytest.mark.gpu


def _dense_cfg(ndim, n, nmat=2):
    dx = W.LAMBDA / 30
    mats = [dict(W.silica_like(), gap_eV=40.0), dict(W.high_index(), gap_eV=40.0),
            dict(W.silica_like(), gap_eV=45.0, me_star=0.4, density_gcc=2.6)][:nmat]
    L = n[0] * dx
    return dict(ndim=ndim, n=n, dx=[dx] * ndim, cfl=0.95, nsteps=10, transverse_bc="periodic",
                # gaps far above the fields the deposit makes: nothing ionizes
                materials=mats,
                layers=[(m, m * L / nmat, (m + 1) * L / nmat) for m in range(nmat)],
                ppc=2, T_K=300.0, shape_order=2, keldysh_terms=500, seed=21,
                laser=dict(lambda_m=W.LAMBDA, fwhm_s=W.cycles(2), peak_Wcm2=1e10, envelope="gauss",
                           pol_axis=1), particle_capacity=0, preionize_eV=0.0, collisions=True)


@pytest.mark.parametrize("ndim,n,npart,nmat", [(1, [48], 1500, 2), (2, [16, 8], 3000, 2), (3, [12, 6, 4], 3000, 2),
                                               (2, [16, 8], 3000, 3)])
def test_collisions_one_step_match_oracle(P, ndim, n, npart, nmat):
    """nmat 3: six kinds, most cells hold more than four of them."""
    cfg = _dense_cfg(ndim, n, nmat)
    st = _state_f32(W.random_state(cfg, npart, seed=300 + ndim, e_scale=1e6, u_scale=0.01, margin=3))
    ctx = P.Context(cfg)
    ctx.set_resort(0)
    ctx.set_state(0, st["E"], st["b"], _records(P, st, ndim))
    ctx.step(1)
    parts = ctx.particles()
    sim = OP.Sim(cfg)
    _to_oracle_state(sim, st)
    sim.step()
    # the dense plasma's own current may ionize a few neutrals (1D): same events,
    # and the births collide too
    assert set(map(tuple, ctx.events().tolist())) == sim.event_set()
    assert len(parts) == len(sim.px)
    npre = len(st["kind"])
    pos_g = parts["cell"][:, :ndim] + parts["off"][:, :ndim].astype(np.float64)
    d = pos_g[:npre] - sim.px[:npre, :ndim]
    for k in range(1, ndim):
        d[:, k] -= n[k] * np.round(d[:, k] / n[k])
    assert np.max(np.abs(d)) < 2e-5
    umax = np.max(np.abs(sim.pu))
    # the collisions moved the momenta far beyond the push's rounding
    sim0 = OP.Sim(dict(cfg, collisions=False))
    _to_oracle_state(sim0, st)
    sim0.step()
    assert np.max(np.abs(sim0.pu[:npre] - sim.pu[:npre])) > 1e-3 * umax
    err = np.max(np.abs(parts["u"][:npre] - sim.pu[:npre]))
    assert err < 1e-5 * umax, err / umax
    assert np.array_equal(parts["kind"][:npre].astype(np.int64), sim.pk[:npre])
    if len(parts) > npre:
        # births (slots in arrival order on the device): matched by kind and position
        kg = parts["kind"][npre:].astype(np.int64)
        og = np.lexsort((pos_g[npre:, 0], kg))
        oo = np.lexsort((sim.px[npre:, 0], sim.pk[npre:]))
        assert np.array_equal(kg[og], sim.pk[npre:][oo])
        assert np.max(np.abs(parts["u"][npre:][og] - sim.pu[npre:][oo])) < 1e-5 * umax
    ctx.close()


def test_collisions_independent_of_the_tile_sort(P):
    """The tile sort reorders the slots and pushes the sorted particles through
    LDS windows: after one step the same particles (matched by kind and
    position) carry the same momenta to FP32 rounding (the pairing follows
    ids and kinds, not slots)."""
    from test_gpu_parity import _match_particles
    cfg = _dense_cfg(2, [16, 8])
    st = _state_f32(W.random_state(cfg, 3000, seed=311, e_scale=1e6, u_scale=0.01, margin=3))
    out = []
    for resort in (0, 1):
        ctx = P.Context(cfg)
        ctx.set_resort(resort)
        ctx.set_state(0, st["E"], st["b"], _records(P, st, 2))
        ctx.step(1)
        p = ctx.particles()
        out.append((p["cell"][:, :2] + p["off"][:, :2].astype(np.float64), p["u"].astype(np.float64),
                    p["kind"].astype(np.int64)))
        ctx.close()
    (pa, ua, ka), (pb, ub, kb) = out
    assert len(ka) == len(kb)
    pb_m, ub_m, kb_m = _match_particles(pb, ub, kb, pa, ka, [None, 8])
    assert np.array_equal(kb_m, ka)
    assert np.max(np.abs(pb_m - pa)) < 1e-5
    umax = np.max(np.abs(ua))
    assert np.max(np.abs(ub_m - ua)) < 1e-5 * umax


def _oracle_l2(a, b):
    num = den = 0.0
    for w in "Eb":
        for c in range(3):
            x, y = a.interior_field(w, c), b.interior_field(w, c)
            num += np.sum((x - y) ** 2)
            den += np.sum(x ** 2)
    return (num / den) ** 0.5


def test_collisions_run_1d_slab(P):
    """A 1D slab run at 1e14 W/cm^2 with collisions.  Pairing is per cell, so a
    particle that crosses a cell face one step earlier in one run than in
    another meets other partners: the runs then separate at O(1) in the
    colliding particles, and the oracle itself does so under a 2e-7 change
    of the laser intensity (field L2 3e-6 at step 800, 0.1 at 1000, 0.5 at
    1400).  So: strict parity at step 800 (ionization and collisions under
    way), and at step 1400 the GPU run within the oracle's own spread."""
    from test_gpu_parity import _field_l2
    cfg = W.config_1d(hi=True, ppc=10, nsteps=1400)
    cfg["collisions"] = True
    ctx, sim = _run_both(P, cfg, 800)
    assert len(sim.pk) > 0
    _compare_run(P, ctx, sim, min_events=5, name="run_1d_collisions_800")
    ctx.step(600)
    sim.run(600)
    spread = []
    for f in (1 + 2e-7, 1 - 2e-7):
        c2 = dict(cfg, laser=dict(cfg["laser"], peak_Wcm2=cfg["laser"]["peak_Wcm2"] * f))
        s2 = OP.Sim(c2)
        s2.run(1400)
        spread.append((_oracle_l2(sim, s2), s2.kinetic_energy("e"), len(s2.event_set())))
    l2 = _field_l2(ctx, sim)
    sc = ctx.scalars()
    l2_spread = max(x[0] for x in spread)
    ke_o = sim.kinetic_energy("e")
    ke_spread = max(abs(x[1] - ke_o) for x in spread)
    ev_spread = max(abs(x[2] - len(sim.event_set())) for x in spread)
    from test_gpu_parity import _record
    _record("run_1d_collisions_1400", field_l2=l2, oracle_spread_l2=l2_spread, ke_e_gpu=sc["ke_e"],
            ke_e_oracle=ke_o, ke_spread=ke_spread, events_gpu=int(sc["events"]), events_oracle=len(sim.event_set()))
    assert l2_spread > 1e-3            # the oracle's own sensitivity is real
    assert l2 <= 3 * l2_spread
    assert abs(sc["ke_e"] - ke_o) <= 3 * ke_spread + 0.02 * ke_o
    assert abs(sc["events"] - len(sim.event_set())) <= 3 * ev_spread + 2
    assert sc["gauss_max"] <= 1e-4 * max(sc["rho_max"], 1.0)
    ctx.close()
