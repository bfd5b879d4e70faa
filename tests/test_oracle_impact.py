"""Pins of the oracle's impact ionization (Keldysh's impact rate, the paper's
future work, Sec. 2.2) to closed forms, statistics and brute force.

* the threshold E_g (1 + 2 mu)/(1 + mu): E_g for an infinitely heavy hole,
  3/2 E_g for equal masses;
* the rate P (eps/E_th - 1)^2: zero at and below the threshold, P at 2 E_th,
  quadrupled at 3 E_th;
* the event frequency of electrons at one energy against 1 - exp(-w dt)
  (binomial, 5 sigma);
* the energy balance: an impacting electron loses exactly the gap;
* each cell's neutrals consumed lowest index first, never twice, none left
  means no event; births at the neutrals' positions, events recorded;
* only electrons in cells of their own material ionize; the result does not
  depend on the order in which the particles are stored."""

import math

import numpy as np

import workloads as W
from oracle import impact as IM
from oracle import pic
from oracle.constants import C, QE
from oracle.problem import Material


def _mat(**kw):
    return Material(dict(W.silica_like(), **kw))


def test_threshold_limits():
    assert abs(IM.threshold_eV(_mat(me_star=1.0, mh_star=1e12)) - 9.0) < 1e-9
    assert abs(IM.threshold_eV(_mat(me_star=0.7, mh_star=0.7)) - 13.5) < 1e-12
    # the benchmark material (m_e* 0.6, m_h* 8): mu = 0.075
    assert abs(IM.threshold_eV(_mat(me_star=0.6, mh_star=8.0)) - 9.0 * 1.15 / 1.075) < 1e-12


def test_rate_shape():
    m = _mat(impact_rate_s=2e15)
    eth = IM.threshold_eV(m)
    assert IM.rate(m, 0.5 * eth) == 0.0 and IM.rate(m, eth) == 0.0
    assert abs(IM.rate(m, 2 * eth) / 2e15 - 1) < 1e-14
    assert abs(IM.rate(m, 3 * eth) / 8e15 - 1) < 1e-14
    assert IM.rate(_mat(), 3 * eth) == 0.0     # rate constant 0: off


def _box(ppc, rate_s, n=64):
    cfg = W.config_1d(n=n, ppc=ppc, nsteps=10)
    dx = cfg["dx"][0]
    cfg["materials"] = [W.with_impact(W.silica_like(), rate_s), W.high_index()]
    cfg["layers"] = [(0, 0.0, 0.75 * n * dx), (1, 0.75 * n * dx, n * dx)]
    return pic.Sim(cfg)


def _place(s, cells, kinds, eps_eV, rng):
    """Electrons (or carriers) in given cells with kinetic energy eps_eV, random directions."""
    m = np.array([s.P.kinds[k]["mass"] for k in kinds])
    g = 1.0 + eps_eV * QE / (m * C * C)
    umag = np.sqrt(g * g - 1.0)
    d = rng.normal(size=(len(cells), 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    s.px = np.column_stack([np.asarray(cells) + rng.uniform(0.05, 0.95, len(cells)), np.zeros((len(cells), 2))])
    s.pu = d * umag[:, None]
    s.pk = np.asarray(kinds, dtype=np.int64)
    s.pid = np.zeros(0, dtype=np.int64)
    s._ensure_ids()


def _ke(s, i):
    k = s.pk[i]
    return (math.sqrt(1 + float(np.dot(s.pu[i], s.pu[i]))) - 1) * s.P.kinds[k]["mass"] * C * C


def test_event_frequency_and_energy_balance():
    rng = np.random.default_rng(5)
    s0 = _box(64, 1.0)
    eth = IM.threshold_eV(s0.P.mats[0])
    eps = 2.0 * eth
    p_target = 0.3
    rate_s = -math.log(1 - p_target) / s0.P.dt       # w(2 E_th) = rate_s
    s = _box(64, rate_s)
    N = 40 * 40
    cells = np.repeat(np.arange(40), 40)              # material-0 cells 0..39, 40 electrons each
    _place(s, cells, [0] * N, eps, rng)
    ke0 = np.array([_ke(s, i) for i in range(N)])
    u0 = s.pu.copy()
    IM.impact(s, 7)
    ev = s.events[-1][0] if s.events else np.zeros(0)
    n_ev = len(ev)
    assert abs(n_ev - p_target * N) < 5 * math.sqrt(N * p_target * (1 - p_target))
    # every impacting electron lost exactly the gap; the others are untouched
    ke1 = np.array([_ke(s, i) for i in range(N)])
    hit = ke1 < ke0 * (1 - 1e-9)
    assert hit.sum() == n_ev
    assert np.max(np.abs((ke0 - ke1)[hit] / (9.0 * QE) - 1)) < 1e-9
    assert np.array_equal(s.pu[:N][~hit], u0[~hit])
    # directions kept
    cosang = np.sum(s.pu[:N][hit] * u0[hit], axis=1) / (np.linalg.norm(s.pu[:N][hit], axis=1) *
                                                       np.linalg.norm(u0[hit], axis=1))
    assert np.min(cosang) > 1 - 1e-12
    # births: two per event at the consumed neutrals' positions, gap energy paid
    assert len(s.pk) == N + 2 * n_ev
    assert abs(s.energy_gap - n_ev * s.P.kinds[0]["weight"] * 9.0 * QE) <= 1e-12 * s.energy_gap


def test_neutrals_lowest_index_first_and_at_most_once():
    rng = np.random.default_rng(6)
    s = _box(3, 1e22)                                 # every hot electron decides "yes"
    eth = IM.threshold_eV(s.P.mats[0])
    cells = [5] * 5 + [9]
    kinds = [0] * 5 + [1]                             # a positive carrier never ionizes
    _place(s, cells, kinds, 3 * eth, rng)
    IM.impact(s, 4)
    ids = np.sort(s.events[-1][0])
    assert list(ids) == [5 * 3 + 0, 5 * 3 + 1, 5 * 3 + 2]     # cell 5's three neutrals, once each
    dead = np.nonzero(~s.nalive)[0]
    assert sorted(s.nid[dead].tolist()) == list(ids) and np.all(s.ndeath[dead] == 4)
    assert len(s.pk) == 6 + 6
    bpos = s.px[6:]
    want = s.npos[np.searchsorted(s.nid, np.concatenate([ids, ids]))]
    assert np.array_equal(np.sort(bpos[:, 0]), np.sort(want[:, 0]))
    # a second step: no neutral left in cell 5, nothing happens
    n_before = len(s.pk)
    IM.impact(s, 5)
    assert len(s.pk) == n_before


def test_only_own_material_and_order_independence():
    rng = np.random.default_rng(7)
    s = _box(8, 1e22)
    eth = IM.threshold_eV(s.P.mats[0])
    # cells 3 (material 0) and 60 (material 1: no impact rate there); kind 2 is
    # material 1's electron sitting in material 0's cell 3
    cells = [3, 3, 3, 60, 60, 3]
    kinds = [0, 0, 0, 0, 2, 2]
    _place(s, cells, kinds, 4 * eth, rng)
    s_copy = (s.px.copy(), s.pu.copy(), s.pk.copy(), s.pid.copy())
    IM.impact(s, 2)
    assert sorted(s.events[-1][0].tolist()) == [24, 25, 26]
    # the same particles stored in another order
    t = _box(8, 1e22)
    perm = rng.permutation(len(cells))
    t.px, t.pu, t.pk, t.pid = (a[perm] for a in s_copy)
    IM.impact(t, 2)
    back = np.empty_like(perm)
    back[perm] = np.arange(len(perm))
    assert np.array_equal(t.pu[:6][back], s.pu[:6])
    assert sorted(t.events[-1][0].tolist()) == [24, 25, 26]


def test_run_with_impact_keeps_gauss_law(monkeypatch):
    """A 1D slab at 3e14 W/cm^2 with impact ionization: some events come from
    impacts, and the Gauss law holds through every birth."""
    cfg = W.config_1d(hi=True, ppc=4, n=512, nsteps=1100, peak=3e14)
    cfg["materials"] = [W.with_impact(cfg["materials"][0], 1e16)]
    s = pic.Sim(cfg)
    real = IM.impact
    n_imp = [0]

    def spy(sim, step):
        n0 = len(sim.events)
        real(sim, step)
        n_imp[0] += sum(len(e[0]) for e in sim.events[n0:])

    monkeypatch.setattr(IM, "impact", spy)
    s.run(1100)
    assert n_imp[0] > 0
    assert sum(len(e[0]) for e in s.events) > n_imp[0]
    rho = s.charge_density()
    assert np.max(np.abs(s.gauss_residual())) < 1e-11 * np.max(np.abs(rho))
    ids = np.concatenate([e[0] for e in s.events])
    assert len(np.unique(ids)) == len(ids)
