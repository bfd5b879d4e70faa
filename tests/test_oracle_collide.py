"""Pins of the oracle's binary collisions (Sec. 2.2, Eq. 4) to conservation
laws, Nanbu's angular law, the rate of Eq. (4), and brute-force bookkeeping.

* every collision conserves the pair's momentum and energy (relativistic);
* the mean deflection cosine is exp(-s) (Nanbu's defining relation), which
  Perez's fit of A(s) and the small- and large-s branches must reproduce;
* a slow electron scattering off a very heavy partner at rest loses its
  forward momentum at the rate nu of Eq. (4): <cos chi> = exp(-nu dt);
* the Coulomb logarithm follows the scalings of its parts (Debye length
  ~ sqrt(T / n), classical distance ~ 1/v^2, quantum ~ 1/v) and is >= 1;
* pairing: each particle's number of collisions per step, half-strength
  collisions for an odd count, the result independent of the order in which
  the particles are stored;
* Nanbu and Yonemura's weight rule updates the heavier-weight particle of an
  unlike pair with probability w_light / w_heavy.
The low-temperature cap's constant is not pinned (only that it bounds s)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import collide as CO
from oracle import pic
from oracle.constants import C, EPS0, ME, QE


def _energy_momentum(u, m):
    g = math.sqrt(1 + float(np.dot(u, u)))
    return g * m * C * C, m * C * np.asarray(u)


@pytest.mark.parametrize("s_scale", [1e-3, 1.0, 1e3])
def test_collision_conserves_momentum_and_energy(s_scale):
    rng = np.random.default_rng(3)
    for _ in range(200):
        m1, m2 = ME * rng.uniform(0.5, 2), ME * 10 ** rng.uniform(0, 5)
        u1, u2 = rng.normal(0, 0.5, 3), rng.normal(0, 0.05, 3)
        words = rng.integers(0, 2 ** 32, 3)
        n = 1e27 * s_scale
        n1, n2 = CO.collide_pair(u1, u2, m1, m2, -QE, QE, 1.0, 1.0, n, 1e-16,
                                 lambda mu, v: 2.0, lambda v: math.inf, False, words)
        E0 = _energy_momentum(u1, m1)[0] + _energy_momentum(u2, m2)[0]
        P0 = _energy_momentum(u1, m1)[1] + _energy_momentum(u2, m2)[1]
        E1 = _energy_momentum(n1, m1)[0] + _energy_momentum(n2, m2)[0]
        P1 = _energy_momentum(n1, m1)[1] + _energy_momentum(n2, m2)[1]
        scale = np.linalg.norm(m1 * C * u1) + np.linalg.norm(m2 * C * u2)
        assert abs(E1 - E0) <= 1e-12 * E0
        assert np.max(np.abs(P1 - P0)) <= 1e-12 * scale
        assert not np.array_equal(n1, u1)


@pytest.mark.parametrize("s", [0.01, 0.05, 0.15, 0.5, 1.0, 2.0, 2.9, 3.5, 5.0, 8.0])
def test_mean_deflection_is_exp_minus_s(s):
    """<cos chi> over U uniform (midpoint rule on 2e5 points) against exp(-s):
    Nanbu's relation coth A - 1/A = exp(-s).  The small-angle branch is exact
    to O(s^2) (its mean is 1 - s), the fit to 3e-3, the large-s branches to
    the size of exp(-s) they drop."""
    N = 200000
    U = (np.arange(N) + 0.5) / N
    mean = np.mean([CO.cos_chi(s, x) for x in U])
    if s < 0.1:
        assert abs(mean - (1 - s)) < 1e-4
        assert abs(mean - math.exp(-s)) < s * s / 2 + 1e-4
    elif s < 3:
        assert abs(mean - math.exp(-s)) < 3e-3
    elif s < 6:
        assert abs(mean - math.exp(-s)) < 1e-3
    else:
        assert abs(mean) < 1e-4 and math.exp(-s) < 3e-3
    # a wrong branch (the isotropic law, or no scattering) would miss it widely
    assert abs(mean - math.exp(-s)) < 0.2 * max(math.exp(-s), 1 - math.exp(-s))


@pytest.mark.parametrize("s_target", [0.04, 0.6])
def test_slowing_down_rate_is_eq4(s_target):
    """An electron at 0.01 c against a partner 1e6 times heavier at rest: the
    forward momentum after one collision, averaged over the deflection draw,
    is exp(-nu dt) of its start, nu from Eq. (4) with the reduced mass."""
    M = 1e6 * ME
    v = 0.01 * C
    u1 = np.array([v / C / math.sqrt(1 - 0.01 ** 2), 0.0, 0.0])
    u2 = np.zeros(3)
    lnL, n = 5.0, 1e27
    mu = ME * M / (ME + M)
    nu = (QE * QE) ** 2 * n * lnL / (4 * math.pi * (EPS0 * mu) ** 2) / v ** 3
    dt = s_target / nu
    K = 4000
    ux = []
    for k in range(K):
        words = [int((k + 0.5) / K * 2 ** 32), int(k * 2654435761 % 2 ** 32), 0]
        n1, _ = CO.collide_pair(u1, u2, ME, M, -QE, QE, 1.0, 1.0, n, dt, lambda m, vr: lnL,
                                lambda vr: math.inf, False, words)
        ux.append(n1[0] / u1[0])
    mean = float(np.mean(ux))
    assert abs(mean - math.exp(-nu * dt)) < 3e-3
    # twice the rate (a dropped factor 2, or mu -> m/2) is far outside
    assert abs(mean - math.exp(-2 * nu * dt)) > 5e-3


def _cell_sim(parts, cfg_extra=None, ndim=1):
    """A 1D box with particles placed in given cells (collisions on, fields
    zero); parts: list of (cell, kind, u)."""
    cfg = W.config_1d(n=16, ppc=4, nsteps=10)
    cfg["materials"] = [W.silica_like(), dict(W.silica_like(), density_gcc=3 * 2.2)]
    cfg["layers"] = [(0, 0, 8 * cfg["dx"][0]), (1, 8 * cfg["dx"][0], 16 * cfg["dx"][0])]
    cfg["collisions"] = True
    if cfg_extra:
        cfg.update(cfg_extra)
    s = pic.Sim(cfg, load_neutrals=False)
    s.px = np.array([[c + 0.25 + 0.5 * (i % 2), 0, 0] for i, (c, k, u) in enumerate(parts)], dtype=float)
    s.pu = np.array([u for (c, k, u) in parts], dtype=float)
    s.pk = np.array([k for (c, k, u) in parts], dtype=np.int64)
    s._ensure_ids()
    return s


def test_pairing_counts_and_order_independence(monkeypatch):
    rng = np.random.default_rng(9)
    parts = []
    # cell 2: 5 electrons (odd: a triangle and a pair) and 2 carriers of material 0;
    # cell 5: 4 electrons; cell 7: one electron alone
    for c, k, m in ((2, 0, 5), (2, 1, 2), (5, 0, 4), (7, 0, 1)):
        parts += [(c, k, rng.normal(0, 0.01, 3)) for _ in range(m)]
    s = _cell_sim(parts)
    calls = []
    real = CO.collide_pair

    def spy(u1, u2, m1, m2, q1, q2, w1, w2, n, dt, lnL_of, cap_of, half, words):
        calls.append((id_of(u1), id_of(u2), half))
        return real(u1, u2, m1, m2, q1, q2, w1, w2, n, dt, lnL_of, cap_of, half, words)

    def id_of(u):
        return int(np.argmin(np.sum((s.pu - u) ** 2, axis=1)))

    monkeypatch.setattr(CO, "collide_pair", spy)
    u_before = s.pu.copy()
    CO.collide(s, 3)
    monkeypatch.setattr(CO, "collide_pair", real)
    # the spy identifies particles by their momentum before each call
    counts = np.zeros(len(parts), dtype=int)
    halves = np.zeros(len(parts), dtype=int)
    for i, j, h in calls:
        counts[i] += 1
        counts[j] += 1
        halves[i] += h
        halves[j] += h
    e2 = [i for i, (c, k, u) in enumerate(parts) if c == 2 and k == 0]
    p2 = [i for i, (c, k, u) in enumerate(parts) if c == 2 and k == 1]
    e5 = [i for i, (c, k, u) in enumerate(parts) if c == 5]
    # cell 2: electrons: the triangle's three 2 half collisions each, the pair's
    # two 1 full collision each; then 5 unlike collisions, one per electron,
    # spread over the 2 carriers
    assert sorted(counts[e2] - halves[e2]) == [1, 1, 1, 2, 2]
    assert sorted(halves[e2]) == [0, 0, 2, 2, 2]
    # carriers: their own pair, then the 5 unlike collisions as 3 and 2
    assert sorted(counts[p2]) == [3, 4]
    assert list(counts[e5]) == [1, 1, 1, 1]
    assert len(calls) == 3 + 1 + 1 + 5 + 2
    assert np.array_equal(s.pu[-1], u_before[-1])   # alone in its cell
    # the result does not depend on the storage order
    s2 = _cell_sim(parts)
    s2.pu = u_before.copy()
    perm = rng.permutation(len(parts))
    s2.px, s2.pu, s2.pk, s2.pid = s2.px[perm], s2.pu[perm], s2.pk[perm], s2.pid[perm]
    CO.collide(s2, 3)
    back = np.empty_like(perm)
    back[perm] = np.arange(len(perm))
    assert np.array_equal(s2.pu[back], s.pu)


def test_weight_rule_updates_heavier_weight_at_the_weight_ratio():
    """Electrons of material 0 against carriers of material 1, whose weight is
    3 x larger (3 x the density): the carrier is updated in 1/3 of the
    collisions, the electron in all."""
    rng = np.random.default_rng(4)
    parts = [(3, 0, rng.normal(0, 0.02, 3)) for _ in range(1)] + \
            [(3, 3, rng.normal(0, 0.0002, 3)) for _ in range(1)]
    s = _cell_sim(parts)
    w0, w3 = s.P.kinds[0]["weight"], s.P.kinds[3]["weight"]
    assert abs(w3 / w0 - 3) < 1e-9
    upd_e = upd_p = 0
    T = 3000
    for step in range(T):
        u0 = s.pu.copy()
        CO.collide(s, step)
        upd_e += not np.array_equal(s.pu[0], u0[0])
        upd_p += not np.array_equal(s.pu[1], u0[1])
        s.pu = u0
    assert upd_e == T
    p = 1 / 3
    assert abs(upd_p - p * T) < 5 * math.sqrt(T * p * (1 - p))


def test_coulomb_log_scalings():
    """ln(Lambda) per collision of a cell: the Debye length ~ sqrt(T/n), the
    classical distance ~ 1/v^2, the quantum one ~ 1/v, never below 1."""
    def lnL_cell(n_scale, T_scale, v):
        # one electron kind at a given density and temperature, read through the
        # function the cell builds (density from counts x weight / V)
        rng = np.random.default_rng(1)
        sig = math.sqrt(T_scale * 1e-2)
        parts = [(4, 0, rng.normal(0, sig, 3)) for _ in range(6)]
        s = _cell_sim(parts, {"ppc": int(4 / n_scale) if n_scale < 1 else 4})
        captured = {}
        real = CO.collide_pair

        def spy(u1, u2, m1, m2, q1, q2, w1, w2, n, dt, lnL_of, cap_of, half, words):
            captured["f"] = lnL_of
            return u1, u2
        CO.collide_pair = spy
        try:
            CO.collide(s, 1)
        finally:
            CO.collide_pair = real
        return captured["f"](ME / 2, v)

    v = 1e6
    # classical regime (slow, below 2 alpha c): a quarter of the density (ppc 16
    # instead of 4: the same particles at a quarter of the weight) raises
    # ln(Lambda) by ln 2
    a, b = lnL_cell(1.0, 100.0, v), lnL_cell(0.25, 100.0, v)
    assert a > 1.5
    assert abs((b - a) - math.log(2)) < 1e-9
    # classical regime: doubling v raises it by ln 4; fast (quantum): by ln 2
    assert abs(lnL_cell(1.0, 100.0, 2 * v) - a - math.log(4)) < 1e-9
    f1, f2 = lnL_cell(1.0, 100.0, 3e7), lnL_cell(1.0, 100.0, 6e7)
    assert abs(f2 - f1 - math.log(2)) < 1e-9
    assert lnL_cell(1.0, 100.0, 1.0) == 1.0


def test_collisions_keep_gauss_law_and_change_only_velocities():
    cfg = W.config_1d(hi=True, ppc=4, nsteps=900, n=512)
    cfg["collisions"] = True
    s = pic.Sim(cfg)
    s.run(900)
    assert sum(len(e[0]) for e in s.events) > 5
    rho = s.charge_density()
    assert np.max(np.abs(s.gauss_residual())) < 1e-11 * np.max(np.abs(rho))
