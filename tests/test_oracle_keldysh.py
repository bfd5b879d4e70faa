"""Pins of the oracle's Keldysh rate (paper Sec. 2.1, Eq. 1-3) to things other
than itself: library special functions, the Legendre relation, the Dawson ODE,
the multiphoton and tunneling limits of the formula, the truncation bound of
the series, the continuity of the rate across channel closings, and the
values the paper prints (Keldysh parameter range, Sec. 2.1; ponderomotive
energies, Sec. 5)."""

import numpy as np
import pytest
import scipy.special as sp

import workloads as W
from oracle import keldysh as K
from oracle.problem import Problem
from oracle.constants import C, QE, ME, HBAR, EPS0

LAM = 800e-9
GAP = 9.0
MRED = 1.0 / (1.0 / 0.6 + 1.0 / 8.0)


def _A_of_gamma(g, lam=LAM, gap=GAP, mred=MRED):
    om = 2 * np.pi * C / lam
    return om * np.sqrt(mred * ME * gap * QE) / (QE * g)


def test_elliptic_against_scipy():
    small = np.geomspace(1e-14, 0.5, 400)
    m = np.concatenate([small, 1.0 - small])
    m1 = np.concatenate([1.0 - small, small])
    Kv, Ev = K.ellip_KE(m, m1)
    Kref = np.where(m < 0.5, sp.ellipk(m), sp.ellipkm1(m1))
    Eref = sp.ellipe(m)
    assert np.max(np.abs(Kv / Kref - 1)) < 4e-15
    assert np.max(np.abs(Ev / Eref - 1)) < 4e-14
    # K(0) = E(0) = pi/2; E -> 1 as m -> 1 (m = 1 itself is the AGM's singular point)
    k0, e0 = K.ellip_KE(np.array([0.0]), np.array([1.0]))
    assert abs(k0[0] - np.pi / 2) < 1e-15 and abs(e0[0] - np.pi / 2) < 1e-15
    _, e1 = K.ellip_KE(np.array([1.0 - 1e-15]), np.array([1e-15]))
    assert abs(e1[0] - 1.0) < 1e-13


def test_legendre_relation():
    g = np.geomspace(1e-3, 1e3, 300)
    g1 = g * g / (1 + g * g)
    g2 = 1 / (1 + g * g)
    K1, E1 = K.ellip_KE(g1, g2)
    K2, E2 = K.ellip_KE(g2, g1)
    res = E1 * K2 + E2 * K1 - K1 * K2 - np.pi / 2
    assert np.max(np.abs(res)) < 2e-14


def test_dawson_against_scipy_and_ode():
    z = np.concatenate([np.linspace(-4, 4, 1001)[np.abs(np.linspace(-4, 4, 1001)) > 0],
                        np.geomspace(1e-8, 60, 3000)])
    F = K.dawson(z)
    assert np.max(np.abs(F / sp.dawsn(z) - 1)) < 5e-14
    # F' = 1 - 2 z F  (central differences)
    zz = np.linspace(0.05, 8, 200)
    h = 1e-5
    dF = (K.dawson(zz + h) - K.dawson(zz - h)) / (2 * h)
    assert np.max(np.abs(dF - (1 - 2 * zz * K.dawson(zz)))) < 1e-9
    # limits: F ~ z (z -> 0), F ~ 1/(2z) (z -> inf)
    assert abs(K.dawson(np.array([1e-9]))[0] / 1e-9 - 1) < 1e-15
    big = np.array([1e4])
    assert abs(K.dawson(big)[0] * 2 * big[0] - 1) < 1e-8


def _w_multiphoton(A, lam=LAM, gap=GAP, mred=MRED):
    """Keldysh's multiphoton limit (gamma >> 1) of Eq. 2-3: the x of Eq. 1 tends
    to (Delta + e^2 A^2 / (4 m* w^2)) / hbar w and kappa(gamma1) ~ ln(4/sqrt(gamma2))."""
    om = 2 * np.pi * C / lam
    Dl = gap * QE
    ms = mred * ME
    xt = (Dl + QE ** 2 * A ** 2 / (4 * ms * om ** 2)) / (HBAR * om)
    N = np.floor(xt) + 1
    return (2 * (2 * om / (9 * np.pi)) * (ms * om / HBAR) ** 1.5 * sp.dawsn(np.sqrt(2 * (N - xt)))
            * np.exp(2 * N) * (QE ** 2 * A ** 2 / (16 * ms * om ** 2 * Dl)) ** N)


@pytest.mark.parametrize("gamma,tol", [(12.6, 1.6e-2), (42.0, 1.5e-3), (126.0, 1.6e-4), (400.0, 2e-5)])
def test_multiphoton_limit(gamma, tol):
    A = _A_of_gamma(gamma)
    W = K.keldysh_rate(A, GAP, MRED, LAM)[0]
    r = W / _w_multiphoton(A)
    assert abs(r - 1) < tol


def test_tunneling_limit_exponent_and_prefactor():
    """gamma << 1: d lnW / d(1/E) -> -(pi/2) sqrt(m*) Delta^1.5 / (hbar e) and the
    prefactor ~ E^(5/2).  Long wavelength makes gamma ~ 0.01 with b/E ~ 30..60."""
    lam = 300e-6
    ms = MRED * ME
    Dl = GAP * QE
    b = (np.pi / 2) * np.sqrt(ms) * Dl ** 1.5 / (HBAR * QE)
    Es = np.linspace(b / 60, b / 30, 6)
    W = K.keldysh_rate(Es, GAP, MRED, lam, terms=400000)
    M = np.stack([-1 / Es, np.log(Es), np.ones_like(Es)], 1)
    coef = np.linalg.lstsq(M, np.log(W), rcond=None)[0]
    assert abs(coef[0] / b - 1) < 1e-3
    assert abs(coef[1] - 2.5) < 0.05


def test_truncation_bound_500_terms():
    """Tail after 500 terms <= q^500/(1-q) max(Dawson), q = exp(-alpha)."""
    for g in (0.15, 0.3, 0.6, 1.0, 3.0):
        A = _A_of_gamma(g)
        p = K.keldysh_parts(np.array([A]), GAP, MRED, LAM)
        W500 = K.keldysh_rate(A, GAP, MRED, LAM, terms=500)[0]
        Wall = K.keldysh_rate(A, GAP, MRED, LAM, terms=200000)[0]
        q = np.exp(-p["alpha"][0])
        n = np.arange(0, 500)
        arg = np.sqrt(p["beta"][0] * (p["N"][0] - p["x"][0] + n))
        S = np.sum(q ** n * sp.dawsn(arg))
        bound = q ** 500 / (1 - q) * 0.5410442246 / S
        assert (Wall - W500) / Wall <= bound * (1 + 1e-9) + 1e-15


def test_continuous_across_channel_closings():
    """With the series summed to convergence, W is continuous where floor(x+1)
    steps (the n = 0 Dawson term vanishes there and the rest re-indexes); a wrong
    index or sign in Eq. 2-3 breaks this."""
    from scipy.optimize import brentq
    for k_int in (7, 8, 9, 10):
        f = lambda A: K.keldysh_parts(np.array([A]), GAP, MRED, LAM)["x"][0] - k_int
        lo, hi = 1e8, 2e11
        if f(lo) > 0 or f(hi) < 0:
            continue
        Ak = brentq(f, lo, hi, xtol=1e-3, rtol=1e-15)
        eps = 1e-9 * Ak
        Wm = K.keldysh_rate(Ak - eps, GAP, MRED, LAM, terms=100000)[0]
        Wp = K.keldysh_rate(Ak + eps, GAP, MRED, LAM, terms=100000)[0]
        assert abs(Wp / Wm - 1) < 1e-3


def test_paper_gamma_range_and_ponderomotive():
    """Sec. 2.1: gamma ~ 0.3..0.9 at the paper's peak fields; Sec. 5: U_p ~ 10 eV
    (m_e* = 0.6) and ~5.5 eV (m_e* = 1.09) at 1e14 W/cm^2 and 800 nm."""
    assert abs(K.ponderomotive_eV(1e14, 0.6, LAM) / 10.0 - 1) < 0.01
    assert abs(K.ponderomotive_eV(1e14, 1.09, LAM) / 5.5 - 1) < 0.01
    E0 = np.sqrt(2 * 1e14 * 1e4 / (C * EPS0))
    Et = 2 / (1 + 1.477) * E0            # transmitted into Table-1 silica
    g = K.keldysh_parts(np.array([Et]), 9.0, MRED, LAM)["gamma"][0]
    assert 0.3 <= g <= 0.9


def test_rate_increases_with_field_between_closings():
    A = np.geomspace(3e9, 4e10, 400)
    W = K.keldysh_rate(A, GAP, MRED, LAM)
    assert np.all(np.isfinite(W)) and np.all(W > 0)
    # steep growth over one decade of field: between A^4 (tunneling side) and
    # A^(2N) with N ~ 7 (multiphoton side)
    assert 1e4 < W[-1] / W[0] < 1e14


@pytest.mark.parametrize("bits", [4, 8, 16, 30])
def test_series_tolerance_bound(bits):
    """The series stopped at tolerance 2^-bits: the terms are positive, so the
    stopped sum is at most the full one and, by the tail bound, within 2^-bits of
    it; coarser tolerances never sum more terms; at 4 bits the stop bites."""
    mt = Problem(W.config_2d()).mats[0]
    lam = W.LAMBDA
    A = np.geomspace(3e8, 3e11, 400)                  # gamma from ~0.1 to ~100
    full = K.keldysh_rate(A, mt.gap_eV, mt.mred, lam, tol_bits=60)
    cut = K.keldysh_rate(A, mt.gap_eV, mt.mred, lam, tol_bits=bits)
    assert np.all(cut <= full * (1 + 1e-15))
    assert np.all((full - cut) / full <= 2.0 ** -bits)
    coarser = K.keldysh_rate(A, mt.gap_eV, mt.mred, lam, tol_bits=max(1, bits // 2))
    assert np.all(coarser <= cut * (1 + 1e-15))
    if bits == 4:
        assert np.max((full - cut) / full) > 1e-6
