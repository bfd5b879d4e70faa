"""Pins of the oracle's Kerr term (the nonlinear extension of the linear
optics of Sec. 2.3, which the paper leaves out): per E component the
displacement gains chi3 E^3, chi3 = (4/3) n0^2 eps0 c n2.

* a standing wave E0 cos(kx) in a periodic Kerr box oscillates slower than in
  the linear medium by the harmonic-balance shift: the fundamental of E^3
  carries (3/4)(3/4) E0^2 (space and time), so eps_eff = eps + (9/16) chi3
  E0^2, and the discrete Yee relation sin^2(w dt/2) = S^2 / eps_eff gives
  dw/w = -(tan t / t) d/2 with t = w dt/2, d = (9/16) chi3 E0^2 / eps; the
  shift grows as E0^2 (the phase-matched third harmonic of a dispersionless
  medium limits the comparison to a few periods: 5 %);
* chi3 from n2: a material with n2 = 0 is the linear medium bit for bit;
* the Gauss law with the Kerr displacement through a run with births."""

import math

import numpy as np

import workloads as W
from oracle import pic
from oracle.constants import C, EPS0


def _box(n2, n=64):
    mat = dict(W.silica_like(), kerr_n2_m2W=n2)
    dx = W.LAMBDA / 40
    cfg = dict(ndim=1, n=[n], dx=[dx], cfl=0.95, nsteps=10, transverse_bc="outflow", materials=[mat],
               layers=[(0, -1.0, 1.0)], ppc=1, T_K=300.0, shape_order=2, keldysh_terms=500, seed=1,
               laser=dict(lambda_m=W.LAMBDA, fwhm_s=W.cycles(2), peak_Wcm2=1e10, envelope="gauss",
                          pol_axis=1), particle_capacity=0, preionize_eV=0.0, periodic_x=True)
    return pic.Sim(cfg, load_neutrals=False)


def _omega(n2, E0, k=3, n=64, steps=100):
    s = _box(n2, n)
    x = np.arange(s.S[0]) - pic.G
    ph = 2 * np.pi * k * x / n
    s.E[1][:, 0, 0] = E0 * np.cos(ph)
    dom = s._domain_slices(s.stE[1])
    basis = np.cos(ph)[dom[0]]
    a = []
    for st in range(steps):
        a.append(np.sum(s.E[1][dom][:, 0, 0] * basis))
        s._b_half()
        s._e_full(st)
        s._b_half()
    a = np.array(a)
    lhs, rhs = a[2:] + a[:-2], 2 * a[1:-1]
    return math.acos(np.dot(lhs, rhs) / np.dot(rhs, rhs)) / s.P.dt, s


def _n2_for(chiE2, E0):
    return chiE2 / E0 ** 2 / (4.0 / 3.0 * 1.45 ** 2 * EPS0 * C)


def test_chi3_from_n2():
    s = _box(2.5e-20)
    want = 4.0 / 3.0 * 1.45 ** 2 * EPS0 * C * 2.5e-20
    assert abs(s.P.mats[0].chi3 / want - 1) < 1e-7


def test_standing_wave_frequency_shift():
    E0 = 1e9
    w0, s0 = _omega(0.0, E0)
    ie = s0.P.mats[0].ie
    S2 = s0.P.Cd[0] ** 2 * math.sin(math.pi * 3 / 64) ** 2
    th = math.asin(math.sqrt(S2 * ie))
    shifts = []
    for c2 in (5e-4, 1e-3):
        w1, s1 = _omega(_n2_for(c2, E0), E0)
        chi = s1.P.mats[0].chi3
        d = (9.0 / 16.0) * chi * E0 ** 2 * ie
        pred = -(math.tan(th) / th) * d / 2
        meas = (w1 - w0) / w0
        shifts.append(meas)
        assert meas < 0
        assert abs(meas / pred - 1) < 0.05, (c2, meas / pred)
    # the shift scales as E0^2 (here as chi3: twice chi3, twice the shift)
    assert abs(shifts[1] / shifts[0] - 2) < 0.1
    # the linear medium: n2 = 0 is the plain update bit for bit
    s_lin = _box(0.0)
    assert s_lin.P.mats[0].chi3 == 0.0


def test_gauss_law_with_kerr_displacement():
    """2D Gaussian beam into a Kerr slab with ionization: div(E/ie + chi3 E^3)
    = rho/eps0 to roundoff; leaving the Kerr term out of the displacement
    breaks it (the beam's E_y varies along y)."""
    cfg = W.config_2d(nx=192, ny=48, nsteps=500, ppc=2, peak=3e14, slab_cells=12, waist=0.6e-6)
    cfg["materials"] = [dict(cfg["materials"][0], kerr_n2_m2W=2.5e-20)]
    s = pic.Sim(cfg)
    s.run(500)
    assert sum(len(e[0]) for e in s.events) > 5
    rho = s.charge_density()
    tol = 1e-11 * np.max(np.abs(rho))
    assert np.max(np.abs(s.gauss_residual())) < tol
    chi = s.chiE
    s.chiE = [np.zeros_like(c) for c in chi]
    assert np.max(np.abs(s.gauss_residual())) > 1e3 * tol
    s.chiE = chi
