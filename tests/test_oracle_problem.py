"""Pins of the oracle's problem definition: the CFL time step (Sec. 3.1), the
FP32 canonical coefficients, the pulse energy/intensity relations (Sec. 3,
Sec. 5), the layer thicknesses printed for the mirror (Fig. 1)."""

import math

import numpy as np

import workloads as W
from oracle.problem import Problem, Laser
from oracle.constants import C, EPS0, QE, ME


def test_cfl_time_step_and_fp32_coefficients():
    for cfg in (W.config_1d(), W.config_2d(), W.config_3d()):
        P = Problem(cfg)
        s = math.sqrt(sum(1.0 / dx ** 2 for dx in cfg["dx"]))
        dt_paper = 0.95 / (C * s)
        assert P.dt <= dt_paper and P.dt > dt_paper * (1 - 2 ** -22)
        for d in range(P.D):
            assert float(np.float32(P.Cd[d])) == P.Cd[d]
            assert abs(P.Cd[d] - C * P.dt / P.dx[d]) <= 2 ** -23 * P.Cd[d]
            assert float(np.float32(P.kmur[d])) == P.kmur[d]
        for m in P.mats:
            assert float(np.float32(m.ie)) == m.ie
            assert abs(m.ie * m.n_index ** 2 - 1) < 2 ** -23


def test_window_length_is_one_cycle():
    P = Problem(W.config_1d())
    assert P.nwin == 43                          # 800 nm / (0.95 * 20 nm) -> 42.1 steps
    P2 = Problem(W.config_2d())
    assert P2.nwin == 48


def test_mirror_layer_thicknesses_fig1():
    """Fig. 1: top SiO2 270.90 nm = lambda/2n, HfO2 98.95 nm and SiO2 135.45 nm =
    lambda/4n, with the indices those printed values imply."""
    L = W.layer_stack([0, 1, 0], [1.4766, 2.0212, 1.4766], 0.0, first_half_wave=True)
    th = [(hi - lo) * 1e9 for (_, lo, hi) in L]
    for got, want in zip(th, (270.90, 98.95, 135.45)):
        assert abs(got / want - 1) < 5e-4


def test_fluence_intensity_and_ponderomotive():
    # 7 fs sine-squared at 0.7 J/cm^2 (Sec. 5) -> peak close to 1e14 W/cm^2 (Sec. 5)
    L = Laser(dict(lambda_m=800e-9, fwhm_s=7e-15, fluence_Jcm2=0.7, envelope="sin2"))
    assert 0.9e14 < L.I0 / 1e4 < 1.05e14
    # sin^2 field envelope: intensity FWHM tau -> full length T = 2.745 tau
    assert abs(L.T / 7e-15 - 2.745) < 3e-3
    # the envelope's intensity FWHM is tau
    t = np.linspace(0, L.T, 200001)
    I = L.env(t) ** 2
    above = t[I >= 0.5]
    assert abs((above[-1] - above[0]) / 7e-15 - 1) < 1e-4
    # integral of the intensity envelope equals the fluence / I0 relation
    assert abs(np.trapezoid(I, t) / L.env2_integral - 1) < 1e-6
    # U_p at 1e14 W/cm^2 from this laser's E0 (Sec. 5: ~10 eV and ~5.5 eV)
    L2 = Laser(dict(lambda_m=800e-9, fwhm_s=7e-15, peak_Wcm2=1e14, envelope="sin2"))
    for mstar, up in ((0.6, 10.0), (1.09, 5.5)):
        Up = QE ** 2 * L2.E0 ** 2 / (4 * mstar * ME * L2.omega ** 2) / QE
        assert abs(Up / up - 1) < 0.01
    # Gaussian: intensity FWHM and integral
    Lg = Laser(dict(lambda_m=800e-9, fwhm_s=5e-15, peak_Wcm2=1e13, envelope="gauss"))
    t = np.linspace(0, 2 * Lg.t0, 400001)
    I = Lg.env(t) ** 2
    above = t[I >= 0.5]
    assert abs((above[-1] - above[0]) / 5e-15 - 1) < 1e-4
    assert abs(np.trapezoid(I, t) / Lg.env2_integral - 1) < 1e-6
    assert abs(0.5 * C * EPS0 * Lg.E0 ** 2 / 1e17 - 1) < 1e-12


def test_materials_table1():
    P = Problem(dict(W.config_1d(), materials=[W.table1_sio2(), W.table1_hfo2()]))
    s, h = P.mats
    assert abs(s.mred - 1 / (1 / 0.6 + 1 / 8)) < 1e-15
    assert abs(h.mred - 1 / (1 / 1.09 + 1 / 1.12)) < 1e-15
    # molecular densities (2.2 g/cc, 60.08 g/mol; 9.68 g/cc, 210.49 g/mol)
    assert abs(s.n0 / 2.205e28 - 1) < 2e-3
    assert abs(h.n0 / 2.769e28 - 1) < 2e-3
