"""Host-side checks of the native library (no GPU compute): the C ABI exports
every symbol include/pic.h declares, the canonical discrete problem equals the
oracle's bit for bit, the C++ Keldysh rate and the FP32 rate table agree with
the oracle's in-situ FP64 evaluation (Sec. 2.1, Eq. 1-3), including both sides
of every channel closing, and invalid configurations are rejected."""

import os
import re

import numpy as np
import pytest
from scipy.optimize import brentq

import workloads as W
from oracle import keldysh as K
from oracle.problem import Problem

P = pytest.importorskip("paper_2502_13695_amd.pic")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libpic.so not built")
    return P.lib()


def test_exports_every_declared_symbol():
    import subprocess
    _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "pic.h")).read()
    declared = set(re.findall(r"\b(pic_[a-z_]+)\s*\(", hdr))
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pic_\w+)", out))
    assert declared <= exported, declared - exported
    assert set(P.SYMBOLS) == declared


@pytest.mark.parametrize("cfg", [W.config_1d(), W.config_1d(hi=True), W.config_2d(), W.config_3d(),
                                 W.batch_scan(4)[3], W.config_2d(nx=100, ny=37),
                                 W.config_1d(dispersive=True), W.config_2d(dispersive=True),
                                 W.config_3d(dispersive=True),
                                 dict(W.config_1d(), materials=[dict(W.silica_like(), kerr_n2_m2W=2.5e-20)])])
def test_canonical_problem_bitwise_equal(cfg):
    _lib_or_skip()
    p = P.canonical(cfg)
    o = Problem(cfg)
    assert p.dt == o.dt
    assert list(p.Cd)[:o.D] == o.Cd[:o.D]
    assert list(p.kmur)[:o.D] == o.kmur[:o.D]
    assert p.nwin == o.nwin
    assert [p.ie[m] for m in range(len(o.mats))] == [m.ie for m in o.mats]
    assert [tuple(p.lor[m]) for m in range(len(o.mats))] == [tuple(m.lor) for m in o.mats]
    assert [p.chi3[m] for m in range(len(o.mats))] == [m.chi3 for m in o.mats]
    assert abs(p.E0 / o.laser.E0 - 1) < 1e-15
    nmat_cells = int(np.sum(o.mat_cell >= 0)) * o.n[1] * o.n[2]
    assert p.n_neutral == nmat_cells * o.ppc


def test_lorentz_stability_check_matches_oracle():
    """pic_init's stability test of a Lorentz medium agrees with the oracle's
    (which its own test ties to the roots of the mode polynomial)."""
    _lib_or_skip()
    from oracle.problem import lorentz_stable
    seen = {True: 0, False: 0}
    for lam0 in (0.1e-6, 0.116e-6, 0.15e-6, 0.2e-6, 0.3e-6):
        for eps_inf in (1.0, 1.3, 1.7, 2.0):
            for dxfrac in (12, 20, 40):
                cfg = W.config_1d(n=64, ppc=1)
                cfg["dx"] = [W.LAMBDA / dxfrac]
                cfg["materials"] = [W.lorentz(W.silica_like(), lam0, eps_inf=eps_inf)]
                try:
                    Problem(cfg)
                    want = True
                except ValueError:
                    want = False
                try:
                    P.canonical(cfg)
                    got = True
                except P.PicError:
                    got = False
                assert got == want, (lam0, eps_inf, dxfrac)
                seen[want] += 1
    assert seen[True] > 5 and seen[False] > 5


def test_keldysh_rate_cpp_equals_oracle():
    _lib_or_skip()
    for m in (W.silica_like(), W.high_index(), W.table1_sio2(), W.table1_hfo2()):
        A = np.geomspace(1e9, 1e11, 300)
        mr = 1 / (1 / m["me_star"] + 1 / m["mh_star"])
        w1 = P.keldysh_rate(m, 800e-9, A)
        w2 = K.keldysh_rate(A, m["gap_eV"], mr, 800e-9)
        assert np.max(np.abs(w1 / w2 - 1)) < 1e-13


def _closings(mt, lam, lo, hi):
    f0 = lambda A, k: K.keldysh_parts(np.array([A]), mt.gap_eV, mt.mred, lam)["x"][0] - k
    out = []
    x_lo = K.keldysh_parts(np.array([lo]), mt.gap_eV, mt.mred, lam)["x"][0]
    x_hi = K.keldysh_parts(np.array([hi]), mt.gap_eV, mt.mred, lam)["x"][0]
    for k in range(int(np.floor(x_lo)) + 1, int(np.floor(x_hi)) + 1):
        out.append(brentq(lambda A: f0(A, k), lo, hi, xtol=1e-6, rtol=1e-15))
    return out


@pytest.mark.parametrize("cfg", [W.config_2d(), W.config_3d(), dict(W.config_2d(), keldysh_tol_bits=12)],
                         ids=["2d", "3d", "2d_tol12"])
def test_rate_table_against_insitu_fp64(cfg):
    """P(A) from the FP32 table vs 1 - exp(-W dt/n0) in FP64 at the same FP32 A,
    over [A_cut, A_sat] and at the FP32 neighbours of every channel closing.  With
    the series stopped at a coarse tolerance (2^-12) the rate jumps where the
    stopping term changes, which the cubic table smooths: there the table must
    agree with the stopped and with the full series within that tolerance."""
    _lib_or_skip()
    o = Problem(cfg)
    for mi, mt in enumerate(o.mats):
        A = np.geomspace(1e9, 9e10, 30000).astype(np.float32)
        for Ak in _closings(mt, o.laser.lam, 1e9, 9e10):
            f = np.float32(Ak)
            nb = [f]
            lo = hi = f
            for _ in range(3):
                lo = np.nextafter(lo, np.float32(0))
                hi = np.nextafter(hi, np.float32(np.inf))
                nb += [lo, hi]
            A = np.concatenate([A, np.array(nb, dtype=np.float32),
                                (np.float64(Ak) * (1 + np.linspace(-1e-3, 1e-3, 41))).astype(np.float32)])
        Pt = P.table_probe(cfg, mi, A)
        Wo = K.keldysh_rate(A.astype(np.float64), mt.gap_eV, mt.mred, o.laser.lam, tol_bits=o.tol_bits)
        Po = -np.expm1(-Wo * o.dt / mt.n0)
        # anything that could fire against a 32-bit draw is tabulated
        assert not np.any((Pt == 0) & (Po >= 2.0 ** -33))
        sel = Po >= 2.0 ** -33
        rel = np.abs(Pt[sel] / Po[sel] - 1)
        if o.tol_bits >= 60:
            assert np.max(rel) < 1e-6
        else:
            Wf = K.keldysh_rate(A.astype(np.float64), mt.gap_eV, mt.mred, o.laser.lam)
            Pf = -np.expm1(-Wf * o.dt / mt.n0)
            assert np.max(rel) < 2.0 ** -o.tol_bits
            assert np.max(np.abs(Pt[sel] / Pf[sel] - 1)) < 2.0 ** -o.tol_bits + 1e-6
        assert np.all(Pt[~sel] < 2.0 ** -32)


@pytest.mark.parametrize("cfg", [W.config_2d(), W.config_3d(), dict(W.config_2d(), keldysh_tol_bits=12)],
                         ids=["2d", "3d", "2d_tol12"])
def test_skip_bound_covers_every_lookup_below(cfg):
    """The bound the ionization step compares a draw with before it reads the
    neutral's amplitude: on a dense sorted sample of FP32 amplitudes, and on
    every FP32 number within 3000 ulp of each channel closing (where the rate
    has its square-root edge), it is nondecreasing, never below the largest
    lookup at any smaller amplitude, zero where nothing can fire and one from
    saturation on; and it stays within 5 % of that running maximum wherever
    P >= 1e-9 (the bound is held per table interval, 0.2 % of A wide, over
    which P ~ A^(2K) rises by about 2K x 0.2 %), so the skip keeps nearly
    every non-firing neutral out."""
    _lib_or_skip()
    o = Problem(cfg)
    for mi, mt in enumerate(o.mats):
        parts = [np.geomspace(5e8, 2e11, 400000).astype(np.float32)]
        for Ak in _closings(mt, o.laser.lam, 5e8, 2e11):
            f = np.float32(Ak)
            bits = f.view(np.int32) + np.arange(-3000, 3001, dtype=np.int32)
            parts.append(bits.view(np.float32))
        A = np.unique(np.concatenate(parts))
        Pt = P.table_probe(cfg, mi, A)
        B = P.table_probe(cfg, mi, A, bound=True)
        run = np.maximum.accumulate(Pt)
        assert np.all(np.diff(B) >= 0)
        assert np.all(B >= run), (A[np.argmax(run - B)], np.max(run - B))
        assert np.all(B[Pt == 0] <= run[Pt == 0] + (2.0 ** -33))
        assert np.all(B[Pt == 1] == 1)
        sel = run >= 1e-9
        assert np.max(B[sel] / run[sel]) < 1.05


def test_invalid_configs_rejected():
    _lib_or_skip()
    import ctypes as C
    c, keep = P.make_config(W.config_1d())
    c.abi_version = 99
    h = C.c_void_p()
    assert P.lib().pic_init(C.byref(c), C.byref(h)) == -7
    c, keep = P.make_config(W.config_1d())
    c.ndim = 4
    assert P.lib().pic_init(C.byref(c), C.byref(h)) == -1
    c, keep = P.make_config(W.config_1d())
    c.shape_order = 3
    assert P.lib().pic_init(C.byref(c), C.byref(h)) == -1
    with pytest.raises(P.PicError):
        P.canonical(dict(W.config_1d(), cfl=1.5))
    with pytest.raises(P.PicError):
        P.canonical(dict(W.config_2d(), n=[2, 512]))
    assert P.lib().pic_status_str(-6) == b"charged-particle capacity exceeded"


def test_size_limits_rejected():
    """The kernels address grids with 32-bit byte offsets and particles with
    32-bit slots: a guarded grid of 2^30 points or more, or a charged capacity
    above 2^30, is refused before anything is allocated."""
    _lib_or_skip()
    big = dict(W.config_3d(), n=[1100, 1000, 1000])             # 1.1e9 guarded points
    with pytest.raises(P.PicError):
        P.footprint(big)
    ok = dict(W.config_3d(), n=[1000, 1000, 1000])              # just below 2^30 with guards
    assert P.footprint(ok) > 0
    with pytest.raises(P.PicError):
        P.footprint(dict(W.config_2d(), particle_capacity=(1 << 30) + 2))


def test_footprint_scales_with_problem():
    _lib_or_skip()
    f2 = P.footprint(W.config_2d())
    f3 = P.footprint(W.config_3d())
    assert 50e6 < f2 < 2e9
    assert f3 > f2
