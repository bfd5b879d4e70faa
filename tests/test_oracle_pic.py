"""Pins of the oracle's PIC step to closed forms, invariants and brute force.

Each check fixes a part a plausible mistake would break: the Boris rotation
(sign, angle, gamma), the Esirkepov weights (index, 1/2 and 1/3 factors), the
Yee curl (sign, staggering, permittivity placement), the outflow/injection
boundary, the coupling of particles and fields (plasma frequency, Gauss law
through ionization births) and the Monte-Carlo ionization statistics."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import pic, keldysh
from oracle.constants import C, EPS0, QE


def _cfg(ndim, n, dxfrac=40, layers=None, periodic_x=False, transverse="outflow", order=2,
         peak=1e13, ppc=4, nsteps=1000):
    dx = W.LAMBDA / dxfrac
    cfg = dict(ndim=ndim, n=list(n), dx=[dx] * ndim, cfl=0.95, nsteps=nsteps,
               transverse_bc=transverse, materials=[W.silica_like(), W.high_index()],
               layers=layers or [], ppc=ppc, T_K=300.0, shape_order=order, keldysh_terms=500,
               seed=3, laser=dict(lambda_m=W.LAMBDA, fwhm_s=W.cycles(2), peak_Wcm2=peak,
                                  envelope="gauss", pol_axis=1),
               particle_capacity=0, preionize_eV=0.0)
    if periodic_x:
        cfg["periodic_x"] = True
    return cfg


def _sim_with_particles(cfg, pos, u, kind):
    s = pic.Sim(cfg, load_neutrals=False)
    s.px = np.array(pos, dtype=float).reshape(-1, 3)
    s.pu = np.array(u, dtype=float).reshape(-1, 3)
    s.pk = np.array(kind, dtype=np.int64).reshape(-1)
    return s


# ------------------------------------------------------------------ Boris push
def test_larmor_rotation_angle_and_speed():
    s = _sim_with_particles(_cfg(1, [256]), [[128.3, 0, 0]], [[0.02, 0.05, 0.0]], [0])
    bz = 2.0e10
    s.b[2][...] = bz
    h = s.P.kinds[0]["h"]
    u0 = s.pu[0].copy()
    for _ in range(200):
        uo = s.pu[0].copy()
        s.push_and_deposit()
        un = s.pu[0]
        g = math.sqrt(1 + uo @ uo)
        ang = math.atan2(uo[0] * un[1] - uo[1] * un[0], uo[0] * un[0] + uo[1] * un[1])
        # Boris: rotation by 2 atan(|t|), t = h b / gamma (sense set by the sign of q)
        assert abs(abs(ang) - 2 * math.atan(abs(h) * bz / g)) < 1e-13
        assert abs(math.sqrt(un @ un) - math.sqrt(u0 @ u0)) < 1e-15
        s.px[0] = [128.3, 0, 0]          # keep it in the uniform field
    # electron (q < 0) in +z field gyrates counter-clockwise in the x-y plane
    assert ang > 0


def test_exb_drift():
    """E_y and b_z uniform, E << cB: guiding-centre velocity E x B / B^2 = c E_y/b_z x."""
    cfg = _cfg(2, [16, 16], transverse="periodic", periodic_x=True)
    s = _sim_with_particles(cfg, [[8.0, 8.0, 0]], [[0.0, 0.0, 0.0]], [0])
    bz, ey = 3.0e12, 3.0e9
    s.b[2][...] = bz
    s.E[1][...] = ey
    h = s.P.kinds[0]["h"]
    # gyro-period in steps from the discrete rotation angle (gamma ~ 1)
    theta = 2 * math.atan(abs(h) * bz)
    nper = 2 * math.pi / theta
    nsteps = int(round(20 * nper))
    x0 = 0.0
    for _ in range(nsteps):
        xb = s.px[0, 0]
        s.push_and_deposit()
        dxp = s.px[0, 0] - xb
        x0 += dxp - 16 * np.round(dxp / 16)
    vdrift = x0 * s.P.dx[0] / (nsteps * s.P.dt)
    assert abs(vdrift / (C * ey / bz) - 1) < 2e-2


def test_pure_e_momentum_and_hyperbolic_motion():
    cfg = _cfg(1, [4096], dxfrac=400)
    s = _sim_with_particles(cfg, [[100.0, 0, 0]], [[0.0, 0, 0]], [0])
    ex = -1.0e9                            # pushes the electron towards +x
    s.E[0][...] = ex
    h = s.P.kinds[0]["h"]
    s.pu[0, 0] = -h * ex                   # at rest at t = 0: u^{-1/2} = -q E dt / (2 m c)
    k = s.P.kinds[0]
    n = 400
    for i in range(n):
        u_before = s.pu[0, 0]
        s.push_and_deposit()
        assert abs(s.pu[0, 0] - (u_before + 2 * h * ex)) <= 1e-15 * max(1.0, abs(s.pu[0, 0]))
    # x(t) = (m c^2 / |q E|) (sqrt(1 + (q E t / m c)^2) - 1) with t = n dt
    a = abs(k["q"] * ex) / (k["mass"] * C)
    t = n * s.P.dt
    xth = (C / a) * (math.sqrt(1 + (a * t) ** 2) - 1)
    xnum = (s.px[0, 0] - 100.0) * s.P.dx[0]
    assert abs(xnum / xth - 1) < 1e-5


# ------------------------------------------------------------- Esirkepov deposit
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_esirkepov_continuity_brute_force(ndim, order):
    rng = np.random.default_rng(10 * ndim + order)
    n = [16, 12, 10][:ndim]
    cfg = _cfg(ndim, n, order=order)
    s = pic.Sim(cfg, load_neutrals=False)
    npart = 40
    x0 = np.zeros((npart, 3))
    for d in range(ndim):
        x0[:, d] = rng.uniform(4, n[d] - 4, npart)
    u = rng.normal(0, 2.0, (npart, 3))
    g = np.sqrt(1 + np.sum(u * u, 1))
    x1 = x0.copy()
    for d in range(ndim):
        x1[:, d] += s.P.Cd[d] * u[:, d] / g
    kind = rng.integers(0, 4, npart)
    qhat = np.array([s.P.kinds[k]["qhat"] for k in kind])
    for J in s.J:
        J[...] = 0
    s._esirkepov(x0, x1, u, g, qhat)
    s.pk = kind
    s.px = x0
    rho0 = s.charge_density()
    s.px = x1
    rho1 = s.charge_density()
    div = np.zeros(s.S)
    for d in range(ndim):
        div += (s.J[d] - np.roll(s.J[d], 1, axis=d)) / s.P.dx[d]
    res = rho1 - rho0 + div
    assert np.max(np.abs(res)) < 1e-13 * np.max(np.abs(rho1))
    # sum of the deposited current = charge x displacement, for each component
    for d in range(3):
        disp = (x1[:, d] - x0[:, d]) * s.P.dx[d] if d < ndim else s.P.Cd[0] * s.P.dx[0] * u[:, d] / g
        assert abs(np.sum(s.J[d]) - np.sum(qhat * disp)) < 1e-12 * np.sum(np.abs(qhat * disp))


def test_esirkepov_order1_1d_is_textbook_cic():
    cfg = _cfg(1, [32], order=1)
    s = pic.Sim(cfg, load_neutrals=False)
    x0 = np.array([[10.2, 0, 0]])
    x1 = np.array([[10.7, 0, 0]])
    qh = s.P.kinds[0]["qhat"]
    s._esirkepov(x0, x1, np.zeros((1, 3)), np.ones(1), np.array([qh]))
    Jx = s.J[0][:, 0, 0]
    nz = np.nonzero(Jx)[0]
    # only the half-node 10+1/2 (array index 10 + G) carries q * displacement
    assert list(nz) == [10 + pic.G]
    assert abs(Jx[10 + pic.G] / (qh * 0.5 * s.P.dx[0]) - 1) < 1e-15


@pytest.mark.parametrize("order", [1, 2])
def test_gather_partition_of_unity_and_linear_exact(order):
    rng = np.random.default_rng(5)
    cfg = _cfg(3, [12, 10, 9], order=order)
    s = pic.Sim(cfg, load_neutrals=False)
    pos = np.stack([rng.uniform(3, 9, 50), rng.uniform(3, 7, 50), rng.uniform(3, 6, 50)], 1)
    one = np.ones(s.S)
    for st in ([False] * 3, [True, False, True]):
        assert np.max(np.abs(s.gather(one, pos, st) - 1)) < 1e-14
        ix, iy, iz = np.meshgrid(*[np.arange(S) - pic.G + (0.5 if st[d] else 0.0)
                                   for d, S in enumerate(s.S)], indexing="ij")
        F = 2.0 + 0.3 * ix - 0.7 * iy + 1.1 * iz
        want = 2.0 + 0.3 * pos[:, 0] - 0.7 * pos[:, 1] + 1.1 * pos[:, 2]
        assert np.max(np.abs(s.gather(F, pos, st) - want)) < 1e-12


# ------------------------------------------------------------------- Yee solver
@pytest.mark.parametrize("ndim,n,k,comp", [(2, [32, 16], (3, 2), 2), (3, [16, 12, 10], (2, 3, 0), 2),
                                           (3, [16, 12, 10], (0, 3, 2), 0), (1, [64], (5,), 1)])
def test_yee_discrete_dispersion(ndim, n, k, comp):
    """Periodic dielectric box, one transverse Fourier mode of E_comp (k_comp = 0):
    a(n+1) + a(n-1) = 2 cos(w dt) a(n) for its projection a, with
    sin^2(w dt/2) = (1/eps_r) sum_d C_d^2 sin^2(k_d dx_d / 2)."""
    cfg = _cfg(ndim, n, layers=[(0, -1.0, 1.0)], periodic_x=True, transverse="periodic")
    s = pic.Sim(cfg, load_neutrals=False)
    G = pic.G
    grids = np.meshgrid(*[np.arange(S) - (G if d < ndim else 0) for d, S in enumerate(s.S)], indexing="ij")
    phase = sum(2 * np.pi * k[d] / n[d] * grids[d] for d in range(ndim))
    s.E[comp][...] = np.cos(phase)
    dom = s._domain_slices(s.stE[comp])
    basis = np.cos(phase)[dom]
    a = []
    for step in range(60):
        a.append(np.sum(s.E[comp][dom] * basis))
        s._b_half()
        s._e_full(step)
        s._b_half()
    a = np.array(a)
    ie = s.P.mats[0].ie
    sin2 = ie * sum(s.P.Cd[d] ** 2 * math.sin(math.pi * k[d] / n[d]) ** 2 for d in range(ndim))
    cos_want = 1 - 2 * sin2
    sel = np.abs(a[1:-1]) > 0.3 * np.max(np.abs(a))
    ratio = (a[2:] + a[:-2]) / (2 * a[1:-1])
    assert np.max(np.abs(ratio[sel] - cos_want)) < 1e-11


def test_yee_energy_invariant():
    """Source-free periodic box: sum E^2/eps + b^{n-1/2} . b^{n+1/2} is conserved."""
    rng = np.random.default_rng(2)
    cfg = _cfg(2, [24, 20], layers=[(0, -1.0, 12 * W.LAMBDA / 40)], periodic_x=True,
               transverse="periodic")
    s = pic.Sim(cfg, load_neutrals=False)
    for c in range(3):
        s.E[c][s._domain_slices(s.stE[c])] = rng.normal(size=s.E[c][s._domain_slices(s.stE[c])].shape)
        s.b[c][s.regB[c]] = rng.normal(size=s.b[c][s.regB[c]].shape)
    vals = []
    for step in range(150):
        bn = [b.copy() for b in s.b]
        s._b_half()
        e2 = sum(np.sum(s.E[c][s._domain_slices(s.stE[c])] ** 2
                        / np.broadcast_to(s.ieE[c], s.S)[s._domain_slices(s.stE[c])]) for c in range(3))
        bb = sum(np.sum(((2 * bn[c] - s.b[c]) * s.b[c])[s.regB[c]]) for c in range(3))
        vals.append(e2 + bb)
        s._e_full(step)
        s._b_half()
    vals = np.array(vals)
    assert np.max(np.abs(vals / vals[0] - 1)) < 1e-13


def _fresnel_R(dxfrac, n_index=1.45):
    """1D: reflected / incident energy at a vacuum probe for a vacuum-dielectric interface."""
    nx = 60 * dxfrac
    xi, xp = 40 * dxfrac, 20 * dxfrac              # interface and probe (cells)
    dx = W.LAMBDA / dxfrac
    mat = dict(W.silica_like(), n_index=n_index)
    cfg = _cfg(1, [nx], dxfrac=dxfrac, layers=[(0, xi * dx, 1.0)])
    cfg["materials"] = [mat]
    s = pic.Sim(cfg, load_neutrals=False)
    L = s.P.laser
    # incident pulse passes the probe around t0 + xp dx / c; reflection 2 (xi - xp) dx / c later
    t_in = L.t0 + xp * dx / C
    t_ref = t_in + 2 * (xi - xp) * dx / C
    split = 0.5 * (t_in + t_ref)
    tend = t_ref + (t_ref - t_in) * 0.9
    nst = int(tend / s.P.dt)
    Ei = Er = 0.0
    for step in range(nst):
        s._b_half()
        s._e_full(step)
        s._b_half()
        v = s.E[1][xp + pic.G, 0, 0] ** 2
        if (step + 1) * s.P.dt < split:
            Ei += v
        else:
            Er += v
    return Er / Ei, Ei * s.P.dt / (0.5 * L.E0 ** 2 * L.env2_integral)


def test_fresnel_reflection_second_order():
    r_exact = ((1 - 1.45) / (1 + 1.45)) ** 2         # R = 3.37 %
    errs = []
    for f in (20, 40, 80):
        R, inj = _fresnel_R(f)
        errs.append(abs(R - r_exact))
        assert abs(inj - 1) < 0.02                  # injected energy at the probe ~ E0
    assert errs[2] < 2e-4
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5


def test_outflow_far_face_reflection():
    cfg = _cfg(1, [1200], dxfrac=40)
    s = pic.Sim(cfg, load_neutrals=False)
    L = s.P.laser
    xp = 1000
    t_in = L.t0 + xp * s.P.dx[0] / C
    split = t_in + 2 * 200 * s.P.dx[0] / C * 0.5
    nst = int((t_in + 2 * 200 * s.P.dx[0] / C + 4 * L.fwhm) / s.P.dt)
    Ei = Er = 0.0
    for step in range(nst):
        s._b_half()
        s._e_full(step)
        s._b_half()
        v = s.E[1][xp + pic.G, 0, 0] ** 2
        if (step + 1) * s.P.dt < split:
            Ei += v
        else:
            Er += v
    assert math.sqrt(Er / Ei) < 1e-2


# ---------------------------------------------------------- particle-field coupling
def test_cold_plasma_oscillation_frequency():
    """k = 0 Langmuir mode of a uniform e- / positive-carrier plasma in a dielectric:
    w = (2/dt) asin(w_p dt / 2), w_p^2 = (1/eps_r) sum_s n q^2 / (m_s eps0)."""
    nx, ppc = 32, 4
    cfg = _cfg(1, [nx], layers=[(0, -1.0, 1.0)], periodic_x=True, ppc=ppc)
    pos = (np.arange(nx * ppc) + 0.5) / ppc
    npart = len(pos)
    px = np.zeros((2 * npart, 3))
    px[:, 0] = np.concatenate([pos, pos])
    pu = np.zeros((2 * npart, 3))
    pu[:npart, 0] = 1e-4
    s = _sim_with_particles(cfg, px, pu, [0] * npart + [1] * npart)
    a = []
    for step in range(120):
        s.step()
        a.append(np.mean(s.E[0][pic.G:pic.G + nx, 0, 0]))
    a = np.array(a)
    mt = s.P.mats[0]
    wp2 = mt.ie * sum(mt.n0 * QE ** 2 / (k["mass"] * EPS0) for k in s.P.kinds[:2])
    w_want = 2 / s.P.dt * math.asin(math.sqrt(wp2) * s.P.dt / 2)
    sel = np.abs(a[1:-1]) > 0.3 * np.max(np.abs(a))
    cosw = (a[2:] + a[:-2]) / (2 * a[1:-1])
    w = np.arccos(np.median(cosw[sel])) / s.P.dt
    assert abs(w / w_want - 1) < 1e-3


@pytest.mark.parametrize("ndim", [1, 2])
def test_gauss_law_through_run_with_births(ndim):
    if ndim == 1:
        cfg = W.config_1d(hi=True, ppc=4, nsteps=1100, n=512)
    else:
        cfg = W.config_2d(nx=192, ny=48, nsteps=500, ppc=2, peak=3e14, slab_cells=12, waist=0.6e-6)
    s = pic.Sim(cfg)
    s.run(cfg["nsteps"])
    nev = sum(len(e[0]) for e in s.events)
    assert nev > 5
    res = s.gauss_residual()
    rho = s.charge_density()
    assert np.max(np.abs(res)) < 1e-11 * np.max(np.abs(rho))
    # births are neutral in pairs and never duplicate a molecule
    ids = np.concatenate([e[0] for e in s.events])
    assert len(np.unique(ids)) == len(ids)
    assert np.sum(s.pk % 2 == 0) == np.sum(s.pk % 2 == 1) or len(s.px) < 2 * nev


def test_window_is_sliding_max_of_node_field():
    cfg = W.config_1d(nsteps=200, n=256, ppc=1)
    s = pic.Sim(cfg)
    hist = []
    for _ in range(150):
        s.step()
        hist.append(s.node_emag())
        want = np.max(np.stack(hist[-s.P.nwin:]), axis=0)
        assert np.array_equal(s.A, want)


def test_ionization_binomial_statistics_at_fixed_amplitude():
    cfg = W.config_1d(n=256, ppc=60)
    s = pic.Sim(cfg)
    mt = s.P.mats[0]
    A = 3.4e10
    Wr = keldysh.keldysh_rate(A, mt.gap_eV, mt.mred, s.P.laser.lam)[0]
    P = -math.expm1(-Wr * s.P.dt / mt.n0)
    s.A[...] = A
    nsteps = int(min(300, max(3, 0.36 / P)))
    for st in range(1, nsteps + 1):
        s.ionize(st)
    N = len(s.nid)
    frac_want = 1 - (1 - P) ** nsteps
    got = np.sum(~s.nalive)
    sigma = math.sqrt(N * frac_want * (1 - frac_want))
    assert abs(got - N * frac_want) < 5 * sigma
    assert 0.05 < frac_want < 0.95
