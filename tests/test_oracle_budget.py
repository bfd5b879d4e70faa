"""Pins of the oracle's loading, exact-skip amplitude and energy diagnostics.

Each check compares an oracle function with a value the physics or the
mathematics fixes independently of the oracle's own formula:

* the 300 K thermal draw (Sec. 3.1) against the Maxwellian's per-component
  variance k_B T / m with the molecule's mass, and its normality;
* the exact-skip amplitude (a reading of Sec. 2.1: a neutral whose
  probability cannot beat the smallest uniform draw is never evaluated)
  against the probability on a fine grid and at the left limit of every
  channel closing below it;
* the number and energy density grids (Sec. 4.1, 4.2) against the particle
  totals and against a uniform lattice load whose density is n0 exactly;
* the field energy against the energy density of uniform fields in a
  dielectric, and the Poynting budget of a pulse crossing vacuum against its
  analytic fluence and against the field energy it leaves in the box;
* the gap energy against the event count times the macroparticle weight and
  the band gap, both computed here from the material's density and molar mass.
"""

import math

import numpy as np
import pytest
from scipy import stats
from scipy.optimize import brentq

import workloads as W
from oracle import keldysh as K
from oracle import pic

KB = 1.380649e-23          # J/K
NA = 6.02214076e23         # 1/mol
CL = 299792458.0           # m/s
E0_VAC = 8.8541878128e-12  # F/m
EV = 1.602176634e-19       # J
M_E = 9.1093837015e-31     # kg


def _cfg(ndim, n, dxfrac=40, layers=None, transverse="outflow", order=2, peak=1e13, ppc=4,
         nsteps=1000, waist=0.0, mats=None):
    dx = W.LAMBDA / dxfrac
    return dict(ndim=ndim, n=list(n), dx=[dx] * ndim, cfl=0.95, nsteps=nsteps,
                transverse_bc=transverse, materials=mats or [W.silica_like(), W.high_index()],
                layers=layers or [], ppc=ppc, T_K=300.0, shape_order=order, keldysh_terms=500,
                seed=5, laser=dict(lambda_m=W.LAMBDA, fwhm_s=W.cycles(2), peak_Wcm2=peak,
                                   waist_m=waist, envelope="gauss", pol_axis=1),
                particle_capacity=0, preionize_eV=0.0)


# ------------------------------------------------------------- thermal load
@pytest.mark.parametrize("mat", [W.silica_like(), W.high_index()], ids=["sio2", "hfo2"])
def test_thermal_velocity_is_maxwellian_at_300K(mat):
    """u = v/c of each Cartesian component: mean 0, variance k_B T / (m c^2) with
    m the molecule's mass M / N_A (5 sigma of the sample statistics), and the
    normalised components standard normal (Kolmogorov-Smirnov)."""
    cfg = _cfg(1, [64], layers=[(0, 0.0, 1.0)], mats=[mat])
    s = pic.Sim(cfg, load_neutrals=False)
    n = 200_000
    ids = np.arange(n, dtype=np.int64) * 7 + 11
    u = s.thermal_u(ids, np.zeros(n, dtype=np.int64))
    m_kg = mat["molar_mass_gmol"] * 1e-3 / NA
    var = KB * 300.0 / (m_kg * CL * CL)
    for c in range(3):
        x = u[:, c]
        assert abs(np.mean(x)) < 5 * math.sqrt(var / n)
        assert abs(np.var(x) / var - 1.0) < 5 * math.sqrt(2.0 / (n - 1))
        assert stats.kstest(x / math.sqrt(var), "norm").pvalue > 1e-4
    # components independent: the sample correlations are noise
    cc = np.corrcoef(u.T)
    assert np.max(np.abs(cc - np.eye(3))) < 5 / math.sqrt(n)


# ------------------------------------------------------ exact skip amplitude
def _closings(mt, lam, lo, hi):
    """Amplitudes in (lo, hi) where x(A) (Eq. 1) crosses an integer."""
    x = lambda A: K.keldysh_parts(np.array([A]), mt.gap_eV, mt.mred, lam)["x"][0]
    out = []
    for k in range(int(np.floor(x(lo))) + 1, int(np.floor(x(hi))) + 1):
        out.append(brentq(lambda A: x(A) - k, lo, hi, xtol=1e-9, rtol=1e-15))
    return out


@pytest.mark.parametrize("which", ["config_1d", "config_3d"])
def test_amp_cut_never_skips_a_possible_event(which):
    """Below the cut every per-step probability is below 2^-33, the smallest
    value a uniform draw (w + 1/2) 2^-32 can take, so skipping those neutrals
    changes no event: checked on a fine grid and at the left limit of every
    channel closing under the cut (where W jumps down as A increases, so the
    supremum of P below the cut is reached there)."""
    cfg = getattr(W, which)()
    s = pic.Sim(cfg, load_neutrals=False)
    P = s.P
    for mi, mt in enumerate(P.mats):
        acut = s.acut[mi]
        assert np.isfinite(acut) and acut > 0
        grid = np.concatenate([np.geomspace(acut * 1e-3, acut, 40001)])
        closings = _closings(mt, P.laser.lam, acut * 1e-3, acut)
        left = np.array([a * (1 - 1e-12) for a in closings])
        A = np.concatenate([grid, left])
        A = A[A <= acut]
        Wr = K.keldysh_rate(A, mt.gap_eV, mt.mred, P.laser.lam, terms=P.terms)
        Pp = -np.expm1(-Wr * P.dt / mt.n0)
        assert np.max(Pp) < 2.0 ** -33, (mt.gap_eV, float(np.max(Pp)))
        # and the cut is not far below the first amplitude that can fire: the
        # probability reaches 2^-34 within one grid step (0.2 %) above it
        above = np.geomspace(acut, acut * 1.0025, 64)
        Pa = -np.expm1(-K.keldysh_rate(above, mt.gap_eV, mt.mred, P.laser.lam, terms=P.terms) * P.dt / mt.n0)
        assert np.max(Pa) >= 2.0 ** -34


# ------------------------------------------------------------ density grids
def _lattice(ndim, n, m):
    """m^ndim particles per cell on a regular lattice (offsets (r + 0.3)/m)."""
    axes = []
    for d in range(ndim):
        axes.append((np.arange(n[d] * m) + 0.3) / m)
    g = np.meshgrid(*axes, indexing="ij")
    pos = np.zeros((g[0].size, 3))
    for d in range(ndim):
        pos[:, d] = g[d].ravel()
    return pos


@pytest.mark.parametrize("ndim,order", [(1, 1), (1, 2), (2, 1), (2, 2)])
def test_density_grid_totals_and_uniform_lattice(ndim, order):
    """Sum of n V over the nodes = the electrons' total weight; a lattice of m
    electrons per cell along each axis (weight n0 V / ppc, ppc = m^ndim) gives
    n0 at every node whose shape support is filled (unit-spaced sublattices:
    the B-spline partition of unity)."""
    m = 2
    n = [24] * ndim
    cfg = _cfg(ndim, n, layers=[(0, -1.0, 1.0)], transverse="periodic", order=order, ppc=m ** ndim)
    s = pic.Sim(cfg, load_neutrals=False)
    pos = _lattice(ndim, n, m)
    s.px = pos
    s.pu = np.zeros_like(pos)
    s.pk = np.zeros(len(pos), dtype=np.int64)             # electrons of material 0
    ne = s.density_grid("e")
    mat = W.silica_like()
    n0 = mat["density_gcc"] * 1e6 / mat["molar_mass_gmol"] * NA
    vcell = np.prod(cfg["dx"])
    w = n0 * vcell / m ** ndim
    assert abs(np.sum(ne) * vcell / (w * len(pos)) - 1.0) < 1e-12
    inner = [slice(pic.G + 3, pic.G + n[0] - 3)] + [slice(pic.G, pic.G + n[d]) for d in range(1, ndim)]
    inner += [slice(0, 1)] * (3 - ndim)
    assert np.max(np.abs(ne[tuple(inner)] / n0 - 1.0)) < 1e-12


@pytest.mark.parametrize("ndim", [1, 2])
def test_energy_density_grid_totals_and_uniform_lattice(ndim):
    """Sum of u V = the electrons' total kinetic energy sum w (gamma - 1) m c^2
    (with random momenta), and a uniform lattice of equal-energy electrons gives
    n0 (gamma - 1) m c^2 at every filled node (Sec. 4.2: density times mean
    energy).  Positive carriers do not enter the electron grid."""
    m = 2
    n = [20] * ndim
    cfg = _cfg(ndim, n, layers=[(0, -1.0, 1.0)], transverse="periodic", ppc=m ** ndim)
    mat = W.silica_like()
    n0 = mat["density_gcc"] * 1e6 / mat["molar_mass_gmol"] * NA
    vcell = np.prod(cfg["dx"])
    w = n0 * vcell / m ** ndim
    me = mat["me_star"] * M_E
    rng = np.random.default_rng(4)
    s = pic.Sim(cfg, load_neutrals=False)
    pos = _lattice(ndim, n, m)
    npart = len(pos)
    s.px = np.concatenate([pos, pos])
    u = rng.normal(scale=0.05, size=(npart, 3))
    s.pu = np.concatenate([u, u])
    s.pk = np.concatenate([np.zeros(npart, dtype=np.int64), np.ones(npart, dtype=np.int64)])
    ue = s.energy_density_grid("e")
    gam = np.sqrt(1.0 + np.sum(u * u, axis=1))
    ke_tot = np.sum(w * (gam - 1.0) * me * CL * CL)
    assert abs(np.sum(ue) * vcell / ke_tot - 1.0) < 1e-10
    # equal energies: (gamma - 1) m c^2 at gamma from |u| = 0.03
    s.pu = np.zeros((2 * npart, 3))
    s.pu[:, 1] = 0.03
    ue = s.energy_density_grid("e")
    want = n0 * (math.sqrt(1.0 + 0.03 ** 2) - 1.0) * me * CL * CL
    inner = [slice(pic.G + 3, pic.G + n[0] - 3)] + [slice(pic.G, pic.G + n[d]) for d in range(1, ndim)]
    inner += [slice(0, 1)] * (3 - ndim)
    assert np.max(np.abs(ue[tuple(inner)] / want - 1.0)) < 1e-10


# -------------------------------------------------------------- field energy
def test_field_energy_of_uniform_fields():
    """Uniform E_y = E0 in a medium of index n filling the box: energy density
    eps0 n^2 E0^2 / 2 over the node positions; uniform b_z = b0 (b = c B):
    B^2 / (2 mu0) = eps0 b0^2 / 2 over the half-staggered positions."""
    nx = 50
    cfg = _cfg(1, [nx], layers=[(0, -1.0, 1.0)])
    s = pic.Sim(cfg, load_neutrals=False)
    dx = cfg["dx"][0]
    nidx = W.silica_like()["n_index"]
    e0, b0 = 3.0e9, 2.0e9
    s.E[1][s._domain_slices(s.stE[1])] = e0
    # 1/eps_r is canonicalised to an FP32 number: the energy uses that medium
    ie = float(np.float32(1.0 / nidx ** 2))
    want_e = 0.5 * E0_VAC * e0 ** 2 / ie * (nx + 1) * dx
    assert abs(s.field_energy() / want_e - 1.0) < 1e-12
    s.E[1][...] = 0.0
    s.b[2][s._domain_slices(s.stB[2])] = b0
    want_b = 0.5 * E0_VAC * b0 ** 2 * nx * dx
    assert abs(s.field_energy() / want_b - 1.0) < 1e-12


def _vacuum_pulse(dxfrac, through=False):
    nx = 40 * dxfrac
    cfg = _cfg(1, [nx], dxfrac=dxfrac, nsteps=40000)
    s = pic.Sim(cfg, load_neutrals=False)
    L = s.P.laser
    env2 = W.cycles(2) * math.sqrt(math.pi / (4.0 * math.log(2.0)))
    fluence = 0.5 * E0_VAC * CL * L.E0 ** 2 * env2
    t_in = 2 * L.t0 + 20 * cfg["dx"][0] / CL            # the whole pulse has crossed x = 20 cells
    while s.step_index * s.P.dt < t_in:
        s.step()
    inside = (s.energy_in / fluence - 1.0, (s.energy_in - s.energy_out) / s.field_energy() - 1.0,
              s.energy_out / s.energy_in)
    if not through:
        return inside
    t_out = 2 * L.t0 + (nx + 20) * cfg["dx"][0] / CL
    while s.step_index * s.P.dt < t_out:
        s.step()
    return inside, (s.energy_out / s.energy_in - 1.0, s.field_energy() / s.energy_in)


def test_poynting_budget_of_a_pulse_crossing_vacuum():
    """1D vacuum: the pulse's energy per unit area entering through the x_min
    plane is its fluence, eps0 c E0^2 / 2 times the integral of env^2 (the
    carrier averages cos^2 to 1/2; for a 2-cycle Gaussian the correction is
    e^-28), up to the second-order discretisation error of the injection (shown
    converging at lambda/20, 40, 80); once the pulse is inside, E_in - E_out is
    the field energy in the box (same order); after it has left through x_max,
    E_out = E_in and the box is empty."""
    errs = [_vacuum_pulse(f) for f in (20, 80)]
    (e40, out40) = _vacuum_pulse(40, through=True)
    errs.insert(1, e40)
    for (fl, bud, leak) in errs:
        assert leak == 0.0                                    # nothing left before the pulse got there
    fl = [abs(e[0]) for e in errs]
    bud = [abs(e[1]) for e in errs]
    assert fl[1] < 8e-3 and fl[2] < 2e-3
    assert fl[0] / fl[1] > 3.5 and fl[1] / fl[2] > 3.5
    assert bud[1] < 4e-3 and bud[0] / bud[1] > 3.5 and bud[1] / bud[2] > 3.5
    assert abs(out40[0]) < 1e-3 and out40[1] < 1e-3


def test_poynting_budget_closes_through_transverse_faces():
    """2D vacuum, a 0.6 um-waist beam diffracting onto the y faces: by the time
    the pulse has left the box, the energy that entered equals the energy that
    left through the x and y planes plus what remains, and a large share left
    through the y planes (a dropped or sign-flipped transverse flux fails)."""
    cfg = _cfg(2, [400, 48], dxfrac=24, waist=0.6e-6, nsteps=4000)
    s = pic.Sim(cfg, load_neutrals=False)
    L = s.P.laser
    mid = 2 * L.t0 + 20 * cfg["dx"][0] / CL             # all of it entered, none reached x_max
    while s.step_index * s.P.dt < mid:
        s.step()
    assert s.energy_out > 0.1 * s.energy_in              # through the y planes only, so far
    late = 2 * L.t0 + 600 * cfg["dx"][0] / CL
    while s.step_index * s.P.dt < late:
        s.step()
    u = s.field_energy()
    assert u < 0.02 * s.energy_in
    assert abs((s.energy_out + u) / s.energy_in - 1.0) < 1e-4


# --------------------------------------------------------------- gap energy
def test_gap_energy_is_events_times_weight_times_gap():
    """Fixed amplitude, ionization only: every event pays the band gap for the
    macroparticle's weight n0 V / ppc, n0 = rho N_A / M."""
    cfg = W.config_1d(n=256, ppc=40)
    s = pic.Sim(cfg)
    s.A[...] = 3.4e10
    for st in range(1, 41):
        s.ionize(st)
    nev = int(np.sum(~s.nalive))
    assert nev > 100
    mat = cfg["materials"][0]
    n0 = mat["density_gcc"] * 1e6 / mat["molar_mass_gmol"] * NA
    w = n0 * cfg["dx"][0] / cfg["ppc"]
    assert abs(s.energy_gap / (nev * w * mat["gap_eV"] * EV) - 1.0) < 1e-12
