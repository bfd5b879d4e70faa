"""The discrete problem a run configuration defines (FP64, oracle side).

TEST INFRASTRUCTURE (part of the oracle).

Sources in the paper:
* time step: 0.95 of the CFL limit, dt = 0.95 / (c sqrt(sum 1/dx_d^2)) (Sec. 3.1)
* materials: band gap, index, density, m_h*, m_e* (Sec. 3.2, Table 1); reduced
  mass m* = 1/(1/m_e* + 1/m_h*) (Sec. 3.2); electrons carry m_e* (Sec. 3.2)
* optical region defined by the same shape that places the neutral species
  (Sec. 2.3); permittivity eps_r = n^2, linear and static (Sec. 2.3), or, as
  the dispersive extension of that linear response, a single-pole Lorentz
  medium whose index at the laser wavelength is n (a reading: the paper keeps
  the static limit; the pole's parameters come with the material)
* pulse: sine-squared envelope with a stated intensity FWHM, spot radius w0,
  fluence F = 2 E_las / (pi w0^2) (Sec. 3); linear polarisation with
  I = c eps0 E0^2 / 2 (the convention the ponderomotive energies of Sec. 5 fix)
* one-cycle amplitude window (Sec. 2.1, last paragraph)

Canonicalisation (a reading; the paper is silent on precision): the time step
is rounded down so that c dt / dx_0 is an FP32 number, and every coefficient of
the discrete operator (c dt / dx_d, 1/eps_r, the outflow coefficients) is an
FP32 number.  These numbers define the discrete problem; this module computes
them from the configuration in FP64 with its own code.

Parity: the canonical coefficients are pinned by tests/test_oracle_problem.py
(CFL formula, Table-1 layer thicknesses lambda/2n and lambda/4n of Fig. 1,
ponderomotive energies of Sec. 5, the fluence/intensity relations).
"""

import math
import numpy as np

from .constants import C, QE, ME, EPS0, NA, AMU, KB


def f32_down(v):
    """Largest FP32 value <= v (as a Python float)."""
    f = np.float32(v)
    if float(f) > v:
        f = np.nextafter(f, np.float32(-np.inf))
    return float(f)


def f32(v):
    return float(np.float32(v))


def lorentz_stable(ie, c, cd, s2max):
    """Von Neumann stability of the Yee update coupled to the explicit
    oscillator (lossless medium).  One mode gives, with w = z - 2 + 1/z,
        f(w) = w^2 / ie + (c / ie + 4 s2 + c deps) w + 4 s2 c = 0
    (the characteristic polynomial divided by z^2), whose roots are real and
    negative; |z| = 1 needs both in [-4, 0]: f(-4) >= 0 with the vertex above
    -4.  Both conditions are monotone in s2, so the largest s2 = sum_d C_d^2
    decides; c < 4 is the oscillator's own leapfrog limit."""
    if not (0.0 <= c < 4.0):
        return False
    f4 = (16.0 - 4.0 * c) / ie - 4.0 * cd - s2max * (16.0 - 4.0 * c)
    vertex_ok = c / ie + 4.0 * s2max + cd <= 8.0 / ie
    return f4 > 0.0 and vertex_ok


class Material:
    def __init__(self, m):
        self.gap_eV = float(m["gap_eV"])
        self.n_index = float(m["n_index"])
        self.density_gcc = float(m["density_gcc"])
        self.molar_mass = float(m["molar_mass_gmol"])
        self.me_star = float(m["me_star"])
        self.mh_star = float(m["mh_star"])
        # molecular number density n0 = rho N_A / M  [m^-3]
        self.n0 = self.density_gcc * 1e6 / self.molar_mass * NA
        # reduced mass of Sec. 3.2, in units of the electron mass
        self.mred = 1.0 / (1.0 / self.me_star + 1.0 / self.mh_star)
        self.mol_mass_kg = self.molar_mass * AMU
        pm = float(m.get("pos_mass_kg", 0.0))
        self.pos_mass_kg = pm if pm > 0 else self.mol_mass_kg
        self.e_mass_kg = self.me_star * ME
        # impact ionization rate constant [1/s] (Keldysh's impact rate; 0 = none)
        self.impact_rate = float(m.get("impact_rate_s", 0.0))
        # single-pole Lorentz response (resonance wavelength > 0), else static
        self.lor_lambda = float(m.get("lorentz_lambda_m", 0.0))
        self.lor_gamma = float(m.get("lorentz_gamma_s", 0.0))
        self.eps_inf = float(m.get("eps_inf", 1.0)) if self.lor_lambda > 0 else self.n_index * self.n_index
        # canonical inverse permittivity 1/eps_r = 1/n^2 (static) or 1/eps_inf
        # (Lorentz: the instantaneous part) as an FP32 number
        self.ie = f32(1.0 / self.eps_inf)
        self.lor = (0.0, 0.0, 0.0)   # (a, c, c deps) of the oscillator update; 0: none
        # instantaneous Kerr response: n = n0 + n2 I; per E component the
        # displacement gains chi3 E^3 with chi3 = (4/3) n0^2 eps0 c n2 (a
        # linearly polarised wave then sees eps + (3/4) chi3 E0^2, i.e. the
        # index change n2 I); chi3 [m^2/V^2] as an FP32 number, 0: none
        n2 = float(m.get("kerr_n2_m2W", 0.0))
        if n2 < 0:
            raise ValueError("negative n2")
        self.chi3 = f32(4.0 / 3.0 * self.n_index * self.n_index * EPS0 * C * n2)


class Laser:
    """Incident pulse at the x_min face (Sec. 3): E(t) = E0 env(t) cos(w (t - t0) + cep)."""

    def __init__(self, L):
        self.lam = float(L["lambda_m"])
        self.omega = 2.0 * math.pi * C / self.lam
        self.fwhm = float(L["fwhm_s"])
        self.envelope = L.get("envelope", "gauss")
        self.waist = float(L.get("waist_m", 0.0))
        self.cep = float(L.get("cep_rad", 0.0))
        self.pol_axis = int(L.get("pol_axis", 1))
        tp = float(L.get("t_peak_s", 0.0))
        if self.envelope == "gauss":
            # field envelope exp(-2 ln2 (t-t0)^2 / tau^2): intensity FWHM tau
            self.t0 = tp if tp > 0 else 3.0 * self.fwhm
            self.T = 0.0
            env2_int = self.fwhm * math.sqrt(math.pi / (4.0 * math.log(2.0)))
        elif self.envelope == "sin2":
            # field envelope sin^2(pi t / T): intensity sin^4 has FWHM tau
            self.T = self.fwhm / (1.0 - (2.0 / math.pi) * math.asin(2.0 ** -0.25))
            self.t0 = tp if tp > 0 else 0.5 * self.T
            env2_int = 3.0 * self.T / 8.0
        else:
            raise ValueError("envelope")
        self.env2_integral = env2_int
        F = float(L.get("fluence_Jcm2", 0.0))
        if F > 0:
            self.I0 = F * 1e4 / env2_int          # W/m^2
        else:
            self.I0 = float(L["peak_Wcm2"]) * 1e4
        self.E0 = math.sqrt(2.0 * self.I0 / (C * EPS0))

    def env(self, t):
        t = np.asarray(t, dtype=np.float64)
        if self.envelope == "gauss":
            return np.exp(-2.0 * math.log(2.0) * (t - self.t0) ** 2 / self.fwhm ** 2)
        s = t - self.t0 + 0.5 * self.T
        return np.where((s >= 0) & (s <= self.T), np.sin(math.pi * s / self.T) ** 2, 0.0)

    def field(self, t):
        t = np.asarray(t, dtype=np.float64)
        return self.E0 * self.env(t) * np.cos(self.omega * (t - self.t0) + self.cep)


class Problem:
    """All derived quantities of one configuration."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.D = int(cfg["ndim"])
        n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
        dx = list(cfg["dx"]) + [0.0] * (3 - len(cfg["dx"]))
        self.n = [int(n[d]) if d < self.D else 1 for d in range(3)]
        self.dx = [float(dx[d]) if d < self.D else 1.0 for d in range(3)]
        per = cfg.get("transverse_bc", "outflow") == "periodic"
        # x is the propagation axis (outflow, laser at x_min); "periodic_x" exists
        # only for the oracle's own invariant checks in a closed box
        self.periodic = [bool(cfg.get("periodic_x", False))] + [per and d < self.D for d in (1, 2)]
        self.nsteps = int(cfg["nsteps"])
        self.ppc = int(cfg["ppc"])
        self.T_K = float(cfg.get("T_K", 300.0))
        self.order = int(cfg.get("shape_order", 2))
        self.terms = int(cfg.get("keldysh_terms", 500))
        self.tol_bits = int(cfg.get("keldysh_tol_bits", 0)) or 60
        self.seed = int(cfg["seed"])
        # binary collisions among the charged particles (Sec. 2.2), off unless asked for
        self.collisions = bool(cfg.get("collisions", False))

        # time step: cfl / (c sqrt(sum_d 1/dx_d^2)), Sec. 3.1; canonicalised
        s = 0.0
        for d in range(self.D):
            s += 1.0 / (self.dx[d] * self.dx[d])
        s = math.sqrt(s)
        c0 = f32_down(float(cfg["cfl"]) / (self.dx[0] * s))
        self.dt = c0 * self.dx[0] / C
        self.Cd = [f32(c0 * (self.dx[0] / self.dx[d])) if d < self.D else 0.0 for d in range(3)]
        self.Cd[0] = c0
        self.kmur = [f32((self.Cd[d] - 1.0) / (self.Cd[d] + 1.0)) if d < self.D else 0.0
                     for d in range(3)]

        self.laser = Laser(cfg["laser"])
        # one laser cycle of samples, Sec. 2.1 (window includes the current step)
        self.nwin = int(math.ceil((self.laser.lam / C) / self.dt))

        self.mats = [Material(m) for m in cfg["materials"]]
        for mt in self.mats:
            if mt.lor_lambda > 0:
                mt.lor = self._lorentz(mt)
        self.layers = [(int(L[0]), float(L[1]), float(L[2])) for L in cfg["layers"]]
        self.vcell = 1.0
        for d in range(self.D):
            self.vcell *= self.dx[d]

        # geometry predicate along the propagation axis (Sec. 2.3)
        nx = self.n[0]
        self.mat_cell = np.array([self.material_at((i + 0.5) * self.dx[0]) for i in range(nx)])
        self.mat_node = np.array([self.material_at(i * self.dx[0]) for i in range(nx + 1)])

        # particle kinds: 2*mat = electron (m_e*), 2*mat+1 = positive carrier
        self.kinds = []
        for mt in self.mats:
            for sp, q, mass in (("e", -QE, mt.e_mass_kg), ("p", QE, mt.pos_mass_kg)):
                self.kinds.append(dict(
                    species=sp, q=q, mass=mass,
                    # q w / (eps0 V) with w = n0 V / ppc  [V/m^2]
                    qhat=q * mt.n0 / (self.ppc * EPS0),
                    # Boris half-step coefficient q dt / (2 m c)  [1/(V/m)]
                    h=q * self.dt / (2.0 * mass * C),
                    weight=mt.n0 * self.vcell / self.ppc,
                    mat=mt))

    def _lorentz(self, mt):
        """Coefficients of the polarisation oscillator of one Lorentz material.

        Medium: eps(w) = eps_inf + deps w0^2 / (w0^2 - w^2 - i g w).  With
        Q = P / eps0 and K = dt J_p / eps0 (J_p = dP/dt) the oscillator
        P'' + g P' + w0^2 P = eps0 deps w0^2 E, centred at step n, reads
            K^{n+1/2} = a K^{n-1/2} + c deps E^n - c Q^n,   Q^{n+1} = Q^n + K^{n+1/2}
        with a = (1 - g dt/2)/(1 + g dt/2), c = (w0 dt)^2 / (1 + g dt/2).  deps is
        fixed by Re eps(w_laser) = n^2 (n is the index at the laser wavelength);
        the static permittivity is then eps_inf + deps.  a, c and c deps are
        canonical FP32 numbers."""
        w0 = 2.0 * math.pi * C / mt.lor_lambda
        w = self.laser.omega
        g = mt.lor_gamma
        if not (w0 > w):
            raise ValueError("Lorentz resonance must lie above the laser frequency")
        t = w0 * w0 - w * w
        re_shape = w0 * w0 * t / (t * t + (g * w) * (g * w))
        mt.deps = (mt.n_index * mt.n_index - mt.eps_inf) / re_shape
        if mt.deps < 0:
            raise ValueError("eps_inf above n^2")
        dt = self.dt
        den = 1.0 + 0.5 * g * dt
        a = (1.0 - 0.5 * g * dt) / den
        c = (w0 * dt) * (w0 * dt) / den
        lor = (f32(a), f32(c), f32(c * mt.deps))
        s2max = sum(self.Cd[d] * self.Cd[d] for d in range(self.D))
        if not lorentz_stable(mt.ie, lor[1], lor[2], s2max):
            raise ValueError("Lorentz medium unstable at this time step")
        return lor

    def material_at(self, x):
        for (m, lo, hi) in self.layers:
            if lo <= x < hi:
                return m
        return -1

    def ie_of(self, mat_idx):
        return np.array([1.0 if m < 0 else self.mats[m].ie for m in mat_idx])

    def lor_of(self, mat_idx):
        """(a, c, c deps) per position; zeros where no oscillator."""
        return np.array([(0.0, 0.0, 0.0) if m < 0 else self.mats[m].lor for m in mat_idx]).reshape(-1, 3)

    def chi3_of(self, mat_idx):
        """Kerr chi3 [m^2/V^2] per position; zero where none."""
        return np.array([0.0 if m < 0 else self.mats[m].chi3 for m in mat_idx])

    def transverse_profile(self, y, z):
        """Gaussian transverse field profile exp(-r^2/w0^2) at the injection plane."""
        w0 = self.laser.waist
        if w0 <= 0 or self.D == 1:
            return np.ones(np.broadcast(y, z).shape)
        return np.exp(-(np.asarray(y) ** 2 + np.asarray(z) ** 2) / (w0 * w0))
