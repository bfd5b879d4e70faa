"""Plain FP64 particle-in-cell time step for laser-dielectric runs.

TEST INFRASTRUCTURE (part of the oracle).  Written for clarity, not speed:
NumPy arrays, whole-array shifted differences for the field solve, loops over
the shape-function stencil with scatter-adds by ``np.bincount``.

The paper builds on a standard PIC code (Sec. 1, 2) and only states the parts
it changes; the inherited parts follow the textbook method named alongside:

* Yee FDTD (Maxwell's equations on a staggered grid) with a spatially varying
  static permittivity eps_r = n^2 in the E update (Sec. 2.3).  Fields are kept
  as E [V/m] and b = c B [V/m].  One step: b^{n+1/2} = b^n - (1/2) C curl E^n,
  E^{n+1} = E^n + (1/eps_r)(C curl b^{n+1/2} - dt J/eps0),
  b^{n+1} = b^{n+1/2} - (1/2) C curl E^{n+1}, where C_d = c dt / dx_d.
* Dispersive extension of that linear response (a reading; the paper keeps it
  static): a single-pole Lorentz medium, eps(w) = eps_inf + deps w0^2 /
  (w0^2 - w^2 - i g w), with the polarisation P and its current J_p = dP/dt as
  the auxiliary differential equation P'' + g P' + w0^2 P = eps0 deps w0^2 E,
  centred at integer steps: J_p^{n+1/2} from J_p^{n-1/2}, E^n and P^n, then
  P^{n+1} = P^n + dt J_p^{n+1/2}, and J_p^{n+1/2} enters the E update beside
  the free current with 1/eps_inf in place of 1/eps_r.
* Its nonlinear extension (a reading; the paper leaves nonlinear optics out,
  Sec. 2.3): an instantaneous Kerr term, per E component chi3 E^3 in the
  displacement, chi3 = (4/3) n0^2 eps0 c n2; the displacement advances by the
  curl and the currents, and E^{n+1} solves the cubic pointwise.
* "Simple outflow" boundaries (Sec. 3.1): first-order Mur on each outflow
  face for the tangential E; the laser enters as the incident field of the
  x_min face condition (Sec. 3, Fig. 1: driven from the minimum boundary).
  A point on several faces follows the first face in the order x, y, z and
  uses its inward neighbour's final value.
* Shape-function gather of each Yee component from its own staggered grid
  (order 1 or 2 B-spline; the paper's number-density output uses the same
  shape, Sec. 4.1).
* Relativistic Boris push (the Lorentz-force push of Sec. 1).
* Esirkepov charge-conserving current deposit (Esirkepov, CPC 135, 144 (2001)),
  with the direct deposit of the velocity components along absent dimensions.
* One-cycle rolling window of the node |E|; its maximum is the amplitude
  entering the Keldysh rate (Sec. 2.1, last paragraph).
* Energy diagnostics: field energy, carriers' kinetic energy, the gap energy
  paid by ionization (absorbed energy, a reading of Sec. 4.2), the number and
  energy density grids (Sec. 4.1, 4.2), and the Poynting flux through the
  faces of the box one cell inside the outflow faces (the field-side budget).
* Binary Coulomb collisions among the charged particles (Sec. 2.2, Eq. 4;
  optional, after ionization): oracle/collide.py.
* Impact ionization by hot electrons (Keldysh's rate, the paper's future work,
  Sec. 2.2; optional per material, after the collisions): oracle/impact.py.
* Monte-Carlo single ionization of immobile neutral molecule macroparticles
  with the per-molecule rate W/n0, probability 1 - exp(-W dt / n0) per step,
  the whole macroparticle converting into one electron (m_e*, Sec. 3.2) and
  one positive carrier at its position and velocity (Sec. 2.1: each molecule
  ionized at most once).  The rate is evaluated in situ per neutral, in FP64,
  with the series of Eq. (3) truncated at 500 terms (Sec. 2.1).

Parity pins (tests/test_oracle_pic.py): Larmor gyration and its discrete
rotation angle, E x B drift, exact pure-E momentum gain and hyperbolic motion,
per-particle discrete continuity of the deposit and the Gauss law through whole
runs with births, the Yee vacuum dispersion relation and the discrete field
energy invariant, Fresnel reflection at a dielectric interface, the cold-plasma
oscillation frequency, brute-force sliding maximum, the binomial statistics of
ionization at a fixed amplitude; for the paper-style diagnostics, kinetic
energies of particles built from a chosen gamma, the particle and range
bookkeeping of the energy histogram, and the maximum accumulated intensity of a
plane wave crossing vacuum against the peak of its incident field
(tests/test_oracle_diagnostics.py); the 300 K thermal draw against the
Maxwellian variance, the exact-skip amplitude against the probability below
it, the number and energy density grids against particle totals and uniform
lattice loads, the field energy against uniform fields in a dielectric, the
Poynting budget against a pulse's analytic fluence and its closure through
transverse faces, and the gap energy against events x weight x gap
(tests/test_oracle_budget.py); for the Lorentz medium, the discrete dispersion
relation of the coupled scheme, Fresnel reflection against the continuum
eps(w) over the pulse's spectrum, and the Gauss law with the bound charge
(tests/test_oracle_lorentz.py); for the Kerr term, the harmonic-balance
frequency shift of a standing wave and the Gauss law with the nonlinear
displacement (tests/test_oracle_kerr.py).
"""

import math
from collections import deque

import numpy as np

from .constants import C, KB, EPS0, QE
from . import collide, impact, keldysh, philox
from .problem import Problem

G = 3  # guard layers on each side of every present dimension


def shape_weights(x, order):
    """B-spline weights on the integer grid: returns (base index, weights (Np, order+1))."""
    if order == 1:
        base = np.floor(x)
        f = x - base
        return base.astype(np.int64), np.stack([1.0 - f, f], axis=1)
    i0 = np.floor(x + 0.5)
    xi = x - i0
    w = np.stack([0.5 * (0.5 - xi) ** 2, 0.75 - xi * xi, 0.5 * (0.5 + xi) ** 2], axis=1)
    return (i0 - 1).astype(np.int64), w


class Sim:
    def __init__(self, cfg, load_neutrals=True):
        P = self.P = Problem(cfg)
        D = self.D = P.D
        self.S = tuple(P.n[d] + 1 + 2 * G if d < D else 1 for d in range(3))
        self.off = [G if d < D else 0 for d in range(3)]
        z = lambda: np.zeros(self.S)
        self.E = [z(), z(), z()]
        self.b = [z(), z(), z()]
        self.J = [z(), z(), z()]
        # staggering: component c of E is half-integer along d == c; b along d != c
        self.stE = [[d == c for d in range(3)] for c in range(3)]
        self.stB = [[d != c for d in range(3)] for c in range(3)]
        # inverse permittivity at each E component's own location (x only)
        nx = P.n[0]
        ie_half = np.ones(self.S[0])
        ie_half[G:G + nx] = P.ie_of(P.mat_cell)
        ie_node = np.ones(self.S[0])
        ie_node[G:G + nx + 1] = P.ie_of(P.mat_node)
        self.ieE = [ie_half.reshape(-1, 1, 1), ie_node.reshape(-1, 1, 1), ie_node.reshape(-1, 1, 1)]
        # Lorentz oscillators (a, c, c deps) at each E component's own location,
        # their polarisation Q = P/eps0 and current K = dt J_p/eps0 (zero where
        # the medium is static or vacuum: the coefficients vanish there)
        lor_half = np.zeros((self.S[0], 3))
        lor_half[G:G + nx] = P.lor_of(P.mat_cell)
        lor_node = np.zeros((self.S[0], 3))
        lor_node[G:G + nx + 1] = P.lor_of(P.mat_node)
        self.lorE = [[t[:, q].reshape(-1, 1, 1) for q in range(3)] for t in (lor_half, lor_node, lor_node)]
        # Kerr: chi3 at each E component's own location (x only)
        chi_half = np.zeros(self.S[0])
        chi_half[G:G + nx] = P.chi3_of(P.mat_cell)
        chi_node = np.zeros(self.S[0])
        chi_node[G:G + nx + 1] = P.chi3_of(P.mat_node)
        self.chiE = [chi_half.reshape(-1, 1, 1), chi_node.reshape(-1, 1, 1), chi_node.reshape(-1, 1, 1)]
        self.Q = [z(), z(), z()]
        self.K = [z(), z(), z()]
        self.regE = [self._region(self.stE[c], True) for c in range(3)]
        self.regB = [self._region(self.stB[c], False) for c in range(3)]
        self.domain_nodes = self._domain_node_mask()
        # amplitude window (brute force over the last nwin samples)
        self.win = deque(maxlen=P.nwin)
        self.A = z()
        # charged particles: positions in cell units, u = gamma v / c, kind index
        self.px = np.zeros((0, 3))
        self.pu = np.zeros((0, 3))
        self.pk = np.zeros(0, dtype=np.int64)
        # particle id: the id of the neutral it was born from (an electron and
        # its positive carrier share it); particles placed directly get
        # cells x ppc + their index, above every neutral id
        self.pid = np.zeros(0, dtype=np.int64)
        self.step_index = 0
        # trajectory sampling (off when track_every == 0)
        self.track_every = 0
        self.track_thr = 0
        self.tracks = []
        # maximum accumulated intensity: node |E|^2 after every imax_every-th step
        self.imax_every = 0
        self.imax = z()
        self.events = []          # list of (id array, step)
        self.energy_gap = 0.0     # sum over events of w * Delta  [J]
        # field energy carried through the flux planes (one cell inside every
        # outflow face) into and out of the box so far [J]
        self.energy_in = 0.0
        self.energy_out = 0.0
        self.acut = [self._amp_cut(m) for m in P.mats]
        if load_neutrals:
            self._load_neutrals()
        else:
            self._no_neutrals()

    # ------------------------------------------------------------------ setup
    def _region(self, st, isE):
        """Index slices of the positions a field update writes."""
        P = self.P
        sl = []
        for d in range(3):
            if d >= self.D:
                sl.append(slice(0, 1))
                continue
            n = P.n[d]
            if P.periodic[d] or st[d]:
                sl.append(slice(G, G + n))
            elif isE:
                sl.append(slice(G + 1, G + n))      # E tangential: faces set by Mur
            else:
                sl.append(slice(G, G + n + 1))
        return tuple(sl)

    def _domain_node_mask(self):
        m = np.zeros(self.S, dtype=bool)
        sl = []
        for d in range(3):
            if d >= self.D:
                sl.append(slice(0, 1))
            else:
                n = self.P.n[d]
                sl.append(slice(G, G + n + (0 if self.P.periodic[d] else 1)))
        m[tuple(sl)] = True
        return m

    def _amp_cut(self, mt):
        """An amplitude below which the per-step probability is < 2^-34 for every
        smaller amplitude; any neutral below it cannot ionize because the uniform
        draw is at least 2^-33.  Used only to avoid evaluating W there."""
        P = self.P
        A = np.geomspace(1e5, 1e13, 20001)
        W = keldysh.keldysh_rate(A, mt.gap_eV, mt.mred, P.laser.lam, terms=P.terms, tol_bits=P.tol_bits)
        Pp = -np.expm1(-W * P.dt / mt.n0)
        hit = np.nonzero(Pp >= 2.0 ** -34)[0]
        if len(hit) == 0:
            return np.inf
        return float(A[max(hit[0] - 1, 0)])

    def _load_neutrals(self):
        P = self.P
        nx, ny, nz = P.n
        ids, pos, mats = [], [], []
        cells = [i for i in range(nx) if P.mat_cell[i] >= 0]
        if cells:
            ii, jj, kk = np.meshgrid(np.array(cells, dtype=np.int64), np.arange(ny),
                                     np.arange(nz), indexing="ij")
            ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
            lin = ii + nx * (jj + ny * kk)          # cell-major, x fastest
            order = np.argsort(lin, kind="stable")
            ii, jj, kk, lin = ii[order], jj[order], kk[order], lin[order]
            k = np.arange(P.ppc, dtype=np.int64)
            nid = (lin[:, None] * P.ppc + k[None, :]).ravel()
            w = philox.draw32(P.seed, nid, 0, philox.PURPOSE_POS)
            cellc = [np.repeat(ii, P.ppc), np.repeat(jj, P.ppc), np.repeat(kk, P.ppc)]
            p = np.zeros((len(nid), 3))
            for d in range(self.D):
                # offset (w >> 8) * 2^-24: an FP32 number in [0, 1)
                p[:, d] = cellc[d] + (w[d] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
            ids.append(nid)
            pos.append(p)
            mats.append(P.mat_cell[np.repeat(ii, P.ppc)])
        if ids:
            self.nid = np.concatenate(ids)
            self.npos = np.concatenate(pos)
            self.nmat = np.concatenate(mats).astype(np.int64)
        else:
            self._no_neutrals()
            return
        self.nalive = np.ones(len(self.nid), dtype=bool)
        self.ndeath = np.full(len(self.nid), -1, dtype=np.int64)
        if float(P.cfg.get("preionize_eV", 0.0)) > 0:
            self._preionize(float(P.cfg["preionize_eV"]))

    def _no_neutrals(self):
        self.nid = np.zeros(0, dtype=np.int64)
        self.npos = np.zeros((0, 3))
        self.nmat = np.zeros(0, dtype=np.int64)
        self.nalive = np.zeros(0, dtype=bool)
        self.ndeath = np.zeros(0, dtype=np.int64)

    def _maxwell_u(self, nid, purpose, sig):
        """u = v/c drawn from a Maxwellian with per-particle velocity spread ``sig``
        [m/s], Box-Muller on one Philox block (counter (id, 0, purpose))."""
        w = philox.draw32(self.P.seed, nid, 0, purpose)
        u1, u2, u3, u4 = [(wi.astype(np.float64) + 0.5) * 2.0 ** -32 for wi in w]
        r1 = np.sqrt(-2.0 * np.log(u1))
        r2 = np.sqrt(-2.0 * np.log(u3))
        nrm = np.stack([r1 * np.cos(2 * np.pi * u2), r1 * np.sin(2 * np.pi * u2),
                        r2 * np.cos(2 * np.pi * u4)], axis=1)
        return nrm * (np.asarray(sig) / C)[:, None]

    def thermal_u(self, nid, mats):
        """Velocity of a neutral at temperature T (molecule mass; Sec. 3.1: 300 K),
        handed to the carriers it creates."""
        sig = np.array([math.sqrt(KB * self.P.T_K / self.P.mats[m].mol_mass_kg) for m in mats])
        return self._maxwell_u(nid, philox.PURPOSE_VEL, sig)

    def _preionize(self, eV):
        """Stress variant: every neutral starts ionized (step 0); electron and positive
        carrier thermal at kT = eV with their own masses."""
        P = self.P
        idx = np.arange(len(self.nid))
        self.nalive[:] = False
        self.ndeath[:] = 0
        pos = self.npos[idx]
        mats = self.nmat[idx]
        ue = self._maxwell_u(self.nid, philox.PURPOSE_STRESS_E,
                             [math.sqrt(eV * 1.602176634e-19 / P.kinds[2 * m]["mass"]) for m in mats])
        up = self._maxwell_u(self.nid, philox.PURPOSE_STRESS_P,
                             [math.sqrt(eV * 1.602176634e-19 / P.kinds[2 * m + 1]["mass"]) for m in mats])
        self.px = np.concatenate([pos, pos])
        self.pu = np.concatenate([ue, up])
        self.pk = np.concatenate([2 * mats, 2 * mats + 1])
        self.pid = np.concatenate([self.nid, self.nid])

    # ------------------------------------------------------------ field solve
    def _fill_periodic(self, a):
        for d in range(self.D):
            if self.P.periodic[d]:
                n = self.P.n[d]
                a = np.moveaxis(a, d, 0)
                a[0:G] = a[n:n + G]
                a[G + n:] = a[G:G + (a.shape[0] - G - n)]
                a = np.moveaxis(a, 0, d)

    def _fold_periodic(self, a):
        for d in range(self.D):
            if self.P.periodic[d]:
                n = self.P.n[d]
                v = np.moveaxis(a, d, 0)
                lo = v[0:G].copy()
                hi = v[G + n:].copy()
                v[n:n + G] += lo
                v[G:G + hi.shape[0]] += hi
                v[0:G] = 0.0
                v[G + n:] = 0.0

    def _fd(self, a, d):
        if d >= self.D:
            return 0.0
        return np.roll(a, -1, axis=d) - a

    def _bd(self, a, d):
        if d >= self.D:
            return 0.0
        return a - np.roll(a, 1, axis=d)

    def _b_half(self):
        Cx, Cy, Cz = self.P.Cd
        E = self.E
        for a in E:
            self._fill_periodic(a)
        curl = [Cy * self._fd(E[2], 1) - Cz * self._fd(E[1], 2),
                Cz * self._fd(E[0], 2) - Cx * self._fd(E[2], 0),
                Cx * self._fd(E[1], 0) - Cy * self._fd(E[0], 1)]
        for c in range(3):
            r = self.regB[c]
            if np.ndim(curl[c]) == 0:
                continue
            self.b[c][r] -= 0.5 * curl[c][r]

    def _e_full(self, n):
        P = self.P
        Cx, Cy, Cz = P.Cd
        b = self.b
        for a in b:
            self._fill_periodic(a)
        old = [e.copy() for e in self.E]
        curl = [Cy * self._bd(b[2], 1) - Cz * self._bd(b[1], 2),
                Cz * self._bd(b[0], 2) - Cx * self._bd(b[2], 0),
                Cx * self._bd(b[1], 0) - Cy * self._bd(b[0], 1)]
        for c in range(3):
            r = self.regE[c]
            cc = curl[c] if np.ndim(curl[c]) else np.zeros(self.S)
            ie = np.broadcast_to(self.ieE[c], self.S)
            # polarisation current of the step from E^n and Q^n, then Q^{n+1}
            la, lc, lcd = (np.broadcast_to(t, self.S)[r] for t in self.lorE[c])
            k_new = la * self.K[c][r] + lcd * self.E[c][r] - lc * self.Q[c][r]
            self.K[c][r] = k_new
            self.Q[c][r] += k_new
            src = cc[r] - self.J[c][r] - k_new
            g = ie[r] * np.broadcast_to(self.chiE[c], self.S)[r]
            if np.any(g != 0):
                # Kerr: the displacement E/ie + chi3 E^3 (+ Q) advances by the
                # curl and the currents; E^{n+1} solves X + g X^3 = R, g = ie chi3
                e0 = self.E[c][r]
                R = e0 + g * e0 ** 3 + ie[r] * src
                X = e0 + ie[r] * src
                for _ in range(60):       # Newton on a monotone cubic, to FP64 convergence
                    dX = (X + g * X ** 3 - R) / (1.0 + 3.0 * g * X * X)
                    X = X - dX
                    if np.all(np.abs(dX) <= 1e-16 * np.abs(X)):
                        break
                self.E[c][r] = X
            else:
                self.E[c][r] += ie[r] * src
        self._mur(old, n)

    def _face_points(self, c, d):
        """Slices (min face, max face) along d of the E_c points whose face
        priority is d, and the inward neighbour slices."""
        P = self.P
        base = []
        for dd in range(3):
            if dd >= self.D:
                base.append(slice(0, 1))
                continue
            nn = P.n[dd]
            if P.periodic[dd] or self.stE[c][dd]:
                base.append(slice(G, G + nn))
            elif dd < d:
                base.append(slice(G + 1, G + nn))   # lower-priority faces excluded
            else:
                base.append(slice(G, G + nn + 1))
        nd = P.n[d]
        out = []
        for p, q in ((G, G + 1), (G + nd, G + nd - 1)):
            sp = list(base)
            sq = list(base)
            sp[d] = slice(p, p + 1)
            sq[d] = slice(q, q + 1)
            out.append((tuple(sp), tuple(sq), p == G))
        return out

    def _inc(self, c, sl_p, sl_q, n):
        """Incident field at the x_min face point and its inward neighbour, time
        levels n and n+1: E_inc(x, t) = g(t - x/c) * transverse profile."""
        P = self.P
        L = P.laser
        if c != L.pol_axis:
            return None
        # transverse coordinates of the E_c points (relative to the box centre)
        coords = []
        for dd in (1, 2):
            if dd >= self.D:
                coords.append(np.zeros(1))
                continue
            s = sl_p[dd]
            idx = np.arange(s.start - G, s.stop - G, dtype=np.float64)
            if self.stE[c][dd]:
                idx = idx + 0.5
            coords.append(idx * P.dx[dd] - 0.5 * P.n[dd] * P.dx[dd])
        y = coords[0].reshape(1, -1, 1)
        z = coords[1].reshape(1, 1, -1)
        T = P.transverse_profile(y, z)
        t0 = n * P.dt
        t1 = (n + 1) * P.dt
        sx = P.dx[0] / C
        g = L.field(np.array([t0, t1, t0 - sx, t1 - sx]))
        return T, g

    def _mur(self, old, n):
        P = self.P
        E = self.E
        for d in (2, 1, 0):
            if d >= self.D or P.periodic[d]:
                continue
            k = P.kmur[d]
            for c in range(3):
                if self.stE[c][d]:
                    continue          # component normal to this face: interior update
                for sl_p, sl_q, is_min in self._face_points(c, d):
                    if d == 0 and is_min:
                        inc = self._inc(c, sl_p, sl_q, n)
                    else:
                        inc = None
                    if inc is None:
                        E[c][sl_p] = old[c][sl_q] + k * (E[c][sl_q] - old[c][sl_p])
                    else:
                        T, g = inc
                        ip0, ip1, iq0, iq1 = g[0] * T, g[1] * T, g[2] * T, g[3] * T
                        E[c][sl_p] = ip1 + (old[c][sl_q] - iq0) + k * (
                            (E[c][sl_q] - iq1) - (old[c][sl_p] - ip0))

    def _poynting(self, E_n, b_half):
        """Energy carried through the flux surface during the step.  The surface
        bounds the inner box whose faces are the node planes one cell inside the
        outflow faces (periodic axes: the whole period).  On the face normal to
        an outflow axis d, the Poynting vector S = E x H = eps0 c (E x b) (b = c B)
        is taken with E at the half step, (E^n + E^{n+1}) / 2, and b^{n+1/2}
        averaged to the plane from its two half-staggered neighbours along d, and
        integrated over the face by the trapezoid rule on the inner box's extent
        along the other axes (cell area dA; absent axes count 1 m).  Each point's
        S dt dA adds to the energy entering (S pointing into the box) or leaving."""
        P = self.P
        for d in range(self.D):
            if P.periodic[d]:
                continue
            a, b_ = (d + 1) % 3, (d + 2) % 3
            area = 1.0
            for e in range(self.D):
                if e != d:
                    area *= P.dx[e]
            for plane, inward in ((1, 1.0), (P.n[d] - 1, -1.0)):
                tot_in = tot_out = 0.0
                for ce, cb, sign in ((a, b_, 1.0), (b_, a, -1.0)):
                    # positions of E_ce on the face (those of b_cb coincide across it)
                    sl, sl_lo, wts = [], [], []
                    for e in range(3):
                        if e == d:
                            sl.append(slice(G + plane, G + plane + 1))
                            sl_lo.append(slice(G + plane - 1, G + plane))
                            wts.append(np.ones(1))
                        elif e >= self.D:
                            sl.append(slice(0, 1))
                            sl_lo.append(slice(0, 1))
                            wts.append(np.ones(1))
                        elif P.periodic[e]:
                            sl.append(slice(G, G + P.n[e]))
                            sl_lo.append(slice(G, G + P.n[e]))
                            wts.append(np.ones(P.n[e]))
                        elif self.stE[ce][e]:            # half-staggered: j + 1/2, 1 <= j <= n - 2
                            sl.append(slice(G + 1, G + P.n[e] - 1))
                            sl_lo.append(slice(G + 1, G + P.n[e] - 1))
                            wts.append(np.ones(P.n[e] - 2))
                        else:                            # nodes 1 .. n - 1, ends weighted 1/2
                            sl.append(slice(G + 1, G + P.n[e]))
                            sl_lo.append(slice(G + 1, G + P.n[e]))
                            w = np.ones(P.n[e] - 1)
                            w[0] = w[-1] = 0.5
                            wts.append(w)
                    wgt = wts[0][:, None, None] * wts[1][None, :, None] * wts[2][None, None, :]
                    e_half = 0.5 * (E_n[ce][tuple(sl)] + self.E[ce][tuple(sl)])
                    b_node = 0.5 * (b_half[cb][tuple(sl_lo)] + b_half[cb][tuple(sl)])
                    flux = inward * sign * EPS0 * C * e_half * b_node * wgt * area * P.dt
                    tot_in += float(np.sum(np.maximum(flux, 0.0)))
                    tot_out += float(np.sum(np.maximum(-flux, 0.0)))
                self.energy_in += tot_in
                self.energy_out += tot_out

    def node_emag(self):
        """|E| at grid nodes from the Yee components averaged to the node."""
        comps = []
        for c in range(3):
            e = self.E[c]
            self._fill_periodic(e)
            if c < self.D:
                e = 0.5 * (np.roll(e, 1, axis=c) + e)
            comps.append(e)
        m = np.sqrt(comps[0] ** 2 + comps[1] ** 2 + comps[2] ** 2)
        m[~self.domain_nodes] = 0.0
        return m

    # -------------------------------------------------------------- particles
    def _stencil(self, pos, st):
        """Per-dimension (indices, weights) for gathering a component with stagger st."""
        P = self.P
        out = []
        for d in range(3):
            if d >= self.D:
                out.append((np.zeros((len(pos), 1), dtype=np.int64), np.ones((len(pos), 1))))
                continue
            x = pos[:, d] - (0.5 if st[d] else 0.0)
            base, w = shape_weights(x, P.order)
            idx = base[:, None] + np.arange(w.shape[1])[None, :] + G
            out.append((idx, w))
        return out

    def gather(self, F, pos, st):
        if any(self.P.periodic):
            self._fill_periodic(F)
        (ix, wx), (iy, wy), (iz, wz) = self._stencil(pos, st)
        val = np.zeros(len(pos))
        for a in range(wx.shape[1]):
            for b_ in range(wy.shape[1]):
                for c in range(wz.shape[1]):
                    val += wx[:, a] * wy[:, b_] * wz[:, c] * F[ix[:, a], iy[:, b_], iz[:, c]]
        return val

    def _kind_arrays(self, pk, key):
        return np.array([k[key] for k in self.P.kinds])[pk] if len(pk) else np.zeros(0)

    def push_and_deposit(self):
        P = self.P
        self._ensure_ids()
        for Jc in self.J:
            Jc[...] = 0.0
        n = len(self.px)
        if n == 0:
            return
        pos = self.px
        Eg = [self.gather(self.E[c], pos, self.stE[c]) for c in range(3)]
        Bg = [self.gather(self.b[c], pos, self.stB[c]) for c in range(3)]
        h = self._kind_arrays(self.pk, "h")
        E = np.stack(Eg, axis=1)
        B = np.stack(Bg, axis=1)
        # relativistic Boris rotation with b = cB and u = gamma v / c
        um = self.pu + h[:, None] * E
        gm = np.sqrt(1.0 + np.sum(um * um, axis=1))
        t = (h / gm)[:, None] * B
        s = 2.0 * t / (1.0 + np.sum(t * t, axis=1))[:, None]
        up = um + np.cross(um + np.cross(um, t), s)
        u_new = up + h[:, None] * E
        g_new = np.sqrt(1.0 + np.sum(u_new * u_new, axis=1))
        x1 = pos.copy()
        for d in range(self.D):
            x1[:, d] = pos[:, d] + P.Cd[d] * u_new[:, d] / g_new
        self._esirkepov(pos, x1, u_new, g_new, self._kind_arrays(self.pk, "qhat"))
        for Jc in self.J:
            self._fold_periodic(Jc)
        keep = np.ones(n, dtype=bool)
        for d in range(self.D):
            nd = P.n[d]
            if P.periodic[d]:
                x1[:, d] = np.where(x1[:, d] < 0, x1[:, d] + nd, x1[:, d])
                x1[:, d] = np.where(x1[:, d] >= nd, x1[:, d] - nd, x1[:, d])
            else:
                keep &= (x1[:, d] >= 0) & (x1[:, d] < nd)
        self.px = x1[keep]
        self.pu = u_new[keep]
        self.pk = self.pk[keep]
        self.pid = self.pid[keep]

    def _esirkepov(self, x0, x1, u, g, qhat):
        P = self.P
        order = P.order
        lo = 2 if order == 2 else 1
        L = 5 if order == 2 else 4
        Np = len(x0)
        S0, DS, ref = [], [], []
        for d in range(3):
            if d >= self.D:
                S0.append(np.ones((Np, 1)))
                DS.append(np.zeros((Np, 1)))
                ref.append(np.zeros(Np, dtype=np.int64))
                continue
            r = (np.floor(x0[:, d] + 0.5) if order == 2 else np.floor(x0[:, d])).astype(np.int64)
            b0, w0 = shape_weights(x0[:, d], order)
            b1, w1 = shape_weights(x1[:, d], order)
            s0 = np.zeros((Np, L))
            s1 = np.zeros((Np, L))
            rows = np.arange(Np)[:, None]
            s0[rows, (b0 - r + lo)[:, None] + np.arange(order + 1)[None, :]] = w0
            s1[rows, (b1 - r + lo)[:, None] + np.arange(order + 1)[None, :]] = w1
            S0.append(s0)
            DS.append(s1 - s0)
            ref.append(r - lo)
        # path-averaged transverse shape products (Esirkepov's W without DS_d)
        def wbar(a, b_):
            return (S0[a][:, :, None] * S0[b_][:, None, :]
                    + 0.5 * DS[a][:, :, None] * S0[b_][:, None, :]
                    + 0.5 * S0[a][:, :, None] * DS[b_][:, None, :]
                    + (1.0 / 3.0) * DS[a][:, :, None] * DS[b_][:, None, :])
        Wb = [wbar(1, 2)[:, None, :, :], wbar(0, 2)[:, :, None, :], wbar(0, 1)[:, :, :, None]]
        shp = (Np, S0[0].shape[1], S0[1].shape[1], S0[2].shape[1])
        # local index grids -> global array indices
        ax = [ref[d][:, None] + np.arange(shp[d + 1])[None, :] + self.off[d] for d in range(3)]
        IX = ax[0][:, :, None, None]
        IY = ax[1][:, None, :, None]
        IZ = ax[2][:, None, None, :]
        flat = np.ravel_multi_index(np.broadcast_arrays(IX, IY, IZ), self.S, mode="raise")
        for d in range(3):
            if d < self.D:
                dsd = DS[d].reshape([Np] + [shp[k + 1] if k == d else 1 for k in range(3)])
                W = dsd * Wb[d]
                Jd = -(qhat * P.dx[d])[:, None, None, None] * np.cumsum(W, axis=d + 1)
            else:
                disp = P.Cd[0] * P.dx[0] * u[:, d] / g     # c dt u_d / gamma [m]
                Jd = (qhat * disp)[:, None, None, None] * np.broadcast_to(Wb[d], shp)
            Jd = np.broadcast_to(Jd, shp)
            self.J[d] += np.bincount(flat.ravel(), weights=Jd.ravel(),
                                     minlength=self.J[d].size).reshape(self.S)

    def charge_density(self):
        """rho/eps0 at nodes [V/m^2] from the charged particles (node shape)."""
        rho = np.zeros(self.S)
        if len(self.px) == 0:
            return rho
        qhat = self._kind_arrays(self.pk, "qhat")
        (ix, wx), (iy, wy), (iz, wz) = self._stencil(self.px, [False] * 3)
        for a in range(wx.shape[1]):
            for b_ in range(wy.shape[1]):
                for c in range(wz.shape[1]):
                    np.add.at(rho, (ix[:, a], iy[:, b_], iz[:, c]), qhat * wx[:, a] * wy[:, b_] * wz[:, c])
        self._fold_periodic(rho)
        return rho

    # ------------------------------------------------------------ ionization
    def ionize(self, step):
        P = self.P
        alive = np.nonzero(self.nalive)[0]
        if len(alive) == 0:
            return
        Ap = self.gather(self.A, self.npos[alive], [False] * 3)
        mats = self.nmat[alive]
        acut = np.array(self.acut)[mats]
        act = Ap >= acut
        if not np.any(act):
            return
        idx = alive[act]
        Aa = Ap[act]
        Pp = np.zeros(len(idx))
        for mi, mt in enumerate(P.mats):
            sel = self.nmat[idx] == mi
            if np.any(sel):
                W = keldysh.keldysh_rate(Aa[sel], mt.gap_eV, mt.mred, P.laser.lam, terms=P.terms,
                                         tol_bits=P.tol_bits)
                Pp[sel] = -np.expm1(-W * P.dt / mt.n0)
        w = philox.draw32(P.seed, self.nid[idx], step, philox.PURPOSE_IONIZE)[0]
        # event iff (w + 1/2) 2^-32 < P, decided exactly in FP64
        ev = (w.astype(np.float64) + 0.5) < Pp * 4294967296.0
        if not np.any(ev):
            return
        eidx = idx[ev]
        self.nalive[eidx] = False
        self.ndeath[eidx] = step
        self.events.append((self.nid[eidx].copy(), step))
        mats_e = self.nmat[eidx]
        u = self.thermal_u(self.nid[eidx], mats_e)
        pos = self.npos[eidx]
        for mi in np.unique(mats_e):
            self.energy_gap += np.sum(mats_e == mi) * P.kinds[2 * mi]["weight"] * P.mats[mi].gap_eV * 1.602176634e-19
        self.px = np.concatenate([self.px, pos, pos])
        self.pu = np.concatenate([self.pu, u, u])
        self.pk = np.concatenate([self.pk, 2 * mats_e, 2 * mats_e + 1])
        self.pid = np.concatenate([self.pid, self.nid[eidx], self.nid[eidx]])

    # ------------------------------------------------------------------ step
    def placed_id_base(self):
        """First id of particles placed directly: cells x ppc (every neutral
        id, cell index x ppc + k, is below it)."""
        return int(np.prod([self.P.n[d] for d in range(self.D)])) * int(self.P.ppc)

    def _ensure_ids(self):
        if len(self.pid) != len(self.pk):
            self.pid = self.placed_id_base() + np.arange(len(self.pk), dtype=np.int64)

    def step(self):
        n = self.step_index
        self.push_and_deposit()
        E_n = [e.copy() for e in self.E]
        self._b_half()
        b_half = [b.copy() for b in self.b]
        self._e_full(n)
        self._poynting(E_n, b_half)
        self._b_half()
        em = self.node_emag()
        self.win.append(em)
        self.A = np.max(np.stack(self.win), axis=0)
        if self.imax_every > 0 and (n + 1) % self.imax_every == 0:
            self.imax = np.maximum(self.imax, em * em)
        self.ionize(n + 1)
        if self.P.collisions:
            collide.collide(self, n + 1)
        impact.impact(self, n + 1)
        self.step_index = n + 1
        if self.track_every > 0 and (n + 1) % self.track_every == 0:
            self._record_tracks(n + 1)

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()

    # ------------------------------------------------------------ diagnostics
    def kinetic_energy(self, species=None):
        if len(self.px) == 0:
            return 0.0
        m = self._kind_arrays(self.pk, "mass")
        w = self._kind_arrays(self.pk, "weight")
        u2 = np.sum(self.pu * self.pu, axis=1)
        ke = m * C * C * u2 / (np.sqrt(1.0 + u2) + 1.0) * w
        if species is not None:
            sp = np.array([k["species"] for k in self.P.kinds])[self.pk]
            ke = ke[sp == species]
        return float(np.sum(ke))

    def field_energy(self):
        """Discrete field energy  sum (eps0/2)(|E|^2/ie + |b|^2) V_cell  [J]."""
        tot = 0.0
        for c in range(3):
            r = self.regE[c]
            ie = np.broadcast_to(self.ieE[c], self.S)
            tot += np.sum(self.E[c][self._domain_slices(self.stE[c])] ** 2
                          / ie[self._domain_slices(self.stE[c])])
            tot += np.sum(self.b[c][self.regB[c]] ** 2)
        return 0.5 * EPS0 * tot * self.P.vcell

    def _domain_slices(self, st):
        sl = []
        for d in range(3):
            if d >= self.D:
                sl.append(slice(0, 1))
                continue
            n = self.P.n[d]
            sl.append(slice(G, G + n + (0 if (self.P.periodic[d] or st[d]) else 1)))
        return tuple(sl)

    def gauss_residual(self):
        """div(E/ie + Q + chi3 E^3) - rho/eps0 at interior nodes [V/m^2] (Sec. 2.3
        medium; Q = P/eps0 of a Lorentz medium, chi3 the Kerr response, zero
        elsewhere)."""
        P = self.P
        div = np.zeros(self.S)
        for c in range(self.D):
            D_ = (self.E[c] / np.broadcast_to(self.ieE[c], self.S) + self.Q[c]
                  + np.broadcast_to(self.chiE[c], self.S) * self.E[c] ** 3)
            self._fill_periodic(D_)
            div += (D_ - np.roll(D_, 1, axis=c)) / P.dx[c]
        res = div - self.charge_density()
        sl = []
        for d in range(3):
            if d >= self.D:
                sl.append(slice(0, 1))
            elif P.periodic[d]:
                sl.append(slice(G, G + P.n[d]))
            else:
                sl.append(slice(G + 1, G + P.n[d]))
        return res[tuple(sl)]

    def density_grid(self, species="e"):
        """Number density [m^-3] at nodes by the particle shape (Sec. 4.1)."""
        out = np.zeros(self.S)
        if len(self.px) == 0:
            return out
        sp = np.array([k["species"] for k in self.P.kinds])[self.pk]
        sel = sp == species
        pos = self.px[sel]
        w = self._kind_arrays(self.pk[sel], "weight")
        (ix, wx), (iy, wy), (iz, wz) = self._stencil(pos, [False] * 3)
        for a in range(wx.shape[1]):
            for b_ in range(wy.shape[1]):
                for c in range(wz.shape[1]):
                    np.add.at(out, (ix[:, a], iy[:, b_], iz[:, c]), w * wx[:, a] * wy[:, b_] * wz[:, c])
        self._fold_periodic(out)
        return out / self.P.vcell

    def energy_density_grid(self, species="e"):
        """Kinetic energy density [J/m^3] at nodes (Sec. 4.2: the number density
        times the mean energy): sum_p w_p KE_p S(x_i - x_p) / V_cell with the
        node shape of the number density and KE = m c^2 |u|^2 / (gamma + 1)."""
        out = np.zeros(self.S)
        if len(self.px) == 0:
            return out
        sp = np.array([k["species"] for k in self.P.kinds])[self.pk]
        sel = sp == species
        pos = self.px[sel]
        w = self._kind_arrays(self.pk[sel], "weight")
        m = self._kind_arrays(self.pk[sel], "mass")
        u2 = np.sum(self.pu[sel] * self.pu[sel], axis=1)
        ke = m * C * C * u2 / (np.sqrt(1.0 + u2) + 1.0)
        (ix, wx), (iy, wy), (iz, wz) = self._stencil(pos, [False] * 3)
        for a in range(wx.shape[1]):
            for b_ in range(wy.shape[1]):
                for c in range(wz.shape[1]):
                    np.add.at(out, (ix[:, a], iy[:, b_], iz[:, c]), w * ke * wx[:, a] * wy[:, b_] * wz[:, c])
        self._fold_periodic(out)
        return out / self.P.vcell

    def set_imax(self, every):
        """Maximum accumulated intensity (Sec. 5, multilayer mirror: the
        intensity recorded at fixed intervals and the largest value over all of
        them kept per point).  From now on, after the field update of every step
        whose new step index is a multiple of `every`, each node's |E|^2 (the
        Yee components averaged to the node, as for the amplitude window) raises
        the node's running maximum; 0 switches it off.  The maximum restarts
        from zero."""
        self.imax_every = int(every)
        self.imax = np.zeros(self.S)

    def set_tracks(self, fraction, every):
        """Trajectory sampling (Sec. 5: tracks of a random 2 % of the
        electrons).  A particle is sampled iff the first word of the Philox
        block (seed; particle id, 0, TRACK) is below floor(fraction 2^32), so an
        electron and its positive carrier are sampled together and the choice
        does not depend on the particle's slot.  After every step whose new step
        index is a multiple of `every` (0 = off), each sampled live particle's
        (id, kind, step, position in cells) is recorded."""
        self.track_every = int(every)
        self.track_thr = int(math.floor(float(fraction) * 2.0 ** 32))
        self.tracks = []

    def _record_tracks(self, step):
        self._ensure_ids()
        if len(self.pid) == 0:
            return
        w = philox.draw32(self.P.seed, self.pid, 0, philox.PURPOSE_TRACK)[0]
        sel = np.nonzero(w.astype(np.int64) < self.track_thr)[0]
        for q in sel:
            self.tracks.append((int(self.pid[q]), int(self.pk[q]), int(step),
                                float(self.px[q, 0]), float(self.px[q, 1]), float(self.px[q, 2])))

    def imax_nodes(self):
        """The running maximum of |E|^2 [V^2/m^2] on the domain nodes."""
        return self.imax[self._domain_slices([False] * 3)].copy()

    def kinetic_energy_eV(self):
        """Kinetic energy of every charged particle [eV]:
        m c^2 |u|^2 / (gamma + 1) = m c^2 (gamma - 1) with gamma = sqrt(1 + |u|^2),
        u = gamma v / c; |u|^2 summed x, y, z in that order."""
        if len(self.px) == 0:
            return np.zeros(0)
        u = self.pu
        u2 = u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1] + u[:, 2] * u[:, 2]
        mc2 = np.array([k["mass"] * C * C / QE for k in self.P.kinds])[self.pk]
        return mc2 * u2 / (np.sqrt(1.0 + u2) + 1.0)

    def energy_spectrum(self, edges_eV, x_lo_cell=0, x_hi_cell=0):
        """Energy histogram of the charged macroparticles (Sec. 5: histograms of
        the electrons' energy in one layer at a given time, fitted with a chi^2
        law).  Counts per kind (row = kind index, 2 m electron, 2 m + 1 positive
        carrier of material m) of the particles whose x cell lies in
        [x_lo_cell, x_hi_cell) (every cell when x_hi_cell <= x_lo_cell), by
        kinetic energy against the increasing bin edges: column 0 below the
        first edge, column j in [edges[j-1], edges[j]), the last column at or
        above the last edge."""
        edges = np.asarray(edges_eV, dtype=np.float64)
        out = np.zeros((len(self.P.kinds), len(edges) + 1), dtype=np.int64)
        if len(self.px) == 0:
            return out
        cell = np.floor(self.px[:, 0]).astype(np.int64)
        sel = np.ones(len(cell), dtype=bool)
        if x_hi_cell > x_lo_cell:
            sel = (cell >= x_lo_cell) & (cell < x_hi_cell)
        col = np.searchsorted(edges, self.kinetic_energy_eV()[sel], side="right")
        np.add.at(out, (self.pk[sel], col), 1)
        return out

    def event_set(self):
        s = set()
        for ids, st in self.events:
            s.update(zip(ids.tolist(), [st] * len(ids)))
        return s

    def interior_field(self, which, c):
        """Field component on its domain positions (no guards)."""
        F = (self.E if which == "E" else self.b)[c]
        st = (self.stE if which == "E" else self.stB)[c]
        return F[self._domain_slices(st)].copy()
