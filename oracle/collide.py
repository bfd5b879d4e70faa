"""Binary Coulomb collisions between charged macroparticles (FP64, scalar).

TEST INFRASTRUCTURE (part of the oracle).  Written for clarity, not speed:
plain Python loops over cells and pairs.

The paper (Sec. 2.2, Eq. 4) uses the Perez/Nanbu binary collision model of
its host code between all charged particles, with the collision frequency of
Eq. (4), nu = (q_a q_b)^2 n_b ln(Lambda) / (4 pi (eps0 mu)^2) / v_r^3, the
Coulomb logarithm computed automatically with a lower bound of 1, and a
low-temperature extension.  The paper gives no more; the published method it
names (Perez et al., Phys. Plasmas 19, 083104 (2012); Nanbu, Phys. Rev. E 55,
4642 (1997); Nanbu & Yonemura, J. Comput. Phys. 145, 639 (1998)) is
restated here, and every choice the paper leaves open is a reading (listed
with the design notes):

* pairing, per cell (the cell holding the particle after the push) and per
  step, after ionization: the particles of each kind in the cell ordered by a
  Philox key (counter (id, kind, step, 7)); each kind with itself (pairs
  (0,1), (2,3), ...; an odd count first makes the triangle (0,1), (1,2),
  (2,0), each with half the scattering parameter), kinds in ascending order;
  then every pair of kinds a < b: collision i = 0 .. max(Na, Nb) - 1 takes
  the (i mod Na)-th of a and the (i mod Nb)-th of b, in that order;
* the density in the scattering parameter: the kind's own for like kinds;
  min(Na, Nb) w_max / V for unlike kinds, and a particle is updated with
  probability w_other / w_max (Nanbu & Yonemura's weight rule);
* per collision one Philox block (counter (id, kind | kind' << 8 | r << 16,
  step, 8) of the first particle, r the round i // min(Na, Nb)): the deflection
  angle from its first word, the azimuth from its second, the weight rule
  from its third, each as (w + 1/2) 2^-32;
* relativistic kinematics of Perez et al.: centre-of-momentum frame, the
  scattering parameter s with the paper's Eq. (4) as its non-relativistic
  limit (s = nu dt), Nanbu's angle distribution through Perez's fit of A(s);
* the Coulomb logarithm per collision: max(1, ln(lambda_D / b_min)) with
  lambda_D^-2 = sum over the cell's kinds of n q^2 / (eps0 T), T = 2/3 of
  the kind's mean kinetic energy in the cell, b_min the larger of the
  classical distance q_a q_b / (4 pi eps0 mu v_rel^2) and hbar / (2 mu v_rel);
* low temperatures: s capped at (4 pi / 3)^(1/3) dt (m_a + m_b) v_rel /
  max(m_a n_a^(-1/3), m_b n_b^(-1/3)), the scattering of one mean free path.

Parity pins (tests/test_oracle_collide.py): energy and momentum conservation
of every collision; Nanbu's mean deflection <cos chi> = exp(-s) against the
fit; the slowing of a slow electron beam on heavy scatterers at the rate of
Eq. (4); the pairing counts (each particle's collisions per step) and the
independence of the particle order; the weight rule's update frequency.
"""

import math

import numpy as np

from .constants import C, EPS0, HBAR
from . import philox

PURPOSE_PAIR = 7
PURPOSE_SCATTER = 8

# Perez et al.'s fit of 1/A(s) on 0.1 <= s < 3 (coth A - 1/A = exp(-s))
_AINV = (0.0056958, 0.9560202, -0.508139, 0.47913906, -0.12788975, 0.02389567)


def cos_chi(s, U):
    """Deflection cosine for scattering parameter s and uniform U in (0, 1)."""
    if s < 0.1:
        return max(-1.0, 1.0 + s * math.log(U))
    if s < 6.0:
        if s < 3.0:
            ainv = sum(c * s ** k for k, c in enumerate(_AINV))
            A = 1.0 / ainv
        else:
            A = 3.0 * math.exp(-s)
            ainv = 1.0 / A
        return min(1.0, max(-1.0, ainv * math.log(math.exp(-A) + 2.0 * U * math.sinh(A))))
    return 2.0 * U - 1.0


def _unif(w):
    return (float(w) + 0.5) * 2.0 ** -32


def pair_kinematics(u1, u2, m1, m2):
    """Centre-of-momentum quantities of two particles (u = gamma v / c)."""
    g1 = math.sqrt(1.0 + float(np.dot(u1, u1)))
    g2 = math.sqrt(1.0 + float(np.dot(u2, u2)))
    bc = (m1 * u1 + m2 * u2) / (m1 * g1 + m2 * g2)        # beta of the CM frame
    bc2 = float(np.dot(bc, bc))
    gc = 1.0 / math.sqrt(1.0 - bc2)
    b1 = u1 / g1
    b2 = u2 / g2
    # particle 1's momentum in the CM frame, in units of kg m/s
    if bc2 > 0.0:
        p1s = m1 * C * (u1 + ((gc - 1.0) / bc2 * float(np.dot(bc, b1)) - gc) * g1 * bc)
    else:
        p1s = m1 * C * u1.copy()
    g1s = gc * g1 * (1.0 - float(np.dot(bc, b1)))
    g2s = gc * g2 * (1.0 - float(np.dot(bc, b2)))
    return g1, g2, bc, bc2, gc, p1s, g1s, g2s


def collide_pair(u1, u2, m1, m2, q1, q2, w1, w2, n, dt, lnL_of, cap_of, half, words):
    """One binary collision.  Returns the new (u1, u2).  lnL_of(mu, v_rel) and
    cap_of(v_rel) give the Coulomb logarithm and the low-temperature cap."""
    g1, g2, bc, bc2, gc, p1s, g1s, g2s = pair_kinematics(u1, u2, m1, m2)
    P = math.sqrt(float(np.dot(p1s, p1s)))
    if P == 0.0:
        return u1, u2
    mu = m1 * m2 / (m1 + m2)
    # relative speed: the two CM velocities composed
    v1s = P / (m1 * g1s)
    v2s = P / (m2 * g2s)
    vrel = (v1s + v2s) / (1.0 + v1s * v2s / (C * C))
    lnL = lnL_of(mu, vrel)
    s = (n * dt * lnL * (q1 * q2) ** 2 / (4.0 * math.pi * EPS0 ** 2 * C ** 4 * m1 * g1 * m2 * g2)
         * gc * P / (m1 * g1 + m2 * g2) * (m1 * g1s * m2 * g2s * C * C / (P * P) + 1.0) ** 2)
    s = min(s, cap_of(vrel))
    if half:
        s *= 0.5
    cchi = cos_chi(s, _unif(words[0]))
    schi = math.sqrt(max(0.0, 1.0 - cchi * cchi))
    phi = 2.0 * math.pi * _unif(words[1])
    cphi, sphi = math.cos(phi), math.sin(phi)
    px, py, pz = p1s
    pperp = math.sqrt(px * px + py * py)
    if pperp > 0.0:
        q = np.array([px * pz / pperp * schi * cphi - py * P / pperp * schi * sphi + px * cchi,
                      py * pz / pperp * schi * cphi + px * P / pperp * schi * sphi + py * cchi,
                      -pperp * schi * cphi + pz * cchi])
    else:
        q = np.array([P * schi * cphi, P * schi * sphi, pz * cchi])
    # back to the lab frame
    if bc2 > 0.0:
        f = (gc - 1.0) / bc2 * float(np.dot(bc, q))
        p1n = q + (f + m1 * C * g1s * gc) * bc
        p2n = -q + (-f + m2 * C * g2s * gc) * bc
    else:
        p1n, p2n = q, -q
    wmax = max(w1, w2)
    U3 = _unif(words[2])
    n1 = p1n / (m1 * C) if U3 < w2 / wmax else u1
    n2 = p2n / (m2 * C) if U3 < w1 / wmax else u2
    return n1, n2


def collide(sim, step):
    """Collisions of one step among the charged particles of ``sim`` (u updated)."""
    P = sim.P
    npart = len(sim.pk)
    if npart < 2:
        return
    sim._ensure_ids()
    D = sim.D
    V = P.vcell
    dt = P.dt
    kinds = P.kinds
    # cell of every particle (periodic positions are inside the box)
    cell = np.zeros(npart, dtype=np.int64)
    stride = 1
    for d in range(D):
        c = np.floor(sim.px[:, d]).astype(np.int64)
        c = np.clip(c, 0, P.n[d] - 1)
        cell += c * stride
        stride *= P.n[d]
    ids = sim.pid.astype(np.uint64)
    kk = sim.pk.astype(np.uint64)
    key = philox.draw32(P.seed, ids | (kk << np.uint64(32)), step, PURPOSE_PAIR)[0]
    order = np.lexsort((sim.pk, sim.pid, key, cell))
    bounds = np.flatnonzero(np.diff(cell[order])) + 1
    for grp in np.split(order, bounds):
        if len(grp) < 2:
            continue
        _collide_cell(sim, grp, step, V, dt, kinds)


def _collide_cell(sim, grp, step, V, dt, kinds):
    P = sim.P
    u = sim.pu
    present = sorted(set(int(k) for k in sim.pk[grp]))
    lists = {k: [int(i) for i in grp if sim.pk[i] == k] for k in present}   # key order
    # densities and temperatures of the cell's kinds
    dens, temp = {}, {}
    for k in present:
        L = lists[k]
        m = kinds[k]["mass"]
        ke = [(math.sqrt(1.0 + float(np.dot(u[i], u[i]))) - 1.0) * m * C * C for i in L]
        dens[k] = len(L) * kinds[k]["weight"] / V
        temp[k] = 2.0 / 3.0 * sum(ke) / len(L)
    inv_ld2 = sum(dens[k] * kinds[k]["q"] ** 2 / (EPS0 * temp[k]) for k in present if temp[k] > 0)

    def lnL_for(qa, qb):
        def f(mu, vrel):
            if inv_ld2 <= 0.0:
                return 1.0
            ld = 1.0 / math.sqrt(inv_ld2)
            bcl = abs(qa * qb) / (4.0 * math.pi * EPS0 * mu * vrel * vrel)
            bqm = HBAR / (2.0 * mu * vrel)
            return max(1.0, math.log(ld / max(bcl, bqm)))
        return f

    def cap_for(ka, kb):
        ma, mb = kinds[ka]["mass"], kinds[kb]["mass"]
        den = max(ma * dens[ka] ** (-1.0 / 3.0), mb * dens[kb] ** (-1.0 / 3.0))
        return lambda vrel: (4.0 * math.pi / 3.0) ** (1.0 / 3.0) * dt * (ma + mb) * vrel / den

    def one(i, j, ka, kb, n, half, r):
        ctr_hi = ka | (kb << 8) | (r << 16)
        words = philox.draw32(P.seed, np.array([int(sim.pid[i]) | (ctr_hi << 32)], dtype=np.uint64),
                              step, PURPOSE_SCATTER)
        words = [int(w[0]) for w in words]
        A, B = kinds[ka], kinds[kb]
        u[i], u[j] = collide_pair(u[i].copy(), u[j].copy(), A["mass"], B["mass"], A["q"], B["q"],
                                  A["weight"], B["weight"], n, dt, lnL_for(A["q"], B["q"]),
                                  cap_for(ka, kb), half, words)

    for k in present:
        L = lists[k]
        N = len(L)
        if N < 2:
            continue
        n = dens[k]
        start = 0
        if N % 2 == 1:
            if N == 1:
                continue
            one(L[0], L[1], k, k, n, True, 0)
            one(L[1], L[2], k, k, n, True, 0)
            one(L[2], L[0], k, k, n, True, 0)
            start = 3
        for a in range(start, N - 1, 2):
            one(L[a], L[a + 1], k, k, n, False, 0)
    for ia, ka in enumerate(present):
        for kb in present[ia + 1:]:
            La, Lb = lists[ka], lists[kb]
            Na, Nb = len(La), len(Lb)
            wmax = max(kinds[ka]["weight"], kinds[kb]["weight"])
            n = min(Na, Nb) * wmax / V
            nmin = min(Na, Nb)
            for i in range(max(Na, Nb)):
                one(La[i % Na], Lb[i % Nb], ka, kb, n, False, i // nmin)
