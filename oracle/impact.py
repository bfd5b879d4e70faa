"""Impact ionization of neutral molecules by hot electrons (FP64, scalar).

TEST INFRASTRUCTURE (part of the oracle).

The paper leaves impact ionization out of its runs and names Keldysh's
impact-ionization rate as the model to use in future work (Sec. 2.2).  That
rate, restated (Keldysh, Sov. Phys. JETP 10, 509 (1960); 21, 1135 (1965)):
an electron of kinetic energy eps above the threshold
    E_th = E_g (1 + 2 mu) / (1 + mu),   mu = m_e* / m_h*
(energy and crystal momentum conserved for parabolic bands) ionizes at
    w(eps) = P (eps / E_th - 1)^2,
P a material constant (`impact_rate_s`, 0 = off).  Readings (listed with the
design notes):

* per step, after photoionization and collisions, every electron in a cell of
  its own material (electron kind 2m in a cell of material m) takes one
  decision: an event iff (w + 1/2) 2^-32 < 1 - exp(-w(eps) dt), w the first
  word of Philox counter (id, kind, step, 9), eps its kinetic energy;
* within a cell the electrons decide in the cell's pairing order (kind, Philox
  key of counter (id, kind, step, 7), id); an event consumes the cell's alive
  neutral with the smallest index; with none left, nothing happens;
* the event is an ionization like a photoionization: the neutral dies at this
  step, an electron and a positive carrier are born at its position with its
  thermal velocity, the gap energy is paid; the impacting electron loses
  E_g of kinetic energy (direction kept), which keeps the energy balance (the
  electron and the neutral carry the same weight).

Parity pins (tests/test_oracle_impact.py): the threshold's limits (heavy
hole: E_g; equal masses: 3/2 E_g), the rate's zero, value P at 2 E_th and
quadratic growth; the event frequency at a fixed energy against
1 - exp(-w dt) (binomial, 5 sigma); the energy balance of every event; the
neutrals consumed lowest index first and never twice; independence of the
particle storage order.
"""

import math

import numpy as np

from .constants import C, QE
from . import philox
from .collide import PURPOSE_PAIR

PURPOSE_IMPACT = 9


def threshold_eV(mt):
    mu = mt.me_star / mt.mh_star
    return mt.gap_eV * (1.0 + 2.0 * mu) / (1.0 + mu)


def rate(mt, eps_eV):
    """Impact-ionization rate [1/s] of one electron of kinetic energy eps_eV."""
    if mt.impact_rate <= 0.0:
        return 0.0
    eth = threshold_eV(mt)
    if eps_eV <= eth:
        return 0.0
    x = eps_eV / eth - 1.0
    return mt.impact_rate * x * x


def impact(sim, step):
    P = sim.P
    if len(sim.pk) == 0 or not any(m.impact_rate > 0 for m in P.mats):
        return
    sim._ensure_ids()
    D = sim.D
    nx, ny = P.n[0], P.n[1]
    cellx = [np.clip(np.floor(sim.px[:, d]).astype(np.int64), 0, P.n[d] - 1) for d in range(D)]
    while len(cellx) < 3:
        cellx.append(np.zeros(len(sim.pk), dtype=np.int64))
    lin = cellx[0] + nx * (cellx[1] + ny * cellx[2])
    ids = sim.pid.astype(np.uint64)
    kk = sim.pk.astype(np.uint64)
    key = philox.draw32(P.seed, ids | (kk << np.uint64(32)), step, PURPOSE_PAIR)[0]
    order = np.lexsort((sim.pid, key, sim.pk, lin))
    U = philox.draw32(P.seed, ids | (kk << np.uint64(32)), step, PURPOSE_IMPACT)[0]
    taken = {}                       # cell -> index of the next neutral slot to look at
    births = []
    for i in order:
        k = int(sim.pk[i])
        if k % 2:
            continue
        m = k // 2
        ix = int(cellx[0][i])
        if P.mat_cell[ix] != m:
            continue
        mt = P.mats[m]
        if mt.impact_rate <= 0.0:
            continue
        u = sim.pu[i]
        mc2 = P.kinds[k]["mass"] * C * C
        ke = (math.sqrt(1.0 + float(np.dot(u, u))) - 1.0) * mc2
        w = rate(mt, ke / QE)
        if w <= 0.0:
            continue
        prob = -math.expm1(-w * P.dt)
        if not (float(U[i]) + 0.5 < prob * 4294967296.0):
            continue
        c = int(lin[i])
        first = int(np.searchsorted(sim.nid, c * P.ppc))
        q = taken.get(c, 0)
        while q < P.ppc and not (first + q < len(sim.nid) and sim.nid[first + q] == c * P.ppc + q
                                 and sim.nalive[first + q]):
            q += 1
        if q >= P.ppc:
            taken[c] = q
            continue
        taken[c] = q + 1
        j = first + q
        sim.nalive[j] = False
        sim.ndeath[j] = step
        births.append(j)
        # the impacting electron pays the gap
        ke2 = ke - mt.gap_eV * QE
        g2 = 1.0 + ke2 / mc2
        sim.pu[i] = u * (math.sqrt(g2 * g2 - 1.0) / math.sqrt(float(np.dot(u, u))))
    if not births:
        return
    b = np.array(births, dtype=np.int64)
    mats = sim.nmat[b]
    sim.events.append((sim.nid[b].copy(), step))
    for mi in np.unique(mats):
        sim.energy_gap += np.sum(mats == mi) * P.kinds[2 * mi]["weight"] * P.mats[mi].gap_eV * QE
    u = sim.thermal_u(sim.nid[b], mats)
    pos = sim.npos[b]
    sim.px = np.concatenate([sim.px, pos, pos])
    sim.pu = np.concatenate([sim.pu, u, u])
    sim.pk = np.concatenate([sim.pk, 2 * mats, 2 * mats + 1])
    sim.pid = np.concatenate([sim.pid, sim.nid[b], sim.nid[b]])
