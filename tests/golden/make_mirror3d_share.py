"""Writes tests/golden/mirror3d_share_2000.npz: the FP64 oracle's state after
2000 steps of the 3D mirror share reduced transversely to 256 x 16 x 16 cells
(periodic, plane wave: every transverse column evolves alike, so the share
carries the full run's per-column physics), seed 2, 8 neutrals per cell,
1 J/cm^2.  Calls only the oracle and the shared workload generator.

Stored: E and b on their own positions after 1000 steps (the layers' plasma
formed, the pulse reflected) and after 2000 (FP32: rounding 6e-8, far below
the 1e-5 field tolerance), the ionization events (neutral id, step), the
electron number and energy density grids at the nodes (FP32), and the
scalars the GPU run is compared with.  Takes about half an hour of one CPU
core.

Usage: python tests/golden/make_mirror3d_share.py
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W          # noqa: E402
from oracle import pic as OP   # noqa: E402

NSTEPS = 2000
MID = 1000


def main():
    cfg = W.config_3d(ny=16, nz=16, nsteps=NSTEPS)
    sim = OP.Sim(cfg)
    t0 = time.perf_counter()
    out = {}
    for s in range(NSTEPS):
        sim.step()
        if s + 1 == MID:
            for c in range(3):
                out[f"E{c}_{MID}"] = sim.interior_field("E", c).astype(np.float32)
                out[f"b{c}_{MID}"] = sim.interior_field("b", c).astype(np.float32)
        if (s + 1) % 100 == 0:
            print(f"step {s + 1}: {len(sim.px)} charged, {time.perf_counter() - t0:.0f} s", flush=True)
    ev = np.array(sorted(sim.event_set()), dtype=np.int64).reshape(-1, 2)
    sl = tuple(slice(OP.G, OP.G + n + (0 if (d > 0) else 1)) for d, n in enumerate(cfg["n"]))
    out.update(events=ev,
               ne=sim.density_grid("e")[sl].astype(np.float32),
               ue=sim.energy_density_grid("e")[sl].astype(np.float32),
               scalars=np.array([len(sim.px), float(np.sum(sim.pk % 2 == 0)), sim.kinetic_energy("e"),
                                 sim.kinetic_energy("p"), sim.energy_gap, sim.field_energy(), sim.energy_in,
                                 sim.energy_out, int(sim.nalive.sum())]))
    for c in range(3):
        out[f"E{c}"] = sim.interior_field("E", c).astype(np.float32)
        out[f"b{c}"] = sim.interior_field("b", c).astype(np.float32)
    np.savez_compressed(os.path.join(HERE, "mirror3d_share_2000.npz"), **out)
    print("written", len(ev), "events")


if __name__ == "__main__":
    main()
