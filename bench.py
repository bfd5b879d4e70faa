"""Benchmark of the laser-dielectric PIC hot path on one MI355X.

Workload (default): the 2D3V slab run -- 2048 x 512 cells at lambda/32, a 2 um
silica-like slab (n = 1.45, 9 eV) across y with 16 neutral macroparticles per
cell, a 3-cycle 800 nm pulse with a 3 um waist at 5e13 W/cm^2, seed 1.  One
step is one pass of the whole hot path (gather, Boris push, Esirkepov deposit,
Yee update with the dielectric, amplitude window, Keldysh ionization and
births).  The timed region is K steps from t = 0 of a fresh run, inputs
resident in HBM; W warmup steps run first on a separate instance.

Metric: particle-steps/s = sum over steps of (charged + alive neutral
macroparticles) / wall time.  Prints one JSON line.  Extra objects:
  roofline     -- the dominant kernel's algorithmic HBM bytes per launch over
                  its mean launch time (HIP events on the kernel's stream)
  cpu_baseline -- the FP64 oracle on a bounded sample of the same workload
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# phases of the step (index into the library's timers)
PHASES = {0: "push", 1: "fields", 2: "ionize", 3: "sort"}


def window_nodes(cfg):
    """Nodes of the amplitude window: material x-range +-1 node, whole transverse."""
    import numpy as np
    D = cfg["ndim"]
    dx = cfg["dx"][0]
    nx = cfg["n"][0]
    cells = [i for i in range(nx)
             if any(lo <= (i + 0.5) * dx < hi for (_, lo, hi) in cfg["layers"])]
    if not cells:
        return 0
    wx = min(nx, cells[-1] + 2) - max(0, cells[0] - 1) + 1
    per = cfg.get("transverse_bc", "outflow") == "periodic"
    t = 1
    for d in range(1, D):
        t *= cfg["n"][d] + (0 if per else 1)
    return int(np.int64(wx) * t)


def phase_bytes(cfg, phase, n_charged_avg, n_alive_avg):
    """Algorithmic HBM bytes of one launch of a phase (FP32 SoA layout)."""
    D = cfg["ndim"]
    per = cfg.get("transverse_bc", "outflow") == "periodic"
    cells = 1
    for d in range(D):
        cells *= cfg["n"][d] + (0 if (per and d > 0) else 1)
    if phase == 1:
        # Yee step: read E, b, J (36 B), write E, b (24 B), clear J (12 B);
        # window node: ring write, prefix read+write, suffix read, A write (20 B)
        # plus the once-per-cycle suffix rebuild (8 B amortised)
        return 72.0 * cells + 28.0 * window_nodes(cfg)
    if phase == 0:           # charged particle: read cell, offsets, u, kind; write back
        rd = 4 + 4 * D + 12 + 1
        wr = 4 + 4 * D + 12
        return float(rd + wr) * n_charged_avg
    if phase == 2:           # alive neutral: offsets (+ alive bit)
        return (4.0 * D + 0.125) * n_alive_avg
    return 0.0


def run_gpu(cfg, steps, warmup):
    import torch
    from paper_2502_13695_amd import pic
    torch.cuda.set_device(0)
    if warmup > 0:
        w = pic.Context(cfg)
        w.step(warmup)
        w.scalars()
        w.close()
    ctx = pic.Context(cfg)
    tune = ctx.autotune(10) if cfg.get("preionize_eV", 0.0) <= 0 else None
    ctx.set_timing(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timers = ctx.timers()
    sort_state = ctx.sort_state()
    sc = ctx.scalars()
    ev = ctx.events()
    nneut = ctx.params().n_neutral
    ctx.close()
    # particle-steps: each neutral counts until its ionization step, each birth
    # pair from its step to the end (carriers leaving the box are not subtracted)
    if len(ev):
        death = ev[:, 1]
        dead_steps = float(sum(min(int(s), steps) for s in death))
        births = float(sum(2 * max(0, steps - int(s)) for s in death))
        neutral_steps = dead_steps + (nneut - len(death)) * steps
    else:
        births = 0.0
        neutral_steps = float(nneut) * steps
    ps = neutral_steps + births
    wall = t1 - t0
    return dict(wall=wall, particle_steps=ps, neutral_steps=neutral_steps, charged_steps=births,
                timers=timers, scalars=sc, nneut=nneut, tune=tune, sort_state=sort_state)


def cpu_baseline(cfg, budget_s=20.0):
    """The FP64 oracle (as it stands) on the first steps of the same run."""
    from oracle import pic as OP
    t0 = time.perf_counter()
    sim = OP.Sim(cfg)
    t_init = time.perf_counter() - t0
    n = 0
    ps = 0.0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        sim.step()
        n += 1
        ps += float(len(sim.px) + int(sim.nalive.sum()))
    dt = time.perf_counter() - t0
    cores = 1
    try:
        import numpy as np  # noqa: F401
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return dict(value=ps / dt, unit="particle-steps/s", cores=cores, kind="oracle",
                sample=f"first {n} steps of the same run from t=0 (init {t_init:.1f} s excluded), "
                       f"FP64 NumPy, in-situ Keldysh rate; numpy may use multiple BLAS threads "
                       f"but the hot loops are single-threaded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="slab2d", choices=["slab2d", "mirror3d", "slab1d",
                                                             "stress2d", "stress3d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 256 MiB once before the run (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); multi-GPU runs are not "
              f"part of this build", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    if args.workload == "slab2d":
        cfg = W.config_2d()
        wl = dict(workload="2D3V silica slab, 2048x512 cells at lambda/32, 16 ppc, 3-cycle 5e13 W/cm^2 "
                           "pulse, w0 3 um", cells=[2048, 512], ppc=16, planned_steps=4000, seed=1)
    elif args.workload == "mirror3d":
        cfg = W.config_3d()
        wl = dict(workload="3D3V multi-layer mirror share, 256x128x128 cells at lambda/24, 8 ppc, "
                           "2-cycle 1 J/cm^2 plane wave", cells=[256, 128, 128], ppc=8,
                  planned_steps=2000, seed=2)
    elif args.workload == "slab1d":
        cfg = W.config_1d()
        wl = dict(workload="1D3V slab, 1024 cells at lambda/40, 100 ppc, 2-cycle 1e13 W/cm^2",
                  cells=[1024], ppc=100, planned_steps=2000, seed=0)
    elif args.workload == "stress2d":
        cfg = W.config_stress(W.config_2d(), eV=2.0)
        wl = dict(workload="2D3V slab, all neutrals pre-ionized (charged-loop stress)", cells=[2048, 512],
                  ppc=16, seed=1)
    else:
        cfg = W.config_stress(W.config_3d(), eV=2.0)
        wl = dict(workload="3D3V mirror share, all neutrals pre-ionized (charged-loop stress)",
                  cells=[256, 128, 128], ppc=8, seed=2)
    cfg = dict(cfg, nsteps=max(cfg["nsteps"], args.steps))
    if args.calib_copy:
        import torch
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    r = run_gpu(cfg, args.steps, args.warmup)
    value = r["particle_steps"] / r["wall"]
    timers = r["timers"]
    # dominant kernel by device time
    tot = {ph: timers[ph] for ph in PHASES if timers[8 + ph] > 0}
    dom = max((ph for ph in tot if ph != 3), key=tot.get)
    n_launch = timers[8 + dom]
    avg_ms = timers[dom] / n_launch
    n_charged_avg = r["charged_steps"] / args.steps
    n_alive_avg = r["neutral_steps"] / args.steps
    bytes_launch = phase_bytes(cfg, dom, n_charged_avg, n_alive_avg)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    step_ms = r["wall"] / args.steps * 1e3
    out = {
        "metric": "particle-steps/sec (gather+push+deposit+ionize) at 1 GPU",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(wl, neutrals=r["nneut"], charged_final=r["scalars"]["n_e"] + r["scalars"]["n_pos"],
                       events=r["scalars"]["events"], particle_steps=r["particle_steps"]),
        "roofline": {"bound": "hbm", "kernel": PHASES[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bytes_launch, "avg_launch_us": avg_ms * 1e3},
        "phases_us_per_step": {PHASES[ph]: timers[ph] / args.steps * 1e3 for ph in tot},
        "phases_us_per_launch": {PHASES[ph]: timers[ph] / max(timers[8 + ph], 1) * 1e3 for ph in tot},
        "field_tile_autotune": r["tune"],
        "tile_sort": r["sort_state"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
