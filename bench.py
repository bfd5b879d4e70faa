"""Benchmark of the laser-dielectric PIC hot path on one MI355X.

Workload (default, ``--workload mirror3d``): the 3D3V one-GPU share of the
multi-layer mirror -- 256 x 128 x 128 cells at lambda/24, eight alternating
quarter-wave layers (n = 1.45 with a 9 eV gap, n = 2.1 with a 4 eV gap) from
x = 64 cells, 8 neutral macroparticles per material cell (3.67e6), a 2-cycle
800 nm plane-wave pulse of 1 J/cm^2, periodic transverse boundaries, seed 2.

One step is one pass of the whole hot path: gather, Boris push, Esirkepov
deposit, Yee update with the dielectric, outflow faces and laser injection,
amplitude window, Keldysh ionization and births, and the tile sort when due.

Timed window: K = --steps steps starting at the interaction step S, the step
at which the pulse peak reaches the front of the first layer
(t_peak + x_front / c; reported as config.start_step, --start overrides).
Untimed before it: context set-up, the in-run timing of the field tile shapes
over the first 28 steps, the advance to step S - W and then W = --warmup more
steps.  Inputs are resident in HBM; the timed region is the K steps bracketed
by device synchronisations.

Metric: particle-steps/s = sum over the K steps of (charged + alive neutral
macroparticles at the start of the step) / wall time of the K steps.

Extra objects in the JSON line:
  roofline     -- the kernel with the most device time in the window: its
                  algorithmic bytes per launch (the per-unit bytes below times
                  the units one launch processes) over its mean launch time,
                  from HIP events stamped by the dispatches of every step of
                  the window on the context's stream
  cpu_baseline -- the FP64 oracle pinned to one host core, on the same window
                  of the workload's transverse share (see cpu_baseline)

Per-unit algorithmic bytes (FP32 SoA layout): a charged particle-step 60
(32 read, 28 written); an alive neutral-step 16, plus 64 per ionization event
(two births); a grid cell-step 73 (E, B, J and the material read; E, B
written; J cleared), 49 where no current can exist; plus 24 per amplitude-
window node-step; a sorted charged particle 120 (read and written once).
"""

import argparse
import ctypes
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec (gather+push+deposit+ionize) at 1 GPU"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
C_LIGHT = 299792458.0

# phases of the step (index into the library's timers)
PHASES = {0: "push", 1: "fields", 2: "ionize", 3: "sort", 4: "collide"}
# algorithmic bytes per unit of work
B_CHARGED, B_NEUTRAL, B_EVENT = 60.0, 16.0, 64.0
B_CELL, B_CELL_NO_J, B_WINDOW, B_SORTED = 73.0, 49.0, 24.0, 120.0
# binary collisions: per charged particle-step, binning (read cell and kind,
# write slot and key: 13), the cell pass (read slot, key, kind, id: 13; read and
# write u: 24) and 10 for the sort's moves; per cell-step the counts, fill
# counters and their scan (16)
B_COLLIDE, B_COLLIDE_CELL = 60.0, 16.0
# algorithmic flops per charged particle-step of the 3D order-2 push: gather
# 160, Boris 60, Esirkepov deposit 770
FLOP_PUSH_3D2 = 990.0
# steps of the in-run timing of the field tile shapes (7 shapes x 4 launches)
TUNE_REPS = 4
TUNE_STEPS = 8 * TUNE_REPS          # at most 8 field tile shapes, TUNE_REPS steps each


class Roctx:
    """roctxProfilerResume / Pause around the timed region, so that a profiler
    run with --selected-regions (which starts paused; a pause before the first
    resume is an error there) sees exactly the window's dispatches.  No-ops
    without a profiler; absent library: nothing happens."""

    def __init__(self):
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so",
                     "/opt/rocm/lib/librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(ctypes.c_uint64(0))

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(ctypes.c_uint64(0))


def window_nodes(cfg):
    """Nodes of the amplitude window: material x-range +-1 node, whole transverse."""
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
    return int(wx * t)


def domain_cells(cfg):
    """Grid cells of the field update (nodes along outflow axes, cells along periodic ones)."""
    per = cfg.get("transverse_bc", "outflow") == "periodic"
    cells = 1
    for d in range(cfg["ndim"]):
        cells *= cfg["n"][d] + (0 if (per and d > 0) else 1)
    return cells


def interaction_start(cfg, params):
    """Step at which the pulse peak reaches the front of the first layer."""
    if not cfg["layers"]:
        return 0
    x0 = min(lo for (_, lo, _) in cfg["layers"])
    return int(round((params.t_peak + x0 / C_LIGHT) / params.dt))


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or
    None when no summary exists or the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    src = os.path.join(ROOT, "paper_2502_13695_amd", "csrc", "pic_kernels.hip")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    ok = False
    for line in open(path):
        f = line.split()
        if len(f) >= 3 and f[0] == "#" and f[1] == "kernels_sha256":
            ok = f[2] == sha
        elif ok and len(f) >= 4 and f[0] == workload and f[1] == kernel:
            return float(f[2]) + float(f[3])
    return None


def stream_copy_gbs(mib=1024, reps=5):
    """Device-to-device copy bandwidth on this GPU (read + write bytes / s),
    the practical ceiling a streaming kernel is also compared with."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def window_counts(sc0, sc1, ev, start, steps):
    """Charged and alive-neutral particle-steps of steps start .. start+steps-1.
    A step counts the particles present when it starts; an event recorded with
    step index s (the ionization of step s - 1) adds two carriers from step s
    on.  Carriers that left the box during the window (rare: the layers are far
    from the outflow faces) are taken off at half the window."""
    import numpy as np
    charged0 = sc0["n_e"] + sc0["n_pos"]
    alive0 = sc0["n_neutral"]
    st = np.asarray(ev[:, 1], dtype=np.int64) if len(ev) else np.zeros(0, dtype=np.int64)
    win = st[(st > start) & (st <= start + steps)]
    later = float(np.sum(start + steps - win))      # steps each birth pair is present
    births = len(win)
    removed = max(0.0, charged0 + 2 * births - (sc1["n_e"] + sc1["n_pos"]))
    charged_steps = steps * charged0 + 2.0 * later - removed * steps / 2.0
    neutral_steps = steps * alive0 - later
    return dict(charged_steps=charged_steps, neutral_steps=neutral_steps, events=births,
                removed=removed, charged_start=charged0, alive_start=alive0,
                charged_end=sc1["n_e"] + sc1["n_pos"], alive_end=sc1["n_neutral"])


def run_window(cfg, start, steps, warmup, field_tile, roctx, resort=None):
    """The benchmark run: one context, untimed advance to the window, K timed
    steps with every dispatch stamped."""
    import torch
    from paper_2502_13695_amd import pic
    torch.cuda.set_device(0)
    ctx = pic.Context(cfg)
    if resort is not None:
        ctx.set_resort(resort)
    pre = start - warmup
    if field_tile is None:
        # field tile shapes timed in-run on the first steps (identical results)
        if pre < TUNE_STEPS:
            raise SystemExit(f"the window starts at step {start}: at least {TUNE_STEPS + warmup} "
                             f"steps are needed before it for the tile timing and the warmup")
        ctx.autotune_steps(TUNE_REPS)
    ctx.step(max(0, pre))
    ctx.step(start - max(0, pre))          # W warmup steps
    torch.cuda.synchronize()
    sc0 = ctx.scalars()
    reg0 = ctx.region()
    sort0 = ctx.sort_state()
    ctx.set_timing(1)                      # every dispatch of the window stamped
    torch.cuda.synchronize()
    roctx.resume()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    roctx.pause()
    timers = ctx.timers()
    sc1 = ctx.scalars()
    reg1 = ctx.region()
    sort1 = ctx.sort_state()
    ev = ctx.events()
    tune = dict(chosen=int(timers[23]), blocks=int(timers[24]),
                ms=[float(x) for x in timers[16:23]] + ([float(timers[26])] if timers[27] > 7 else []))
    ctx.close()
    assert sc1["health"] == 0, f"health word {sc1['health']}"
    return dict(wall=t1 - t0, timers=timers, sc0=sc0, sc1=sc1, reg0=reg0, reg1=reg1, sort0=sort0,
                sort1=sort1, ev=ev, tune=tune)


def phase_bytes(cfg, r, cnt, steps):
    """Algorithmic bytes per launch of each phase over the window."""
    timers = r["timers"]
    out = {}
    n_launch = {ph: max(1.0, timers[8 + ph]) for ph in PHASES}
    out[0] = B_CHARGED * cnt["charged_steps"] / n_launch[0]
    out[2] = (B_NEUTRAL * cnt["neutral_steps"] + B_EVENT * cnt["events"]) / n_launch[2]
    # field update: tiles updated per launch (device counter), near tiles with
    # current, the rest without; tiles beyond the field front move nothing
    reg0, reg1 = r["reg0"], r["reg1"]
    ntiles = max(1, reg1["near_tiles"] + reg1["far_tiles"])
    upd = (reg1["tiles_updated"] - reg0["tiles_updated"]) / max(1.0, timers[9])
    near = min(upd, 0.5 * (reg0["near_tiles"] + reg1["near_tiles"]))
    far_upd = max(0.0, upd - near)
    cells = domain_cells(cfg)
    out[1] = cells * (B_CELL * near + B_CELL_NO_J * far_upd) / ntiles + B_WINDOW * window_nodes(cfg)
    # tile sort: every slot read and written once per sort performed
    nsort = r["sort1"]["sorts"] - r["sort0"]["sorts"]
    slots = 0.5 * (cnt["charged_start"] + cnt["charged_end"])
    out[3] = B_SORTED * slots * nsort / n_launch[3]
    # binary collisions (when on): the charged slots binned by cell and their
    # momenta read and written, plus the per-cell counts and scan
    out[4] = (B_COLLIDE * cnt["charged_steps"] + B_COLLIDE_CELL * domain_cells(cfg) * steps) / n_launch[4]
    return out, dict(tiles=ntiles, updated_per_launch=upd, near=near, far_updated=far_upd,
                     sorts=nsort)


def _oracle_child(spec):
    """The oracle on the window, in this (pinned, single-threaded) process."""
    os.sched_setaffinity(0, {int(spec["cpu"])})
    from oracle import pic as OP
    cfg = spec["cfg"]
    t0 = time.perf_counter()
    sim = OP.Sim(cfg)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    while sim.step_index < spec["start"]:
        sim.step()
    t_ff = time.perf_counter() - t0
    n, ps = 0, 0.0
    charged = 0.0
    t0 = time.perf_counter()
    K = spec["steps"]
    while True:
        el = time.perf_counter() - t0
        if not ((n < K and el < 3 * spec["budget"]) or (el < spec["budget"] and n < 10 * K)):
            break
        c = float(len(sim.px))
        ps += c + float(sim.nalive.sum())
        charged += c
        sim.step()
        n += 1
    dt = time.perf_counter() - t0
    print(json.dumps(dict(steps=n, seconds=dt, particle_steps=ps, charged_steps=charged,
                          init_s=t_init, advance_s=t_ff, cpus=sorted(os.sched_getaffinity(0)))), flush=True)


def cpu_baseline(cfg, start, steps, budget_s, share_note):
    """The FP64 oracle (as it stands, untuned) on the same window, pinned to one
    host core with single-threaded numpy: a child process advances to `start`
    (untimed), then times the window's steps (and more while the time budget
    lasts, up to 10x the window)."""
    cpus = sorted(os.sched_getaffinity(0))
    spec = dict(cfg=cfg, start=start, budget=budget_s, steps=steps, cpu=cpus[-1])
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               NUMEXPR_NUM_THREADS="1")
    p = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-child", json.dumps(spec)],
                       env=env, capture_output=True, text=True, timeout=1800)
    if p.returncode != 0:
        raise RuntimeError(f"oracle child failed: {p.stderr[-2000:]}")
    res = json.loads(p.stdout.strip().splitlines()[-1])
    return dict(value=res["particle_steps"] / res["seconds"], unit="particle-steps/s", cores=1,
                kind="oracle",
                sample=f"steps {start}..{start + res['steps'] - 1} ({res['steps']} steps, "
                       f"{res['seconds']:.1f} s, {res['particle_steps'] / res['steps']:.3g} particles per step) "
                       f"of {share_note}; FP64 NumPy with in-situ Keldysh rates, one process pinned to "
                       f"host CPU {res['cpus']} with single-threaded BLAS; the advance to step {start} "
                       f"({res['advance_s']:.1f} s) and set-up ({res['init_s']:.1f} s) untimed",
                cpus_on_host=len(cpus))


def trace_summary(path, steps):
    """Per-kernel statistics of the timed window from a rocprofv3 kernel trace
    (kernel_trace.csv of a run of this script): the window is the span from
    the start of the last `steps` push dispatches (no push follows the window)
    to the end of the last ionization dispatch; every dispatch starting inside
    it is counted."""
    import csv
    rows = list(csv.DictReader(open(path)))
    for r in rows:
        r["t0"], r["t1"] = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
    rows.sort(key=lambda r: r["t0"])
    push = [r for r in rows if "k_push" in r["Kernel_Name"]]
    ion = [r for r in rows if "k_ionize" in r["Kernel_Name"]]
    if len(push) < steps or not ion:
        raise SystemExit(f"{path}: {len(push)} push dispatches, fewer than the window's {steps} steps")
    w0, w1 = push[-steps]["t0"], ion[-1]["t1"]
    stats = {}
    for r in rows:
        if w0 <= r["t0"] <= w1:
            name = r["Kernel_Name"].split("(")[0]
            s = stats.setdefault(name, [0, 0.0, 1e30, 0.0])
            d = (r["t1"] - r["t0"]) / 1e3
            s[0] += 1
            s[1] += d
            s[2] = min(s[2], d)
            s[3] = max(s[3], d)
    total = sum(v[1] for v in stats.values())
    lines = [f"window: {steps} steps, {(w1 - w0) / 1e6:.3f} ms from the first push of the window to the "
             f"end of the last ionization",
             "| kernel | calls | total us | avg us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for name, (n, tot, lo, hi) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {name} | {n} | {tot:.1f} | {tot / n:.2f} | {lo:.2f} | {hi:.2f} | {tot / total:.1%} |")
    return "\n".join(lines)


WORKLOADS = {
    "mirror3d": "3D3V multi-layer mirror share, 256x128x128 cells at lambda/24, 8 alternating quarter-wave "
                "layers (n 1.45 / 9 eV, n 2.1 / 4 eV), 8 ppc, 2-cycle 1 J/cm^2 plane wave, periodic transverse, "
                "seed 2",
    "slab2d": "2D3V silica slab, 2048x512 cells at lambda/32, 16 ppc, 3-cycle 5e13 W/cm^2 pulse, w0 3 um, seed 1",
    "slab1d": "1D3V slab, 1024 cells at lambda/40, 100 ppc, 2-cycle 1e13 W/cm^2, seed 0",
    "stress2d": "2D3V slab grid, every neutral pre-ionized at 2 eV (charged-loop stress), seed 1",
    "stress3d": "3D3V mirror-share grid, every neutral pre-ionized at 2 eV (charged-loop stress), seed 2",
    "stress2d-cap": "2D3V slab grid, 4.0e7 pre-ionized carriers (charged-loop stress at the particle cap)",
    "stress3d-cap": "3D3V mirror-share grid, 2.5e8 pre-ionized carriers (charged-loop stress at the particle cap)",
}


DISPERSIVE_NOTE = "; layers as single-pole Lorentz media (index at 800 nm unchanged)"


def workload_config(name, dispersive=False):
    """(benchmark configuration, oracle configuration for the CPU baseline, its description).
    dispersive: the layers respond as single-pole Lorentz media."""
    import workloads as W
    d = dict(dispersive=dispersive)
    if name == "mirror3d":
        cfg = W.config_3d(**d)
        # periodic transverse plane-wave run: every transverse column evolves
        # alike, so a 16 x 16 share carries the same per-particle work
        return cfg, W.config_3d(ny=16, nz=16, **d), "the 256x16x16 transverse share of the same run"
    if name == "slab2d":
        cfg = W.config_2d(**d)
        return cfg, cfg, "the same run"
    if name == "slab1d":
        cfg = W.config_1d(**d)
        return cfg, cfg, "the same run"
    if name == "stress2d":
        cfg = W.config_stress(W.config_2d(**d), eV=2.0)
        return cfg, W.config_stress(W.config_2d(ny=32, **d), eV=2.0), "a 2048x32 outflow strip of the same slab"
    if name == "stress3d":
        cfg = W.config_stress(W.config_3d(**d), eV=2.0)
        return cfg, W.config_stress(W.config_3d(ny=16, nz=16, **d), eV=2.0), "the 256x16x16 transverse share"
    if name == "stress2d-cap":
        # 488 neutrals per slab cell, all pre-ionized: 2 x 40960 x 488 = 4.0e7 charged
        return W.config_stress(W.config_2d(ppc=488, **d), eV=2.0), None, ""
    if name == "stress3d-cap":
        # 272 neutrals per material cell, all pre-ionized: 2 x 458752 x 272 = 2.5e8 charged
        return W.config_stress(W.config_3d(ppc=272, **d), eV=2.0), None, ""
    raise SystemExit(f"unknown workload {name}")


def bench_window(args):
    from paper_2502_13695_amd import pic
    cfg, ocfg, share_note = workload_config(args.workload, args.dispersive)
    if args.collisions:
        cfg = dict(cfg, collisions=True)
        ocfg = dict(ocfg, collisions=True) if ocfg is not None else None
    params = pic.canonical(cfg)
    if args.start is not None:
        start = args.start
    elif cfg.get("preionize_eV", 0.0) > 0:
        start = TUNE_STEPS + args.warmup + 12
    else:
        start = interaction_start(cfg, params)
    cfg = dict(cfg, nsteps=max(cfg["nsteps"], start + args.steps + 1))
    if args.calib_copy:
        import torch
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.field_tile is not None:
        os.environ["PIC_FIELD_TILE"] = str(args.field_tile)
    roctx = Roctx()
    r = run_window(cfg, start, args.steps, args.warmup, args.field_tile, roctx, args.resort)
    cnt = window_counts(r["sc0"], r["sc1"], r["ev"], start, args.steps)
    timers = r["timers"]
    ps = cnt["charged_steps"] + cnt["neutral_steps"]
    value = ps / r["wall"]
    bytes_launch, fdetail = phase_bytes(cfg, r, cnt, args.steps)
    tot_ms = {ph: timers[ph] for ph in PHASES if timers[8 + ph] > 0}
    dom = max(tot_ms, key=tot_ms.get)
    avg_ms = timers[dom] / timers[8 + dom]
    achieved = bytes_launch[dom] / (avg_ms * 1e-3) / 1e9
    copy_gbs = stream_copy_gbs()
    # the other ceiling of the push: its algorithmic flops at the FP32 vector
    # peak (3D order 2 only); bound = the larger of the two floors
    roof = {"kernel": PHASES[dom], "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload, PHASES[dom]),
            "bytes_per_launch": bytes_launch[dom], "avg_launch_us": avg_ms * 1e3, "launches": int(timers[8 + dom]),
            "stream_copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs}
    bound = "hbm"
    if dom == 0 and cfg["ndim"] == 3 and cfg.get("shape_order", 2) == 2:
        flops = FLOP_PUSH_3D2 * cnt["charged_steps"] / timers[8]
        tflops = flops / (avg_ms * 1e-3) / 1e12
        roof["alu"] = {"flop_per_launch": flops, "achieved_TFLOPs": tflops, "peak_TFLOPs": FP32_PEAK_TFLOPS,
                       "frac": tflops / FP32_PEAK_TFLOPS}
        if flops / (FP32_PEAK_TFLOPS * 1e12) > bytes_launch[dom] / (HBM_PEAK_GBS * 1e9):
            bound = "alu"
    roof = {"bound": bound, **roof}
    steps = args.steps
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + (DISPERSIVE_NOTE if args.dispersive else "")
                   + ("; binary collisions every step" if args.collisions else ""),
                   "cells": list(cfg["n"]), "ppc": cfg["ppc"],
                   "seed": cfg["seed"], "start_step": start,
                   "sort_check_every": args.resort if args.resort is not None else 8,
                   "window": f"steps {start}..{start + steps - 1}" +
                             (" (the pulse peak reaches the first layer at the start)" if args.start is None
                              and not cfg.get("preionize_eV", 0.0) else ""),
                   "charged_start": cnt["charged_start"], "charged_end": cnt["charged_end"],
                   "alive_neutrals_start": cnt["alive_start"], "alive_neutrals_end": cnt["alive_end"],
                   "events_in_window": cnt["events"], "removed_in_window": cnt["removed"],
                   "charged_steps": cnt["charged_steps"], "neutral_steps": cnt["neutral_steps"],
                   "particle_steps": ps},
        "roofline": roof,
        "phases_us_per_step": {PHASES[ph]: timers[ph] / steps * 1e3 for ph in tot_ms},
        "phases_us_per_launch": {PHASES[ph]: timers[ph] / timers[8 + ph] * 1e3 for ph in tot_ms},
        "phases_GBs": {PHASES[ph]: bytes_launch[ph] / (timers[ph] / timers[8 + ph] * 1e-3) / 1e9
                       for ph in tot_ms},
        "field_tiles": fdetail,
        "field_tile_autotune": r["tune"],
        "tile_sort": dict(start=r["sort0"], end=r["sort1"]),
        "health": r["sc1"]["health"],
    }
    if not args.no_cpu_baseline and ocfg is not None:
        out["cpu_baseline"] = cpu_baseline(dict(ocfg, nsteps=cfg["nsteps"]), start, steps, args.cpu_budget,
                                           share_note)
    return out


def _run_alone(cfg, steps):
    """The plain one-run-at-a-time GPU path: init, step, read the result."""
    import torch
    from paper_2502_13695_amd import pic
    from paper_2502_13695_amd.serve import particle_steps
    ctx = pic.Context(cfg)
    ctx.step(steps)
    sc = ctx.scalars()
    ev = ctx.events()
    nps, cps = particle_steps(ev, ctx.params().n_neutral, steps)
    ctx.close()
    torch.cuda.synchronize()
    return sc, ev, nps + cps


def bench_scan(args):
    """Batched fluence scan: N independent 2D3V instances advanced by one launch
    per phase, against running the same instances one at a time."""
    import torch
    import workloads as W
    from paper_2502_13695_amd import pic
    from paper_2502_13695_amd.serve import particle_steps
    torch.cuda.set_device(0)
    steps = args.scan_steps
    cfgs = [dict(c, nsteps=steps) for c in W.batch_scan(args.instances, steps)]
    # warm the kernels and the rate-table cache
    _run_alone(dict(cfgs[0], nsteps=20), 20)
    # one at a time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = [_run_alone(c, steps) for c in cfgs]
    t_alone = time.perf_counter() - t0
    # batched: contexts initialised up front (outside the timed region, like the
    # resident state of the one-at-a-time runs is not re-initialised either)
    ctxs = [pic.Context(c) for c in cfgs]
    b = pic.Batch(ctxs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ps_b = 0.0
    ev_match = 0
    print(f"scan: one at a time {t_alone:.3f} s, batched {t_batch:.3f} s", file=sys.stderr, flush=True)
    for x, (_, ev_a, _) in zip(ctxs, alone):
        ev = x.events()
        nps, cps = particle_steps(ev, x.params().n_neutral, steps)
        ps_b += nps + cps
        ev_match += int(set(map(tuple, ev.tolist())) == set(map(tuple, ev_a.tolist())))
    b.close()
    for x in ctxs:
        x.close()
    ps_a = sum(r[2] for r in alone)
    return {
        "metric": "particle-steps/sec, batched fluence scan at 1 GPU",
        "value": ps_b / t_batch, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.instances} independent 2D3V slab instances, grids 256x128 .. "
                               f"1536x512 at lambda/32, fluences 0.05 .. 3 J/cm^2 log-spaced, 8 .. 32 ppc, "
                               f"seeds 100..", "instances": args.instances},
        "batched_s": t_batch, "one_at_a_time_s": t_alone,
        "one_at_a_time_value": ps_a / t_alone,
        "speedup_vs_one_at_a_time": (ps_b / t_batch) / (ps_a / t_alone),
        "instances_with_identical_events": ev_match,
    }


def bench_serve(args):
    """Served scan: Poisson arrivals of mixed 1D/2D/3D runs, admitted by HBM
    footprint into a continuously batched set of resident runs; p50/p99 latency
    and aggregate particle-steps/s, against serving them one at a time (FIFO)."""
    import torch
    import workloads as W
    from paper_2502_13695_amd import serve as S
    torch.cuda.set_device(0)
    reqs = W.served_requests(args.requests, scale=args.scale)
    if args.burst:
        reqs = [dict(r, arrival_s=0.0) for r in reqs]
    _run_alone(dict(reqs[0]["cfg"], nsteps=20), 20)
    for r in reqs[:3]:   # fill the rate-table cache (1D, 2D, 3D time steps)
        _run_alone(dict(r["cfg"], nsteps=1), 1)
    def progress(r):
        if (srv.stats["completed"]) % 20 == 0:
            print(f"served {srv.stats['completed']}/{len(reqs)}  latency {r['latency_s']:.3f} s",
                  file=sys.stderr, flush=True)
    srv = S.Server(chunk=50, on_result=progress)
    res = srv.run(reqs)
    summ = S.summarize(res)
    # one at a time, first come first served, same arrivals
    t0 = time.perf_counter()
    clock_free = 0.0
    lat = []
    ps = 0.0
    for r in reqs:
        now = time.perf_counter() - t0
        if now < r["arrival_s"]:
            time.sleep(r["arrival_s"] - now)
        _, _, p = _run_alone(r["cfg"], r["cfg"]["nsteps"])
        ps += p
        lat.append(time.perf_counter() - t0 - r["arrival_s"])
        if len(lat) % 20 == 0:
            print(f"one at a time {len(lat)}/{len(reqs)}  latency {lat[-1]:.3f} s", file=sys.stderr, flush=True)
    span = time.perf_counter() - t0 - reqs[0]["arrival_s"]
    import numpy as np
    lat = np.array(lat)
    return {
        "metric": "served scan: aggregate particle-steps/sec and p50/p99 run latency at 1 GPU",
        "value": summ["particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "p50_s": summ["p50_s"], "p99_s": summ["p99_s"],
        "config": {"workload": f"{args.requests} requests, "
                               f"{'all arriving at t = 0' if args.burst else 'Poisson arrivals 4/s'}, mixed "
                               f"1D/2D/3D mirror runs (1-8 layers, 0.05-3 J/cm^2), scale {args.scale}, seed 7"},
        "served": summ, "server_stats": srv.stats,
        "one_at_a_time": {"particle_steps_per_s": ps / span, "p50_s": float(np.percentile(lat, 50)),
                          "p99_s": float(np.percentile(lat, 99)), "makespan_s": span},
        "speedup_vs_one_at_a_time": summ["particle_steps_per_s"] / (ps / span),
    }


def bench_diag(args):
    """Sec. 5 diagnostics at the 2D slab grid (2048 x 512).  The energy
    histogram of 1.2e6 charged particles (a seeded synthetic state, |u| log-
    uniform from 1e-4 to 3, not stepped) over 200 log bins, for the whole box
    and for one 80-cell layer.  On the 2D stress run (the slab pre-ionized at
    2 eV, 1.31e6 carriers): the node |E|^2 maximum sampled every step, and
    trajectory records of 2 % of the particles every 10th step.  Reported: the
    wall time of one histogram call (host edges in, counts out, synchronous)
    and the step times with each sampling on; kernel durations come from a
    kernel trace of this command."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2502_13695_amd import pic
    cfg = W.config_2d()
    npart = 1_200_000
    st = W.random_state(cfg, npart, seed=77, e_scale=1e8)
    rng = np.random.default_rng(78)
    d = st["u"] / np.linalg.norm(st["u"], axis=1, keepdims=True)
    st["u"] = (d * (10.0 ** rng.uniform(-4.0, 0.5, npart))[:, None]).astype(np.float32)
    rec = np.zeros(npart, dtype=pic.PARTICLE_DTYPE)
    rec["cell"][:, :2] = st["cell"][:, :2]
    rec["off"] = st["off"]
    rec["u"] = st["u"]
    rec["kind"] = st["kind"]
    ctx = pic.Context(cfg)
    ctx.set_state(0, st["E"], st["b"], rec)
    edges = np.geomspace(1e-4, 3e6, 201)
    out = {}
    for name, (lo, hi) in (("box", (0, 0)), ("layer", (512, 592))):
        for _ in range(3):
            ctx.spectrum(edges, lo, hi)
        ts = []
        for _ in range(50):
            t0 = time.perf_counter()
            ctx.spectrum(edges, lo, hi)
            ts.append(time.perf_counter() - t0)
        out[name] = dict(call_us=1e6 * float(np.median(ts)), counted=int(ctx.spectrum(edges, lo, hi).sum()))
    ctx.close()

    scfg = W.config_stress(W.config_2d())
    ctx = pic.Context(scfg)
    ncharged = int(ctx.scalars()["slots"])
    nstep = 400

    def timed_steps():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(nstep)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / nstep

    ctx.step(40)
    off1 = timed_steps()
    ctx.set_imax(1)
    on = timed_steps()
    ctx.set_imax(0)
    off2 = timed_steps()
    # trajectory records of 2 % of the particles every 10th step
    ctx.set_tracks(0.02, 10, max_records=1 << 21)
    timed_steps()
    nrec = len(ctx.tracks())
    ctx.set_tracks(0.02, 0)
    assert ctx.scalars()["health"] == 0
    nodes = (cfg["n"][0] + 1) * (cfg["n"][1] + 1)
    ctx.close()
    return {"metric": "Sec. 5 diagnostics at the 2D slab grid", "unit": "us", "data": "synthetic",
            "config": {"workload": "2048x512 slab; histogram of 1.2e6 charged particles (seeded state), "
                                   "200 log bins; sampling on the 2 eV pre-ionized slab",
                       "particles": npart, "nodes": nodes, "stress_charged": ncharged},
            "spectrum": out,
            # algorithmic bytes: kind 1 + cell 4 + u 12 per slot; E 12 + maximum read and write 8 per node
            "spectrum_bytes": 17 * npart, "imax_bytes_per_sample": 20 * nodes,
            "step_us_without_sampling": 1e6 * 0.5 * (off1 + off2), "step_us_sampling_every_step": 1e6 * on,
            "track_records": nrec,
            # kind 1 + id 4 per slot; a sampled one reads cell 4 + offsets 8 and writes 40
            "tracks_bytes_per_launch": 5 * ncharged + int(0.02 * ncharged) * 52}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (the window)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps right before the window")
    ap.add_argument("--start", type=int, default=None,
                    help="first step of the window (default: the pulse peak reaches the first layer)")
    ap.add_argument("--workload", default="mirror3d",
                    choices=list(WORKLOADS) + ["scan", "serve", "diag"])
    ap.add_argument("--instances", type=int, default=32, help="scan: fluence-scan instances")
    ap.add_argument("--scan-steps", type=int, default=3000, help="scan: steps of every instance")
    ap.add_argument("--requests", type=int, default=400, help="serve: requests")
    ap.add_argument("--scale", type=float, default=1.0, help="serve: grid/step scale of the mix")
    ap.add_argument("--burst", action="store_true",
                    help="serve: every request arrives at t = 0 (capacity, not latency, is measured)")
    ap.add_argument("--field-tile", type=int, default=None,
                    help="fixed field tile shape (default: timed in-run over the first steps)")
    ap.add_argument("--dispersive", action="store_true",
                    help="the workload's layers respond as single-pole Lorentz media")
    ap.add_argument("--collisions", action="store_true",
                    help="binary collisions among the charged particles every step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 256 MiB once before the run (HBM counter calibration)")
    ap.add_argument("--resort", type=int, default=None,
                    help="tile-sort check period in steps (default: the library's, 8)")
    ap.add_argument("--trace-summary", default=None, metavar="KERNEL_TRACE_CSV",
                    help="print the per-kernel statistics of the timed window of a rocprofv3 kernel "
                         "trace of this script (same --steps) and exit")
    ap.add_argument("--oracle-child", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_child is not None:
        _oracle_child(json.loads(args.oracle_child))
        return
    if args.trace_summary is not None:
        print(trace_summary(args.trace_summary, args.steps))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library has no multi-GPU "
              f"path, and the design notes describe how a run would shard", file=sys.stderr)
        sys.exit(2)
    if args.workload == "scan":
        print(json.dumps(bench_scan(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "diag":
        print(json.dumps(bench_diag(args)), flush=True)
        return
    print(json.dumps(bench_window(args)), flush=True)


if __name__ == "__main__":
    main()
