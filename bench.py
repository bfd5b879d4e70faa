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

TIMING_PERIOD = 16

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


def phase_bytes(cfg, phase, n_charged_avg, n_alive_avg, far_frac=0.0, far_updated=None):
    """Algorithmic HBM bytes of one launch of a phase (FP32 SoA layout).
    far_frac: share of the field tiles that skip the current (no charged
    particle has come within their margin); far_updated: share of the field
    tiles that skip the current and are updated (the rest lie beyond the
    field front and move nothing), default all of them."""
    D = cfg["ndim"]
    per = cfg.get("transverse_bc", "outflow") == "periodic"
    cells = 1
    for d in range(D):
        cells *= cfg["n"][d] + (0 if (per and d > 0) else 1)
    if phase == 1:
        # Yee step: read E, b, J (36 B), write E, b (24 B), clear J (12 B);
        # far tiles: no current to read or clear (48 B);
        # window node: ring write, prefix read+write, suffix read, A write (20 B)
        # plus the once-per-cycle suffix rebuild (8 B amortised)
        fu = far_frac if far_updated is None else far_updated
        return (72.0 * (1.0 - far_frac) + 48.0 * fu) * cells + 28.0 * window_nodes(cfg)
    if phase == 0:           # charged particle: read cell, offsets, u, kind; write back
        rd = 4 + 4 * D + 12 + 1
        wr = 4 + 4 * D + 12
        return float(rd + wr) * n_charged_avg
    if phase == 2:           # alive neutral: offsets (+ alive bit)
        return (4.0 * D + 0.125) * n_alive_avg
    return 0.0


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


def run_gpu(cfg, steps, warmup, field_tile=None):
    import torch
    from paper_2502_13695_amd import pic
    torch.cuda.set_device(0)
    if warmup > 0:
        w = pic.Context(cfg)
        w.step(warmup)
        w.scalars()
        w.close()
    ctx = pic.Context(cfg)
    region0 = ctx.region()
    # field tile shape: timed on the first steps of the timed run itself (every
    # shape computes identical fields); the choice is reported after the run
    if field_tile is None:
        ctx.autotune_steps(4)
    # HIP events stamped by the dispatches of one step in every 16 of the timed
    # region (the sampled position cycles through the window, so the tile sort
    # check, due every 8 steps, is sampled in proportion)
    ctx.set_timing(TIMING_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timers = ctx.timers()
    tune = dict(chosen=int(timers[23]), blocks=int(timers[24]), ms=[float(x) for x in timers[16:23]])
    sort_state = ctx.sort_state()
    region = ctx.region()
    sc = ctx.scalars()
    ev = ctx.events()
    nneut = ctx.params().n_neutral
    ctx.close()
    # particle-steps: each neutral counts until its ionization step, each birth
    # pair from its step to the end (carriers leaving the box are not subtracted)
    if len(ev):
        import numpy as np
        death = np.asarray(ev[:, 1], dtype=np.int64)
        dead_steps = float(np.minimum(death, steps).sum())
        births = float(2 * np.maximum(0, steps - death).sum())
        neutral_steps = dead_steps + (nneut - len(death)) * steps
    else:
        births = 0.0
        neutral_steps = float(nneut) * steps
    ps = neutral_steps + births
    wall = t1 - t0
    return dict(wall=wall, particle_steps=ps, neutral_steps=neutral_steps, charged_steps=births,
                timers=timers, scalars=sc, nneut=nneut, tune=tune, sort_state=sort_state, region=region,
                region0=region0)


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
    steps = args.steps if args.steps != 4000 else 3000
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
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="slab2d", choices=["slab2d", "mirror3d", "slab1d",
                                                             "stress2d", "stress3d", "stress2d-cap",
                                                             "stress3d-cap", "scan", "serve", "diag"])
    ap.add_argument("--instances", type=int, default=32, help="scan: fluence-scan instances")
    ap.add_argument("--requests", type=int, default=400, help="serve: requests")
    ap.add_argument("--scale", type=float, default=1.0, help="serve: grid/step scale of the mix")
    ap.add_argument("--burst", action="store_true",
                    help="serve: every request arrives at t = 0 (capacity, not latency, is measured)")
    ap.add_argument("--field-tile", type=int, default=None,
                    help="fixed field tile shape (default: timed in-run over the first steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 256 MiB once before the run (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    if args.workload == "scan":
        print(json.dumps(bench_scan(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "diag":
        print(json.dumps(bench_diag(args)), flush=True)
        return
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
    elif args.workload == "stress2d-cap":
        # 488 neutrals per slab cell, all pre-ionized: 2 x 40960 x 488 = 4.0e7 charged
        cfg = W.config_stress(W.config_2d(ppc=488), eV=2.0)
        wl = dict(workload="2D3V slab grid, 4.0e7 pre-ionized carriers (charged-loop stress at the "
                           "particle cap)", cells=[2048, 512], ppc=488, seed=1)
    elif args.workload == "stress3d-cap":
        # 272 neutrals per material cell, all pre-ionized: 2 x 458752 x 272 = 2.5e8 charged
        cfg = W.config_stress(W.config_3d(ppc=272), eV=2.0)
        wl = dict(workload="3D3V mirror-share grid, 2.5e8 pre-ionized carriers (charged-loop stress at "
                           "the particle cap)", cells=[256, 128, 128], ppc=272, seed=2)
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
    if args.field_tile is not None:
        # fixed field tile shape, read by the library when a context is created
        os.environ["PIC_FIELD_TILE"] = str(args.field_tile)
    r = run_gpu(cfg, args.steps, args.warmup, args.field_tile)
    value = r["particle_steps"] / r["wall"]
    timers = r["timers"]
    # dominant kernel by device time
    tot = {ph: timers[ph] for ph in PHASES if timers[8 + ph] > 0}
    dom = max((ph for ph in tot if ph != 3), key=tot.get)
    n_launch = timers[8 + dom]
    avg_ms = timers[dom] / n_launch
    n_charged_avg = r["charged_steps"] / args.steps
    n_alive_avg = r["neutral_steps"] / args.steps
    # share of the field tiles that skip the current: it only shrinks during a
    # run (the charged region only grows), so the share at the start gives the
    # fewest bytes per launch, the share at the end the most; the achieved rate
    # uses the fewest
    share = lambda g: g["far_tiles"] / max(1, g["near_tiles"] + g["far_tiles"])
    reg, reg0 = r["region"], r["region0"]
    far_frac, far_frac_end = share(reg0), share(reg)
    # far tiles beyond the field front are not updated: the device counts the
    # tiles every field launch updated; the mean over the timed launches,
    # less the near tiles, is the share of far tiles that moved bytes
    ntiles = max(1, reg["near_tiles"] + reg["far_tiles"])
    upd = (reg["tiles_updated"] - reg0["tiles_updated"]) / max(1, args.steps)
    far_updated = min(far_frac, max(0.0, upd - reg0["near_tiles"]) / ntiles)
    bytes_launch = phase_bytes(cfg, dom, n_charged_avg, n_alive_avg, far_frac, far_updated)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    copy_gbs = stream_copy_gbs()
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
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, PHASES[dom]),
                     "bytes_per_launch": bytes_launch, "avg_launch_us": avg_ms * 1e3,
                     "stream_copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "phases_us_per_step": {PHASES[ph]: timers[ph] / max(timers[8], 1) * 1e3 for ph in tot},
        "phases_us_per_launch": {PHASES[ph]: timers[ph] / max(timers[8 + ph], 1) * 1e3 for ph in tot},
        "field_tile_autotune": r["tune"],
        "far_tiles": dict(start=reg0, end=reg, far_frac_start=far_frac, far_frac_end=far_frac_end,
                          tiles_updated_per_launch=upd, far_updated_frac=far_updated,
                          bytes_per_launch_end=phase_bytes(cfg, 1, 0, 0, far_frac_end)),
        "tile_sort": r["sort_state"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
