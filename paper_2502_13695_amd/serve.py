"""Continuous batching of PIC runs on one GPU (fluence-scan serving).

Requests (a run configuration plus an arrival time) are admitted as soon as
they have arrived, a member slot is free and their device footprint
(``pic_footprint``) fits the HBM budget next to the runs already resident.  An
admitted run is initialised on the device and joins the running batch at the
next step boundary; every batch step advances all members with one launch per
phase; a member leaves the batch when it has taken its own number of steps,
its diagnostics are read and its memory returns to the pool.  Runs that arrive
while others are on the GPU therefore overlap with them on the device, and
each run computes exactly what it would compute alone (members share no state;
only the summation order of FP32 atomics can differ).

Latency of a request = time from its arrival to its result being on the host.
"""

import collections
import time

from . import pic


def particle_steps(events, nneut, steps):
    """(alive-neutral, charged) particle-steps of a run of ``steps`` steps from
    t = 0, from its ionization events (neutral id, step): each neutral counts
    until its ionization step, each birth pair from that step on (carriers
    leaving the box are not subtracted)."""
    import numpy as np
    if len(events) == 0:
        return float(nneut) * steps, 0.0
    death = np.asarray(events[:, 1], dtype=np.int64)
    dead = float(np.minimum(death, steps).sum())
    births = float(2 * np.maximum(0, steps - death).sum())
    return dead + (nneut - len(death)) * steps, births


class Server:
    """Admit, batch and retire runs; see the module docstring.

    hbm_budget: bytes available to resident runs (default: 90 % of the free
    device memory when the server starts); max_members: batch slots; chunk:
    largest number of batch steps between admission checks.
    """

    def __init__(self, hbm_budget=None, max_members=64, chunk=50, on_result=None):
        import torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.9 * free)
        self.hbm_budget = int(hbm_budget)
        self.max_members = int(max_members)
        self.chunk = int(chunk)
        self.on_result = on_result
        self.stats = dict(admitted=0, completed=0, batch_steps=0, max_resident=0, max_bytes=0)

    def run(self, requests, clock=time.perf_counter, keep_fields=False):
        """Serve ``requests`` (dicts with 'cfg' and 'arrival_s', seconds from the
        start) in real time; returns one result dict per request, in input order."""
        import torch
        order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival_s"])
        pending = collections.deque(order)
        results = [None] * len(requests)
        active = {}   # request index -> dict(ctx, left, steps, bytes, t_admit)
        used = 0
        batch = pic.Batch([])
        t0 = clock()
        try:
            while pending or active:
                now = clock() - t0
                # ---- admission: arrived, a slot free, footprint fits
                while pending and len(active) < self.max_members:
                    i = pending[0]
                    req = requests[i]
                    if req["arrival_s"] > now:
                        break
                    need = pic.footprint(req["cfg"])
                    if need > self.hbm_budget:
                        raise ValueError(f"request {i} needs {need} bytes, more than the HBM budget")
                    if used + need > self.hbm_budget:
                        break   # wait for a resident run to finish
                    pending.popleft()
                    ctx = pic.Context(req["cfg"])
                    batch.add(ctx)
                    steps = int(req.get("steps", req["cfg"]["nsteps"]))
                    active[i] = dict(ctx=ctx, left=steps, steps=steps, bytes=need, t_admit=clock() - t0)
                    used += need
                    self.stats["admitted"] += 1
                self.stats["max_resident"] = max(self.stats["max_resident"], len(active))
                self.stats["max_bytes"] = max(self.stats["max_bytes"], used)
                if not active:
                    nxt = requests[pending[0]]["arrival_s"]
                    time.sleep(max(0.0, min(0.05, nxt - (clock() - t0))))
                    continue
                # ---- advance every member by the same number of steps
                k = min(self.chunk, min(a["left"] for a in active.values()))
                batch.step(k)
                torch.cuda.current_stream().synchronize()
                self.stats["batch_steps"] += k
                # ---- retire finished members
                done = [i for i, a in active.items() if a["left"] == k]
                for a in active.values():
                    a["left"] -= k
                for i in done:
                    a = active.pop(i)
                    ctx = a["ctx"]
                    batch.remove(ctx)
                    sc = ctx.scalars()
                    ev = ctx.events()
                    neutral_ps, charged_ps = particle_steps(ev, ctx.params().n_neutral, a["steps"])
                    res = dict(index=i, arrival_s=requests[i]["arrival_s"], admit_s=a["t_admit"],
                               done_s=clock() - t0, steps=a["steps"], scalars=sc,
                               events=ev, particle_steps=neutral_ps + charged_ps,
                               neutral_steps=neutral_ps, charged_steps=charged_ps)
                    res["latency_s"] = res["done_s"] - res["arrival_s"]
                    if keep_fields:
                        res["fields"] = ctx.fields()
                    ctx.close()
                    used -= a["bytes"]
                    results[i] = res
                    self.stats["completed"] += 1
                    if self.on_result:
                        self.on_result(res)
        finally:
            batch.close()
            for a in active.values():
                a["ctx"].close()
        return results


def summarize(results):
    """p50 / p99 latency and aggregate particle-steps/s of a served run."""
    import numpy as np
    lat = np.array([r["latency_s"] for r in results])
    span = max(r["done_s"] for r in results) - min(r["arrival_s"] for r in results)
    ps = sum(r["particle_steps"] for r in results)
    return dict(requests=len(results), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()), max_s=float(lat.max()),
                makespan_s=float(span), particle_steps=float(ps),
                particle_steps_per_s=float(ps / span) if span > 0 else 0.0)
