"""Serving workload: a Poisson stream of independent imaging jobs through the
continuous-batching server of libwsg (wsg_server_*).

Jobs are drawn from a pool of pre-generated datasets held in pinned host
memory (mesh 512^2 .. 4096^2, 8 .. 64 w-planes, 1e5 .. 5e7 complex64
visibilities, random array layouts); each job's image comes back to pinned
host memory.  Two schedules are compared on the same trace:
  * batched:    n_slots concurrent jobs, admitted by device-memory footprint;
  * sequential: one job at a time (a single slot), in arrival order.
Latency is arrival -> image on the host; output images are pinned before the clock
starts and recycled, so a job waits at the client until an image of its size is free.  Run `python -m
paper_2411_07321_amd.serve --help` for the command-line driver.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from paper_2411_07321_amd import synth, wsg


class PinnedJob:
    """One pooled dataset in pinned host memory plus its imaging parameters."""

    def __init__(self, ds: synth.Dataset, **param_overrides):
        import torch
        self.ds = ds
        self.uvw = torch.from_numpy(ds.uvw).pin_memory()
        self.vis = torch.from_numpy(np.ascontiguousarray(ds.vis)).pin_memory()
        self.wts = torch.from_numpy(np.ascontiguousarray(ds.weights)).pin_memory()
        self.params = wsg.params_for(ds, **param_overrides)
        self.vb = wsg.make_vis(self.uvw, self.vis, self.wts, None, ds.freq_hz, ds.row_period)
        self.n_vis = ds.n_vis
        self.grid_n = ds.grid_n


def make_pool(n_datasets: int, seed: int = synth.CONFIG_SEED0 + 4, device=None,
              m_cap: float | None = None, log=None, **param_overrides) -> list[PinnedJob]:
    """Pre-generate the pool (job shapes from the seeded job_spec draw)."""
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(n_datasets):
        spec = synth.job_spec(rng)
        if m_cap is not None and spec["m_target"] > m_cap:
            n_bl = spec["n_ant"] * (spec["n_ant"] - 1) // 2
            spec["m_target"] = m_cap
            spec["n_times"] = max(1, int(round(m_cap / n_bl)))
        ds = synth.make_job(spec, seed * 1000 + i, device=device)
        pool.append(PinnedJob(ds, **param_overrides))
        if log:
            log(f"pool {i + 1}/{n_datasets}: N={ds.grid_n} Nw={ds.n_wplanes} M={ds.n_vis:,}")
    return pool


class OutputBuffers:
    """Pinned host images, allocated before the clock starts and recycled by size: a
    client holds `per_size` images of each mesh size, and a job whose image is not free
    waits at the client (pinned allocation inside the timed loop would stall the run)."""

    def __init__(self, sizes, per_size: int):
        import torch
        self.free = {n: [torch.empty((1, n, n), dtype=torch.float64).pin_memory()
                         for _ in range(per_size)] for n in sorted(set(sizes))}

    def take(self, n: int):
        lst = self.free[n]
        return lst.pop() if lst else None

    def give(self, n: int, buf):
        self.free[n].append(buf)


def replay(pool, order, arrivals, n_slots: int, hbm_budget: int = 0, device: int = 0,
           keep_images: set | None = None, log=None, per_size: int | None = None) -> dict:
    """Job k (pool index order[k]) arrives at time arrivals[k] (s after the start) and is
    submitted to a server with n_slots slots once an output image of its size is free
    (arrived jobs are submitted in arrival order, skipping those still waiting for an
    image); returns per-job latency (arrival -> image on the host) and the throughput."""
    per_size = per_size or 2 * max(n_slots, 4)
    outs = OutputBuffers([pool[i].grid_n for i in order], per_size)
    srv = wsg.Server(device, n_slots, hbm_budget)
    pending = {}
    lat, infos, kept, wait_ms = [], [], {}, []
    waiting = []                # arrived, not yet submitted (client queue)
    k = 0
    n = len(order)
    t0 = time.perf_counter()
    t_end_last = t0
    try:
        while k < n or pending or waiting:
            now = time.perf_counter() - t0
            while k < n and arrivals[k] <= now:
                waiting.append(k)
                k += 1
            still = []
            for kk in waiting:
                job = pool[order[kk]]
                buf = outs.take(job.grid_n)
                if buf is None:
                    still.append(kk)
                    continue
                t = srv.submit(job.params, job.vb, buf)
                pending[t] = (kk, job, buf)
            waiting = still
            done_any = False
            for t in list(pending):
                ok, info = srv.poll(t)
                if ok:
                    kk, job, buf = pending.pop(t)
                    if info["status"] != wsg.OK:
                        raise wsg.WsgError(info["status"], f"job {kk} failed")
                    t_done = time.perf_counter()
                    lat.append(t_done - (t0 + arrivals[kk]))
                    wait_ms.append((info["t_start"] - info["t_submit"]) * 1e3)
                    infos.append(info)
                    t_end_last = max(t_end_last, t_done)
                    if keep_images is not None and kk in keep_images:
                        kept[kk] = buf.numpy().copy()
                    outs.give(job.grid_n, buf)
                    done_any = True
            if not done_any:
                nxt = arrivals[k] - (time.perf_counter() - t0) if k < n else 0.0002
                time.sleep(max(0.0, min(0.0002, nxt)))
        wall = time.perf_counter() - t0
        held, peak = srv.memory()
    finally:
        srv.close()
    lat = np.array(lat)
    span = t_end_last - t0
    return {"jobs": n, "wall_s": wall, "jobs_per_s": n / span,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "peak_device_bytes": peak,
            "server_queue_wait_p50_ms": float(np.percentile(wait_ms, 50)),
            "visibilities_per_s": sum(pool[i].n_vis for i in order) / span,
            "images": kept}


def protocol(n_pool: int = 64, n_jobs: int = 600, rates=(20, 50, 100, 200, 400), slots: int = 4,
             budget: int = 96 << 30, n_check: int = 24, log=None) -> dict:
    """The serving measurement: one seeded job list of n_jobs drawn from a pool of n_pool
    datasets, replayed as a backlog (every job arrives at t = 0: jobs/s at saturation) and
    as Poisson arrivals at each rate, batched (slots) and sequential (one slot).  The
    images of n_check jobs of the backlog runs are compared, batched against
    sequential (a sequential job runs alone on the device), on the raw image (the grid
    correction, which multiplies FP32 rounding near the field edge by up to ~3000, is
    off; the work per job is the same)."""
    pool = make_pool(n_pool, device="cuda", log=log, grid_correct=False)
    rng = np.random.default_rng(synth.CONFIG_SEED0 + 40)
    order = rng.integers(0, len(pool), n_jobs)
    check = set(range(0, n_jobs, max(1, n_jobs // n_check)))
    out = {"workload": "config4_serving", "pool": n_pool, "jobs": n_jobs, "slots": slots,
           "mean_visibilities": float(np.mean([pool[i].n_vis for i in order])),
           "backlog": {}, "sweep": []}
    imgs = {}
    for name, sl in (("batched", slots), ("sequential", 1)):
        if log:
            log(f"backlog, {name}")
        r = replay(pool, order, np.zeros(n_jobs), sl, budget, keep_images=check)
        imgs[name] = r.pop("images")
        out["backlog"][name] = r
    worst = 0.0
    for k in check:
        a, b = imgs["batched"][k], imgs["sequential"][k]
        nb = np.linalg.norm(b)
        worst = max(worst, float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)))
    out["batched_vs_alone_max_rel"] = worst
    out["checked_jobs"] = len(check)
    for rate in rates:
        arr = synth.poisson_arrivals(n_jobs, rate, np.random.default_rng(synth.CONFIG_SEED0 + 41))
        row = {"rate_hz": rate}
        for name, sl in (("batched", slots), ("sequential", 1)):
            if log:
                log(f"rate {rate}/s, {name}")
            r = replay(pool, order, arr, sl, budget)
            r.pop("images")
            row[name] = {k: r[k] for k in ("jobs_per_s", "p50_ms", "p99_ms", "mean_ms", "wall_s",
                                           "server_queue_wait_p50_ms")}
        out["sweep"].append(row)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--pool", type=int, default=24)
    ap.add_argument("--jobs", type=int, default=600)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=96.0)
    ap.add_argument("--backlog", action="store_true", help="all jobs arrive at t=0")
    ap.add_argument("--m-cap", type=float, default=None, help="cap visibilities per job")
    ap.add_argument("--protocol", action="store_true",
                    help="the full measurement: backlog and a rate sweep, batched vs sequential")
    ap.add_argument("--rates", default="20,50,100,200,400")
    ap.add_argument("--modes", default="batched,sequential",
                    help="which replays to run (without --protocol)")
    args = ap.parse_args()
    log = lambda m: print(f"[serve] {m}", file=sys.stderr, flush=True)
    if args.protocol:
        res = protocol(args.pool, args.jobs, tuple(float(x) for x in args.rates.split(",")),
                       args.slots, int(args.budget_gb * 2**30), log=log)
        print(json.dumps(res))
        return
    pool = make_pool(args.pool, device="cuda", m_cap=args.m_cap, log=log)
    rng = np.random.default_rng(synth.CONFIG_SEED0 + 40)
    order = rng.integers(0, len(pool), args.jobs)
    arr = np.zeros(args.jobs) if args.backlog else synth.poisson_arrivals(args.jobs, args.rate, rng)
    res = {}
    modes = [(n, sl) for n, sl in (("batched", args.slots), ("sequential", 1))
             if n in args.modes.split(",")]
    for name, slots in modes:
        log(f"replaying {args.jobs} jobs, {name}")
        r = replay(pool, order, arr, slots, int(args.budget_gb * 2**30), log=log)
        r.pop("images")
        res[name] = r
        log(f"{name}: {r['jobs_per_s']:.2f} jobs/s p50 {r['p50_ms']:.1f} ms p99 {r['p99_ms']:.1f} ms")
    print(json.dumps({"workload": "config4_serving", "rate_hz": None if args.backlog else args.rate,
                      "backlog": args.backlog, "pool": args.pool, **res}))


if __name__ == "__main__":
    main()
