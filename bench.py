#!/usr/bin/env python3
"""Benchmark of the w-stacking imager on one MI355X.

A step is one whole imaging job through the C ABI (wsg_image): validity pass,
binning, gridding (Eq. 3), per-plane 2D inverse transforms and the w-correction
with plane sum (Eq. 2), on the single-large-image workload: 256 antennas
(log-radial, 20 km), 2,048 times, 4 channels -> 267,386,880 complex64
visibilities onto a 4096^2 x 64-plane complex64 stack, support 7, FP64 phase.
Inputs are synthetic (seeded), generated on and resident in HBM before timing.
The gridding kernel is the Gaussian of width 0.9 cells, or with --kernel kb the
Kaiser-Bessel window of the paper's runs (default beta for the support).

Prints ONE JSON line.  Roofline figures credit the method's own traffic: every
input byte read once (B_in), the w-stack written once by the gridder and read
once by the transform (2 B_grid), the image written once (B_img); binning and
intermediate passes are implementation overhead and earn nothing.  The gridding
kernel itself is bound by VALU and LDS atomics, not HBM, and is rated by its
useful arithmetic (392 flop per visibility: 49 complex multiply-adds) against
the FP32 vector peak the library's kernels can issue (no packed FP32 instructions: 256 CUs x
4 SIMDs x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s); the FP64 LDS atomic-add rate
and the copy bandwidth the device reaches are measured by the library's probes.
The same JSON line carries the job at the paper's own arithmetic (complex128 mesh
and transform, FP64 throughout) as "f64_config1".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP32_VENDOR_TFLOPS = 157.3     # MI355X FP32 vector, vendor figure (counts packed FP32)
# FP32 vector issue without packed instructions (the library is built without them):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
DTYPE = "c64 mesh+FFT, f64 phase argument with f32 sin/cos, f64 plane sum and image"
GRID_FLOP_PER_VIS = 392        # 49 complex multiply-adds per visibility
TILE = 64                      # binning tile of the FP32 mesh (set explicitly)
STAGES = ("ms_prep", "ms_count", "ms_scatter", "ms_zero", "ms_grid", "ms_occupancy", "ms_fft1",
          "ms_fft2_wcorr", "ms_total")


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_bin.hip", "k_grid.hip", "k_fft.hip", "wsg_lib.cpp", "wsg_internal.h"):
        with open(os.path.join(ROOT, "paper_2411_07321_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# Per stage of wsg_stats: its main kernel, the bytes the method credits to it, and the
# bytes the stage itself has to move in this design (sparse w-stack: only occupied
# tiles are written and read, rows of empty tile-rows are skipped by the transform).
def stage_bytes(job) -> tuple[dict, dict]:
    m, rows = job["n_elem"], job["n_rows"]
    n, nw = job["grid_n"], job["n_pl"]
    f64 = job["precision"] == "f64"
    csz = 16 if f64 else 8
    vsz, wsz = (16, 8) if f64 else (8, 4)
    b_in = rows * 24 + m * (vsz + wsz)
    b_grid = nw * n * n * csz
    b_img = n * n * 8
    rec = 32 if f64 else 16
    n_rec = job["n_records"]
    tiles = job["n_tiles"] * job["tile"] ** 2 * csz
    trows = job["n_tile_rows"] * job["tile"] * n * csz
    st = {
        "ms_prep": ("k_prep", b_in, b_in + m),
        "ms_count": ("k_count", 0, rows * 24 + m * (1 + wsz)),
        "ms_scatter": ("k_scatter", 0, rows * 24 + m * (1 + vsz + wsz) + n_rec * rec),
        "ms_zero": ("k_zero_tiles", 0, 0),
        "ms_grid": ("k_grid", b_grid, n_rec * rec + tiles),
        "ms_occupancy": ("k_occupancy", 0, 0),
        "ms_fft1": ("k_pass1", b_grid, tiles + trows),
        "ms_fft2_wcorr": ("k_pass2_wcorr", b_img, trows + b_img),
    }
    return st, {"B_in": b_in, "B_grid": b_grid, "B_img": b_img, "B_alg": b_in + 2 * b_grid + b_img}


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy-kernel calibration), if recorded for the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    rec = t.get(workload, {}).get(kernel)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def host_cpu() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def cpu_baseline(ds_host: dict, params: dict, n_total: int) -> dict:
    """The FP64 oracle (unchanged) on a bounded sample of the same workload, scaled to the
    whole job: gridding of a row subsample with every measurement on one plane (the
    per-visibility work does not depend on the plane count), plus one plane's transform
    and w-correction, extrapolated to all visibilities and planes.  Timed with one
    thread and with every thread the host gives this process (the oracle's gridding
    splits the mesh rows over threads; its transform is numpy's, one thread)."""
    import numpy as np
    import oracle
    uvw, vis, wts, freq = ds_host["uvw"], ds_host["vis"], ds_host["weights"], ds_host["freq"]
    m_s = vis.size
    inp = oracle.Inputs.make(uvw, freq, vis, wts)
    n = params["grid_n"]
    prm1 = oracle.Params(n, 1, params["support"], params["cell_rad"], params["kernel_sigma"],
                         kernel=params.get("kernel", "gauss"))
    nw = params["n_wplanes"]
    cpu = host_cpu()
    all_threads = cpu["nproc"]
    runs = {}
    for threads in (1, all_threads):
        oracle.threads(threads)
        t0 = time.perf_counter()
        wmin, wmax = oracle.w_range(inp, prm1)
        g, cnt = oracle.grid(inp, prm1, wmin, wmax)
        t_grid = time.perf_counter() - t0
        t0 = time.perf_counter()
        F = oracle.fft_planes(g)
        t_fft = time.perf_counter() - t0
        t0 = time.perf_counter()
        A = oracle.wcorrect(F, wmin, wmax, 1, params["cell_rad"])
        D = oracle.post(A, cnt["sum_w"], prm1)
        t_wc = time.perf_counter() - t0
        del g, F, A, D
        t_est = t_grid * (n_total / m_s) + nw * (t_fft + t_wc)
        runs[threads] = {"value": n_total / t_est, "t_grid": t_grid, "t_fft": t_fft, "t_wc": t_wc,
                         "t_job_est": t_est}
        progress(f"oracle, {threads} thread(s): {n_total / t_est:.3e} vis/s")
    one, full = runs[1], runs[all_threads]
    return {"value": full["value"], "unit": "visibilities/s", "cores": all_threads, "kind": "oracle",
            "value_1_thread": one["value"], "host_cpu": cpu,
            "sample": (f"FP64 oracle on {all_threads} threads ({cpu['model']}; 1 thread: "
                       f"{one['value']:.3e} vis/s): {m_s:,} visibilities (row subsample) gridded "
                       f"on the {n}^2 mesh in {full['t_grid']:.2f} s (1 thread {one['t_grid']:.2f} s), "
                       f"one plane transformed in {full['t_fft']:.2f} s and w-corrected in "
                       f"{full['t_wc']:.2f} s; extrapolated to {n_total:,} visibilities and {nw} "
                       f"planes = {full['t_job_est']:.0f} s per job "
                       f"(1 thread {one['t_job_est']:.0f} s)")}


def chunked(args, d, prm, ctx, out):
    """The same workload as a chunked job: begin, one add per time chunk, finish, with
    the w range of the data given up front.  A step is the whole job, accumulator
    set-up included; host chunks are copied from pinned memory inside the step."""
    import torch
    from paper_2411_07321_amd import wsg
    c = 299792458.0
    scale = [f / c for f in d["freq_hz"]]
    w = d["uvw"][:, 2]
    lo, hi = float(w.min()), float(w.max())
    prm.w_min = min(min(lo * x, hi * x) for x in scale)
    prm.w_max = max(max(lo * x, hi * x) for x in scale)
    rows, rp = d["uvw"].shape[0], d["row_period"]
    step = -(-rows // args.chunks)
    step = -(-step // rp) * rp
    bounds = [(a, min(rows, a + step)) for a in range(0, rows, step)]
    src = {k: d[k] for k in ("uvw", "vis", "weights")}
    if args.host_chunks:
        progress("copying the workload to pinned host memory")
        src = {k: v.cpu().pin_memory() for k, v in src.items()}
    chunks = [wsg.make_vis(src["uvw"][a:b], src["vis"][a:b], src["weights"][a:b], None,
                           d["freq_hz"], rp) for a, b in bounds]

    def job():
        with wsg.Accum(ctx, prm, d["vis"].shape[1], stream=ctx.stream) as acc:
            for vb in chunks:
                acc.add(vb, stream=ctx.stream)
            st = acc.finish(out, stream=ctx.stream)
        return st

    for i in range(args.warmup):
        job()
        progress(f"warmup {i}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = job()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / args.steps * 1e3
    n_used = int(st[0]["n_used"])
    progress(f"timed {args.steps} chunked jobs: {ms_step:.2f} ms/job")
    b_in = sum(x.numel() * x.element_size() for x in (d["uvw"], d["vis"], d["weights"]))
    where = "host_pinned" if args.host_chunks else "device"
    result = {
        "metric": "visibilities gridded+imaged/s", "value": n_used / (ms_step * 1e-3),
        "unit": "visibilities/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE,
        "data": "synthetic (seeded, device-generated config-1 interferometer data)",
        "config": {"workload": f"config1_4096sq_64w_2.67e8vis_{len(bounds)}chunks_{where}",
                   "grid_n": d["params"]["grid_n"], "n_wplanes": d["params"]["n_wplanes"],
                   "support": 7, "visibilities": int(d["vis"].numel()), "n_used": n_used,
                   "chunks": len(bounds), "chunk_rows": step, "inputs": where,
                   "kernel": args.kernel, "tile": TILE},
        "input_bytes": b_in,
        "input_rate_GBps": round(b_in / (ms_step * 1e-3) / 1e9, 1),
    }
    ctx.close()
    print(json.dumps(result), flush=True)


def f64_job(args, d, n) -> dict:
    """The same job at the paper's own arithmetic: complex128 visibilities and mesh, FP64
    transform, phase and image (FP64 weights), the library's default binning tile (64).
    Its own context; 1 warm-up and 3 timed jobs."""
    import numpy as np
    import torch
    from paper_2411_07321_amd import wsg
    progress("f64 job: converting inputs")
    vis = d["vis"].to(torch.complex128)
    wts = d["weights"].to(torch.float64)
    prm = wsg.make_params(**{**d["params"], "precision": "f64"})
    vb = wsg.make_vis(d["uvw"], vis, wts, None, d["freq_hz"], d["row_period"])
    out = torch.empty((1, n, n), dtype=torch.float64, device=vis.device)
    with wsg.Context(0) as c:
        c.set_timing(True)
        c.image(prm, vb, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [c.image(prm, vb, out)[0] for _ in range(3)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 3 * 1e3
    del vis, wts
    torch.cuda.empty_cache()
    n_used = int(sts[-1]["n_used"])
    progress(f"f64 job: {ms:.2f} ms/job")
    return {"ms_per_step": round(ms, 3), "value": n_used / (ms * 1e-3), "unit": "visibilities/s",
            "dtype": "c128 mesh+FFT, f64 phase and image (the paper's arithmetic)",
            "tile": int(prm.tile) if prm.tile else 64,
            "stages_ms": {k: round(float(np.mean([s[k] for s in sts])), 3) for k in STAGES}}


def config3_job(steps: int = 5) -> dict:
    """Batched channels: 32 channels sharing one uvw set (128 antennas, 512 times), uneven
    flagging, one 1024^2 x 16-plane stack and image per channel, every stage one launch
    over all channels (the gridder one persistent launch over every channel's (plane,
    tile) items, largest first), tile and planes per pass autotuned on the data."""
    import numpy as np
    import torch
    from paper_2411_07321_amd import synth, wsg
    progress("config 3: generating")
    ds = synth.config3(device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    vb = wsg.make_vis(dev(ds.uvw), dev(ds.vis), dev(ds.weights), dev(ds.flags), ds.freq_hz,
                      ds.row_period)
    n = ds.grid_n
    out = torch.empty((ds.n_chan, n, n), dtype=torch.float64, device="cuda")
    with wsg.Context(0) as c:
        tile, ppp = c.autotune(wsg.params_for(ds), vb)
        prm = wsg.params_for(ds)
        c.image(prm, vb, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = c.image(prm, vb, out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
    used = int(sum(x["n_used"] for x in st))
    rows, nch = ds.uvw.shape[0], ds.n_chan
    b_in = rows * 24 + rows * nch * (8 + 4 + 1)
    b_grid = nch * ds.n_wplanes * n * n * 8
    b_alg = b_in + 2 * b_grid + nch * n * n * 8
    rate = used / (ms * 1e-3)
    progress(f"config 3: {ms:.2f} ms/job, {rate:.3e} unflagged vis/s (tile {tile}, ppp {ppp})")
    return {"ms_per_step": round(ms, 3), "value": rate, "unit": "unflagged visibilities/s",
            "target": 3.5e10, "vs_target": round(rate / 3.5e10, 4), "n_used": used,
            "visibilities": rows * nch, "tile": tile, "planes_per_pass": ppp,
            "B_alg_bytes": b_alg,
            "path_roofline_frac": round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rows-stride", type=int, default=1,
                    help="keep every k-th row (quick runs only; not the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true",
                    help="skip the extra timing of the job at the paper's FP64 arithmetic")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the extra timing of the 32-channel cube (config 3)")
    ap.add_argument("--kernel", choices=("gauss", "kb"), default="gauss",
                    help="gridding kernel: Gaussian (sigma 0.9) or Kaiser-Bessel")
    ap.add_argument("--w-support", type=int, default=1,
                    help="planes each visibility spreads over (the gridding kernel in w)")
    ap.add_argument("--chunks", type=int, default=0,
                    help="image the workload as a chunked job of this many time chunks "
                         "(wsg_accum_*) instead of one call")
    ap.add_argument("--host-chunks", action="store_true",
                    help="with --chunks: chunks come from pinned host memory (PCIe included)")
    ap.add_argument("--cpu-sample-rows", type=int, default=400_000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a reference elementwise pass of known traffic (2 GiB read, "
                         "2 GiB written per launch) for calibrating rocprofv3 byte counters")
    args = ap.parse_args()
    if args.w_support > 1:
        args.no_cpu_baseline = True   # the oracle's rate is taken on the nearest-plane workload
    if args.copy_calibration:
        import torch
        n = 2 ** 29
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.add(x, 0.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": n * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library images on one GPU; multi-GPU runs (w-plane "
                                   "sharding) are not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2411_07321_amd import synth, wsg

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    progress("generating config 1 on the device")
    t0 = time.perf_counter()
    d = synth.config1_device(dev, rows_stride=args.rows_stride)
    torch.cuda.synchronize()
    progress(f"inputs ready in {time.perf_counter() - t0:.1f} s: vis {tuple(d['vis'].shape)}")
    d["params"]["kernel"] = args.kernel
    d["params"]["w_support"] = args.w_support
    prm = wsg.make_params(**d["params"], tile=TILE)
    vb = wsg.make_vis(d["uvw"], d["vis"], d["weights"], None, d["freq_hz"], d["row_period"])
    n = d["params"]["grid_n"]
    out = torch.empty((1, n, n), dtype=torch.float64, device=dev)
    ctx = wsg.Context(0)
    if args.chunks > 0:
        chunked(args, d, prm, ctx, out)
        return
    ctx.set_timing(True)
    for i in range(args.warmup):
        st = ctx.image(prm, vb, out)
        progress(f"warmup {i}: {st[0]['ms_total']:.2f} ms")
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = ctx.image(prm, vb, out)
        stages.append(st[0])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    s0 = stages[-1]
    n_used = int(s0["n_used"])
    progress(f"timed {args.steps} steps: {ms_step:.2f} ms/step, {n_used} visibilities used")

    mean = {k: float(np.mean([s[k] for s in stages])) for k in STAGES}
    job = {"n_elem": d["vis"].numel(), "n_rows": d["uvw"].shape[0], "n_chan": d["vis"].shape[1],
           "grid_n": n, "n_pl": d["params"]["n_wplanes"], "precision": d["params"]["precision"],
           "n_records": int(s0["n_records"]), "n_tiles": int(s0["n_tiles"]),
           "n_tile_rows": int(s0["n_tile_rows"]), "tile": TILE}
    sb, model = stage_bytes(job)
    dom = max(sb, key=lambda k: mean[k])
    kname = sb[dom][0]
    workload = "config1_4096sq_64w_2.67e8vis" if args.rows_stride == 1 else \
        f"config1_rows_stride_{args.rows_stride}"
    if args.kernel == "kb":
        workload += "_kaiser_bessel"
    if args.w_support > 1:
        workload += f"_w_support{args.w_support}"
    if kname == "k_grid":
        # VALU / LDS-atomic bound: useful arithmetic per launch over the launch time,
        # against the FP32 rate without packed instructions
        flops = GRID_FLOP_PER_VIS * n_used
        achieved = flops / (mean[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": kname, "achieved": round(achieved, 2),
                "peak": round(FP32_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "vendor_peak_packed_fp32": FP32_VENDOR_TFLOPS,
                "frac_of_vendor_peak": round(achieved / FP32_VENDOR_TFLOPS, 4),
                "traffic": load_traffic(kname, workload), "avg_ms": round(mean[dom], 3),
                "alg_flops": flops}
    else:
        kb = sb[dom][1]
        achieved = kb / (mean[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(kname, workload), "avg_ms": round(mean[dom], 3),
                "alg_bytes": kb}
    path_gbs = model["B_alg"] / (ms_step * 1e-3) / 1e9
    stage_rates = {k: {"kernel": v[0], "ms": round(mean[k], 3), "credited_bytes": v[1],
                       "moved_bytes_est": v[2],
                       "moved_GBps": round(v[2] / (mean[k] * 1e-3) / 1e9, 1) if mean[k] > 0 else None}
                   for k, v in sb.items()}
    result = {
        "metric": "visibilities gridded+imaged/s", "value": n_used / (ms_step * 1e-3),
        "unit": "visibilities/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE,
        "data": "synthetic (seeded, device-generated config-1 interferometer data)",
        "config": {"workload": workload, "grid_n": n, "n_wplanes": d["params"]["n_wplanes"],
                   "support": 7, "visibilities": int(d["vis"].numel()), "n_used": n_used,
                   "precision": d["params"]["precision"], "tile": TILE,
                   "kernel": args.kernel, "w_support": args.w_support},
        "roofline": roof,
        "path_roofline": {"bound": "hbm", "B_alg_bytes": model["B_alg"],
                          "achieved": round(path_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(path_gbs / HBM_PEAK_GBS, 4)},
        "stages": stage_rates,
        "occupancy": {"n_records": job["n_records"], "n_tiles": job["n_tiles"],
                      "n_tile_rows": job["n_tile_rows"]},
    }
    try:
        probes = wsg.probe_rates(0, 1 << 31)
        result["device_probes"] = {
            "lds_f64_atomic_adds_per_s": probes["lds_f64_adds_per_s"],
            "copy_GBps": round(probes["copy_bytes_per_s"] / 1e9, 1),
            "note": "measured by wsg_probe_rates: FP64 LDS atomic adds (no return, no bank "
                    "conflicts) and a 2 GiB 16-byte streaming copy (read + write bytes)"}
        lds = wsg.probe_lds(0)
        result["device_probes"]["lds_atomic_adds_per_s"] = {k: float(f"{v:.4g}") for k, v in lds.items()}
        result["device_probes"]["note_lds"] = (
            "wsg_probe_lds: LDS atomic adds without a returned value, FP64 and FP32 with every "
            "lane on its own bank, FP64 with 2 and 16 lanes per bank pair")
        result["path_roofline"]["frac_of_measured_copy"] = round(
            path_gbs / (probes["copy_bytes_per_s"] / 1e9), 4)
        progress(f"probes: LDS f64 adds {probes['lds_f64_adds_per_s']:.3e}/s, copy "
                 f"{probes['copy_bytes_per_s'] / 1e9:.0f} GB/s")
    except wsg.WsgError as e:
        progress(f"probes failed: {e}")
    if not args.no_f64:
        ctx.close()
        result["f64_config1"] = f64_job(args, d, n)
    if not args.no_config3:
        ctx.close()
        result["config3"] = config3_job()
    if not args.no_cpu_baseline:
        progress("cpu baseline: oracle on a bounded sample")
        k = max(1, d["uvw"].shape[0] // args.cpu_sample_rows)
        host = {"uvw": d["uvw"][::k].cpu().numpy().copy(),
                "vis": d["vis"][::k].cpu().numpy().astype(np.complex128),
                "weights": d["weights"][::k].cpu().numpy().astype(np.float64),
                "freq": d["freq_hz"]}
        result["cpu_baseline"] = cpu_baseline(host, d["params"], int(d["vis"].numel()))
        progress(f"cpu baseline {result['cpu_baseline']['value']:.3e} vis/s")
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
