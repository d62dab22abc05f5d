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
the FP32 vector peak.
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
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector, vendor figure
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
    rec = 40 if f64 else 16
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


def cpu_baseline(ds_host: dict, params: dict, n_total: int) -> dict:
    """The FP64 oracle (unchanged) on a bounded sample of the same workload, scaled to the
    whole job: gridding of a row subsample with every measurement on one plane (the
    per-visibility work does not depend on the plane count), plus one plane's transform
    and w-correction, extrapolated to all visibilities and planes."""
    import numpy as np
    import oracle
    uvw, vis, wts, freq = ds_host["uvw"], ds_host["vis"], ds_host["weights"], ds_host["freq"]
    m_s = vis.size
    inp = oracle.Inputs.make(uvw, freq, vis, wts)
    n = params["grid_n"]
    prm1 = oracle.Params(n, 1, params["support"], params["cell_rad"], params["kernel_sigma"],
                         kernel=params.get("kernel", "gauss"))

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
    nw = params["n_wplanes"]
    t_est = t_grid * (n_total / m_s) + nw * (t_fft + t_wc)
    return {"value": n_total / t_est, "unit": "visibilities/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 oracle, 1 thread: {m_s:,} visibilities (row subsample) gridded on "
                       f"the {n}^2 mesh in {t_grid:.2f} s, one plane transformed in "
                       f"{t_fft:.2f} s and w-corrected in {t_wc:.2f} s; extrapolated to "
                       f"{n_total:,} visibilities and {nw} planes = {t_est:.0f} s per job")}


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
        "vs_baseline": None, "dtype": "c64 mesh+FFT, f64 phase+image",
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rows-stride", type=int, default=1,
                    help="keep every k-th row (quick runs only; not the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
        print(json.dumps({"error": "this build images on one GPU; multi-GPU runs (w-plane "
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
        # VALU / LDS-atomic bound: useful arithmetic per launch over the launch time
        flops = GRID_FLOP_PER_VIS * n_used
        achieved = flops / (mean[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": kname, "achieved": round(achieved, 2),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
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
        "vs_baseline": None, "dtype": "c64 mesh+FFT, f64 phase+image",
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
