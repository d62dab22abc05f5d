"""Shared helpers of the GPU parity tests: run the HIP library and the FP64 oracle on
the same seeded inputs."""
import math
import sys

import numpy as np

import oracle
from paper_2411_07321_amd import wsg

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


# per-pixel bar of the FP32 paths next to the relative L2 one: the largest pixel error
# against the largest oracle pixel (the precision study measures about 2e-7)
PEAK32 = 1e-6


def peak(a, b):
    """max |a - b| / max |b|: a bad column or tile row cannot hide in a norm."""
    mb = np.abs(b).max()
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0))


def cast_inputs(precision, vis, wts):
    if precision == "f64":
        return (np.ascontiguousarray(vis, np.complex128),
                None if wts is None else np.ascontiguousarray(wts, np.float64))
    return (np.ascontiguousarray(vis, np.complex64),
            None if wts is None else np.ascontiguousarray(wts, np.float32))


def both_params(grid_n, n_wplanes, support, cell_rad, precision="f64", kernel_sigma=0.9,
                w_min=None, w_max=None, plane_lo=0, plane_hi=0, grid_correct=True,
                normalize=True, per_channel=False, naive_nm1=False, tile=0, kernel="gauss",
                kernel_beta=0.0, w_fold=False, w_support=1):
    wp = wsg.make_params(grid_n, n_wplanes, support, cell_rad, precision, kernel_sigma, w_min,
                         w_max, plane_lo, plane_hi, grid_correct, normalize, per_channel,
                         naive_nm1, tile, kernel, kernel_beta, w_fold, w_support)
    op = oracle.Params(grid_n, n_wplanes, support, cell_rad, kernel_sigma,
                       math.nan if w_min is None else w_min, math.nan if w_max is None else w_max,
                       plane_lo, plane_hi, grid_correct, normalize, per_channel, kernel,
                       kernel_beta, w_fold, w_support)
    return wp, op


def gpu_image(ctx, wp, uvw, vis, wts=None, flags=None, freq=None, on_device=True, row_period=0):
    """Image through the C ABI; returns (image [n_img,N,N] numpy, stats list)."""
    import torch
    n_img = wsg.n_images(wp, wsg.make_vis(uvw, vis, wts, flags, freq))
    n = wp.grid_n
    if on_device:
        vb = wsg.make_vis(dev(uvw), dev(vis), None if wts is None else dev(wts),
                          None if flags is None else dev(flags), freq, row_period)
        out = torch.full((n_img, n, n), float("nan"), dtype=torch.float64, device=DEV)
        st = ctx.image(wp, vb, out)
        torch.cuda.synchronize()
        return out.cpu().numpy(), st
    vb = wsg.make_vis(np.ascontiguousarray(uvw), np.ascontiguousarray(vis),
                      None if wts is None else np.ascontiguousarray(wts),
                      None if flags is None else np.ascontiguousarray(flags), freq, row_period)
    out = np.full((n_img, n, n), np.nan)
    st = ctx.image(wp, vb, out)
    return out, st


def oracle_image(op, uvw, vis, wts=None, flags=None, freq=None, **kw):
    return oracle.image(oracle.Inputs.make(uvw, freq, vis, wts, flags), op, **kw)


def assert_stats(st, ost, sum_w_rel=1e-12):
    for a, b in zip(st, ost):
        assert a["n_used"] == b["n_used"], (a, b)
        assert a["n_flagged"] == b["n_flagged"], (a, b)
        assert a["n_dropped"] == b["n_dropped"], (a, b)
        assert abs(a["sum_w"] - b["sum_w"]) <= sum_w_rel * max(1.0, abs(b["sum_w"])), (a, b)
        assert a["w_min"] == b["w_min"] and a["w_max"] == b["w_max"], (a, b)
