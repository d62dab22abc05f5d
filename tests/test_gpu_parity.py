"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on the same
seeded inputs.  Tolerances: FP64 path rel-L2 <= 1e-12; FP32 mesh paths rel-L2 <= 1e-5
on the raw image (Re A before the post factors), the bar stated for the plain path."""
import math

import numpy as np
import pytest

import oracle
from paper_2411_07321_amd import synth, wsg
from tests.gpuutil import (DEV, assert_stats, both_params, cast_inputs, dev, gpu_image, log,
                           oracle_image, rel, PEAK32, peak)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = wsg.Context(0)
    yield c
    c.close()


# ---------------------------------------------------------------- end to end, config 0
@pytest.mark.parametrize("on_device,row_period", [(True, 496), (False, 496), (True, 0), (True, 37)])
def test_config0_f64_image(ctx, config0, on_device, row_period):
    # row_period: the baselines per time slice (496), no hint, and a wrong hint; the
    # hint only changes the traversal order of the binning passes
    ds = config0
    log(f"config0 f64 image on_device={on_device} row_period={row_period}")
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64")
    img, st = gpu_image(ctx, wp, ds.uvw, ds.vis, ds.weights, on_device=on_device,
                        row_period=row_period)
    ref = oracle_image(op, ds.uvw, ds.vis, ds.weights)
    assert_stats(st, ref["stats"])
    assert rel(img[0], ref["image"][0]) <= TOL64


@pytest.mark.parametrize("ppp", [1, 3])
def test_config0_f64_passes_over_planes(ctx, config0, ppp):
    # the 8 planes in passes of 1 or 3 (3, 3, 2) planes: each pass grids, transforms
    # and w-corrects its planes into the image
    ds = config0
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64")
    wp.planes_per_pass = ppp
    img, st = gpu_image(ctx, wp, ds.uvw, ds.vis, ds.weights, row_period=ds.row_period)
    ref = oracle_image(op, ds.uvw, ds.vis, ds.weights)
    assert_stats(st, ref["stats"])
    assert rel(img[0], ref["image"][0]) <= TOL64


def test_config0_f64_raw(ctx, config0):
    ds = config0
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64",
                         grid_correct=False, normalize=False)
    img, st = gpu_image(ctx, wp, ds.uvw, ds.vis, ds.weights, row_period=ds.row_period)
    ref = oracle_image(op, ds.uvw, ds.vis, ds.weights)
    assert rel(img[0], ref["raw"][0].real) <= TOL64


@pytest.mark.parametrize("precision", ["f32_phase64", "f32_phase32"])
def test_config0_f32_paths(ctx, config0, precision):
    ds = config0
    vis, wts = cast_inputs(precision, ds.vis, ds.weights)
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, precision,
                         grid_correct=False, normalize=False)
    img, st = gpu_image(ctx, wp, ds.uvw, vis, wts, row_period=ds.row_period)
    ref = oracle_image(op, ds.uvw, vis, wts)
    assert_stats(st, ref["stats"], sum_w_rel=1e-12)
    e = rel(img[0], ref["raw"][0].real)
    log(f"config0 {precision}: raw rel err {e:.3e}")
    assert e <= TOL32
    assert peak(img[0], ref["raw"][0].real) <= PEAK32


# ---------------------------------------------------------------- stages
@pytest.mark.parametrize("precision", ["f64", "f32_phase64"])
def test_stage_grid(ctx, config0, precision):
    import torch
    ds = config0
    vis, wts = cast_inputs(precision, ds.vis, ds.weights)
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, precision)
    ctype = torch.complex128 if precision == "f64" else torch.complex64
    out = torch.zeros((ds.n_wplanes, ds.grid_n, ds.grid_n), dtype=ctype, device=DEV)
    st = ctx.stage_grid(wp, wsg.make_vis(dev(ds.uvw), dev(vis), dev(wts), row_period=ds.row_period),
                        out)
    inp = oracle.Inputs.make(ds.uvw, None, vis, wts)
    wmin, wmax = oracle.w_range(inp, op)
    g, cnt = oracle.grid(inp, op, wmin, wmax)
    got = out.cpu().numpy()
    e = rel(got, g)
    log(f"stage grid {precision}: rel err {e:.3e}")
    assert e <= (TOL64 if precision == "f64" else 1e-6)
    assert st[0]["n_used"] == cnt["n_used"]


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384])
@pytest.mark.parametrize("precision", ["f64", "f32_phase64"])
def test_stage_fft(ctx, n, precision):
    # 8192 and 16384: one or two rows per workgroup, components exchanged one at a time
    import torch
    n_pl = 3 if n <= 1024 else (2 if n <= 4096 else 1)
    g = synth.random_planes(n_pl, n, seed=100 + n)
    ctype = torch.complex128 if precision == "f64" else torch.complex64
    x = dev(g).to(ctype)
    wp, _ = both_params(n, n_pl, 7, 0.2 / n, precision)
    ctx.stage_fft(wp, x)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    ref = oracle.fft_planes(g.astype(np.complex64).astype(np.complex128)
                            if precision != "f64" else g)
    e = rel(got, ref)
    log(f"stage fft N={n} {precision}: rel err {e:.3e}")
    assert e <= (TOL64 if precision == "f64" else 2e-6)


def test_stage_fft_host_buffers(ctx):
    g = synth.random_planes(2, 64, seed=5)
    wp, _ = both_params(64, 2, 7, 0.2 / 64, "f64")
    x = g.copy()
    ctx.stage_fft(wp, x)
    assert rel(x, oracle.fft_planes(g)) <= TOL64


@pytest.mark.parametrize("precision", ["f64", "f32_phase64", "f32_phase32"])
def test_stage_wcorrect(ctx, precision):
    import torch
    n, nw = 256, 6
    F = synth.random_planes(nw, n, seed=77)
    cell = 0.35 / n                        # field edge at l, m = 0.175
    w_min, w_max, sum_w = -3000.0, 4200.0, 123.5
    wp, op = both_params(n, nw, 7, cell, precision)
    ctype = torch.complex128 if precision == "f64" else torch.complex64
    Fd = dev(F).to(ctype)
    out = torch.empty((n, n), dtype=torch.float64, device=DEV)
    ctx.stage_wcorrect(wp, Fd, w_min, w_max, sum_w, out)
    torch.cuda.synchronize()
    Fin = Fd.cpu().numpy().astype(np.complex128)
    A = oracle.wcorrect(Fin, w_min, w_max, nw, cell)
    ref = oracle.post(A, sum_w, op)
    e = rel(out.cpu().numpy(), ref)
    log(f"stage wcorrect {precision}: rel err {e:.3e}")
    # f32_phase64: FP64 argument reduced exactly, FP32 sin/cos of the reduced angle
    tol = {"f64": TOL64, "f32_phase64": 1e-6, "f32_phase32": 1e-3}[precision]
    assert e <= tol


# ---------------------------------------------------------------- FP32 at a larger mesh
def test_f32_random_1024_ragged(ctx):
    n, nw = 1024, 16
    uvw, vis, wts = synth.random_visibilities(300_001, 1, n, 0.2 / n, seed=31, w_extent=800.0)
    vis, wts = cast_inputs("f32_phase64", vis, wts)
    wp, op = both_params(n, nw, 7, 0.2 / n, "f32_phase64", grid_correct=False, normalize=False)
    # row period 1000: 301 time slices, the last one ragged
    img, st = gpu_image(ctx, wp, uvw, vis, wts, row_period=1000)
    ref = oracle_image(op, uvw, vis, wts)
    assert_stats(st, ref["stats"])
    e = rel(img[0], ref["raw"][0].real)
    log(f"f32 1024^2 x 16, 300001 vis: raw rel err {e:.3e}")
    assert e <= TOL32
    assert peak(img[0], ref["raw"][0].real) <= PEAK32


# ---------------------------------------------------------------- edge cases
def _small(n_rows, seed=3, n=64, nw=4, prec="f64", **kw):
    uvw, vis, wts = synth.random_visibilities(n_rows, 1, n, 0.2 / n, seed=seed, **kw)
    return uvw, *cast_inputs(prec, vis, wts)


def test_empty_input(ctx):
    wp, op = both_params(64, 4, 7, 0.2 / 64, "f64")
    img, st = gpu_image(ctx, wp, np.zeros((0, 3)), np.zeros((0, 1), np.complex128))
    assert np.all(img == 0) and st[0]["n_used"] == 0 and st[0]["n_dropped"] == 0


def test_all_flagged(ctx):
    uvw, vis, wts = _small(500)
    flags = np.ones(vis.shape, np.uint8)
    wp, op = both_params(64, 4, 7, 0.2 / 64, "f64")
    img, st = gpu_image(ctx, wp, uvw, vis, wts, flags)
    assert np.all(img == 0)
    assert st[0]["n_flagged"] == 500 and st[0]["n_used"] == 0


def test_bad_values_and_footprint_edges(ctx):
    n, cell = 64, 1.0 / 100
    du = 1.0 / (n * cell)
    uvw = np.array([[10.0, 5.0, 1.0], [10.0, 5.0, 2.0], [np.nan, 5.0, 1.0], [10.0, 5.0, 1.0],
                    [(n / 2 - 3) * du, 0.0, 1.0], [(n / 2 - 4) * du, 0.0, 3.0],
                    [-(n / 2 - 3) * du, 0.0, 1.5], [10.0, 5.0, 1.0], [0.0, (n / 2 - 4) * du, -2.0],
                    [1.0, 1.0, np.inf]])
    vis = np.array([1, 1, 1, 1, 1, 2, 3, np.inf + 0j, 4j, 1], complex)[:, None]
    wts = np.array([1, 1, 1, 0, 1, 1, 1, 1, 0.5, 1], float)[:, None]
    fl = np.array([0, 1, 0, 0, 0, 0, 0, 0, 0, 0], np.uint8)[:, None]
    wp, op = both_params(n, 3, 7, cell, "f64")
    img, st = gpu_image(ctx, wp, uvw, vis, wts, fl)
    ref = oracle_image(op, uvw, vis, wts, fl)
    assert_stats(st, ref["stats"])
    assert rel(img[0], ref["image"][0]) <= TOL64


@pytest.mark.parametrize("precision,per_channel", [("f64", False), ("f32_phase64", False),
                                                   ("f64", True)])
def test_w_range_edge_rows_invalid(ctx, precision, per_channel):
    """The rows at both ends of the w range carry a NaN visibility and a zero weight,
    so the rows whose uvw and flags pass span a wider range than the valid data; the
    planes follow the valid data alone (the planes, counts and image equal the
    oracle's).  Cube variant: 3 channels in metres, and only one channel of each edge
    row fails, so only that image's range is narrower than its uvw range."""
    rng = np.random.default_rng(77)
    nch = 3 if per_channel else 1
    uvw, vis, wts = synth.random_visibilities(4000, nch, 64, 0.2 / 64, seed=78, w_extent=150.0)
    freq = None
    if per_channel:
        freq = 150e6 * (1.0 + 0.05 * np.arange(nch))
        uvw = uvw * (299792458.0 / 150e6)
    hi, lo = int(np.argmax(uvw[:, 2])), int(np.argmin(uvw[:, 2]))
    ch = 1 if per_channel else 0
    vis[hi, ch] = np.nan
    wts[lo, ch] = 0.0
    vis[rng.integers(0, 4000, 20), 0] = np.inf       # scattered bad values as well
    vis, wts = cast_inputs(precision, vis, wts)
    wp, op = both_params(64, 5, 7, 0.2 / 64, precision, per_channel=per_channel)
    img, st = gpu_image(ctx, wp, uvw, vis, wts, freq=freq)
    ref = oracle_image(op, uvw, vis, wts, freq=freq)
    assert_stats(st, ref["stats"])
    assert st[ch]["w_max"] < uvw[hi, 2] * (freq[ch] / 299792458.0 if per_channel else 1.0)
    assert st[ch]["w_min"] > uvw[lo, 2] * (freq[ch] / 299792458.0 if per_channel else 1.0)
    for k in range(img.shape[0]):
        assert rel(img[k], ref["image"][k]) <= (TOL64 if precision == "f64" else TOL32)


@pytest.mark.parametrize("n_chan,offset", [(4, 0), (2, 0), (4, 1)])
def test_f32_channels_flags_and_bad_values(ctx, n_chan, offset):
    """Single-image complex64 jobs of 2 and 4 channels (the validity pass takes one
    thread per row with vector loads of the channels), with flags, weights <= 0, NaN
    and infinite values and footprints off the mesh; offset 1: the arrays start one
    row into their buffers, so the loads are not 16-byte aligned and the pass takes
    one thread per (row, channel) instead.  Counts equal the oracle's, raw image
    within the FP32 bar."""
    import torch
    rng = np.random.default_rng(40 + n_chan + offset)
    m, n = 6001, 128
    uvw, vis1, wts1 = synth.random_visibilities(m + offset, 1, n, 0.2 / n, seed=41, w_extent=300.0)
    freq = 150e6 * (1.0 + 0.01 * np.arange(n_chan))
    uvw = uvw * (299792458.0 / 150e6)              # metres: channels scale u, v, w
    vis = (rng.standard_normal((m + offset, n_chan)) + 1j * rng.standard_normal((m + offset, n_chan)))
    wts = rng.uniform(0.5, 1.5, (m + offset, n_chan))
    flags = (rng.random((m + offset, n_chan)) < 0.1).astype(np.uint8)
    wts[rng.random(wts.shape) < 0.02] = 0.0
    vis[rng.random(vis.shape) < 0.01] = np.nan
    uvw[rng.random(m + offset) < 0.01, 0] = np.inf
    uvw[::97, 0] = 1e6                               # off the mesh
    vis, wts = cast_inputs("f32_phase64", vis, wts)
    wp, op = both_params(n, 6, 7, 0.2 / n, "f32_phase64", grid_correct=False, normalize=False)
    sl = slice(offset, None)
    vb = wsg.make_vis(dev(uvw)[sl], dev(vis)[sl], dev(wts)[sl], dev(flags)[sl], freq)
    out = torch.full((1, n, n), float("nan"), dtype=torch.float64, device=DEV)
    st = ctx.image(wp, vb, out)
    torch.cuda.synchronize()
    ref = oracle_image(op, uvw[sl], vis[sl], wts[sl], flags[sl], freq)
    assert_stats(st, ref["stats"])
    e = rel(out.cpu().numpy()[0], ref["raw"][0].real)
    log(f"f32 {n_chan} channels offset {offset}: {st[0]['n_used']} used of {m * n_chan}, rel {e:.2e}")
    assert e <= TOL32


def test_single_visibility_and_zero_w_spread(ctx):
    uvw = np.array([[37.0, -12.5, 55.0]])
    vis = np.array([[0.3 + 0.4j]])
    wp, op = both_params(128, 5, 7, 0.3 / 128, "f64")
    img, st = gpu_image(ctx, wp, uvw, vis)
    ref = oracle_image(op, uvw, vis)
    assert st[0]["w_min"] == st[0]["w_max"] == 55.0
    assert rel(img[0], ref["image"][0]) <= TOL64


@pytest.mark.parametrize("support", [1, 3, 5, 9, 15])
def test_supports(ctx, support):
    # compared before the grid correction: for wide kernels 1/C(nu) reaches ~1e12 at the
    # field edge and amplifies the last-bit differences of two independent quadratures
    uvw, vis, wts = _small(4001, n=128, nw=3)
    wp, op = both_params(128, 3, support, 0.2 / 128, "f64", kernel_sigma=0.5 + support / 8,
                         grid_correct=False)
    img, st = gpu_image(ctx, wp, uvw, vis, wts)
    ref = oracle_image(op, uvw, vis, wts)
    assert_stats(st, ref["stats"])
    assert rel(img[0], ref["image"][0]) <= TOL64


@pytest.mark.parametrize("n", [16, 32])
def test_tiny_meshes(ctx, n):
    uvw, vis, wts = _small(777, n=n)
    wp, op = both_params(n, 2, 7, 0.2 / n, "f64")
    img, st = gpu_image(ctx, wp, uvw, vis, wts)
    ref = oracle_image(op, uvw, vis, wts)
    assert rel(img[0], ref["image"][0]) <= TOL64


@pytest.mark.parametrize("tile", [16, 32, 64])
def test_tiles_f32(ctx, tile):
    n = 256
    uvw, vis, wts = _small(20_000, n=n, prec="f32_phase64", seed=8)
    wp, op = both_params(n, 4, 7, 0.2 / n, "f32_phase64", tile=tile, grid_correct=False,
                         normalize=False)
    img, st = gpu_image(ctx, wp, uvw, vis, wts)
    ref = oracle_image(op, uvw, vis, wts)
    assert rel(img[0], ref["raw"][0].real) <= TOL32
    assert peak(img[0], ref["raw"][0].real) <= PEAK32


@pytest.mark.parametrize("tile,support", [(16, 15), (32, 7), (64, 1)])
def test_tiles_f64(ctx, tile, support):
    """The complex128 records at every tile size: the widest kernel on the smallest tile
    (the largest cell field of a record), and a one-cell kernel with visibilities at the
    low edge of the mesh (coordinates below 2 cells, where a record's sub-cell offset
    can round in its last bit).  Before the grid correction, as in test_supports."""
    n = 256
    cell = 0.2 / n
    uvw, vis, wts = _small(6000, n=n, seed=31)
    if support == 1:
        du = 1.0 / (n * cell)
        x = np.array([0.3, 0.7, 1.2, 1.49, 1.51, 1.999])
        uvw[:6, 0] = (x - n / 2) * du
        uvw[:6, 1] = (x[::-1] - n / 2) * du
    wp, op = both_params(n, 4, support, cell, "f64", tile=tile, kernel_sigma=0.5 + support / 8,
                         grid_correct=False)
    img, st = gpu_image(ctx, wp, uvw, vis, wts)
    ref = oracle_image(op, uvw, vis, wts)
    assert_stats(st, ref["stats"])
    assert st[0]["n_dropped"] == 0
    assert rel(img[0], ref["image"][0]) <= TOL64


def test_split_hot_tiles(ctx):
    # 60,000 visibilities packed into a few cells: bins far above one work item
    rng = np.random.default_rng(12)
    n, cell = 128, 0.2 / 128
    du = 1.0 / (n * cell)
    m = 60_000
    uvw = np.stack([rng.normal(0, 2 * du, m), rng.normal(0, 2 * du, m),
                    rng.uniform(-10, 10, m)], axis=1)
    vis = (rng.standard_normal(m) + 1j * rng.standard_normal(m))[:, None]
    for prec, tol in (("f64", TOL64), ("f32_phase64", TOL32)):
        v, w = cast_inputs(prec, vis, np.ones(vis.shape))
        wp, op = both_params(n, 2, 7, cell, prec, grid_correct=False, normalize=False)
        img, st = gpu_image(ctx, wp, uvw, v, w)
        ref = oracle_image(op, uvw, v, w)
        e = rel(img[0], ref["raw"][0].real)
        log(f"split hot tiles {prec}: {e:.3e}")
        assert e <= tol
        if prec != "f64":
            assert peak(img[0], ref["raw"][0].real) <= PEAK32


def test_plane_shards_sum(ctx, config0):
    ds = config0
    wp, op = both_params(ds.grid_n, ds.n_wplanes, 7, ds.cell_rad, "f64", grid_correct=False,
                         normalize=False)
    full, st = gpu_image(ctx, wp, ds.uvw, ds.vis, ds.weights)
    acc = 0
    for lo, hi in ((0, 3), (3, 8)):
        wp2, _ = both_params(ds.grid_n, ds.n_wplanes, 7, ds.cell_rad, "f64", w_min=st[0]["w_min"],
                             w_max=st[0]["w_max"], plane_lo=lo, plane_hi=hi, grid_correct=False,
                             normalize=False)
        part, _ = gpu_image(ctx, wp2, ds.uvw, ds.vis, ds.weights)
        acc = acc + part
    assert rel(acc, full) <= 1e-13


def test_given_w_range_drops_outside(ctx):
    uvw, vis, wts = _small(3000, w_extent=100.0)
    wp, op = both_params(64, 4, 7, 0.2 / 64, "f64", w_min=-50.0, w_max=60.0)
    img, st = gpu_image(ctx, wp, uvw, vis, wts)
    ref = oracle_image(op, uvw, vis, wts)
    assert_stats(st, ref["stats"])
    assert st[0]["n_dropped"] > 0
    assert rel(img[0], ref["image"][0]) <= TOL64


# ---------------------------------------------------------------- channels
def test_channels_metres_mfs_and_cube(ctx):
    rng = np.random.default_rng(21)
    rows, nch, n = 5000, 5, 128
    uvw = rng.uniform(-60, 60, (rows, 3))
    freq = np.linspace(120e6, 180e6, nch)
    vis = rng.standard_normal((rows, nch)) + 1j * rng.standard_normal((rows, nch))
    wts = rng.uniform(0.5, 2.0, (rows, nch))
    flags = (rng.random((rows, nch)) < 0.2).astype(np.uint8)
    for per_channel in (False, True):
        wp, op = both_params(n, 4, 7, 0.2 / n, "f64", per_channel=per_channel)
        img, st = gpu_image(ctx, wp, uvw, vis, wts, flags, freq, row_period=50)
        ref = oracle_image(op, uvw, vis, wts, flags, freq)
        assert_stats(st, ref["stats"])
        assert img.shape[0] == (nch if per_channel else 1)
        for i in range(img.shape[0]):
            assert rel(img[i], ref["image"][i]) <= TOL64
