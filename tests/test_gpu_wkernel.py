"""Gridding kernel in w (Eq. 3's G over u, v and w; w_support planes): library against
the FP64 oracle with the same kernel: rel-L2 <= 1e-12 (FP64 mesh), <= 1e-5 raw (FP32
mesh); the gridded stack itself; and the accuracy gain against the exact transform."""
import numpy as np
import pytest

import oracle
from paper_2411_07321_amd import synth, wsg
from tests import pinlib
from tests.gpuutil import (DEV, assert_stats, both_params, cast_inputs, dev, gpu_image, log,
                           oracle_image, rel, PEAK32, peak)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = wsg.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kernel,sw,corrected", [("gauss", 5, True), ("kb", 5, True),
                                                 ("kb", 3, True), ("kb", 7, False)])
def test_config0_w_kernel_f64(ctx, config0, kernel, sw, corrected):
    """Grid-corrected where the window's transform stays within a factor of a few of its
    peak over the field; S_w = 7 on 8 planes leaves 2 planes for the data, so dw (n - 1)
    reaches 0.7 at the corners, where 1/C_w of the Kaiser-Bessel window is 1.2e4 and
    lifts last-bit differences of the two summation orders above 1e-12: compared raw."""
    ds = config0
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64", kernel=kernel,
                         w_support=sw, grid_correct=corrected)
    img, st = gpu_image(ctx, wp, ds.uvw, ds.vis, ds.weights, row_period=ds.row_period)
    ref = oracle_image(op, ds.uvw, ds.vis, ds.weights)
    assert_stats(st, ref["stats"])
    e = rel(img[0], ref["image"][0])
    log(f"w kernel {kernel} S_w={sw} config0 f64: rel err {e:.3e}, records {st[0]['n_records']}")
    assert e <= TOL64


@pytest.mark.parametrize("precision", ["f32_phase64", "f32_phase32"])
def test_config0_w_kernel_f32(ctx, config0, precision):
    ds = config0
    vis, wts = cast_inputs(precision, ds.vis, ds.weights)
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, precision,
                         grid_correct=False, normalize=False, w_support=7)
    img, st = gpu_image(ctx, wp, ds.uvw, vis, wts, row_period=ds.row_period)
    ref = oracle_image(op, ds.uvw, vis, wts)
    assert_stats(st, ref["stats"])
    e = rel(img[0], ref["raw"][0].real)
    log(f"w kernel S_w=7 config0 {precision}: raw rel err {e:.3e}")
    assert e <= TOL32
    assert peak(img[0], ref["raw"][0].real) <= PEAK32


@pytest.mark.parametrize("precision,kernel", [("f64", "gauss"), ("f32_phase64", "gauss"),
                                              ("f64", "kb")])
def test_w_kernel_stage_grid(ctx, precision, kernel):
    """The stack itself: every visibility on its 3 planes with the window's weights,
    including rows at the very ends of the w range, whose outer planes sit exactly at
    |d| = S_w / 2, the edge of the Kaiser-Bessel window (1/I0(beta) inside, 0 beyond)."""
    import torch
    n, nw = 128, 6
    uvw, vis, wts = synth.random_visibilities(30_000, 1, n, 0.2 / n, seed=83, w_extent=60.0)
    uvw[:3, 2] = [uvw[:, 2].min(), uvw[:, 2].max(), 0.0]
    vis, wts = cast_inputs(precision, vis, wts)
    wp, op = both_params(n, nw, 7, 0.2 / n, precision, w_support=3, tile=32, kernel=kernel)
    ctype = torch.complex128 if precision == "f64" else torch.complex64
    out = torch.zeros((nw, n, n), dtype=ctype, device=DEV)
    st = ctx.stage_grid(wp, wsg.make_vis(dev(uvw), dev(vis), dev(wts)), out)
    torch.cuda.synchronize()
    inp = oracle.Inputs.make(uvw, None, vis, wts)
    wmin, wmax = oracle.w_range(inp, op)
    g, cnt = oracle.grid(inp, op, wmin, wmax)
    e = rel(out.cpu().numpy(), g)
    log(f"w kernel stage grid {precision} {kernel}: rel err {e:.3e}")
    assert st[0]["n_used"] == cnt["n_used"]
    assert e <= (TOL64 if precision == "f64" else 1e-6)


def test_w_kernel_approaches_the_exact_transform(ctx):
    """Wide field (0.5 rad), 12 planes over |w| <= 30: 7 planes of kernel and its
    correction bring the image far closer to the exact transform (the oracle: 26x)."""
    n, cell = 256, 0.5 / 256
    rng = np.random.default_rng(71)
    m = 6000
    du = 1.0 / (n * cell)
    uvw = np.stack([rng.uniform(-0.3, 0.3, m) * n * du, rng.uniform(-0.3, 0.3, m) * n * du,
                    rng.uniform(-30.0, 30.0, m)], axis=1)
    vis = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    wts = np.ones(m)
    q = np.array([40, 60, 200, 220, 128, 30, 100, 160])
    p = np.array([50, 210, 45, 190, 20, 128, 100, 170])
    De = pinlib.exact_dft(uvw, vis, wts, n, cell, q, p)
    err = {}
    for sw in (1, 7):
        wp, op = both_params(n, 12, 7, cell, "f32_phase64", w_support=sw)
        v32, w32 = cast_inputs("f32_phase64", vis[:, None], wts[:, None])
        img, _ = gpu_image(ctx, wp, uvw, v32, w32)
        err[sw] = np.abs(img[0][q, p] - De).max()
    log(f"w kernel vs exact: nearest plane {err[1]:.3e}, 7 planes {err[7]:.3e}")
    assert err[7] < 0.1 * err[1]


def test_w_kernel_in_chunks_and_degenerate_range(ctx, config0):
    import torch
    ds = config0
    lo, hi = float(ds.uvw[:, 2].min()) - 1.0, float(ds.uvw[:, 2].max()) + 1.0
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64", w_min=lo,
                         w_max=hi, w_support=5)
    m = ds.uvw.shape[0]
    out = torch.zeros((1, ds.grid_n, ds.grid_n), dtype=torch.float64, device=DEV)
    with wsg.Accum(ctx, wp, 1) as acc:
        for a, b in ((0, m // 3), (m // 3, m)):
            acc.add(wsg.make_vis(dev(ds.uvw[a:b]), dev(ds.vis[a:b]), dev(ds.weights[a:b])))
        st = acc.finish(out)
    torch.cuda.synchronize()
    ref = oracle_image(op, ds.uvw, ds.vis, ds.weights)
    assert_stats(st, ref["stats"])
    assert rel(out.cpu().numpy()[0], ref["image"][0]) <= TOL64
    # every w equal: the plane width is 0 and the kernel in w does nothing
    uvw = ds.uvw.copy()
    uvw[:, 2] = 12.5
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64", w_support=5)
    img, st = gpu_image(ctx, wp, uvw, ds.vis, ds.weights)
    ref = oracle_image(op, uvw, ds.vis, ds.weights)
    assert_stats(st, ref["stats"])
    assert rel(img[0], ref["image"][0]) <= TOL64


@pytest.mark.parametrize("precision", ["f64", "f32_phase64"])
def test_w_kernel_stage_wcorrect(ctx, precision):
    """The w-correction entry point alone with a kernel in w: planes at w0 + (k + 1/2) dw
    of the padded geometry, and the window's transform divided out per pixel."""
    import torch
    n, nw = 256, 9
    F = synth.random_planes(nw, n, seed=78)
    cell = 0.35 / n
    w_min, w_max, sum_w = -20.0, 28.0, 77.25     # dw |n - 1| <= 0.3 over the field
    wp, op = both_params(n, nw, 7, cell, precision, w_support=5)
    ctype = torch.complex128 if precision == "f64" else torch.complex64
    Fd = dev(F).to(ctype)
    out = torch.empty((n, n), dtype=torch.float64, device=DEV)
    ctx.stage_wcorrect(wp, Fd, w_min, w_max, sum_w, out)
    torch.cuda.synchronize()
    Fin = Fd.cpu().numpy().astype(np.complex128)
    A = oracle.wcorrect(Fin, w_min, w_max, nw, cell, 0, 5)
    ref = oracle.post(A, sum_w, op, w_min, w_max)
    e = rel(out.cpu().numpy(), ref)
    log(f"w kernel stage wcorrect {precision}: rel err {e:.3e}")
    assert e <= (TOL64 if precision == "f64" else 1e-6)
