"""wsg_image_noalloc (the entry point for callers that cannot allocate) against
wsg_image on the same device inputs: two calls in a row, the second with a smaller
input, so that the second runs on a scratch array that still holds the first call's
workspace.  Bar: FP64 mesh rel-L2 <= 1e-12 and equal counts; FP32 mesh rel-L2 <= 1e-6
with a per-pixel bound, on the raw image (both results sum the same terms in different
orders)."""
import numpy as np
import pytest

from paper_2411_07321_amd import synth, wsg
from tests.gpuutil import DEV, both_params, cast_inputs, dev, log, peak, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = wsg.Context(0)
    yield c
    c.close()


def _pair(ctx, wp, uvw, vis, wts, freq=None, row_period=0, n_img=1):
    import torch
    vb = wsg.make_vis(dev(uvw), dev(vis), dev(wts), None, freq, row_period)
    n = wp.grid_n
    a = torch.full((n_img, n, n), np.nan, dtype=torch.float64, device=DEV)
    b = torch.full((n_img, n, n), np.nan, dtype=torch.float64, device=DEV)
    st_a = ctx.image(wp, vb, a)
    st_b = ctx.image_noalloc(wp, vb, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), st_a, st_b


def _same_counts(st_a, st_b):
    for x, y in zip(st_a, st_b):
        for k in ("n_used", "n_flagged", "n_dropped", "n_records", "n_tiles", "n_tile_rows"):
            assert x[k] == y[k], (k, x[k], y[k])
        assert x["w_min"] == y["w_min"] and x["w_max"] == y["w_max"]


@pytest.mark.parametrize("precision", ["f64", "f32_phase64"])
def test_noalloc_equals_image_twice(ctx, config0, precision):
    ds = config0
    vis, wts = cast_inputs(precision, ds.vis, ds.weights)
    # FP32 meshes are compared on the raw image: the grid correction amplifies the
    # rounding of differently ordered FP32 sums near the field edge
    f32 = precision != "f64"
    wp, _ = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, precision,
                        grid_correct=not f32, normalize=not f32)
    # whole config 0, then every third time slice of it (a smaller job on the same array)
    sub = np.concatenate([np.arange(t * ds.row_period, (t + 1) * ds.row_period)
                          for t in range(0, ds.uvw.shape[0] // ds.row_period, 3)])
    for name, rows in (("full", slice(None)), ("smaller", sub)):
        log(f"noalloc {precision} {name}: {ds.uvw[rows].shape[0]} rows")
        a, b, st_a, st_b = _pair(ctx, wp, ds.uvw[rows], vis[rows], wts[rows],
                                 row_period=ds.row_period)
        assert np.isfinite(b).all()
        _same_counts(st_a, st_b)
        e = rel(b[0], a[0])
        log(f"  rel {e:.3e} peak {peak(b[0], a[0]):.3e} records {st_b[0]['n_records']}")
        if precision == "f64":
            assert e <= 1e-12
            assert abs(st_a[0]["sum_w"] - st_b[0]["sum_w"]) <= 1e-12 * st_a[0]["sum_w"]
        else:
            assert e <= 1e-6
            assert peak(b[0], a[0]) <= 1e-6


def test_noalloc_cube_kaiser_bessel_and_fold(ctx):
    # channels in metres as a cube, the Kaiser-Bessel window (its tables in the
    # scratch array) and w-folding, after a larger call left other contents behind
    ds = synth.config0()
    rows = slice(0, ds.uvw.shape[0] // 2)
    uvw_m = ds.uvw[rows] * (299792458.0 / 150e6)
    freq = np.array([140e6, 150e6, 160e6])
    vis = np.ascontiguousarray(np.repeat(ds.vis[rows, :1], 3, axis=1), np.complex128)
    wts = np.ones(vis.shape, np.float64)
    wp, _ = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64",
                        per_channel=True, kernel="kb", w_fold=True)
    a, b, st_a, st_b = _pair(ctx, wp, uvw_m, vis, wts, freq=freq, row_period=ds.row_period,
                             n_img=3)
    _same_counts(st_a, st_b)
    for c in range(3):
        assert rel(b[c], a[c]) <= 1e-12, c


def test_noalloc_refuses_large_and_host_jobs(ctx, config0):
    import torch
    ds = config0
    # 4096^2 x 8 planes of complex64 is 1 GiB of stack: far above the scratch array
    wp, _ = both_params(4096, 8, 7, ds.cell_rad / 16, "f32_phase64")
    vis, wts = cast_inputs("f32_phase64", ds.vis, ds.weights)
    vb = wsg.make_vis(dev(ds.uvw), dev(vis), dev(wts), row_period=ds.row_period)
    out = torch.empty((1, 4096, 4096), dtype=torch.float64, device=DEV)
    with pytest.raises(wsg.WsgError) as e:
        ctx.image_noalloc(wp, vb, out)
    assert e.value.status == wsg.ENOMEM
    with pytest.raises(ValueError):
        ctx.image_noalloc(wp, wsg.make_vis(ds.uvw, vis, wts), out)
