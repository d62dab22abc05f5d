"""The imaging path grids only non-empty (plane, tile) bins and its transform passes
read only what the gridder wrote (tile occupancy).  These cases cluster the uv
coverage so that most tiles, most tile-rows and whole w-planes are empty, with one
blob dense enough to split its bin, at tile sizes where one transform workgroup
spans several tile-rows (N = 64 and 128 with T = 16) and where the tile-row
bitmap needs four words (N = 4096, T = 16), and on the meshes above 4096 (8192,
16384), whose transform rows take a workgroup each.  Raw image against the FP64 oracle:
rel-L2 <= 1e-12 (FP64 path) and <= 1e-5 (FP32 mesh)."""
import numpy as np
import pytest

import oracle
from paper_2411_07321_amd import wsg
from tests.gpuutil import DEV, both_params, cast_inputs, dev, gpu_image, log, oracle_image, rel, PEAK32, peak

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32_phase64": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    c = wsg.Context(0)
    yield c
    c.close()


def _clustered(n, seed, n_clusters=5, per=300, dense=0):
    """uvw in wavelengths for cell 0.2/n: a few compact blobs at three w values
    (so most planes of 8 are empty); with dense > 0 one blob of that many points
    within two cells."""
    rng = np.random.default_rng(seed)
    du = 1.0 / 0.2                       # one cell in wavelengths
    h = 3
    lo, hi = h + 2 - n / 2, n / 2 - h - 3
    ws = np.array([-40.0, 5.0, 60.0])
    parts = []
    for k in range(n_clusters):
        cx, cy = rng.uniform(lo, hi, 2)
        x = np.clip(cx + rng.normal(0, 1.5, per), lo, hi)
        y = np.clip(cy + rng.normal(0, 1.5, per), lo, hi)
        w = ws[k % 3] + rng.normal(0, 0.5, per)
        parts.append(np.stack([x * du, y * du, w], axis=1))
    if dense:
        cx, cy = rng.uniform(lo, hi, 2)
        x = np.clip(cx + rng.normal(0, 0.4, dense), lo, hi)
        y = np.clip(cy + rng.normal(0, 0.4, dense), lo, hi)
        parts.append(np.stack([x * du, y * du, ws[1] + rng.normal(0, 0.2, dense)], axis=1))
    uvw = np.concatenate(parts)
    m = len(uvw)
    vis = (rng.standard_normal(m) + 1j * rng.standard_normal(m))[:, None]
    wts = rng.uniform(0.5, 2.0, (m, 1))
    return uvw, vis, wts


@pytest.mark.parametrize("n,tile,n_w,dense,precisions", [
    (64, 16, 8, 0, ("f64", "f32_phase64")),
    (128, 16, 8, 40_000, ("f64", "f32_phase64")),
    (1024, 32, 8, 40_000, ("f64", "f32_phase64")),
    (4096, 16, 4, 0, ("f32_phase64",)),
    # meshes above 4096: transform rows of one workgroup each, at least N/256 per tile
    (8192, 32, 2, 0, ("f32_phase64",)),
    (16384, 64, 2, 0, ("f32_phase64", "f64")),
])
def test_sparse_stack(ctx, n, tile, n_w, dense, precisions):
    uvw, vis, wts = _clustered(n, seed=n + tile, dense=dense)
    for prec in precisions:
        v, w = cast_inputs(prec, vis, wts)
        wp, op = both_params(n, n_w, 7, 0.2 / n, prec, tile=tile, grid_correct=False,
                             normalize=False)
        img, st = gpu_image(ctx, wp, uvw, v, w)
        ref = oracle_image(op, uvw, v, w, plane_chunk=2)
        assert st[0]["n_used"] == ref["stats"][0]["n_used"]
        e = rel(img[0], ref["raw"][0].real)
        log(f"sparse N={n} T={tile} {prec}: {st[0]['n_used']} used, rel {e:.3e}")
        assert e <= TOL[prec]
        if prec != "f64":
            assert peak(img[0], ref["raw"][0].real) <= PEAK32


def test_dense_stage_grid_still_writes_every_cell(ctx):
    """The stage entry point returns the whole mesh: empty tiles read back as zeros
    even where the buffer held other values."""
    import torch
    n = 256
    uvw, vis, wts = _clustered(n, seed=5)
    v, w = cast_inputs("f32_phase64", vis, wts)
    wp, op = both_params(n, 8, 7, 0.2 / n, "f32_phase64", tile=16)
    out = torch.full((8, n, n), float("nan"), dtype=torch.complex64, device=DEV)
    st = ctx.stage_grid(wp, wsg.make_vis(dev(uvw), dev(v), dev(w)), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.isfinite(got.real).all() and np.isfinite(got.imag).all()
    inp = oracle.Inputs.make(uvw, None, v, w)
    wmin, wmax = oracle.w_range(inp, op)
    g, cnt = oracle.grid(inp, op, wmin, wmax)
    assert st[0]["n_used"] == cnt["n_used"]
    assert rel(got, g) <= 1e-6
