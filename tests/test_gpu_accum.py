"""Chunked imaging (data loaded chunk after chunk by time or by frequency, Sec. 5):
an accumulator keeps the w-stack resident while chunks are binned and gridded into
it, then transforms and w-corrects once.  Its image must equal the FP64 oracle's
image of all chunks together: rel-L2 <= 1e-12 (FP64 mesh), <= 1e-5 on the raw
image (FP32 mesh); counts equal, weight sums to 1e-12."""
import numpy as np
import pytest

from paper_2411_07321_amd import synth, wsg
from tests.gpuutil import (DEV, assert_stats, both_params, cast_inputs, dev, log, oracle_image,
                           rel, PEAK32, peak)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = wsg.Context(0)
    yield c
    c.close()


def _w_range(uvw, freq=None):
    w = uvw[:, 2] if freq is None else np.concatenate([uvw[:, 2] * f / 299792458.0 for f in freq])
    return float(w.min()) - 1.0, float(w.max()) + 1.0


def _accumulate(ctx, wp, chunks, n_chan, n, n_img=1, on_device=True, freq_of=None):
    """chunks: list of (row slice, channel slice); returns (image, stats)."""
    import torch
    with wsg.Accum(ctx, wp, n_chan) as acc:
        for uvw, vis, wts, flags, freq in chunks:
            if on_device:
                vb = wsg.make_vis(dev(uvw), dev(vis), None if wts is None else dev(wts),
                                  None if flags is None else dev(flags), freq)
            else:
                vb = wsg.make_vis(np.ascontiguousarray(uvw), np.ascontiguousarray(vis),
                                  None if wts is None else np.ascontiguousarray(wts),
                                  None if flags is None else np.ascontiguousarray(flags), freq)
            acc.add(vb)
        if on_device:
            out = torch.full((n_img, n, n), float("nan"), dtype=torch.float64, device=DEV)
            st = acc.finish(out)
            torch.cuda.synchronize()
            return out.cpu().numpy(), st
        out = np.full((n_img, n, n), np.nan)
        st = acc.finish(out)
        return out, st


def _row_chunks(uvw, vis, wts, cuts, flags=None, freq=None):
    out = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        out.append((uvw[a:b], vis[a:b], None if wts is None else wts[a:b],
                    None if flags is None else flags[a:b], freq))
    return out


@pytest.mark.parametrize("on_device", [True, False])
def test_time_chunks_f64(ctx, config0, on_device):
    """Config 0 in four chunks of time (one empty), grid-corrected and normalised."""
    ds = config0
    lo, hi = _w_range(ds.uvw)
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64", w_min=lo, w_max=hi)
    m = ds.uvw.shape[0]
    cuts = [0, 4_960, 4_960, 17_000, m]
    img, st = _accumulate(ctx, wp, _row_chunks(ds.uvw, ds.vis, ds.weights, cuts), 1, ds.grid_n,
                          on_device=on_device)
    ref = oracle_image(op, ds.uvw, ds.vis, ds.weights)
    assert_stats(st, ref["stats"])
    e = rel(img[0], ref["image"][0])
    log(f"accum config0 f64 on_device={on_device}: rel err {e:.3e}")
    assert e <= TOL64


@pytest.mark.parametrize("on_device", [True, False])
def test_time_chunks_f32_with_a_hot_bin(ctx, on_device):
    """1024^2 x 16 planes, 200,001 visibilities in three uneven chunks; 60,000 of them in
    one cell, so that bin splits over work items inside a chunk."""
    n, nw = 1024, 16
    uvw, vis, wts = synth.random_visibilities(200_001, 1, n, 0.2 / n, seed=91, w_extent=500.0)
    uvw[70_000:130_000, :2] = uvw[70_000:130_000, :2] * 1e-3 + np.array([40.0, -25.0])
    vis, wts = cast_inputs("f32_phase64", vis, wts)
    lo, hi = _w_range(uvw)
    wp, op = both_params(n, nw, 7, 0.2 / n, "f32_phase64", w_min=lo, w_max=hi, grid_correct=False,
                         normalize=False, tile=32)
    cuts = [0, 65_001, 140_000, 200_001]
    img, st = _accumulate(ctx, wp, _row_chunks(uvw, vis, wts, cuts), 1, n, on_device=on_device)
    ref = oracle_image(op, uvw, vis, wts)
    assert_stats(st, ref["stats"])
    e = rel(img[0], ref["raw"][0].real)
    log(f"accum f32 1024^2 x 16 on_device={on_device}: raw rel err {e:.3e}")
    assert e <= TOL32
    assert peak(img[0], ref["raw"][0].real) <= PEAK32


def _channel_data(rows=4000, nch=4, seed=23):
    rng = np.random.default_rng(seed)
    uvw = rng.uniform(-60, 60, (rows, 3))
    freq = np.linspace(120e6, 180e6, nch)
    vis = rng.standard_normal((rows, nch)) + 1j * rng.standard_normal((rows, nch))
    wts = rng.uniform(0.5, 2.0, (rows, nch))
    flags = (rng.random((rows, nch)) < 0.2).astype(np.uint8)
    return uvw, freq, vis, wts, flags


def test_frequency_chunks_into_one_image(ctx):
    """Multi-frequency synthesis from chunks of channels, uvw in metres."""
    n = 128
    uvw, freq, vis, wts, flags = _channel_data()
    lo, hi = _w_range(uvw, freq)
    wp, op = both_params(n, 4, 7, 0.2 / n, "f64", w_min=lo, w_max=hi)
    chunks = [(uvw, np.ascontiguousarray(vis[:, c]), np.ascontiguousarray(wts[:, c]),
               np.ascontiguousarray(flags[:, c]), freq[c]) for c in (slice(0, 1), slice(1, 4))]
    img, st = _accumulate(ctx, wp, chunks, 1, n)
    ref = oracle_image(op, uvw, vis, wts, flags, freq)
    assert_stats(st, ref["stats"])
    assert rel(img[0], ref["image"][0]) <= TOL64


def test_time_chunks_of_a_cube(ctx):
    n, nch = 128, 4
    uvw, freq, vis, wts, flags = _channel_data(nch=nch, seed=29)
    lo, hi = _w_range(uvw, freq)
    wp, op = both_params(n, 4, 7, 0.2 / n, "f64", w_min=lo, w_max=hi, per_channel=True)
    img, st = _accumulate(ctx, wp, _row_chunks(uvw, vis, wts, [0, 1500, 4000], flags, freq), nch, n,
                          n_img=nch)
    ref = oracle_image(op, uvw, vis, wts, flags, freq)
    assert_stats(st, ref["stats"])
    for i in range(nch):
        assert rel(img[i], ref["image"][i]) <= TOL64


def test_plane_range_and_kaiser_bessel(ctx, config0):
    """A shard of planes [2, 6) of 8, with the Kaiser-Bessel window."""
    ds = config0
    lo, hi = _w_range(ds.uvw)
    wp, op = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64", w_min=lo, w_max=hi,
                         plane_lo=2, plane_hi=6, kernel="kb")
    m = ds.uvw.shape[0]
    img, st = _accumulate(ctx, wp, _row_chunks(ds.uvw, ds.vis, ds.weights, [0, m // 3, m]), 1,
                          ds.grid_n)
    ref = oracle_image(op, ds.uvw, ds.vis, ds.weights)
    assert_stats(st, ref["stats"])
    assert rel(img[0], ref["image"][0]) <= TOL64


def test_no_chunks_gives_a_zero_image(ctx):
    wp, _ = both_params(64, 4, 7, 0.2 / 64, "f32_phase64", w_min=-10.0, w_max=10.0)
    img, st = _accumulate(ctx, wp, [], 1, 64)
    assert np.array_equal(img, np.zeros_like(img))
    assert st[0]["n_used"] == 0 and st[0]["n_records"] == 0 and st[0]["sum_w"] == 0.0


def test_rules(ctx):
    import torch
    wp, _ = both_params(64, 4, 7, 0.2 / 64, "f64")               # no w range
    with pytest.raises(wsg.WsgError) as e:
        wsg.Accum(ctx, wp, 1)
    assert e.value.status == wsg.EINVAL
    wp, _ = both_params(64, 4, 7, 0.2 / 64, "f64", w_min=-10.0, w_max=10.0, per_channel=True)
    uvw, vis, wts = synth.random_visibilities(100, 2, 64, 0.2 / 64, seed=1, w_extent=5.0)
    with wsg.Accum(ctx, wp, 3) as acc:
        with pytest.raises(wsg.WsgError) as e:
            acc.add(wsg.make_vis(dev(uvw), dev(vis), dev(wts)))   # 2 channels, cube of 3
        assert e.value.status == wsg.EINVAL
    wp, _ = both_params(64, 4, 7, 0.2 / 64, "f64", w_min=-10.0, w_max=10.0)
    out = torch.zeros((1, 64, 64), dtype=torch.float64, device=DEV)
    with wsg.Accum(ctx, wp, 2) as acc:
        acc.add(wsg.make_vis(dev(uvw), dev(vis), dev(wts)))
        acc.finish(out)
        with pytest.raises(wsg.WsgError):
            acc.finish(out)                                        # finished once
        with pytest.raises(wsg.WsgError):
            acc.add(wsg.make_vis(dev(uvw), dev(vis), dev(wts)))
    # the context still runs ordinary jobs afterwards
    st = ctx.image(wp, wsg.make_vis(dev(uvw), dev(vis), dev(wts)), out)
    assert st[0]["n_used"] > 0


def test_blocks_are_reused_across_jobs(ctx):
    """Consecutive chunked jobs on one context reuse (or replace) the previous job's
    w-stack block and chunk slots; every job starts from a clear stack."""
    for n, nw, rows, host in ((128, 4, 3000, True), (256, 8, 9000, True), (128, 4, 2000, True),
                              (128, 2, 2500, False)):
        uvw, vis, wts = synth.random_visibilities(rows, 1, n, 0.2 / n, seed=n + rows, w_extent=50.0)
        lo, hi = _w_range(uvw)
        wp, op = both_params(n, nw, 7, 0.2 / n, "f64", w_min=lo, w_max=hi)
        img, st = _accumulate(ctx, wp, _row_chunks(uvw, vis, wts, [0, rows // 2, rows]), 1, n,
                              on_device=not host)
        ref = oracle_image(op, uvw, vis, wts)
        assert_stats(st, ref["stats"])
        assert rel(img[0], ref["image"][0]) <= TOL64, (n, nw, rows)
