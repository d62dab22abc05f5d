"""Batched channels (config 3, all 512 time samples): 32 channels at 120-180 MHz
sharing one uvw set, uneven per-channel flagging, one image per channel, every
stage one launch over all channels.  Each channel of the batched call equals the
single-channel call on that channel, and the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2411_07321_amd import synth, wsg
from tests.gpuutil import DEV, dev, log, rel, PEAK32, peak

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    return synth.config3()


def test_cube_matches_single_channels_and_oracle(c3):
    import torch
    ds = c3
    n = ds.grid_n
    prm = wsg.params_for(ds, grid_correct=False, normalize=True)
    vb = wsg.make_vis(dev(ds.uvw), dev(ds.vis), dev(ds.weights), dev(ds.flags), ds.freq_hz,
                      ds.row_period)
    cube = torch.empty((ds.n_chan, n, n), dtype=torch.float64, device=DEV)
    with wsg.Context(0) as ctx:
        st = ctx.image(prm, vb, cube)
        torch.cuda.synchronize()
        cube = cube.cpu().numpy()
        used = [s["n_used"] for s in st]
        log(f"cube: used per channel {min(used)}..{max(used)} of {ds.n_rows}")
        assert max(used) > 2 * min(used)          # uneven flagging
        prm1 = wsg.params_for(ds, grid_correct=False, normalize=True, per_channel=False)
        for c in (0, 7, 19, 31):
            one = torch.empty((1, n, n), dtype=torch.float64, device=DEV)
            vb1 = wsg.make_vis(dev(ds.uvw), dev(np.ascontiguousarray(ds.vis[:, c:c + 1])),
                               dev(np.ascontiguousarray(ds.weights[:, c:c + 1])),
                               dev(np.ascontiguousarray(ds.flags[:, c:c + 1])),
                               ds.freq_hz[c:c + 1], ds.row_period)
            s1 = ctx.image(prm1, vb1, one)
            torch.cuda.synchronize()
            assert s1[0]["n_used"] == st[c]["n_used"]
            assert rel(cube[c], one.cpu().numpy()[0]) <= 1e-6
    op = oracle.Params(n, ds.n_wplanes, 7, ds.cell_rad, 0.9, grid_correct=False,
                       normalize=True, per_channel=True)
    for c in (0, 13, 31):
        inp = oracle.Inputs.make(ds.uvw, ds.freq_hz[c:c + 1],
                                 ds.vis[:, c:c + 1].astype(np.complex128),
                                 ds.weights[:, c:c + 1], ds.flags[:, c:c + 1])
        ref = oracle.image(inp, op)
        assert ref["stats"][0]["n_used"] == st[c]["n_used"]
        e = rel(cube[c], ref["image"][0])
        log(f"channel {c}: rel err vs oracle {e:.2e}")
        assert e <= 1e-5
        assert peak(cube[c], ref["image"][0]) <= PEAK32


def test_passes_over_the_planes_equal_one_pass(c3):
    """planes_per_pass: the cube imaged 4 and 5 planes at a time (passes of 4, 4, 4, 4 and
    5, 5, 5, 1 planes) equals the one-pass cube."""
    import torch
    ds = c3
    n = ds.grid_n
    vb = wsg.make_vis(dev(ds.uvw), dev(ds.vis), dev(ds.weights), dev(ds.flags), ds.freq_hz,
                      ds.row_period)
    with wsg.Context(0) as ctx:
        ref = torch.empty((ds.n_chan, n, n), dtype=torch.float64, device=DEV)
        st = ctx.image(wsg.params_for(ds, grid_correct=False, normalize=False), vb, ref)
        for ppp in (4, 5):
            out = torch.empty_like(ref)
            st2 = ctx.image(wsg.params_for(ds, grid_correct=False, normalize=False,
                                           planes_per_pass=ppp), vb, out)
            torch.cuda.synchronize()
            a, b = out.cpu().numpy(), ref.cpu().numpy()
            worst = max(rel(a[c], b[c]) for c in range(ds.n_chan))
            log(f"{ppp} planes per pass: worst channel rel {worst:.2e}")
            assert worst <= 1e-6
            assert [x["n_used"] for x in st2] == [x["n_used"] for x in st]
            assert [x["n_tiles"] for x in st2] == [x["n_tiles"] for x in st]


def test_autotune_picks_tile_and_passes_and_reads_its_cache(c3, tmp_path):
    ds = c3
    prm = wsg.params_for(ds)
    vb = wsg.make_vis(dev(ds.uvw), dev(ds.vis), dev(ds.weights), dev(ds.flags), ds.freq_hz,
                      ds.row_period)
    cache = str(tmp_path / "tune.txt")
    with wsg.Context(0) as ctx:
        tile, ppp = ctx.autotune(prm, vb, cache)
        assert tile in (16, 32, 64)
        assert ppp in (0, 8, 4)
        log(f"autotuned tile {tile}, planes per pass {ppp or 'all'}")
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split()[5:7] == [str(tile), str(ppp)]
    # a new context takes the stored choice without timing (no new line)
    with open(cache, "a") as f:
        f.write(lines[0].replace(f" {tile} {ppp} ", " 32 4 ", 1) + "\n")
    with wsg.Context(0) as ctx:
        assert ctx.autotune(prm, vb, cache) == (32, 4)
    assert len(open(cache).read().splitlines()) == 2
