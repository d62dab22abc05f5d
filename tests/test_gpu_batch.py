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


def test_autotune_picks_a_tile(c3):
    ds = c3
    prm = wsg.params_for(ds)
    vb = wsg.make_vis(dev(ds.uvw), dev(ds.vis), dev(ds.weights), dev(ds.flags), ds.freq_hz,
                      ds.row_period)
    with wsg.Context(0) as ctx:
        best = ctx.autotune(prm, vb)
        assert best in (16, 32, 64)
        log(f"autotuned tile: {best}")
