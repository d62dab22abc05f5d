"""Stream ordering through the C ABI: a call runs on the caller's stream (torch's
default stream is HIP's null stream), after the work already queued there, and
later work on that stream sees its output, with no host synchronisation between.
The inputs are written by torch behind a slow matrix product, so a call that ran
on another stream would read them still zero."""
import numpy as np
import pytest

from paper_2411_07321_amd import wsg
from tests.gpuutil import DEV, dev, log, rel

pytestmark = pytest.mark.gpu


def _queue_slow_work(torch):
    a = torch.randn(8192, 8192, device=DEV)
    for _ in range(6):
        a = (a @ a) * (1.0 / 8192)
    return a


@pytest.mark.parametrize("precision", ["f32_phase64", "f64"])
def test_call_is_ordered_on_the_callers_stream(config0, precision):
    import torch
    ds = config0
    vt = torch.complex128 if precision == "f64" else torch.complex64
    wt = torch.float64 if precision == "f64" else torch.float32
    prm = wsg.params_for(ds, precision=precision, grid_correct=False)
    uvw = dev(ds.uvw)
    vis = dev(ds.vis).to(vt)
    wts = dev(ds.weights).to(wt)
    n = ds.grid_n
    ref_out = torch.empty((1, n, n), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    with wsg.Context(0) as ctx:
        st_ref = ctx.image(prm, wsg.make_vis(uvw, vis, wts, None, ds.freq_hz, ds.row_period),
                           ref_out)
        torch.cuda.synchronize()
        ref = ref_out.cpu().numpy()
        assert st_ref[0]["n_used"] > 0
        for trial in range(3):
            vis2 = torch.zeros_like(vis)
            wts2 = torch.zeros_like(wts)
            out = torch.full((1, n, n), float("nan"), dtype=torch.float64, device=DEV)
            torch.cuda.synchronize()
            _queue_slow_work(torch)
            vis2.copy_(vis)
            wts2.copy_(wts)
            vb = wsg.make_vis(uvw, vis2, wts2, None, ds.freq_hz, ds.row_period)
            if trial == 0:
                st = ctx.image(prm, vb, out)
                assert st[0]["n_used"] == st_ref[0]["n_used"]
            else:
                ctx.image(prm, vb, out, stats=False)
            # read back on torch's stream only
            total = out.sum()
            got = out.cpu().numpy()
            e = rel(got, ref)
            log(f"{precision} trial {trial}: rel diff to the synchronised call {e:.2e}")
            assert np.isfinite(total.item())
            assert e <= 1e-6


def test_context_stream_is_usable(config0):
    import torch
    ds = config0
    prm = wsg.params_for(ds, grid_correct=False)
    vb = wsg.make_vis(dev(ds.uvw), dev(ds.vis), dev(ds.weights), None, ds.freq_hz,
                      ds.row_period)
    n = ds.grid_n
    a = torch.empty((1, n, n), dtype=torch.float64, device=DEV)
    b = torch.empty((1, n, n), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    with wsg.Context(0) as ctx:
        assert ctx.stream
        ctx.image(prm, vb, a)
        ctx.image(prm, vb, b, stream=ctx.stream)
        torch.cuda.synchronize()
    assert rel(b.cpu().numpy(), a.cpu().numpy()) <= 1e-12
