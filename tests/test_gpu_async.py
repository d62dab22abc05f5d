"""Jobs submitted to a context (wsg_submit / wsg_poll / wsg_wait / wsg_cancel): each
result equals the synchronous wsg_image result on the same inputs (FP64: rel-L2 <=
1e-12 and equal counts), jobs finish in submission order, a job still queued can be
canceled (reported WSG_ECANCELED), one on the device cannot (WSG_EBUSY), and the
synchronous calls refuse to overlap submitted work (WSG_EBUSY)."""
import numpy as np
import pytest

from paper_2411_07321_amd import wsg
from tests.gpuutil import DEV, both_params, dev, log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = wsg.Context(0)
    yield c
    c.close()


def _jobs(ds, n):
    """n jobs: every k-th time slice of config 0 for k = 1 .. n (different sizes)."""
    nt = ds.uvw.shape[0] // ds.row_period
    out = []
    for k in range(1, n + 1):
        rows = np.concatenate([np.arange(t * ds.row_period, (t + 1) * ds.row_period)
                               for t in range(0, nt, k)])
        out.append(rows)
    return out


def test_submitted_jobs_equal_synchronous(ctx, config0):
    import torch
    ds = config0
    wp, _ = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64")
    jobs = _jobs(ds, 5)
    vbs = [wsg.make_vis(dev(ds.uvw[r]), dev(ds.vis[r]), dev(ds.weights[r]),
                        row_period=ds.row_period) for r in jobs]
    n = ds.grid_n
    ref, ref_st = [], []
    for vb in vbs:
        o = torch.empty((1, n, n), dtype=torch.float64, device=DEV)
        ref_st.append(ctx.image(wp, vb, o))
        ref.append(o)
    torch.cuda.synchronize()
    outs = [torch.full((1, n, n), np.nan, dtype=torch.float64, device=DEV) for _ in vbs]
    tickets = [ctx.submit(wp, vb, o) for vb, o in zip(vbs, outs)]
    assert tickets == sorted(tickets)
    # poll the last one until done: the stream runs the jobs in order, so the others
    # are then finished too
    while True:
        done, rc, st = ctx.poll(tickets[-1])
        if done:
            break
    assert rc == wsg.OK
    results = [ctx.wait(t) for t in tickets[:-1]] + [(rc, st)]
    for i, ((rc_i, st_i), o) in enumerate(zip(results, outs)):
        assert rc_i == wsg.OK
        e = rel(o.cpu().numpy()[0], ref[i].cpu().numpy()[0])
        log(f"job {i}: {len(jobs[i])} rows, rel {e:.2e}")
        assert e <= 1e-12
        for k in ("n_used", "n_flagged", "n_dropped", "n_records", "n_tiles"):
            assert st_i[0][k] == ref_st[i][0][k], (i, k)
    with pytest.raises(KeyError):
        ctx.wait(tickets[0])   # reported once, then forgotten


def test_cancel_queued_and_busy(ctx, config0):
    import torch
    ds = config0
    wp, _ = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64")
    vb = wsg.make_vis(dev(ds.uvw), dev(ds.vis), dev(ds.weights), row_period=ds.row_period)
    n = ds.grid_n
    outs = [torch.empty((1, n, n), dtype=torch.float64, device=DEV) for _ in range(4)]
    t = [ctx.submit(wp, vb, o) for o in outs]
    # two jobs go to the device at submission, the other two wait on the host
    assert ctx.cancel(t[0]) == wsg.EBUSY
    assert ctx.cancel(t[3]) == wsg.OK
    with pytest.raises(wsg.WsgError) as e:
        ctx.image(wp, vb, outs[0])
    assert e.value.status == wsg.EBUSY
    rc3, st3 = ctx.wait(t[3])
    assert rc3 == wsg.ECANCELED and st3 is None
    for k in (0, 1, 2):
        rc, st = ctx.wait(t[k])
        assert rc == wsg.OK and st[0]["n_used"] > 0
    # all reported: synchronous calls work again
    ctx.image(wp, vb, outs[0])


def test_submitted_host_buffers_and_failure(ctx, config0):
    ds = config0
    wp, _ = both_params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, "f64")
    vb = wsg.make_vis(ds.uvw, ds.vis, ds.weights, row_period=ds.row_period)
    n = ds.grid_n
    ref = np.empty((1, n, n))
    ctx.image(wp, vb, ref)
    out = np.full((1, n, n), np.nan)
    t = ctx.submit(wp, vb, out)
    rc, st = ctx.wait(t)
    assert rc == wsg.OK
    assert rel(out[0], ref[0]) <= 1e-12
    # a job the device cannot hold fails alone; the next job runs
    ctx.set_budget(1 << 20)
    t_bad = ctx.submit(wp, vb, out)
    ctx.set_budget(0)
    t_ok = ctx.submit(wp, vb, out)
    assert ctx.wait(t_bad)[0] == wsg.ENOMEM
    rc, st = ctx.wait(t_ok)
    assert rc == wsg.OK and rel(out[0], ref[0]) <= 1e-12
