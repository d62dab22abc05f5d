"""Serving: each job's image is the same alone and in the mix; admission keeps the
device memory held by the slots within the budget; a failing job fails alone.
Images are compared raw (before the grid correction, which amplifies FP32 rounding
near the field edge by up to ~3000x), normalised by the sum of weights."""
import os

import numpy as np
import pytest

from paper_2411_07321_amd import serve, synth, wsg
from tests.gpuutil import log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    # small versions of the serving mix: mesh 512^2 and 1024^2, up to 3e5 visibilities
    rng = np.random.default_rng(77)
    jobs = []
    for i in range(6):
        spec = synth.job_spec(rng)
        spec["grid_n"] = (512, 1024)[i % 2]
        spec["n_wplanes"] = (8, 16, 32)[i % 3]
        n_bl = spec["n_ant"] * (spec["n_ant"] - 1) // 2
        spec["n_times"] = max(1, int(3e5 // n_bl) - i)
        jobs.append(serve.PinnedJob(synth.make_job(spec, 500 + i), grid_correct=False))
    return jobs


def _solo(job):
    out = np.empty((1, job.grid_n, job.grid_n))
    with wsg.Context(0) as ctx:
        ctx.image(job.params, job.vb, out)
    return out


def test_mix_equals_solo(pool):
    solo = [_solo(j) for j in pool]
    order = np.array([0, 1, 2, 3, 4, 5, 1, 0, 3, 2, 5, 4])
    log(f"burst of {len(order)} jobs on 3 slots")
    r = serve.replay(pool, order, np.zeros(len(order)), n_slots=3,
                     keep_images=set(range(len(order))))
    assert len(r["images"]) == len(order)
    for k, img in r["images"].items():
        e = rel(img, solo[order[k]])
        assert e <= 1e-6, (k, e)
    log(f"mix: {r['jobs_per_s']:.1f} jobs/s, p99 {r['p99_ms']:.1f} ms")


def test_budget_admission(pool):
    fps = [wsg.footprint(j.params, j.vb) for j in pool]
    budget = int(1.5 * max(fps))
    order = np.arange(len(pool)).repeat(2)
    r = serve.replay(pool, order, np.zeros(len(order)), n_slots=4, hbm_budget=budget)
    assert r["peak_device_bytes"] <= budget * 1.15, (r["peak_device_bytes"], budget)
    with wsg.Server(0, 2, hbm_budget=min(fps) // 2) as srv:
        out = np.empty((1, pool[0].grid_n, pool[0].grid_n))
        with pytest.raises(wsg.WsgError) as e:
            srv.submit(pool[0].params, pool[0].vb, out)
        assert e.value.status == wsg.ENOMEM


def test_failure_isolated(pool, monkeypatch):
    monkeypatch.setenv("WSG_SERVER_FAIL_GRID_N", "1024")
    solo512 = {i: _solo(j) for i, j in enumerate(pool) if j.grid_n == 512}
    with wsg.Server(0, 3) as srv:
        tickets = []
        for i, j in enumerate(pool):
            out = np.full((1, j.grid_n, j.grid_n), np.nan)
            tickets.append((i, srv.submit(j.params, j.vb, out), out))
        for i, t, out in tickets:
            info = srv.wait(t)
            if pool[i].grid_n == 1024:
                assert info["status"] == wsg.EDEVICE
            else:
                assert info["status"] == wsg.OK
                assert rel(out, solo512[i]) <= 1e-6


def test_mix_of_kernels_and_plane_mappings(pool):
    """Jobs in one mix may use different gridding kernels and plane mappings (the
    Kaiser-Bessel window, w-folding, a kernel in w): each image equals the job alone."""
    import copy
    variants = []
    for i, (kernel, fold, sw) in enumerate((("kb", False, 1), ("gauss", True, 1), ("kb", True, 3))):
        job = copy.copy(pool[i])
        job.params = wsg.params_for(pool[i].ds, grid_correct=False, kernel=kernel, w_fold=fold,
                                    w_support=sw)
        variants.append(job)
    solo = [_solo(j) for j in variants]
    order = np.array([0, 1, 2, 2, 1, 0])
    r = serve.replay(variants, order, np.zeros(len(order)), n_slots=3,
                     keep_images=set(range(len(order))))
    for k, img in r["images"].items():
        e = rel(img, solo[order[k]])
        assert e <= 1e-6, (k, e)
