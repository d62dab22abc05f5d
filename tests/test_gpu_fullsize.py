"""Parity at the benchmark's full size and launch configuration (config 1: 4096^2 x 64
planes, 267,386,880 complex64 visibilities, FP64 phase): sampled pixels of the raw
image against the oracle's direct per-pixel evaluation, and the counts."""
import numpy as np
import pytest

import oracle
from paper_2411_07321_amd import synth, wsg
from tests.gpuutil import DEV, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kernel,fold", [("gauss", False), ("kb", True)])
def test_config1_sampled_pixels(kernel, fold):
    """The Gaussian of the workload, and the paper's Kaiser-Bessel window with w-folding."""
    import torch
    d = synth.config1_device(DEV)
    prm = wsg.make_params(**{**d["params"], "grid_correct": False, "normalize": False,
                             "kernel": kernel, "w_fold": fold})
    vb = wsg.make_vis(d["uvw"], d["vis"], d["weights"], None, d["freq_hz"], d["row_period"])
    out = torch.empty((1, 4096, 4096), dtype=torch.float64, device=DEV)
    with wsg.Context(0) as ctx:
        st = ctx.image(prm, vb, out)
    torch.cuda.synchronize()
    img = out[0]
    log(f"config 1 ({kernel}, fold {fold}) imaged: {st[0]['n_used']} used, "
        f"{st[0]['n_dropped']} dropped")
    # the 8 brightest sources and 8 random pixels
    sky = d["sky"]
    cell = 0.2 / 4096
    top = np.argsort(sky.flux)[-8:]
    q = list(np.round(sky.m[top] / cell).astype(int) + 2048)
    p = list(np.round(sky.l[top] / cell).astype(int) + 2048)
    rng = np.random.default_rng(5)
    q += list(rng.integers(0, 4096, 8))
    p += list(rng.integers(0, 4096, 8))
    got = img[torch.tensor(q), torch.tensor(p)].cpu().numpy()
    inp = oracle.Inputs.make(d["uvw"].cpu().numpy(), d["freq_hz"],
                             d["vis"].cpu().numpy().astype(np.complex128),
                             d["weights"].cpu().numpy().astype(np.float64))
    op = oracle.Params(4096, 64, 7, cell, 0.9, grid_correct=False, normalize=False,
                       kernel=kernel, w_fold=fold)
    log("oracle: direct evaluation of 16 pixels")
    ref = oracle.pixels(inp, op, q, p).real
    err = np.abs(got - ref)
    log(f"max abs diff {err.max():.3e}, max |A| {np.abs(ref).max():.3e}")
    assert err.max() <= 1e-5 * np.abs(ref).max()
    assert st[0]["n_used"] + st[0]["n_dropped"] == d["vis"].numel()
