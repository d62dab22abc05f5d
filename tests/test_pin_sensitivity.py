"""The pins are sharp: plausible mistakes planted in the oracle (on the CPU, by
substituting a wrong step) are caught by the same checks the pins use."""
import numpy as np

import oracle
from paper_2411_07321_amd import synth
from tests import pinlib


def _fft_wrong_sign(g):
    x = np.fft.ifftshift(g, axes=(-2, -1))
    return np.fft.fftshift(np.fft.fft2(x, axes=(-2, -1)), axes=(-2, -1))


def _fft_wrong_origin(g):
    return np.fft.ifft2(g, axes=(-2, -1), norm="forward")


def _fft_normalised(g):
    return oracle.fft_planes(g) / (g.shape[-1] ** 2)


def test_transform_mistakes_are_caught():
    g = synth.random_planes(1, 16, seed=3)
    ref = pinlib.direct_centred_idft(g[0])
    ok = np.linalg.norm(oracle.fft_planes(g)[0] - ref) / np.linalg.norm(ref)
    assert ok < 1e-13
    for bad in (_fft_wrong_sign, _fft_wrong_origin, _fft_normalised):
        err = np.linalg.norm(bad(g)[0] - ref) / np.linalg.norm(ref)
        assert err > 1e-3, bad.__name__


def test_naive_n_minus_1_is_caught():
    n, cell = 64, 1e-4                          # small eta: the naive form cancels
    c = (np.arange(n) - n / 2) * cell
    eta = (c[None, :] ** 2 + c[:, None] ** 2).ravel()[1:200]
    ref = pinlib.n_minus_1_ld(eta)
    naive = np.sqrt(1.0 - eta) - 1.0
    stable = oracle.n_minus_1(n, cell)[0].ravel()[1:200]
    ok = eta > 0
    assert np.all(np.abs(stable[ok] - ref[ok]) <= 6e-16 * np.abs(ref[ok]))
    assert np.any(np.abs(naive[ok] - ref[ok]) > 1e-12 * np.abs(ref[ok]))


def test_wrong_plane_w_is_caught(config0, monkeypatch):
    # planes at their lower edge instead of their centre: the quantised-DFT bound fails
    ds = config0
    sub = slice(0, None, 16)
    uvw, vis, wts = ds.uvw[sub], ds.vis[sub, 0], ds.weights[sub, 0]
    prm = oracle.Params(ds.grid_n, 2, ds.support, ds.cell_rad, 0.9)
    good = oracle.image(oracle.Inputs.make(uvw, None, vis, wts), prm)
    st = good["stats"][0]
    q = np.arange(70, 190, 24).repeat(5)
    p = np.tile(np.arange(70, 190, 24), 5)
    Dq = pinlib.quantised_dft(uvw, vis, wts, st["w_min"], st["w_max"], 2, ds.grid_n,
                              ds.cell_rad, q, p)
    eps = pinlib.kernel_eps(ds.support, 0.9, 0.25)
    bound = (2 * eps + eps * eps) * np.abs(vis).mean() * 1.1
    assert np.abs(good["image"][0][q, p] - Dq).max() <= bound

    def lower_edge(k, w_min, w_max, n_w, w_support=1):
        return w_min + np.asarray(k, dtype=np.float64) * (w_max - w_min) / n_w
    monkeypatch.setattr(oracle, "plane_w", lower_edge)
    bad = oracle.image(oracle.Inputs.make(uvw, None, vis, wts), prm)
    assert np.abs(bad["image"][0][q, p] - Dq).max() > bound


def test_kaiser_bessel_mistakes_are_caught():
    """Plausible slips in the Kaiser-Bessel window (argument scaled by S instead of S/2,
    no 1/I0(beta), the default beta without the oversampling factor) each fail the
    kernel-value pin against scipy's I0."""
    from scipy.special import i0
    S = 7
    beta = oracle.kb_default_beta(S)
    x = np.linspace(0.0, S / 2, 21)
    d = np.concatenate([-x[::-1], x])

    def ref(d, b=beta):
        t = 2.0 * d / S
        return i0(b * np.sqrt(np.clip(1.0 - t * t, 0.0, None))) / i0(b)

    good = oracle.kernel_value(oracle.Params(64, 1, S, 1.0, kernel="kb"), d)
    assert np.abs(good - ref(d)).max() <= 1e-14
    slips = {
        "d/S": i0(beta * np.sqrt(np.clip(1.0 - (d / S) ** 2, 0.0, None))) / i0(beta),
        "no 1/I0(beta)": ref(d) * i0(beta),
        "beta without 1.5": ref(d, np.pi * np.sqrt((S / 2) ** 2 - 0.8)),
    }
    for name, bad in slips.items():
        assert np.abs(bad - ref(d)).max() > 1e-6, name


def test_fold_without_conjugation_is_caught(config0):
    """Folding the coordinates but not conjugating the visibility breaks the Hermitian
    identity that the fold pin checks."""
    ds = config0
    sub = slice(0, None, 16)
    uvw, vis, wts = ds.uvw[sub], ds.vis[sub, 0], ds.weights[sub, 0]
    q, p = np.array([100, 140, 90]), np.array([120, 70, 160])
    De = pinlib.exact_dft(uvw, vis, wts, ds.grid_n, ds.cell_rad, q, p)
    neg = uvw[:, 2] < 0
    bad = pinlib.exact_dft(np.where(neg[:, None], -uvw, uvw), vis, wts, ds.grid_n, ds.cell_rad, q, p)
    assert np.abs(bad - De).max() > 1e-3 * np.abs(De).max()


def _planted_oracle(tmp_path, old: str, new: str):
    """A copy of the C oracle with one line changed, built with gcc on the CPU."""
    import subprocess
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "wsg_oracle_planted.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_planted.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared",
                    "-fPIC", "-o", str(lib), str(path), "-lm"], check=True)
    return str(lib)


def test_w_kernel_edge_clamp_slip_is_caught(tmp_path, monkeypatch):
    """The clamp that keeps a kernel-in-w visibility's planes inside the stack, planted one
    plane off (N_w - h_w instead of N_w - 1 - h_w): the edge-plane pin fails."""
    from tests.test_oracle_pins import w_kernel_edge_plane_error
    lib = _planted_oracle(tmp_path, "if (k0 > n_w - 1 - hw) k0 = n_w - 1 - hw;",
                          "if (k0 > n_w - hw) k0 = n_w - hw;")
    monkeypatch.setattr(oracle, "_LIB_PATH", lib)
    monkeypatch.setattr(oracle, "_lib", None)
    try:
        for sw in (3, 5):
            err, _ = w_kernel_edge_plane_error(sw)
            assert err > 1e-2
    finally:
        oracle._lib = None
