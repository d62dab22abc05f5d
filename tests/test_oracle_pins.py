"""Pins of the FP64 oracle against things other than itself: brute-force transforms,
closed forms, invariants and error bounds (De Rubeis et al., Sec. 2, Eqs. 1-3).

A plausible slip anywhere in the oracle -- a sign in the transform, the origin
at N/2, the plane index, the kernel argument, a dropped weight, the stable
n - 1 -- fails at least one of these."""
import math

import numpy as np
import pytest

import oracle
from paper_2411_07321_amd import synth
from tests import pinlib

SIG = 0.9


def _inputs(uvw, vis, wts=None, flags=None, freq=None):
    return oracle.Inputs.make(uvw, freq, vis, wts, flags)


def _raw(inp, prm):
    prm.grid_correct = False
    prm.normalize = False
    return oracle.image(inp, prm)["raw"][0]


# ---------------------------------------------------------------- P1, P2: transform
@pytest.mark.parametrize("n", [8, 16, 32])
def test_fft_matches_direct_dft(n):
    g = synth.random_planes(2, n, seed=n)
    F = oracle.fft_planes(g)
    for k in range(2):
        ref = pinlib.direct_centred_idft(g[k])
        assert np.linalg.norm(F[k] - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("n", [64, 256])
def test_fft_parseval(n):
    g = synth.random_planes(3, n, seed=11)
    F = oracle.fft_planes(g)
    for k in range(3):
        lhs = np.sum(np.abs(F[k]) ** 2)
        rhs = n * n * np.sum(np.abs(g[k]) ** 2)
        assert abs(lhs - rhs) / rhs < 1e-13


def test_fft_single_cell_is_fringe():
    # g = delta at (j, i) -> F[q,p] = exp(2 pi i ((i-N/2)(p-N/2) + (j-N/2)(q-N/2))/N)
    n, i, j = 32, 21, 6
    g = np.zeros((1, n, n), complex)
    g[0, j, i] = 1.0
    F = oracle.fft_planes(g)[0]
    c = np.arange(n) - n / 2
    ref = np.exp(2j * np.pi * ((i - n / 2) * c[None, :] + (j - n / 2) * c[:, None]) / n)
    assert np.abs(F - ref).max() < 1e-13


# ---------------------------------------------------------------- P3, single-visibility grid
def test_grid_single_visibility_footprint():
    n, cell, S = 64, 1.0 / 100, 7
    uvw = np.array([[12.34567, -8.7654, 5.0]])
    vis = np.array([[0.3 - 0.8j]])
    wts = np.array([[1.7]])
    prm = oracle.Params(n, 1, S, cell, SIG)
    g, cnt = oracle.grid(_inputs(uvw, vis, wts), prm, 5.0, 5.0)
    x, y = pinlib.positions(uvw, n, cell)
    i0, j0 = int(math.floor(x[0] + 0.5)), int(math.floor(y[0] + 0.5))
    ref = np.zeros((n, n), complex)
    for b in range(-3, 4):
        for a in range(-3, 4):
            ref[j0 + b, i0 + a] = 1.7 * vis[0, 0] * pinlib.gauss(i0 + a - x[0], SIG) * \
                pinlib.gauss(j0 + b - y[0], SIG)
    assert np.abs(g[0] - ref).max() < 1e-15
    assert cnt["n_used"] == 1 and cnt["sum_w"] == 1.7


def test_grid_sum_invariant(config0):
    ds = config0
    prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG)
    inp = _inputs(ds.uvw, ds.vis, ds.weights)
    wmin, wmax = oracle.w_range(inp, prm)
    g, _ = oracle.grid(inp, prm, wmin, wmax)
    x, y = pinlib.positions(ds.uvw, ds.grid_n, ds.cell_rad)
    k, _ = pinlib.planes(ds.uvw[:, 2], wmin, wmax, ds.n_wplanes)
    a = np.arange(-3, 4)
    i0 = np.floor(x + 0.5)
    j0 = np.floor(y + 0.5)
    sx = pinlib.gauss(i0[:, None] + a[None, :] - x[:, None], SIG).sum(1)
    sy = pinlib.gauss(j0[:, None] + a[None, :] - y[:, None], SIG).sum(1)
    contrib = ds.weights[:, 0] * ds.vis[:, 0] * sx * sy
    for kk in range(ds.n_wplanes):
        ref = contrib[k == kk].sum()
        got = g[kk].sum()
        assert abs(got - ref) <= 1e-13 * max(1.0, np.abs(contrib[k == kk]).sum())
    # planes are populated roughly evenly for an Earth-rotation track
    assert all(np.any(k == kk) for kk in range(ds.n_wplanes))


# ---------------------------------------------------------------- P4: pure fringe
def test_pure_fringe_closed_form():
    # N dl = 1/2 exactly, so x = u/2 + N/2 is exact for even u: the visibility sits on a cell
    n, cell, S = 64, 1.0 / 128, 7
    u, v, w = 2.0 * 9, 2.0 * -13, 37.5
    inp = _inputs(np.array([[u, v, w]]), np.array([[1.0 + 0j]]))
    A = _raw(inp, oracle.Params(n, 4, S, cell, SIG))
    c = (np.arange(n) - n / 2)
    l = c * cell
    nu = c / n
    a = np.arange(-3, 4)
    cd = (pinlib.gauss(a, SIG)[None, :] * np.cos(2 * np.pi * a[None, :] * nu[:, None])).sum(1)
    nm1 = np.sqrt(1 - l[None, :] ** 2 - l[:, None] ** 2) - 1
    ref = np.exp(2j * np.pi * (u * l[None, :] + v * l[:, None] + w * nm1)) * cd[None, :] * cd[:, None]
    assert np.abs(A - ref).max() < 1e-12


# ---------------------------------------------------------------- P5: flat image
def test_flat_image_from_zero_spacing():
    n, cell, S = 64, 1.0 / 200, 7
    inp = _inputs(np.array([[0.0, 0.0, 0.0]]), np.array([[1.0 + 0j]]))
    prm = oracle.Params(n, 1, S, cell, SIG)
    A = _raw(inp, oracle.Params(n, 1, S, cell, SIG))
    nu = (np.arange(n) - n / 2) / n
    a = np.arange(-3, 4)
    cd = (pinlib.gauss(a, SIG)[None, :] * np.cos(2 * np.pi * a[None, :] * nu[:, None])).sum(1)
    assert np.abs(A - cd[None, :] * cd[:, None]).max() < 1e-13
    D = oracle.image(inp, prm)["image"][0]
    # corrected by the continuous transform C: 1 within (1+e)^2 - 1 in the inner half
    eps = np.abs(cd / pinlib.c_closed_form(nu, S, SIG) - 1.0)
    inner = np.abs(nu) <= 0.25
    bound = (1 + eps[inner][None, :]) * (1 + eps[inner][:, None]) - 1
    assert np.all(np.abs(D[np.ix_(inner, inner)] - 1.0) <= bound * 1.0001 + 1e-14)


# ---------------------------------------------------------------- P6: unit point source
def test_unit_source_at_phase_centre(config0):
    ds = config0
    vis = np.ones_like(ds.vis)                    # what Eq. 1 gives for S = 1 at l = m = 0
    prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG)
    D = oracle.image(_inputs(ds.uvw, vis, ds.weights), prm)["image"][0]
    eps = pinlib.kernel_eps(ds.support, SIG, 0.0, n_nu=1)
    assert abs(D[128, 128] - 1.0) <= (2 * eps + eps * eps) * 1.1
    assert eps < 1e-3


# ---------------------------------------------------------------- P7: permutation, linearity
def test_permutation_and_linearity(config0):
    ds = config0
    prm = lambda: oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG)
    rng = np.random.default_rng(5)
    perm = rng.permutation(ds.n_rows)
    A = _raw(_inputs(ds.uvw, ds.vis, ds.weights), prm())
    Ap = _raw(_inputs(ds.uvw[perm], ds.vis[perm], ds.weights[perm]), prm())
    assert np.linalg.norm(A - Ap) / np.linalg.norm(A) < 1e-13
    v2 = (rng.standard_normal(ds.vis.shape) + 1j * rng.standard_normal(ds.vis.shape))
    A2 = _raw(_inputs(ds.uvw, v2, ds.weights), prm())
    Al = _raw(_inputs(ds.uvw, 0.7 * ds.vis - 1.3j * v2, ds.weights), prm())
    ref = 0.7 * A - 1.3j * A2
    assert np.linalg.norm(Al - ref) / np.linalg.norm(ref) < 1e-13


# ---------------------------------------------------------------- P8, P9: error bounds vs DFT
def _inner_pixels(n, step):
    c = np.arange(n // 4, 3 * n // 4 + 1, step)
    q, p = np.meshgrid(c, c, indexing="ij")
    return q.ravel(), p.ravel()


def test_against_quantised_and_exact_dft(config0):
    ds = config0
    sub = slice(0, None, 8)                      # 3,968 measurements
    uvw, vis, wts = ds.uvw[sub], ds.vis[sub, 0], ds.weights[sub, 0]
    prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG)
    out = oracle.image(_inputs(uvw, vis, wts), prm)
    D = out["image"][0]
    st = out["stats"][0]
    q, p = _inner_pixels(ds.grid_n, 8)
    Dq = pinlib.quantised_dft(uvw, vis, wts, st["w_min"], st["w_max"], ds.n_wplanes,
                              ds.grid_n, ds.cell_rad, q, p)
    eps = pinlib.kernel_eps(ds.support, SIG, 0.25)
    amp = (wts * np.abs(vis)).sum() / wts.sum()
    err_q = np.abs(D[q, p] - Dq)
    assert err_q.max() <= (2 * eps + eps * eps) * amp * 1.1
    assert err_q.max() > 0.0
    # w quantisation: |D_q - D| <= 2 pi (dw/2) |n - 1| * sum W|V| / sum W
    De = pinlib.exact_dft(uvw, vis, wts, ds.grid_n, ds.cell_rad, q, p)
    dw = (st["w_max"] - st["w_min"]) / ds.n_wplanes
    l = (p - ds.grid_n / 2) * ds.cell_rad
    m = (q - ds.grid_n / 2) * ds.cell_rad
    nm1 = np.abs(np.sqrt(1 - l * l - m * m) - 1)
    assert np.all(np.abs(Dq - De) <= 2 * np.pi * dw / 2 * nm1 * amp * 1.0001 + 1e-14)


def test_sources_recovered(config0):
    ds = config0
    prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG)
    D = oracle.image(_inputs(ds.uvw, ds.vis, ds.weights), prm)["image"][0]
    for l, m, f in zip(ds.sky.l, ds.sky.m, ds.sky.flux):
        p = int(round(l / ds.cell_rad)) + 128
        q = int(round(m / ds.cell_rad)) + 128
        assert abs(D[q, p] - f) < 0.1 * max(f, 0.3)


# ---------------------------------------------------------------- P10: stable n - 1
def test_stable_n_minus_1():
    n, cell = 512, 0.9 / 256 * math.sqrt(0.5)        # eta up to 0.81 at the corners
    nm1, inside = oracle.n_minus_1(n, cell)
    rng = np.random.default_rng(2)
    idx = rng.integers(0, n, (400, 2))
    c = (np.arange(n) - n / 2) * cell
    eta = c[idx[:, 1]] ** 2 + c[idx[:, 0]] ** 2
    ref = pinlib.n_minus_1_ld(eta)
    got = nm1[idx[:, 0], idx[:, 1]]
    ok = eta > 0
    assert np.all(np.abs(got[ok] - ref[ok]) <= 6e-16 * np.abs(ref[ok]))
    assert got[~ok].size == 0 or np.all(got[~ok] == 0)
    assert inside.all()


def test_off_sphere_pixels_are_zero():
    # dl large enough that the corners have l^2 + m^2 >= 1
    n, cell = 16, 0.1
    F = np.ones((1, n, n), complex)
    A = oracle.wcorrect(F, 0.0, 10.0, 1, cell)
    c = (np.arange(n) - n / 2) * cell
    off = (c[None, :] ** 2 + c[:, None] ** 2) >= 1.0
    assert off.any() and np.all(A[off] == 0) and np.all(A[~off] != 0)


# ---------------------------------------------------------------- P11: grid correction
@pytest.mark.parametrize("S,sig", [(7, 0.9), (7, 1.0), (5, 0.7), (15, 2.0)])
def test_kernel_transform_quadrature(S, sig):
    n = 128
    c = oracle.kernel_transform(n, S, sig)
    nu = (np.arange(n) - n / 2) / n
    ref = pinlib.c_closed_form(nu, S, sig)
    assert np.abs(c - ref).max() <= 2e-15 * np.abs(ref).max()
    # converged: another rule agrees to the accuracy of numpy's nodes (~1e-14)
    c2 = oracle.kernel_transform(n, S, sig, nodes=48)
    assert np.abs(c - c2).max() <= 2e-14 * np.abs(ref).max()


def test_kernel_width_reading():
    # sigma = 0.9 cells keeps the worst per-visibility error below 1e-3 over |nu| <= 1/4
    assert pinlib.kernel_eps(7, 0.9, 0.25) < 1e-3
    assert pinlib.kernel_eps(7, 1.0, 0.25) > pinlib.kernel_eps(7, 0.9, 0.25)


# ---------------------------------------------------------------- O2/O3: counts, planes
def test_validity_counts():
    n, cell = 64, 1.0 / 100
    du = 1.0 / (n * cell)
    uvw = np.array([[10.0, 5.0, 1.0],          # used
                    [10.0, 5.0, 2.0],          # flagged
                    [np.nan, 5.0, 1.0],        # non-finite u
                    [10.0, 5.0, 1.0],          # weight 0
                    [(n / 2 - 3) * du, 0.0, 1.0],   # i0 = N-3 > N-1-h: off the grid
                    [(n / 2 - 4) * du, 0.0, 3.0],   # i0 = N-4 = N-1-h: last that fits
                    [-(n / 2 - 3) * du, 0.0, 1.5],  # i0 = 3 = h: first that fits
                    [10.0, 5.0, 1.0]])         # vis inf
    vis = np.array([1, 1, 1, 1, 1, 1, 1, np.inf + 0j], complex)[:, None]
    wts = np.array([1, 1, 1, 0, 1, 1, 1, 1], float)[:, None]
    fl = np.array([0, 1, 0, 0, 0, 0, 0, 0], np.uint8)[:, None]
    inp = _inputs(uvw, vis, wts, fl)
    prm = oracle.Params(n, 2, 7, cell, SIG)
    wmin, wmax = oracle.w_range(inp, prm)
    assert (wmin, wmax) == (1.0, 3.0)
    _, cnt = oracle.grid(inp, prm, wmin, wmax)
    assert cnt == {"n_used": 3, "n_flagged": 1, "n_dropped": 4, "sum_w": 3.0}
    # a caller-given range that excludes w = 3 drops it too
    _, cnt2 = oracle.grid(inp, prm, 0.0, 2.0)
    assert cnt2["n_used"] == 2 and cnt2["n_dropped"] == 5


def test_plane_rule_and_degenerate_range():
    k, wk = pinlib.planes(np.array([0.0, 0.999, 1.0, 3.99, 4.0]), 0.0, 4.0, 4)
    assert list(k) == [0, 0, 1, 3, 3] and list(wk) == [0.5, 0.5, 1.5, 3.5, 3.5]
    assert list(oracle.plane_w(np.arange(4), 0.0, 4.0, 4)) == [0.5, 1.5, 2.5, 3.5]
    assert list(oracle.plane_w(np.arange(2), 2.0, 2.0, 2)) == [2.0, 2.0]


def test_empty_input_gives_zero_image():
    inp = _inputs(np.zeros((0, 3)), np.zeros((0, 1), complex))
    out = oracle.image(inp, oracle.Params(32, 2, 7, 0.01, SIG))
    assert np.all(out["image"] == 0) and out["stats"][0]["n_used"] == 0


# ---------------------------------------------------------------- sharding and sampling
def test_plane_shards_sum_to_whole(config0):
    ds = config0
    inp = _inputs(ds.uvw, ds.vis, ds.weights)
    full = _raw(inp, oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG))
    wmin, wmax = oracle.w_range(inp, oracle.Params(ds.grid_n, 8, 7, ds.cell_rad))
    parts = 0
    for lo, hi in [(0, 3), (3, 8)]:
        prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG,
                            w_min=wmin, w_max=wmax, plane_lo=lo, plane_hi=hi)
        parts = parts + _raw(inp, prm)
    assert np.linalg.norm(parts - full) / np.linalg.norm(full) < 1e-13


def test_pixel_evaluator_matches_mesh_path(config0):
    ds = config0
    inp = _inputs(ds.uvw, ds.vis, ds.weights)
    prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG)
    A = _raw(inp, prm)
    rng = np.random.default_rng(9)
    q = rng.integers(0, ds.grid_n, 12)
    p = rng.integers(0, ds.grid_n, 12)
    got = oracle.pixels(inp, prm, q, p)
    assert np.abs(got - A[q, p]).max() < 1e-12 * np.abs(A).max()


def test_channels_cube_and_metres():
    # uvw in metres with per-channel frequencies equals uvw pre-scaled per channel
    rng = np.random.default_rng(4)
    uvw_m = rng.uniform(-300, 300, (300, 3))
    freq = np.array([120e6, 150e6, 180e6])
    vis = rng.standard_normal((300, 3)) + 1j * rng.standard_normal((300, 3))
    prm = oracle.Params(64, 4, 7, 0.2 / 64, SIG, per_channel=True)
    cube = oracle.image(oracle.Inputs.make(uvw_m, freq, vis), prm)["image"]
    for c in range(3):
        one = oracle.image(oracle.Inputs.make(uvw_m * (freq[c] / oracle.C_LIGHT), None,
                                              vis[:, c:c + 1]),
                           oracle.Params(64, 4, 7, 0.2 / 64, SIG))["image"][0]
        assert np.linalg.norm(cube[c] - one) <= 1e-13 * np.linalg.norm(one)


# ---------------------------------------------------------------- Kaiser-Bessel kernel
# The paper's runs grid with a Kaiser-Bessel window (Sec. 2, after Eq. 3; Jackson
# et al. 1991): G(d) = I0(beta sqrt(1 - (2d/S)^2)) / I0(beta) on |d| <= S/2.
def _kb_ref(d, S, beta):
    from scipy.special import i0
    t = 2.0 * np.asarray(d, dtype=np.float64) / S
    u = np.clip(1.0 - t * t, 0.0, None)
    return np.where(1.0 - t * t >= 0.0, i0(beta * np.sqrt(u)) / i0(beta), 0.0)


def test_bessel_i0_against_scipy():
    from scipy.special import i0
    lib = oracle._load()
    for x in (0.0, 1e-3, 0.5, 1.0, 3.75, 7.0, 10.0, 16.252239469813198, 25.0, 40.0):
        assert abs(lib.oracle_bessel_i0(x) - i0(x)) <= 2e-15 * i0(x), x


@pytest.mark.parametrize("S", [5, 7, 9])
def test_kb_kernel_values(S):
    beta = oracle.kb_default_beta(S)
    prm = oracle.Params(64, 1, S, 1.0, kernel="kb")
    x = np.linspace(0.0, S / 2, 21)
    d = np.concatenate([-x[::-1], x])                       # exact mirror images
    g = oracle.kernel_value(prm, d)
    assert np.abs(g - _kb_ref(d, S, beta)).max() <= 1e-14
    assert oracle.kernel_value(prm, np.array([0.0]))[0] == 1.0
    assert np.array_equal(g, g[::-1])                       # even
    assert oracle.kernel_value(prm, np.array([S / 2 + 1e-9]))[0] == 0.0


def test_kb_default_beta_reading():
    # Beatty et al. (2005) for twofold oversampling: beta = pi sqrt((S/2)^2 1.5^2 - 0.8)
    assert abs(oracle.kb_default_beta(7) - 16.252239469813198) < 1e-12
    assert abs(oracle.kb_default_beta(5) - math.pi * math.sqrt(6.25 * 2.25 - 0.8)) < 1e-12


@pytest.mark.parametrize("S,beta", [(7, 0.0), (5, 0.0), (9, 0.0), (7, 9.0)])
def test_kb_kernel_transform_closed_form(S, beta):
    # the window's continuous transform: S sinh(sqrt(beta^2 - (pi S nu)^2)) / sqrt(...) / I0(beta)
    from scipy.special import i0
    n = 128
    b = beta if beta > 0 else oracle.kb_default_beta(S)
    c = oracle.kernel_transform(n, S, SIG, kernel="kb", beta=beta)
    nu = (np.arange(n) - n / 2) / n
    z2 = b * b - (np.pi * S * nu) ** 2
    ref = np.where(z2 > 0, S * np.sinh(np.sqrt(np.abs(z2))) / np.sqrt(np.abs(z2)),
                   S * np.sin(np.sqrt(np.abs(z2))) / np.sqrt(np.abs(z2))) / i0(b)
    assert np.abs(c - ref).max() <= 1e-13 * np.abs(ref).max()


def test_kb_single_visibility_footprint():
    n, cell, S = 64, 1.0 / 100, 7
    uvw = np.array([[12.34567, -8.7654, 5.0]])
    vis = np.array([[0.3 - 0.8j]])
    wts = np.array([[1.7]])
    prm = oracle.Params(n, 1, S, cell, kernel="kb")
    g, cnt = oracle.grid(_inputs(uvw, vis, wts), prm, 5.0, 5.0)
    x, y = pinlib.positions(uvw, n, cell)
    i0_, j0 = int(math.floor(x[0] + 0.5)), int(math.floor(y[0] + 0.5))
    beta = oracle.kb_default_beta(S)
    ref = np.zeros((n, n), complex)
    for b in range(-3, 4):
        for a in range(-3, 4):
            ref[j0 + b, i0_ + a] = 1.7 * vis[0, 0] * _kb_ref(i0_ + a - x[0], S, beta) * \
                _kb_ref(j0 + b - y[0], S, beta)
    assert np.abs(g[0] - ref).max() < 1e-15
    assert cnt["n_used"] == 1


def test_kb_pure_fringe_closed_form():
    # a visibility on a cell: its image is the fringe times the discrete kernel transform
    n, cell, S = 64, 1.0 / 128, 7
    u, v, w = 2.0 * 9, 2.0 * -13, 37.5
    inp = _inputs(np.array([[u, v, w]]), np.array([[1.0 + 0j]]))
    A = _raw(inp, oracle.Params(n, 4, S, cell, kernel="kb"))
    c = (np.arange(n) - n / 2)
    l = c * cell
    nu = c / n
    a = np.arange(-3, 4)
    kb = _kb_ref(a, S, oracle.kb_default_beta(S))
    cd = (kb[None, :] * np.cos(2 * np.pi * a[None, :] * nu[:, None])).sum(1)
    nm1 = np.sqrt(1 - l[None, :] ** 2 - l[:, None] ** 2) - 1
    ref = np.exp(2j * np.pi * (u * l[None, :] + v * l[:, None] + w * nm1)) * cd[None, :] * cd[:, None]
    assert np.abs(A - ref).max() < 1e-12


# ---------------------------------------------------------------- w-folding
# A real sky has a Hermitian visibility function, V(-u,-v,-w) = conj V(u,v,w) (Eq. 1),
# so rows with w < 0 may be gridded at (-u,-v,-w) with conj(V): Re of Eq. 2 is unchanged
# and the planes cover only w >= 0.
def test_fold_preserves_the_exact_dft(config0):
    ds = config0
    sub = slice(0, None, 8)
    uvw, vis, wts = ds.uvw[sub], ds.vis[sub, 0], ds.weights[sub, 0]
    f = oracle.fold_w(_inputs(uvw, vis, wts))
    assert (f.uvw[:, 2] >= 0).all()
    neg = uvw[:, 2] < 0
    assert np.array_equal(f.uvw[~neg], uvw[~neg]) and np.array_equal(f.uvw[neg], -uvw[neg])
    q, p = _inner_pixels(ds.grid_n, 6)
    De = pinlib.exact_dft(uvw, vis, wts, ds.grid_n, ds.cell_rad, q, p)
    Df = pinlib.exact_dft(f.uvw, f.vis[:, 0], wts, ds.grid_n, ds.cell_rad, q, p)
    assert np.abs(Df - De).max() <= 1e-12 * np.abs(De).max()


def test_folded_image_against_exact_dft(config0):
    """The folded image obeys the same two bounds as the plain one (kernel error against
    the w-quantised transform, quantisation error against the exact transform of the
    ORIGINAL data), with the folded plane width, about half the plain one here."""
    ds = config0
    sub = slice(0, None, 8)
    uvw, vis, wts = ds.uvw[sub], ds.vis[sub, 0], ds.weights[sub, 0]
    prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, SIG, w_fold=True)
    out = oracle.image(_inputs(uvw, vis, wts), prm)
    D = out["image"][0]
    st = out["stats"][0]
    assert st["w_min"] >= 0.0
    plain = oracle.w_range(_inputs(uvw, vis, wts), oracle.Params(ds.grid_n, 1, ds.support,
                                                                 ds.cell_rad, SIG))
    dw = (st["w_max"] - st["w_min"]) / ds.n_wplanes
    assert dw <= 0.55 * (plain[1] - plain[0]) / ds.n_wplanes
    q, p = _inner_pixels(ds.grid_n, 8)
    neg = uvw[:, 2] < 0
    uf = np.where(neg[:, None], -uvw, uvw)
    vf = np.where(neg, np.conj(vis), vis)
    Dq = pinlib.quantised_dft(uf, vf, wts, st["w_min"], st["w_max"], ds.n_wplanes, ds.grid_n,
                              ds.cell_rad, q, p)
    eps = pinlib.kernel_eps(ds.support, SIG, 0.25)
    amp = (wts * np.abs(vis)).sum() / wts.sum()
    assert np.abs(D[q, p] - Dq).max() <= (2 * eps + eps * eps) * amp * 1.1
    De = pinlib.exact_dft(uvw, vis, wts, ds.grid_n, ds.cell_rad, q, p)
    l = (p - ds.grid_n / 2) * ds.cell_rad
    m = (q - ds.grid_n / 2) * ds.cell_rad
    nm1 = np.abs(np.sqrt(1 - l * l - m * m) - 1)
    assert np.all(np.abs(Dq - De) <= 2 * np.pi * dw / 2 * nm1 * amp * 1.0001 + 1e-14)


def test_fold_without_negative_w_changes_nothing():
    rng = np.random.default_rng(5)
    n = 64
    uvw = np.stack([rng.uniform(-200, 200, 500), rng.uniform(-200, 200, 500),
                    rng.uniform(0.0, 30.0, 500)], axis=1)
    vis = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    a = oracle.image(_inputs(uvw, vis), oracle.Params(n, 4, 7, 1.0 / (n * 10), SIG))
    b = oracle.image(_inputs(uvw, vis), oracle.Params(n, 4, 7, 1.0 / (n * 10), SIG, w_fold=True))
    assert np.array_equal(a["image"], b["image"])


# ---------------------------------------------------------------- kernel in w
# Eq. 3's G acts in u, v and w: with w_support = 2 h_w + 1 a visibility adds
# W V G(u) G(v) G_w((w_k - w)/dw) to the planes k0 - h_w .. k0 + h_w around its own,
# the data range covering the middle N_w - 2 h_w planes; after the plane sum with
# the phases of Eq. 2 the image carries C_w(dw (n - 1)), the window's transform,
# which the grid correction divides out.
def test_w_kernel_single_visibility_planes():
    n, cell, S, SW, nw = 64, 1.0 / 100, 7, 5, 9
    uvw = np.array([[12.34567, -8.7654, 3.21]])
    vis = np.array([[0.3 - 0.8j]])
    wts = np.array([[1.7]])
    w_lo, w_hi = -10.0, 10.0
    prm = oracle.Params(n, nw, S, cell, SIG, w_support=SW)
    g, cnt = oracle.grid(_inputs(uvw, vis, wts), prm, w_lo, w_hi)
    dw = (w_hi - w_lo) / (nw - 4)
    w0 = w_lo - 2 * dw
    assert cnt["n_used"] == 1
    k0 = int(np.floor((3.21 - w0) / dw))
    x, y = pinlib.positions(uvw, n, cell)
    i0_, j0 = int(math.floor(x[0] + 0.5)), int(math.floor(y[0] + 0.5))
    gx = pinlib.gauss(i0_ + np.arange(-3, 4) - x[0], SIG)
    gy = pinlib.gauss(j0 + np.arange(-3, 4) - y[0], SIG)
    ref = np.zeros((nw, n, n), complex)
    for k in range(k0 - 2, k0 + 3):
        gw = pinlib.gauss((w0 + (k + 0.5) * dw - 3.21) / dw, SIG)
        ref[k, j0 - 3:j0 + 4, i0_ - 3:i0_ + 4] = 1.7 * vis[0, 0] * gw * np.outer(gy, gx)
    assert np.abs(g - ref).max() < 1e-15
    assert np.count_nonzero(np.abs(g).reshape(nw, -1).max(1)) == 5


def test_w_kernel_transform_closed_form():
    prm = oracle.Params(64, 8, 7, 1.0, SIG, w_support=7)
    nu = np.array([0.0, 0.01, 0.05, 0.13, 0.25, 0.4])
    ref = pinlib.c_closed_form(nu, 7, SIG)
    assert np.abs(oracle.w_kernel_transform(nu, prm) - ref).max() <= 1e-13 * ref.max()


def test_w_kernel_pure_fringe():
    """One visibility on a cell: Re A = Re[fringe_uv * Cd(p) Cd(q) *
    sum_k G_w((w_k - w)/dw) e^{2 pi i w_k (n - 1)}]."""
    n, cell, S, SW, nw = 64, 1.0 / 128, 7, 5, 10
    u, v, w = 2.0 * 9, 2.0 * -13, 37.5
    prm = oracle.Params(n, nw, S, cell, SIG, w_min=-40.0, w_max=40.0, w_support=SW)
    A = _raw(_inputs(np.array([[u, v, w]]), np.array([[1.0 + 0j]])), prm)
    c = np.arange(n) - n / 2
    l = c * cell
    nu = c / n
    a = np.arange(-3, 4)
    cd = (pinlib.gauss(a, SIG)[None, :] * np.cos(2 * np.pi * a[None, :] * nu[:, None])).sum(1)
    nm1 = np.sqrt(1 - l[None, :] ** 2 - l[:, None] ** 2) - 1
    dw = 80.0 / (nw - 4)
    w0 = -40.0 - 2 * dw
    k0 = int(np.floor((w - w0) / dw))
    ws = sum(pinlib.gauss((w0 + (k + 0.5) * dw - w) / dw, SIG) *
             np.exp(2j * np.pi * (w0 + (k + 0.5) * dw) * nm1) for k in range(k0 - 2, k0 + 3))
    ref = np.exp(2j * np.pi * (u * l[None, :] + v * l[:, None])) * cd[None, :] * cd[:, None] * ws
    assert np.abs(A - ref).max() < 1e-12


def test_w_kernel_approaches_the_exact_transform():
    """Wide field (0.5 rad), 12 planes over |w| <= 30: with a kernel of 7 planes and its
    C_w correction the image is far closer to the exact transform than with nearest
    planes (or than the same stack without the C_w division)."""
    n, cell = 256, 0.5 / 256
    rng = np.random.default_rng(71)
    m = 6000
    du = 1.0 / (n * cell)
    uvw = np.stack([rng.uniform(-0.3, 0.3, m) * n * du, rng.uniform(-0.3, 0.3, m) * n * du,
                    rng.uniform(-30.0, 30.0, m)], axis=1)
    vis = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    wts = np.ones(m)
    q = np.array([40, 60, 200, 220, 128, 30, 100, 160])
    p = np.array([50, 210, 45, 190, 20, 128, 100, 170])
    De = pinlib.exact_dft(uvw, vis, wts, n, cell, q, p)
    inp = _inputs(uvw, vis, wts)
    err = {}
    for sw in (1, 7):
        out = oracle.image(inp, oracle.Params(n, 12, 7, cell, SIG, w_support=sw))
        err[sw] = np.abs(out["image"][0][q, p] - De).max()
    prm = oracle.Params(n, 12, 7, cell, SIG, w_support=7)
    out = oracle.image(inp, prm)
    st = out["stats"][0]
    # the same stack, divided by the uv correction and sum W only
    d = out["raw"][0].real / (oracle.kernel_transform(n, 7, SIG)[:, None] *
                              oracle.kernel_transform(n, 7, SIG)[None, :]) / st["sum_w"]
    err_no_cw = np.abs(d[q, p] - De).max()
    assert err[7] < 0.1 * err[1]
    assert err[7] < 0.1 * err_no_cw


def w_kernel_edge_plane_error(sw):
    """Largest difference between the oracle's planes and hand-computed ones for the
    visibilities at the ends of the data's own w range (see test_w_kernel_edge_planes),
    and the number of planes that hold anything."""
    n, cell, S, nw = 64, 1.0 / 100, 7, 9
    hw = (sw - 1) // 2
    w_lo, w_mid, w_hi = -7.3, 2.0, 11.9
    # three visibilities on separate cells, so their footprints do not touch
    uvw = np.array([[-12.25, -8.5, w_lo], [13.5, 9.75, w_hi], [0.5, 0.25, w_mid]])
    vis = np.array([[0.3 - 0.8j], [1.1 + 0.2j], [-0.4 + 0.5j]])
    prm = oracle.Params(n, nw, S, cell, SIG, w_support=sw)
    lo, hi = oracle.w_range(_inputs(uvw, vis), prm)
    assert (lo, hi) == (w_lo, w_hi)
    g, cnt = oracle.grid(_inputs(uvw, vis), prm, lo, hi)
    assert cnt["n_used"] == 3
    x, y = pinlib.positions(uvw, n, cell)
    dw = (w_hi - w_lo) / (nw - 2 * hw)
    expect = {0: (hw, 0.5), 1: (nw - 1 - hw, -0.5)}   # visibility -> (k0, offset of j = 0)
    err = 0.0
    for r, (k0, off) in expect.items():
        i0_, j0 = int(math.floor(x[r] + 0.5)), int(math.floor(y[r] + 0.5))
        foot = np.outer(pinlib.gauss(j0 + np.arange(-3, 4) - y[r], SIG),
                        pinlib.gauss(i0_ + np.arange(-3, 4) - x[r], SIG))
        sl = (slice(j0 - 3, j0 + 4), slice(i0_ - 3, i0_ + 4))
        for k in range(nw):
            ref = np.zeros((7, 7), complex)
            if abs(k - k0) <= hw:
                # w_k from the geometry written out, as a check of the offset itself
                wk = w_lo + (k - hw + 0.5) * dw
                assert abs((wk - uvw[r, 2]) / dw - ((k - k0) + off)) < 1e-12
                ref = vis[r, 0] * pinlib.gauss((k - k0) + off, SIG) * foot
            err = max(err, float(np.abs(g[k][sl] - ref).max()))
    # planes holding anything: every one of the stack, the padding planes holding only
    # the tails of the edge visibilities
    return err, int(np.count_nonzero(np.abs(g).reshape(nw, -1).max(1)))


@pytest.mark.parametrize("sw", [3, 5])
def test_w_kernel_edge_planes(sw):
    """The visibilities at the ends of the data's own w range: the range covers the middle
    N_w - 2 h_w planes, so the one at w_max lies on the upper edge of plane N_w - h_w and
    the one at w_min on the lower edge of plane h_w (where rounding may place it one plane
    lower).  Each must spread over planes k0 - h_w .. k0 + h_w with k0 = N_w - 1 - h_w and
    k0 = h_w, the kernel's planes staying inside the stack.  Plane geometry by hand:
    dw = (w_max - w_min)/(N_w - 2 h_w), w_k = w_min + (k - h_w + 1/2) dw, so the offsets
    (w_k - w)/dw are j - 1/2 at w_max and j + 1/2 at w_min, j = -h_w .. h_w."""
    err, n_planes = w_kernel_edge_plane_error(sw)
    assert err < 1e-14
    assert n_planes == 9


def test_grid_threads_bit_identical():
    """The oracle's gridding splits mesh rows over threads; each cell still receives its
    terms in input order, so any thread count gives the one-thread result bit for bit."""
    from paper_2411_07321_amd import synth
    ds = synth.config0()
    op = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad)
    inp = oracle.Inputs.make(ds.uvw, None, ds.vis, ds.weights)
    wmin, wmax = oracle.w_range(inp, op)
    before = oracle.threads()
    try:
        res = []
        for t in (1, 3, 8):
            oracle.threads(t)
            res.append(oracle.grid(inp, op, wmin, wmax))
    finally:
        oracle.threads(before)
    for g, cnt in res[1:]:
        assert np.array_equal(g, res[0][0])
        assert cnt == res[0][1]
