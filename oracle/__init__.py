"""FP64 CPU oracle of the w-stacking imager -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP library never calls it and shares no code with
it.  Everything here runs in float64 / complex128.

Method (De Rubeis et al., "Accelerating radio astronomy imaging with RICK",
arXiv 2411.07321, Sec. 2):

  O1 geometry   pixel p has l_p = (p - N/2) dl, cell i has u_i = (i - N/2)/(N dl)
                (Sec. 2: the N_u x N_v x N_w mesh; u,v,w in wavelengths).
  O2 validity   unflagged, finite, weight > 0, footprint inside the mesh.
  O3 planes     nearest of N_w cell-centred w-planes (Sec. 2, w-stacking paragraph).
  O4 gridding   Eq. 3 with a separable Gaussian of support S    (wsg_oracle.c)
  O5 transform  unnormalised centred 2D inverse DFT of every plane (Sec. 2, third
                component; sign + from Eq. 2).  numpy.fft is the library step.
  O6 w-correct  A = sum_k F_k exp(+2 pi i w_k (n - 1)) (Eq. 2; fourth component).
  O7 post       D = Re A / (sum W * C(nu_p) C(nu_q)): grid correction by the
                continuous transform C of the truncated kernel, and weight
                normalisation (a reading: the paper does not state either).
  O8 channels   one image per channel, or all channels into one image.

Parity status: every step is pinned by tests/test_oracle_pins.py against
brute-force direct transforms, closed forms (pure fringe, flat field,
quadrature vs complex-erf) and invariants (Parseval, grid sum, permutation,
linearity).  The paper prints no image or accuracy figure, so agreement with
the paper's own outputs is unpinned.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

C_LIGHT = 299792458.0
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wsg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Counts(ctypes.Structure):
    _fields_ = [("n_used", ctypes.c_int64), ("n_flagged", ctypes.c_int64),
                ("n_dropped", ctypes.c_int64), ("sum_w", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_w_range.restype = ctypes.c_int64
        lib.oracle_w_range.argtypes = [ctypes.c_int64, ctypes.c_int, P, P, P, P, P,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       P, P]
        lib.oracle_grid.restype = ctypes.c_int
        lib.oracle_grid.argtypes = [ctypes.c_int64, ctypes.c_int, P, P, P, P, P,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, P, P]
        lib.oracle_plane_geometry.restype = None
        lib.oracle_plane_geometry.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, P, P]
        lib.oracle_pixels.restype = ctypes.c_int
        lib.oracle_pixels.argtypes = [ctypes.c_int64, ctypes.c_int, P, P, P, P, P,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, P]
        lib.oracle_bessel_i0.restype = ctypes.c_double
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_bessel_i0.argtypes = [ctypes.c_double]
        lib.oracle_kernel_value.restype = ctypes.c_double
        lib.oracle_kernel_value.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_double]
        _lib = lib
    return _lib


@dataclass
class Params:
    """Imaging parameters (the same quantities the library takes)."""
    grid_n: int
    n_wplanes: int
    support: int
    cell_rad: float
    kernel_sigma: float = 0.9
    w_min: float = float("nan")        # nan -> range of the data
    w_max: float = float("nan")
    plane_lo: int = 0
    plane_hi: int = 0                  # 0 -> all planes
    grid_correct: bool = True
    normalize: bool = True
    per_channel: bool = False
    kernel: str = "gauss"              # "gauss" or "kb" (Kaiser-Bessel)
    kernel_beta: float = 0.0           # Kaiser-Bessel beta; 0 -> kb_default_beta(support)
    w_fold: bool = False               # grid rows with w < 0 at (-u, -v, -w) with conj(V)
    w_support: int = 1                 # planes a visibility spreads over (kernel in w)


@dataclass
class Inputs:
    """Measurements in float64: uvw [rows,3]; vis [rows,n_chan] complex128."""
    uvw: np.ndarray
    freq_hz: np.ndarray | None
    vis: np.ndarray
    weights: np.ndarray | None
    flags: np.ndarray | None

    @staticmethod
    def make(uvw, freq_hz, vis, weights=None, flags=None) -> "Inputs":
        uvw = np.ascontiguousarray(uvw, dtype=np.float64)
        vis = np.ascontiguousarray(vis, dtype=np.complex128)
        if vis.ndim == 1:
            vis = vis[:, None]
        if weights is not None:
            weights = np.ascontiguousarray(weights, dtype=np.float64).reshape(vis.shape)
        if flags is not None:
            flags = np.ascontiguousarray(flags, dtype=np.uint8).reshape(vis.shape)
        f = None if freq_hz is None else np.ascontiguousarray(freq_hz, dtype=np.float64)
        return Inputs(uvw, f, vis, weights, flags)

    @property
    def n_rows(self):
        return self.uvw.shape[0]

    @property
    def n_chan(self):
        return self.vis.shape[1]

    def chan_scale(self) -> np.ndarray:
        """Per-channel factor from metres to wavelengths (f/c), or 1 for uvw in wavelengths."""
        if self.freq_hz is None:
            return np.ones(self.n_chan, dtype=np.float64)
        return self.freq_hz / C_LIGHT


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def fold_w(inp: Inputs) -> Inputs:
    """w-folding.  The sky is real, so its visibility function is Hermitian:
    V(-u,-v,-w) = conj V(u,v,w) (Eq. 1).  A row with w < 0 is therefore the same
    sample as (-u, -v, -w) carrying conj(V) in every channel (f/c > 0 keeps the sign
    of w), and Re of the image of Eq. 2 is the same for both.  After folding every
    w is >= 0, so the planes span half the range for symmetric coverage."""
    neg = inp.uvw[:, 2] < 0.0
    if not neg.any():
        return inp
    uvw = inp.uvw.copy()
    uvw[neg] = -uvw[neg]
    vis = inp.vis.copy()
    vis[neg] = np.conj(vis[neg])
    return Inputs(uvw, inp.freq_hz, vis, inp.weights, inp.flags)


def _prepared(inp: Inputs, prm: Params) -> Inputs:
    return fold_w(inp) if prm.w_fold else inp


# ----------------------------------------------------------------------------
# O2/O3: data range of w and counts
# ----------------------------------------------------------------------------
def w_range(inp: Inputs, prm: Params, chan: int = -1):
    """(w_min, w_max) for the plane placement: the caller's range if given, else the
    range over valid measurements; (0, 0) when nothing is valid."""
    if math.isfinite(prm.w_min) and math.isfinite(prm.w_max):
        return float(prm.w_min), float(prm.w_max)
    inp = _prepared(inp, prm)
    lib = _load()
    sc = inp.chan_scale()
    lo, hi = ctypes.c_double(0.0), ctypes.c_double(0.0)
    lib.oracle_w_range(inp.n_rows, inp.n_chan, _ptr(inp.uvw), _ptr(sc), _ptr(inp.vis),
                       _ptr(inp.weights), _ptr(inp.flags), prm.grid_n, prm.support,
                       prm.cell_rad, chan, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def plane_w(k: np.ndarray | int, w_min: float, w_max: float, n_w: int, w_support: int = 1):
    """w of plane k: w0 + (k + 1/2) dw, or w0 when dw = 0 (O3; plane_geometry)."""
    w0, dw = plane_geometry(w_min, w_max, n_w, w_support)
    k = np.asarray(k, dtype=np.float64)
    if dw == 0.0:
        return np.full_like(k, w0)
    return w0 + (k + 0.5) * dw


# ----------------------------------------------------------------------------
# O4: gridding (Eq. 3)
# ----------------------------------------------------------------------------
def grid(inp: Inputs, prm: Params, w_min: float, w_max: float, plane_lo: int = 0,
         plane_hi: int | None = None, chan: int = -1):
    """Gridded planes [plane_hi-plane_lo, N, N] complex128 (row j = v index, column i =
    u index) and the counts (used, flagged, dropped, sum of weights)."""
    if plane_hi is None:
        plane_hi = prm.n_wplanes
    inp = _prepared(inp, prm)
    lib = _load()
    n = prm.grid_n
    g = np.zeros((plane_hi - plane_lo, n, n), dtype=np.complex128)
    cnt = _Counts()
    sc = inp.chan_scale()
    rc = lib.oracle_grid(inp.n_rows, inp.n_chan, _ptr(inp.uvw), _ptr(sc), _ptr(inp.vis),
                         _ptr(inp.weights), _ptr(inp.flags), n, prm.n_wplanes, prm.support,
                         prm.cell_rad, *_kernel_args(prm), *_w_kernel_args(prm), w_min, w_max,
                         plane_lo, plane_hi, chan, _ptr(g), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_grid: unsupported support")
    return g, {"n_used": cnt.n_used, "n_flagged": cnt.n_flagged, "n_dropped": cnt.n_dropped,
               "sum_w": cnt.sum_w}


# ----------------------------------------------------------------------------
# O5: transform
# ----------------------------------------------------------------------------
def fft_planes(g: np.ndarray) -> np.ndarray:
    """F[q,p] = sum_{j,i} g[j,i] exp(+2 pi i ((i-N/2)(p-N/2) + (j-N/2)(q-N/2))/N):
    the unnormalised inverse DFT with the origin at index N/2 on both sides."""
    x = np.fft.ifftshift(g, axes=(-2, -1))
    x = np.fft.ifft2(x, axes=(-2, -1), norm="forward")
    return np.fft.fftshift(x, axes=(-2, -1))


# ----------------------------------------------------------------------------
# O6: w-correction and plane sum (Eq. 2)
# ----------------------------------------------------------------------------
def n_minus_1(n: int, cell: float):
    """(n - 1) on the pixel grid in the cancellation-free form -eta/(1 + sqrt(1 - eta)),
    eta = l^2 + m^2; and the mask eta < 1 of pixels on the celestial sphere."""
    c = (np.arange(n, dtype=np.float64) - n / 2) * cell
    eta = c[None, :] ** 2 + c[:, None] ** 2          # [q, p]
    inside = eta < 1.0
    e = np.where(inside, eta, 0.0)
    return -e / (1.0 + np.sqrt(1.0 - e)), inside


def wcorrect(F: np.ndarray, w_min: float, w_max: float, n_w: int, cell: float,
             plane_lo: int = 0, w_support: int = 1) -> np.ndarray:
    """A[q,p] = sum_k F_k[q,p] exp(+2 pi i w_k (n_pq - 1)); 0 off the sphere."""
    n = F.shape[-1]
    nm1, inside = n_minus_1(n, cell)
    acc = np.zeros((n, n), dtype=np.complex128)
    for kk in range(F.shape[0]):
        wk = float(plane_w(plane_lo + kk, w_min, w_max, n_w, w_support))
        acc += F[kk] * np.exp(2j * np.pi * wk * nm1)
    acc[~inside] = 0.0
    return acc


# ----------------------------------------------------------------------------
# O7: grid correction and normalisation
# ----------------------------------------------------------------------------
def kb_default_beta(support: int) -> float:
    """Kaiser-Bessel shape for a mesh oversampled twice over the image, after Beatty,
    Nishimura and Pauly (2005): beta = pi sqrt((S/2)^2 (2 - 1/2)^2 - 0.8).  The paper
    names the Kaiser-Bessel kernel of Jackson et al. (1991) without its beta."""
    return math.pi * math.sqrt((support / 2.0) ** 2 * 1.5 ** 2 - 0.8)


def _kernel_args(prm: Params) -> tuple[int, float]:
    if prm.kernel == "gauss":
        return 0, prm.kernel_sigma
    if prm.kernel == "kb":
        return 1, (prm.kernel_beta if prm.kernel_beta > 0 else kb_default_beta(prm.support))
    raise ValueError(f"unknown kernel {prm.kernel!r}")


def _w_kernel_args(prm: Params) -> tuple[int, float]:
    """(w_support, shape) of the kernel in w: the uv kernel's kind over w_support
    planes (Gaussian: the same sigma in planes; Kaiser-Bessel: the given beta, else
    the default for w_support)."""
    if prm.w_support <= 1:
        return 1, 0.0
    if prm.kernel == "kb":
        return prm.w_support, (prm.kernel_beta if prm.kernel_beta > 0
                               else kb_default_beta(prm.w_support))
    return prm.w_support, prm.kernel_sigma


def plane_geometry(w_min: float, w_max: float, n_w: int, w_support: int = 1):
    """(w0, dw): plane k sits at w0 + (k + 1/2) dw.  With a kernel in w over
    w_support = 2 h_w + 1 planes, [w_min, w_max] covers the middle N_w - 2 h_w planes."""
    w0, dw = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _load().oracle_plane_geometry(w_min, w_max, n_w, w_support, ctypes.byref(w0), ctypes.byref(dw))
    return w0.value, dw.value


def kernel_value(prm: Params, d) -> np.ndarray:
    """G(d) of the gridding kernel (Eq. 3), elementwise over d (cells)."""
    lib = _load()
    kind, par = _kernel_args(prm)
    return np.vectorize(lambda x: lib.oracle_kernel_value(kind, par, prm.support, float(x)))(d)


def kernel_transform(n: int, support: int, sigma: float, nodes: int = 64, kernel: str = "gauss",
                     beta: float = 0.0) -> np.ndarray:
    """C(nu_p) = int_{-S/2}^{S/2} G(d) cos(2 pi nu_p d) dd at nu_p = (p - N/2)/N, by
    Gauss-Legendre quadrature (G is analytic on the support for both kernels)."""
    x, wq = np.polynomial.legendre.leggauss(nodes)
    a = support / 2.0
    d = a * x
    nu = (np.arange(n, dtype=np.float64) - n / 2) / n
    prm = Params(n, 1, support, 1.0, sigma, kernel=kernel, kernel_beta=beta)
    f = kernel_value(prm, d)
    return a * (np.cos(2.0 * np.pi * nu[:, None] * d[None, :]) * (wq * f)[None, :]).sum(axis=1)


def w_kernel_transform(nu: np.ndarray, prm: Params, nodes: int = 64) -> np.ndarray:
    """C_w(nu) = int G_w(d) cos(2 pi nu d) dd over the w support (in planes), by
    Gauss-Legendre quadrature, at arbitrary nu."""
    sw, par = _w_kernel_args(prm)
    x, wq = np.polynomial.legendre.leggauss(nodes)
    a = sw / 2.0
    d = a * x
    lib = _load()
    kind = 1 if prm.kernel == "kb" else 0
    f = np.array([lib.oracle_kernel_value(kind, par, sw, float(t)) for t in d])
    nu = np.asarray(nu, dtype=np.float64)
    return a * (np.cos(2.0 * np.pi * nu[..., None] * d) * (wq * f)).sum(axis=-1)


def post(A: np.ndarray, sum_w: float, prm: Params, w_min: float = 0.0,
         w_max: float = 0.0) -> np.ndarray:
    """D = Re A / (sum W * C(nu_p) C(nu_q) [* C_w(dw (n_pq - 1))]), each factor
    switchable; 0 if sum W = 0.  The C_w factor undoes a kernel in w: summing the
    planes with their phases turns the visibility's spread over planes into the
    window's transform at dw (n - 1) (Poisson summation; 1 with w_support 1)."""
    d = A.real.copy()
    if prm.grid_correct:
        c = kernel_transform(prm.grid_n, prm.support, prm.kernel_sigma, kernel=prm.kernel,
                             beta=prm.kernel_beta)
        d /= c[:, None] * c[None, :]
        if prm.w_support > 1:
            _, dw = plane_geometry(w_min, w_max, prm.n_wplanes, prm.w_support)
            if dw > 0.0:
                nm1, inside = n_minus_1(prm.grid_n, prm.cell_rad)
                cw = w_kernel_transform(dw * nm1, prm)
                d = np.where(inside, d / cw, 0.0)
    if prm.normalize:
        if sum_w > 0.0:
            d /= sum_w
        else:
            d[:] = 0.0
    return d


# ----------------------------------------------------------------------------
# whole method
# ----------------------------------------------------------------------------
def image(inp: Inputs, prm: Params, plane_chunk: int | None = None, keep_stages: bool = False):
    """The imaging method end to end.  Returns dict(image [n_img,N,N] f64, raw
    [n_img,N,N] complex128 (A before post), stats per image, and, with keep_stages,
    grid and planes of the first image)."""
    chans = list(range(inp.n_chan)) if prm.per_channel else [-1]
    lo = prm.plane_lo
    hi = prm.plane_hi if prm.plane_hi > 0 else prm.n_wplanes
    step = plane_chunk or (hi - lo)
    imgs, raws, stats = [], [], []
    stages = {}
    for ci, ch in enumerate(chans):
        wmin, wmax = w_range(inp, prm, ch)
        acc = np.zeros((prm.grid_n, prm.grid_n), dtype=np.complex128)
        cnt = None
        for k0 in range(lo, hi, step):
            k1 = min(hi, k0 + step)
            g, cnt = grid(inp, prm, wmin, wmax, k0, k1, ch)
            F = fft_planes(g)
            if keep_stages and ci == 0 and step == hi - lo:
                stages = {"grid": g, "planes": F}
            acc += wcorrect(F, wmin, wmax, prm.n_wplanes, prm.cell_rad, k0, prm.w_support)
            del g, F
        if cnt is None:
            _, cnt = grid(inp, prm, wmin, wmax, 0, 0, ch)
        raws.append(acc)
        imgs.append(post(acc, cnt["sum_w"], prm, wmin, wmax))
        stats.append(dict(cnt, w_min=wmin, w_max=wmax))
    out = {"image": np.stack(imgs), "raw": np.stack(raws), "stats": stats}
    out.update(stages)
    return out


def pixels(inp: Inputs, prm: Params, pix_q, pix_p, chan: int = -1) -> np.ndarray:
    """Raw image A at the listed pixels, evaluated directly from the measurements
    (for sampled checks at full size).  complex128 [n_pix]."""
    if prm.w_support > 1:
        raise ValueError("the pixel evaluator takes each visibility on its nearest plane only")
    lib = _load()
    wmin, wmax = w_range(inp, prm, chan)
    inp = _prepared(inp, prm)
    q = np.ascontiguousarray(pix_q, dtype=np.int32)
    p = np.ascontiguousarray(pix_p, dtype=np.int32)
    out = np.zeros(len(q), dtype=np.complex128)
    sc = inp.chan_scale()
    rc = lib.oracle_pixels(inp.n_rows, inp.n_chan, _ptr(inp.uvw), _ptr(sc), _ptr(inp.vis),
                           _ptr(inp.weights), _ptr(inp.flags), prm.grid_n, prm.n_wplanes,
                           prm.support, prm.cell_rad, *_kernel_args(prm), wmin, wmax, chan,
                           len(q), _ptr(q), _ptr(p), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_pixels failed")
    return out


def threads(n: int = 0) -> int:
    """Threads of the oracle's parallel loops (gridding by row bands, pixel sums); n > 0
    sets them.  Results do not depend on the count."""
    return int(_load().oracle_threads(int(n)))
