"""Seeded synthetic interferometer data: the inputs of the w-stacking imager.

This module only *produces inputs*: antenna layouts, Earth-rotation (u,v,w)
tracks, point-source visibilities from the measurement equation (Eq. 1 of
De Rubeis et al., "Accelerating radio astronomy imaging with RICK", Sec. 2),
noise, weights and flags.  It holds none of the imaging arithmetic (no
gridding kernel, no transform, no w-correction); both the FP64 oracle and
the HIP library are fed from here.

The observations of the paper (LOFAR HBA, 8 h tracks, Table 1) are not
available; these generators stand in for them with the same structure:
an 8 h Earth-rotation track, a LOFAR-like latitude, time-major row order
(rows of one time slice are contiguous, as in a measurement set) and
channels as the fastest index.

uvw follow the textbook relation between an equatorial baseline vector and
the (u,v,w) frame (Thompson, Moran & Swenson, "Interferometry and Synthesis
in Radio Astronomy", eq. 4.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0            # m/s
LATITUDE_DEG = 52.91             # LOFAR-like site
DEC_DEG = 45.0                   # phase-centre declination


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def layout_uniform_disc(n_ant: int, radius_m: float, rng: np.random.Generator) -> np.ndarray:
    """Antennas uniform in a disc: r = R*sqrt(U), theta ~ U[0, 2pi).  Returns (E, N) [n_ant, 2]."""
    r = radius_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * np.pi * rng.random(n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def layout_log_radial(n_ant: int, r_min: float, r_max: float, rng: np.random.Generator) -> np.ndarray:
    """Antennas with log-uniform radius r = r_min*(r_max/r_min)^U: dense core, sparse outskirts."""
    r = r_min * (r_max / r_min) ** rng.random(n_ant)
    th = 2.0 * np.pi * rng.random(n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def baselines_xyz(en: np.ndarray, lat_deg: float = LATITUDE_DEG) -> np.ndarray:
    """Equatorial baseline vectors (X, Y, Z) of all pairs a < b (no autocorrelations).

    Antennas lie on the local horizontal plane (U = 0), so X = -N sin(lat),
    Y = E, Z = N cos(lat).
    """
    lat = math.radians(lat_deg)
    e, n = en[:, 0], en[:, 1]
    xyz = np.stack([-n * math.sin(lat), e, n * math.cos(lat)], axis=1)
    a, b = np.triu_indices(en.shape[0], k=1)
    return xyz[b] - xyz[a]


def hour_angles(n_times: int, track_h: float = 8.0) -> np.ndarray:
    """Hour angles (rad) of an n_times-sample track centred on transit."""
    t = np.arange(n_times, dtype=np.float64)
    h_hours = -track_h / 2.0 + track_h * (t + 0.5) / n_times
    return h_hours * (2.0 * np.pi / 24.0)


def uvw_tracks(bxyz: np.ndarray, ha: np.ndarray, dec_deg: float = DEC_DEG) -> np.ndarray:
    """(u,v,w) in the units of bxyz, time-major rows (row = t*n_bl + b)."""
    d = math.radians(dec_deg)
    sd, cd = math.sin(d), math.cos(d)
    sh = np.sin(ha)[:, None]
    ch = np.cos(ha)[:, None]
    bx, by, bz = bxyz[None, :, 0], bxyz[None, :, 1], bxyz[None, :, 2]
    u = sh * bx + ch * by
    v = -sd * ch * bx + sd * sh * by + cd * bz
    w = cd * ch * bx - cd * sh * by + sd * bz
    return np.stack([u, v, w], axis=-1).reshape(-1, 3)


# ----------------------------------------------------------------------------
# sky and visibilities
# ----------------------------------------------------------------------------
@dataclass
class Sky:
    l: np.ndarray
    m: np.ndarray
    flux: np.ndarray


def point_sources(n: int, half_box: float, grid_n: int, cell: float,
                  rng: np.random.Generator) -> Sky:
    """n sources uniform in |l|,|m| <= half_box, snapped to pixel centres (p - N/2)*cell."""
    l = rng.uniform(-half_box, half_box, n)
    m = rng.uniform(-half_box, half_box, n)
    l = np.round(l / cell) * cell
    m = np.round(m / cell) * cell
    flux = rng.uniform(0.1, 1.0, n)
    return Sky(l=l, m=m, flux=flux)


def _torch_device(device):
    import torch
    return torch.device(device if device is not None else "cpu")


def visibilities(uvw: np.ndarray, scale: np.ndarray, sky: Sky, *, device=None,
                 chunk: int = 1 << 18) -> np.ndarray:
    """Point-source visibilities from the measurement equation with apparent fluxes.

    V[r, c] = sum_s S_s exp(-2 pi i (u l_s + v m_s + w (n_s - 1))), with
    (u,v,w) = uvw[r] * scale[c] (scale = f_c/c for uvw in metres, 1 for
    uvw already in wavelengths).  Computed in FP64 with torch on `device`.
    Returns complex128 [rows, n_chan].
    """
    import torch
    dev = _torch_device(device)
    eta = sky.l ** 2 + sky.m ** 2
    nm1 = -eta / (1.0 + np.sqrt(1.0 - eta))
    lmn = torch.tensor(np.stack([sky.l, sky.m, nm1], axis=0), dtype=torch.float64, device=dev)
    flux = torch.tensor(sky.flux, dtype=torch.float64, device=dev)
    rows = uvw.shape[0]
    n_chan = len(scale)
    out = np.empty((rows, n_chan), dtype=np.complex128)
    two_pi = 2.0 * math.pi
    for r0 in range(0, rows, chunk):
        r1 = min(rows, r0 + chunk)
        b = torch.tensor(uvw[r0:r1], dtype=torch.float64, device=dev)
        ph0 = b @ lmn                                   # [chunk, S] (uvw units)
        acc = torch.empty((r1 - r0, n_chan), dtype=torch.complex128, device=dev)
        for c in range(n_chan):
            ph = ph0 * (-two_pi * float(scale[c]))
            re = (torch.cos(ph) * flux).sum(dim=1)
            im = (torch.sin(ph) * flux).sum(dim=1)
            acc[:, c] = torch.complex(re, im)
        out[r0:r1] = acc.cpu().numpy()
    return out


def add_noise(vis: np.ndarray, sigma: float, rng: np.random.Generator, chunk: int = 1 << 20) -> None:
    """Add independent N(0, sigma^2) to real and imaginary parts, in place."""
    flat = vis.reshape(-1)
    for i0 in range(0, flat.size, chunk):
        i1 = min(flat.size, i0 + chunk)
        z = rng.standard_normal((i1 - i0, 2))
        flat[i0:i1] += sigma * (z[:, 0] + 1j * z[:, 1])


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
@dataclass
class Dataset:
    """One imaging job: inputs plus the imaging parameters."""
    name: str
    uvw: np.ndarray                 # [rows, 3] f64; metres if freq_hz is not None else wavelengths
    freq_hz: np.ndarray | None      # [n_chan] or None
    vis: np.ndarray                 # [rows, n_chan] complex128 or complex64
    weights: np.ndarray | None      # [rows, n_chan] f64 or f32
    flags: np.ndarray | None        # [rows, n_chan] u8
    grid_n: int
    n_wplanes: int
    support: int
    cell_rad: float
    precision: str                  # "f64" | "f32_phase64" | "f32_phase32"
    kernel_sigma: float = 0.9
    per_channel: bool = False       # one image per channel (cube) instead of one image
    row_period: int = 0             # baselines per time slice (rows are time-major)
    sky: Sky | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_rows(self) -> int:
        return self.uvw.shape[0]

    @property
    def n_chan(self) -> int:
        return self.vis.shape[1]

    @property
    def n_vis(self) -> int:
        return self.vis.shape[0] * self.vis.shape[1]


CONFIG_SEED0 = 1000


def config0(seed: int = CONFIG_SEED0 + 0, device=None) -> Dataset:
    """Tiny FP64 case: 32 antennas in a 2 km disc, 64 times, 150 MHz, 5 sources within +-1 deg,
    256^2 grid, 8 w-planes, support 7.  31,744 complex128 visibilities, uvw in wavelengths."""
    rng = np.random.default_rng(seed)
    en = layout_uniform_disc(32, 1000.0, rng)
    uvw_m = uvw_tracks(baselines_xyz(en), hour_angles(64))
    lam = C_LIGHT / 150e6
    uvw = uvw_m / lam
    n, cell = 256, math.radians(4.0) / 256
    sky = point_sources(5, math.radians(1.0), n, cell, rng)
    vis = visibilities(uvw, np.array([1.0]), sky, device=device)
    w = np.ones(vis.shape, dtype=np.float64)
    return Dataset("config0", uvw, None, vis, w, None, n, 8, 7, cell, "f64", sky=sky,
                   row_period=32 * 31 // 2)


def _config1_inputs(seed: int, device, rows_stride: int = 1):
    rng = np.random.default_rng(seed)
    en = layout_log_radial(256, 30.0, 10000.0, rng)
    uvw = uvw_tracks(baselines_xyz(en), hour_angles(2048))
    if rows_stride > 1:
        uvw = np.ascontiguousarray(uvw[::rows_stride])
    freq = (150.5 + (np.arange(4) - 1.5) * 0.48828) * 1e6
    # sources are drawn once in the +-0.095 box on the 4096 grid's pixel centres
    sky = point_sources(200, 0.095, 4096, 0.2 / 4096, rng)
    vis = visibilities(uvw, freq / C_LIGHT, sky, device=device)
    add_noise(vis, 0.01, rng)
    return uvw, freq, vis, sky


def config1(seed: int = CONFIG_SEED0 + 1, device=None, rows_stride: int = 1) -> Dataset:
    """Single large image: 256 antennas, log-radial 30 m..10 km radius (20 km extent),
    2048 times, 4 channels around 150.5 MHz (1953.1 kHz sub-band), 200 sources within
    +-0.095 rad, noise sigma 0.01; 4096^2 grid, 64 w-planes, support 7, FP32 grid,
    FP64 w-phase.  66,846,720 rows x 4 channels = 267,386,880 complex64 visibilities.
    `rows_stride` > 1 keeps every k-th row (a thinned copy for quick checks)."""
    uvw, freq, vis, sky = _config1_inputs(seed, device, rows_stride)
    vis = vis.astype(np.complex64)
    w = np.ones(vis.shape, dtype=np.float32)
    return Dataset("config1", uvw, freq, vis, w, None, 4096, 64, 7, 0.2 / 4096,
                   "f32_phase64", sky=sky, row_period=0 if rows_stride > 1 else 256 * 255 // 2)


def config2(precision: str = "f32_phase64", seed: int = CONFIG_SEED0 + 1, device=None,
            rows_stride: int = 1) -> Dataset:
    """Precision study: the config-1 inputs at 2048^2 with 32 w-planes (field edges at
    l, m = +-0.1).  Baselines beyond the grid are dropped and counted."""
    uvw, freq, vis, sky = _config1_inputs(seed, device, rows_stride)
    if precision == "f64":
        w = np.ones(vis.shape, dtype=np.float64)
    else:
        vis = vis.astype(np.complex64)
        w = np.ones(vis.shape, dtype=np.float32)
    return Dataset("config2", uvw, freq, vis, w, None, 2048, 32, 7, 0.2 / 2048,
                   precision, sky=sky, row_period=0 if rows_stride > 1 else 256 * 255 // 2)


def config3(seed: int = CONFIG_SEED0 + 3, device=None, n_times: int = 512) -> Dataset:
    """Batched channels: 128 antennas in a 2 km disc, 512 times, 32 channels at
    120 + 60*c/31 MHz sharing one uvw set (metres), per-channel flag fraction
    p_c ~ U[0, 0.6]; one 1024^2 x 16-plane stack and one image per channel."""
    rng = np.random.default_rng(seed)
    en = layout_uniform_disc(128, 1000.0, rng)
    uvw = uvw_tracks(baselines_xyz(en), hour_angles(n_times))
    freq = (120.0 + 60.0 * np.arange(32) / 31.0) * 1e6
    n, cell = 1024, 0.2 / 1024
    sky = point_sources(5, 0.05, n, cell, rng)
    vis = visibilities(uvw, freq / C_LIGHT, sky, device=device).astype(np.complex64)
    p = rng.uniform(0.0, 0.6, 32)
    flags = np.empty(vis.shape, dtype=np.uint8)
    for c in range(32):
        flags[:, c] = (rng.random(vis.shape[0]) < p[c]).astype(np.uint8)
    w = np.ones(vis.shape, dtype=np.float32)
    return Dataset("config3", uvw, freq, vis, w, flags, n, 16, 7, cell, "f32_phase64",
                   per_channel=True, sky=sky, meta={"flag_fraction": p},
                   row_period=128 * 127 // 2)


# ----------------------------------------------------------------------------
# serving jobs
# ----------------------------------------------------------------------------
JOB_GRID_N = (512, 1024, 2048, 4096)
JOB_WPLANES = (8, 16, 32, 64)


def job_spec(rng: np.random.Generator) -> dict:
    """Draw one serving job's shape: N, N_w, target visibility count, antennas, times."""
    n = int(rng.choice(JOB_GRID_N))
    nw = int(rng.choice(JOB_WPLANES))
    m_target = float(np.exp(rng.uniform(math.log(1e5), math.log(5e7))))
    n_ant = int(rng.integers(32, 257))
    n_bl = n_ant * (n_ant - 1) // 2
    n_times = max(1, int(round(m_target / n_bl)))
    return {"grid_n": n, "n_wplanes": nw, "m_target": m_target, "n_ant": n_ant,
            "n_times": n_times}


def make_job(spec: dict, seed: int, device=None) -> Dataset:
    """Materialise a job: uniform disc of diameter 4.5*N m, 150 MHz, 5 sources within
    +-0.05 rad, cell 0.2/N, complex64 visibilities, uvw in wavelengths."""
    rng = np.random.default_rng(seed)
    n = spec["grid_n"]
    en = layout_uniform_disc(spec["n_ant"], 4.5 * n / 2.0, rng)
    lam = C_LIGHT / 150e6
    uvw = uvw_tracks(baselines_xyz(en), hour_angles(spec["n_times"])) / lam
    cell = 0.2 / n
    sky = point_sources(5, 0.05, n, cell, rng)
    vis = visibilities(uvw, np.array([1.0]), sky, device=device).astype(np.complex64)
    w = np.ones(vis.shape, dtype=np.float32)
    return Dataset(f"job{seed}", uvw, None, vis, w, None, n, spec["n_wplanes"], 7, cell,
                   "f32_phase64", sky=sky, meta=dict(spec),
                   row_period=spec["n_ant"] * (spec["n_ant"] - 1) // 2)


def poisson_arrivals(n_jobs: int, rate_hz: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate_hz, n_jobs))


# ----------------------------------------------------------------------------
# small random inputs for stage tests
# ----------------------------------------------------------------------------
def random_planes(n_planes: int, n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Gaussian complex planes [n_planes, n, n] (stage inputs for transform tests)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n_planes, n, n)) + 1j * rng.standard_normal((n_planes, n, n))
    return z.astype(dtype)


def random_visibilities(n_rows: int, n_chan: int, grid_n: int, cell: float, seed: int,
                        w_extent: float = 200.0, fill: float = 0.45) -> tuple:
    """Uniformly scattered (u,v,w) in wavelengths with |u|,|v| <= fill * N * du, complex
    Gaussian visibilities and U(0.5, 1.5) weights (stage inputs with ragged counts)."""
    rng = np.random.default_rng(seed)
    du = 1.0 / (grid_n * cell)
    ext = fill * grid_n * du
    uvw = np.empty((n_rows, 3))
    uvw[:, 0] = rng.uniform(-ext, ext, n_rows)
    uvw[:, 1] = rng.uniform(-ext, ext, n_rows)
    uvw[:, 2] = rng.uniform(-w_extent, w_extent, n_rows)
    vis = rng.standard_normal((n_rows, n_chan)) + 1j * rng.standard_normal((n_rows, n_chan))
    wts = rng.uniform(0.5, 1.5, (n_rows, n_chan))
    return uvw, vis, wts


# ----------------------------------------------------------------------------
# large configurations generated on the device (torch), for benchmarks
# ----------------------------------------------------------------------------
def visibilities_device(uvw_dev, scale, sky: Sky, noise_sigma: float, seed: int,
                        dtype=None, chunk: int = 1 << 18):
    """As `visibilities` (Eq. 1, apparent fluxes, FP64) but on the device holding uvw_dev,
    plus complex Gaussian noise from a seeded torch generator on that device; returns a
    [rows, n_chan] tensor of `dtype` (complex64 by default) on the device."""
    import torch
    dev = uvw_dev.device
    dtype = dtype or torch.complex64
    eta = sky.l ** 2 + sky.m ** 2
    nm1 = -eta / (1.0 + np.sqrt(1.0 - eta))
    lmn = torch.tensor(np.stack([sky.l, sky.m, nm1], axis=0), dtype=torch.float64, device=dev)
    flux = torch.tensor(sky.flux, dtype=torch.float64, device=dev)
    rows, n_chan = uvw_dev.shape[0], len(scale)
    out = torch.empty((rows, n_chan), dtype=dtype, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    two_pi = 2.0 * math.pi
    for r0 in range(0, rows, chunk):
        r1 = min(rows, r0 + chunk)
        ph0 = uvw_dev[r0:r1] @ lmn
        for c in range(n_chan):
            ph = ph0 * (-two_pi * float(scale[c]))
            re = (torch.cos(ph) * flux).sum(dim=1)
            im = (torch.sin(ph) * flux).sum(dim=1)
            if noise_sigma > 0:
                z = torch.randn((r1 - r0, 2), dtype=torch.float64, device=dev, generator=gen)
                re = re + noise_sigma * z[:, 0]
                im = im + noise_sigma * z[:, 1]
            out[r0:r1, c] = torch.complex(re, im).to(dtype)
    return out


def config1_device(device="cuda", seed: int = CONFIG_SEED0 + 1, grid_n: int = 4096,
                   n_wplanes: int = 64, precision: str = "f32_phase64", rows_stride: int = 1):
    """Config 1 (or, with grid_n=2048 / n_wplanes=32, config 2) with the arrays resident on
    the device: dict(uvw f64 [rows,3], vis complex64/128 [rows,4], weights f32/f64
    [rows,4], freq_hz numpy, params dict, sky).  Same layout, frequencies and sky as
    config1(); the noise comes from a seeded torch generator on the device."""
    import torch
    rng = np.random.default_rng(seed)
    en = layout_log_radial(256, 30.0, 10000.0, rng)
    uvw = uvw_tracks(baselines_xyz(en), hour_angles(2048))
    if rows_stride > 1:
        uvw = np.ascontiguousarray(uvw[::rows_stride])
    freq = (150.5 + (np.arange(4) - 1.5) * 0.48828) * 1e6
    sky = point_sources(200, 0.095, 4096, 0.2 / 4096, rng)
    uvw_d = torch.from_numpy(uvw).to(device)
    f64 = precision == "f64"
    vis = visibilities_device(uvw_d, freq / C_LIGHT, sky, 0.01, seed,
                              dtype=torch.complex128 if f64 else torch.complex64)
    wts = torch.ones(vis.shape, dtype=torch.float64 if f64 else torch.float32, device=device)
    return {"uvw": uvw_d, "vis": vis, "weights": wts, "freq_hz": freq, "sky": sky,
            "row_period": 0 if rows_stride > 1 else 256 * 255 // 2,
            "params": dict(grid_n=grid_n, n_wplanes=n_wplanes, support=7,
                           cell_rad=0.2 / grid_n, precision=precision, kernel_sigma=0.9)}
