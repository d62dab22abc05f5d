"""Input generator checks: array geometry, rotation invariance, measurement-equation
special cases.  (uvw relation: Thompson, Moran & Swenson, eq. 4.1.)"""
import math

import numpy as np

from paper_2411_07321_amd import synth


def test_baseline_count_and_rows(config0):
    # 32 antennas -> 32*31/2 = 496 baselines; 64 times -> 31,744 rows, one channel
    assert config0.uvw.shape == (31744, 3)
    assert config0.vis.shape == (31744, 1)
    assert config0.vis.dtype == np.complex128


def test_uvw_rotation_invariance():
    # |(u,v,w)| = |B| at every hour angle: the (u,v,w) frame is a rotation of (X,Y,Z)
    rng = np.random.default_rng(7)
    en = synth.layout_uniform_disc(12, 1000.0, rng)
    b = synth.baselines_xyz(en)
    uvw = synth.uvw_tracks(b, synth.hour_angles(37)).reshape(37, -1, 3)
    nb = np.linalg.norm(b, axis=1)
    assert np.allclose(np.linalg.norm(uvw, axis=2), nb[None, :], rtol=1e-12, atol=0)


def test_uvw_at_transit_matches_closed_form():
    # at H = 0: u = B_Y, v = -sin(dec) B_X + cos(dec) B_Z, w = cos(dec) B_X + sin(dec) B_Z
    b = np.array([[3.0, -5.0, 7.0]])
    uvw = synth.uvw_tracks(b, np.array([0.0]), dec_deg=30.0)[0]
    d = math.radians(30.0)
    assert np.allclose(uvw, [-5.0, -math.sin(d) * 3 + math.cos(d) * 7,
                             math.cos(d) * 3 + math.sin(d) * 7], atol=1e-14)


def test_phase_centre_source_is_flat():
    # a unit source at l = m = 0 gives V = 1 + 0i exactly on every baseline (Eq. 1)
    rng = np.random.default_rng(3)
    uvw = rng.uniform(-1e4, 1e4, (500, 3))
    sky = synth.Sky(l=np.array([0.0]), m=np.array([0.0]), flux=np.array([1.0]))
    v = synth.visibilities(uvw, np.array([1.0, 1.3]), sky)
    assert np.all(v == 1.0 + 0.0j)


def test_point_source_phase():
    # one source: V = S exp(-2 pi i (u l + v m + w (n - 1))) with n - 1 from sqrt(1 - l^2 - m^2)
    uvw = np.array([[100.0, -250.0, 30.0]])
    sky = synth.Sky(l=np.array([0.01]), m=np.array([-0.02]), flux=np.array([0.5]))
    v = synth.visibilities(uvw, np.array([1.0]), sky)[0, 0]
    n = math.sqrt(1 - 0.01 ** 2 - 0.02 ** 2)
    ph = -2 * math.pi * (100 * 0.01 + (-250) * (-0.02) + 30 * (n - 1))
    assert abs(v - 0.5 * complex(math.cos(ph), math.sin(ph))) < 1e-13


def test_config_seeds_are_reproducible():
    a = synth.config0()
    b = synth.config0()
    assert np.array_equal(a.uvw, b.uvw) and np.array_equal(a.vis, b.vis)


def test_job_spec_ranges():
    rng = np.random.default_rng(1004)
    for _ in range(50):
        s = synth.job_spec(rng)
        assert s["grid_n"] in synth.JOB_GRID_N and s["n_wplanes"] in synth.JOB_WPLANES
        assert 1e5 <= s["m_target"] <= 5e7 and 32 <= s["n_ant"] <= 256
