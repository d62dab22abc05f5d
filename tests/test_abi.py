"""C ABI contract checks that need no GPU: the library loads, exports every symbol
include/wsg.h declares, validates parameters and reports footprints."""
import math
import os
import re

import numpy as np
import pytest

from paper_2411_07321_amd import wsg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "wsg.h")).read()
    decl = r"^\s*(?:wsg_status|void|const char \*|int32_t)\s*\*?\s*(wsg_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


def test_header_symbols_exported():
    lib = wsg.load()
    names = _declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(wsg.SYMBOLS)


def _p(**kw):
    base = dict(grid_n=256, n_wplanes=8, support=7, cell_rad=1e-4, precision="f64")
    base.update(kw)
    return wsg.make_params(**base)


def _v(n_rows=10, n_chan=1, **kw):
    uvw = np.zeros((n_rows, 3))
    vis = np.zeros((n_rows, n_chan), np.complex128)
    return wsg.make_vis(uvw, vis, **kw)


@pytest.mark.parametrize("kw,code", [
    (dict(), wsg.OK),
    (dict(grid_n=100), wsg.EINVAL),
    (dict(grid_n=8), wsg.EUNSUPPORTED),
    (dict(grid_n=8192), wsg.OK),
    (dict(grid_n=16384), wsg.OK),
    (dict(grid_n=32768), wsg.EUNSUPPORTED),
    (dict(grid_n=16384, tile=32, precision="f32_phase64"), wsg.EUNSUPPORTED),  # > 256 tiles per axis
    (dict(grid_n=16384, tile=64, precision="f32_phase64"), wsg.OK),
    (dict(support=6), wsg.EINVAL),
    (dict(support=0), wsg.EINVAL),
    (dict(support=17), wsg.EUNSUPPORTED),
    (dict(n_wplanes=0), wsg.EINVAL),
    (dict(cell_rad=0.0), wsg.EINVAL),
    (dict(cell_rad=math.nan), wsg.EINVAL),
    (dict(kernel_sigma=-1.0), wsg.EINVAL),
    (dict(w_min=1.0), wsg.EINVAL),                       # one-sided range
    (dict(w_min=2.0, w_max=1.0), wsg.EINVAL),
    (dict(w_min=-1.0, w_max=math.inf), wsg.EINVAL),
    (dict(plane_lo=2, plane_hi=4), wsg.EINVAL),          # shard without a given range
    (dict(plane_lo=2, plane_hi=4, w_min=0.0, w_max=1.0), wsg.OK),
    (dict(plane_lo=4, plane_hi=4, w_min=0.0, w_max=1.0), wsg.EINVAL),
    (dict(plane_lo=0, plane_hi=9, w_min=0.0, w_max=1.0), wsg.EINVAL),
    (dict(tile=48), wsg.EINVAL),
    (dict(planes_per_pass=-1), wsg.EINVAL),
    (dict(planes_per_pass=3), wsg.OK),
    (dict(planes_per_pass=20), wsg.OK),                 # more than N_w: one pass
    (dict(tile=128), wsg.EUNSUPPORTED),                  # FP64 LDS tile limit
    (dict(tile=128, precision="f32_phase64"), wsg.EUNSUPPORTED),
    (dict(tile=16, precision="f32_phase64"), wsg.OK),
    (dict(kernel="kb"), wsg.OK),
    (dict(kernel="kb", kernel_sigma=-1.0), wsg.OK),      # sigma is the Gaussian's
    (dict(kernel="kb", kernel_beta=-1.0), wsg.EINVAL),
    (dict(kernel="kb", kernel_beta=math.nan), wsg.EINVAL),
    (dict(kernel="kb", kernel_beta=65.0), wsg.EUNSUPPORTED),
    (dict(kernel="kb", support=1), wsg.EINVAL),           # no default beta for S = 1
    (dict(kernel="kb", support=1, kernel_beta=2.0), wsg.OK),
    (dict(kernel="kb", kernel_beta=60.0), wsg.OK),        # FP64: exact series
    # FP32 mesh: per-tap degree-8 fit, 1.7e-6 off at beta = 60, S = 7
    (dict(kernel="kb", kernel_beta=60.0, precision="f32_phase64"), wsg.EUNSUPPORTED),
    (dict(kernel="kb", kernel_beta=25.0, precision="f32_phase64"), wsg.OK),
    (dict(kernel="kb", support=3, kernel_beta=10.0, precision="f32_phase32"), wsg.EUNSUPPORTED),
    (dict(w_support=7), wsg.OK),
    (dict(w_support=7, kernel="kb"), wsg.OK),
    (dict(w_support=4), wsg.EINVAL),
    (dict(w_support=-1), wsg.EINVAL),
    (dict(w_support=17), wsg.EUNSUPPORTED),
    (dict(w_support=9), wsg.EINVAL),                      # more planes of kernel than planes
    (dict(w_support=3, plane_lo=2, plane_hi=4, w_min=0.0, w_max=1.0), wsg.EUNSUPPORTED),
    (dict(w_support=3, plane_lo=0, plane_hi=8, w_min=0.0, w_max=1.0), wsg.OK),
])
def test_parameter_validation(kw, code):
    assert wsg.check(_p(**kw), _v()) == code


def test_unknown_kernel():
    p = _p()
    p.kernel = 2
    assert wsg.check(p, _v()) == wsg.EINVAL


@pytest.mark.parametrize("support", [3, 5, 7, 9, 11, 13, 15])
def test_kb_default_beta_fits_fp32_mesh(support):
    """The default Kaiser-Bessel shape of every support passes the FP32 mesh's fit
    check (its per-tap polynomials within 2e-7 of the exact kernel)."""
    assert wsg.check(_p(kernel="kb", support=support, precision="f32_phase64"), _v()) == wsg.OK


def test_vis_validation():
    assert wsg.check(_p(), _v(n_rows=0)) == wsg.OK
    bad = _v()
    bad.desc.n_chan = 0
    assert wsg.check(_p(), bad) == wsg.EINVAL
    bad = _v()
    bad.desc.uvw = None
    assert wsg.check(_p(), bad) == wsg.EINVAL
    bad = _v()
    bad.desc.mem = 7
    assert wsg.check(_p(), bad) == wsg.EINVAL
    assert wsg.check(_p(), _v(freq_hz=np.array([-1.0]))) == wsg.EINVAL
    assert wsg.check(_p(per_channel=True), _v(n_chan=300)) == wsg.EUNSUPPORTED


def test_footprint_scales_with_mesh():
    f1 = wsg.footprint(_p(grid_n=256), _v(n_rows=1000))
    f2 = wsg.footprint(_p(grid_n=512), _v(n_rows=1000))
    # the plane stack dominates: 8 planes x N^2 x 16 bytes
    assert f1 >= 8 * 256 * 256 * 16
    assert 3.5 < f2 / f1 < 4.5
    f3 = wsg.footprint(_p(grid_n=256, precision="f32_phase64"), _v(n_rows=1000))
    assert f3 < f1
    assert wsg.n_images(_p(per_channel=True), _v(n_chan=5)) == 5
    assert wsg.n_images(_p(), _v(n_chan=5)) == 1


def test_footprint_shrinks_with_planes_per_pass():
    """A pass over a quarter of the planes holds a quarter of the w-stack."""
    full = wsg.footprint(_p(n_wplanes=8), _v(n_rows=1000))
    quarter = wsg.footprint(_p(n_wplanes=8, planes_per_pass=2), _v(n_rows=1000))
    stack = 8 * 256 * 256 * 16
    assert full - quarter >= 0.74 * stack


def test_strerror():
    assert wsg.strerror(wsg.OK) == "ok"
    assert "invalid" in wsg.strerror(wsg.EINVAL)
    assert "unknown" in wsg.strerror(-99)


def test_no_device_is_a_loud_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(wsg.WsgError) as e:
        wsg.Context(0)
    assert e.value.status in (wsg.EDEVICE, wsg.EINVAL)


def test_load_binds_to_torchs_hip_runtime():
    """Loading the library imports torch first, so both use one HIP runtime (a second
    runtime initialised first would leave torch without devices)."""
    import subprocess
    import sys
    code = ("import sys; from paper_2411_07321_amd import wsg; "
            "assert 'torch' not in sys.modules; wsg.load(); print('torch' in sys.modules)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "True"


def test_accum_footprint_and_rules():
    """The chunked accumulator holds the w-stack (N_w x N^2 cells) and needs a given w
    range; its footprint is known before any device work."""
    ok = _p(w_min=-5.0, w_max=5.0)
    f = wsg.accum_footprint(ok, 1)
    assert f >= 8 * 256 * 256 * 16
    assert wsg.accum_footprint(_p(w_min=-5.0, w_max=5.0, precision="f32_phase64"), 1) < f
    cube = wsg.accum_footprint(_p(w_min=-5.0, w_max=5.0, per_channel=True), 3)
    assert cube >= 3 * 8 * 256 * 256 * 16
    for bad, code in ((_p(), wsg.EINVAL), (_p(w_min=1.0, w_max=0.0), wsg.EINVAL)):
        with pytest.raises(wsg.WsgError) as e:
            wsg.accum_footprint(bad, 1)
        assert e.value.status == code
    with pytest.raises(wsg.WsgError) as e:
        wsg.accum_footprint(ok, 0)
    assert e.value.status == wsg.EINVAL


def test_record_offsets_guard():
    """Binning records are addressed with 32-bit offsets; a call whose worst case
    (4 records per visibility on each of the w_support planes) reaches 2^32 is refused
    before any device work, and the largest safe call is accepted."""
    largest = (2 ** 32 - 1) // (4 * 7)
    uvw = np.zeros((1, 3))
    vis = np.zeros((1, 1), np.complex128)

    def desc(n_rows):
        vb = wsg.make_vis(uvw, vis)
        vb.desc.n_rows = n_rows        # pointers are not dereferenced by the check
        return vb

    assert wsg.check(_p(w_support=7), desc(2 ** 29)) == wsg.EUNSUPPORTED
    assert wsg.check(_p(w_support=7), desc(largest + 1)) == wsg.EUNSUPPORTED
    assert wsg.check(_p(w_support=7), desc(largest)) == wsg.OK
    assert wsg.check(_p(w_support=3), desc(2 ** 29)) == wsg.EUNSUPPORTED
    assert wsg.check(_p(), desc(2 ** 29)) == wsg.OK           # 2^31 records at most
    assert wsg.check(_p(), desc(2 ** 29 + 1)) == wsg.EUNSUPPORTED


@pytest.mark.parametrize("prec,vdt,wdt,ok", [
    ("f64", np.complex128, np.float64, True),
    ("f64", np.complex64, np.float32, False),
    ("f64", np.complex128, np.float32, False),
    ("f32_phase64", np.complex64, np.float32, True),
    ("f32_phase64", np.complex128, np.float64, False),
    ("f32_phase32", np.complex64, np.float64, False),
])
def test_binding_checks_element_types(prec, vdt, wdt, ok):
    """The C ABI carries no sizes or element types: the binding refuses buffers whose
    element type or extent does not match the precision before calling it."""
    uvw = np.zeros((10, 3))
    vb = wsg.make_vis(uvw, np.zeros((10, 2), vdt), np.ones((10, 2), wdt))
    p = _p(precision=prec)
    if ok:
        wsg._check_inputs(p, vb)
    else:
        with pytest.raises(ValueError):
            wsg._check_inputs(p, vb)


def test_binding_checks_outputs():
    with pytest.raises(ValueError):
        wsg._check_out(np.zeros((1, 256, 256), np.float32), 256 * 256, ("f", 8), "the image")
    with pytest.raises(ValueError):
        wsg._check_out(np.zeros((1, 255, 256)), 256 * 256, ("f", 8), "the image")
    wsg._check_out(np.zeros((1, 256, 256)), 256 * 256, ("f", 8), "the image")
    with pytest.raises(ValueError):
        wsg._check_inputs(_p(), wsg.make_vis(np.zeros((10, 2)), np.zeros((10, 1), np.complex128)))
    with pytest.raises(ValueError):
        wsg._check_inputs(_p(), wsg.make_vis(np.zeros((10, 3)), np.zeros((10, 1), np.complex128),
                                             None, np.zeros((9, 1), np.uint8)))


def test_context_refuses_mismatched_buffers_before_the_call():
    """A float32 image or complex64 visibilities under the FP64 precision raise ValueError
    in the binding (no device is touched: the check comes first)."""
    ctx = wsg.Context.__new__(wsg.Context)      # no device needed for the check
    ctx._h = None
    vb = wsg.make_vis(np.zeros((10, 3)), np.zeros((10, 1), np.complex64))
    with pytest.raises(ValueError):
        ctx.image(_p(), vb, np.zeros((1, 256, 256)))
    vb = wsg.make_vis(np.zeros((10, 3)), np.zeros((10, 1), np.complex128))
    with pytest.raises(ValueError):
        ctx.image(_p(), vb, np.zeros((1, 256, 256), np.float32))
