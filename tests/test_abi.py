"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before touching a GPU (CPU only)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2203_02300_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dco_stereo.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dco_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2203_02300_amd import build
        build.build()
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    syms = declared_symbols()
    assert len(syms) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (dco_\w+)", out))
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    assert set(syms) == set(_lib.EXPORTS)


def test_default_params(L):
    p = _lib.Params()
    assert L.dco_default_params(C.byref(p)) == 0
    assert (p.census_w, p.census_h, p.arm_L1, p.arm_tau1) == (9, 7, 17, 20)
    assert (p.lambda_ad, p.lambda_census, p.gamma_L) == (10.0, 40.0, 1.0)
    assert abs(p.eps - 0.8) < 1e-7 and p.agg_iters == 2 and p.subpixel == 1
    assert p.vote_iters == 0
    assert L.dco_default_params(None) == -1


def create(L, W, H, D, **kw):
    p = _lib.Params()
    L.dco_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    h = C.c_void_p()
    st = L.dco_stereo_create(C.byref(h), W, H, D, C.byref(p), None)
    return st, h


@pytest.mark.parametrize("W,H,D", [(64, 48, 64), (64, 48, 0), (8, 48, 4), (64, 6, 4),
                                   (20000, 8, 4), (16384, 16384, 16),
                                   # W * H above 2^27 with W * H * D < 2^31
                                   (16384, 16384, 1), (16384, 8193, 1)])
def test_bad_shapes_rejected(L, W, H, D):
    st, h = create(L, W, H, D)
    assert st == -2 and not h.value
    assert b"shape" in L.dco_last_error()


@pytest.mark.parametrize("kw", [dict(census_w=8), dict(census_w=11), dict(census_h=0),
                                dict(arm_L1=18), dict(arm_L1=-1), dict(arm_tau1=0),
                                dict(lambda_ad=0.0), dict(lambda_census=-1.0),
                                dict(eps=float("nan")), dict(agg_iters=3),
                                dict(lr_max_diff=-1), dict(subpixel=2), dict(vote_iters=-1),
                                dict(vote_iters=65)])
def test_bad_params_rejected(L, kw):
    st, h = create(L, 64, 48, 16, **kw)
    assert st == -1 and not h.value


def test_null_arguments_rejected(L):
    assert L.dco_stereo_create(None, 64, 48, 16, None, None) == -1
    assert L.dco_census(None, None, None, None) == -1
    assert L.dco_cost_volume(None, 0, None, None, None, None, None, None) == -1
    assert L.dco_aggregate(None, None, None, None) == -1
    assert L.dco_wta_lrcheck(None, None, None, None, None, None, None) == -1
    assert L.dco_stereo_match(None, None, None, None, None) == -1
    assert L.dco_vote_refine(None, None, None, None, None, 1, None, None, None) == -1
    assert L.dco_stereo_match_half(None, None, None, 2, 2, 1.0, None, None, None) == -1
    assert L.dco_densify_run(None, None, None, None, None, None, None) == -1
    assert L.dco_densify_create(None, 4, 4, None, None) == -1
    assert L.dco_contour_create(None, 4, 4, None, None) == -1
    assert L.dco_contour_run(None, None, None, None, None, None, None) == -1
    L.dco_contour_destroy(None)
    L.dco_densify_destroy(None)


def test_densify_defaults_and_bad_params(L):
    p = _lib.DensifyParams()
    assert L.dco_densify_default_params(C.byref(p)) == 0
    assert abs(p.lambda_d - 0.8) < 1e-7 and abs(p.lambda_s - 1.2) < 1e-7
    assert abs(p.lambda_s2 - 0.02) < 1e-9
    assert p.iters_per_launch % 2 == 0 and p.max_iters > 0
    for k, v in (("lambda_s", -1.0), ("tol", float("nan")), ("iters_per_launch", 3),
                 ("max_iters", -1)):
        q = _lib.DensifyParams()
        L.dco_densify_default_params(C.byref(q))
        setattr(q, k, v)
        h = C.c_void_p()
        assert L.dco_densify_create(C.byref(h), 8, 8, C.byref(q), None) == -1 and not h.value
    h = C.c_void_p()
    assert L.dco_densify_create(C.byref(h), 0, 8, None, None) == -2
    assert L.dco_densify_create(C.byref(h), 4096, 2049, None, None) == -2 and not h.value
    assert L.dco_stereo_set_stream(None, None) == -1
    L.dco_stereo_destroy(None)


def test_contour_defaults_and_bad_params(L):
    p = _lib.ContourParams()
    assert L.dco_contour_default_params(C.byref(p)) == 0
    assert abs(p.T_high - 0.06) < 1e-8 and abs(p.T_low - 0.03) < 1e-8
    assert abs(p.T_depth - 0.03) < 1e-8 and p.box_radius == 2
    for k, v in (("T_high", -1.0), ("T_low", float("inf")), ("box_radius", 17),
                 ("box_radius", -1)):
        q = _lib.ContourParams()
        L.dco_contour_default_params(C.byref(q))
        setattr(q, k, v)
        h = C.c_void_p()
        assert L.dco_contour_create(C.byref(h), 8, 8, C.byref(q), None) == -1 and not h.value
    h = C.c_void_p()
    assert L.dco_contour_create(C.byref(h), 1, 8, None, None) == -2


def test_status_strings(L):
    assert L.dco_status_string(0) == b"ok"
    assert L.dco_status_string(-4) == b"out of device memory"
    assert L.dco_status_string(99) == b"unknown status"


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.lib()


def test_noalloc_match_checks_arguments_before_any_launch(L):
    """dco_stereo_match_noalloc rejects bad arguments and shapes whose buffers
    do not fit its static scratch on the host, before touching a GPU."""
    p = _lib.Params()
    L.dco_default_params(C.byref(p))
    buf = C.create_string_buffer(16)
    ptr = C.cast(buf, C.c_void_p)
    assert L.dco_stereo_match_noalloc(64, 48, 16, C.byref(p), None, None, ptr, ptr, ptr) == -1
    assert L.dco_stereo_match_noalloc(64, 48, 64, C.byref(p), None, ptr, ptr, ptr, ptr) == -2
    # 1280 x 720 with D = 128 needs about 1 GB: more than the 160 MiB array
    assert L.dco_stereo_match_noalloc(1280, 720, 128, C.byref(p), None, ptr, ptr, ptr, ptr) == -2
    assert b"static scratch" in L.dco_last_error()
    bad = _lib.Params()
    L.dco_default_params(C.byref(bad))
    bad.agg_iters = 3
    assert L.dco_stereo_match_noalloc(64, 48, 16, C.byref(bad), None, ptr, ptr, ptr, ptr) == -1
