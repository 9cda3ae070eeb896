"""The C ABI: every function declared in include/swe.h is exported by
libswe.so and declared by the Python binding; host-only calls work without a
GPU.  The FP64 checker's library exports its entry points too."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_12010_amd import swe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swe.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = header_functions()
    for required in ("swe_create", "swe_step", "swe_read", "swe_destroy", "swe_submit", "swe_poll",
                     "swe_batch_create", "swe_batch_add", "swe_batch_run", "swe_server_create",
                     "swe_autotune"):
        assert required in names


def test_library_exports_every_header_function():
    if not swe.LIB_PATH.exists():
        pytest.fail("libswe.so is not built")
    L = ctypes.CDLL(str(swe.LIB_PATH))
    missing = [n for n in header_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_declares_every_header_function():
    missing = set(header_functions()) - set(swe.exported_names())
    assert not missing, missing


def test_host_only_calls():
    L = swe.lib()
    assert L.swe_strerror(swe.ENONFINITE).decode().startswith("non-finite")
    assert L.swe_strerror(12345) == b"unknown error"
    # 11 planes of 4096 floats x 4096 rows plus ghosts and scalars
    fp = swe.footprint(4096, 4096)
    assert 11 * 4096 * 4096 * 4 <= fp < 11 * 4096 * 4096 * 4 + 2 ** 20
    assert swe.footprint(0, 5) == 0
    assert L.swe_tile_count() >= 4
    v = swe.tile_variants()
    assert all(t["tx"] * t["ty"] // t["r"] == t["threads"] and t["threads"] % 64 == 0 for t in v)
    # null handles are rejected without touching the GPU
    assert L.swe_step(None, 1) == swe.EINVAL
    assert L.swe_read(None, None, None, None, None) == swe.EINVAL
    L.swe_destroy(None)
    L.swe_batch_destroy(None)
    L.swe_server_destroy(None)
    assert L.swe_set_outputs(None, None, 0) == swe.EINVAL
    assert L.swe_output_get(None, 0, 0, None, None, None, None, None) == swe.EINVAL
    assert L.swe_track_max_depth(None, 1) == swe.EINVAL
    assert L.swe_read_max_depth(None, None) == swe.EINVAL
    assert L.swe_batch_track_max_depth(None, 0, 1) == swe.EINVAL
    assert L.swe_batch_read_max_depth(None, 0, None) == swe.EINVAL
    assert L.swe_batch_set_option(None, swe.OPT_FRICTION_IMPLICIT, 1) == swe.EINVAL
    assert L.swe_server_set_option(None, swe.OPT_FRICTION_IMPLICIT, 1) == swe.EINVAL
    # allocator hook: both callbacks or neither
    assert L.swe_set_allocator(swe.ALLOC_FN(lambda n, d, u: None), swe.RELEASE_FN(), None) == swe.EINVAL
    assert L.swe_set_allocator(swe.ALLOC_FN(), swe.RELEASE_FN(lambda p, d, u: None), None) == swe.EINVAL
    assert L.swe_set_allocator(swe.ALLOC_FN(), swe.RELEASE_FN(), None) == swe.OK
    with pytest.raises(swe.SweError):
        swe.set_allocator(lambda n, d: 0, None)
    swe.set_allocator(None, None)


def test_create_rejects_bad_sizes_before_reading_fields():
    # parameters are validated before any field is read or any device call
    # is made: a 1-element dummy array stands for every field
    import ctypes
    dummy = np.zeros(1, np.float32)
    ptr = dummy.ctypes.data
    out = ctypes.c_void_p()

    def create(**kw):
        base = dict(nx=8, ny=8, dx=1.0, dy=1.0, g=9.81, cfl=0.4, dt_fixed=0.0, h_dry=1e-3,
                    weno_eps=1e-6, kappa_cap=0.0, bc=(0, 0, 0, 0))
        base.update(kw)
        p = swe.make_params(base)
        return swe.lib().swe_create(ctypes.byref(p), ptr, ptr, ptr, ptr, ptr, None, ctypes.byref(out))

    assert create(nx=2) == swe.EINVAL and create(ny=0) == swe.EINVAL
    # planes of 2^30 elements or more (rows padded to 64) are refused
    assert create(nx=32768, ny=32768) == swe.EINVAL
    assert create(nx=32705, ny=32768) == swe.EINVAL   # pitch 32768
    assert create(nx=3, ny=(1 << 30) // 64) == swe.EINVAL  # pitch 64
    assert create(dx=0.0) == swe.EINVAL and create(dy=-1.0) == swe.EINVAL
    assert create(g=float("nan")) == swe.EINVAL
    assert create(cfl=0.0, dt_fixed=0.0) == swe.EINVAL
    assert create(weno_eps=0.0) == swe.EINVAL
    assert create(bc=(0, 0, 0, 7)) == swe.EINVAL
    assert out.value is None


def test_params_struct_layout_matches_header():
    # int32 nx, ny; 8 doubles; int32 bc[4]  -> 4 + 4 + 64 + 16 = 88 bytes
    assert ctypes.sizeof(swe.Params) == 88
    # t, step, mass, clamp_mass, dt (8 bytes each); alpha_x, alpha_y, runup, status
    assert ctypes.sizeof(swe.Stats) == 8 * 5 + 4 * 4


def test_checker_library_exports():
    import oracle
    L = oracle.lib()
    for n in ("oracle_create", "oracle_step", "oracle_read", "oracle_scalars", "oracle_rhs",
              "oracle_weno5", "oracle_destroy"):
        assert hasattr(L, n)


def test_calibration_library_exports_and_rejects_bad_arguments():
    # the benchmark's vector-ALU calibration: a library of its own, outside
    # the solver's ABI; argument checks run before any GPU call
    path = swe.LIB_PATH.parent / "libswe_calib.so"
    if not path.exists():
        pytest.fail("libswe_calib.so is not built")
    L = ctypes.CDLL(str(path))
    f = L.swe_calib_valu
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                  ctypes.POINTER(ctypes.c_double)]
    f.restype = ctypes.c_int
    ms, wi = ctypes.c_float(), ctypes.c_double()
    assert f(3, 2, 10, ctypes.byref(ms), ctypes.byref(wi)) == -1
    assert f(0, 3, 10, ctypes.byref(ms), ctypes.byref(wi)) == -1
    assert f(0, 2, 0, ctypes.byref(ms), ctypes.byref(wi)) == -1
    assert f(0, 2, 10, None, ctypes.byref(wi)) == -1
