"""Python binding of libswe.so (argument marshalling only).

Every step of the solver runs in the HIP library; this module converts
arguments (NumPy host arrays or torch CUDA tensors) to plain pointers and
sizes and raises on error codes.  It never falls back to another
implementation: without a built ``libswe.so`` it raises.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libswe.so"

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
BC_REFLECT, BC_FIXED = 0, 1
OPT_GRAPH_STEPS, OPT_TILE, OPT_COMPENSATED, OPT_FRICTION_IMPLICIT, OPT_LOCAL_SPLIT = 1, 2, 3, 4, 5
BATCH_PERSISTENT, BATCH_ROUNDS = 0, 1
PENDING, DONE, FAILED, CANCELLED = 0, 1, 2, 3
SUBMIT_MAX_DEPTH = 1
NOALLOC_MAX_BYTES = 64 << 20  # SWE_NOALLOC_MAX_BYTES: working array of swe_run_noalloc


class SweError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib().swe_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("g", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt_fixed", ctypes.c_double), ("h_dry", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("kappa_cap", ctypes.c_double),
                ("bc", ctypes.c_int32 * 4)]


class Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("step", ctypes.c_int64),
                ("mass", ctypes.c_double), ("clamp_mass", ctypes.c_double),
                ("dt", ctypes.c_double), ("alpha_x", ctypes.c_float),
                ("alpha_y", ctypes.c_float), ("runup", ctypes.c_float),
                ("status", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("error", ctypes.c_int32),
                ("t", ctypes.c_double), ("mass", ctypes.c_double),
                ("runup", ctypes.c_float), ("steps", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("active", ctypes.c_int64),
                ("mem_in_use", ctypes.c_size_t), ("mem_high_water", ctypes.c_size_t),
                ("mem_budget", ctypes.c_size_t), ("segments", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# exported symbols and their signatures (also checked by the CPU test-suite
# against include/swe.h)
_VP = ctypes.c_void_p
_FP = ctypes.c_void_p  # float* (host or device address)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)
_SIGS = {
    "swe_create": (ctypes.c_int, [ctypes.POINTER(Params), _FP, _FP, _FP, _FP, _FP, _VP, ctypes.POINTER(_VP)]),
    "swe_step": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "swe_read": (ctypes.c_int, [_VP, _FP, _FP, _FP, ctypes.POINTER(Stats)]),
    "swe_destroy": (None, [_VP]),
    "swe_set_option": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64]),
    "swe_state_device": (ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                        ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int64)]),
    "swe_time_stages": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "swe_set_outputs": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]),
    "swe_output_get": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, _FP, _FP, _FP,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "swe_track_max_depth": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "swe_read_max_depth": (ctypes.c_int, [_VP, _FP]),
    "swe_tile_info": (ctypes.c_int, [ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 4),
    "swe_tile_count": (ctypes.c_int, []),
    "swe_autotune": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "swe_batch_create": (ctypes.c_int, [_VP, ctypes.POINTER(_VP)]),
    "swe_batch_add": (ctypes.c_int, [_VP, ctypes.POINTER(Params), _FP, _FP, _FP, _FP, _FP,
                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "swe_batch_run": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "swe_batch_read": (ctypes.c_int, [_VP, ctypes.c_int32, _FP, _FP, _FP, ctypes.POINTER(Stats)]),
    "swe_batch_set_mode": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "swe_batch_set_tile": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "swe_batch_set_option": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64]),
    "swe_batch_track_max_depth": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "swe_batch_read_max_depth": (ctypes.c_int, [_VP, ctypes.c_int32, _FP]),
    "swe_batch_destroy": (None, [_VP]),
    "swe_server_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_size_t, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(_VP)]),
    "swe_submit": (ctypes.c_int, [_VP, ctypes.POINTER(Params), _FP, _FP, _FP, _FP, _FP,
                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "swe_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(Result), _FP, _FP, _FP]),
    "swe_submit_ex": (ctypes.c_int, [_VP, ctypes.POINTER(Params), _FP, _FP, _FP, _FP, _FP,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "swe_poll_ex": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(Result), _FP, _FP, _FP, _FP]),
    "swe_cancel": (ctypes.c_int, [_VP, ctypes.c_uint64]),
    "swe_server_set_mode": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "swe_server_set_option": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64]),
    "swe_server_get_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ServerStats)]),
    "swe_server_destroy": (None, [_VP]),
    "swe_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "swe_footprint": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "swe_set_allocator": (ctypes.c_int, [ALLOC_FN, RELEASE_FN, _VP]),
    "swe_run_noalloc": (ctypes.c_int, [ctypes.POINTER(Params), _FP, _FP, _FP, _FP, _FP, ctypes.c_int32,
                                       _VP, ctypes.POINTER(Stats)]),
}

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        # torch bundles its own HIP runtime under the same soname as the
        # system one; loading torch first makes libswe bind to that single
        # runtime, so torch streams and buffers can be handed to the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950) first")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def lib():
    return _lib()


def exported_names():
    return list(_SIGS)


def _check(rc: int, what: str):
    if rc != OK:
        raise SweError(rc, what)


def make_params(p) -> Params:
    """swe_params from an object or dict with the same field names."""
    get = (lambda k: p[k]) if isinstance(p, dict) else (lambda k: getattr(p, k))
    q = Params()
    q.nx, q.ny = int(get("nx")), int(get("ny"))
    q.dx, q.dy, q.g = float(get("dx")), float(get("dy")), float(get("g"))
    q.cfl, q.dt_fixed = float(get("cfl")), float(get("dt_fixed"))
    q.h_dry, q.weno_eps = float(get("h_dry")), float(get("weno_eps"))
    q.kappa_cap = float(get("kappa_cap"))
    bc = get("bc")
    for k in range(4):
        q.bc[k] = int(bc[k])
    return q


def _ptr(a, ny: int, nx: int, keep: list):
    """Address of a float32 [ny][nx] array: NumPy (host) or torch (host/device)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):  # torch tensor
        if a.dtype.__repr__() != "torch.float32" or tuple(a.shape) != (ny, nx) or not a.is_contiguous():
            raise ValueError("tensor must be contiguous float32 of shape (ny, nx)")
        keep.append(a)
        return a.data_ptr()
    arr = np.ascontiguousarray(a, dtype=np.float32)
    if arr.shape != (ny, nx):
        raise ValueError(f"array shape {arr.shape} != ({ny}, {nx})")
    keep.append(arr)
    return arr.ctypes.data


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def run_noalloc(params, b, n, h, hu, hv, nsteps: int, stream=None, stats: bool = True):
    """swe_run_noalloc: advance the device arrays (h, hu, hv) in place by
    nsteps steps, with no device allocation (the library's fixed working
    array).  Inputs are contiguous float32 (ny, nx) device tensors.  With
    stats the call waits and returns the diagnostics as a dict; without, it
    only enqueues kernels on `stream` and returns None."""
    q = make_params(params)
    keep = []
    ptrs = [_ptr(a, q.ny, q.nx, keep) for a in (b, n, h, hu, hv)]
    st = Stats() if stats else None
    rc = _lib().swe_run_noalloc(ctypes.byref(q), *ptrs, int(nsteps), _stream_handle(stream),
                                ctypes.byref(st) if st is not None else None)
    _check(rc, "swe_run_noalloc")
    return st.as_dict() if st is not None else None


class Solver:
    """A single scenario resident on the GPU."""

    def __init__(self, params, b, n, h, hu, hv, stream=None):
        self.params = make_params(params)
        ny, nx = self.params.ny, self.params.nx
        keep = []
        ptrs = [_ptr(a, ny, nx, keep) for a in (b, n, h, hu, hv)]
        out = _VP()
        rc = _lib().swe_create(ctypes.byref(self.params), *ptrs, _stream_handle(stream), ctypes.byref(out))
        _check(rc, "swe_create")
        self._ctx = out
        self.nx, self.ny = nx, ny

    @classmethod
    def from_scenario(cls, sc, stream=None):
        return cls(sc.params, *sc.fields(), stream=stream)

    def step(self, nsteps: int):
        _check(_lib().swe_step(self._ctx, int(nsteps)), "swe_step")

    def read(self, check: bool = True):
        h = np.empty((self.ny, self.nx), np.float32)
        hu = np.empty_like(h)
        hv = np.empty_like(h)
        st = Stats()
        rc = _lib().swe_read(self._ctx, h.ctypes.data, hu.ctypes.data, hv.ctypes.data, ctypes.byref(st))
        if check:
            _check(rc, "swe_read")
        return h, hu, hv, st.as_dict()

    def read_into(self, h=None, hu=None, hv=None):
        """Copy the state into caller arrays or tensors (host or device)."""
        keep = []
        p = [_ptr(a, self.ny, self.nx, keep) for a in (h, hu, hv)]
        st = Stats()
        _check(_lib().swe_read(self._ctx, *p, ctypes.byref(st)), "swe_read")
        return st.as_dict()

    def stats(self):
        st = Stats()
        rc = _lib().swe_read(self._ctx, None, None, None, ctypes.byref(st))
        return st.as_dict() | {"rc": rc}

    def time_stages(self, nsteps: int):
        """Mean device time [ms] of the stage-1, -2, -3 kernels over nsteps steps."""
        ms = (ctypes.c_double * 3)()
        _check(_lib().swe_time_stages(self._ctx, int(nsteps), ms), "swe_time_stages")
        return [ms[0], ms[1], ms[2]]

    def set_option(self, key: int, value: int):
        _check(_lib().swe_set_option(self._ctx, int(key), int(value)), "swe_set_option")

    def set_outputs(self, times):
        """Request snapshots at the given simulated times (see swe_set_outputs)."""
        t = np.ascontiguousarray(times, dtype=np.float64)
        arr = (ctypes.c_double * max(len(t), 1))(*t.tolist())
        _check(_lib().swe_set_outputs(self._ctx, arr, len(t)), "swe_set_outputs")

    def output(self, k: int, wait: bool = False):
        """Snapshot k as (h, hu, hv, t, step), or None while it is not available."""
        h = np.empty((self.ny, self.nx), np.float32)
        hu = np.empty_like(h)
        hv = np.empty_like(h)
        t = ctypes.c_double()
        st = ctypes.c_int64()
        rc = _lib().swe_output_get(self._ctx, int(k), int(bool(wait)), h.ctypes.data, hu.ctypes.data,
                                   hv.ctypes.data, ctypes.byref(t), ctypes.byref(st))
        if rc < 0:
            raise SweError(rc, "swe_output_get")
        return (h, hu, hv, t.value, st.value) if rc == 1 else None

    def output_ready(self, k: int, wait: bool = False) -> bool:
        """Whether snapshot k is on the host (copies nothing; moves the
        transfers of newly taken snapshots onto the copy stream)."""
        rc = _lib().swe_output_get(self._ctx, int(k), int(bool(wait)), None, None, None, None, None)
        if rc < 0:
            raise SweError(rc, "swe_output_get")
        return rc == 1

    def track_max_depth(self, enable: bool = True):
        _check(_lib().swe_track_max_depth(self._ctx, int(bool(enable))), "swe_track_max_depth")

    def max_depth(self):
        hm = np.empty((self.ny, self.nx), np.float32)
        _check(_lib().swe_read_max_depth(self._ctx, hm.ctypes.data), "swe_read_max_depth")
        return hm

    def close(self):
        if getattr(self, "_ctx", None):
            _lib().swe_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tile_variants():
    L = _lib()
    out = []
    for i in range(L.swe_tile_count()):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(L.swe_tile_info(i, *[ctypes.byref(x) for x in v]), "swe_tile_info")
        out.append(dict(index=i, tx=v[0].value, ty=v[1].value, r=v[2].value, threads=v[3].value))
    return out


def autotune(nx: int, ny: int, cache_path: str | None = None):
    best = ctypes.c_int32()
    ms = ctypes.c_double()
    cp = cache_path.encode() if cache_path else None
    _check(_lib().swe_autotune(int(nx), int(ny), cp, ctypes.byref(best), ctypes.byref(ms)), "swe_autotune")
    return best.value, ms.value


def footprint(nx: int, ny: int) -> int:
    return int(_lib().swe_footprint(int(nx), int(ny)))


# Every callback pair ever handed to the library: memory keeps the allocator
# that made it, so a replaced pair may still be called to release it.
_ALLOCATORS = []


def set_allocator(alloc=None, release=None):
    """Route the library's device allocations through ``alloc(nbytes, device)
    -> address`` and ``release(address, device)`` (swe_set_allocator); both
    None restores hipMalloc/hipFree.  An exception in ``alloc`` reads as out
    of memory."""
    if alloc is None and release is None:
        _check(_lib().swe_set_allocator(ALLOC_FN(), RELEASE_FN(), None), "swe_set_allocator")
        return

    def _alloc(nbytes, device, _user):
        try:
            return int(alloc(int(nbytes), int(device))) or None
        except Exception:
            return None

    def _release(ptr, device, _user):
        release(int(ptr), int(device))

    pair = (ALLOC_FN(_alloc) if alloc is not None else ALLOC_FN(),
            RELEASE_FN(_release) if release is not None else RELEASE_FN())
    _ALLOCATORS.append(pair)
    _check(_lib().swe_set_allocator(pair[0], pair[1], None), "swe_set_allocator")


def use_torch_allocator(enable: bool = True):
    """Allocate the library's device memory from torch's caching allocator
    (counted by torch.cuda.memory_allocated), or go back to hipMalloc."""
    if not enable:
        set_allocator(None, None)
        return
    import torch

    set_allocator(lambda n, dev: torch.cuda.caching_allocator_alloc(n, dev),
                  lambda p, dev: torch.cuda.caching_allocator_delete(p))


class Batch:
    """Many scenarios advanced together: by default one launch per stage
    round over every active scenario, captured as one hipGraph per run;
    set_mode selects the persistent launch instead."""

    def __init__(self, stream=None):
        out = _VP()
        _check(_lib().swe_batch_create(_stream_handle(stream), ctypes.byref(out)), "swe_batch_create")
        self._bt = out
        self._shapes = []

    def add(self, params, b, n, h, hu, hv, nsteps: int) -> int:
        p = make_params(params)
        keep = []
        ptrs = [_ptr(a, p.ny, p.nx, keep) for a in (b, n, h, hu, hv)]
        idx = ctypes.c_int32()
        _check(_lib().swe_batch_add(self._bt, ctypes.byref(p), *ptrs, int(nsteps), ctypes.byref(idx)),
               "swe_batch_add")
        self._shapes.append((p.ny, p.nx))
        return idx.value

    def add_scenario(self, sc, nsteps: int | None = None) -> int:
        return self.add(sc.params, *sc.fields(), sc.nsteps if nsteps is None else nsteps)

    def set_mode(self, mode: int, use_graph: bool = False):
        _check(_lib().swe_batch_set_mode(self._bt, int(mode), int(bool(use_graph))), "swe_batch_set_mode")

    def set_tile(self, tile: int):
        _check(_lib().swe_batch_set_tile(self._bt, int(tile)), "swe_batch_set_tile")

    def set_option(self, key: int, value: int):
        _check(_lib().swe_batch_set_option(self._bt, int(key), int(value)), "swe_batch_set_option")

    def run(self, max_steps: int = -1):
        _check(_lib().swe_batch_run(self._bt, int(max_steps)), "swe_batch_run")

    def read(self, index: int, check: bool = True):
        ny, nx = self._shapes[index]
        h = np.empty((ny, nx), np.float32)
        hu = np.empty_like(h)
        hv = np.empty_like(h)
        st = Stats()
        rc = _lib().swe_batch_read(self._bt, int(index), h.ctypes.data, hu.ctypes.data, hv.ctypes.data,
                                   ctypes.byref(st))
        if check:
            _check(rc, "swe_batch_read")
        return h, hu, hv, st.as_dict()

    def stats(self, index: int):
        st = Stats()
        rc = _lib().swe_batch_read(self._bt, int(index), None, None, None, ctypes.byref(st))
        return st.as_dict() | {"rc": rc}

    def track_max_depth(self, index: int, enable: bool = True):
        _check(_lib().swe_batch_track_max_depth(self._bt, int(index), int(bool(enable))),
               "swe_batch_track_max_depth")

    def max_depth(self, index: int):
        ny, nx = self._shapes[index]
        hm = np.empty((ny, nx), np.float32)
        _check(_lib().swe_batch_read_max_depth(self._bt, int(index), hm.ctypes.data), "swe_batch_read_max_depth")
        return hm

    def close(self):
        if getattr(self, "_bt", None):
            _lib().swe_batch_destroy(self._bt)
            self._bt = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server: requests are admitted by memory footprint."""

    def __init__(self, device: int = 0, mem_budget: int = 0, max_slots: int = 256,
                 segment_steps: int = 100):
        out = _VP()
        _check(_lib().swe_server_create(int(device), int(mem_budget), int(max_slots),
                                        int(segment_steps), ctypes.byref(out)), "swe_server_create")
        self._sv = out
        self._shapes = {}

    def submit(self, params, b, n, h, hu, hv, nsteps: int, max_depth: bool = False) -> int:
        """Queue a request; max_depth keeps its maximum-depth map (swe_submit_ex)."""
        p = make_params(params)
        keep = []
        ptrs = [_ptr(a, p.ny, p.nx, keep) for a in (b, n, h, hu, hv)]
        t = ctypes.c_uint64()
        flags = SUBMIT_MAX_DEPTH if max_depth else 0
        _check(_lib().swe_submit_ex(self._sv, ctypes.byref(p), *ptrs, int(nsteps), flags, ctypes.byref(t)),
               "swe_submit_ex")
        self._shapes[t.value] = (p.ny, p.nx)
        return t.value

    def submit_scenario(self, sc, nsteps: int | None = None, max_depth: bool = False) -> int:
        return self.submit(sc.params, *sc.fields(), sc.nsteps if nsteps is None else nsteps,
                           max_depth=max_depth)

    def poll(self, ticket: int, want_state: bool = True, want_max_depth: bool = False):
        """-> (result dict, (h, hu, hv) or None); with want_max_depth the
        tuple also holds the maximum-depth map (swe_poll_ex)."""
        r = Result()
        ny, nx = self._shapes.get(ticket, (1, 1))
        arrs = [np.empty((ny, nx), np.float32) for _ in range(3)] if want_state else [None] * 3
        hmax = np.empty((ny, nx), np.float32) if want_max_depth else None
        ptrs = [a.ctypes.data if a is not None else None for a in arrs]
        rc = _lib().swe_poll_ex(self._sv, int(ticket), ctypes.byref(r), *ptrs,
                                hmax.ctypes.data if hmax is not None else None)
        _check(rc, "swe_poll_ex")
        d = r.as_dict()
        if d["status"] != PENDING:
            self._shapes.pop(ticket, None)
        state = None
        if d["status"] == DONE and (want_state or want_max_depth):
            state = (tuple(arrs) if want_state else ()) + ((hmax,) if want_max_depth else ())
        return d, state

    def set_mode(self, mode: int):
        _check(_lib().swe_server_set_mode(self._sv, int(mode)), "swe_server_set_mode")

    def set_option(self, key: int, value: int):
        _check(_lib().swe_server_set_option(self._sv, int(key), int(value)), "swe_server_set_option")

    def cancel(self, ticket: int):
        _check(_lib().swe_cancel(self._sv, int(ticket)), "swe_cancel")

    def stats(self):
        st = ServerStats()
        _check(_lib().swe_server_get_stats(self._sv, ctypes.byref(st)), "swe_server_get_stats")
        return st.as_dict()

    def close(self):
        if getattr(self, "_sv", None):
            _lib().swe_server_destroy(self._sv)
            self._sv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
