"""ctypes binding of libfram.so with the C ABI's names (include/fram.h).

Module-level functions carry the exact C names and take a context handle;
the ``Context`` class wraps them with numpy in/out.  Device-memory variants
take raw device pointers (e.g. ``tensor.data_ptr()`` of a torch tensor) and a
HIP stream handle; torch is only a source of device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
import pathlib

import numpy as np

FRAM_OK, FRAM_EINVAL, FRAM_ENOMEM, FRAM_EDEVICE, FRAM_ENUMERIC, FRAM_EBUSY = range(6)
FRAM_FP32, FRAM_BF16, FRAM_FP16 = 0, 1, 2
PRECISIONS = {"fp32": FRAM_FP32, "bf16": FRAM_BF16, "fp16": FRAM_FP16}

_HERE = pathlib.Path(__file__).resolve().parent


def library_path() -> pathlib.Path:
    return pathlib.Path(os.environ.get("FRAM_LIBRARY", _HERE / "libfram.so"))


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int),
        ("sdsn_passes", ctypes.c_int),
        ("sdsn_passes_last", ctypes.c_int),
        ("sdsn_passes_max", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("sdsn_capped", ctypes.c_int),
        ("lap_paths", ctypes.c_int),
        ("gemm_tile", ctypes.c_int),
        ("delta", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("ms_total", ctypes.c_double),
        ("gemm_launches", ctypes.c_int),
        ("sdsn_launches", ctypes.c_int),
        ("ms_gemm", ctypes.c_double),
        ("ms_sdsn", ctypes.c_double),
        ("ms_stats", ctypes.c_double),
        ("ms_update", ctypes.c_double),
        ("stalled", ctypes.c_int),
        ("ms_discretize", ctypes.c_double),
        ("sdsn_onchip", ctypes.c_int),
        ("sdsn_fallbacks", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Options(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int),
        ("alpha", ctypes.c_double),
        ("gamma_tol", ctypes.c_double),
        ("sdsn_max", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("profile", ctypes.c_int),
        ("stable_iters", ctypes.c_int),
        ("sdsn_mode", ctypes.c_int),
        ("stall_iters", ctypes.c_int),
        ("stall_delta", ctypes.c_double),
        ("variant", ctypes.c_int),
        ("dsn_iters", ctypes.c_int),
        ("many_workers", ctypes.c_int),
        ("N0", ctypes.c_void_p),
        ("N_out", ctypes.c_void_p),
        ("onchip_roll_us", ctypes.c_int),
        ("onchip_barrier_us", ctypes.c_int),
    ]


class FramError(RuntimeError):
    def __init__(self, status: int, where: str, message: str = ""):
        self.status = status
        super().__init__(f"{where}: status {status} ({message})")


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "fram_default_options": (None, [_P]),
    "fram_struct_sizes": (None, [_P, _P]),
    "fram_create": (_I, [ctypes.POINTER(_P), _I, ctypes.c_size_t]),
    "fram_destroy": (None, [_P]),
    "fram_workspace_bytes": (ctypes.c_size_t, [_I, _I, _I]),
    "fram_set_tile_table": (_I, [_P, _P, _I]),
    "fram_auto_tile": (_I, [_I]),
    "fram_solve": (_I, [_P, _P, _P, _I, _D, _I, _D, _P, _P]),
    "fram_solve_ex": (_I, [_P, _P, _P, _I, _D, _I, _D, _P, _P, _P, _P]),
    "fram_solve_dev": (_I, [_P, _P, _P, _I, _D, _I, _D, _P, _P, _P, _P, _P]),
    "fram_solve_attr_ex": (_I, [_P, _P, _P, _P, _I, _D, _D, _I, _D, _P, _P, _P, _P]),
    "fram_solve_attr_dev": (_I, [_P, _P, _P, _P, _I, _D, _D, _I, _D, _P, _P, _P, _P, _P]),
    "fram_sdsn_project": (_I, [_P, _P, _I, _D, _P]),
    "fram_sdsn_project_ex": (_I, [_P, _P, _I, _D, _P, _P, _P]),
    "fram_sdsn_project_dev": (_I, [_P, _P, _I, _I, _D, _P, _P, _I, _P, _P]),
    "fram_sdsn_project_noalloc": (_I, [_P, _I, _I, _D, _P, _P, _I, _P, _P]),
    "fram_gradient": (_I, [_P, _P, _P, _P, _I, _I, _P]),
    "fram_assign": (_I, [_P, _P, _I, _P]),
    "fram_assign_dev": (_I, [_P, _P, _I, _I, _P, _P]),
    "fram_solve_many": (_I, [_P, _I, _P, _P, _P, _D, _I, _D, _P, _P]),
    "fram_solve_many_ex": (_I, [_P, _I, _P, _P, _P, _D, _I, _D, _P, _P, _P, _P]),
    "fram_resident_bytes": (ctypes.c_size_t, [_P]),
    "fram_trim": (_I, [_P]),
    "fram_last_stats": (_I, [_P, _P]),
    "fram_status_str": (ctypes.c_char_p, [_I]),
    "fram_last_error": (ctypes.c_char_p, [_P]),
}


def load_library():
    """Load libfram.so; raises if it is missing (build with
    ``python -m paper_2508_00887_amd.build``).  There is no fallback.

    torch is imported first when available: it carries its own HIP runtime
    (libamdhip64.so.7), and libfram must bind to that same runtime so that
    device pointers and streams from torch are valid in the library (two HIP
    runtimes in one process do not share devices)."""
    global _lib
    if _lib is not None:
        return _lib
    # Concurrent solves (fram_solve_many's workers, the server's slots) each
    # use a stream; HIP maps the streams of a process onto GPU_MAX_HW_QUEUES
    # hardware queues (4 by default), and kernels of streams that share a
    # queue run one after the other.  16 queues measured 1.9x the throughput
    # of 4 on 512 small pairs.  Read when HIP starts, so set before torch or
    # the library touch the device; a value the caller set is kept.
    os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    path = library_path()
    if not path.exists():
        raise ImportError(f"{path} not found: build it with `python -m paper_2508_00887_amd.build`")
    lib = ctypes.CDLL(str(path))
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    ob, sb = ctypes.c_size_t(), ctypes.c_size_t()
    lib.fram_struct_sizes(ctypes.byref(ob), ctypes.byref(sb))
    if (ob.value, sb.value) != (ctypes.sizeof(Options), ctypes.sizeof(Stats)):
        raise ImportError(f"{path}: fram_options / fram_stats are {ob.value} / {sb.value} bytes, "
                          f"the binding expects {ctypes.sizeof(Options)} / {ctypes.sizeof(Stats)}")
    _lib = lib
    cache = os.environ.get("FRAM_TUNE_CACHE")
    if cache:
        from . import tune
        tune.apply(tune.load(cache))
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------- C names
def fram_default_options() -> Options:
    o = Options()
    load_library().fram_default_options(ctypes.byref(o))
    return o


def fram_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = _P()
    st = load_library().fram_create(ctypes.byref(h), device, hbm_budget_bytes)
    if st != FRAM_OK:
        raise FramError(st, "fram_create")
    return h.value


def fram_destroy(ctx: int) -> None:
    load_library().fram_destroy(ctx)


def fram_workspace_bytes(n: int, prec: int = FRAM_FP32, tile: int = 0) -> int:
    return int(load_library().fram_workspace_bytes(n, prec, tile))


def fram_set_tile_table(n_max, tile) -> None:
    """fram_set_tile_table: bucket k covers n_max[k-1] < n <= n_max[k] and
    selects tile[k]; empty sequences clear the table."""
    n_max = np.ascontiguousarray(n_max, dtype=np.int32)
    tile = np.ascontiguousarray(tile, dtype=np.int32)
    if n_max.shape != tile.shape or n_max.ndim != 1:
        raise ValueError("n_max and tile must be 1-D sequences of the same length")
    st = load_library().fram_set_tile_table(_ptr(n_max) if n_max.size else None,
                                            _ptr(tile) if tile.size else None, int(n_max.size))
    if st != FRAM_OK:
        raise FramError(st, "fram_set_tile_table")


def fram_auto_tile(n: int) -> int:
    return int(load_library().fram_auto_tile(n))


def fram_status_str(status: int) -> str:
    return load_library().fram_status_str(status).decode()


def fram_last_error(ctx: int) -> str:
    return load_library().fram_last_error(ctx).decode()


def fram_sdsn_project_noalloc(dK: int, ldk: int, n: int, dX: int, ldx: int, theta=2.0,
                              gamma_tol=1e-6, sdsn_max=1000, tile=0, stream=0) -> dict:
    """fram_sdsn_project_noalloc on device pointers (no context); returns the
    stats dict."""
    stats = Stats()
    o = _options("fp32", 0.95, gamma_tol, sdsn_max, tile, False, "stream")
    st = load_library().fram_sdsn_project_noalloc(dK, ldk, n, theta, ctypes.byref(o), dX, ldx,
                                                  ctypes.byref(stats), stream or None)
    if st != FRAM_OK:
        raise FramError(st, "fram_sdsn_project_noalloc", fram_status_str(st))
    return stats.as_dict()


def _check(ctx: int, st: int, where: str):
    if st != FRAM_OK:
        raise FramError(st, where, f"{fram_status_str(st)}; {fram_last_error(ctx)}")


SDSN_MODES = {"auto": 0, "stream": 1, "onchip": 2}
VARIANTS = {"fram": 0, "dspfp": 1}


def _options(prec="fp32", alpha=0.95, gamma_tol=1e-6, sdsn_max=1000, tile=0,
             profile=False, sdsn_mode="auto", stable_iters=0, stall_iters=0,
             stall_delta=1e-3, variant="fram", dsn_iters=30, many_workers=16,
             onchip_roll_us=0, onchip_barrier_us=0) -> Options:
    o = Options()
    o.many_workers = int(many_workers)
    o.onchip_roll_us = int(onchip_roll_us)
    o.onchip_barrier_us = int(onchip_barrier_us)
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.dsn_iters = int(dsn_iters)
    o.stable_iters = int(stable_iters)
    o.stall_iters = int(stall_iters)
    o.stall_delta = float(stall_delta)
    # profile: False/0 off, True/1 each launch timed alone, 2 timed without
    # serialising the launches.
    o.profile = int(profile)
    o.sdsn_mode = SDSN_MODES[sdsn_mode] if isinstance(sdsn_mode, str) else int(sdsn_mode)
    o.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    o.alpha = alpha
    o.gamma_tol = gamma_tol
    o.sdsn_max = sdsn_max
    o.tile = tile
    return o


class Context:
    """One FRAM context (device, stream, workspace).  Not thread-safe."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.lib = load_library()
        self.handle = fram_create(device, hbm_budget_bytes)

    def close(self):
        if self.handle:
            fram_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ FRAM
    def solve(self, A, B, theta=2.0, iters=100, tol=0.0, K=None, node_weight=1.0, N0=None,
              N_out=None, **opts):
        """fram_solve_ex (or fram_solve_attr_ex when node similarities K are
        given) on host arrays; returns (perm, objective, stats dict).  N0: warm
        start (n x n); N_out: an n x n float32 C-contiguous array that receives
        the final iterate."""
        A, B = _f64(A), _f64(B)
        n = A.shape[0]
        perm = np.empty(n, dtype=np.int32)
        obj = ctypes.c_double()
        stats = Stats()
        o = _options(**opts)
        if N0 is not None:
            N0 = _f32(N0)
            o.N0 = _ptr(N0)
        if N_out is not None:
            if N_out.dtype != np.float32 or not N_out.flags.c_contiguous or N_out.shape != (n, n):
                raise ValueError("N_out must be a C-contiguous n x n float32 array")
            o.N_out = _ptr(N_out)
        if K is None:
            st = self.lib.fram_solve_ex(self.handle, _ptr(A), _ptr(B), n, theta, iters, tol,
                                        ctypes.byref(o), _ptr(perm), ctypes.byref(obj),
                                        ctypes.byref(stats))
            _check(self.handle, st, "fram_solve_ex")
        else:
            K = _f64(K)
            st = self.lib.fram_solve_attr_ex(self.handle, _ptr(A), _ptr(B), _ptr(K), n,
                                             node_weight, theta, iters, tol, ctypes.byref(o),
                                             _ptr(perm), ctypes.byref(obj), ctypes.byref(stats))
            _check(self.handle, st, "fram_solve_attr_ex")
        return perm.astype(np.int64), obj.value, stats.as_dict()

    def solve_dev(self, dA: int, dB: int, n: int, theta=2.0, iters=100, tol=0.0, stream=0,
                  dK: int = 0, node_weight=1.0, dN0: int = 0, dN_out: int = 0, **opts):
        """fram_solve_dev (fram_solve_attr_dev with dK) on device pointers
        (n*n doubles each; dN0 / dN_out: n*n floats, or 0)."""
        perm = np.empty(n, dtype=np.int32)
        obj = ctypes.c_double()
        stats = Stats()
        o = _options(**opts)
        o.N0 = dN0 or None
        o.N_out = dN_out or None
        if not dK:
            st = self.lib.fram_solve_dev(self.handle, dA, dB, n, theta, iters, tol,
                                         ctypes.byref(o), _ptr(perm), ctypes.byref(obj),
                                         ctypes.byref(stats), stream or None)
            _check(self.handle, st, "fram_solve_dev")
        else:
            st = self.lib.fram_solve_attr_dev(self.handle, dA, dB, dK, n, node_weight, theta,
                                              iters, tol, ctypes.byref(o), _ptr(perm),
                                              ctypes.byref(obj), ctypes.byref(stats),
                                              stream or None)
            _check(self.handle, st, "fram_solve_attr_dev")
        return perm.astype(np.int64), obj.value, stats.as_dict()

    def sdsn_project(self, K, theta=2.0, gamma_tol=1e-6, sdsn_max=1000, tile=0,
                     sdsn_mode="auto", profile=False, onchip_roll_us=0, onchip_barrier_us=0):
        """fram_sdsn_project_ex on a host matrix; returns (X, stats dict)."""
        K = _f32(K)
        n = K.shape[0]
        X = np.empty((n, n), dtype=np.float32)
        stats = Stats()
        o = _options("fp32", 0.95, gamma_tol, sdsn_max, tile, profile, sdsn_mode,
                     onchip_roll_us=onchip_roll_us, onchip_barrier_us=onchip_barrier_us)
        st = self.lib.fram_sdsn_project_ex(self.handle, _ptr(K), n, theta, ctypes.byref(o),
                                           _ptr(X), ctypes.byref(stats))
        _check(self.handle, st, "fram_sdsn_project_ex")
        return X, stats.as_dict()

    def sdsn_project_dev(self, dK: int, ldk: int, n: int, dX: int, ldx: int, theta=2.0,
                         gamma_tol=1e-6, sdsn_max=1000, tile=0, stream=0, sdsn_mode="auto",
                         profile=False):
        stats = Stats()
        o = _options("fp32", 0.95, gamma_tol, sdsn_max, tile, profile, sdsn_mode)
        st = self.lib.fram_sdsn_project_dev(self.handle, dK, ldk, n, theta, ctypes.byref(o), dX,
                                            ldx, ctypes.byref(stats), stream or None)
        _check(self.handle, st, "fram_sdsn_project_dev")
        return stats.as_dict()

    def gradient(self, A, N, B, prec="fp32"):
        """fram_gradient: X = A N B with GEMM inputs rounded to `prec`."""
        A, N, B = _f32(A), _f32(N), _f32(B)
        n = A.shape[0]
        X = np.empty((n, n), dtype=np.float32)
        st = self.lib.fram_gradient(self.handle, _ptr(A), _ptr(N), _ptr(B), n,
                                    PRECISIONS[prec] if isinstance(prec, str) else prec, _ptr(X))
        _check(self.handle, st, "fram_gradient")
        return X

    def assign(self, W) -> np.ndarray:
        """fram_assign: exact assignment maximising sum_i W[i, perm[i]] (eq. 2)."""
        W = _f32(W)
        n = W.shape[0]
        perm = np.empty(n, dtype=np.int32)
        _check(self.handle, self.lib.fram_assign(self.handle, _ptr(W), n, _ptr(perm)),
               "fram_assign")
        return perm.astype(np.int64)

    def assign_dev(self, dW: int, ldw: int, n: int, dperm: int, stream=0):
        """fram_assign_dev on device pointers (dperm: n int32)."""
        _check(self.handle, self.lib.fram_assign_dev(self.handle, dW, ldw, n, dperm, stream),
               "fram_assign_dev")

    def solve_many(self, As, Bs, theta=2.0, iters=100, tol=0.0, **opts):
        """fram_solve_many_ex; returns (list of perms, objectives array, list of stats)."""
        As = [_f64(a) for a in As]
        Bs = [_f64(b) for b in Bs]
        count = len(As)
        ns = np.array([a.shape[0] for a in As], dtype=np.int32)
        perms = [np.empty(int(n), dtype=np.int32) for n in ns]
        pa = (ctypes.c_void_p * count)(*[_ptr(a) for a in As])
        pb = (ctypes.c_void_p * count)(*[_ptr(b) for b in Bs])
        pp = (ctypes.c_void_p * count)(*[_ptr(p) for p in perms])
        objs = np.empty(count, dtype=np.float64)
        stats = (Stats * count)()
        o = _options(**opts)
        st = self.lib.fram_solve_many_ex(self.handle, count, pa, pb, _ptr(ns), theta, iters, tol,
                                         ctypes.byref(o), pp, _ptr(objs), stats)
        _check(self.handle, st, "fram_solve_many_ex")
        return [p.astype(np.int64) for p in perms], objs, [s.as_dict() for s in stats]

    def resident_bytes(self) -> int:
        """fram_resident_bytes: device memory this context holds between calls."""
        return int(self.lib.fram_resident_bytes(self.handle))

    def trim(self) -> None:
        """fram_trim: release the context's device workspace."""
        _check(self.handle, self.lib.fram_trim(self.handle), "fram_trim")

    def last_stats(self) -> dict:
        s = Stats()
        _check(self.handle, self.lib.fram_last_stats(self.handle, ctypes.byref(s)), "fram_last_stats")
        return s.as_dict()



