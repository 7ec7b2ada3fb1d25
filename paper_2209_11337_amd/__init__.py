"""MI355X QMC-CPW Greeks: Python binding of the C ABI in include/qmc_cpw.h.

Argument marshalling only: every step of the estimator runs in the HIP
library ``libqmccpw.so`` built from ``csrc/`` (``python -m
paper_2209_11337_amd.build`` or ``__graft_entry__.build()``).  Importing this
package without the built library raises; there is no CPU fallback.

Torch, when used, only provides device buffers and the current stream
(``greeks(..., device_outputs=True)``).
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmccpw.so")

ARITH_ASIAN, BINARY_ASIAN, LOOKBACK, GEOMETRIC_ASIAN = 0, 1, 2, 3
ARITH_ASIAN_PUT, BINARY_ASIAN_PUT, LOOKBACK_PUT, GEOMETRIC_ASIAN_PUT = 4, 5, 6, 7
BASKET_ASIAN, BASKET_ASIAN_PUT = 8, 9
MAX_ASSETS, MAX_BASKET_DIMS = 8, 384
PATH_BB, PATH_PCA, PATH_STANDARD, PATH_PCA_FULL = 0, 1, 2, 3
FP64, FP32_MIXED = 0, 1
GEMM_FP32, GEMM_BF16X3 = 0, 1
FLAG_GRAPH, FLAG_OWEN = 1, 2
OUTPUTS = ("price", "delta", "vega", "gamma")
MAX_D, MAX_D_PCA, MAX_D_PCA_FULL = 385, 257, 256

STATUS = {0: "QCPW_OK", -1: "QCPW_EINVAL", -2: "QCPW_ENOMEM", -3: "QCPW_EDEVICE", -4: "QCPW_EDIMS",
          -5: "QCPW_EBUSY", -6: "QCPW_ECANCELLED", -7: "QCPW_ENOTFOUND"}

# names of every entry point declared in include/qmc_cpw.h
EXPORTS = ("qmc_cpw_greeks", "qmc_cpw_greeks_ex", "qmc_cpw_greeks_noalloc", "qcpw_sobol_points", "qcpw_scrambled_points",
           "qcpw_path_coordinates", "qcpw_path_factor",
           "qcpw_kernel_timer", "qcpw_last_error", "qcpw_version", "qcpw_server_create", "qcpw_submit", "qcpw_poll",
           "qcpw_wait", "qcpw_cancel", "qcpw_server_stats", "qcpw_server_destroy")


class QcpwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class OptionSpec(C.Structure):
    _fields_ = [("type", C.c_int32), ("d", C.c_int32), ("S0", C.c_double), ("K", C.c_double),
                ("r", C.c_double), ("sigma", C.c_double), ("T", C.c_double), ("seed", C.c_uint64),
                ("n_points", C.c_int64), ("n_assets", C.c_int32), ("reserved", C.c_int32), ("rho", C.c_double)]


class RunConfig(C.Structure):
    _fields_ = [("precision", C.c_int32), ("pca_gemm", C.c_int32), ("device", C.c_int32),
                ("outputs_on_device", C.c_int32), ("stream", C.c_void_p),
                ("out_per_shift", C.c_void_p), ("block_threads", C.c_int32), ("flags", C.c_int32),
                ("out_paper_sigma", C.c_void_p)]


_lib = None
_lock = threading.Lock()


def lib() -> C.CDLL:
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libqmccpw.so is not built (run paper_2209_11337_amd/build.py); "
                                  "there is no fallback path")
            # One HIP runtime per process: torch ships its own libamdhip64.so.7;
            # loading it first lets the library bind to that copy (same soname),
            # so device pointers and streams from torch are valid here.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = C.CDLL(LIB_PATH)
            vp, i32, i64, u64, f64p = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
            L.qmc_cpw_greeks.argtypes = [vp, i32, i32, i64, i32, i32, f64p, f64p]
            L.qmc_cpw_greeks_ex.argtypes = [vp, i32, i32, i64, i32, i32, f64p, f64p, vp]
            L.qmc_cpw_greeks_noalloc.argtypes = [vp, i32, i32, i64, i32, i32, f64p, f64p, vp]
            L.qcpw_sobol_points.argtypes = [u64, i32, i32, i64, i64, vp]
            L.qcpw_scrambled_points.argtypes = [u64, i32, i32, i64, i64, vp]
            L.qcpw_path_coordinates.argtypes = [vp, i32, i32, i32, i32, vp]
            L.qcpw_path_factor.argtypes = [i32, i32, C.c_double, vp]
            L.qcpw_kernel_timer.argtypes = [i32, i32, C.POINTER(C.c_double), C.POINTER(i64)]
            L.qcpw_last_error.restype = C.c_char_p
            L.qcpw_version.restype = C.c_char_p
            L.qcpw_server_create.argtypes = [vp, i64, C.POINTER(vp)]
            L.qcpw_submit.argtypes = [vp, vp, i32, i32, i32, C.c_double, C.POINTER(u64)]
            L.qcpw_poll.argtypes = [vp, u64, vp, vp, vp]
            L.qcpw_wait.argtypes = [vp, u64, vp, vp, vp]
            L.qcpw_cancel.argtypes = [vp, u64]
            L.qcpw_server_stats.argtypes = [vp, vp]
            L.qcpw_server_destroy.argtypes = [vp]
            for name in EXPORTS:
                f = getattr(L, name)
                if f.restype is C.c_int or f.restype is None:
                    if name not in ("qcpw_last_error", "qcpw_version"):
                        f.restype = C.c_int32
            _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise QcpwError(st, lib().qcpw_last_error().decode())


def last_error() -> str:
    return lib().qcpw_last_error().decode()


def version() -> str:
    return lib().qcpw_version().decode()


def make_specs(options: Sequence[dict]) -> C.Array:
    arr = (OptionSpec * len(options))()
    for i, o in enumerate(options):
        arr[i] = OptionSpec(int(o["type"]), int(o.get("d", 0)), float(o["S0"]), float(o["K"]),
                            float(o["r"]), float(o["sigma"]), float(o["T"]),
                            int(o.get("seed", 0)) & (2**64 - 1), int(o.get("n_points", 0)),
                            int(o.get("n_assets", 0)), 0, float(o.get("rho", 1.0)))
    return arr


def greeks(options: Sequence[dict], n_shifts: int, path: int = PATH_BB, precision: int = FP64,
           d: int = 0, n_points: int = 0, pca_gemm: int = GEMM_FP32, per_shift: bool = False,
           block_threads: int = 0, stream=None, device_outputs: bool = False, device: int = -1,
           out=None, graph: bool = False, owen: bool = False, paper_sigma: bool = False):
    """Greeks of many options in one launch.

    Host mode (default): returns (greeks[n][4], stderr[n][4]) numpy arrays,
    followed by per_shift[n][L][4] and paper_sigma[n][4] (the spread of the
    single replications) when asked for.  Device mode: ``out`` is a tuple of
    torch CUDA tensors (greeks, stderr[, per_shift][, paper_sigma]) the
    results are written to on ``stream`` (default: torch's current stream);
    returns ``out``.
    """
    specs = make_specs(options)
    n = len(options)
    cfg = RunConfig(precision, pca_gemm, device, 1 if device_outputs else 0, None, None,
                    block_threads, (FLAG_GRAPH if graph else 0) | (FLAG_OWEN if owen else 0))
    if device_outputs:
        import torch
        if out is None:
            dev = torch.device("cuda", torch.cuda.current_device() if device < 0 else device)
            out = (torch.empty((n, 4), dtype=torch.float64, device=dev),
                   torch.empty((n, 4), dtype=torch.float64, device=dev))
            if per_shift:
                out = out + (torch.empty((n, n_shifts, 4), dtype=torch.float64, device=dev),)
            if paper_sigma:
                out = out + (torch.empty((n, 4), dtype=torch.float64, device=dev),)
        s = stream if stream is not None else torch.cuda.current_stream()
        cfg.stream = C.c_void_p(s.cuda_stream)
        if per_shift:
            cfg.out_per_shift = C.c_void_p(out[2].data_ptr())
        if paper_sigma:
            cfg.out_paper_sigma = C.c_void_p(out[3 if per_shift else 2].data_ptr())
        _check(lib().qmc_cpw_greeks_ex(specs, n, d, n_points, n_shifts, path, out[0].data_ptr(),
                                       out[1].data_ptr(), C.byref(cfg)))
        return out
    g = np.zeros((n, 4))
    e = np.zeros((n, 4))
    ps = np.zeros((n, n_shifts, 4)) if per_shift else None
    sg = np.zeros((n, 4)) if paper_sigma else None
    if per_shift:
        cfg.out_per_shift = C.c_void_p(ps.ctypes.data)
    if paper_sigma:
        cfg.out_paper_sigma = C.c_void_p(sg.ctypes.data)
    if stream is not None:
        cfg.stream = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(lib().qmc_cpw_greeks_ex(specs, n, d, n_points, n_shifts, path, g.ctypes.data, e.ctypes.data,
                                   C.byref(cfg)))
    return (g, e) + ((ps,) if per_shift else ()) + ((sg,) if paper_sigma else ())


NOALLOC_BYTES = 64 << 20


def greeks_noalloc(options: Sequence[dict], n_shifts: int, path: int = PATH_BB, precision: int = FP64,
                   d: int = 0, n_points: int = 0, block_threads: int = 0, owen: bool = False, out=None,
                   stream=None):
    """qmc_cpw_greeks_noalloc: the launch workspace in the library's fixed
    device array (no device allocation).  out=None: host outputs, returns
    (greeks[n][4], stderr[n][4]); out = (greeks, stderr) torch CUDA tensors:
    written on `stream` (default: torch's current stream), returns out."""
    specs = make_specs(options)
    n = len(options)
    cfg = RunConfig(precision, GEMM_FP32, -1, 1 if out is not None else 0, None, None, block_threads,
                    FLAG_OWEN if owen else 0)
    if out is not None:
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        cfg.stream = C.c_void_p(s.cuda_stream)
        _check(lib().qmc_cpw_greeks_noalloc(specs, n, d, n_points, n_shifts, path, out[0].data_ptr(),
                                            out[1].data_ptr(), C.byref(cfg)))
        return out
    g = np.zeros((n, 4))
    e = np.zeros((n, 4))
    _check(lib().qmc_cpw_greeks_noalloc(specs, n, d, n_points, n_shifts, path, g.ctypes.data, e.ctypes.data,
                                        C.byref(cfg)))
    return g, e


def greeks_plain(options: Sequence[dict], n_shifts: int, path: int = PATH_BB, d: int = 0,
                 n_points: int = 0):
    """The plain entry point qmc_cpw_greeks (FP64, host buffers)."""
    specs = make_specs(options)
    n = len(options)
    g = np.zeros((n, 4))
    e = np.zeros((n, 4))
    _check(lib().qmc_cpw_greeks(specs, n, d, n_points, n_shifts, path, g.ctypes.data, e.ctypes.data))
    return g, e


def sobol_points(seed: int, shift_index: int, n_dims: int, k0: int, count: int,
                 owen: bool = False) -> np.ndarray:
    """The randomised Sobol integers the kernels use: digital shift, or nested
    scrambling with owen=True."""
    out = np.zeros((count, n_dims), dtype=np.uint32)
    f = lib().qcpw_scrambled_points if owen else lib().qcpw_sobol_points
    _check(f(seed & (2**64 - 1), shift_index, n_dims, k0, count, out.ctypes.data))
    return out


def path_coordinates(option: dict, n_shifts: int, path: int = PATH_BB, precision: int = FP32_MIXED,
                     owen: bool = False) -> np.ndarray:
    """The randomised Sobol integers the per-path kernel consumes for one
    option: [n_shifts][n_points][dimensions 1..], recorded by the kernel."""
    spec = make_specs([option])
    d = int(option["d"])
    nd = d - 1 + (int(option.get("n_assets", 0)) * d if option["type"] in (BASKET_ASIAN, BASKET_ASIAN_PUT) else 0)
    out = np.zeros((n_shifts, int(option["n_points"]), nd), dtype=np.uint32)
    _check(lib().qcpw_path_coordinates(spec, n_shifts, path, precision, FLAG_OWEN if owen else 0,
                                       out.ctypes.data))
    return out


def path_factor(path: int, d: int, T: float) -> np.ndarray:
    """The factor A: (d-1) x (d-1), or d x d for PATH_PCA_FULL."""
    m = d if path == PATH_PCA_FULL else d - 1
    out = np.zeros((max(m, 0), max(m, 0)))
    buf = out if m > 0 else np.zeros(1)
    _check(lib().qcpw_path_factor(path, d, T, buf.ctypes.data))
    return out


TIMER_START, TIMER_READ, TIMER_STOP = 1, 2, 3


def kernel_timer(op: int, device: int = -1) -> tuple[float, int]:
    """qcpw_kernel_timer: (summed main-kernel milliseconds, timed launches)."""
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _check(lib().qcpw_kernel_timer(device, op, C.byref(ms), C.byref(n)))
    return ms.value, n.value


class Server:
    """Continuous-batching request server (qcpw_server_*)."""

    def __init__(self, hbm_budget_bytes: int, precision: int = FP32_MIXED, device: int = -1,
                 block_threads: int = 0, owen: bool = False):
        cfg = RunConfig(precision, GEMM_FP32, device, 0, None, None, block_threads, FLAG_OWEN if owen else 0)
        h = C.c_void_p()
        _check(lib().qcpw_server_create(C.byref(cfg), hbm_budget_bytes, C.byref(h)))
        self._h = h

    def submit(self, options: Sequence[dict], n_shifts: int, target_stderr: float,
               path: int = PATH_BB) -> int:
        specs = make_specs(options)
        rid = C.c_uint64()
        _check(lib().qcpw_submit(self._h, specs, len(options), n_shifts, path, target_stderr, C.byref(rid)))
        return rid.value

    def _result(self, fn, rid: int, n: int):
        g = np.zeros((n, 4))
        e = np.zeros((n, 4))
        pts = C.c_int64()
        st = fn(self._h, rid, g.ctypes.data, e.ctypes.data, C.byref(pts))
        return st, g, e, pts.value

    def poll(self, rid: int, n: int):
        """None while running; else (greeks, stderr, points_used)."""
        st, g, e, p = self._result(lib().qcpw_poll, rid, n)
        if st == -5:
            return None
        _check(st)
        return g, e, p

    def wait(self, rid: int, n: int):
        st, g, e, p = self._result(lib().qcpw_wait, rid, n)
        _check(st)
        return g, e, p

    def cancel(self, rid: int):
        _check(lib().qcpw_cancel(self._h, rid))

    def stats(self) -> dict:
        out = (C.c_int64 * 8)()
        _check(lib().qcpw_server_stats(self._h, out))
        keys = ("admitted", "completed", "cancelled", "launches", "bytes_in_use", "peak_bytes", "queued",
                "workspace_bytes")
        return dict(zip(keys, list(out)))

    def close(self):
        if self._h:
            _check(lib().qcpw_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
