"""ctypes binding of libspamm (include/spamm.h): argument marshalling only.

Every step of SpAMM and SP2 runs in the library's HIP kernels; this module
converts Python arguments (torch tensors on the GPU, numpy arrays on the
host, streams) to the C ABI and the C results back.  If the shared library
is missing or cannot be loaded, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspamm.so")

FP64, FP32, BF16, FP16, BF16X3, FP16X3 = 0, 1, 2, 3, 4, 5
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp16": FP16, "bf16x3": BF16X3,
              "fp16x3": FP16X3}
SP2_MAX_ITER = 256
N_PHASES = 6
PHASES = ("tree", "pyramid", "cull", "gemm", "epilogue", "dense")
STOP_REASONS = ("converged", "stalled", "max_iter")

OK, NOT_CONVERGED, PENDING = 0, 1, 2
ERR_NAMES = {-1: "INVALID_ARG", -2: "NONFINITE", -3: "NOT_SYMMETRIC", -4: "OOM", -5: "DEVICE",
             -6: "SHAPE"}


class SpammError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"SPAMM_ERR_{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class SpammInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_pad", ctypes.c_int64), ("nb", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_blocks", ctypes.c_int64),
                ("frobenius", ctypes.c_double)]


class MultStats(ctypes.Structure):
    _fields_ = [("n_exec", ctypes.c_int64), ("n_cblocks", ctypes.c_int64),
                ("n_nonzero_pairs", ctypes.c_int64), ("n_dense", ctypes.c_int64),
                ("err_bound", ctypes.c_double), ("cull_restarts", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Sp2Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("min_iter", ctypes.c_int32), ("stall_rule", ctypes.c_int32),
                ("tol", ctypes.c_double), ("stall_floor", ctypes.c_double),
                ("symmetric", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Sp2Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("symmetric", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eps_min", ctypes.c_double), ("eps_max", ctypes.c_double),
                ("trace_final", ctypes.c_double), ("n_exec_total", ctypes.c_int64),
                ("branch", ctypes.c_int8 * SP2_MAX_ITER),
                ("trace", ctypes.c_double * SP2_MAX_ITER),
                ("err", ctypes.c_double * SP2_MAX_ITER),
                ("n_exec", ctypes.c_int64 * SP2_MAX_ITER),
                ("n_blocks", ctypes.c_int64 * SP2_MAX_ITER)]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * N_PHASES), ("ms", ctypes.c_double * N_PHASES),
                ("gemm_products", ctypes.c_int64)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("batch_gemm", ctypes.c_int32),
                ("device", ctypes.c_int32), ("fill_products", ctypes.c_int32)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("active", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("gemm_launches", ctypes.c_int64), ("solve_iterations", ctypes.c_int64),
                ("budget_bytes", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64),
                ("cached_bytes", ctypes.c_uint64), ("peak_used_bytes", ctypes.c_uint64)]


# Exported symbols and their signatures (kept in step with include/spamm.h).
_VP, _I64, _I32, _D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
SIGNATURES = {
    "sp2_options_default": (None, [ctypes.POINTER(Sp2Options)]),
    "spamm_tree_build": (ctypes.c_int, [_VP, _I64, _I64, _I32, _VP, ctypes.POINTER(_VP)]),
    "spamm_multiply": (ctypes.c_int, [_VP, _VP, _D, _VP, ctypes.POINTER(_VP),
                                      ctypes.POINTER(MultStats)]),
    "spamm_cull": (ctypes.c_int, [_VP, _VP, _D, _VP, ctypes.POINTER(_VP)]),
    "spamm_tasks_info": (ctypes.c_int, [_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "spamm_tasks_copy": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "spamm_tasks_destroy": (None, [_VP]),
    "sp2_solve": (ctypes.c_int, [_VP, _I64, _I64, _I64, _D, ctypes.POINTER(Sp2Options), _VP, _VP,
                                 _I64, ctypes.POINTER(Sp2Stats)]),
    "sp2_initial_guess": (ctypes.c_int, [_VP, _I64, _I64, _I32, _VP, ctypes.POINTER(_VP),
                                         ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "spamm_to_dense": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "spamm_matrix_info": (ctypes.c_int, [_VP, ctypes.POINTER(SpammInfo)]),
    "spamm_matrix_norms": (ctypes.c_int, [_VP, _VP, _VP]),
    "spamm_matrix_destroy": (None, [_VP]),
    "spamm_last_error": (ctypes.c_char_p, []),
    "spamm_version": (ctypes.c_char_p, []),
    "spamm_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "spamm_profile_phases": (ctypes.c_int, [ctypes.c_uint]),
    "spamm_profile_reset": (ctypes.c_int, []),
    "spamm_profile_read": (ctypes.c_int, [ctypes.POINTER(Profile)]),
    "sp2_footprint_bytes": (ctypes.c_size_t, [_I64, _I32]),
    "spamm_server_options_default": (None, [ctypes.POINTER(ServerOptions)]),
    "spamm_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(ServerOptions),
                                           ctypes.POINTER(_VP)]),
    "spamm_server_submit": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I64, _D,
                                           ctypes.POINTER(Sp2Options),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "spamm_server_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _I64,
                                         ctypes.POINTER(Sp2Stats)]),
    "spamm_server_wait": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _I64,
                                         ctypes.POINTER(Sp2Stats)]),
    "spamm_server_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ServerInfo)]),
    "spamm_server_destroy": (None, [_VP]),
}

_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Load libspamm.so (raises if it is missing: there is no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise ImportError(f"{path} is missing: build it with "
                                  "`python -m paper_1403_7458_amd.build`")
            lib = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _check(rc: int, allow=(OK,)) -> int:
    if rc in allow:
        return rc
    msg = load().spamm_last_error().decode(errors="replace")
    raise SpammError(rc, msg)


def _stream(stream):
    """hipStream_t of `stream` (torch stream, int, None = torch's current)."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dense_arg(a):
    """(pointer, n, ld, keepalive) of a square FP64 row-major matrix."""
    if hasattr(a, "data_ptr"):      # torch tensor (device or host)
        if a.dtype != __import__("torch").float64 or a.dim() != 2 or a.shape[0] != a.shape[1]:
            raise ValueError("square float64 tensor expected")
        if a.stride(1) != 1:
            a = a.contiguous()
        return ctypes.c_void_p(a.data_ptr()), a.shape[0], a.stride(0), a
    arr = np.asarray(a)
    if arr.dtype != np.float64 or arr.ndim != 2 or arr.shape[0] != arr.shape[1]:
        raise ValueError("square float64 array expected")
    if arr.strides[1] != 8 or arr.strides[0] % 8:
        arr = np.ascontiguousarray(arr)
    return ctypes.c_void_p(arr.ctypes.data), arr.shape[0], arr.strides[0] // 8, arr


class SpammMatrix:
    """Owning wrapper of a spamm_matrix handle."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = SpammInfo()
        _check(load().spamm_matrix_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in SpammInfo._fields_ if f != "reserved"}

    def close(self):
        if self._h is not None and self._h.value:
            load().spamm_matrix_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spamm_tree_build(a, prec="fp32", stream=None) -> SpammMatrix:
    p, n, ld, keep = _dense_arg(a)
    h = ctypes.c_void_p()
    _check(load().spamm_tree_build(p, n, ld, PRECISIONS.get(prec, prec), _stream(stream),
                                   ctypes.byref(h)))
    del keep
    return SpammMatrix(h)


def _stats_dict(st) -> dict:
    return {f: getattr(st, f) for f, _ in st._fields_ if f != "reserved"}


def spamm_multiply(a: SpammMatrix, b: SpammMatrix, tau: float, stream=None, stats: bool = True):
    """(C, statistics dict); stats=False skips the passes only the
    statistics need and returns (C, None)."""
    h = ctypes.c_void_p()
    st = MultStats()
    _check(load().spamm_multiply(a.handle, b.handle, float(tau), _stream(stream), ctypes.byref(h),
                                 ctypes.byref(st) if stats else None))
    return SpammMatrix(h), (_stats_dict(st) if stats else None)


def spamm_cull(a: SpammMatrix, b: SpammMatrix, tau: float, stream=None) -> dict:
    """Task list E(tau) grouped by C block, as host numpy arrays."""
    lib = load()
    h = ctypes.c_void_p()
    _check(lib.spamm_cull(a.handle, b.handle, float(tau), _stream(stream), ctypes.byref(h)))
    try:
        nc, nt = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.spamm_tasks_info(h, ctypes.byref(nc), ctypes.byref(nt)))
        ci = np.empty(max(nc.value, 1), np.int32)
        cj = np.empty(max(nc.value, 1), np.int32)
        cp = np.empty(nc.value + 1, np.int64)
        ks = np.empty(max(nt.value, 1), np.int32)
        _check(lib.spamm_tasks_copy(h, ci.ctypes.data, cj.ctypes.data, cp.ctypes.data,
                                    ks.ctypes.data, _stream(stream)))
    finally:
        lib.spamm_tasks_destroy(h)
    return {"c_i": ci[:nc.value], "c_j": cj[:nc.value], "c_ptr": cp, "k": ks[:nt.value]}


def sp2_initial_guess(f, prec="fp32", stream=None):
    """Tree of X_0 = (eps_max I - F) / (eps_max - eps_min); returns (X_0, eps_min, eps_max)."""
    p, n, ld, keep = _dense_arg(f)
    h = ctypes.c_void_p()
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(load().sp2_initial_guess(p, n, ld, PRECISIONS.get(prec, prec), _stream(stream),
                                    ctypes.byref(h), ctypes.byref(lo), ctypes.byref(hi)))
    return SpammMatrix(h), lo.value, hi.value


def spamm_to_dense(m: SpammMatrix, out=None, stream=None):
    """Dense FP64 copy: into `out` (torch tensor or numpy array) or a new numpy array."""
    n = m.info()["n"]
    if out is None:
        out = np.empty((n, n), np.float64)
    p, n2, ld, keep = _dense_arg(out)
    if n2 != n:
        raise ValueError("output size mismatch")
    _check(load().spamm_to_dense(m.handle, p, ld, _stream(stream)))
    return out


def spamm_matrix_norms(m: SpammMatrix, stream=None) -> list:
    """Norms of every tier: list of 2^t x 2^t arrays, t = 0 (root) .. depth."""
    d = m.info()["depth"]
    total = ((1 << (2 * (d + 1))) - 1) // 3
    buf = np.empty(total, np.float64)
    _check(load().spamm_matrix_norms(m.handle, buf.ctypes.data, _stream(stream)))
    out = []
    for t in range(d + 1):
        off = ((1 << (2 * t)) - 1) // 3
        out.append(buf[off:off + (1 << (2 * t))].reshape(1 << t, 1 << t))
    return out


def sp2_options(precision="fp32", max_iter=100, min_iter=0, stall_rule=True, tol=1e-8,
                stall_floor=0.0, symmetric=True) -> Sp2Options:
    o = Sp2Options()
    load().sp2_options_default(ctypes.byref(o))
    o.precision = PRECISIONS.get(precision, precision)
    o.max_iter, o.min_iter, o.stall_rule = int(max_iter), int(min_iter), int(bool(stall_rule))
    o.tol, o.stall_floor = float(tol), float(stall_floor)
    o.symmetric = int(bool(symmetric))
    return o


def sp2_solve(f, n_occ: int, tau: float, out=None, stream=None, **opts):
    """Run SP2 on F; returns (P, stats dict).  P goes to `out` if given
    (torch tensor or numpy array), else to a new numpy array."""
    pf, n, ldf, keep_f = _dense_arg(f)
    if out is None:
        out = np.empty((n, n), np.float64)
    pp, n2, ldp, keep_p = _dense_arg(out)
    if n2 != n:
        raise ValueError("output size mismatch")
    o = sp2_options(**opts)
    st = Sp2Stats()
    rc = load().sp2_solve(pf, n, ldf, int(n_occ), float(tau), ctypes.byref(o), _stream(stream), pp,
                          ldp, ctypes.byref(st))
    _check(rc, allow=(OK, NOT_CONVERGED))
    return out, _sp2_stats(rc, st)


def _sp2_stats(rc: int, st: Sp2Stats) -> dict:
    it = st.iterations
    return {
        "status": rc, "iterations": it, "stop": STOP_REASONS[st.stop_reason],
        "symmetric": bool(st.symmetric),
        "eps_min": st.eps_min, "eps_max": st.eps_max, "trace_final": st.trace_final,
        "n_exec_total": st.n_exec_total,
        "branches": [int(x) for x in st.branch[:it]],
        "traces": list(st.trace[:it]), "errors": list(st.err[:it]),
        "n_exec": [int(x) for x in st.n_exec[:it]], "n_blocks": [int(x) for x in st.n_blocks[:it]],
    }


def sp2_footprint_bytes(n: int, precision="fp32") -> int:
    """Peak device memory of one SP2 solve of order n (an upper bound)."""
    return int(load().sp2_footprint_bytes(int(n), PRECISIONS.get(precision, precision)))


class Sp2Server:
    """Owning wrapper of a spamm_server: SP2 requests solved together on one
    device, one iteration of every running request per step."""

    def __init__(self, budget_bytes: int, max_active: int = 64, batch_gemm: bool = True,
                 device: int = -1, fill_products=None):
        lib = load()
        o = ServerOptions()
        lib.spamm_server_options_default(ctypes.byref(o))
        o.max_active, o.batch_gemm, o.device = int(max_active), int(bool(batch_gemm)), int(device)
        if fill_products is not None:
            o.fill_products = int(fill_products)
        self._h = ctypes.c_void_p()
        _check(lib.spamm_server_create(int(budget_bytes), ctypes.byref(o), ctypes.byref(self._h)))
        self._inputs = {}   # device inputs, kept alive until their request finishes

    def submit(self, f, n_occ: int, tau: float, **opts) -> int:
        pf, n, ldf, keep = _dense_arg(f)
        o = sp2_options(**opts)
        rid = ctypes.c_uint64()
        _check(load().spamm_server_submit(self._h, pf, n, ldf, int(n_occ), float(tau),
                                          ctypes.byref(o), ctypes.byref(rid)))
        self._inputs[rid.value] = (keep, n)
        return rid.value

    def _collect(self, fn, rid: int, out):
        if rid not in self._inputs:  # unknown or already collected: the library says which
            _check(fn(self._h, ctypes.c_uint64(rid), None, 0, None))
        keep, n = self._inputs[rid]
        if out is None:
            out = np.empty((n, n), np.float64)
        pp, n2, ldp, keep_p = _dense_arg(out)
        if n2 != n:
            raise ValueError("output size mismatch")
        st = Sp2Stats()
        rc = fn(self._h, ctypes.c_uint64(rid), pp, ldp, ctypes.byref(st))
        if rc == PENDING:
            return None
        del self._inputs[rid]
        _check(rc, allow=(OK, NOT_CONVERGED))
        return out, _sp2_stats(rc, st)

    def poll(self, rid: int, out=None):
        """None while pending, else (P, stats) as sp2_solve returns them."""
        return self._collect(load().spamm_server_poll, rid, out)

    def wait(self, rid: int, out=None):
        return self._collect(load().spamm_server_wait, rid, out)

    def stats(self) -> dict:
        inf = ServerInfo()
        _check(load().spamm_server_stats(self._h, ctypes.byref(inf)))
        return {f: int(getattr(inf, f)) for f, _ in ServerInfo._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            load().spamm_server_destroy(self._h)
        self._h = None
        self._inputs = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True):
    _check(load().spamm_profile_enable(int(bool(on))))


def profile_phases(*names: str):
    """Time only the named phases (PHASES); no names: every phase."""
    unknown = [x for x in names if x not in PHASES]
    if unknown:
        raise ValueError(f"unknown phase {unknown[0]!r}; known: {PHASES}")
    mask = sum(1 << PHASES.index(x) for x in set(names)) if names else (1 << N_PHASES) - 1
    _check(load().spamm_profile_phases(mask))


def profile_reset():
    _check(load().spamm_profile_reset())


def profile_read() -> dict:
    p = Profile()
    _check(load().spamm_profile_read(ctypes.byref(p)))
    return {"launches": dict(zip(PHASES, list(p.launches))), "ms": dict(zip(PHASES, list(p.ms))),
            "gemm_products": int(p.gemm_products)}


def version() -> str:
    return load().spamm_version().decode()
