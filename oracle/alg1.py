"""ctypes wrapper of the recursive Alg. 1 oracle in `alg1.c`.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg of the
benchmark).  The shared object is compiled with gcc from `alg1.c` by the
package build step, or here on first use if it is missing; it never links
against the device library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from .spamm_oracle import LEAF, blocks, check_tau, depth_of, pad, padded_size

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alg1.c")
_LIB = os.path.join(_HERE, "liboracle_alg1.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile alg1.c into liboracle_alg1.so (plain C, OpenMP, portable x86-64-v3)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_spamm_alg1.restype = ctypes.c_int
            lib.oracle_spamm_alg1.argtypes = [
                ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                ctypes.POINTER(ctypes.c_double)]
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def to_blocked(a_pad: np.ndarray) -> np.ndarray:
    """Contiguous [nb, nb, 32, 32] copy of a padded matrix."""
    return np.ascontiguousarray(blocks(a_pad))


def from_blocked(cb: np.ndarray) -> np.ndarray:
    nb = cb.shape[0]
    return np.ascontiguousarray(cb.transpose(0, 2, 1, 3)).reshape(nb * LEAF, nb * LEAF)


def spamm_alg1(a: np.ndarray, b: np.ndarray, tau: float, threads: int = 0,
               n_pad: int | None = None):
    """SpAMM product by the recursive task form (Alg. 1), FP64.

    Returns (c_pad, info) like `spamm_oracle.spamm`: the padded product and a
    dict with the executed-task count and the culled-product error bound.
    """
    tau = check_tau(tau)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    n_pad = padded_size(a.shape[0]) if n_pad is None else n_pad
    ab = to_blocked(a if a.shape[0] == n_pad else pad(a, n_pad))
    bb = to_blocked(b if b.shape[0] == n_pad else pad(b, n_pad))
    cb = np.empty_like(ab)
    n_exec = ctypes.c_int64(0)
    bound = ctypes.c_double(0.0)
    rc = _load().oracle_spamm_alg1(depth_of(n_pad), ab.ctypes.data, bb.ctypes.data, tau,
                                   cb.ctypes.data, int(threads), ctypes.byref(n_exec),
                                   ctypes.byref(bound))
    if rc != 0:
        raise RuntimeError(f"oracle_spamm_alg1 failed ({rc})")
    return from_blocked(cb), {"n_exec": int(n_exec.value), "culled_bound": float(bound.value)}
