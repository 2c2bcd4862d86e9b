"""FP64 CPU oracle of second-order spectral projection (SP2) with SpAMM.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg of the
benchmark).  It shares no code with the device library.

The paper builds the spectral projector (the Heaviside step function of the
Fockian, Sec. 4) by SP2 purification run to convergence, each iteration one
SpAMM square, and cites Niklasson (2002) for the scheme without writing it
out.  The steps below are that scheme as read for this build:

1. Gershgorin bounds over the N active rows (the paper gives none):
   eps_min = min_i (F_ii - R_i), eps_max = max_i (F_ii + R_i),
   R_i = sum_{j != i} |F_ij|.
2. X_0 = (eps_max I_N - F) / (eps_max - eps_min) on the active N x N block,
   zero in the padding (I_N, not the padded identity, so the padding adds
   nothing to the trace): low energies map towards 1, so the
   projector is onto the n_occ lowest eigenvectors of F.
3. For n = 0, 1, ...:
     t_n = tr X_n;  C = SpAMM(X_n, X_n, tau);  e_n = ||C - X_n||_F
     X_{n+1} = C if t_n > n_occ else 2 X_n - C
     stop if e_n < tol (converged), or, with the stall rule on, if n >= 2,
     e_n < stall_floor * sqrt(max(n_occ, 1)) and e_n >= e_{n-2} (stalled at
     the precision or culling floor, which grows with ||P||_F = sqrt(n_occ);
     past it the iteration drifts and, in finite precision, eventually
     diverges), or when n + 1 = max_iter (not converged).
   The returned projector is X_{n+1} of the stopping iteration.
   Stopping is only allowed once n + 1 >= min_iter.

The SpAMM product is the flat definition (`spamm_oracle.spamm`) or the
recursive Alg. 1 form (`alg1.spamm_alg1`), which execute the same leaf set.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .spamm_oracle import check_tau, pad, padded_size, spamm

STOP_CONVERGED = 0
STOP_STALLED = 1
STOP_MAX_ITER = 2


@dataclasses.dataclass
class SP2Result:
    p: np.ndarray                 # [n, n] projector, FP64
    iterations: int
    branches: list                # 1 = X^2 branch, 0 = 2X - X^2 branch
    traces: list                  # t_n = tr X_n
    errors: list                  # e_n = ||X~_n^2 - X_n||_F
    n_exec: list                  # executed leaf products per iteration
    n_exec_upper: list            # the same, C blocks with i <= j only
    eps_min: float
    eps_max: float
    stop: int


def gershgorin(f: np.ndarray) -> tuple[float, float]:
    """Gershgorin bounds of the spectrum of symmetric F over its rows."""
    f = np.asarray(f, dtype=np.float64)
    d = np.diag(f)
    r = np.abs(f).sum(axis=1) - np.abs(d)
    return float((d - r).min()), float((d + r).max())


def initial_x(f: np.ndarray, eps_min: float, eps_max: float, n_pad: int) -> np.ndarray:
    """X_0 = (eps_max I_N - F) / (eps_max - eps_min), zero-padded."""
    n = f.shape[0]
    x = (eps_max * np.eye(n) - f) / (eps_max - eps_min)
    return pad(x, n_pad)


def sp2(f: np.ndarray, n_occ: int, tau: float, tol: float = 1e-8, max_iter: int = 100,
        min_iter: int = 0, stall: bool = True, stall_floor: float = 1e-3,
        product=None) -> SP2Result:
    """Run SP2 on symmetric F; returns the projector and the iteration history."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    if f.ndim != 2 or f.shape[1] != n or n < 1:
        raise ValueError("square F expected")
    if not (0 <= n_occ <= n):
        raise ValueError("n_occ out of range")
    if max_iter < 1:
        raise ValueError("max_iter must be >= 1")
    tau = check_tau(tau)
    product = spamm if product is None else product
    n_pad = padded_size(n)
    eps_min, eps_max = gershgorin(f)
    if not eps_max > eps_min:
        raise ValueError("degenerate spectrum bounds")
    x = initial_x(f, eps_min, eps_max, n_pad)
    floor = stall_floor * math.sqrt(max(n_occ, 1))
    branches, traces, errors, execs, uppers = [], [], [], [], []
    stop = STOP_MAX_ITER
    it = 0
    for it in range(max_iter):
        t = float(np.trace(x))
        c, info = product(x, x, tau, n_pad=n_pad)
        e = float(np.linalg.norm(c - x))
        square = t > n_occ
        x = c if square else 2.0 * x - c
        branches.append(1 if square else 0)
        traces.append(t)
        errors.append(e)
        execs.append(int(info["n_exec"]))
        uppers.append(int(info.get("n_exec_upper", -1)))
        if it + 1 >= min_iter:
            if e < tol:
                stop = STOP_CONVERGED
                break
            if stall and it >= 2 and e < floor and e >= errors[it - 2]:
                stop = STOP_STALLED
                break
    return SP2Result(p=x[:n, :n].copy(), iterations=it + 1, branches=branches, traces=traces,
                     errors=errors, n_exec=execs, n_exec_upper=uppers, eps_min=eps_min,
                     eps_max=eps_max, stop=stop)


def energy_error(f: np.ndarray, p_ref: np.ndarray, p: np.ndarray) -> float:
    """Tr[F (P - P~)], the paper's accumulated-error measure (Sec. 4.1)."""
    return float(np.sum(f * (p_ref - p).T))


def idempotency_error(p: np.ndarray) -> float:
    """||P^2 - P||_F with an exact dense FP64 square."""
    return float(np.linalg.norm(p @ p - p))
