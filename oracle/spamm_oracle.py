"""FP64 CPU oracle of the Sparse Approximate Matrix Multiply (SpAMM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the device library.

What is computed (Sec. 2 of the paper, Eqs. 1-4):

* The matrix is zero-padded to N_pad = 32 * 2^d (the smallest such size
  >= N; Fig. 4's caption pads 2,250 to 4,096) and split into a quadtree whose
  tier d holds 32 x 32 dense leaf blocks (Eq. 1; leaf size N_b = 32).
* Each node carries its Frobenius norm: a leaf's norm is the square root of
  the sum of its squared entries (Eq. 2); a parent's norm is the square root
  of the sum of its four children's squared norms (Eq. 3).
* SpAMM adds a sub-product A_ik B_kj into C_ij only when
  ||A_ik|| * ||B_kj|| > tau (strict; Eq. 4), at every tier.

Because a parent's norm is never below any child's norm (Eq. 3, and the
same holds in floating point since rounding is monotone), a leaf product
passes every ancestor test whenever it passes its own.  The recursive
(Alg. 1) and breadth-first (Algs. 2-3) forms therefore execute exactly the
flat leaf set

    E(tau) = {(i, j, k) : ||A_ik|| * ||B_kj|| > tau}

and C~_ij = sum_{k : (i,j,k) in E} A_ik B_kj.  `spamm` below is that plain
definition; `executed_set_breadth_first` walks the tiers as Algs. 2-3 do
and serves as a check of the equivalence; `oracle/alg1.c` is the recursive
Alg. 1 form with tasks and per-block locks.

Readings where the paper is silent or garbled: ties are culled (strict >);
the test uses the children's norms (Alg. 3; Alg. 1's superscripts are off by
one tier); with depth 0 the single leaf product is itself tested against tau;
tau is absolute, tau = 0 culls only exact-zero products, tau < 0 or NaN
is rejected.
"""
from __future__ import annotations

import math

import numpy as np

LEAF = 32


def padded_size(n: int) -> int:
    """N_pad = 32 * 2^d, the smallest such size >= n (Fig. 4 caption pads 2,250 to 4,096)."""
    if n < 1:
        raise ValueError("matrix dimension must be >= 1")
    nb = 1
    while LEAF * nb < n:
        nb *= 2
    return LEAF * nb


def depth_of(n_pad: int) -> int:
    nb = n_pad // LEAF
    d = int(round(math.log2(nb)))
    if LEAF * (1 << d) != n_pad:
        raise ValueError("not a padded size")
    return d


def pad(a: np.ndarray, n_pad: int | None = None) -> np.ndarray:
    """Zero-padded FP64 copy of a square matrix."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("square matrix expected")
    n = a.shape[0]
    n_pad = padded_size(n) if n_pad is None else n_pad
    out = np.zeros((n_pad, n_pad), dtype=np.float64)
    out[:n, :n] = a
    return out


def blocks(a_pad: np.ndarray) -> np.ndarray:
    """View of a padded matrix as [nb, nb, 32, 32] leaf blocks (Eq. 1 at tier d)."""
    nb = a_pad.shape[0] // LEAF
    return a_pad.reshape(nb, LEAF, nb, LEAF).transpose(0, 2, 1, 3)


def leaf_norms(a_pad: np.ndarray) -> np.ndarray:
    """Frobenius norm of every leaf block (Eq. 2)."""
    b = blocks(a_pad)
    return np.sqrt((b * b).sum(axis=(2, 3)))


def tier_norms(leaf: np.ndarray) -> list[np.ndarray]:
    """Norms of every tier, index t = 0 (root) .. d (leaves), by Eq. 3."""
    tiers = [leaf]
    cur = leaf
    while cur.shape[0] > 1:
        h = cur.shape[0] // 2
        sq = cur * cur
        parent = np.sqrt(sq[0::2, 0::2] + sq[0::2, 1::2] + sq[1::2, 0::2] + sq[1::2, 1::2])
        tiers.append(parent)
        cur = parent
    return tiers[::-1]


def check_tau(tau: float) -> float:
    tau = float(tau)
    if not math.isfinite(tau) or tau < 0.0:
        raise ValueError("tau must be finite and >= 0")
    return tau


def executed_ks(na: np.ndarray, nb_: np.ndarray, tau: float, i: int, j: int) -> np.ndarray:
    """Ascending k with ||A_ik|| ||B_kj|| > tau: the flat culling test (Eq. 4)."""
    return np.nonzero(na[i, :] * nb_[:, j] > tau)[0]


def executed_mask(na: np.ndarray, nb_: np.ndarray, tau: float) -> np.ndarray:
    """Boolean [nb, nb, nb] mask E[i, j, k] of executed leaf products (small nb)."""
    return na[:, None, :] * nb_.T[None, :, :] > tau


def spamm(a: np.ndarray, b: np.ndarray, tau: float, n_pad: int | None = None,
          rows=None, cols=None):
    """SpAMM product C~ = sum over E(tau) of A_ik B_kj, in FP64.

    a, b: square matrices of equal size (unpadded or already padded).
    rows/cols: optional iterables of block indices restricting which C
    blocks are formed (for sampling large cases); other blocks stay zero.
    Returns (c_pad, info) with c_pad the padded product and info holding the
    executed-task count, the count restricted to the C blocks with i <= j
    (what a product known to be symmetric has to execute), and the leaf
    norms.
    """
    tau = check_tau(tau)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    n_pad = padded_size(a.shape[0]) if n_pad is None else n_pad
    ap = a if a.shape[0] == n_pad else pad(a, n_pad)
    bp = b if b.shape[0] == n_pad else pad(b, n_pad)
    ab, bb = blocks(ap), blocks(bp)
    na, nbn = leaf_norms(ap), leaf_norms(bp)
    nb = n_pad // LEAF
    c = np.zeros((n_pad, n_pad), dtype=np.float64)
    cb = blocks(c)
    n_exec = n_exec_upper = 0
    rows = range(nb) if rows is None else rows
    cols = list(range(nb)) if cols is None else list(cols)
    for i in rows:
        for j in cols:
            ks = executed_ks(na, nbn, tau, i, j)
            if ks.size == 0:
                continue
            acc = np.zeros((LEAF, LEAF), dtype=np.float64)
            for k in ks:
                acc += ab[i, k] @ bb[k, j]
            cb[i, j] = acc
            n_exec += int(ks.size)
            if i <= j:
                n_exec_upper += int(ks.size)
    return c, {"n_exec": n_exec, "n_exec_upper": n_exec_upper, "norms_a": na, "norms_b": nbn}


def executed_set_breadth_first(tiers_a: list[np.ndarray], tiers_b: list[np.ndarray],
                               tau: float) -> set:
    """Leaf triples enabled by tier-by-tier occlusion (Algs. 2-3).

    Tier 0 is enabled.  On every tier t < d each enabled triple (i, j, k)
    tests its eight children (2i+a, 2j+b, 2k+c) with the norms of tier t+1
    and enables those whose norm product exceeds tau.  With d = 0 the single
    leaf is tested directly.
    """
    tau = check_tau(tau)
    d = len(tiers_a) - 1
    if d == 0:
        return {(0, 0, 0)} if tiers_a[0][0, 0] * tiers_b[0][0, 0] > tau else set()
    enabled = {(0, 0, 0)}
    for t in range(d):
        na, nbn = tiers_a[t + 1], tiers_b[t + 1]
        nxt = set()
        for (i, j, k) in enabled:
            for ci in (2 * i, 2 * i + 1):
                for cj in (2 * j, 2 * j + 1):
                    for ck in (2 * k, 2 * k + 1):
                        if na[ci, ck] * nbn[ck, cj] > tau:
                            nxt.add((ci, cj, ck))
        enabled = nxt
    return enabled


def culled_error_bound(na: np.ndarray, nb_: np.ndarray, tau: float) -> tuple[float, float]:
    """Bounds on ||C~ - AB||_F from the culled leaf products.

    By sub-multiplicativity (||XY|| <= ||X|| ||Y||, Sec. 2) and the triangle
    inequality, block (i, j) of the error is at most the sum over culled k of
    ||A_ik|| ||B_kj||.  Returns (blockwise bound, total sum bound), the first
    the Frobenius norm of the blockwise sums, the second their plain sum.
    """
    tau = check_tau(tau)
    prod = na[:, None, :] * nb_.T[None, :, :]          # [i, j, k]
    culled = np.where(prod > tau, 0.0, prod)
    per_block = culled.sum(axis=2)
    return float(np.sqrt((per_block ** 2).sum())), float(per_block.sum())
