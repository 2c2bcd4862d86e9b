"""Pins of the SpAMM oracle against what the paper and the mathematics fix.

Each test fixes the oracle to something other than itself: a dense BLAS
product (tau = 0), closed forms built from scalar coefficients, the paper's
own padding example, sub-multiplicativity error bounds, brute force over
matrix elements, and the equivalence of the flat, breadth-first (Algs. 2-3)
and recursive (Alg. 1) forms.
"""
import math

import numpy as np
import pytest

from oracle import alg1
from oracle import spamm_oracle as so
from watergen import synthetic as syn


@pytest.mark.parametrize("n,expect", [(1, 32), (32, 32), (33, 64), (750, 1024), (2250, 4096),
                                      (3750, 4096), (25000, 32768), (10000, 16384)])
def test_padded_size(n, expect):
    # Fig. 4 caption: the native 2,250 x 2,250 matrix is padded to 4,096 x 4,096.
    assert so.padded_size(n) == expect


def test_padded_size_rejects_empty():
    with pytest.raises(ValueError):
        so.padded_size(0)


def test_leaf_norm_known_blocks():
    a = np.zeros((64, 64))
    a[:32, :32] = 1.0                 # all-ones block: norm 32 (Eq. 2)
    a[40, 33], a[41, 60] = 3.0, 4.0   # 3-4-5 block
    n = so.leaf_norms(a)
    assert n[0, 0] == 32.0 and n[1, 1] == 5.0 and n[0, 1] == 0.0 and n[1, 0] == 0.0
    tiers = so.tier_norms(n)
    assert len(tiers) == 2 and tiers[0][0, 0] == pytest.approx(math.sqrt(32.0 ** 2 + 25.0), rel=1e-15)


def test_tier_norms_invariants():
    a = so.pad(syn.decaying(200, seed=3, rate=0.02))
    tiers = so.tier_norms(so.leaf_norms(a))
    assert len(tiers) == so.depth_of(a.shape[0]) + 1
    # Root norm equals the Frobenius norm of the whole matrix (Eqs. 2-3).
    assert tiers[0][0, 0] == pytest.approx(np.linalg.norm(a), rel=1e-14)
    for t in range(len(tiers) - 1):
        ch = tiers[t + 1] ** 2
        par = ch[0::2, 0::2] + ch[0::2, 1::2] + ch[1::2, 0::2] + ch[1::2, 1::2]
        np.testing.assert_allclose(tiers[t] ** 2, par, rtol=1e-14)
        # A parent is never smaller than any child (monotonicity used by O-2).
        for a_ in (0, 1):
            for b_ in (0, 1):
                assert np.all(tiers[t] >= tiers[t + 1][a_::2, b_::2])


@pytest.mark.parametrize("n", [1, 31, 32, 33, 100, 200])
def test_tau_zero_equals_dense_gemm(n):
    a = syn.decaying(n, seed=n, rate=0.03)
    b = syn.decaying(n, seed=n + 1000, rate=0.07)
    c, info = so.spamm(a, b, 0.0)
    ref = a @ b
    assert np.linalg.norm(c[:n, :n] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.all(c[n:, :] == 0) and np.all(c[:, n:] == 0)


def test_tau_zero_culls_only_exact_zero_products():
    a = syn.decaying(96, seed=5)
    a[0:32, 32:64] = 0.0               # an exactly zero block of A
    c, info = so.spamm(a, a, 0.0)
    nb = 4
    na = so.leaf_norms(so.pad(a))
    nonzero_pairs = sum(1 for i in range(nb) for j in range(nb) for k in range(nb)
                        if na[i, k] > 0 and na[k, j] > 0)
    assert info["n_exec"] == nonzero_pairs
    np.testing.assert_allclose(c[:96, :96], a @ a, rtol=0, atol=1e-12 * np.linalg.norm(a) ** 2)


def _coeffs(nb, seed):
    g = syn.generator(seed)
    # Magnitudes spread over many decades, values far apart so no product
    # lands near the thresholds used below.
    return 10.0 ** g.integers(-8, 1, size=(nb, nb)) * g.choice([1.0, 1.5, 2.5], size=(nb, nb))


@pytest.mark.parametrize("tau", [0.0, 3e-9, 3e-7, 3e-5, 3e-3, 0.7])
def test_scaled_block_closed_form(tau):
    """A_ik = alpha_ik U, B_kj = beta_kj V with ||U|| = ||V|| = 1: the executed set and
    the product follow from scalar arithmetic on alpha and beta alone."""
    nb = 4
    alpha, beta = _coeffs(nb, 1), _coeffs(nb, 2)
    u, v = syn.unit_block(3), syn.unit_block(4)
    a, b = syn.block_scaled(alpha, u), syn.block_scaled(beta, v)
    c, info = so.spamm(a, b, tau)
    uv = u @ v
    count = 0
    for i in range(nb):
        for j in range(nb):
            s = 0.0
            for k in range(nb):
                if alpha[i, k] * beta[k, j] > tau:   # Eq. 4, strict
                    s += alpha[i, k] * beta[k, j]
                    count += 1
            scale = sum(alpha[i, k] * beta[k, j] for k in range(nb)) * np.abs(uv).max()
            np.testing.assert_allclose(c[32 * i:32 * i + 32, 32 * j:32 * j + 32], s * uv,
                                       rtol=1e-13, atol=1e-14 * scale)
    assert info["n_exec"] == count


def test_elementwise_brute_force_tiny():
    """Element-level loops, no block views: c_rs = sum_q a_rq b_qs over kept block triples."""
    n = 40
    a = syn.decaying(n, seed=7, rate=0.3)
    b = syn.decaying(n, seed=8, rate=0.2)
    tau = 0.02
    ap, bp = so.pad(a), so.pad(b)
    npad = ap.shape[0]
    na = np.zeros((2, 2))
    nbn = np.zeros((2, 2))
    for r in range(npad):
        for s in range(npad):
            na[r // 32, s // 32] += ap[r, s] ** 2
            nbn[r // 32, s // 32] += bp[r, s] ** 2
    na, nbn = np.sqrt(na), np.sqrt(nbn)
    ref = np.zeros((npad, npad))
    for r in range(npad):
        for s in range(npad):
            acc = 0.0
            for q in range(npad):
                if na[r // 32, q // 32] * nbn[q // 32, s // 32] > tau:
                    acc += ap[r, q] * bp[q, s]
            ref[r, s] = acc
    c, _ = so.spamm(a, b, tau)
    np.testing.assert_allclose(c, ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("n,tau", [(32, 0.5), (32, 1e9), (100, 1e-3), (200, 1e-2),
                                   (300, 1e-4), (260, 0.0)])
def test_flat_equals_breadth_first_equals_alg1(n, tau):
    a = syn.decaying(n, seed=n, rate=0.04)
    b = syn.decaying(n, seed=n + 1, rate=0.04)
    ap, bp = so.pad(a), so.pad(b)
    na, nbn = so.leaf_norms(ap), so.leaf_norms(bp)
    flat = {tuple(int(x) for x in t) for t in np.argwhere(so.executed_mask(na, nbn, tau))}
    bfs = so.executed_set_breadth_first(so.tier_norms(na), so.tier_norms(nbn), tau)
    assert flat == bfs
    c1, i1 = so.spamm(a, b, tau)
    c2, i2 = alg1.spamm_alg1(a, b, tau)
    assert i1["n_exec"] == len(flat) == i2["n_exec"]
    np.testing.assert_allclose(c2, c1, rtol=1e-14, atol=1e-14 * max(1.0, np.abs(c1).max()))


@pytest.mark.parametrize("tau", [1e-6, 1e-4, 1e-3, 1e-2])
def test_error_bound(tau):
    a = syn.decaying(300, seed=11, rate=0.03)
    b = syn.decaying(300, seed=12, rate=0.03)
    c, info = so.spamm(a, b, tau)
    err = np.linalg.norm(c[:300, :300] - a @ b)
    blockwise, total = so.culled_error_bound(info["norms_a"], info["norms_b"], tau)
    slack = 1e-14 * np.linalg.norm(a) * np.linalg.norm(b)
    assert err <= blockwise * (1 + 1e-12) + slack
    assert blockwise <= total * (1 + 1e-12) + slack
    _, i2 = alg1.spamm_alg1(a, b, tau)
    assert err <= i2["culled_bound"] * (1 + 1e-12) + slack


def test_huge_tau_gives_zero_and_sets_are_nested():
    a = syn.decaying(150, seed=21, rate=0.05)
    b = syn.decaying(150, seed=22, rate=0.05)
    big = np.linalg.norm(a) * np.linalg.norm(b)
    c, info = so.spamm(a, b, big)
    assert info["n_exec"] == 0 and not np.any(c)
    na, nbn = so.leaf_norms(so.pad(a)), so.leaf_norms(so.pad(b))
    prev = None
    for tau in [0.0, 1e-8, 1e-5, 1e-3, 1e-1, 10.0, big]:
        m = so.executed_mask(na, nbn, tau)
        if prev is not None:
            assert np.all(prev | ~m)      # E(tau) shrinks as tau grows
        prev = m


def test_block_diagonal_products_stay_block_diagonal():
    a = np.zeros((128, 128))
    a[:64, :64] = syn.decaying(64, seed=1)
    a[64:, 64:] = syn.decaying(64, seed=2)
    c, _ = so.spamm(a, a, 1e-12)
    assert not np.any(c[:64, 64:]) and not np.any(c[64:, :64])
    np.testing.assert_allclose(c, a @ a, rtol=0, atol=1e-12 * np.linalg.norm(a) ** 2)


def test_symmetric_square_is_symmetric():
    a = syn.decaying(250, seed=31, rate=0.05, symmetric=True)
    c, _ = so.spamm(a, a, 1e-4)
    np.testing.assert_allclose(c, c.T, rtol=0, atol=1e-13 * np.abs(c).max())


@pytest.mark.parametrize("tau", [-1.0, float("nan"), float("inf")])
def test_invalid_tau_rejected(tau):
    a = np.eye(4)
    with pytest.raises(ValueError):
        so.spamm(a, a, tau)
    with pytest.raises(ValueError):
        alg1.spamm_alg1(a, a, tau)


def test_depth_zero_leaf_is_tested():
    a = np.eye(4)                                # ||A|| = 2 exactly, product of norms 4
    c, info = so.spamm(a, a, 4.0)                # tie: culled (strict > of Eq. 4)
    assert info["n_exec"] == 0 and not np.any(c)
    c2, i2 = alg1.spamm_alg1(a, a, 4.0)
    assert i2["n_exec"] == 0 and not np.any(c2)
    c3, i3 = alg1.spamm_alg1(a, a, 3.99)
    assert i3["n_exec"] == 1
    np.testing.assert_allclose(c3[:4, :4], a @ a)


def test_upper_count_is_the_restriction_of_the_executed_set(rng):
    """n_exec_upper counts the executed (i, j, k) with i <= j (brute force);
    for a symmetric matrix the task sets of (i, j) and (j, i) coincide, so
    n_exec = 2 n_exec_upper - (executed products of diagonal blocks)."""
    n = 200
    a = rng.standard_normal((n, n)) * np.exp(-np.abs(np.subtract.outer(np.arange(n), np.arange(n))) / 30)
    a = a + a.T
    tau = 0.3
    _, info = so.spamm(a, a, tau)
    na = info["norms_a"]
    nb = na.shape[0]
    upper = diag = 0
    for i in range(nb):
        for j in range(nb):
            for k in range(nb):
                if na[i, k] * na[k, j] > tau:
                    upper += i <= j
                    diag += i == j
    assert info["n_exec_upper"] == upper
    assert info["n_exec"] == 2 * upper - diag
