"""Pins of the SP2 oracle: eigendecomposition, scalar recurrence, closed forms."""
import math

import numpy as np
import pytest

from oracle import alg1
from oracle import sp2_oracle as sp
from watergen import synthetic as syn
from watergen import water_cluster


def eigh_projector(f, n_occ):
    w, v = np.linalg.eigh(f)
    return v[:, :n_occ] @ v[:, :n_occ].T


@pytest.mark.parametrize("n,n_occ,seed", [(40, 10, 1), (100, 37, 2), (129, 64, 3), (256, 100, 4)])
def test_tau_zero_equals_eigh_projector(n, n_occ, seed):
    f = syn.random_symmetric_with_gap(n, n_occ, seed=seed, gap=0.5)
    r = sp.sp2(f, n_occ, 0.0)
    p = eigh_projector(f, n_occ)
    assert r.stop == sp.STOP_CONVERGED
    assert np.linalg.norm(r.p - p) <= 1e-8
    assert abs(np.trace(r.p) - n_occ) <= 1e-8
    assert sp.idempotency_error(r.p) < 1e-8
    assert np.linalg.norm(r.p @ f - f @ r.p) <= 1e-8 * np.linalg.norm(f)


@pytest.mark.parametrize("molecules,seed", [(4, 0), (8, 2), (10, 2)])
def test_water_cluster_tau_zero_equals_eigh(molecules, seed):
    w = water_cluster(molecules, 1.5, seed)
    ev = np.linalg.eigvalsh(w.f)
    lo, hi = sp.gershgorin(w.f)
    gap = (ev[w.n_occ] - ev[w.n_occ - 1]) / (hi - lo)
    assert gap >= 1e-3, "seed chosen for a scaled gap >= 1e-3"
    r = sp.sp2(w.f, w.n_occ, 0.0)
    assert np.linalg.norm(r.p - eigh_projector(w.f, w.n_occ)) <= 1e-8
    assert abs(np.trace(r.p) - w.n_occ) <= 1e-8


def scalar_sp2(lams, n_occ, tol, max_iter, stall_floor=1e-3):
    floor = stall_floor * math.sqrt(max(n_occ, 1))
    """The same recurrence on the eigenvalues of X_0 (X_n is a polynomial in F)."""
    lam = np.array(lams, dtype=np.float64)
    bits, errs = [], []
    for it in range(max_iter):
        t = lam.sum()
        e = math.sqrt(((lam * lam - lam) ** 2).sum())
        sq = t > n_occ
        lam = lam * lam if sq else 2 * lam - lam * lam
        bits.append(1 if sq else 0)
        errs.append(e)
        if e < tol:
            break
        if it >= 2 and e < floor and e >= errs[it - 2]:
            break
    return bits, errs


@pytest.mark.parametrize("molecules,seed", [(4, 0), (12, 5)])
def test_branch_sequence_matches_scalar_recurrence(molecules, seed):
    w = water_cluster(molecules, 1.5, seed)
    lo, hi = sp.gershgorin(w.f)
    lam0 = (hi - np.linalg.eigvalsh(w.f)) / (hi - lo)
    bits, errs = scalar_sp2(lam0, w.n_occ, 1e-8, 100)
    r = sp.sp2(w.f, w.n_occ, 0.0)
    assert r.branches == bits
    assert r.iterations == len(bits)
    np.testing.assert_allclose(r.errors, errs, rtol=1e-6, atol=1e-11)
    # Traces agree with sums of the transformed eigenvalues.
    assert abs(r.traces[0] - lam0.sum()) < 1e-10


def test_gershgorin_contains_spectrum():
    w = water_cluster(20, 1.5, 3)
    lo, hi = sp.gershgorin(w.f)
    ev = np.linalg.eigvalsh(w.f)
    assert lo <= ev[0] and hi >= ev[-1]
    f = np.array([[2.0, -1.0, 0.5], [-1.0, 0.0, 0.25], [0.5, 0.25, -3.0]])
    lo, hi = sp.gershgorin(f)
    assert lo == min(2 - 1.5, 0 - 1.25, -3 - 0.75) and hi == max(2 + 1.5, 0 + 1.25, -3 + 0.75)


def test_diagonal_f_gives_exact_zero_one_projector():
    g = syn.generator(9)
    d = g.permutation(np.linspace(-2.0, 3.0, 70))
    f = np.diag(d)
    n_occ = 25
    r = sp.sp2(f, n_occ, 0.0, tol=0.0)
    expect = np.diag((d <= np.sort(d)[n_occ - 1]).astype(float))
    assert np.max(np.abs(r.p - expect)) <= 1e-12


def test_idempotent_start_stops_immediately():
    # F = diag(-1 x 5, +1 x 20): X_0 = diag(1 x 5, 0 x 20) is already idempotent.
    f = np.diag([-1.0] * 5 + [1.0] * 20)
    r = sp.sp2(f, 5, 0.0)
    assert r.iterations == 1 and r.errors[0] == 0.0 and r.stop == sp.STOP_CONVERGED
    np.testing.assert_array_equal(r.p, np.diag([1.0] * 5 + [0.0] * 20))


@pytest.mark.parametrize("a,b,c", [(1.0, 0.3, -0.5), (-2.0, 1.0, 2.0), (0.1, -0.7, 0.4)])
def test_two_by_two_closed_form(a, b, c):
    f = np.array([[a, b], [b, c]])
    lam = 0.5 * (a + c) - math.sqrt(0.25 * (a - c) ** 2 + b * b)   # lower eigenvalue
    v = np.array([b, lam - a]) if abs(b) > 0 else np.array([1.0, 0.0])
    v /= np.linalg.norm(v)
    r = sp.sp2(f, 1, 0.0, tol=0.0)          # run to the rounding floor (stall rule)
    assert r.stop == sp.STOP_STALLED
    np.testing.assert_allclose(r.p, np.outer(v, v), atol=1e-12)


def test_block_diagonal_f_gives_blockwise_projector():
    f1 = syn.random_symmetric_with_gap(30, 10, seed=1, gap=0.8)
    f2 = syn.random_symmetric_with_gap(50, 20, seed=2, gap=0.8)
    f = np.zeros((80, 80))
    f[:30, :30], f[30:, 30:] = f1, f2
    r = sp.sp2(f, 30, 0.0, tol=0.0)
    np.testing.assert_allclose(r.p[:30, :30], eigh_projector(f1, 10), atol=1e-9)
    np.testing.assert_allclose(r.p[30:, 30:], eigh_projector(f2, 20), atol=1e-9)
    assert np.max(np.abs(r.p[:30, 30:])) <= 1e-12


def test_stop_rules():
    f = syn.random_symmetric_with_gap(60, 20, seed=7, gap=0.2)
    r = sp.sp2(f, 20, 0.0, max_iter=1)
    assert r.iterations == 1 and r.stop == sp.STOP_MAX_ITER
    r = sp.sp2(f, 20, 0.0, tol=1e9)
    assert r.iterations == 1 and r.stop == sp.STOP_CONVERGED
    r = sp.sp2(f, 20, 0.0, tol=1e9, min_iter=4)
    assert r.iterations == 4
    # Without the stall rule and with an unreachable tolerance the cap is hit.
    r = sp.sp2(f, 20, 0.0, tol=0.0, stall=False, max_iter=60)
    assert r.iterations == 60 and r.stop == sp.STOP_MAX_ITER
    # With it, the run stops at the rounding floor well before the cap.
    r = sp.sp2(f, 20, 0.0, tol=0.0, max_iter=200)
    assert r.stop == sp.STOP_STALLED and r.iterations < 200


def test_invalid_arguments():
    f = np.eye(4)
    with pytest.raises(ValueError):
        sp.sp2(f, 5, 0.0)
    with pytest.raises(ValueError):
        sp.sp2(f, 2, -1.0)
    with pytest.raises(ValueError):
        sp.sp2(np.ones((3, 4)), 1, 0.0)


def test_alg1_product_gives_same_sp2():
    w = water_cluster(12, 1.5, 5)
    r1 = sp.sp2(w.f, w.n_occ, 1e-6)
    r2 = sp.sp2(w.f, w.n_occ, 1e-6, product=alg1.spamm_alg1)
    assert r1.branches == r2.branches and r1.n_exec == r2.n_exec
    np.testing.assert_allclose(r2.p, r1.p, atol=1e-12)


def test_error_grows_with_tau():
    """Accumulated SpAMM error against the tau = 0 projector (Sec. 4.1 measure)."""
    w = water_cluster(10, 1.5, 2)
    ref = sp.sp2(w.f, w.n_occ, 0.0).p
    errs = []
    for tau in [1e-10, 1e-6, 1e-3]:
        p = sp.sp2(w.f, w.n_occ, tau).p
        errs.append(abs(sp.energy_error(w.f, ref, p)))
    assert errs[0] <= 1e-7 and errs[0] <= errs[2]
