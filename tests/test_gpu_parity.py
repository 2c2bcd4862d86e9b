"""Parity of the HIP path against the FP64 oracle, through the C ABI.

Every case runs the device library (libspamm.so) on cuda:0 and compares
with the oracle on the same seeded inputs: element by element at sizes the
oracle finishes in seconds (several tiles and a ragged tail), and on sampled
blocks or size-independent properties at the full workload sizes.

Tolerances:
* FP64 leaves: products differ from the oracle only by summation order,
  |error| <= ~2 * 32 * (#k) * u64 * sum |a||b| -> relative 1e-13.
* FP32 leaves: FP32 tiles (relative rounding 2^-24 ~ 6e-8 per input) and
  FP32 accumulation over 32 * (#k) terms; the relative Frobenius error is
  held to 1e-5 (the stated FP32 target).
* Task lists: identical sets, except products inside the tie band
  |‖A_ik‖‖B_kj‖ - tau| <= 1e-12 tau, where norm rounding may decide either way.
"""
import numpy as np
import pytest

from oracle import alg1
from oracle import sp2_oracle as sp2o
from oracle import spamm_oracle as so
from watergen import synthetic as syn
from watergen import water_cluster, water_cluster_torch

pytestmark = pytest.mark.gpu

TIE = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def lib():
    import paper_1403_7458_amd as sp
    sp.load()
    return sp


def to_dev(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def morton(i, j):
    z = 0
    for bit in range(16):
        z |= ((i >> bit) & 1) << (2 * bit + 1)
        z |= ((j >> bit) & 1) << (2 * bit)
    return z


SIZES = [1, 31, 32, 33, 100, 257, 300]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", SIZES)
def test_tree_norms_match_oracle(torch_dev, lib, n, prec):
    a = syn.decaying(n, seed=n, rate=0.05)
    m = lib.spamm_tree_build(to_dev(torch_dev, a), prec)
    info = m.info()
    ap = so.pad(a)
    tiers = so.tier_norms(so.leaf_norms(ap))
    assert info["n"] == n and info["n_pad"] == ap.shape[0] and info["depth"] == len(tiers) - 1
    assert info["n_blocks"] == int((tiers[-1] > 0).sum())
    got = lib.spamm_matrix_norms(m)
    for g, o in zip(got, tiers):
        np.testing.assert_allclose(g, o, rtol=1e-13, atol=0)
    assert info["frobenius"] == pytest.approx(np.linalg.norm(a), rel=1e-13)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_to_dense_roundtrip_host_and_device(torch_dev, lib, prec):
    a = syn.decaying(300, seed=7, rate=0.02)
    ref = a if prec == "fp64" else a.astype(np.float32).astype(np.float64)
    m_dev = lib.spamm_tree_build(to_dev(torch_dev, a), prec)
    m_host = lib.spamm_tree_build(a, prec)              # host input, staged by the library
    np.testing.assert_array_equal(lib.spamm_to_dense(m_dev), ref)
    np.testing.assert_array_equal(lib.spamm_to_dense(m_host), ref)
    torch, dev = torch_dev
    out = torch.full((300, 300), np.nan, dtype=torch.float64, device=dev)
    lib.spamm_to_dense(m_dev, out=out)
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


def test_exact_zero_blocks_are_not_stored(torch_dev, lib):
    a = syn.decaying(128, seed=3)
    a[0:32, 64:96] = 0.0
    a[96:128, 0:32] = 0.0
    m = lib.spamm_tree_build(to_dev(torch_dev, a), "fp64")
    assert m.info()["n_blocks"] == 16 - 2
    np.testing.assert_array_equal(lib.spamm_to_dense(m), a)


def oracle_tasks(na, nbn, tau):
    """Per C block (i, j) in Morton order: ascending k with ||A_ik|| ||B_kj|| > tau,
    plus the tie-band triples whose decision may go either way."""
    nb = na.shape[0]
    prod = na[:, None, :] * nbn.T[None, :, :]            # [i, j, k]
    keep = prod > tau
    tie = np.abs(prod - tau) <= TIE * tau
    return keep, tie


def check_task_list(t, na, nbn, tau):
    keep, tie = oracle_tasks(na, nbn, tau)
    nb = na.shape[0]
    ci, cj, cp, ks = t["c_i"], t["c_j"], t["c_ptr"], t["k"]
    # Morton order of the C blocks, ascending k inside each.
    codes = [morton(int(i), int(j)) for i, j in zip(ci, cj)]
    assert codes == sorted(codes) and len(set(codes)) == len(codes)
    assert cp[0] == 0 and cp[-1] == len(ks) and np.all(np.diff(cp) > 0)
    got = np.zeros((nb, nb, nb), bool)
    for x in range(len(ci)):
        kk = ks[cp[x]:cp[x + 1]]
        assert np.all(np.diff(kk) > 0)
        got[ci[x], cj[x], kk] = True
    diff = got != keep
    assert not np.any(diff & ~tie), "task set differs outside the tie band"
    return int(got.sum()), int(diff.sum())


@pytest.mark.parametrize("tau", [0.0, 1e-4, 1e-2, 1e-1, 1.0])
@pytest.mark.parametrize("n", [33, 300, 700])
def test_cull_task_list_matches_oracle(torch_dev, lib, n, tau):
    a = syn.decaying(n, seed=11 + n, rate=0.04)
    b = syn.decaying(n, seed=12 + n, rate=0.07)
    ma = lib.spamm_tree_build(to_dev(torch_dev, a), "fp64")
    mb = lib.spamm_tree_build(to_dev(torch_dev, b), "fp64")
    t = lib.spamm_cull(ma, mb, tau)
    na, nbn = so.leaf_norms(so.pad(a)), so.leaf_norms(so.pad(b))
    check_task_list(t, na, nbn, tau)
    # The breadth-first tier walk of the oracle gives the same set (Algs. 2-3).
    if n <= 300:
        bf = so.executed_set_breadth_first(so.tier_norms(na), so.tier_norms(nbn), tau)
        assert len(bf) == len(t["k"])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
@pytest.mark.parametrize("tau", [0.0, 1e-3, 1e-1])
@pytest.mark.parametrize("n", [33, 100, 300, 700])
def test_multiply_matches_oracle(torch_dev, lib, n, tau, prec, tol):
    a = syn.decaying(n, seed=n, rate=0.05)
    b = syn.decaying(n, seed=n + 1, rate=0.08)
    ma = lib.spamm_tree_build(to_dev(torch_dev, a), prec)
    mb = lib.spamm_tree_build(to_dev(torch_dev, b), prec)
    mc, st = lib.spamm_multiply(ma, mb, tau)
    c = lib.spamm_to_dense(mc)
    cref, info = so.spamm(a, b, tau)
    assert rel(c, cref[:n, :n]) <= tol
    assert st["n_exec"] == info["n_exec"]
    nb = so.padded_size(n) // 32
    assert st["n_dense"] == nb ** 3
    na, nbn = info["norms_a"], info["norms_b"]
    assert st["n_nonzero_pairs"] == int(((na[:, None, :] > 0) & (nbn.T[None, :, :] > 0)).sum())
    # Stored C blocks: exactly those with an executed product.
    assert mc.info()["n_blocks"] == st["n_cblocks"]
    assert st["n_cblocks"] == int((so.executed_mask(na, nbn, tau).sum(axis=2) > 0).sum())
    # Error bound: the sum over maximal culled octree nodes, as the recursive
    # Alg. 1 oracle accumulates it; it bounds the true error.
    _, inf1 = alg1.spamm_alg1(a, b, tau)
    assert st["err_bound"] == pytest.approx(inf1["culled_bound"], rel=1e-10, abs=1e-300)
    exact = a @ b
    assert np.linalg.norm(c - exact) <= st["err_bound"] * (1 + 1e-12) + tol * np.linalg.norm(exact) + 1e-300


@pytest.mark.parametrize("n", [64, 250])
def test_multiply_tau_zero_equals_dense_gemm(torch_dev, lib, n):
    a = syn.decaying(n, seed=5, rate=0.01)
    b = syn.decaying(n, seed=6, rate=0.01)
    mc, st = lib.spamm_multiply(lib.spamm_tree_build(to_dev(torch_dev, a), "fp64"),
                                lib.spamm_tree_build(to_dev(torch_dev, b), "fp64"), 0.0)
    assert rel(lib.spamm_to_dense(mc), a @ b) <= 1e-13
    assert st["err_bound"] == 0.0


def test_multiply_huge_tau_culls_everything(torch_dev, lib):
    a = syn.decaying(200, seed=9)
    ma = lib.spamm_tree_build(to_dev(torch_dev, a), "fp32")
    tau = 1.01 * np.linalg.norm(a) ** 2
    mc, st = lib.spamm_multiply(ma, ma, tau)
    assert st["n_exec"] == 0 and st["n_cblocks"] == 0 and mc.info()["n_blocks"] == 0
    assert np.all(lib.spamm_to_dense(mc) == 0.0)
    assert lib.spamm_cull(ma, ma, tau)["k"].size == 0


def test_multiply_block_diagonal_and_symmetric(torch_dev, lib):
    n = 256
    a = np.zeros((n, n))
    for b0 in range(0, n, 64):
        blk = syn.decaying(64, seed=b0, rate=0.1, symmetric=True)
        a[b0:b0 + 64, b0:b0 + 64] = blk
    ma = lib.spamm_tree_build(to_dev(torch_dev, a), "fp64")
    mc, st = lib.spamm_multiply(ma, ma, 1e-6)
    c = lib.spamm_to_dense(mc)
    t = lib.spamm_cull(ma, ma, 1e-6)
    for i, j in zip(t["c_i"], t["c_j"]):
        assert i // 2 == j // 2, "off-diagonal block of a block-diagonal product"
    np.testing.assert_allclose(c, c.T, rtol=0, atol=1e-14 * np.abs(c).max())


def test_multiply_is_deterministic(torch_dev, lib):
    a = syn.decaying(500, seed=21, rate=0.03)
    ma = lib.spamm_tree_build(to_dev(torch_dev, a), "fp32")
    c1 = lib.spamm_to_dense(lib.spamm_multiply(ma, ma, 1e-3)[0])
    c2 = lib.spamm_to_dense(lib.spamm_multiply(ma, ma, 1e-3)[0])
    np.testing.assert_array_equal(c1, c2)
    # Without statistics: the same product (only the statistics passes go).
    c3, st3 = lib.spamm_multiply(ma, ma, 1e-3, stats=False)
    assert st3 is None
    np.testing.assert_array_equal(lib.spamm_to_dense(c3), c1)


def test_error_paths(torch_dev, lib):
    a = syn.decaying(64, seed=1)
    ma = lib.spamm_tree_build(to_dev(torch_dev, a), "fp64")
    mb = lib.spamm_tree_build(to_dev(torch_dev, syn.decaying(96, seed=2)), "fp64")
    m32 = lib.spamm_tree_build(to_dev(torch_dev, a), "fp32")
    with pytest.raises(lib.SpammError) as e:
        lib.spamm_multiply(ma, mb, 0.0)
    assert e.value.code == -6
    with pytest.raises(lib.SpammError) as e:
        lib.spamm_multiply(ma, m32, 0.0)
    assert e.value.code == -6
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(lib.SpammError) as e:
            lib.spamm_multiply(ma, ma, bad)
        assert e.value.code == -1
    b = a.copy()
    b[3, 5] = np.nan
    with pytest.raises(lib.SpammError) as e:
        lib.spamm_tree_build(to_dev(torch_dev, b), "fp64")
    assert e.value.code == -2
    f = syn.decaying(64, seed=4, symmetric=True)
    out = np.zeros((64, 64))
    with pytest.raises(lib.SpammError) as e:
        lib.sp2_solve(to_dev(torch_dev, f), 65, 0.0, out=out)
    assert e.value.code == -1
    g = f.copy()
    g[1, 2] += 1e-6
    with pytest.raises(lib.SpammError) as e:
        lib.sp2_solve(to_dev(torch_dev, g), 10, 0.0, out=out)
    assert e.value.code == -3
    g = f.copy()
    g[7, 7] = np.inf
    with pytest.raises(lib.SpammError) as e:
        lib.sp2_solve(to_dev(torch_dev, g), 10, 0.0, out=out)
    assert e.value.code == -2
    assert np.all(out == 0.0), "output untouched on error"


def eigh_projector(f, n_occ):
    w, v = np.linalg.eigh(f)
    return v[:, :n_occ] @ v[:, :n_occ].T


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("tau", [0.0, 1e-6])
def test_sp2_fp64_matches_oracle(torch_dev, lib, tau, symmetric):
    w = water_cluster(8, 1.5, 2)
    p, st = lib.sp2_solve(to_dev(torch_dev, w.f), w.n_occ, tau, precision="fp64",
                          symmetric=symmetric)
    r = sp2o.sp2(w.f, w.n_occ, tau)
    assert st["iterations"] == r.iterations
    assert st["branches"] == r.branches
    assert st["symmetric"] == symmetric
    # Symmetric squares execute the products of the C blocks with i <= j.
    assert st["n_exec"] == (r.n_exec_upper if symmetric else r.n_exec)
    if symmetric:
        np.testing.assert_array_equal(p, p.T)
    np.testing.assert_allclose(st["traces"], r.traces, rtol=1e-12)
    np.testing.assert_allclose(st["errors"], r.errors, rtol=1e-6, atol=1e-12)
    assert rel(p, r.p) <= 1e-10
    assert st["eps_min"] == pytest.approx(r.eps_min, rel=1e-14)
    assert st["eps_max"] == pytest.approx(r.eps_max, rel=1e-14)
    if tau == 0.0:
        assert rel(p, eigh_projector(w.f, w.n_occ)) <= 1e-8
        assert abs(np.trace(p) - w.n_occ) <= 1e-8


def test_sp2_fp32_matches_oracle(torch_dev, lib):
    w = water_cluster(8, 1.5, 2)
    torch, dev = torch_dev
    out = torch.empty((w.n, w.n), dtype=torch.float64, device=dev)
    p, st = lib.sp2_solve(to_dev(torch_dev, w.f), w.n_occ, 1e-6, out=out, precision="fp32")
    r = sp2o.sp2(w.f, w.n_occ, 1e-6)
    p = p.cpu().numpy()
    assert rel(p, r.p) <= 1e-5
    assert abs(np.trace(p) - w.n_occ) <= 1e-4
    assert st["branches"][:20] == r.branches[:20]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3", "bf16"])
def test_sp2_symmetric_squares_match_full_squares(torch_dev, lib, prec):
    """Upper-triangle squares with mirrored blocks against full squares: the
    same iteration count and branches, about half the leaf products, P equal
    to rounding (exactly symmetric), and the full form is used when F is not
    exactly symmetric."""
    w = water_cluster(16, 1.8, 4)
    f = to_dev(torch_dev, w.f)
    ps, ss = lib.sp2_solve(f, w.n_occ, 1e-6, precision=prec)
    pf, sf = lib.sp2_solve(f, w.n_occ, 1e-6, precision=prec, symmetric=False)
    assert ss["symmetric"] and not sf["symmetric"]
    np.testing.assert_array_equal(ps, ps.T)
    tol = {"fp64": 1e-12, "fp32": 1e-5, "fp16x3": 1e-5, "bf16": 1e-1}[prec]
    assert rel(ps, pf) <= tol
    if prec in ("fp64", "fp32"):
        assert ss["branches"] == sf["branches"] and ss["iterations"] == sf["iterations"]
        for a, b in zip(ss["n_exec"], sf["n_exec"]):
            assert b / 2 <= a <= b / 2 + b / 8      # the diagonal blocks count once
    g = w.f.copy()
    g[3, 7] *= 1.0 + 2.0 ** -50                   # within the symmetry check, not exact
    _, sg = lib.sp2_solve(to_dev(torch_dev, g), w.n_occ, 1e-6, precision=prec)
    assert not sg["symmetric"]


def test_sp2_c1_workload_fp64(torch_dev, lib):
    """30 molecules, N = 750 -> 1024, FP64, tau = 1e-10, until ||X^2 - X|| < 1e-8."""
    w = water_cluster(30, 1.5, 0)
    p, st = lib.sp2_solve(to_dev(torch_dev, w.f), w.n_occ, 1e-10, precision="fp64")
    r = sp2o.sp2(w.f, w.n_occ, 1e-10, product=alg1.spamm_alg1)
    assert st["stop"] == "converged" and r.stop == sp2o.STOP_CONVERGED
    assert st["iterations"] == r.iterations and st["branches"] == r.branches
    assert rel(p, r.p) <= 1e-9
    assert abs(np.trace(p) - w.n_occ) <= 1e-6
    assert sp2o.idempotency_error(p) <= 1e-6


def test_sp2_closed_forms(torch_dev, lib):
    # F = diag(-1.., +1..): X_0 is already the projector, e_0 = 0.
    d = np.array([-1.0] * 40 + [1.0] * 60)
    f = np.diag(d)
    p, st = lib.sp2_solve(to_dev(torch_dev, f), 40, 0.0, precision="fp64")
    np.testing.assert_array_equal(p, np.diag((d < 0).astype(float)))
    assert st["iterations"] == 1 and st["errors"][0] == 0.0 and st["stop"] == "converged"
    # 2 x 2, n_occ = 1: projector on the lower eigenvector.
    f = np.array([[0.3, -0.7], [-0.7, 1.1]])
    p, st = lib.sp2_solve(f, 1, 0.0, precision="fp64")
    np.testing.assert_allclose(p, eigh_projector(f, 1), atol=1e-9)


def test_sp2_max_iter_returns_last_iterate(torch_dev, lib):
    w = water_cluster(6, 1.5, 0)
    p, st = lib.sp2_solve(to_dev(torch_dev, w.f), w.n_occ, 0.0, precision="fp64", max_iter=3)
    assert st["status"] == 1 and st["stop"] == "max_iter" and st["iterations"] == 3
    r = sp2o.sp2(w.f, w.n_occ, 0.0, max_iter=3)
    assert rel(p, r.p) <= 1e-13


def test_spamm_multiply_c2_sampled(torch_dev, lib):
    """150 molecules, N = 3750 -> 4096, FP32 leaves: X_0 * X_0 at three tau."""
    w = water_cluster(150, 1.5, 0)
    lo, hi = sp2o.gershgorin(w.f)
    x0 = sp2o.initial_x(w.f, lo, hi, 4096)
    mx = lib.spamm_tree_build(to_dev(torch_dev, x0[:w.n, :w.n]), "fp32")
    na = so.leaf_norms(x0)
    rng = np.random.Generator(np.random.PCG64(0))
    for tau in (1e-8, 1e-6, 1e-4):
        mc, st = lib.spamm_multiply(mx, mx, tau)
        keep, tie = oracle_tasks(na, na, tau)
        assert abs(st["n_exec"] - int(keep.sum())) <= int(tie.sum())
        c = lib.spamm_to_dense(mc)
        rows = sorted(set(rng.integers(0, 118, 4).tolist()) | {0, 117})
        cols = sorted(set(rng.integers(0, 118, 4).tolist()) | {5})
        cref, _ = so.spamm(x0, x0, tau, rows=rows, cols=cols)
        for i in rows:
            for j in cols:
                g = c[i * 32:(i + 1) * 32, j * 32:(j + 1) * 32]
                o = cref[i * 32:(i + 1) * 32, j * 32:(j + 1) * 32][:g.shape[0], :g.shape[1]]
                # FP32 error scale of block (i, j): sum over its executed k of
                # ||A_ik|| ||B_kj||, the size of the terms being added.
                ks = so.executed_ks(na, na, tau, i, j)
                scale = float((na[i, ks] * na[ks, j]).sum())
                assert np.linalg.norm(g - o) <= 1e-5 * scale + 1e-30


@pytest.mark.slow
def test_spamm_multiply_c3_sampled(torch_dev, lib):
    """1000 molecules, N = 25000 -> 32768 (nb 1024, depth 10), FP32 leaves:
    the Gershgorin bounds, the executed-task count of X_0 * X_0 at tau 1e-6
    and sampled C blocks against the oracle, at the full size."""
    torch, dev = torch_dev
    f_dev, n_occ = water_cluster_torch(1000, 1.5, 0, device=dev)
    n = f_dev.shape[0]
    mx, glo, ghi = lib.sp2_initial_guess(f_dev, "fp32")
    f = f_dev.cpu().numpy()
    lo, hi = sp2o.gershgorin(f)
    assert glo == pytest.approx(lo, rel=1e-13) and ghi == pytest.approx(hi, rel=1e-13)
    x0 = sp2o.initial_x(f, lo, hi, 32768)
    del f
    na = so.leaf_norms(x0)
    tau = 1e-6
    mc, st = lib.spamm_multiply(mx, mx, tau)
    keep = tie = 0
    for i in range(na.shape[0]):                      # the flat test, row by row
        prod = na[i, None, :] * na.T
        keep += int((prod > tau).sum())
        tie += int((np.abs(prod - tau) <= TIE * tau).sum())
    assert abs(st["n_exec"] - keep) <= tie
    assert st["n_dense"] == 1024 ** 3
    c = torch.empty((n, n), dtype=torch.float64, device=dev)
    lib.spamm_to_dense(mc, out=c)
    rng = np.random.Generator(np.random.PCG64(1))
    rows = sorted(set(rng.integers(0, 782, 4).tolist()) | {0, 781})
    cols = sorted(set(rng.integers(0, 782, 4).tolist()) | {390})
    cref, _ = so.spamm(x0, x0, tau, rows=rows, cols=cols)
    for i in rows:
        for j in cols:
            g = c[i * 32:(i + 1) * 32, j * 32:(j + 1) * 32].cpu().numpy()
            o = cref[i * 32:(i + 1) * 32, j * 32:(j + 1) * 32][:g.shape[0], :g.shape[1]]
            ks = so.executed_ks(na, na, tau, i, j)
            scale = float((na[i, ks] * na[ks, j]).sum())
            assert np.linalg.norm(g - o) <= 1e-5 * scale + 1e-30


@pytest.mark.slow
def test_sp2_c3_full_size_properties(torch_dev, lib):
    """1000-molecule SP2 with FP32 leaves at tau 1e-6: stops on the stall
    rule below its floor, and P is symmetric, has trace n_occ and is
    idempotent to the FP32 floor (properties that hold at any size; the
    oracle is checked on the same system block by block above)."""
    torch, dev = torch_dev
    f_dev, n_occ = water_cluster_torch(1000, 1.5, 0, device=dev)
    p = torch.empty_like(f_dev)
    _, st = lib.sp2_solve(f_dev, n_occ, 1e-6, out=p, precision="fp32")
    floor = 1e-3 * np.sqrt(n_occ)
    assert st["stop"] in ("converged", "stalled") and st["errors"][-1] < floor
    assert float(torch.linalg.norm(p - p.T)) <= 1e-4 * float(torch.linalg.norm(p))
    assert abs(float(torch.trace(p)) - n_occ) <= 0.1
    assert float(torch.linalg.norm(p @ p - p)) <= floor


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sp2_initial_guess_matches_oracle(torch_dev, lib, prec):
    w = water_cluster(12, 1.5, 1)
    x0, lo, hi = lib.sp2_initial_guess(to_dev(torch_dev, w.f), prec)
    olo, ohi = sp2o.gershgorin(w.f)
    assert lo == pytest.approx(olo, rel=1e-14) and hi == pytest.approx(ohi, rel=1e-14)
    ox = sp2o.initial_x(w.f, olo, ohi, so.padded_size(w.n))
    got = lib.spamm_to_dense(x0)
    ref = ox[:w.n, :w.n] if prec == "fp64" else ox[:w.n, :w.n].astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-16)
    # Leaf norms of the FP64 values of X_0, in either precision.
    for g, o in zip(lib.spamm_matrix_norms(x0), so.tier_norms(so.leaf_norms(ox))):
        np.testing.assert_allclose(g, o, rtol=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_leaf_kernels_agree_bitwise(torch_dev, lib, prec, monkeypatch):
    """Every leaf-product kernel (one wave per C block, 2 x 2 and 4 x 4 block
    groups) adds the same products in the same ascending k order."""
    w = water_cluster(40, 1.5, 3)
    f = to_dev(torch_dev, w.f)
    x0, _, _ = lib.sp2_initial_guess(f, prec)
    out = {}
    sym = {}
    for kern in ("block", "2x2", "4x4", "w2x2", "w2x2s"):
        monkeypatch.setenv("SPAMM_LEAF_KERNEL", kern)
        c, st = lib.spamm_multiply(x0, x0, 1e-7)
        p, s2 = lib.sp2_solve(f, w.n_occ, 1e-7, precision=prec, max_iter=6, symmetric=False)
        out[kern] = (lib.spamm_to_dense(c), st["n_exec"], p, s2["errors"])
        if kern in ("block", "w2x2", "w2x2s"):   # the kernels with a mirrored epilogue
            sym[kern] = lib.sp2_solve(f, w.n_occ, 1e-7, precision=prec, max_iter=6)
    ref = out["block"]
    for kern in ("2x2", "4x4", "w2x2", "w2x2s"):
        np.testing.assert_array_equal(out[kern][0], ref[0])
        assert out[kern][1] == ref[1]
        np.testing.assert_array_equal(out[kern][2], ref[2])
        assert out[kern][3] == ref[3]
    for kern in ("w2x2", "w2x2s"):
        np.testing.assert_array_equal(sym[kern][0], sym["block"][0])
        assert sym[kern][1]["errors"] == sym["block"][1]["errors"]
        assert sym[kern][1]["symmetric"]


# ---- 16-bit forms ----------------------------------------------------------------
#
# Tolerances follow the unit roundoff u of each form: BF16 u = 2^-8, FP16
# u = 2^-11, BF16X3 (hi + lo) u ~ 2^-16, FP16X3 u ~ 2^-22, with FP32
# accumulation (2^-24 per addition) on top.  A product's relative Frobenius
# error is a few u (inputs rounded once each, errors averaging over the 32 k
# of a leaf and over the k of a block): held to 2.5u, 4u, 3u and 8u.

HALF_TOL = {"bf16": 1e-2, "fp16": 2e-3, "bf16x3": 5e-5, "fp16x3": 2e-6}


def round_bf16(x):
    f = np.asarray(x, np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return b.view(np.float32).astype(np.float64)


def round_fp16(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


@pytest.mark.parametrize("n", [20, 300])
def test_half_tiles_roundtrip(torch_dev, lib, n):
    a = syn.decaying(n, seed=31 + n, rate=0.03)
    np.testing.assert_array_equal(lib.spamm_to_dense(lib.spamm_tree_build(to_dev(torch_dev, a), "bf16")),
                                  round_bf16(a))
    # FP16: rounded to nearest (directly or through FP32, which may differ in
    # the last bit): within half an FP16 unit in the last place, plus a hair.
    d = lib.spamm_to_dense(lib.spamm_tree_build(to_dev(torch_dev, a), "fp16"))
    ulp = np.spacing(np.abs(round_fp16(a)).astype(np.float16)).astype(np.float64)
    assert np.all(np.abs(d - a) <= 0.5 * ulp * (1 + 2.0 ** -9))
    assert np.mean(d == round_fp16(a)) > 0.999
    # Split forms: hi + lo reproduces the value to the hi + lo precision.
    d = lib.spamm_to_dense(lib.spamm_tree_build(to_dev(torch_dev, a), "bf16x3"))
    assert np.all(np.abs(d - a) <= 2.0 ** -16 * np.abs(a) + 1e-38)
    d = lib.spamm_to_dense(lib.spamm_tree_build(to_dev(torch_dev, a), "fp16x3"))
    assert np.all(np.abs(d - a) <= 2.0 ** -21 * np.abs(a) + 2.0 ** -24 * 2.0 ** -11)
    # Norms stay those of the FP64 input.
    for g, o in zip(lib.spamm_matrix_norms(lib.spamm_tree_build(to_dev(torch_dev, a), "bf16")),
                    so.tier_norms(so.leaf_norms(so.pad(a)))):
        np.testing.assert_allclose(g, o, rtol=1e-13)


@pytest.mark.parametrize("prec", list(HALF_TOL))
@pytest.mark.parametrize("n,tau", [(20, 0.0), (300, 1e-3), (700, 1e-2)])
def test_half_multiply_matches_oracle(torch_dev, lib, prec, n, tau):
    a = syn.decaying(n, seed=n, rate=0.05)
    b = syn.decaying(n, seed=n + 1, rate=0.08)
    ma = lib.spamm_tree_build(to_dev(torch_dev, a), prec)
    mb = lib.spamm_tree_build(to_dev(torch_dev, b), prec)
    mc, st = lib.spamm_multiply(ma, mb, tau)
    cref, info = so.spamm(a, b, tau)
    assert st["n_exec"] == info["n_exec"]          # culling uses FP64 norms in every form
    assert rel(lib.spamm_to_dense(mc), cref[:n, :n]) <= HALF_TOL[prec]


def test_fp16_range_checks(torch_dev, lib):
    a = np.full((64, 64), 1.0)
    a[3, 4] = 7e4
    with pytest.raises(lib.SpammError) as e:
        lib.spamm_tree_build(to_dev(torch_dev, a), "fp16")
    assert e.value.code == -1
    big = np.full((64, 64), 100.0)                  # products reach 64 * 1e4 > 65504
    mb = lib.spamm_tree_build(to_dev(torch_dev, big), "fp16x3")
    with pytest.raises(lib.SpammError) as e:
        lib.spamm_multiply(mb, mb, 0.0)
    assert e.value.code == -2
    mb = lib.spamm_tree_build(to_dev(torch_dev, big), "bf16")   # BF16 has FP32's range
    c, _ = lib.spamm_multiply(mb, mb, 0.0)
    assert np.all(lib.spamm_to_dense(c) == round_bf16(640000.0))


SP2_HALF_TOL = {"fp16x3": 1e-5, "bf16x3": 3e-4, "fp16": 2e-2, "bf16": 1e-1}


@pytest.mark.parametrize("prec", list(SP2_HALF_TOL))
def test_half_sp2_against_fp64_oracle(torch_dev, lib, prec):
    """SP2 error of each 16-bit form against the FP64 oracle at the same tau,
    on a well-gapped matrix (gap 0.5 of the spectrum width ~ 3)."""
    f = syn.random_symmetric_with_gap(200, 60, seed=3, gap=0.5)
    r = sp2o.sp2(f, 60, 1e-6)
    p, st = lib.sp2_solve(to_dev(torch_dev, f), 60, 1e-6, precision=prec)
    p = p.cpu().numpy() if hasattr(p, "cpu") else p
    assert st["stop"] in ("converged", "stalled")
    assert rel(p, r.p) <= SP2_HALF_TOL[prec]
    assert abs(np.trace(p) - 60) <= 60 * SP2_HALF_TOL[prec]
