"""CPU pins of the reference adaptive HSS compression (Algorithm 1)."""
import numpy as np
import pytest

import workloads
from oracle import hss


def _tree_ranges(lo, hi, leaf):
    """Index-halving tree as nested tuples (lo, hi, children) — written here
    independently of the oracle's tree code."""
    if hi - lo <= leaf:
        return (lo, hi, None)
    mid = lo + (hi - lo) // 2
    return (lo, hi, (_tree_ranges(lo, mid, leaf), _tree_ranges(mid, hi, leaf)))


def _exact_hss(n, leaf, r, seed, symmetric=False):
    """A dense matrix with exact HSS rank r: random D, leaf bases, transfer
    matrices and couplings assembled by the nested-basis formula of section 2.2."""
    g = np.random.Generator(np.random.PCG64(seed))
    A = np.zeros((n, n))

    def build(node):
        lo, hi, ch = node
        if ch is None:
            A[lo:hi, lo:hi] = g.standard_normal((hi - lo, hi - lo))
            U = g.standard_normal((hi - lo, r))
            V = U if symmetric else g.standard_normal((hi - lo, r))
            return U, V
        (U1, V1), (U2, V2) = build(ch[0]), build(ch[1])
        (l1, h1, _), (l2, h2, _) = ch
        B12 = g.standard_normal((r, r))
        B21 = B12.T if symmetric else g.standard_normal((r, r))
        A[l1:h1, l2:h2] = U1 @ B12 @ V2.T
        A[l2:h2, l1:h1] = U2 @ B21 @ V1.T
        Tu = g.standard_normal((2 * r, r))
        Tv = Tu if symmetric else g.standard_normal((2 * r, r))
        Ub = np.zeros((h2 - l1, 2 * r))
        Ub[:h1 - l1, :r] = U1
        Ub[h1 - l1:, r:] = U2
        Vb = np.zeros((h2 - l1, 2 * r))
        Vb[:h1 - l1, :r] = V1
        Vb[h1 - l1:, r:] = V2
        return Ub @ Tu, Vb @ Tv

    build(_tree_ranges(0, n, leaf))
    return A


@pytest.mark.parametrize("kind", ["gaussian", "sjlt", "srht"])
@pytest.mark.parametrize("symmetric", [True, False])
def test_exact_hss_recovery(kind, symmetric):
    n, leaf, r = 256, 32, 4
    A = _exact_hss(n, leaf, r, seed=10, symmetric=symmetric)
    if symmetric:
        A = 0.5 * (A + A.T)
    sk = hss.OracleSketcher(A, kind, seed=3, alpha=4, symmetric=symmetric)
    res = hss.compress(A, leaf, sk, d0=16, dd=16, eps_r=1e-12, eps_a=1e-14, symmetric=symmetric)
    assert res.converged
    assert hss.relative_error(A, res) < 1e-10
    # exact rank r is found at every non-root node
    assert set(res.ranks()) == {r}
    assert res.max_rank() == r


def test_block_diagonal_has_rank_zero():
    n, leaf = 128, 16
    g = np.random.Generator(np.random.PCG64(2))
    A = np.zeros((n, n))
    for lo in range(0, n, leaf):
        A[lo:lo + leaf, lo:lo + leaf] = g.standard_normal((leaf, leaf))
    sk = hss.OracleSketcher(A, "sjlt", seed=1, alpha=4)
    res = hss.compress(A, leaf, sk, d0=16, dd=16, eps_r=1e-10, eps_a=1e-12)
    assert res.converged and res.max_rank() == 0 and res.extensions == 0
    assert hss.relative_error(A, res) == 0.0


def test_symmetric_input_through_nonsymmetric_path_gives_U_equal_V():
    w = workloads
    X = w.uniform_points(256, 2, 5)
    X = X[w.bisection_order(X, 32)]
    A = w.gaussian_kernel_dense(X, 0.5, 1e-2)
    sk = hss.OracleSketcher(A, "gaussian", seed=4, symmetric=False)
    res = hss.compress(A, 32, sk, d0=32, dd=16, eps_r=1e-8, eps_a=1e-10, symmetric=False)
    assert res.converged
    for t in res.order:
        if t.U is not None:
            assert np.allclose(t.U, t.V, atol=1e-12) and list(t.J) == list(t.Jt)


@pytest.mark.parametrize("kind", ["gaussian", "sjlt", "srht"])
def test_kernel_matrix_meets_tolerance(kind):
    """A small instance of the n = 1024 kernel workload (n = 512, leaf 64):
    the relative Frobenius error of the compressed matrix is within 10 eps_r and
    the final d stays close to the HSS rank (section 8 reports d/rank of 1-1.8)."""
    w = workloads
    X = w.uniform_points(512, 2, 7)
    X = X[w.bisection_order(X, 64)]
    A = w.gaussian_kernel_dense(X, 0.5, 1e-2)
    eps = 1e-6
    sk = hss.OracleSketcher(A, kind, seed=11, alpha=4, symmetric=True)
    res = hss.compress(A, 64, sk, d0=64, dd=64, eps_r=eps, eps_a=1e-8, symmetric=True)
    assert res.converged
    err = hss.relative_error(A, res)
    assert err < 10 * eps
    assert res.final_d >= res.max_rank()


def test_nonsymmetric_cauchy_meets_tolerance():
    A = workloads.cauchy_dense(512)
    sk = hss.OracleSketcher(A, "sjlt", seed=2, alpha=4, symmetric=False)
    res = hss.compress(A, 64, sk, d0=32, dd=32, eps_r=1e-8, eps_a=1e-8, symmetric=False)
    assert res.converged
    assert hss.relative_error(A, res) < 1e-7


def test_extension_happens_when_d0_too_small():
    """With d0 far below the rank the algorithm must extend R (Algorithm 1,
    extension branch) and still meet the tolerance."""
    n, leaf, r = 256, 32, 12
    A = _exact_hss(n, leaf, r, seed=3, symmetric=True)
    A = 0.5 * (A + A.T)
    sk = hss.OracleSketcher(A, "gaussian", seed=5, symmetric=True)
    res = hss.compress(A, leaf, sk, d0=4, dd=4, eps_r=1e-12, eps_a=1e-14, symmetric=True)
    assert res.converged and res.extensions >= 2
    assert hss.relative_error(A, res) < 1e-9
    assert len(sk.widths) == 2 + res.extensions


def test_interpolative_decomposition():
    """ID of a rank-5 matrix: 5 skeleton columns, an identity block on them, exact
    reconstruction, and the ID rank at a tolerance is at least the SVD rank."""
    g = np.random.Generator(np.random.PCG64(8))
    M = g.standard_normal((30, 5)) @ g.standard_normal((5, 40))
    J, Y = hss.interpolative(M, 1e-12, 1e-14)
    assert len(J) == 5
    assert np.allclose(Y[:, J], np.eye(5), atol=0)
    assert np.linalg.norm(M - M[:, J] @ Y) < 1e-11 * np.linalg.norm(M)
    Mn = M + 1e-6 * g.standard_normal(M.shape)
    J2, _ = hss.interpolative(Mn, 1e-3, 0.0)
    s = np.linalg.svd(Mn, compute_uv=False)
    assert len(J2) >= int((s > 1e-3 * s[0]).sum())
    J0, Y0 = hss.interpolative(np.zeros((4, 6)), 1e-8, 1e-8)
    assert len(J0) == 0 and Y0.shape == (0, 6)


def test_node_ranks_match_lapack_pivoted_qr_at_level_scaled_tolerance():
    """Every node's ID rank equals the number of pivoted-QR diagonal entries of
    its final local sketch above max(eps_a, eps_r |R_00|) / level(node)
    (Algorithm 1: tolerances divided by the node level; LAPACK dgeqp3 via scipy
    is the library routine the truncated CPQR reduces to)."""
    import scipy.linalg as sla
    w = workloads
    X = w.uniform_points(512, 2, 9)
    X = X[w.bisection_order(X, 32)]
    A = w.gaussian_kernel_dense(X, 0.3, 1e-2)
    eps_r, eps_a = 1e-5, 1e-9
    sk = hss.OracleSketcher(A, "gaussian", seed=12, symmetric=True)
    res = hss.compress(A, 32, sk, d0=48, dd=16, eps_r=eps_r, eps_a=eps_a, symmetric=True)
    assert res.converged
    checked = 0
    for t in res.order:
        if t.J is None:
            continue
        R = sla.qr(t.S.T, mode="r", pivoting=True)[0]
        dg = np.abs(np.diag(R))
        if dg.size == 0:
            continue
        tol = max(eps_a / t.level, eps_r / t.level * dg[0])
        # skip nodes whose cut lies within rounding of the tolerance
        if np.any(np.abs(dg / tol - 1) < 1e-6):
            continue
        k = int(np.argmax(dg < tol)) if np.any(dg < tol) else dg.size
        assert len(t.J) == k, (t.lo, t.hi, t.level)
        checked += 1
    assert checked >= 10


def test_qchem_toeplitz_hss_meets_tolerance():
    """The paper's QChem Toeplitz matrix (section 8.1, d = 0.1) compressed by the
    oracle's adaptive HSS with SJLT sketches: the error meets the tolerance and
    the ranks stay small (the paper notes they grow slowly with n)."""
    import workloads as w
    n = 512
    A = w.qchem_toeplitz_dense(n, 0.1)
    sk = hss.OracleSketcher(A, "sjlt", 77, alpha=4, symmetric=True)
    res = hss.compress(A, 64, sk, d0=64, dd=64, eps_r=1e-6, eps_a=1e-8, symmetric=True)
    assert res.converged
    err = hss.relative_error(A, res)
    assert err <= 10 * 1e-6
    assert res.max_rank() <= 48
