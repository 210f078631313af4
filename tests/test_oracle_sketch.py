"""CPU pins of the oracle's sketches, adjoint and matrix-free gradient.

Each oracle result (explicit R times A by a dense product) is checked against an
independent formulation: the paper's own SJLT outer-product (CRS) and
inner-product (CCS) algorithms of section 6.3, a fast Walsh-Hadamard transform for
SRHT, brute-force loops, and central finite differences for the gradient."""
import math

import numpy as np
import pytest

from oracle import operators as ops
from oracle import sketch as osk
from oracle.sketch import rel_fro


def _rand(m, n, seed):
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((m, n))


def _sjlt_AR_outer(A, n, w, alpha, block, seed, construction="block"):
    """Section 6.3, "Efficiently computing AR": S = sum_i A(:, i) R(i, :) by walking
    the rows of R in CRS form: add column A_i to S_j for each +1 in row i of B+,
    subtract it for each 1 in B-, and scale by s at the end."""
    R = ops.sjlt_block(n, w, alpha, block, seed, construction)
    s, Bp, Bm = ops.sjlt_split(R)
    rp, ip = ops.crs(Bp)
    rm, im = ops.crs(Bm)
    S = np.zeros((A.shape[0], w))
    for i in range(n):
        for j in ip[rp[i]:rp[i + 1]]:
            S[:, j] += A[:, i]
        for j in im[rm[i]:rm[i + 1]]:
            S[:, j] -= A[:, i]
    return s * S


def _sjlt_AtR_inner(A, n, w, alpha, block, seed, construction="block"):
    """Section 6.3, A^* R by inner products: for each column of A, signed sums over
    the CCS row lists of every column of R, scaled at the end."""
    R = ops.sjlt_block(n, w, alpha, block, seed, construction)
    s, Bp, Bm = ops.sjlt_split(R)
    cp, jp = ops.ccs(Bp)
    cm, jm = ops.ccs(Bm)
    St = np.zeros((A.shape[1], w))
    for k in range(A.shape[1]):
        col = A[:, k]
        for j in range(w):
            St[k, j] = col[jp[cp[j]:cp[j + 1]]].sum() - col[jm[cm[j]:cm[j + 1]]].sum()
    return s * St


@pytest.mark.parametrize("construction", ["block", "graph"])
@pytest.mark.parametrize("m,n,w,alpha", [(37, 64, 16, 4), (20, 50, 24, 8), (64, 128, 64, 1), (30, 40, 20, 3)])
def test_sjlt_sketch_matches_paper_algorithms(m, n, w, alpha, construction):
    if construction == "block" and w % alpha:
        pytest.skip("the block construction needs alpha | w")
    A = _rand(m, n, 1)
    R = ops.sjlt_block(n, w, alpha, 2, 99, construction)
    assert rel_fro(osk.sketch(A, R), _sjlt_AR_outer(A, n, w, alpha, 2, 99, construction)) < 1e-14
    B = _rand(n, m, 2)            # S' = B^T R with B n x m (rows of R index rows of B)
    assert rel_fro(osk.sketch_t(B, R), _sjlt_AtR_inner(B, n, w, alpha, 2, 99, construction)) < 1e-14


def _fwht_rows(X):
    """In-place radix-2 fast Walsh-Hadamard transform of every row (natural
    order, unnormalised)."""
    X = X.copy()
    nu = X.shape[1]
    h = 1
    while h < nu:
        for i in range(0, nu, 2 * h):
            a = X[:, i:i + h].copy()
            b = X[:, i + h:i + 2 * h].copy()
            X[:, i:i + h] = a + b
            X[:, i + h:i + 2 * h] = a - b
        h *= 2
    return X


@pytest.mark.parametrize("m,n,w,col0", [(9, 64, 16, 0), (33, 256, 40, 72)])
def test_srht_sketch_matches_fwht(m, n, w, col0):
    """Section 7.1: S = A D H P computed by a fast transform of each row of A D,
    then column sampling and the scale sqrt(nu/w)/sqrt(nu) = 1/sqrt(w)."""
    A = _rand(m, n, 3)
    D = ops.srht_diag(n, 17)
    mu = ops.srht_samples(n, col0, col0 + w, 17)
    ref = _fwht_rows(A * D[None, :])[:, mu] / math.sqrt(w)
    R = ops.srht_block(n, w, col0, 17)
    assert rel_fro(osk.sketch(A, R), ref) < 1e-14
    B = _rand(n, m, 4)             # S' = B^T R: transform every column of B
    refT = _fwht_rows(B.T * D[None, :])[:, mu] / math.sqrt(w)
    assert rel_fro(osk.sketch_t(B, R), refT) < 1e-14


def test_gaussian_sketch_brute_force():
    m, n, w = 7, 11, 5
    A = _rand(m, n, 5)
    R = ops.gaussian_block(n, w, 3, 8)
    S = np.zeros((m, w))
    for i in range(m):
        for j in range(w):
            acc = 0.0
            for k in range(n):
                acc += A[i, k] * R[k, j]
            S[i, j] = acc
    assert rel_fro(osk.sketch(A, R), S) < 1e-14


@pytest.mark.parametrize("kind", ops.KINDS)
def test_sketch_identities(kind):
    """A = I gives S = R; linearity; block concatenation equals the sketch with
    the concatenated operator; sampled columns equal full columns; adjoint dot
    test <A R, W> = <A, W R^T>."""
    n = 64
    widths = [16, 16, 32]
    R = ops.operator(kind, n, widths, 31, alpha=4)
    assert np.array_equal(osk.sketch(np.eye(n), R), R)
    A, B = _rand(20, n, 6), _rand(20, n, 7)
    assert rel_fro(osk.sketch(2 * A - 3 * B, R), 2 * osk.sketch(A, R) - 3 * osk.sketch(B, R)) < 1e-14
    parts = [osk.sketch(A, ops.operator_block(kind, n, w, b, c0, 31, 4))
             for b, (w, c0) in enumerate(zip(widths, np.cumsum([0] + widths[:-1])))]
    assert rel_fro(np.hstack(parts), osk.sketch(A, R)) < 1e-15
    cols = [0, 5, 17, 40, 63]
    sc = osk.sketch_columns(A, kind, n, widths, 31, cols, alpha=4)
    assert rel_fro(sc, osk.sketch(A, R)[:, cols]) < 1e-14
    Asq = _rand(n, n, 8)
    sct = osk.sketch_columns(Asq, kind, n, widths, 31, cols, alpha=4, transpose=True)
    assert rel_fro(sct, osk.sketch_t(Asq, R)[:, cols]) < 1e-14
    W = _rand(20, R.shape[1], 9)
    lhs = float((osk.sketch(A, R) * W).sum())
    rhs = float((A * osk.adjoint(W, R)).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_kernel_sketch_and_matrix():
    X = np.random.Generator(np.random.PCG64(2)).random((300, 3))
    R = ops.sjlt_block(300, 32, 4, 0, 5)
    K = osk.kernel_matrix(X, X, 0.3, shift=1e-3)
    assert rel_fro(osk.kernel_sketch(X, 0.3, R, shift=1e-3, block_rows=64), K @ R) < 1e-14
    # brute force one entry of K
    i, j = 3, 250
    r2 = sum((X[i, a] - X[j, a]) ** 2 for a in range(3))
    assert abs(K[i, j] - math.exp(-r2 / (2 * 0.09))) < 1e-16


def test_kernel_gradient_matches_finite_differences():
    """dL/dX and dL/dh (closed form) against central differences in FP64."""
    g = np.random.Generator(np.random.PCG64(4))
    N = 96
    X = g.random((N, 3))
    R = ops.sjlt_block(N, 16, 4, 0, 3)
    W = g.standard_normal((N, 16))
    h = 0.3
    dX, dh = osk.kernel_grad(X, h, R, W, block_rows=40)
    coords = [(i, a) for i in (0, 7, 50, 95) for a in range(3)]
    fd, fdh = osk.finite_difference_grad(X, h, R, W, coords, step=1e-5)
    got = np.array([dX[i, a] for i, a in coords])
    assert np.max(np.abs(got - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd)))
    assert abs(dh - fdh) < 1e-7 * max(1.0, abs(fdh))


def test_bf16x3_split_is_exact():
    """a = a1 + a2 + a3 exactly for FP32 a, every part on the bfloat16 grid: three
    8-bit significands cover FP32's 24 bits (with the sign absorbing the rounding)."""
    g = np.random.Generator(np.random.PCG64(6))
    a = (g.standard_normal(100000) * np.exp(g.uniform(-30, 30, 100000))).astype(np.float32)
    a1, a2, a3 = osk.split_bf16x3(a)
    assert ((a1 + a2) + a3 == a.astype(np.float64)).all()
    for p in (a1, a2, a3):
        assert (ops.bf16_round(p) == p).all()
    # a single bf16 part leaves ~2^-9 relative error
    rel = np.abs(a1 - a) / np.abs(a)
    assert rel.max() <= 2.0 ** -8


def test_kernel_row_helpers_match_full_forms_and_differences():
    """The row-wise helpers (used for sampled rows of the N = 32768 workload) give
    the same rows as the full forms, which are pinned above by the kernel matrix
    and finite differences; dL/dx_i from the row helper is also checked directly
    against central differences of the FP64 loss, so a dropped G_ji term, a
    misplaced diagonal shift or a wrong sign in either helper fails here."""
    g = np.random.Generator(np.random.PCG64(11))
    N, w = 300, 32
    X = g.random((N, 3))
    R = ops.sjlt_block(N, w, 4, 0, 17)
    W = g.standard_normal((N, w))
    h, shift = 0.25, 0.7
    rows = np.array([0, 5, 149, 150, 298, 299])
    S = osk.kernel_sketch(X, h, R, shift=shift, block_rows=64)
    assert rel_fro(osk.kernel_sketch_rows(X, h, R, rows, shift=shift), S[rows]) < 1e-14
    # the shift sits on the diagonal only: rows differ from the unshifted ones by shift R(i, :)
    d = osk.kernel_sketch_rows(X, h, R, rows, shift=shift) - osk.kernel_sketch_rows(X, h, R, rows)
    assert np.allclose(d, shift * R[rows], rtol=0, atol=1e-14)
    dX, _ = osk.kernel_grad(X, h, R, W, block_rows=77)
    gr = osk.kernel_grad_rows(X, h, R, W, rows)
    assert rel_fro(gr, dX[rows]) < 1e-13
    coords = [(int(i), a) for i in rows for a in range(3)]
    fd, _ = osk.finite_difference_grad(X, h, R, W, coords, step=1e-5)
    assert np.max(np.abs(gr.reshape(-1) - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd)))
    # G_ji matters: with W R^T nonsymmetric, the one-sided sum differs
    one_sided = np.zeros_like(gr)
    for t, i in enumerate(rows):
        diff = X[i][None, :] - X
        K = np.exp(-(diff ** 2).sum(1) / (2 * h * h))
        one_sided[t] = -((2 * (R @ W[i]) * K)[:, None] * diff).sum(0) / (h * h)
    assert rel_fro(one_sided, gr) > 1e-2


@pytest.mark.parametrize("n", [1, 2, 5, 12, 33, 64, 100, 257])
def test_hadamard_split_is_the_padded_transform(n):
    """Section 7.1, eqs. (had1) and (hadiden): the k-point / p-point split equals
    [A 0] H_nu (A padded with zero columns to nu = 2^ceil(log2 n)) as a matrix
    identity, checked against the explicit Sylvester matrix; for n a power of
    two it is the plain transform."""
    A = _rand(7, n, 30 + n)
    nu = ops.srht_nu(n)
    Apad = np.zeros((7, nu))
    Apad[:, :n] = A
    assert rel_fro(osk.hadamard_split(A), Apad @ ops.hadamard(nu)) < 1e-14
    # the two halves of the split: A_k H_k +- A^ H_p [I ... I]
    if n & (n - 1):
        k = nu // 2
        assert rel_fro(osk.hadamard_split(A)[:, :k] - osk.hadamard_split(A)[:, k:],
                       2 * osk.hadamard_split(np.concatenate([np.zeros((7, k)), A[:, k:]], 1))[:, :k]) < 1e-13


@pytest.mark.parametrize("m,n,w,col0", [(9, 100, 16, 0), (20, 1000, 40, 24), (5, 3, 8, 8), (33, 129, 64, 0)])
def test_srht_any_n_fast_path_matches_explicit(m, n, w, col0):
    """S = A D H P for n not a power of two: the section 7.1 transform path equals
    the explicit operator of section 7.2 times A (and S' likewise on A^T)."""
    A = _rand(m, n, 3)
    D = ops.srht_diag(n, 17)
    mu = ops.srht_samples(ops.srht_nu(n), col0, col0 + w, 17)
    R = ops.srht_block(n, w, col0, 17)
    assert rel_fro(osk.srht_sketch_fast(A, D, mu, w), osk.sketch(A, R)) < 1e-13
    B = _rand(n, m, 4)
    assert rel_fro(osk.srht_sketch_fast(B.T, D, mu, w), osk.sketch_t(B, R)) < 1e-13
    # A = I: the sketch is R itself
    assert rel_fro(osk.srht_sketch_fast(np.eye(n), D, mu, w), R) < 1e-14

