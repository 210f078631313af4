"""CPU pins of the oracle's generator and operators against facts fixed by the
paper, by published test vectors, or by mathematics."""
import math
import os

import numpy as np
import pytest
import torch

from oracle import operators as ops
from oracle.philox import key_from_seed, mulhi32, philox4x32_10

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_sections(path):
    sec, out = None, {}
    for line in open(path):
        line = line.strip()
        if line.startswith("# section:"):
            sec = line.split(":", 1)[1].strip()
            out[sec] = []
        elif line and not line.startswith("#") and sec:
            out[sec].append([int(x) for x in line.split()])
    return {k: np.array(v) for k, v in out.items()}


# ------------------------------------------------------------------- Philox
def test_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        out = philox4x32_10(v[0], v[1], v[2], v[3], (v[4], v[5]))
        assert [int(x) for x in out] == v[6:10]


def test_key_and_mulhi():
    assert key_from_seed(0x0123456789ABCDEF) == (0x89ABCDEF, 0x01234567)
    # mulhi32 maps [0, 2^32) onto [0, r) monotonically and hits the endpoints
    u = np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint64)
    assert list(mulhi32(u, 10)) == [0, 0, 5, 9]
    assert list(mulhi32(u, 2**32)) == [int(x) for x in u]


# --------------------------------------------------------------------- SJLT
@pytest.mark.parametrize("n,w,alpha", [(100, 64, 4), (257, 64, 8), (64, 256, 4), (33, 8, 1)])
def test_sjlt_structure(n, w, alpha):
    """Section 2.4.3, block construction (alpha chunks of w/alpha columns, one
    nonzero +-1/sqrt(alpha) each): exactly alpha nonzeros per row, one per chunk,
    unit row norms, ||R||_F^2 = n."""
    R = ops.sjlt_block(n, w, alpha, block=3, seed=77)
    wc = w // alpha
    nz = R != 0
    assert (nz.sum(1) == alpha).all()
    for c in range(alpha):
        assert (nz[:, c * wc:(c + 1) * wc].sum(1) == 1).all()
    assert np.allclose(np.abs(R[nz]), 1 / math.sqrt(alpha), rtol=0, atol=0)
    assert np.allclose((R * R).sum(1), 1.0, rtol=1e-15)
    assert abs((R * R).sum() - n) < 1e-9


def test_sjlt_blocks_differ_and_are_deterministic():
    a = ops.sjlt_hash(500, 64, 4, 0, 11)
    b = ops.sjlt_hash(500, 64, 4, 0, 11)
    c = ops.sjlt_hash(500, 64, 4, 1, 11)
    d = ops.sjlt_hash(500, 64, 4, 0, 12)
    assert all((x == y).all() for x, y in zip(a, b))
    assert (a[0] != c[0]).any() and (a[0] != d[0]).any()


def test_sjlt_positions_uniform_and_signs_balanced():
    """Offsets are uniform over each chunk and signs are fair coins (section 2.4.3)."""
    n, w, alpha = 40000, 64, 4
    cols, signs = ops.sjlt_hash(n, w, alpha, 0, 5)
    wc = w // alpha
    offs = cols - np.arange(alpha)[None, :] * wc
    cnt = np.bincount(offs.ravel(), minlength=wc)
    exp = n * alpha / wc
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < wc + 6 * math.sqrt(2 * wc)          # ~ chi^2(wc-1), > 6 sigma fails
    assert abs(signs.mean()) < 6 / math.sqrt(signs.size)


def test_sjlt_worked_example_split():
    """Section 6.1: R = s (B+ - B-) with binary B+/B-, stored in CRS and CCS
    without value arrays.  The printed 4x3 example pins the split."""
    g = _read_sections(os.path.join(GOLD, "sjlt_worked_example.txt"))
    R = g["M"] / math.sqrt(2)
    s, Bp, Bm = ops.sjlt_split(R)
    assert abs(s - 1 / math.sqrt(2)) < 1e-15
    assert (Bp == g["Bplus"]).all() and (Bm == g["Bminus"]).all()
    assert np.allclose(s * (Bp - Bm), R, atol=0)
    # CRS of B+ : rows 0, 2, 3 hold column 0, row 3 also column 2
    assert ops.crs(Bp) == ([0, 1, 1, 2, 4], [0, 0, 0, 2])
    assert ops.ccs(Bm) == ([0, 0, 2, 4], [1, 2, 0, 1])


# --------------------------------------------------------------------- SRHT
@pytest.mark.parametrize("nu", [1, 2, 4, 64, 1024])
def test_hadamard_orthogonal(nu):
    """Section 2.4.2: the Sylvester recursion gives H H^T = nu I (unnormalised)."""
    H = ops.hadamard(nu)
    assert (H @ H.T == nu * np.eye(nu)).all()


def test_hadamard_element_formula_matches_recursion():
    """Section 7.2: (H_nu)_ij = (-1)^{i . j} with i . j the dot product of the
    binary digits (0-based indices, natural order)."""
    nu = 256
    i = np.arange(nu, dtype=np.uint64)
    par = ops.popcount(i[:, None] & i[None, :]) & 1
    assert ((1 - 2 * par) == ops.hadamard(nu)).all()


def test_srht_block_equals_DHP():
    """Section 2.4.2 R = D H P with P's columns sqrt(nu/w) e_mu; the element formula
    of section 7.2 must give the same matrix as the explicit product."""
    n, w, col0, seed = 128, 24, 40, 9
    D = ops.srht_diag(n, seed)
    mu = ops.srht_samples(n, col0, col0 + w, seed)
    Hn = ops.hadamard(n) / math.sqrt(n)
    P = np.zeros((n, w))
    P[mu, np.arange(w)] = math.sqrt(n / w)
    R = np.diag(D.astype(float)) @ Hn @ P
    assert np.allclose(ops.srht_block(n, w, col0, seed), R, atol=1e-14)


def test_srht_rows_unit_norm_and_samples_uniform():
    R = ops.srht_block(512, 64, 0, 3)
    assert np.allclose((R * R).sum(1), 1.0, atol=1e-14)
    mu = ops.srht_samples(16, 0, 160000, 4)
    cnt = np.bincount(mu, minlength=16)
    exp = 10000
    assert ((cnt - exp) ** 2 / exp).sum() < 16 + 6 * math.sqrt(32)


@pytest.mark.parametrize("n", [100, 129, 1000, 3])
def test_srht_any_n_is_padded_DHP(n):
    """Section 7.2, eq. (DtildeH): for n not a power of two, R = D~ H_nu P with
    nu = 2^ceil(log2 n) and D~ = [D 0]; the element formula gives exactly the
    first n rows of that explicit product, with unit row norms."""
    w, col0, seed = 24, 8, 5
    nu = ops.srht_nu(n)
    assert nu >= n > nu // 2
    D = ops.srht_diag(n, seed)
    mu = ops.srht_samples(nu, col0, col0 + w, seed)
    assert mu.max() < nu
    Dt = np.zeros((n, nu))
    Dt[np.arange(n), np.arange(n)] = D
    P = np.zeros((nu, w))
    P[mu, np.arange(w)] = math.sqrt(nu / w)
    R = Dt @ (ops.hadamard(nu) / math.sqrt(nu)) @ P
    Rb = ops.srht_block(n, w, col0, seed)
    assert np.allclose(Rb, R, rtol=0, atol=1e-14)
    assert np.allclose((Rb * Rb).sum(1), 1.0, atol=1e-14)
    # for a power of two the operator is unchanged: nu = n
    assert ops.srht_nu(128) == 128


# ----------------------------------------------------------------- Gaussian
def test_bf16_round_matches_library_on_fp32_values():
    """For FP32-representable inputs, rounding to bf16 must agree with torch's
    float32 -> bfloat16 conversion (round to nearest even)."""
    g = np.random.Generator(np.random.PCG64(0))
    x = (g.standard_normal(200000) * np.exp(g.uniform(-20, 20, 200000))).astype(np.float32)
    # add exact ties: values with the 16 low mantissa bits equal to 0x8000
    bits = g.integers(0, 2**32, 5000, dtype=np.uint64).astype(np.uint32)
    expo = g.integers(100, 150, 5000).astype(np.uint32) << np.uint32(23)
    bits = (bits & np.uint32(0x807F0000)) | np.uint32(0x00008000) | expo
    x = np.concatenate([x, bits.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert (ops.bf16_round(x.astype(np.float64)) == ref).all()


def test_gaussian_draws_moments():
    g = ops.gaussian_raw(20000, 0, 16, 123).ravel()
    assert abs(g.mean()) < 5 / math.sqrt(g.size)
    assert abs(g.var() - 1) < 5 * math.sqrt(2 / g.size) + 2e-5
    # on the bf16 grid
    assert (ops.bf16_round(g) == g).all()
    # Kolmogorov-Smirnov distance to N(0,1)
    s = np.sort(g)
    cdf = 0.5 * (1 + np.vectorize(math.erf)(s / math.sqrt(2)))
    ks = np.max(np.abs(cdf - np.arange(1, s.size + 1) / s.size))
    assert ks < 1.63 / math.sqrt(s.size) + 4e-3      # bf16 grid adds <= 2^-9 rel. jitter


def test_gaussian_block_columns_are_global():
    """Column j of R depends only on the global column index (blocks are slices of
    one infinite column sequence), scaled by the block's own width."""
    assert np.array_equal(ops.gaussian_raw(50, 0, 64, 7)[:, 32:], ops.gaussian_raw(50, 32, 32, 7))
    b = ops.gaussian_block(50, 32, 32, 7)
    assert np.allclose(b * math.sqrt(32), ops.gaussian_raw(50, 32, 32, 7), rtol=1e-15, atol=0)


# ------------------------------------------------------------ JL statistics
@pytest.mark.parametrize("kind", ["gaussian", "sjlt", "srht"])
def test_jl_norm_preservation_statistics(kind):
    """E ||x^T R||^2 = ||x||^2 with the variance fixed by each construction:
    Gaussian 2||x||^4/w (entries N(0, 1/w)); SJLT block construction
    (2/w)(||x||^4 - sum x^4); SRHT given D: (1/w)(nu sum z^4 - ||x||^4) with
    z = H D x / sqrt(nu).  Checked over 4000 seeds to 5 sigma."""
    n, w, alpha, trials = 64, 16, 4, 4000
    g = np.random.Generator(np.random.PCG64(1))
    x = g.standard_normal(n)
    x[:4] *= 6                                      # non-flat vector
    nx2 = x @ x
    vals = []
    for s in range(trials):
        R = ops.operator_block(kind, n, w, 0, 0, 1000 + s, alpha)
        y = x @ R
        vals.append(y @ y)
    vals = np.array(vals)
    if kind == "gaussian":
        var = 2 * nx2 ** 2 / w
        se = math.sqrt(var / trials)
        assert abs(vals.mean() - nx2) < 5 * se
        assert abs(vals.var() / var - 1) < 0.25
    elif kind == "sjlt":
        var = 2 / w * (nx2 ** 2 - (x ** 4).sum())
        se = math.sqrt(var / trials)
        assert abs(vals.mean() - nx2) < 5 * se
        assert abs(vals.var() / var - 1) < 0.2
    else:
        # condition on D by averaging the conditional variance over seeds
        cv = []
        for s in range(trials):
            D = ops.srht_diag(n, 1000 + s)
            z = ops.hadamard(n) @ (D * x) / math.sqrt(n)
            cv.append((n * (z ** 4).sum() - nx2 ** 2) / w)
        var = float(np.mean(cv))
        se = math.sqrt(var / trials)
        assert abs(vals.mean() - nx2) < 5 * se
        assert abs(vals.var() / var - 1) < 0.2


def test_gaussian_frobenius_bound_worked_value():
    """Theorem 4.2 worked value: eps = 0.5, delta = 0.01 -> d >= 424; and at that
    d the fraction of draws with | ||AR||_F^2 / ||A||_F^2 - 1 | > eps stays below
    delta (checked over 400 seeds on a fixed 40 x 300 matrix)."""
    for line in open(os.path.join(GOLD, "jl_gaussian_bound.txt")):
        if line.startswith("#") or not line.strip():
            continue
        eps, delta, dmin = line.split()
        eps, delta, dmin = float(eps), float(delta), int(dmin)
    assert math.ceil(20 / eps ** 2 * math.log(2 / delta)) == dmin
    from oracle.sketch import frobenius_ratio
    A = np.random.Generator(np.random.PCG64(3)).standard_normal((40, 300))
    bad = sum(abs(frobenius_ratio(A, ops.gaussian_block(300, dmin, 0, s)) - 1) > eps
              for s in range(400))
    assert bad / 400 <= delta


# ------------------------------------------------------- SJLT graph construction
@pytest.mark.parametrize("n,w,alpha", [(300, 64, 4), (257, 16, 16), (100, 256, 8), (64, 7, 1), (50, 32, 32)])
def test_sjlt_graph_structure(n, w, alpha):
    """Section 2.4.3, graph construction: alpha nonzeros +-1/sqrt(alpha) per row at
    distinct columns of the block (reading: without replacement), unit row norms."""
    cols, signs = ops.sjlt_graph_hash(n, w, alpha, 2, 31)
    assert cols.min() >= 0 and cols.max() < w
    assert all(len(set(r)) == alpha for r in cols.tolist())
    assert set(np.unique(signs)) <= {-1, 1}
    R = ops.sjlt_block(n, w, alpha, 2, 31, construction="graph")
    assert ((R != 0).sum(1) == alpha).all()
    assert np.allclose((R * R).sum(1), 1.0, rtol=1e-15)
    # not the block construction: positions are not confined to chunks
    # (alpha = w leaves one subset, all columns)
    if 1 < alpha < w and w % alpha == 0:
        wc = w // alpha
        assert (cols // wc != np.arange(alpha)[None, :]).any()


def test_sjlt_graph_subsets_uniform():
    """Floyd's algorithm draws every alpha-subset of the w columns with probability
    1/C(w, alpha): w = 6, alpha = 3 gives 20 subsets, counted over 60000 rows
    (chi-square with 19 degrees of freedom, 6 sigma); every column is hit with
    probability alpha/w."""
    n, w, alpha = 60000, 6, 3
    cols, signs = ops.sjlt_graph_hash(n, w, alpha, 0, 9)
    keys = np.sort(cols, axis=1) @ np.array([36, 6, 1])
    _, cnt = np.unique(keys, return_counts=True)
    assert cnt.size == math.comb(w, alpha)
    exp = n / cnt.size
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < 19 + 6 * math.sqrt(2 * 19)
    hits = np.bincount(cols.ravel(), minlength=w) / n
    assert np.abs(hits - alpha / w).max() < 6 * math.sqrt(0.25 / n)
    assert abs(signs.mean()) < 6 / math.sqrt(signs.size)


def test_sjlt_graph_jl_statistics():
    """E ||x^T R||^2 = ||x||^2 and, with alpha distinct uniform columns per row,
    Var = (2/w)(||x||^4 - sum x^4): the cross terms x_i x_k s_ij s_kj survive only
    in pairs and P(j in S_i) = alpha/w for every row.  4000 seeds, 5 sigma."""
    n, w, alpha, trials = 64, 16, 4, 4000
    g = np.random.Generator(np.random.PCG64(1))
    x = g.standard_normal(n)
    x[:4] *= 6
    nx2 = x @ x
    vals = np.array([(lambda y: y @ y)(x @ ops.operator_block("sjlt_graph", n, w, 0, 0, 3000 + s, alpha))
                     for s in range(trials)])
    var = 2 / w * (nx2 ** 2 - (x ** 4).sum())
    assert abs(vals.mean() - nx2) < 5 * math.sqrt(var / trials)
    assert abs(vals.var() / var - 1) < 0.2


def test_qchem_toeplitz_input_matches_the_closed_form():
    """Section 8.1, QChem Toeplitz: T_ii = pi^2 / (6 d^2), T_ij = (-1)^(i-j) /
    (d^2 (i-j)^2) with d = 0.1, checked entry by entry on a small n; T is
    symmetric and Toeplitz."""
    import workloads
    n, d = 40, 0.1
    T = workloads.qchem_toeplitz_dense(n, d)
    for i in range(n):
        for j in range(n):
            ref = math.pi ** 2 / (6 * d * d) if i == j else (-1) ** (i - j) / (d * d * (i - j) ** 2)
            assert abs(T[i, j] - ref) <= 1e-13 * abs(ref)
    assert (T == T.T).all()
    assert (T[1:, 1:] == T[:-1, :-1]).all()
