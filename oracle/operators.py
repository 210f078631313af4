"""Explicit sketching operators R (FP64), built entry by entry from the operator spec.

Test infrastructure only (see ``oracle/__init__.py``).

The operator R = [R_0 | R_1 | ...] is a concatenation of blocks; block b has width
w_b and starts at global column c_b.  Each block is its own JL operator normalised
by its own width (reading of section 2.4.1 "Gaussian Sketching Operator" together
with the extension step of Algorithm 1, which appends a fresh JL-Operator(dd, n)).

Random draws come from Philox4x32-10 (``oracle.philox``) under key = seed, with
these counters (all indices 0-based):

  SJLT offset, row k, chunk c, block b : ctr (1, b, k, c >> 2), word c & 3
                                         offset = mulhi32(word, w_b / alpha)
  SJLT sign,   row k, chunk c, block b : ctr (2, b, k, 0), word 0, bit c
                                         sigma = +1 if the bit is 0 else -1
  SRHT diagonal D_k                    : ctr (3, 0, k, 0), word 0, bit 0
  SRHT sample mu_j (global column j)   : ctr (4, 0, j >> 2, 0), word j & 3
                                         mu = mulhi32(word, nu)
  Gaussian g_{k,j} (global column j)   : ctr (5, j, k, 0), words 0 and 1
  SJLT graph draw, row k, step c, blk b: ctr (6, b, k, c >> 2), word c & 3
                                         t_c = mulhi32(word, w_b - alpha + c + 1)
"""
import math

import numpy as np

from .philox import key_from_seed, mulhi32, philox4x32_10

SJLT_MAX_ALPHA = 32


# --------------------------------------------------------------------------- SJLT
def sjlt_hash(n, w, alpha, block, seed):
    """Nonzero positions and signs of one SJLT block (block construction).

    Section 2.4.3 "Sparse Johnson-Lindenstrauss Transform": every row holds alpha
    nonzeros +-1/sqrt(alpha).  Block construction, read as: the row of width w is
    cut into alpha chunks of w/alpha consecutive columns and each chunk holds
    exactly one nonzero at a uniform position (the printed text says d/alpha
    chunks, which contradicts alpha nonzeros per row; alpha chunks is the reading
    consistent with "alpha nonzeros per row" and "d/alpha must be an integer").

    Returns (cols, signs): int64 arrays of shape (n, alpha); cols[k, c] is the
    column inside the block, signs[k, c] is +1 or -1.
    """
    if alpha < 1 or alpha > SJLT_MAX_ALPHA or w % alpha:
        raise ValueError("alpha must divide w and be in [1, 32]")
    key = key_from_seed(seed)
    wc = w // alpha
    k = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(alpha, dtype=np.uint64)[None, :]
    words = philox4x32_10(1, block, k, c >> np.uint64(2), key)
    word = np.choose((c & np.uint64(3)).astype(np.int64) + np.zeros((n, 1), np.int64), words)
    offs = mulhi32(word, wc).astype(np.int64)
    cols = c.astype(np.int64) * wc + offs
    sw = philox4x32_10(2, block, np.arange(n, dtype=np.uint64), 0, key)[0]
    bits = (sw[:, None] >> c) & np.uint64(1)
    signs = 1 - 2 * bits.astype(np.int64)
    return cols, signs


def sjlt_graph_hash(n, w, alpha, block, seed):
    """Nonzero positions and signs of one SJLT block, graph construction.

    Section 2.4.3: each row holds alpha nonzeros +-1/sqrt(alpha) at positions
    drawn uniformly from the w columns of the block.  The text does not say
    whether positions may repeat; the reading here is without replacement
    (alpha distinct columns, a uniformly random alpha-subset per row), which
    keeps exactly alpha nonzeros per row as the construction requires.

    The subset is drawn with Floyd's sampling algorithm (Bentley and Floyd,
    "A sample of brilliance", CACM 1987): for step c = 0 .. alpha-1 let
    j = w - alpha + c and draw t uniform in [0, j]; take t unless an earlier
    step already took it, in which case take j.  Every alpha-subset of [w] then
    has probability 1 / C(w, alpha), with exactly alpha draws per row.  Signs use
    the block construction's counter (2, b, k, 0), bit c.

    Returns (cols, signs) of shape (n, alpha); cols[k, c] is the column chosen
    at step c.
    """
    if alpha < 1 or alpha > SJLT_MAX_ALPHA or alpha > w:
        raise ValueError("graph construction needs 1 <= alpha <= min(w, 32)")
    key = key_from_seed(seed)
    k = np.arange(n, dtype=np.uint64)
    cols = np.zeros((n, alpha), dtype=np.int64)
    for c in range(alpha):
        j = w - alpha + c
        word = philox4x32_10(6, block, k, c >> 2, key)[c & 3]
        t = mulhi32(word, j + 1).astype(np.int64)
        taken = (cols[:, :c] == t[:, None]).any(axis=1)
        cols[:, c] = np.where(taken, j, t)
    sw = philox4x32_10(2, block, k, 0, key)[0]
    bits = (sw[:, None] >> np.arange(alpha, dtype=np.uint64)[None, :]) & np.uint64(1)
    signs = 1 - 2 * bits.astype(np.int64)
    return cols, signs


def sjlt_block(n, w, alpha, block, seed, construction="block"):
    """Dense FP64 SJLT block R_b (n x w): R[k, cols[k,c]] = signs[k,c] / sqrt(alpha),
    with the positions of the block (default) or graph construction."""
    hashf = sjlt_graph_hash if construction == "graph" else sjlt_hash
    cols, signs = hashf(n, w, alpha, block, seed)
    R = np.zeros((n, w), dtype=np.float64)
    rows = np.repeat(np.arange(n), alpha)
    R[rows, cols.ravel()] = signs.ravel() / math.sqrt(alpha)
    return R


def sjlt_split(R):
    """Split R = s (B+ - B-) with binary B+ and B- (section 6.1 data structure).

    Returns (s, Bplus, Bminus) where s is the common magnitude of the nonzeros.
    """
    nz = R[R != 0]
    s = float(np.abs(nz[0])) if nz.size else 1.0
    return s, (R > 0).astype(np.int8), (R < 0).astype(np.int8)


def crs(B):
    """Compressed row storage of a binary matrix without a value array."""
    rowptr = [0]
    idx = []
    for i in range(B.shape[0]):
        nz = np.nonzero(B[i])[0].tolist()
        idx += nz
        rowptr.append(len(idx))
    return rowptr, idx


def ccs(B):
    """Compressed column storage of a binary matrix without a value array."""
    return crs(B.T)


# --------------------------------------------------------------------------- SRHT
def is_pow2(n):
    return n >= 1 and (n & (n - 1)) == 0


def srht_diag(n, seed):
    """Rademacher diagonal D (section 2.4.2 SRHT): int64 array of +-1, length n."""
    key = key_from_seed(seed)
    w0 = philox4x32_10(3, 0, np.arange(n, dtype=np.uint64), 0, key)[0]
    return 1 - 2 * (w0 & np.uint64(1)).astype(np.int64)


def srht_samples(nu, j0, j1, seed):
    """Sampled Hadamard columns mu_j for global columns j0 <= j < j1.

    Each column of P is drawn independently and uniformly from the nu canonical
    vectors (section 2.4.2 SRHT and section 7.2), i.e. with replacement.
    """
    key = key_from_seed(seed)
    j = np.arange(j0, j1, dtype=np.uint64)
    words = philox4x32_10(4, 0, j >> np.uint64(2), 0, key)
    word = np.choose((j & np.uint64(3)).astype(np.int64), words)
    return mulhi32(word, nu).astype(np.int64)


def hadamard(nu):
    """Unnormalised Sylvester-Hadamard matrix H_nu (+-1 entries, natural order).

    Built by the recursion H_1 = [1], H_2m = [[H_m, H_m], [H_m, -H_m]] of section 2.4.2.
    """
    H = np.ones((1, 1), dtype=np.float64)
    while H.shape[0] < nu:
        H = np.block([[H, H], [H, -H]])
    return H


def popcount(x):
    x = np.asarray(x, dtype=np.uint64)
    cnt = np.zeros(x.shape, dtype=np.int64)
    while np.any(x):
        cnt += (x & np.uint64(1)).astype(np.int64)
        x = x >> np.uint64(1)
    return cnt


def srht_nu(n):
    """nu = 2^ceil(log2 n): the Hadamard dimension of section 7.2 (nu = n when n
    is a power of two)."""
    nu = 1
    while nu < n:
        nu *= 2
    return nu


def srht_block(n, w, col0, seed):
    """Dense FP64 SRHT block from the element formula of section 7.2:

        R[k, jj] = D_k * (-1)^{popcount(k & mu_{col0 + jj})} / sqrt(w),   k < n,

    with nu = 2^ceil(log2 n) and mu uniform over [nu].  For n not a power of two
    this is D~ H_nu P with the padded diagonal D~ = [D 0] of eq. (DtildeH): only
    the first n rows of H_nu are ever used.  Indices are 0-based, so the
    Hadamard entry (-1)^{i . j} uses the bits of the 0-based i and j.
    """
    nu = srht_nu(n)
    D = srht_diag(n, seed)
    mu = srht_samples(nu, col0, col0 + w, seed)
    k = np.arange(n, dtype=np.uint64)[:, None]
    par = popcount(k & mu.astype(np.uint64)[None, :]) & 1
    return D[:, None] * (1.0 - 2.0 * par) / math.sqrt(w)


# ------------------------------------------------------------------------ Gaussian
def bf16_round(z):
    """Round FP64 values to the nearest bfloat16 value (8 significant bits),
    ties to even, returned as FP64.  Inputs are finite normal numbers well inside
    bfloat16 range (Box-Muller output)."""
    z = np.asarray(z, dtype=np.float64)
    m, e = np.frexp(z)                      # z = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)   # rint rounds half to even


def gaussian_raw(n, col0, w, seed):
    """Unscaled Gaussian draws g[k, jj] for global columns col0 .. col0+w-1.

    Box-Muller on two Philox words: U = (u + 0.5) 2^-32, z = sqrt(-2 ln U1) cos(2 pi U2),
    evaluated in FP64 and rounded to bfloat16 so that the value is exactly
    representable in bf16, fp32 and fp64 (section 2.4.1 "Gaussian Sketching Operator"
    asks for N(0, 1/d) entries; the bf16 grid is this build's reading, see the
    design notes).
    """
    key = key_from_seed(seed)
    k = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(col0, col0 + w, dtype=np.uint64)[None, :]
    u0, u1, _, _ = philox4x32_10(5, j, k, 0, key)
    U1 = (u0.astype(np.float64) + 0.5) * 2.0 ** -32
    U2 = (u1.astype(np.float64) + 0.5) * 2.0 ** -32
    z = np.sqrt(-2.0 * np.log(U1)) * np.cos(2.0 * math.pi * U2)
    return bf16_round(z)


def gaussian_block(n, w, col0, seed):
    """Dense FP64 Gaussian block: R[k, jj] = g[k, col0+jj] / sqrt(w)."""
    return gaussian_raw(n, col0, w, seed) / math.sqrt(w)


# ----------------------------------------------------------------- concatenation
KINDS = ("gaussian", "sjlt", "srht", "sjlt_graph")


def operator_block(kind, n, w, block, col0, seed, alpha=4):
    """One block of R in FP64.  ``block`` is the block index b, ``col0`` = c_b.
    ``sjlt_graph`` is the SJLT operator with the graph construction."""
    if kind == "sjlt":
        return sjlt_block(n, w, alpha, block, seed)
    if kind == "sjlt_graph":
        return sjlt_block(n, w, alpha, block, seed, construction="graph")
    if kind == "srht":
        return srht_block(n, w, col0, seed)
    if kind == "gaussian":
        return gaussian_block(n, w, col0, seed)
    raise ValueError(kind)


def operator(kind, n, widths, seed, alpha=4):
    """R = [R_0 | R_1 | ...] for the given block widths (FP64, n x sum(widths))."""
    blocks = []
    col0 = 0
    for b, w in enumerate(widths):
        blocks.append(operator_block(kind, n, w, b, col0, seed, alpha))
        col0 += w
    return np.concatenate(blocks, axis=1) if blocks else np.zeros((n, 0))
