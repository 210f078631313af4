"""Plain FP64 sketches, adjoints and matrix-free kernel gradients.

Test infrastructure only (see ``oracle/__init__.py``).

Everything here is the plain definition written out with an explicit operator R
from ``oracle.operators`` and a dense product (a library matmul serves as the
product step).  Section 1 states the two sketches used by HSS construction:
S = A R for the column space and, for nonsymmetric A, S' = A^* R for the row
space (A is real in this build, so A^* = A^T).
"""
import numpy as np

from . import operators as ops


def sketch(A, R):
    """S = A R in FP64."""
    return np.asarray(A, dtype=np.float64) @ np.asarray(R, dtype=np.float64)


def sketch_t(A, R):
    """S' = A^T R in FP64."""
    return np.asarray(A, dtype=np.float64).T @ np.asarray(R, dtype=np.float64)


def operator_columns(kind, n, widths, seed, cols, alpha=4):
    """The selected global columns of R = [R_0 | R_1 | ...] (FP64, n x len(cols)),
    each formed from its block's element formulas."""
    offs = np.cumsum([0] + list(widths))
    Rsel = np.zeros((n, len(cols)))
    cache = {}
    for t, j in enumerate(cols):
        b = int(np.searchsorted(offs, j, side="right") - 1)
        if b not in cache:
            cache[b] = ops.operator_block(kind, n, widths[b], b, int(offs[b]), seed, alpha)
        Rsel[:, t] = cache[b][:, j - offs[b]]
    return Rsel


def sketch_columns(A, kind, n, widths, seed, cols, alpha=4, transpose=False, block=4096):
    """Selected columns of S = A R (or S' = A^T R): S(:, j) = sum_k A(:, k) R(k, j),
    evaluated for the requested global columns j only, in FP64, over row blocks
    of the result so that an FP32 A is promoted one block at a time."""
    A = np.asarray(A)
    Rsel = operator_columns(kind, n, widths, seed, cols, alpha)
    rows = A.shape[1] if transpose else A.shape[0]
    out = np.zeros((rows, len(cols)))
    for r0 in range(0, rows, block):
        r1 = min(rows, r0 + block)
        blk = A[:, r0:r1].T if transpose else A[r0:r1, :]
        out[r0:r1] = blk.astype(np.float64) @ Rsel
    return out


def fwht_rows(X):
    """Unnormalised natural-order Walsh-Hadamard transform of every row of X
    (row length a power of two), by the Sylvester recursion
    [a b] H_2m = [a H_m + b H_m, a H_m - b H_m]."""
    X = np.asarray(X, dtype=np.float64)
    nu = X.shape[1]
    if nu == 1:
        return X.copy()
    h = nu // 2
    a, b = fwht_rows(X[:, :h]), fwht_rows(X[:, h:])
    return np.concatenate([a + b, a - b], axis=1)


def hadamard_split(A):
    """A H_nu for A with n columns, nu = 2^ceil(log2 n), A padded with zero
    columns, by the split of section 7.1: with k = 2^floor(log2 n), n = k + r,
    p = 2^ceil(log2 r) and q = k / p,

        A H_2k = [A_k H_k + A^ H_p [I ... I],  A_k H_k - A^ H_p [I ... I]]

    (eqs. (had1) and (hadiden)), A_k the first k columns and A^ the last r
    padded to p.  Two transforms of dimensions k and p replace the one of
    dimension 2k.  For n a power of two it is the plain transform."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    k = 1
    while 2 * k <= n:
        k *= 2
    r = n - k
    if r == 0:
        return fwht_rows(A)
    p = 1
    while p < r:
        p *= 2
    q = k // p
    Ak = fwht_rows(A[:, :k])
    Ahat = np.zeros((m, p))
    Ahat[:, :r] = A[:, k:]
    T = np.tile(fwht_rows(Ahat), (1, q))        # A^ H_p [I ... I]
    return np.concatenate([Ak + T, Ak - T], axis=1)


def srht_sketch_fast(A, D, mu, w):
    """S = A D H_nu P / sqrt(w) by the transform of section 7.1 (any n): the
    rows of A D are transformed with ``hadamard_split`` and the sampled columns
    mu are kept."""
    AD = np.asarray(A, dtype=np.float64) * np.asarray(D, dtype=np.float64)[None, :]
    return hadamard_split(AD)[:, np.asarray(mu)] / np.sqrt(w)


def adjoint(dS, R):
    """dA = dS R^T: the adjoint of A -> A R applied to dS (FP64)."""
    return np.asarray(dS, dtype=np.float64) @ np.asarray(R, dtype=np.float64).T


# ------------------------------------------------------------- matrix-free kernel
def kernel_matrix(X, Y, h, shift=0.0):
    """K_ij = exp(-|x_i - y_j|^2 / (2 h^2)) in FP64, plus shift on the diagonal
    when X and Y are the same point set."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    d2 = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    K = np.exp(-d2 / (2.0 * h * h))
    if shift and X.shape == Y.shape and np.array_equal(X, Y):
        K = K + shift * np.eye(X.shape[0])
    return K


def kernel_sketch(X, h, R, shift=0.0, block_rows=2048):
    """S = K(X, h) R without storing K: row blocks of K are formed one at a time."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    S = np.zeros((N, R.shape[1]))
    for i0 in range(0, N, block_rows):
        i1 = min(N, i0 + block_rows)
        d2 = ((X[i0:i1, None, :] - X[None, :, :]) ** 2).sum(-1)
        Kb = np.exp(-d2 / (2.0 * h * h))
        S[i0:i1] = Kb @ R
        if shift:
            S[i0:i1] += shift * R[i0:i1]
    return S


def kernel_loss(X, h, R, W, shift=0.0):
    """L = sum(W o S) with S = K(X, h) R."""
    return float(np.sum(np.asarray(W, np.float64) * kernel_sketch(X, h, R, shift)))


def kernel_grad(X, h, R, W, block_rows=1024):
    """Closed-form gradient of L = sum(W o (K R)) with respect to X and h.

    With G = W R^T (dL/dK) and K_ij = exp(-r_ij^2 / (2h^2)):
      dK_ij/dx_i = -K_ij (x_i - x_j) / h^2,   dK_ij/dx_j = +K_ij (x_i - x_j) / h^2,
      dK_ij/dh   =  K_ij r_ij^2 / h^3,
    so dL/dx_i = -(1/h^2) sum_j (G_ij + G_ji) K_ij (x_i - x_j) (K is symmetric) and
    dL/dh = sum_ij G_ij K_ij r_ij^2 / h^3.  The diagonal shift does not depend on
    X or h and drops out.  Returns (dX, dh) in FP64.
    """
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    N = X.shape[0]
    dX = np.zeros_like(X)
    dh = 0.0
    for i0 in range(0, N, block_rows):
        i1 = min(N, i0 + block_rows)
        diff = X[i0:i1, None, :] - X[None, :, :]           # (b, N, dim)
        d2 = (diff ** 2).sum(-1)
        K = np.exp(-d2 / (2.0 * h * h))
        G = W[i0:i1] @ R.T                                   # G_ij for rows i0..i1
        Gt = R[i0:i1] @ W.T                                  # G_ji = (W R^T)_ji
        M = (G + Gt) * K
        dX[i0:i1] = -(M[:, :, None] * diff).sum(1) / (h * h)
        dh += float((G * K * d2).sum()) / h ** 3
    return dX, dh


def kernel_grad_rows(X, h, R, W, rows):
    """dL/dx_i of L = sum(W o (K R)) for the listed rows i only (same closed
    form as ``kernel_grad``), O(len(rows) N) work."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    out = np.zeros((len(rows), X.shape[1]))
    for t, i in enumerate(rows):
        diff = X[i][None, :] - X                      # (N, dim)
        K = np.exp(-(diff ** 2).sum(1) / (2.0 * h * h))
        Gi = R @ W[i]                                 # G_ij over j
        Gti = W @ R[i]                                # G_ji over j
        out[t] = -(((Gi + Gti) * K)[:, None] * diff).sum(0) / (h * h)
    return out


def kernel_sketch_rows(X, h, R, rows, shift=0.0):
    """Rows i of S = K(X, h) R (plus shift R(i, :)) in FP64."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((len(rows), R.shape[1]))
    for t, i in enumerate(rows):
        K = np.exp(-((X[i][None, :] - X) ** 2).sum(1) / (2.0 * h * h))
        out[t] = K @ R + shift * R[i]
    return out


def finite_difference_grad(X, h, R, W, coords, step=1e-4):
    """Central finite differences of L = sum(W o (K(X,h) R)) in FP64.

    coords: list of (i, a) coordinates of X; also returns dL/dh.
    """
    X = np.asarray(X, dtype=np.float64).copy()
    out = []
    for i, a in coords:
        x0 = X[i, a]
        X[i, a] = x0 + step
        lp = kernel_loss(X, h, R, W)
        X[i, a] = x0 - step
        lm = kernel_loss(X, h, R, W)
        X[i, a] = x0
        out.append((lp - lm) / (2 * step))
    dh = (kernel_loss(X, h + step, R, W) - kernel_loss(X, h - step, R, W)) / (2 * step)
    return np.array(out), dh


def rel_fro(x, ref):
    """||x - ref||_F / ||ref||_F in FP64."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def frobenius_ratio(A, R):
    """||A R||_F^2 / ||A||_F^2: the quantity the Frobenius stopping test relies on
    (section 4, Theorems 4.1-4.4: it concentrates at 1 for JL operators)."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A @ R) ** 2 / np.linalg.norm(A) ** 2)


def split_bf16x3(A):
    """Split FP32 values a = a1 + a2 + a3 with each part on the bfloat16 grid
    (round-to-nearest-even at every step).  Returns three FP64 arrays."""
    a = np.asarray(A, dtype=np.float32).astype(np.float64)
    a1 = ops.bf16_round(a)
    r1 = a - a1
    a2 = ops.bf16_round(r1)
    r2 = r1 - a2
    a3 = ops.bf16_round(r2)
    return a1, a2, a3

