"""Seeded synthetic inputs for the sketch workloads.

This module only builds inputs (point sets, dense test matrices, batch
descriptions, loss weights).  It holds none of the sketching arithmetic and is the
only code shared by the oracle-side tests and the GPU-side tests and benchmarks.

Matrices are returned as numpy arrays in Fortran (column-major) order, so that
``A[i, j]`` is entry (i, j) and ``A.T`` is a C-contiguous array whose memory is the
column-major matrix expected by the sketch library.

The paper's own test matrices (an exponential-kernel covariance on a finite
element mesh, a Toeplitz kinetic-energy operator, a boundary-element impedance
matrix and a multifrontal root front, section "Test Problems") are replaced by
the synthetic workloads below: Gaussian-kernel matrices on uniform random points
(smooth kernels, the same class as the covariance matrix), a Cauchy matrix (the
classical nonsymmetric HSS test matrix), and a batch of kernel matrices of
uneven size.
"""
import math

import numpy as np

DATA_SEED = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}
OP_SEED = {1: 2001, 2: 2002, 3: 2003, 4: 2004, 5: 2005}


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(n, dim, seed):
    """n points uniform in [0, 1]^dim (FP64, shape n x dim)."""
    return rng(seed).random((n, dim))


def bisection_order(X, leaf):
    """Permutation from recursive coordinate bisection.

    At each node the points are split along the coordinate of larger extent
    (first coordinate on ties) at the median position of a stable sort, into
    halves of floor(m/2) and ceil(m/2) points, until a node holds <= leaf points.
    The halves are emitted left to right, so index halving of the reordered set
    reproduces the bisection tree.
    """
    X = np.asarray(X)
    out = []
    stack = [np.arange(X.shape[0])]
    while stack:
        P = stack.pop()
        if P.size <= leaf:
            out.append(P)
            continue
        ext = X[P].max(0) - X[P].min(0)
        ax = int(np.argmax(ext))
        srt = P[np.argsort(X[P, ax], kind="stable")]
        h = P.size // 2
        stack.append(srt[h:])
        stack.append(srt[:h])
    return np.concatenate(out)


def gaussian_kernel_dense(X, h, shift, dtype=np.float64, threads=8):
    """K_ij = exp(-|x_i - x_j|^2 / (2 h^2)) + shift * delta_ij evaluated in FP64
    and rounded once to ``dtype``; column-major n x n.  Built column block by
    column block on a small thread pool (numpy releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    out = np.empty((n, n), dtype=dtype, order="F")
    inv = 1.0 / (2.0 * h * h)
    bs = 256

    def work(j0):
        j1 = min(n, j0 + bs)
        d2 = np.zeros((n, j1 - j0))
        for a in range(X.shape[1]):
            diff = X[:, a][:, None] - X[j0:j1, a][None, :]
            d2 += diff * diff
        blk = np.exp(-d2 * inv)
        if shift:
            blk[np.arange(j0, j1), np.arange(j1 - j0)] += shift
        out[:, j0:j1] = blk.astype(dtype)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, range(0, n, bs)))
    return out


def cauchy_dense(n, dtype=np.float64):
    """Nonsymmetric Cauchy matrix A_ij = 1 / (x_i - y_j), column-major.

    Interleaved points on a uniform grid: x_i = i/n, y_j = x_j + 0.5/n, so
    x_0 < y_0 < x_1 < y_1 < ... and |x_i - y_j| >= 0.5/n.  Every value is exact in
    FP64 before the single division (n a power of two)."""
    x = np.arange(n, dtype=np.float64) / n
    y = x + 0.5 / n
    A = np.empty((n, n), dtype=dtype, order="F")
    bs = 1024
    for j0 in range(0, n, bs):
        j1 = min(n, j0 + bs)
        A[:, j0:j1] = (1.0 / (x[:, None] - y[None, j0:j1])).astype(dtype)
    return A


# ------------------------------------------------------------------ the workloads
def cfg1():
    """Adaptive HSS of one n=1024 FP64 Gaussian-kernel matrix: points uniform in
    [0,1]^2, reordered by recursive coordinate bisection (leaf 64), h = 0.5,
    diagonal shift 1e-2; SJLT alpha = 4, d0 = 64, grown by 64 to eps_r = 1e-6."""
    n = 1024
    X = uniform_points(n, 2, DATA_SEED[1])
    X = X[bisection_order(X, 64)]
    A = gaussian_kernel_dense(X, 0.5, 1e-2, np.float64)
    return dict(n=n, X=X, A=A, h=0.5, shift=1e-2, leaf=64, alpha=4, d0=64, dd=64,
                eps_r=1e-6, eps_a=1e-8, seed=OP_SEED[1], symmetric=True)


def cfg2(n=16384):
    """Nonsymmetric FP64 Cauchy matrix, S = A R and S' = A^T R at d = 256 for the
    Gaussian, SJLT (alpha 4) and SRHT operators; HSS tolerance 1e-8."""
    return dict(n=n, A=cauchy_dense(n), d=256, alpha=4, eps_r=1e-8, eps_a=1e-8,
                leaf=256, seed=OP_SEED[2], symmetric=False)


def gaussian_kernel_device(X, h, shift, dtype="float32", bs=1024):
    """The same matrix as ``gaussian_kernel_dense``, built on the GPU with torch:
    FP64 evaluation (squared coordinate differences summed in coordinate order,
    exp, shift on the diagonal), rounded once to ``dtype``.  Returns an n x n
    column-major view (the transpose of a row-major buffer)."""
    import torch
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Xd = torch.from_numpy(X).cuda()
    T = torch.empty((n, n), dtype=getattr(torch, dtype), device="cuda")  # T[j, i] = K(i, j)
    inv = 1.0 / (2.0 * h * h)
    for j0 in range(0, n, bs):
        j1 = min(n, j0 + bs)
        d2 = torch.zeros((j1 - j0, n), dtype=torch.float64, device="cuda")
        for a in range(X.shape[1]):
            diff = Xd[:, a][None, :] - Xd[j0:j1, a][:, None]
            d2 += diff * diff
        K = torch.exp(-d2 * inv)
        if shift:
            r = torch.arange(j1 - j0, device="cuda")
            K[r, r + j0] += shift
        T[j0:j1, :] = K.to(T.dtype)
        del d2, K
    return T.t()


def cfg3_points(n=65536):
    return uniform_points(n, 3, DATA_SEED[3])


def cfg3(n=65536, threads=16):
    """FP32 Gaussian-kernel matrix on points uniform in [0,1]^3, h = 0.2, shift
    1e-3; d = 512 built in 8 blocks of 64; SJLT alpha = 8."""
    X = cfg3_points(n)
    A = gaussian_kernel_dense(X, 0.2, 1e-3, np.float32, threads=threads)
    return dict(n=n, X=X, A=A, h=0.2, shift=1e-3, d=512, block=64, alpha=8,
                seed=OP_SEED[3], sample_cols=sample_columns(512, 64, DATA_SEED[3]))


def sample_columns(d, count, seed):
    """``count`` distinct sketch columns in [0, d), sorted (seeded)."""
    return np.sort(rng(seed + 7).choice(d, size=min(count, d), replace=False))


def cfg4_specs(count=96, seed=DATA_SEED[4]):
    """Batch of ``count`` kernel matrices of uneven size.

    n_i = 64 * round(exp(U[ln 512, ln 8192]) / 64), points uniform in [0,1]^2,
    h_i ~ U[0.1, 1], sketch width d_i uniform on {64, 128, 192, 256}."""
    g = rng(seed)
    specs = []
    for i in range(count):
        n = int(64 * round(math.exp(g.uniform(math.log(512), math.log(8192))) / 64))
        n = max(64, n)
        h = float(g.uniform(0.1, 1.0))
        d = int(64 * g.integers(1, 5))
        specs.append(dict(n=n, h=h, d=d, point_seed=seed * 1000 + i))
    return specs


def cfg4_matrix(spec, dtype=np.float32):
    X = uniform_points(spec["n"], 2, spec["point_seed"])
    return gaussian_kernel_dense(X, spec["h"], 0.0, dtype)


def qchem_toeplitz_vector(n, spacing=0.1):
    """The defining vector of the paper's QChem Toeplitz test matrix (1-D kinetic
    energy, section 8.1): t[n - 1 + (i - j)] = T_ij with T_ii = pi^2 / (6 d^2) and
    T_ij = (-1)^(i-j) / (d^2 (i - j)^2) otherwise, d = ``spacing``.  Length 2n - 1,
    FP64 (symmetric, so t is a palindrome)."""
    r = np.arange(-(n - 1), n, dtype=np.float64)
    t = np.empty(2 * n - 1)
    off = r != 0
    t[off] = np.where(np.abs(r[off]) % 2 == 1, -1.0, 1.0) / (spacing * spacing * r[off] * r[off])
    t[~off] = math.pi ** 2 / (6.0 * spacing * spacing)
    return t


def qchem_toeplitz_dense(n, spacing=0.1, dtype=np.float64):
    """The QChem Toeplitz matrix stored dense, column-major: T_ij = t[n - 1 + i - j]."""
    t = qchem_toeplitz_vector(n, spacing)
    i = np.arange(n)
    return np.asfortranarray(t[n - 1 + i[:, None] - i[None, :]].astype(dtype))


def cfg5(N=32768):
    """Matrix-free differentiation: N points uniform in [0,1]^3 (FP32), bandwidth
    h = 0.3, SJLT alpha = 4, d = 256, loss weights W ~ N(0, 1) (N x 256)."""
    X = uniform_points(N, 3, DATA_SEED[5]).astype(np.float32)
    W = rng(DATA_SEED[5] + 1).standard_normal((N, 256)).astype(np.float32)
    return dict(N=N, X=X, W=np.asfortranarray(W), h=0.3, alpha=4, d=256,
                seed=OP_SEED[5])


def random_dense(m, n, seed, dtype=np.float64):
    """Dense column-major m x n with N(0, 1) entries (for property tests)."""
    return np.asfortranarray(rng(seed).standard_normal((m, n)).astype(dtype))
