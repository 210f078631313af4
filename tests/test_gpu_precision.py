"""Full-size precision workload: an n = 65536 FP32 Gaussian-kernel matrix
(17.2 GB on the device; points uniform in [0,1]^3, h = 0.2, diagonal shift 1e-3),
sketched to d = 512 in 8 blocks of 64 (apply, then seven extensions) with the
Gaussian operator in BF16 and bf16x3 MFMA, FP32 SJLT (alpha = 8) and FP32 SRHT.
Each result is checked against the FP64 oracle on 64 seeded sampled rows of S:
row i of S is row i of A times the explicit operator, so the oracle needs only
those rows of A, evaluated in FP64 and rounded once to FP32 exactly as the
device copy was."""
import numpy as np
import pytest
import torch

import workloads
from oracle import operators as ops
from oracle import sketch as osk

pytestmark = pytest.mark.gpu

N = 65536
H = 0.2
SHIFT = 1e-3
BLOCK = 64
NBLK = 8
ALPHA = 8


@pytest.fixture(scope="module")
def ctx():
    from paper_2302_01977_amd import api
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def big():
    """Device A (column-major FP32) built in FP64 and rounded once, and the
    oracle's copy of 64 sampled rows of it (the same arithmetic on the host)."""
    X = workloads.cfg3_points(N)
    A = workloads.gaussian_kernel_device(X, H, SHIFT, "float32")
    torch.cuda.synchronize()
    rows = workloads.sample_columns(N, 64, workloads.DATA_SEED[3])
    inv = 1.0 / (2.0 * H * H)
    Ar = np.empty((len(rows), N))
    for r, i in enumerate(rows):
        d2 = np.zeros(N)
        for a in range(X.shape[1]):
            diff = X[i, a] - X[:, a]
            d2 += diff * diff
        k = np.exp(-d2 * inv)
        k[i] += SHIFT
        Ar[r] = k.astype(np.float32).astype(np.float64)
    yield A, rows, Ar
    del A
    torch.cuda.empty_cache()


def _sketch(ctx, A, kind, prec):
    from paper_2302_01977_amd import api
    kw = {"alpha": ALPHA} if kind == "sjlt" else {}
    if prec:
        kw["prec"] = prec
    sk = api.Sketch(ctx, A, kind, BLOCK, workloads.OP_SEED[3], **kw)
    for _ in range(NBLK - 1):
        sk.extend(BLOCK)
    torch.cuda.synchronize()
    return sk


@pytest.mark.parametrize("kind,prec,tol", [("sjlt", None, 1e-5), ("srht", None, 1e-5),
                                           ("gaussian", "bf16x3", 1e-5), ("gaussian", "bf16", 2e-2)])
def test_full_size_sampled_rows(ctx, big, kind, prec, tol):
    A, rows, Ar = big
    sk = _sketch(ctx, A, kind, prec)
    assert sk.width == (BLOCK * NBLK, NBLK)
    got = sk.S[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    sk.release()
    R = ops.operator(kind, N, [BLOCK] * NBLK, workloads.OP_SEED[3], alpha=ALPHA)
    ref = Ar @ R
    err = osk.rel_fro(got, ref)
    print("n=65536 %s %s: rel. error %.3e on 64 sampled rows" % (kind, prec or "fp32", err))
    assert err <= tol
    if prec == "bf16":
        assert err > 1e-5   # plain bf16 really rounds A
