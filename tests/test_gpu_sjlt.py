"""GPU parity of the SJLT path against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import operators as ops
from oracle import sketch as osk

pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-12, np.float32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    from paper_2302_01977_amd import api
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    import gc
    gc.collect()
    c.close()


def _api():
    from paper_2302_01977_amd import api
    return api


@pytest.mark.parametrize("n,w,alpha,block,seed", [(1000, 64, 4, 0, 5), (4096, 256, 4, 0, 6),
                                                  (333, 32, 8, 0, 9), (64, 16, 1, 0, 1)])
def test_hash_bit_exact(ctx, n, w, alpha, block, seed):
    api = _api()
    A = api.to_device_colmajor(np.ones((1, n)))
    sk = api.Sketch(ctx, A, "sjlt", w, seed, alpha=alpha)
    codes = sk.sjlt_codes(0, alpha)
    cols, signs = ops.sjlt_hash(n, w, alpha, block, seed)
    assert np.array_equal(codes >> 1, cols)
    assert np.array_equal(codes & 1, (signs < 0).astype(np.uint32))
    sk.release()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("m,n,w,alpha", [(1000, 1000, 64, 4), (1024, 1024, 256, 4), (777, 777, 64, 8),
                                         (130, 70, 32, 4), (65, 4097, 48, 16)])
def test_sketch_parity(ctx, dtype, m, n, w, alpha):
    api = _api()
    A = workloads.random_dense(m, n, 11, dtype)
    Ad = api.to_device_colmajor(A)
    square = m == n
    sk = api.Sketch(ctx, Ad, "sjlt", w, 123, alpha=alpha, transpose=square)
    torch.cuda.synchronize()
    R = ops.sjlt_block(n, w, alpha, 0, 123)
    A64 = A.astype(np.float64)
    assert osk.rel_fro(sk.S.cpu().numpy(), osk.sketch(A64, R)) <= TOL[dtype]
    if square:
        assert osk.rel_fro(sk.St.cpu().numpy(), osk.sketch_t(A64, R)) <= TOL[dtype]
    sk.release()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,w,alpha", [(1536, 512, 4), (2048, 256, 8), (1100, 256, 4)])
def test_wide_and_dense_buckets(ctx, dtype, n, w, alpha):
    """Passes of 256 and more columns (16-wave launches), long buckets
    (alpha = 8) and a ragged square matrix: S and S' against the oracle."""
    api = _api()
    A = workloads.random_dense(n, n, 17, dtype)
    sk = api.Sketch(ctx, api.to_device_colmajor(A), "sjlt", w, 321, alpha=alpha, transpose=True)
    torch.cuda.synchronize()
    R = ops.sjlt_block(n, w, alpha, 0, 321)
    A64 = A.astype(np.float64)
    assert osk.rel_fro(sk.S.cpu().numpy(), osk.sketch(A64, R)) <= TOL[dtype]
    assert osk.rel_fro(sk.St.cpu().numpy(), osk.sketch_t(A64, R)) <= TOL[dtype]
    sk.release()


def _device_view(A, ld, off, dtype):
    """Column-major device copy of A with leading dimension ld >= rows, starting
    off elements into its buffer (off = 1 leaves the columns without 16-byte
    alignment for FP64 and FP32)."""
    m, n = A.shape
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    buf = torch.zeros(off + ld * n, dtype=tdt, device="cuda")
    M = buf[off:].view(n, ld).t()[:m, :]
    M.copy_(torch.from_numpy(np.ascontiguousarray(A)).to("cuda"))
    return M


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("m,n,w,alpha,ld,off", [(700, 700, 1024, 4, 700, 0),    # widest block
                                                (500, 500, 256, 32, 500, 0),    # 32 nonzeros per row
                                                (3, 1, 16, 4, 3, 0),            # one source
                                                (1, 5, 16, 1, 1, 0),            # one row
                                                (257, 257, 64, 4, 260, 1)])     # padded, unaligned
def test_edge_shapes(ctx, dtype, m, n, w, alpha, ld, off):
    """Extremes of the block width and of alpha, single rows and sources, and a
    matrix whose columns are neither contiguous nor 16-byte aligned."""
    api = _api()
    A = workloads.random_dense(m, n, 23, dtype)
    Ad = _device_view(A, ld, off, dtype)
    sk = api.Sketch(ctx, Ad, "sjlt", w, 55, alpha=alpha, transpose=m == n)
    torch.cuda.synchronize()
    R = ops.sjlt_block(n, w, alpha, 0, 55)
    A64 = A.astype(np.float64)
    assert osk.rel_fro(sk.S.cpu().numpy(), osk.sketch(A64, R)) <= TOL[dtype]
    if m == n:
        assert osk.rel_fro(sk.St.cpu().numpy(), osk.sketch_t(A64, R)) <= TOL[dtype]
    sk.release()


def test_extension_multiblock_and_determinism(ctx):
    api = _api()
    n = 2048
    A = workloads.random_dense(n, n, 2, np.float64)
    Ad = api.to_device_colmajor(A)
    sk = api.Sketch(ctx, Ad, "sjlt", 64, 77, alpha=4, transpose=True)
    Sn, Stn = sk.extend(64, nblocks=3)          # three new blocks in one pass
    sk.extend(128, nblocks=1)
    torch.cuda.synchronize()
    assert sk.width == (64 + 192 + 128, 5)
    R = ops.operator("sjlt", n, [64, 64, 64, 64, 128], 77, alpha=4)
    assert osk.rel_fro(sk.S.cpu().numpy(), A @ R) <= 1e-12
    assert osk.rel_fro(sk.St.cpu().numpy(), A.T @ R) <= 1e-12
    # same blocks drawn one at a time give bit-identical columns
    sk2 = api.Sketch(ctx, Ad, "sjlt", 64, 77, alpha=4, transpose=True)
    for _ in range(3):
        sk2.extend(64)
    sk2.extend(128)
    torch.cuda.synchronize()
    assert torch.equal(sk.S, sk2.S) and torch.equal(sk.St, sk2.St)
    # rerun with the same seed reproduces everything bit for bit
    S0 = sk.S.clone()
    sk.rerun(77)
    torch.cuda.synchronize()
    assert torch.equal(S0, sk.S)
    # rerun with a new seed matches the oracle's operator for that seed
    sk.rerun(78)
    torch.cuda.synchronize()
    R78 = ops.operator("sjlt", n, [64, 64, 64, 64, 128], 78, alpha=4)
    assert osk.rel_fro(sk.S.cpu().numpy(), A @ R78) <= 1e-12
    sk.release()
    sk2.release()


@pytest.mark.parametrize("dtype,n,w,alpha,nb", [(np.float32, 2085, 64, 8, 3), (np.float32, 2085, 64, 8, 4),
                                                 (np.float32, 1500, 64, 8, 7), (np.float32, 1100, 128, 4, 3),
                                                 (np.float64, 1300, 64, 8, 3)])
def test_wide_passes(ctx, dtype, n, w, alpha, nb):
    """Passes wider than eight waves of columns (16 waves of 16 columns with
    several rows per lane, one workgroup per 256 columns): S and S' of the new
    blocks against the oracle, ragged n."""
    api = _api()
    A = workloads.random_dense(n, n, 12, dtype)
    Ad = api.to_device_colmajor(A)
    sk = api.Sketch(ctx, Ad, "sjlt", w, 31, alpha=alpha, transpose=True)
    Sn, Stn = sk.extend(w, nblocks=nb)
    torch.cuda.synchronize()
    Rall = ops.operator("sjlt", n, [w] * (nb + 1), 31, alpha=alpha)
    R = Rall[:, w:]
    A64 = A.astype(np.float64)
    assert osk.rel_fro(Sn.cpu().numpy().astype(np.float64), A64 @ R) <= TOL[dtype]
    assert osk.rel_fro(Stn.cpu().numpy().astype(np.float64), A64.T @ R) <= TOL[dtype]
    # the apply (one block of w columns: a narrow pass)
    assert osk.rel_fro(sk.S[:, :w].cpu().numpy().astype(np.float64), A64 @ Rall[:, :w]) <= TOL[dtype]
    assert osk.rel_fro(sk.St[:, :w].cpu().numpy().astype(np.float64), A64.T @ Rall[:, :w]) <= TOL[dtype]
    sk.release()


def test_identity_gives_R_and_linearity(ctx):
    api = _api()
    n, w = 512, 64
    I = api.to_device_colmajor(np.eye(n))
    sk = api.Sketch(ctx, I, "sjlt", w, 5, alpha=4, transpose=True)
    torch.cuda.synchronize()
    R = ops.sjlt_block(n, w, 4, 0, 5)
    assert np.array_equal(sk.S.cpu().numpy(), R)
    assert np.array_equal(sk.St.cpu().numpy(), R)
    sk.release()
    A = workloads.random_dense(n, n, 1)
    B = workloads.random_dense(n, n, 2)
    outs = []
    for M in (A, B, 2 * A - 3 * B):
        s = api.Sketch(ctx, api.to_device_colmajor(M), "sjlt", w, 5, alpha=4)
        torch.cuda.synchronize()
        outs.append(s.S.cpu().numpy())
        s.release()
    assert osk.rel_fro(outs[2], 2 * outs[0] - 3 * outs[1]) < 1e-13


def test_get_rows_matches_oracle(ctx):
    api = _api()
    n = 300
    A = api.to_device_colmajor(np.ones((2, n)))
    sk = api.Sketch(ctx, A, "sjlt", 32, 4, alpha=4)
    sk.extend(48)
    R = ops.operator("sjlt", n, [32, 48], 4, alpha=4)
    assert np.array_equal(sk.get_rows(0, n, 0, 80), R)
    assert np.array_equal(sk.get_rows(17, 250, 30, 70), R[17:250, 30:70])
    sk.release()


def test_argument_errors(ctx):
    api = _api()
    A = api.to_device_colmajor(np.ones((8, 8)))
    with pytest.raises(api.SketchError) as e:
        api.Sketch(ctx, A, "sjlt", 30, 1, alpha=4)      # alpha does not divide 30
    assert e.value.code == -1
    # SRHT takes any n (nu = 16 for n = 12)
    sk = api.Sketch(ctx, api.to_device_colmajor(np.ones((8, 12))), "srht", 16, 1)
    torch.cuda.synchronize()
    assert osk.rel_fro(sk.S.cpu().numpy(), np.ones((8, 12)) @ ops.srht_block(12, 16, 0, 1)) <= 1e-12
    sk.release()
    with pytest.raises(api.SketchError) as e:
        api.Sketch(ctx, A, "sjlt", 24, 1, alpha=4)      # widths are multiples of 16
    assert e.value.code == -1
    with pytest.raises(api.SketchError) as e:
        api.Sketch(ctx, A, "sjlt", 1040, 1, alpha=4)    # wider than a block may be
    assert e.value.code == -1
    A2 = api.to_device_colmajor(np.ones((8, 12)))
    with pytest.raises(api.SketchError):
        api.Sketch(ctx, A2, "sjlt", 16, 1, alpha=4, transpose=True)   # S' needs square A


def test_cauchy_full_size_sampled_columns(ctx):
    """The n = 16384 FP64 Cauchy workload at d = 256: S and S' on the GPU, 64
    seeded columns of each checked against the oracle (sampled-column form)."""
    api = _api()
    c = workloads.cfg2()
    A, n, d = c["A"], c["n"], c["d"]
    Ad = api.to_device_colmajor(A)
    sk = api.Sketch(ctx, Ad, "sjlt", d, c["seed"], alpha=c["alpha"], transpose=True)
    torch.cuda.synchronize()
    cols = workloads.sample_columns(d, 64, 99)
    ref = osk.sketch_columns(A, "sjlt", n, [d], c["seed"], cols, alpha=4)
    reft = osk.sketch_columns(A, "sjlt", n, [d], c["seed"], cols, alpha=4, transpose=True)
    assert osk.rel_fro(sk.S[:, cols].cpu().numpy(), ref) <= 1e-12
    assert osk.rel_fro(sk.St[:, cols].cpu().numpy(), reft) <= 1e-12
    sk.release()
