"""sketch_rerun_static, the allocation-free entry point, against sketch_rerun
(the entry point it mirrors) through the C ABI: two calls in a row, the second
on a smaller input, each bit-identical to sketch_rerun and within the oracle
tolerance; a call whose scratch exceeds the fixed array is refused cleanly."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from oracle import operators as ops
from oracle import sketch as osk

pytestmark = pytest.mark.gpu


def _static(api, sk, seed, S, St):
    lib = api.abi.load()
    out = api._output(S, St)
    return lib.sketch_rerun_static(sk.h, ctypes.byref(sk._in), seed, ctypes.byref(out),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _case(api, ctx, kind, dtype, n, d, alpha, prec="native", transpose=True):
    A = workloads.random_dense(n, n, 40 + n, dtype)
    sk = api.Sketch(ctx, api.to_device_colmajor(A), kind, d, 11, alpha=alpha, prec=prec, transpose=transpose)
    sk.extend(d)  # two blocks: one pass of 2d columns
    seed = 900 + n
    sk.rerun(seed)
    torch.cuda.synchronize()
    ref, reft = sk.S.clone(), (sk.St.clone() if transpose else None)
    S = torch.full_like(sk.S, float("nan"))
    St = torch.full_like(sk.St, float("nan")) if transpose else None
    rc = _static(api, sk, seed, S, St)
    assert rc == 0, api.abi.load().sketch_last_error()
    torch.cuda.synchronize()
    assert torch.equal(S, ref)
    if transpose:
        assert torch.equal(St, reft)
    if prec == "native":
        R = ops.operator(kind, n, [d, d], seed, alpha=alpha)
        tol = 1e-12 if dtype == np.float64 else 1e-5
        assert osk.rel_fro(S.cpu().numpy(), osk.sketch(A.astype(np.float64), R)) <= tol
    sk.release()


def test_rerun_static_matches_rerun():
    api = pytest.importorskip("paper_2302_01977_amd.api")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with api.Context(0) as ctx:
        # first call: n = 3000 FP64 SJLT, two blocks of 32, S and S': the source
        # range is split 22 ways, 34 MB of partial sums in the fixed array
        _case(api, ctx, "sjlt", np.float64, 3000, 32, 4)
        # second call, smaller input: the array keeps the first call's partials
        _case(api, ctx, "sjlt", np.float32, 1000, 32, 8)
        _case(api, ctx, "srht", np.float64, 1024, 64, 1)
        _case(api, ctx, "gaussian", np.float32, 768, 64, 1, prec="bf16x3", transpose=False)
        # matrix-free input
        X = torch.from_numpy(workloads.uniform_points(700, 3, 4).astype(np.float32)).cuda()
        sk = api.Sketch(ctx, None, "sjlt", 64, 3, alpha=4, points=(X, 0.3, 0.0))
        sk.rerun(17)
        torch.cuda.synchronize()
        ref = sk.S.clone()
        S = torch.full_like(ref, float("nan"))
        assert _static(api, sk, 17, S, None) == 0
        torch.cuda.synchronize()
        assert torch.equal(S, ref)
        sk.release()


def test_rerun_static_refuses_oversized_scratch():
    """bf16x3 Gaussian, m = 12288, n = 8192, 1024 columns: two source slices of
    12288 x 1024 FP32 partials (96 MiB) exceed the 64 MiB array."""
    api = pytest.importorskip("paper_2302_01977_amd.api")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with api.Context(0) as ctx:
        m, n, d = 12288, 8192, 1024
        A = torch.randn(n, m, dtype=torch.float32, device="cuda").T
        sk = api.Sketch(ctx, A, "gaussian", d, 5, prec="bf16x3")
        torch.cuda.synchronize()
        first = sk.S.clone()
        S = torch.empty_like(sk.S)
        rc = _static(api, sk, 6, S, None)
        msg = api.abi.load().sketch_last_error().decode()
        assert rc == api.abi.SK_EINVAL and "scratch" in msg and str(64 << 20) in msg
        # the handle keeps its operator: a rerun with the original seed reproduces the first sketch
        sk.rerun(5)
        torch.cuda.synchronize()
        assert torch.equal(sk.S, first)
        sk.release()
