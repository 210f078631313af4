"""Adaptive HSS compression (the oracle's Algorithm 1) driven by sketches computed
on the GPU through the C ABI: the n = 1024 kernel workload with SJLT, Gaussian
and SRHT operators and a nonsymmetric Cauchy matrix (S and S').  Several
results are correct (rounding can move a pivot), so runs are compared by final
width, ranks and error, not bit for bit."""
import numpy as np
import pytest
import torch

import workloads
from oracle import hss

pytestmark = pytest.mark.gpu


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


class GPUSketcher:
    """add_block / R_rows for ``hss.compress``: sketch_apply for the first block,
    sketch_extend for the following ones, R rows from sketch_get_rows."""

    def __init__(self, ctx, A, kind, seed, alpha=4, symmetric=True):
        from paper_2302_01977_amd import api
        self.api, self.ctx = api, ctx
        self.Ad = api.to_device_colmajor(A)
        self.kind, self.seed, self.alpha, self.symmetric = kind, seed, alpha, symmetric
        self.sk = None
        self.widths = []

    def add_block(self, w):
        if self.sk is None:
            self.sk = self.api.Sketch(self.ctx, self.Ad, self.kind, w, self.seed, alpha=self.alpha,
                                      transpose=not self.symmetric)
            S, St = self.sk.S, self.sk.St
        else:
            S, St = self.sk.extend(w)
        self.widths.append(w)
        torch.cuda.synchronize()
        return S.cpu().numpy(), (None if self.symmetric else St.cpu().numpy())

    def R_rows(self, rows, c0, c1):
        rows = np.asarray(rows)
        i0, i1 = int(rows.min()), int(rows.max()) + 1
        return self.sk.get_rows(i0, i1, c0, c1)[rows - i0]

    def release(self):
        if self.sk is not None:
            self.sk.release()


@pytest.mark.parametrize("kind", ["sjlt", "gaussian", "srht"])
def test_kernel_matrix_hss_with_gpu_sketches(ctx, kind):
    c = workloads.cfg1()
    A = c["A"]
    gs = GPUSketcher(ctx, A, kind, c["seed"], alpha=c["alpha"], symmetric=True)
    res = hss.compress(A, c["leaf"], gs, d0=c["d0"], dd=c["dd"], eps_r=c["eps_r"], eps_a=c["eps_a"],
                       symmetric=True)
    gs.release()
    os_ = hss.OracleSketcher(A, kind, c["seed"], alpha=c["alpha"], symmetric=True)
    ref = hss.compress(A, c["leaf"], os_, d0=c["d0"], dd=c["dd"], eps_r=c["eps_r"], eps_a=c["eps_a"],
                       symmetric=True)
    err, err_ref = hss.relative_error(A, res), hss.relative_error(A, ref)
    print("%s: final d %d (oracle %d), max rank %d (%d), error %.2e (%.2e)"
          % (kind, res.final_d, ref.final_d, res.max_rank(), ref.max_rank(), err, err_ref))
    assert res.converged and ref.converged
    assert err <= 10 * c["eps_r"]
    assert res.final_d == ref.final_d
    assert abs(res.max_rank() - ref.max_rank()) <= 2


def test_nonsymmetric_cauchy_hss_with_gpu_sketches(ctx):
    n = 2048
    A = workloads.cauchy_dense(n)
    gs = GPUSketcher(ctx, A, "sjlt", 77, alpha=4, symmetric=False)
    res = hss.compress(A, 256, gs, d0=64, dd=64, eps_r=1e-8, eps_a=1e-8, symmetric=False)
    gs.release()
    err = hss.relative_error(A, res)
    print("cauchy n=%d: final d %d, max rank %d, error %.2e" % (n, res.final_d, res.max_rank(), err))
    assert res.converged
    assert err <= 1e-7


@pytest.mark.parametrize("kind", ["sjlt", "srht"])
def test_qchem_toeplitz_hss_with_gpu_sketches(ctx, kind):
    """The paper's QChem Toeplitz matrix (section 8.1, d = 0.1) at n = 1000 (SRHT
    on a non-power-of-two n): GPU sketches against the oracle's own, compared by
    final width, ranks and error."""
    n = 1000
    A = workloads.qchem_toeplitz_dense(n, 0.1)
    gs = GPUSketcher(ctx, A, kind, 91, alpha=4, symmetric=True)
    res = hss.compress(A, 64, gs, d0=64, dd=64, eps_r=1e-6, eps_a=1e-8, symmetric=True)
    gs.release()
    os_ = hss.OracleSketcher(A, kind, 91, alpha=4, symmetric=True)
    ref = hss.compress(A, 64, os_, d0=64, dd=64, eps_r=1e-6, eps_a=1e-8, symmetric=True)
    err = hss.relative_error(A, res)
    print("toeplitz %s: final d %d (oracle %d), max rank %d (%d), error %.2e"
          % (kind, res.final_d, ref.final_d, res.max_rank(), ref.max_rank(), err))
    assert res.converged and err <= 1e-5
    assert res.final_d == ref.final_d and abs(res.max_rank() - ref.max_rank()) <= 2
