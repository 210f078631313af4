"""GPU parity of the batched persistent SJLT sketch (many matrices of uneven size,
each grown in blocks) against the FP64 oracle, graph replays against eager runs,
reseeding, the autotuner, and the full 96-matrix batch on sampled columns."""
import numpy as np
import pytest
import torch

import workloads
from oracle import operators as ops
from oracle import sketch as osk

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


def _api():
    from paper_2302_01977_amd import api
    return api


def _small_batch(count, dtype, seed, square=True):
    g = np.random.Generator(np.random.PCG64(seed))
    mats, d, seeds = [], [], []
    for i in range(count):
        n = int(64 * g.integers(1, 17))          # 64 .. 1024, some ragged against the row tiles
        m = n if square else int(g.integers(40, 900))
        mats.append(workloads.random_dense(m, n, seed * 100 + i, dtype))
        d.append(int(64 * g.integers(1, 5)))
        seeds.append(int(g.integers(1, 2 ** 40)))
    return mats, d, seeds


def _oracle(A, d, dd, seed, transpose=False):
    R = ops.operator("sjlt", A.shape[1] if not transpose else A.shape[0], [dd] * (d // dd), seed, alpha=4)
    A64 = A.astype(np.float64)
    return (A64.T @ R) if transpose else (A64 @ R)


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_parity(ctx, dtype, tol, graph):
    api = _api()
    mats, d, seeds = _small_batch(11, dtype, 3)
    dev = [api.to_device_colmajor(A) for A in mats]
    b = api.Batch(ctx, dev, d, 64, seeds, graph=graph, transpose=True)
    nr, shape = b.info()
    assert nr == max(d) // 64
    b.run()
    torch.cuda.synchronize()
    for i, A in enumerate(mats):
        assert osk.rel_fro(b.S[i].cpu().numpy(), _oracle(A, d[i], 64, seeds[i])) <= tol, i
        assert osk.rel_fro(b.St[i].cpu().numpy(), _oracle(A, d[i], 64, seeds[i], True)) <= tol, i
    b.release()


def test_batch_rectangular_and_round_by_round(ctx):
    """m != n (S only), rounds run one at a time; every round writes only its block."""
    api = _api()
    mats, d, seeds = _small_batch(7, np.float32, 5, square=False)
    dev = [api.to_device_colmajor(A) for A in mats]
    b = api.Batch(ctx, dev, d, 64, seeds, graph=False)
    nr = b.info()[0]
    for S in b.S:
        S.fill_(float("nan"))
    for r in range(nr):
        b.run(r, r + 1)
        torch.cuda.synchronize()
        for i, A in enumerate(mats):
            got = b.S[i].cpu().numpy()
            if d[i] > 64 * r:
                ref = _oracle(A, 64 * (r + 1), 64, seeds[i])[:, 64 * r:]
                assert osk.rel_fro(got[:, 64 * r:64 * (r + 1)], ref) <= 1e-5, (i, r)
            assert np.isnan(got[:, 64 * (r + 1):]).all()  # later blocks untouched
    b.release()


def test_graph_replays_match_eager(ctx):
    """The captured rounds, replayed several times with eager work and
    synchronisations in between, reproduce the eager results bit for bit."""
    api = _api()
    mats, d, seeds = _small_batch(9, np.float32, 7)
    dev = [api.to_device_colmajor(A) for A in mats]
    eager = api.Batch(ctx, dev, d, 64, seeds, graph=False)
    eager.run()
    torch.cuda.synchronize()
    ref = [S.clone() for S in eager.S]
    eager.release()
    g = api.Batch(ctx, dev, d, 64, seeds, graph=True)
    for rep in range(4):
        for S in g.S:
            S.zero_()
        g.run()
        x = torch.randn(512, 512, device="cuda")     # the program's own eager work
        (x @ x).sum().item()
        torch.cuda.synchronize()
        for i in range(len(mats)):
            assert torch.equal(g.S[i], ref[i]), (rep, i)
    g.release()


def test_reseed_and_single_matrix_path(ctx):
    api = _api()
    mats, d, seeds = _small_batch(6, np.float64, 9)
    dev = [api.to_device_colmajor(A) for A in mats]
    b = api.Batch(ctx, dev, d, 64, seeds, graph=True)
    b.run()
    new = [s + 17 for s in seeds]
    b.reseed(new)
    b.run()
    torch.cuda.synchronize()
    for i, A in enumerate(mats):
        assert osk.rel_fro(b.S[i].cpu().numpy(), _oracle(A, d[i], 64, new[i])) <= 1e-12
        # the same operator through sketch_apply / sketch_extend
        sk = api.Sketch(ctx, dev[i], "sjlt", 64, new[i])
        if d[i] > 64:
            sk.extend(64, nblocks=d[i] // 64 - 1)
        torch.cuda.synchronize()
        assert osk.rel_fro(b.S[i].cpu().numpy(), sk.S.cpu().numpy()) <= 1e-13
        sk.release()
    b.release()


def test_autotune_picks_a_valid_shape(ctx):
    api = _api()
    mats, d, seeds = _small_batch(8, np.float32, 11)
    dev = [api.to_device_colmajor(A) for A in mats]
    b = api.Batch(ctx, dev, d, 64, seeds, graph=True, autotune=True)
    nr, shape = b.info()
    assert shape[0] in (64, 128, 256) and shape[1] * shape[2] == 64
    b.run()
    torch.cuda.synchronize()
    for i, A in enumerate(mats):
        assert osk.rel_fro(b.S[i].cpu().numpy(), _oracle(A, d[i], 64, seeds[i])) <= 1e-5
    # a second batch with the same signature reuses the cached shape
    b2 = api.Batch(ctx, dev, d, 64, seeds, graph=False, autotune=True)
    assert b2.info()[1] == shape
    b.release()
    b2.release()


def test_batch_errors(ctx):
    api = _api()
    A = api.to_device_colmajor(workloads.random_dense(64, 64, 1, np.float32))
    B = api.to_device_colmajor(workloads.random_dense(64, 64, 1, np.float64))
    with pytest.raises(api.SketchError):
        api.Batch(ctx, [A], [96], 64, [1])             # d not a multiple of dd
    with pytest.raises(api.SketchError):
        api.Batch(ctx, [A, B], [64, 64], 64, [1, 2])   # mixed dtypes
    with pytest.raises(api.SketchError):
        api.Batch(ctx, [A], [96], 32, [1])             # unsupported block width
    b = api.Batch(ctx, [A], [128], 64, [1], graph=False)
    with pytest.raises(api.SketchError):
        b.run(0, 3)                                    # only two rounds
    b.release()


def test_full_batch_96_matrices_sampled(ctx):
    """The 96-matrix batch (n_i log-uniform in [512, 8192], FP32 Gaussian kernel
    matrices, d_i in {64, ..., 256}): every matrix's 8 seeded sketch columns
    against the oracle."""
    api = _api()
    specs = workloads.cfg4_specs()
    seeds = [workloads.OP_SEED[4] + i for i in range(len(specs))]
    dev, hosts = [], []
    for sp in specs:
        A = workloads.cfg4_matrix(sp)
        hosts.append(A)
        dev.append(api.to_device_colmajor(A))
    d = [sp["d"] for sp in specs]
    b = api.Batch(ctx, dev, d, 64, seeds, graph=True)
    b.run()
    torch.cuda.synchronize()
    worst = 0.0
    for i, (sp, A) in enumerate(zip(specs, hosts)):
        cols = workloads.sample_columns(d[i], 8, 400 + i)
        ref = osk.sketch_columns(A, "sjlt", sp["n"], [64] * (d[i] // 64), seeds[i], cols)
        err = osk.rel_fro(b.S[i][:, cols].cpu().numpy(), ref)
        worst = max(worst, err)
        assert err <= 1e-5, (i, sp["n"], err)
    print("96-matrix batch: worst sampled rel.err %.2e" % worst)
    b.release()
