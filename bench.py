"""Benchmark of the sketch hot path on one MI355X.

Default workload: the nonsymmetric FP64 Cauchy matrix, n = 16384, column-major,
S = A R and S' = A^T R at d = 256 (one block).  One step = draw the operator
block on the device (hash + bucket tables) and compute S and S' through the C
ABI.  The metric is the effective bandwidth of the SJLT sketch (alpha = 4):
algorithmic bytes (read A once per sketch + write the new columns) divided by the
step time, with A already resident in HBM.

Reported beside it, on the same GPU and in the same run:
  * the other operator kinds on the same FP64 matrix (SRHT, FP64 Gaussian on
    MFMA) and the library FP64 GEMM (rocBLAS through torch) on the same shapes;
  * the same matrix rounded to FP32: SJLT, SRHT, Gaussian in BF16 and bf16x3,
    each with its relative error against the FP64-arithmetic Gaussian path;
  * the matrix-free kernel sketch and its backward (N = 32768 points in 3-D,
    d = 256);
  * the batched sketch of 96 kernel matrices of uneven size, one persistent
    graph launch per round, against per-matrix launches;
  * a measured copy bandwidth (torch copy of A), the reference for the HBM
    counters, and a measured read bandwidth (torch column sums of A);
  * the FP64 CPU oracle timed on the host cores (a reported baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KERNELS = {"sjlt": ("sjlt_gather", "sjlt_gather_t", "sjlt_reduce", "sjlt_meta"),
           "srht": ("srht", "srht_t"),
           "gaussian": ("gauss_f64", "gauss_f64_t"),
           "bf16": ("gauss_bf16", "gauss_bf16_t"),
           "bf16x3": ("gauss_bf16x3", "gauss_bf16x3_t")}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
# VALU issue without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
# the step kernels' sources: the recorded traffic figures are valid only for them
GATHER_SOURCES = ("paper_2302_01977_amd/csrc/sjlt.hip", "paper_2302_01977_amd/csrc/sjlt_dma.hip",
                  "paper_2302_01977_amd/csrc/sjlt_tile.hpp", "paper_2302_01977_amd/csrc/gather.hpp")
# rocprofv3 FETCH_SIZE / WRITE_SIZE summaries of the step's two kernels (S, S')
TRAFFIC_FILES = {"sjlt_gather": os.path.join(ROOT, "profiles", "sjlt_gather_S_cauchy16k_traffic.txt"),
                 "sjlt_gather_t": os.path.join(ROOT, "profiles", "sjlt_gather_St_cauchy16k_traffic.txt")}
STEP_KERNELS = {"sjlt_gather": "sjlt_gather_kernel<double, false, 16, 16, 1, 256, true, false> (S = A R)",
                "sjlt_gather_t": "sjlt_gather_kernel<double, true, 16, 16, 1, 256, true, false> (S' = A^T R)"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default="cauchy16k", choices=["cauchy16k"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--leg", default="all",
                   choices=["all", "main", "srht", "gaussian", "fp32", "mf", "batch", "precision", "hss",
                            "hss_device"],
                   help="run one leg only and print its figures (for profiling); 'main' = the SJLT step with "
                        "the copy and read references")
    p.add_argument("--only-main", action="store_true", help="same as --leg main")
    p.add_argument("--only-mf", action="store_true", help="same as --leg mf")
    a = p.parse_args()
    if a.only_main:
        a.leg = "main"
    if a.only_mf:
        a.leg = "mf"
    return a


def time_steps(fn, steps, warmup):
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(steps):
        fn(warmup + i)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def kernel_times(ctx, fn, names, reps):
    """Average duration per launch of each kernel family, from the HIP events the
    library records on the stream it launches on."""
    import torch
    ctx.profile(True)
    ctx.profile_read("", reset=True)
    for i in range(reps):
        fn(1000 + i)
    torch.cuda.synchronize()
    out = {}
    for name in names:
        tot, cnt = ctx.profile_read(name)
        if cnt:
            out[name] = {"avg_ms": tot / cnt, "launches": cnt}
    ctx.profile_read("", reset=True)
    ctx.profile(False)
    return out


def sources_digest():
    h = hashlib.sha256()
    for rel in GATHER_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(path):
    """HBM bytes per launch of a step kernel from its committed rocprofv3
    counter summary, if it was taken on the current kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_digest") != sources_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(A, d, alpha, seed, budget_s=12.0, max_reps=50):
    """The FP64 oracle on the host: operator materialisation + S = A R + S' = A^T R
    for the full workload, repeated until ~budget_s of CPU work."""
    from oracle import operators as ops
    from oracle import sketch as osk
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    reps, t_tot = 0, 0.0
    while t_tot < budget_s and reps < max_reps:
        t = time.perf_counter()
        R = ops.sjlt_block(A.shape[1], d, alpha, 0, seed + reps)
        osk.sketch(A, R)
        osk.sketch_t(A, R)
        t_tot += time.perf_counter() - t
        reps += 1
    return t_tot / reps, cores, reps


def cpu_baseline_extras(A, d, alpha, seed):
    """Beside the main figure: the same oracle step on one thread (a few
    repetitions), and the oracle's adaptive HSS compression of the n = 1024
    kernel matrix with its own SJLT sketches (the whole Algorithm 1 run)."""
    import workloads
    from oracle import hss
    out = {}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1, _, r1 = cpu_baseline(A, d, alpha, seed, budget_s=4.0, max_reps=3)
        out["one_thread"] = {"s_per_step": round(t1, 6), "reps": r1}
    except ImportError:
        pass
    c = workloads.cfg1()
    t = time.perf_counter()
    sk = hss.OracleSketcher(c["A"], "sjlt", c["seed"], alpha=c["alpha"], symmetric=True)
    res = hss.compress(c["A"], c["leaf"], sk, d0=c["d0"], dd=c["dd"], eps_r=c["eps_r"], eps_a=c["eps_a"],
                       symmetric=True)
    out["hss_1024_compress"] = {"s": round(time.perf_counter() - t, 4), "final_d": int(res.final_d),
                                "max_rank": int(res.max_rank()), "converged": bool(res.converged)}
    return out


def cpu_baseline_workloads(A2, seed2):
    """The oracle on samples of the other workloads, each timed on the host and
    scaled to the whole workload by its arithmetic (clearly a per-unit
    extrapolation, not a run of the whole thing):
      * n = 65536 FP32 kernel matrix, SJLT alpha = 8, d = 512: the 64 sampled
        columns of S on the first 512 rows, scaled by 65536 / 512 rows and
        512 / 64 columns;
      * the 96-matrix batch: S = A_i R_i for 8 of the matrices, scaled by
        sum n_i^2 d_i over the batch;
      * the matrix-free forward (N = 32768, d = 256): 1024 rows of S = K R,
        scaled by N / 1024;
      * the adaptive HSS compression of the n = 16384 Cauchy matrix (SJLT,
        eps_r = 1e-8): the whole oracle run."""
    import numpy as np

    import workloads
    from oracle import hss
    from oracle import operators as ops
    from oracle import sketch as osk
    out = {}
    # n = 65536: sampled columns on a row block
    n3, rows = 65536, 512
    X = workloads.cfg3_points(n3)
    d2 = np.zeros((rows, n3))
    for a in range(3):
        diff = X[:rows, a][:, None] - X[:, a][None, :]
        d2 += diff * diff
    blk = np.exp(-d2 / (2.0 * 0.2 * 0.2))
    blk[np.arange(rows), np.arange(rows)] += 1e-3
    blk = blk.astype(np.float32)
    del d2
    cols = workloads.sample_columns(512, 64, workloads.DATA_SEED[3])
    t = time.perf_counter()
    osk.sketch_columns(blk, "sjlt", n3, [64] * 8, workloads.OP_SEED[3], cols, alpha=8)
    dt = time.perf_counter() - t
    out["n65536_sjlt8_d512"] = {"sample": "64 sampled columns of S on rows 0..511", "sample_s": round(dt, 4),
                                "extrapolated_full_s": round(dt * (n3 / rows) * (512 / 64), 2)}
    del blk
    # batch: 8 of the 96 matrices
    specs = workloads.cfg4_specs()
    tot = sum(sp["n"] ** 2 * sp["d"] for sp in specs)
    smp, t_s = 0, 0.0
    for i, sp in enumerate(specs[:8]):
        Ai = workloads.cfg4_matrix(sp)
        t = time.perf_counter()
        osk.sketch(Ai, ops.operator("sjlt", sp["n"], [64] * (sp["d"] // 64), workloads.OP_SEED[4] + i, alpha=4))
        t_s += time.perf_counter() - t
        smp += sp["n"] ** 2 * sp["d"]
    out["batch96"] = {"sample": "S = A_i R_i for 8 of the 96 matrices", "sample_s": round(t_s, 4),
                      "extrapolated_full_s": round(t_s * tot / smp, 3)}
    # matrix-free forward
    c5 = workloads.cfg5()
    R5 = ops.sjlt_block(c5["N"], c5["d"], c5["alpha"], 0, c5["seed"])
    t = time.perf_counter()
    osk.kernel_sketch_rows(c5["X"].astype(np.float64), float(np.float32(c5["h"])), R5, np.arange(1024))
    dt = time.perf_counter() - t
    out["matrix_free_forward"] = {"sample": "1024 of the 32768 rows of S = K(X, h) R", "sample_s": round(dt, 4),
                                  "extrapolated_full_s": round(dt * c5["N"] / 1024, 2)}
    # adaptive HSS of the Cauchy matrix, whole run
    t = time.perf_counter()
    sk = hss.OracleSketcher(A2, "sjlt", seed2, alpha=4, symmetric=False)
    res = hss.compress(A2, 256, sk, d0=64, dd=64, eps_r=1e-8, eps_a=1e-8, symmetric=False)
    out["cauchy16k_hss_compress"] = {"s": round(time.perf_counter() - t, 3), "final_d": int(res.final_d),
                                     "max_rank": int(res.max_rank()), "converged": bool(res.converged)}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def rel_err(x, ref):
    import torch
    return float(torch.linalg.norm((x.double() - ref.double())) / torch.linalg.norm(ref.double()))


def stored_leg(api, ctx, A, kind, d, seed, alpha, prec, steps, warmup, bytes_step, construction="block"):
    import torch
    try:
        sk = api.Sketch(ctx, A, kind, d, seed, alpha=alpha, prec=prec, transpose=True, construction=construction)
    except api.SketchError as e:
        return {"unavailable": str(e)}, None
    ms = time_steps(lambda i: sk.rerun(seed + i), steps, warmup)
    names = KERNELS[prec if kind == "gaussian" and prec != "native" else kind]
    kern = kernel_times(ctx, lambda i: sk.rerun(seed + i), names, max(3, steps // 2))
    sk.rerun(seed)
    torch.cuda.synchronize()
    r = {"ms_per_step": ms, "GBps": bytes_step / (ms * 1e-3) / 1e9, "kernels": kern}
    return r, sk


def matrix_free_leg(api, ctx, steps, warmup):
    import numpy as np
    import torch

    import workloads
    c = workloads.cfg5()
    N, d = c["N"], c["d"]
    X = torch.from_numpy(c["X"]).cuda()
    W = api.to_device_colmajor(np.asarray(c["W"]))
    sk = api.Sketch(ctx, None, "sjlt", d, c["seed"], alpha=c["alpha"], points=(X, c["h"], 0.0))
    fwd_ms = time_steps(lambda i: sk.rerun(c["seed"] + i), steps, warmup)
    bsteps = max(2, steps // 4)
    bwd_ms = time_steps(lambda i: sk.adjoint(W), bsteps, 1)
    kern = kernel_times(ctx, lambda i: (sk.rerun(c["seed"] + i), sk.adjoint(W)),
                        ("mf_fwd", "mf_bwd", "sjlt_meta", "sjlt_reduce"), max(2, steps // 4))
    sk.release()
    pairs = float(N) * N
    # VALU lane-operations per (i, k) pair, counted from the kernels' arithmetic
    # (dim = 3, alpha = 4; the transcendental exp2 issues at a quarter rate):
    #   forward : 3 sub + 3 fma + 1 mul + exp2 (4 slots) + 4 signed fma          = 15
    #   backward: 3 sub + 3 fma + 1 mul + exp2 (4) + 8 fma (G_ij, G_ji) + 3 fma
    #             (dX terms) + 2 mul + cvt + f64 add (dh term)                   = 28
    out = {"workload": "N=%d points in [0,1]^3, h=%.1f, SJLT alpha=%d, d=%d" % (N, c["h"], c["alpha"], d),
           "forward_ms": round(fwd_ms, 4), "backward_ms": round(bwd_ms, 4), "kernels": kern}
    for key, ops, name in (("forward", 15, "mf_fwd"), ("backward", 28, "mf_bwd")):
        if name in kern:
            ms = kern[name]["avg_ms"]
            out[key + "_pairs_per_s"] = pairs / (ms * 1e-3)
            out[key + "_valu_frac"] = round(pairs * ops / (ms * 1e-3) / VALU_LANE_OPS_PEAK, 4)
    return out


def hss_device_leg(api, ctx, A16=None, reps=3):
    """Adaptive HSS compression on the GPU end to end (Algorithm 1: sketch,
    extensions and the per-node work of every tree level in the library's
    batched kernels; the tree walk and the decisions on the host): the n = 1024
    Gaussian-kernel matrix (leaf 64, d0 = dd = 64, eps_r 1e-6) for each kind,
    and the n = 16384 nonsymmetric Cauchy matrix (leaf 256, d0 = dd = 64,
    eps_r = eps_a = 1e-8) with SJLT.  Wall time per compression (mean of
    ``reps`` after two warm-ups) and the device time of each kernel family."""
    import torch

    import workloads
    from paper_2302_01977_amd import hss as dhss

    def run(A, kind, seed, leaf, d0, dd, eps_r, eps_a, sym, alpha=4):
        for _ in range(2):  # warm-up (first pinned staging buffers, metadata kernels)
            res = dhss.compress(ctx, A, kind, seed, leaf, d0, dd, eps_r, eps_a, symmetric=sym, alpha=alpha)
            res.sketch.release()
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read("", reset=True)
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            res = dhss.compress(ctx, A, kind, seed, leaf, d0, dd, eps_r, eps_a, symmetric=sym, alpha=alpha)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            res.sketch.release()
        kern = {}
        for name in ("sjlt_gather", "sjlt_gather_t", "sjlt_meta", "sjlt_reduce", "srht", "srht_t", "srht_reduce",
                     "srht_reduce_t", "gauss_f64", "gauss_f64_t", "gauss_reduce", "hss_gemm", "hss_qr", "hss_id",
                     "hss_norm", "hss_gather", "hss_rrows"):
            ms, cnt = ctx.profile_read(name)
            if cnt:
                kern[name] = {"ms_per_compression": round(ms / reps, 4), "launches_per_compression": cnt // reps}
        ctx.profile(False)
        sk_ms = sum(v["ms_per_compression"] for k, v in kern.items() if not k.startswith("hss_"))
        node_ms = sum(v["ms_per_compression"] for k, v in kern.items() if k.startswith("hss_"))
        return {"ms": round(1e3 * sum(times) / len(times), 3), "final_d": int(res.final_d),
                "extensions": int(res.extensions), "max_rank": int(res.max_rank()), "converged": bool(res.converged),
                "sketch_kernels_ms": round(sk_ms, 4), "per_node_kernels_ms": round(node_ms, 4), "kernels": kern}

    c = workloads.cfg1()
    A1 = api.to_device_colmajor(c["A"])
    out = {"workload": "adaptive HSS on the GPU: n=1024 FP64 Gaussian kernel (leaf 64, d0=dd=64, eps 1e-6) per "
                       "kind; n=16384 FP64 Cauchy (leaf 256, d0=dd=64, eps 1e-8) with SJLT alpha=4"}
    for kind in ("sjlt", "gaussian", "srht"):
        out["kernel1024_" + kind] = run(A1, kind, c["seed"], c["leaf"], c["d0"], c["dd"], c["eps_r"], c["eps_a"],
                                        True, c["alpha"])
    if A16 is None:
        A16 = api.to_device_colmajor(workloads.cfg2()["A"])
    out["cauchy16k_sjlt"] = run(A16, "sjlt", workloads.OP_SEED[2], 256, 64, 64, 1e-8, 1e-8, False)
    # the QChem Toeplitz matrix of section 8.1 (n = 1000, spacing 0.1) with SRHT
    # (n not a power of two) and with the SJLT graph construction
    T = api.to_device_colmajor(workloads.qchem_toeplitz_dense(1000, 0.1))
    out["toeplitz1000_srht"] = run(T, "srht", 91, 64, 64, 64, 1e-6, 1e-8, True)
    out["workload"] += "; QChem Toeplitz n=1000 (spacing 0.1, leaf 64, d0=dd=64, eps 1e-6) with SRHT"
    return out


def hss_leg(api, ctx, reps=50):
    """The n = 1024 FP64 Gaussian-kernel matrix of the adaptive HSS workload
    (points in [0,1]^2 in bisection order, h = 0.5, shift 1e-2): the sketch of
    the adaptive loop's initial width d0 + dd = 128 (an apply of 64 columns and
    one extension of 64) per operator kind, in FP64.  At eps_r = 1e-6 the loop
    stops at d = 64 for all three kinds (HSS ranks <= 24, no extension), so this
    is the whole sketching work of the adaptive run.  The matrix (8 MB) stays
    in cache between back-to-back sketches, so the main figure is warm; the
    cold one is the mean of single sketches each preceded by a 1 GiB write
    that evicts the L2 caches and the 256 MB last-level cache."""
    import torch

    import workloads
    c = workloads.cfg1()
    A = api.to_device_colmajor(c["A"])
    out = {"workload": "n=1024 FP64 Gaussian kernel (cfg of the adaptive HSS run), d = 64 + 64"}
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    for kind in ("gaussian", "sjlt", "srht"):
        kw = {"alpha": c["alpha"]} if kind == "sjlt" else {}
        sk = api.Sketch(ctx, A, kind, c["d0"], c["seed"], symmetric=True, **kw)
        sk.extend(c["dd"])
        for i in range(3):
            sk.rerun(c["seed"] + i)
        torch.cuda.synchronize()
        t0.record()
        for i in range(reps):
            sk.rerun(c["seed"] + i)
        t1.record()
        torch.cuda.synchronize()
        warm = t0.elapsed_time(t1) / reps
        cold = 0.0
        for i in range(5):
            flush.zero_()
            t0.record()
            sk.rerun(c["seed"] + i)
            t1.record()
            torch.cuda.synchronize()
            cold += t0.elapsed_time(t1) / 5
        out[kind] = {"ms_per_sketch": round(warm, 4), "cold_ms_per_sketch": round(cold, 4)}
        sk.release()
    del flush
    g = out["gaussian"]["ms_per_sketch"]
    for kind in ("sjlt", "srht"):
        out[kind]["speedup_vs_fp64_gaussian"] = round(g / out[kind]["ms_per_sketch"], 2)
    return out


def precision_leg(api, ctx, reps):
    """The n = 65536 FP32 Gaussian-kernel matrix (17.2 GB; points uniform in
    [0,1]^3, h = 0.2, shift 1e-3) sketched to d = 512 in 8 blocks of 64 (one
    apply and seven extensions, each a pass over A): BF16 and bf16x3 Gaussian,
    FP32 SJLT (alpha = 8) and FP32 SRHT, against the Gaussian sketch in FP64
    arithmetic.  Errors are against the same operator applied in FP64
    arithmetic on the GPU: the FP64-arithmetic Gaussian kernel for the
    Gaussian kinds, an FP64 copy of A (34 GB) for SJLT and SRHT.  SJLT and SRHT
    are also timed with look-ahead: the same 8 blocks in 3 passes over A."""
    import torch

    import workloads
    n, blk, nblk, alpha, seed = 65536, 64, 8, 8, workloads.OP_SEED[3]
    A = workloads.gaussian_kernel_device(workloads.cfg3_points(n), 0.2, 1e-3, "float32")
    torch.cuda.synchronize()
    bytes_build = nblk * (n * n * 4 + n * blk * 4)

    def build(kind, prec, M, keep=False, plan=(1,) * nblk):
        # plan: blocks per call (the first call is the apply of one block)
        kw = {"alpha": alpha} if kind == "sjlt" else {}
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        times = []
        sk = None
        for r in range(reps + 1):
            if sk is not None:
                sk.release()
            torch.cuda.synchronize()
            t0.record()
            sk = api.Sketch(ctx, M, kind, blk, seed, prec=prec, **kw)
            for nb in plan[1:]:
                sk.extend(blk, nblocks=nb)
            t1.record()
            torch.cuda.synchronize()
            if r:  # the first build warms up
                times.append(t0.elapsed_time(t1))
        S = sk.S.clone() if keep else None
        sk.release()
        return sum(times) / len(times), S

    out = {"workload": "n=65536 FP32 Gaussian kernel (h=0.2, shift 1e-3, points in [0,1]^3), d=512 in 8 blocks "
                       "of 64 (apply + 7 extend), SJLT alpha=8", "bytes_per_build": bytes_build}
    base_ms, ref_g = build("gaussian", "native", A, keep=True)
    out["gaussian_fp64_arith"] = {"ms": round(base_ms, 3), "TFLOPs": round(2.0 * n * n * blk * nblk / (base_ms * 1e-3) / 1e12, 2)}
    for key, kind, prec in (("bf16x3", "gaussian", "bf16x3"), ("bf16", "gaussian", "bf16"),
                            ("sjlt", "sjlt", "native"), ("srht", "srht", "native")):
        ms, S = build(kind, prec, A, keep=True)
        r = {"ms": round(ms, 3), "GBps": round(bytes_build / (ms * 1e-3) / 1e9, 1),
             "speedup_vs_fp64_gaussian": round(base_ms / ms, 2)}
        if kind == "gaussian":
            r["rel_err_vs_fp64_arith"] = rel_err(S, ref_g)
            r["mfma_TFLOPs"] = round((3 if prec == "bf16x3" else 1) * 2.0 * n * n * blk * nblk / (ms * 1e-3) / 1e12, 1)
        if kind != "gaussian":
            # look-ahead: the same 8 blocks in 3 passes over A (1, 3 and 4 blocks)
            ms3, S3 = build(kind, prec, A, keep=True, plan=(1, 3, 4))
            r["lookahead_3_passes"] = {"ms": round(ms3, 3), "speedup_vs_fp64_gaussian": round(base_ms / ms3, 2),
                                       "rel_diff_vs_8_passes": rel_err(S3, S)}
            del S3
        out[key] = r
        del S
    del ref_g
    # FP64 references of the SJLT and SRHT results (same operators, A promoted)
    A64 = A.double()
    del A
    torch.cuda.empty_cache()
    # the library FP64 GEMM (rocBLAS through torch) on the same values: 8 products
    # of n x n by n x 64 (R drawn by torch: timing only); the FP64 Gaussian
    # baseline is the faster of it and the FP64-arithmetic kernel above
    Rg = torch.randn(n, blk, dtype=torch.float64, device="cuda")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.mm(A64, Rg)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(nblk):
        torch.mm(A64, Rg)
    t1.record()
    torch.cuda.synchronize()
    lib_ms = t0.elapsed_time(t1)
    del Rg
    out["fp64_gemm_library"] = {"ms": round(lib_ms, 3),
                                "TFLOPs": round(2.0 * n * n * blk * nblk / (lib_ms * 1e-3) / 1e12, 2)}
    best = min(base_ms, lib_ms)
    out["fp64_gaussian_baseline_ms"] = round(best, 3)
    for key in ("bf16x3", "bf16", "sjlt", "srht"):
        out[key]["speedup_vs_fp64_gaussian"] = round(best / out[key]["ms"], 2)
        if "lookahead_3_passes" in out[key]:
            la = out[key]["lookahead_3_passes"]
            la["speedup_vs_fp64_gaussian"] = round(best / la["ms"], 2)
    for key, kind in (("sjlt", "sjlt"), ("srht", "srht")):
        _, S64 = build(kind, "native", A64, keep=True)
        _, S32 = build(kind, "native", A64.float(), keep=True)
        out[key]["rel_err_vs_fp64_arith"] = rel_err(S32, S64)
        del S64, S32
    del A64
    torch.cuda.empty_cache()
    return out


def batch_leg(api, ctx, steps, warmup):
    """96 FP32 Gaussian-kernel matrices of uneven size (n_i log-uniform in
    [512, 8192]), SJLT alpha = 4, each grown in blocks of 64 to its own d_i in
    {64, ..., 256}: every round as one persistent launch replayed from a HIP
    graph, against one launch pair (operator block + sketch) per matrix and
    round.  The matrices are formed on the device from the seeded points."""
    import torch

    import workloads
    specs = workloads.cfg4_specs()
    seeds = [workloads.OP_SEED[4] + i for i in range(len(specs))]
    mats = []
    for sp in specs:
        X = torch.from_numpy(workloads.uniform_points(sp["n"], 2, sp["point_seed"])).cuda()
        D2 = torch.cdist(X, X) ** 2
        K = torch.exp(-D2 / (2.0 * sp["h"] ** 2)).float().contiguous()
        mats.append(K.t())  # symmetric: the transposed view is the column-major matrix
        del X, D2
    d = [sp["d"] for sp in specs]
    nbytes = sum(sp["n"] * sp["n"] * 4 * (sp["d"] // 64) + sp["n"] * sp["d"] * 4 for sp in specs)
    b = api.Batch(ctx, mats, d, 64, seeds, graph=True, autotune=True)
    nr, shape = b.info()
    ms_b = time_steps(lambda i: b.run(), steps, warmup)
    kern = kernel_times(ctx, lambda i: b.run(), ("sjlt_batch",), max(2, steps // 4))
    b.release()
    # baseline: one single-block handle per (matrix, round), rerun one by one
    hs = []
    for r in range(nr):
        for i, sp in enumerate(specs):
            if d[i] > 64 * r:
                hs.append((api.Sketch(ctx, mats[i], "sjlt", 64, seeds[i] + 7919 * r), seeds[i] + 7919 * r))
    ms_p = time_steps(lambda i: [h.rerun(s0) for h, s0 in hs], steps, warmup)
    for h, _ in hs:
        h.release()
    del mats
    torch.cuda.empty_cache()
    return {"workload": "96 FP32 Gaussian-kernel matrices, n_i in [512, 8192], d_i in {64..256}, blocks of 64, "
                        "SJLT alpha=4", "rounds": nr, "tile_shape": shape, "launches_per_matrix_path": 2 * len(hs),
            "batched_graph_ms": round(ms_b, 4), "per_matrix_ms": round(ms_p, 4),
            "batched_GBps": round(nbytes / (ms_b * 1e-3) / 1e9, 1),
            "per_matrix_GBps": round(nbytes / (ms_p * 1e-3) / 1e9, 1),
            "speedup_vs_per_matrix": round(ms_p / ms_b, 3), "kernels": kern}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sketch library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads
    from paper_2302_01977_amd import api

    single = {"mf": ("matrix_free", lambda ctx: matrix_free_leg(api, ctx, args.steps, args.warmup)),
              "batch": ("batched", lambda ctx: batch_leg(api, ctx, max(3, args.steps // 2), 2)),
              "precision": ("precision_65536", lambda ctx: precision_leg(api, ctx, 2)),
              "hss": ("hss_1024", lambda ctx: hss_leg(api, ctx)),
              "hss_device": ("hss_device", lambda ctx: hss_device_leg(api, ctx))}
    if args.leg in single:
        key, fn = single[args.leg]
        ctx = api.Context(0)
        print(json.dumps({key: fn(ctx)}))
        ctx.close()
        return

    c = workloads.cfg2()
    A_host, n, d, alpha, seed = c["A"], c["n"], c["d"], c["alpha"], c["seed"]
    A = api.to_device_colmajor(A_host)

    def step_bytes(esz):
        # read A once and write the new columns, for S and for S'
        return 2 * (n * n * esz + n * d * esz)

    ctx = api.Context(0)
    results = {}
    sketches = {}

    # measured copy bandwidth on this GPU (read + write of A's bytes)
    B = torch.empty_like(A)
    copy_ms = time_steps(lambda i: B.copy_(A), 10, 2)
    del B
    copy_gbps = 2 * A.numel() * 8 / (copy_ms * 1e-3) / 1e9
    results["copy_reference"] = {"bytes_per_launch": 2 * A.numel() * 8, "ms": round(copy_ms, 4),
                                 "GBps": round(copy_gbps, 1)}
    # measured read-only bandwidth: a column-sum reduction over A (reads A once,
    # writes n values), the closest library kernel to the sketch's access pattern
    colsum = torch.empty(n, dtype=A.dtype, device="cuda")
    read_ms = time_steps(lambda i: torch.sum(A, dim=0, out=colsum), 10, 2)
    del colsum
    read_gbps = A.numel() * 8 / (read_ms * 1e-3) / 1e9
    results["read_reference"] = {"bytes_per_launch": A.numel() * 8, "ms": round(read_ms, 4),
                                 "GBps": round(read_gbps, 1), "kernel": "torch.sum over the columns of A"}

    if args.leg in ("srht", "gaussian"):
        r, sk = stored_leg(api, ctx, A, args.leg, d, seed, alpha, "native", args.steps, args.warmup, step_bytes(8))
        if sk is not None:
            sk.release()
        print(json.dumps({args.leg: r}))
        ctx.close()
        return
    kinds = ["sjlt"] if args.leg in ("main", "fp32") else ["sjlt", "srht", "gaussian"]
    for kind in kinds:
        r, sk = stored_leg(api, ctx, A, kind, d, seed, alpha, "native", args.steps, args.warmup, step_bytes(8))
        results[kind] = r
        if sk is not None:
            sketches[kind] = sk
    if args.leg == "all":
        # the SJLT graph construction (alpha distinct positions per row) on the
        # same matrix, and the SRHT for a size that is not a power of two (the
        # leading 15000 x 15000 block of A, nu = 16384: zero-padded chunks)
        r, sk = stored_leg(api, ctx, A, "sjlt", d, seed, alpha, "native", args.steps, args.warmup, step_bytes(8),
                           construction="graph")
        results["sjlt_graph"] = r
        if sk is not None:
            sk.release()
        n2 = 15000
        r, sk = stored_leg(api, ctx, A[:n2, :n2], "srht", d, seed, alpha, "native", args.steps, args.warmup,
                           2 * (n2 * n2 * 8 + n2 * d * 8))
        r["n"], r["nu"] = n2, 16384
        results["srht_n15000"] = r
        if sk is not None:
            sk.release()

    if args.leg in ("all", "fp32"):
        # library FP64 GEMM (rocBLAS through torch) on the same shapes, for the
        # "faster of the two" FP64 Gaussian baseline; R drawn by torch (timing only)
        Rt = torch.randn(n, d, dtype=torch.float64, device="cuda")
        At_row = A.T  # row-major view of the column-major A

        def dgemm(i):
            torch.mm(A, Rt)
            torch.mm(At_row, Rt)
        lib_ms = time_steps(dgemm, max(3, args.steps // 2), 1)
        del Rt
        g64 = results.get("gaussian", {})
        base_ms = min([x for x in (g64.get("ms_per_step"), lib_ms) if x])
        for kind in ("sjlt", "srht"):
            if "ms_per_step" in results.get(kind, {}):
                results[kind]["speedup_vs_fp64_gaussian"] = round(base_ms / results[kind]["ms_per_step"], 3)
        if "ms_per_step" in g64:
            flops = 2 * 2 * n * n * d
            g64["TFLOPs"] = round(flops / (g64["ms_per_step"] * 1e-3) / 1e12, 2)
            g64["frac_fp64_peak"] = round(g64["TFLOPs"] / FP64_PEAK_TFLOPS, 4)
        results["fp64_gemm_library_ms"] = round(lib_ms, 4)
        results["fp64_gaussian_baseline_ms"] = round(base_ms, 4)

        # the same matrix rounded to FP32
        A32 = A.float()
        ref = {}
        try:
            sk = api.Sketch(ctx, A32, "gaussian", d, seed, prec="native", transpose=True)
            torch.cuda.synchronize()
            ref = {"S": sk.S.clone(), "St": sk.St.clone()}
            sk.release()
        except api.SketchError:
            pass
        fp32 = {}
        for kind, prec in (("sjlt", "native"), ("srht", "native"), ("gaussian", "bf16x3"), ("gaussian", "bf16")):
            key = kind if prec == "native" else prec
            r, sk = stored_leg(api, ctx, A32, kind, d, seed, alpha, prec, args.steps, args.warmup, step_bytes(4))
            if sk is not None:
                if kind == "gaussian" and ref:
                    r["rel_err_vs_fp64_arith"] = max(rel_err(sk.S, ref["S"]), rel_err(sk.St, ref["St"]))
                    flops = (3 if prec == "bf16x3" else 1) * 2 * 2 * n * n * d
                    r["mfma_TFLOPs"] = round(flops / (r["ms_per_step"] * 1e-3) / 1e12, 2)
                    r["frac_bf16_peak"] = round(r["mfma_TFLOPs"] / BF16_PEAK_TFLOPS, 4)
                r["speedup_vs_fp64_gaussian"] = round(base_ms / r["ms_per_step"], 3)
                sk.release()
            fp32[key] = r
        del A32, ref
        results["fp32_matrix"] = fp32
    if args.leg == "fp32":
        print(json.dumps({"fp32_matrix": results["fp32_matrix"]}))
        for sk in sketches.values():
            sk.release()
        ctx.close()
        return
    if args.leg == "all":
        results["matrix_free"] = matrix_free_leg(api, ctx, args.steps, args.warmup)
        results["batched"] = batch_leg(api, ctx, max(3, args.steps // 2), 2)
        results["precision_65536"] = precision_leg(api, ctx, 2)
        results["hss_1024"] = hss_leg(api, ctx)
        results["hss_device"] = hss_device_leg(api, ctx, A16=A)

    # the timed step: SJLT, S and S' of the FP64 matrix
    r = results["sjlt"]
    ms = r["ms_per_step"]
    value = r["GBps"]
    # roofline of the step's dominant kernel (the longer of S and S'), the
    # other one beside it; per-launch times from the library's HIP events on
    # the launch stream
    bytes_sketch = n * n * 8 + n * d * 8
    per_kernel = {}
    for name in STEP_KERNELS:
        g = r["kernels"].get(name)
        if not g:
            continue
        ach = bytes_sketch / (g["avg_ms"] * 1e-3) / 1e9
        per_kernel[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(TRAFFIC_FILES[name]),
                            "kernel": STEP_KERNELS[name], "bytes_per_launch": bytes_sketch,
                            "avg_launch_ms": round(g["avg_ms"], 5), "launches": g["launches"],
                            "frac_of_measured_copy": round(ach / copy_gbps, 4),
                            "frac_of_measured_read": round(ach / read_gbps, 4)}
    roof = None
    if per_kernel:
        dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_launch_ms"])
        roof = dict(per_kernel[dom])
        roof["dominant"] = dom
        roof["source_digest"] = sources_digest()
        roof["other"] = {k: v for k, v in per_kernel.items() if k != dom}
    for sk in sketches.values():
        sk.release()

    cpu = None
    if not args.no_cpu_baseline:
        t_cpu, cores, reps = cpu_baseline(A_host, d, alpha, seed)
        cpu = {"value": round(step_bytes(8) / t_cpu / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
               "sample": "full workload (operator + S + S', n=16384, d=256) x %d reps, %.2f s each" % (reps, t_cpu),
               "cpu_model": cpu_model()}
        cpu.update(cpu_baseline_extras(A_host, d, alpha, seed))
        if args.leg == "all":
            cpu["other_workloads"] = cpu_baseline_workloads(A_host, seed)

    out = {
        "metric": "S=AR effective GB/s & % HBM peak, SJLT/SRHT/bf16x3 vs FP64 Gaussian at 1e-6",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cauchy16k: FP64 Cauchy A_ij = 1/(x_i - y_j), n=16384, column-major, "
                               "SJLT alpha=4, d=256, S and S' per step", "n": n, "d": d, "alpha": alpha},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "pct_measured_copy": round(100 * value / copy_gbps, 2),
        "pct_measured_read": round(100 * value / read_gbps, 2),
        "roofline": roof,
        "cpu_baseline": cpu,
        "kinds": results,
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
