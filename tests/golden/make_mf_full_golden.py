"""Writes mf_n32768_dh.txt: dL/dh of the full matrix-free workload (N = 32768
points uniform in [0,1]^3, h = 0.3 as an FP32 value, SJLT alpha = 4, d = 256,
L = sum(W o S) with the seeded W), from the FP64 oracle's closed-form gradient
over all N^2 pairs.  Calls only ``oracle`` and the input generators in
``workloads``; run from the repository root:

    python tests/golden/make_mf_full_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import operators as ops  # noqa: E402
from oracle import sketch as osk  # noqa: E402


def main():
    c = workloads.cfg5()
    X = c["X"].astype(np.float64)
    W = np.asarray(c["W"], dtype=np.float64)
    h = float(np.float32(c["h"]))
    R = ops.sjlt_block(c["N"], c["d"], c["alpha"], 0, c["seed"])
    t = time.time()
    _, dh = osk.kernel_grad(X, h, R, W, block_rows=512)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mf_n32768_dh.txt")
    with open(out, "w") as f:
        f.write("# dL/dh of L = sum(W o (K(X, h) R)) for the N = 32768 matrix-free workload\n")
        f.write("# (points uniform in [0,1]^3 from data seed %d, h = float32(0.3), SJLT alpha = 4,\n" % 1005)
        f.write("# d = 256, operator seed %d, W ~ N(0, 1) from data seed %d).\n" % (c["seed"], 1006))
        f.write("# FP64 closed form dL/dh = sum_ij G_ij K_ij |x_i - x_j|^2 / h^3, G = W R^T,\n")
        f.write("# written by tests/golden/make_mf_full_golden.py from the oracle alone.\n")
        f.write("%.17e\n" % dh)
    print("dh = %.17e  (%.0f s)" % (dh, time.time() - t))


if __name__ == "__main__":
    main()
