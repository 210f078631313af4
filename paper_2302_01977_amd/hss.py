"""Adaptive HSS compression driven from the GPU (Algorithm 1 of the paper and the
appendix "HSS Algorithm Detailed Description"), with every numerical step in the
library's kernels: the sketches S = A R, S' = A^T R and their extensions
(sketch_apply / sketch_extend), the rows of R (sketch_get_rows_device), and the
per-node work of each tree level in batched FP64 kernels (sketch_batched_*):
local sketches, the QR and the twice-applied projection of the stopping test
(section 3), the Frobenius norms, the interpolative decomposition by
column-pivoted QR and the local operators for the parent.

The host keeps the tree, the node states and the index sets; it reads back only
scalars (norms, |R_jj|, ranks) and the ID pivots.  Torch provides the device
buffers and nothing else.

Order of work.  Algorithm 1 visits the nodes bottom-up, level by level, and
restarts the sweep after the first node that fails its test (once the sketch is
extended).  Here all nodes of a level are processed together; the results are
then committed in the serial order up to and including the first failing node,
and the later nodes of that level are left as they were (they are visited
again after the extension, as in the serial sweep).  Every committed result is
computed from the same data as in the serial order, so the final width and the
states match the serial algorithm; pivots may differ where rounding does.

Readings where the paper is silent (the same as the library's other parts):
each block of R is its own JL operator; the nonsymmetric column side applies the
algorithm to A^T and a node passes only if both sides pass; the ID stops at
the first |R_kk| < max(eps_a, eps_r |R_00|) with the tolerances divided by the
node's level; a failing node appends the new orthonormal directions of every
side before the extension.
"""
import ctypes

import numpy as np
import torch

from . import _abi as abi
from .api import Sketch, _check, _stream

UNTOUCHED, PARTIAL, COMPRESSED = 0, 1, 2


def _f64(rows, cols):
    """Uninitialised FP64 device buffer, column-major rows x cols (ld = rows)."""
    return torch.empty((max(cols, 1), max(rows, 1)), dtype=torch.float64, device="cuda").T


def _ptr(t, i=0, j=0):
    """Device address of element (i, j) of a column-major FP64 tensor."""
    return t.data_ptr() + 8 * (i + j * t.stride(1))


def _ld(t):
    return max(1, t.stride(1))


class _Node:
    def __init__(self, lo, hi, level, parent=None):
        self.lo, self.hi, self.level, self.parent = lo, hi, level, parent
        self.children = None
        self.state = UNTOUCHED
        self.B12 = self.B21 = None          # device couplings (internal nodes)
        self.S = self.St = None             # local sketches (device, capacity buffers)
        self.w = 0                          # committed columns of S / St
        self.Q = self.Qt = None             # orthonormal bases (device) and their widths
        self.nq = self.nqt = 0
        self.om = self.omt = 0.0            # |Omega_00| of the first QR, per side
        self.Y = self.Yt = None             # ID coefficients (k x m) per side: U = Y^T
        self.J = self.Jt = None             # skeleton positions (host)
        self.Itil = self.Itilt = None       # skeleton rows / columns of A (host)
        self.Rl = self.Rlt = None           # local operators (device, capacity buffers)
        self.wl = 0

    @property
    def is_leaf(self):
        return self.children is None

    @property
    def m(self):
        """Rows of the node's local sketch: its size (leaf) or the children's ranks."""
        if self.is_leaf:
            return self.hi - self.lo
        return len(self.children[0].J) + len(self.children[1].J)

    @property
    def mt(self):
        if self.is_leaf:
            return self.hi - self.lo
        return len(self.children[0].Jt) + len(self.children[1].Jt)


def _tree(n, leaf):
    root = _Node(0, n, 0)
    stack = [root]
    while stack:
        t = stack.pop()
        if t.hi - t.lo > leaf:
            mid = t.lo + (t.hi - t.lo) // 2
            t.children = (_Node(t.lo, mid, t.level + 1, t), _Node(mid, t.hi, t.level + 1, t))
            stack.extend(t.children)
    return root


def _levels(root):
    by = {}
    stack = [root]
    while stack:
        t = stack.pop()
        by.setdefault(t.level, []).append(t)
        if t.children:
            stack.extend(t.children)
    return [sorted(by[lv], key=lambda t: t.lo) for lv in sorted(by, reverse=True)]


class _Batch:
    """Descriptor lists of one batched call each."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.lib = abi.load()

    def gemm(self, descs):
        if descs:
            arr = (abi.SkGemmDesc * len(descs))(*descs)
            _check(self.lib.sketch_batched_gemm(self.ctx.ptr, arr, len(descs), _stream(None)))

    def qr(self, descs):
        if descs:
            arr = (abi.SkQrDesc * len(descs))(*descs)
            _check(self.lib.sketch_batched_qr(self.ctx.ptr, arr, len(descs), _stream(None)))

    def ident(self, descs):
        if descs:
            arr = (abi.SkIdDesc * len(descs))(*descs)
            _check(self.lib.sketch_batched_id(self.ctx.ptr, arr, len(descs), _stream(None)))

    def norm(self, descs):
        if descs:
            arr = (abi.SkNormDesc * len(descs))(*descs)
            _check(self.lib.sketch_batched_norm(self.ctx.ptr, arr, len(descs), _stream(None)))

    def gather(self, descs):
        if descs:
            arr = (abi.SkGatherDesc * len(descs))(*descs)
            _check(self.lib.sketch_batched_gather(self.ctx.ptr, arr, len(descs), _stream(None)))


def _gemm(C, A, B, m, n, k, alpha=1.0, beta=0.0, ta=False, tb=False):
    """Descriptor of C = beta C + alpha op(A) op(B); A, B, C are (tensor, i, j)."""
    (Ct, ci, cj), (At, ai, aj), (Bt, bi, bj) = C, A, B
    return abi.SkGemmDesc(m=m, n=n, k=k, transA=int(ta), transB=int(tb), alpha=alpha, beta=beta,
                          A=_ptr(At, ai, aj), lda=_ld(At), B=_ptr(Bt, bi, bj), ldb=_ld(Bt),
                          C=_ptr(Ct, ci, cj), ldc=_ld(Ct))


def _copy(dst, src, m, n, rows=None, trans=False):
    """Descriptor of dst(i, j) = src(rows[i] or i, j) (or the transpose)."""
    (Dt, di, dj), (St, si, sj) = dst, src
    return abi.SkGatherDesc(m=m, n=n, trans=int(trans), src=St.data_ptr(), lds=_ld(St),
                            rows=rows.data_ptr() if rows is not None else None, cols=None,
                            row0=si, col0=sj, dst=_ptr(Dt, di, dj), ldd=_ld(Dt))


class HSSResult:
    """Outcome of ``compress``: the tree (nodes with device generators), the
    final width d of Algorithm 1, and the counts."""

    def __init__(self, root, levels, d, dd, n, symmetric, converged, extensions):
        self.root, self.levels, self.d, self.dd = root, levels, d, dd
        self.n, self.symmetric, self.converged, self.extensions = n, symmetric, converged, extensions

    @property
    def final_d(self):
        return self.d

    def max_rank(self):
        r = [len(t.J) for lv in self.levels for t in lv if t.J is not None]
        r += [len(t.Jt) for lv in self.levels for t in lv if t.Jt is not None]
        return max(r) if r else 0

    def generators(self):
        """Host copies of the generators of every non-root node: dict keyed by
        (lo, hi) with U = Y^T, V = Yt^T, J, Jt, and B12, B21 for internal nodes."""
        out = {}
        for lv in self.levels:
            for t in lv:
                g = {}
                if t.Y is not None:
                    g["U"] = t.Y.cpu().numpy().T.copy()
                    g["V"] = g["U"] if self.symmetric else t.Yt.cpu().numpy().T.copy()
                    g["J"], g["Jt"] = np.asarray(t.J), np.asarray(t.Jt)
                if t.B12 is not None:
                    g["B12"] = t.B12.cpu().numpy().copy()
                    g["B21"] = t.B21.cpu().numpy().copy()
                out[(t.lo, t.hi)] = g
        return out


class _Compressor:
    def __init__(self, ctx, A, kind, seed, leaf, d0, dd, eps_r, eps_a, symmetric, alpha, d_max):
        self.ctx, self.A, self.kind, self.seed = ctx, A, kind, seed
        self.leaf, self.d0, self.dd = leaf, d0, dd
        self.eps_r, self.eps_a, self.sym = eps_r, eps_a, symmetric
        self.n = A.shape[0]
        self.d_max = self.n if d_max is None else d_max
        self.batch = _Batch(ctx)
        self.lib = abi.load()
        self._keep = []     # temporaries of the launches in flight (device index arrays, work buffers)
        self._pend = []     # copies of grown buffers not yet issued
        # Algorithm 1: R <- JL-Operator(d0 + dd, n), here a block of d0 columns
        # and one of dd; S <- A R (and S' <- A^T R)
        self.sk = Sketch(ctx, A, kind, d0, seed, alpha=alpha, transpose=not symmetric)
        self.sk.extend(dd)
        self.d = d0
        self.R = None
        self._rows_of_R()

    # ------------------------------------------------------------ storage
    @property
    def S(self):
        return self.sk.S

    @property
    def St(self):
        return self.sk.S if self.sym else self.sk.St

    def _rows_of_R(self):
        """All rows of R, columns [0, d + dd), on the device."""
        w = self.d + self.dd
        self.R = _f64(self.n, w)
        _check(self.lib.sketch_get_rows_device(self.sk.h, 0, self.n, 0, w, ctypes.c_void_p(self.R.data_ptr()),
                                               self.n, _stream(None)))

    def _grow(self, buf, rows, width, keep):
        """A buffer of at least ``width`` columns holding the first ``keep``
        columns of ``buf`` (capacity doubles); the copy joins the pending ones,
        which ``_flush`` issues in one batched launch."""
        if buf is not None and buf.shape[1] >= width:
            return buf
        cap = max(width, 2 * (buf.shape[1] if buf is not None else 0))
        nb = _f64(rows, cap)
        if buf is not None and keep and rows:
            self._pend.append(_copy((nb, 0, 0), (buf, 0, 0), rows, keep))
            self._keep.append(buf)
        return nb

    def _flush(self):
        self.batch.gather(self._pend)
        self._pend = []

    def _stage(self, reqs):
        """Index lists of one phase in one upload: ``reqs`` holds (descriptor,
        field, host array); the arrays go through one pinned buffer and one
        asynchronous copy, and each descriptor field receives its device
        pointer."""
        if not reqs:
            return
        tot = sum(len(a) for _, _, a in reqs)
        host = torch.empty(max(tot, 1), dtype=torch.int64, pin_memory=True)
        hv = host.numpy()
        offs, o = [], 0
        for _, _, a in reqs:
            hv[o:o + len(a)] = a
            offs.append(o)
            o += len(a)
        dev = host.to("cuda", non_blocking=True)
        self._keep += [host, dev]
        base = dev.data_ptr()
        for (desc, field, _), off in zip(reqs, offs):
            setattr(desc, field, base + 8 * off)

    # ------------------------------------------------------------- sweep
    def run(self):
        root = _tree(self.n, self.leaf)
        levels = _levels(root)
        extensions = 0
        while root.state != COMPRESSED and self.d < self.d_max:
            failed = False
            for lv in levels:
                if lv[0] is root:
                    self._couplings([root])
                    root.state = COMPRESSED
                    break
                if self._level(lv):
                    failed = True
                    break
            if failed:
                # extension: R <- [R, Rbar], S <- [S, A Rbar]; the sweep restarts
                self.sk.extend(self.dd)
                self.d += self.dd
                extensions += 1
                self._rows_of_R()
        torch.cuda.synchronize()
        return HSSResult(root, levels, self.d, self.dd, self.n, self.sym, root.state == COMPRESSED,
                         extensions)

    def _couplings(self, nodes):
        """B12 = A(I~_1, I~'_2) and B21 = A(I~_2, I~'_1) of the untouched internal nodes."""
        gat, reqs = [], []
        for t in nodes:
            if t.state == UNTOUCHED and not t.is_leaf:
                c1, c2 = t.children
                bl = []
                for (ra, ca) in ((c1.Itil, c2.Itilt), (c2.Itil, c1.Itilt)):
                    B = _f64(len(ra), len(ca))
                    bl.append(B)
                    g = abi.SkGatherDesc(m=len(ra), n=len(ca), trans=0, src=self.A.data_ptr(), lds=_ld(self.A),
                                         rows=None, cols=None, row0=0, col0=0, dst=B.data_ptr(), ldd=_ld(B))
                    reqs += [(g, "rows", ra), (g, "cols", ca)]
                    gat.append(g)
                t.B12, t.B21 = bl
        self._stage(reqs)
        self.batch.gather(gat)

    def _sides(self):
        return ("S",) if self.sym else ("S", "St")

    def _level(self, nodes):
        """Visit every node of one level; commit in order up to the first node
        that fails.  Returns True when a node failed (the sketch must grow)."""
        d, dd = self.d, self.dd
        i1 = d + dd
        self._keep = []
        self._couplings(nodes)
        plan = [{"t": t, "i0": 0 if t.state == UNTOUCHED else d} for t in nodes]
        self._local_sketches(plan, i1)
        tests = [p for p in plan if p["t"].state != COMPRESSED]
        for p in tests:
            lv = p["t"].level
            p["eps"] = (self.eps_r / lv, self.eps_a / lv)
        self._stopping_test(tests, d, dd)
        fail = None
        for i, p in enumerate(plan):
            if p["t"].state != COMPRESSED and not all(p["pass"].values()):
                fail = i
                break
        commit = plan if fail is None else plan[:fail]
        self._interpolate([p for p in commit if p["t"].state != COMPRESSED], i1)
        for p in commit:
            t = p["t"]
            t.S, t.w = p["S"], i1
            if not self.sym:
                t.St = p["St"]
        if fail is not None:
            self._keep_failing(plan[fail], i1)
        self._local_operators(commit, i1)
        return fail is not None

    def _local_sketches(self, plan, i1):
        """Columns [i0, i1) of every node's local sketch: the rows of S (leaf) or
        the skeleton rows of the children's local sketches, minus the diagonal
        block times R (leaf) or the couplings times the children's local
        operators (internal node)."""
        gat, gem, reqs = [], [], []
        for p in plan:
            t, i0 = p["t"], p["i0"]
            w = i1 - i0
            for side in self._sides():
                m = t.m if side == "S" else t.mt
                buf = self._grow(getattr(t, side) if t.state != UNTOUCHED else None, m, i1,
                                 t.w if t.state != UNTOUCHED else 0)
                p[side] = buf
                if not m:
                    continue
                if t.is_leaf:
                    src = self.S if side == "S" else self.St
                    gat.append(_copy((buf, 0, i0), (src, t.lo, i0), m, w))
                    gem.append(_gemm((buf, 0, i0), (self.A, t.lo, t.lo), (self.R, t.lo, i0), m, w, m,
                                     alpha=-1.0, beta=1.0, ta=(side == "St")))
                    continue
                c1, c2 = t.children
                if side == "S":
                    # [c1.S(J1) - B12 R'_2 ; c2.S(J2) - B21 R'_1]
                    parts = ((c1.J, c1.S, t.B12, c2.Rlt, len(c2.Jt), False),
                             (c2.J, c2.S, t.B21, c1.Rlt, len(c1.Jt), False))
                else:
                    # [c1.S'(J'1) - B21^T R_2 ; c2.S'(J'2) - B12^T R_1]
                    parts = ((c1.Jt, c1.St, t.B21, c2.Rl, len(c2.J), True),
                             (c2.Jt, c2.St, t.B12, c1.Rl, len(c1.J), True))
                r0 = 0
                for (J, cS, B, Rl, kk, tb) in parts:
                    k = len(J)
                    if k:
                        gd = abi.SkGatherDesc(m=k, n=w, trans=0, src=cS.data_ptr(), lds=_ld(cS), rows=None,
                                              cols=None, row0=0, col0=i0, dst=_ptr(buf, r0, i0), ldd=_ld(buf))
                        reqs.append((gd, "rows", J))
                        gat.append(gd)
                        if kk:
                            gem.append(_gemm((buf, r0, i0), (B, 0, 0), (Rl, 0, i0), k, w, kk,
                                             alpha=-1.0, beta=1.0, ta=tb))
                    r0 += k
        self._flush()  # old columns of grown buffers (disjoint from the new ones written here)
        self._stage(reqs)
        self.batch.gather(gat)
        self.batch.gemm(gem)

    def _stopping_test(self, tests, d, dd):
        """Section 3's test for every side of every node not yet compressed:
        QR of the first d columns (untouched nodes), projection of the next dd
        columns applied twice, Frobenius test, and for the sides that fail it the
        QR of the projected block and the test on its smallest |R_jj|."""
        sides = [(p, side) for p in tests for side in self._sides()]
        nsd = len(sides)
        # per side: ||S^||_F, ||S~||_F, |R_00| of the first QR
        scal = torch.zeros((max(1, 3 * nsd), 1), dtype=torch.float64, device="cuda")
        self._keep.append(scal)
        gat, qrs, r00 = [], [], []
        for q, (p, side) in enumerate(sides):
            t = p["t"]
            m = t.m if side == "S" else t.mt
            if t.state == UNTOUCHED:
                r = min(m, d)
                Q = self._grow(None, m, r + dd, 0)
                p[side + "_Q"], p[side + "_nq"] = Q, r
                if m and r:
                    W = _f64(m, d)
                    rd = torch.empty(r, dtype=torch.float64, device="cuda")
                    self._keep += [W, rd]
                    gat.append(_copy((W, 0, 0), (p[side], 0, 0), m, d))
                    qrs.append(abi.SkQrDesc(m=m, n=d, A=W.data_ptr(), lda=_ld(W), rdiag=rd.data_ptr(),
                                            Q=Q.data_ptr(), ldq=_ld(Q)))
                    r00.append(_copy((scal, 3 * q + 2, 0), (rd.view(r, 1), 0, 0), 1, 1))
            else:
                nq = t.nq if side == "S" else t.nqt
                p[side + "_Q"] = self._grow(t.Q if side == "S" else t.Qt, m, nq + dd, nq)
                p[side + "_nq"] = nq
        self._flush()
        self.batch.gather(gat)
        self.batch.qr(qrs)
        self.batch.gather(r00)
        gem1, gem2, gem3, gem4, cps, nrm = [], [], [], [], [], []
        for q, (p, side) in enumerate(sides):
            t = p["t"]
            m = t.m if side == "S" else t.mt
            Q, nq, Sl = p[side + "_Q"], p[side + "_nq"], p[side]
            Sh = _f64(m, dd)
            p[side + "_hat"] = Sh
            if not m:
                continue
            cps.append(_copy((Sh, 0, 0), (Sl, 0, d), m, dd))
            if nq:
                Wt = _f64(nq, dd)
                self._keep.append(Wt)
                gem1.append(_gemm((Wt, 0, 0), (Q, 0, 0), (Sl, 0, d), nq, dd, m, ta=True))
                gem2.append(_gemm((Sh, 0, 0), (Q, 0, 0), (Wt, 0, 0), m, dd, nq, alpha=-1.0, beta=1.0))
                gem3.append(_gemm((Wt, 0, 0), (Q, 0, 0), (Sh, 0, 0), nq, dd, m, ta=True))
                gem4.append(_gemm((Sh, 0, 0), (Q, 0, 0), (Wt, 0, 0), m, dd, nq, alpha=-1.0, beta=1.0))
            nrm.append(abi.SkNormDesc(m=m, n=dd, A=_ptr(Sh), lda=_ld(Sh), out=scal.data_ptr() + 8 * (3 * q)))
            nrm.append(abi.SkNormDesc(m=m, n=dd, A=_ptr(Sl, 0, d), lda=_ld(Sl), out=scal.data_ptr() + 8 * (3 * q + 1)))
        self.batch.gather(cps)
        for g in (gem1, gem2, gem3, gem4):
            self.batch.gemm(g)
        self.batch.norm(nrm)
        vals = scal.cpu().numpy()[:, 0]
        for p in tests:
            p["pass"] = {}
        hat = []
        for q, (p, side) in enumerate(sides):
            t = p["t"]
            eps_r_t, eps_a_t = p["eps"]
            nh, ns = float(vals[3 * q]), float(vals[3 * q + 1])
            if t.state == UNTOUCHED:
                p[side + "_om"] = float(vals[3 * q + 2])
            else:
                p[side + "_om"] = t.om if side == "S" else t.omt
            if nh < eps_a_t or nh < eps_r_t * ns:
                p["pass"][side] = True
            else:
                hat.append((p, side))
        mins = self._qr_hats(hat)
        for (p, side), mn in zip(hat, mins):
            eps_r_t, eps_a_t = p["eps"]
            p["pass"][side] = mn < eps_a_t or mn < eps_r_t * p[side + "_om"]

    def _qr_hats(self, hat):
        """QR of S^ of each (node, side) into the columns after the side's
        current basis; returns min |R_jj| per entry and advances the bases."""
        if not hat:
            return []
        dd = self.dd
        gat, qrs, offs = [], [], []
        total = sum(min(p["t"].m if s == "S" else p["t"].mt, dd) for p, s in hat)
        rd = torch.zeros(max(1, total), dtype=torch.float64, device="cuda")
        self._keep.append(rd)  # |R_jj| of every QR, one after the other
        o = 0
        for (p, side) in hat:
            t = p["t"]
            m = t.m if side == "S" else t.mt
            r = min(m, dd)
            offs.append((o, r))
            if r:
                W = _f64(m, dd)
                self._keep.append(W)
                Q, nq = p[side + "_Q"], p[side + "_nq"]
                gat.append(_copy((W, 0, 0), (p[side + "_hat"], 0, 0), m, dd))
                qrs.append(abi.SkQrDesc(m=m, n=dd, A=W.data_ptr(), lda=_ld(W), rdiag=rd.data_ptr() + 8 * o,
                                        Q=_ptr(Q, 0, nq), ldq=_ld(Q)))
            p[side + "_nq"] += r
            p[side + "_hatqr"] = True
            o += r
        self.batch.gather(gat)
        self.batch.qr(qrs)
        v = rd.cpu().numpy()
        return [float(v[a:a + r].min()) if r else 0.0 for (a, r) in offs]

    def _interpolate(self, newly, i1):
        """Interpolative decompositions S_tau^T ~ S_tau^T(:, J) Y of the nodes that
        pass (per side), their skeleton positions J and the U = Y^T factors."""
        if not newly:
            return
        sides = [(p, side) for p in newly for side in self._sides()]
        qtot = sum((p["t"].m if s == "S" else p["t"].mt) for p, s in sides)
        # ranks, then the permutations: one read-back
        iw = torch.zeros(len(sides) + max(1, qtot), dtype=torch.int32, device="cuda")
        rank, perm = iw[:len(sides)], iw[len(sides):]
        gat, ids, offs = [], [], []
        o = 0
        for q, (p, side) in enumerate(sides):
            t = p["t"]
            eps_r_t, eps_a_t = p["eps"]
            m = t.m if side == "S" else t.mt
            Y = _f64(min(i1, m), m)
            offs.append((o, m, Y))
            if m:
                M = _f64(i1, m)
                self._keep.append(M)
                gat.append(_copy((M, 0, 0), (p[side], 0, 0), i1, m, trans=True))
                ids.append(abi.SkIdDesc(p=i1, q=m, M=M.data_ptr(), ldm=_ld(M), eps_r=eps_r_t, eps_a=eps_a_t,
                                        perm=perm.data_ptr() + 4 * o, rank=rank.data_ptr() + 4 * q,
                                        Y=Y.data_ptr(), ldy=_ld(Y)))
            o += m
        self.batch.gather(gat)
        self.batch.ident(ids)
        iv = iw.cpu().numpy()
        rv, pv = iv[:len(sides)], iv[len(sides):]
        for q, (p, side) in enumerate(sides):
            t = p["t"]
            a, m, Y = offs[q]
            k = int(rv[q])
            J = pv[a:a + k].astype(np.int64)
            if side == "S":
                t.J, t.Y = J, Y[:k, :]
            else:
                t.Jt, t.Yt = J, Y[:k, :]
        for p in newly:
            t = p["t"]
            if self.sym:
                t.Jt, t.Yt = t.J, t.Y
            t.Q = t.Qt = None
            t.state = COMPRESSED
            t._fresh = True

    def _keep_failing(self, p, i1):
        """The failing node keeps its local sketch and appends to every side's
        basis the new orthonormal directions (sides that passed the Frobenius
        test get the QR of their S^ now), so that the basis spans the first
        d + dd columns after the extension."""
        t = p["t"]
        self._qr_hats([(p, side) for side in self._sides() if not p.get(side + "_hatqr")])
        t.S, t.w = p["S"], i1
        t.Q, t.nq, t.om = p["S_Q"], p["S_nq"], p["S_om"]
        if not self.sym:
            t.St, t.Qt, t.nqt, t.omt = p["St"], p["St_Q"], p["St_nq"], p["St_om"]
        t.state = PARTIAL

    def _local_operators(self, commit, i1):
        """R_tau = U_tau^T R(I_tau, :) (leaf) or U_tau^T [R_nu1; R_nu2] (internal
        node), on all columns for the nodes compressed in this visit and on the
        new columns for the nodes compressed before; skeleton rows I~ for the
        parent."""
        gem = []
        for p in commit:
            t = p["t"]
            fresh = getattr(t, "_fresh", False)
            t._fresh = False
            j0 = 0 if fresh else p["i0"]
            w = i1 - j0
            t.Rl = self._grow(None if fresh else t.Rl, len(t.J), i1, 0 if fresh else t.wl)
            if self.sym:
                t.Rlt = t.Rl
            else:
                t.Rlt = self._grow(None if fresh else t.Rlt, len(t.Jt), i1, 0 if fresh else t.wl)
            pairs = [(t.Y, t.Rl, "Rl", "J")] + ([] if self.sym else [(t.Yt, t.Rlt, "Rlt", "Jt")])
            for (Y, Rl, rname, jname) in pairs:
                k = Y.shape[0]
                if not k:
                    continue
                if t.is_leaf:
                    gem.append(_gemm((Rl, 0, j0), (Y, 0, 0), (self.R, t.lo, j0), k, w, t.hi - t.lo))
                    continue
                c1, c2 = t.children
                k1, k2 = len(getattr(c1, jname)), len(getattr(c2, jname))
                if k1:
                    gem.append(_gemm((Rl, 0, j0), (Y, 0, 0), (getattr(c1, rname), 0, j0), k, w, k1))
                if k2:
                    gem.append(_gemm((Rl, 0, j0), (Y, 0, k1), (getattr(c2, rname), 0, j0), k, w, k2,
                                     beta=1.0 if k1 else 0.0))
            t.wl = i1
            if t.is_leaf:
                idx = np.arange(t.lo, t.hi)
                t.Itil, t.Itilt = idx[t.J], idx[t.Jt]
            else:
                c1, c2 = t.children
                t.Itil = np.concatenate([c1.Itil, c2.Itil])[t.J]
                t.Itilt = np.concatenate([c1.Itilt, c2.Itilt])[t.Jt]
        self._flush()
        # two products into one Rl column block (k1 then k2 with beta = 1) must
        # not run concurrently: split them over two launches
        first, second = [], []
        seen = set()
        for g in gem:
            (second if g.C in seen else first).append(g)
            seen.add(g.C)
        self.batch.gemm(first)
        self.batch.gemm(second)


def compress(ctx, A, kind, seed, leaf, d0, dd, eps_r, eps_a, symmetric=False, alpha=4, d_max=None):
    """Adaptive HSS compression of the dense FP64 n x n device matrix ``A``
    (column-major) with a ``kind`` sketching operator drawn from ``seed``:
    Algorithm 1 with initial width d0 + dd, blocks of dd, relative and absolute
    tolerances eps_r, eps_a, leaves of at most ``leaf`` indices (index
    halving).  Returns an ``HSSResult``."""
    if A.dtype != torch.float64 or not A.is_cuda or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square FP64 device matrix")
    c = _Compressor(ctx, A, kind, seed, leaf, d0, dd, eps_r, eps_a, symmetric, alpha, d_max)
    res = c.run()
    res.sketch = c.sk
    return res
