"""Reference adaptive HSS compression (Algorithm 1 of the paper), FP64, on the CPU.

Test infrastructure only (see ``oracle/__init__.py``).

The HSS format is the one of section 2.2: a binary cluster tree of contiguous
index ranges (the same tree for rows and columns); leaves keep D_tau = A(I, I);
every non-root node keeps row and column bases U_tau, V_tau which are nested
(U^big_tau = diag(U^big_nu1, U^big_nu2) U_tau, equation "nestedUV"); every
internal node keeps B_{nu1,nu2} = A(I~_nu1, I~'_nu2) and B_{nu2,nu1}.

Compression follows Algorithm 1 ("HSSCompressAdaptive", appendix "HSS Algorithm
Detailed Description") with the walk-through of the same appendix:
local sketches with the diagonal block (leaf) or the sibling coupling (internal
node) subtracted, a QR of the first d columns, the block Gram-Schmidt projection
of the last dd columns applied twice (remark after the stopping criteria of
section 3), the Frobenius tests of equation "stopping_criteria-1" with the
tolerances divided by the node level, the rank-deficiency test on the new R
factor, an interpolative decomposition (section 2.3 and its remark on row
bases), and an extension of R by a fresh block of dd columns when a node fails,
after which the sweep restarts.

Readings taken where the paper is silent (listed with the design notes):
  * nonsymmetric column side: Algorithm 1 is applied to A^T (B_{nu2,nu1}^T and
    B_{nu1,nu2}^T, row and column local operators swapped); a node passes only
    if both sides pass;
  * when a node fails, every side whose new columns were not yet appended to its
    orthonormal basis gets them appended too, so that Q always spans the first d
    columns of the local sketch;
  * a node that becomes compressed in a visit forms its local operator
    R_tau = U_tau^T R(...) on all columns; an already compressed node revisited
    after an extension forms only the new columns;
  * ID: column-pivoted Householder QR with exact column norms, first index of
    maximal norm, truncated at the first k with |R_kk| < max(eps_a, eps_r |R_00|).
"""
import numpy as np

UNTOUCHED = 0
PARTIALLY_COMPRESSED = 1
COMPRESSED = 2


# ----------------------------------------------------------------------- tree
class Node:
    def __init__(self, lo, hi, level, parent=None):
        self.lo, self.hi, self.level, self.parent = lo, hi, level, parent
        self.children = None
        self.state = UNTOUCHED
        self.D = self.B12 = self.B21 = None
        # local sketches (row side S, column side St) and their orthonormal bases
        self.S = self.St = None
        self.Q = self.Qt = None
        self.om11 = self.omt11 = 0.0
        # interpolative bases, skeleton positions (local) and skeleton rows (global)
        self.U = self.V = None
        self.J = self.Jt = None
        self.Itil = self.Itilt = None
        # local operators R_tau = U^T R(...), R'_tau = V^T R(...)
        self.Rl = self.Rlt = None

    @property
    def is_leaf(self):
        return self.children is None

    @property
    def idx(self):
        return np.arange(self.lo, self.hi)


def build_tree(n, leaf):
    """Cluster tree by index halving of [0, n) until a node holds <= leaf indices.
    Section 2.2: nodes are contiguous index sets, children partition the parent."""
    root = Node(0, n, 0)
    stack = [root]
    while stack:
        t = stack.pop()
        if t.hi - t.lo > leaf:
            mid = t.lo + (t.hi - t.lo) // 2
            t.children = (Node(t.lo, mid, t.level + 1, t), Node(mid, t.hi, t.level + 1, t))
            stack.extend(t.children)
    return root


def topological(root):
    """Bottom-up level-by-level order (section 2.2): deepest level first,
    left to right within a level; the root comes last."""
    levels = {}
    stack = [root]
    while stack:
        t = stack.pop()
        levels.setdefault(t.level, []).append(t)
        if t.children:
            stack.extend(t.children)
    order = []
    for lev in sorted(levels, reverse=True):
        order += sorted(levels[lev], key=lambda t: t.lo)
    return order


# ------------------------------------------------------------------ ID via CPQR
def interpolative(M, eps_r, eps_a):
    """Column interpolative decomposition M ~ M(:, J) Y (helper table of the
    appendix: ID(S, eps_r, eps_a)).

    Column-pivoted Householder QR with exact recomputation of the remaining
    column norms at every step; the pivot is the first column of maximal norm;
    the factorisation stops at the first k with |R_kk| < max(eps_a, eps_r |R_00|).
    Returns (J, Y) with J the k pivot columns and Y = [I, R11^{-1} R12] P^T.
    """
    M = np.array(M, dtype=np.float64, copy=True)
    m, n = M.shape
    perm = np.arange(n)
    rank = 0
    r00 = None
    for k in range(min(m, n)):
        norms = np.linalg.norm(M[k:, k:], axis=0)
        p = int(np.argmax(norms))          # argmax returns the first maximal index
        nk = float(norms[p])
        if r00 is None:
            r00 = nk
        if nk == 0.0 or nk < max(eps_a, eps_r * r00):
            break
        p += k
        if p != k:
            M[:, [k, p]] = M[:, [p, k]]
            perm[[k, p]] = perm[[p, k]]
        x = M[k:, k].copy()
        alpha = -np.copysign(np.linalg.norm(x), x[0] if x[0] != 0 else 1.0)
        v = x.copy()
        v[0] -= alpha
        vn = np.linalg.norm(v)
        if vn > 0:
            v /= vn
            M[k:, k:] -= 2.0 * np.outer(v, v @ M[k:, k:])
        M[k + 1:, k] = 0.0
        rank = k + 1
    else:
        rank = min(m, n)
    R11 = np.triu(M[:rank, :rank])
    R12 = M[:rank, rank:]
    T = np.linalg.solve(R11, R12) if rank else np.zeros((0, n - rank))
    Y = np.zeros((rank, n))
    Y[:, perm[:rank]] = np.eye(rank)
    Y[:, perm[rank:]] = T
    return perm[:rank].copy(), Y


def _qr(S):
    """Householder QR (library routine), reduced: S = Q Omega."""
    if S.shape[1] == 0 or S.shape[0] == 0:
        return np.zeros((S.shape[0], 0)), np.zeros((0, S.shape[1]))
    return np.linalg.qr(S, mode="reduced")


# ------------------------------------------------------------------- sketchers
class OracleSketcher:
    """Explicit-R sketcher: R = [R_0 | R_1 | ...] from ``oracle.operators`` and
    S = A R, S' = A^T R by dense products.  Any object with the same two methods
    (add_block, R_rows) can drive ``compress``."""

    def __init__(self, A, kind, seed, alpha=4, symmetric=False):
        from . import operators as ops
        self._ops = ops
        self.A = np.asarray(A, dtype=np.float64)
        self.kind, self.seed, self.alpha = kind, seed, alpha
        self.symmetric = symmetric
        self.n = self.A.shape[1]
        self.widths = []
        self.R = np.zeros((self.n, 0))

    def add_block(self, w):
        b = len(self.widths)
        c0 = int(sum(self.widths))
        Rb = self._ops.operator_block(self.kind, self.n, w, b, c0, self.seed, self.alpha)
        self.widths.append(w)
        self.R = np.concatenate([self.R, Rb], axis=1)
        S = self.A @ Rb
        St = None if self.symmetric else self.A.T @ Rb
        return S, St

    def R_rows(self, rows, c0, c1):
        return self.R[rows, c0:c1]


# ----------------------------------------------------------------- compression
class HSSResult:
    def __init__(self, root, order, d, dd, n, symmetric, converged, extensions):
        self.root, self.order, self.d, self.dd = root, order, d, dd
        self.n, self.symmetric, self.converged = n, symmetric, converged
        self.extensions = extensions

    @property
    def final_d(self):
        """d of Algorithm 1 at exit (the sketch holds d + dd columns)."""
        return self.d

    def ranks(self):
        return [len(t.J) for t in self.order if t.J is not None]

    def max_rank(self):
        r = [len(t.J) for t in self.order if t.J is not None]
        r += [len(t.Jt) for t in self.order if t.Jt is not None]
        return max(r) if r else 0


def compress(A, leaf, sketcher, d0, dd, eps_r, eps_a, symmetric=False, d_max=None):
    """Adaptive HSS compression of the dense n x n matrix A (Algorithm 1).

    A supplies D_tau and B blocks (partially matrix-free: O(n r) entries are read);
    ``sketcher`` supplies the sketch columns and the entries R(I, cols).
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    d_max = n if d_max is None else d_max
    root = build_tree(n, leaf)
    order = topological(root)

    # Algorithm 1: R <- JL-Operator(d + dd, n); S <- A R, built here as a block of
    # d0 columns followed by a block of dd columns.
    S_parts, St_parts = [], []
    for w in (d0, dd):
        s, st = sketcher.add_block(w)
        S_parts.append(s)
        St_parts.append(st)
    S = np.concatenate(S_parts, axis=1)
    St = S if symmetric else np.concatenate(St_parts, axis=1)
    d = d0
    extensions = 0

    def Rcols(rows, c0, c1):
        return np.asarray(sketcher.R_rows(rows, c0, c1), dtype=np.float64)

    while root.state != COMPRESSED and d < d_max:
        for t in order:
            if t.state == UNTOUCHED:
                if t.is_leaf:
                    t.D = A[t.lo:t.hi, t.lo:t.hi].copy()
                else:
                    c1, c2 = t.children
                    t.B12 = A[np.ix_(c1.Itil, c2.Itilt)]
                    t.B21 = A[np.ix_(c2.Itil, c1.Itilt)]
                i0, i1 = 0, d + dd
            else:
                i0, i1 = d, d + dd
            if t is root:
                t.state = COMPRESSED
                break

            # local sketches on columns i0:i1
            if t.is_leaf:
                Ri = Rcols(t.idx, i0, i1)
                s_new = S[t.lo:t.hi, i0:i1] - t.D @ Ri
                st_new = None if symmetric else St[t.lo:t.hi, i0:i1] - t.D.T @ Ri
            else:
                c1, c2 = t.children
                s_new = np.vstack([c1.S[c1.J, i0:i1] - t.B12 @ c2.Rlt[:, i0:i1],
                                   c2.S[c2.J, i0:i1] - t.B21 @ c1.Rlt[:, i0:i1]])
                st_new = None if symmetric else np.vstack(
                    [c1.St[c1.Jt, i0:i1] - t.B21.T @ c2.Rl[:, i0:i1],
                     c2.St[c2.Jt, i0:i1] - t.B12.T @ c1.Rl[:, i0:i1]])
            t.S = s_new if i0 == 0 else np.hstack([t.S, s_new])
            if not symmetric:
                t.St = st_new if i0 == 0 else np.hstack([t.St, st_new])

            newly = False
            if t.state != COMPRESSED:
                eps_r_t = eps_r / t.level
                eps_a_t = eps_a / t.level
                sides = [("S", "Q", "om11")] + ([] if symmetric else [("St", "Qt", "omt11")])
                passed, pending = [], []
                for sk, qk, ok in sides:
                    Sloc = getattr(t, sk)
                    if t.state == UNTOUCHED:
                        Q, Om = _qr(Sloc[:, :d])
                        setattr(t, qk, Q)
                        setattr(t, ok, abs(Om[0, 0]) if Om.size else 0.0)
                    Q = getattr(t, qk)
                    Stil = Sloc[:, d:d + dd]
                    Shat = Stil - Q @ (Q.T @ Stil)
                    Shat = Shat - Q @ (Q.T @ Shat)
                    nh = np.linalg.norm(Shat)
                    if nh < eps_a_t or nh < eps_r_t * np.linalg.norm(Stil):
                        passed.append(True)
                        pending.append((qk, Shat))
                        continue
                    Qh, Oh = _qr(Shat)
                    setattr(t, qk, np.hstack([Q, Qh]))
                    mn = float(np.min(np.abs(np.diag(Oh)))) if Oh.size else 0.0
                    passed.append(mn < eps_a_t or mn < eps_r_t * getattr(t, ok))
                if all(passed):
                    t.J, Y = interpolative(t.S.T, eps_r_t, eps_a_t)
                    t.U = Y.T
                    if symmetric:
                        t.Jt, t.V = t.J, t.U
                    else:
                        t.Jt, Yt = interpolative(t.St.T, eps_r_t, eps_a_t)
                        t.V = Yt.T
                    t.state = COMPRESSED
                    newly = True
                else:
                    for qk, Shat in pending:
                        Qh, _ = _qr(Shat)
                        setattr(t, qk, np.hstack([getattr(t, qk), Qh]))
                    s, st = sketcher.add_block(dd)
                    d += dd
                    extensions += 1
                    S = np.hstack([S, s])
                    St = S if symmetric else np.hstack([St, st])
                    t.state = PARTIALLY_COMPRESSED
                    break

            # local operators and skeletons for the parent
            j0 = 0 if newly else i0
            if t.is_leaf:
                Ri = Rcols(t.idx, j0, d + dd)
                rl = t.U.T @ Ri
                rlt = rl if symmetric else t.V.T @ Ri
                t.Itil = t.idx[t.J]
                t.Itilt = t.idx[t.Jt]
            else:
                c1, c2 = t.children
                rl = t.U.T @ np.vstack([c1.Rl[:, j0:d + dd], c2.Rl[:, j0:d + dd]])
                rlt = rl if symmetric else t.V.T @ np.vstack([c1.Rlt[:, j0:d + dd],
                                                              c2.Rlt[:, j0:d + dd]])
                t.Itil = np.concatenate([c1.Itil, c2.Itil])[t.J]
                t.Itilt = np.concatenate([c1.Itilt, c2.Itilt])[t.Jt]
            if j0 == 0:
                t.Rl, t.Rlt = rl, rlt
            else:
                t.Rl = np.hstack([t.Rl, rl])
                t.Rlt = t.Rl if symmetric else np.hstack([t.Rlt, rlt])

    return HSSResult(root, order, d, dd, n, symmetric, root.state == COMPRESSED, extensions)


# ---------------------------------------------------------------- reconstruction
def _ubig(t, which):
    B = t.U if which == "U" else t.V
    if t.is_leaf:
        return B
    c1, c2 = t.children
    u1, u2 = _ubig(c1, which), _ubig(c2, which)
    blk = np.zeros((u1.shape[0] + u2.shape[0], u1.shape[1] + u2.shape[1]))
    blk[:u1.shape[0], :u1.shape[1]] = u1
    blk[u1.shape[0]:, u1.shape[1]:] = u2
    return blk @ B


def reconstruct(res):
    """Dense A_HSS from D, nested U/V and B (section 2.2, the worked example of
    equation "HSSexamplematrix")."""
    n = res.n
    out = np.zeros((n, n))
    stack = [res.root]
    while stack:
        t = stack.pop()
        if t.is_leaf:
            out[t.lo:t.hi, t.lo:t.hi] = t.D
            continue
        c1, c2 = t.children
        out[c1.lo:c1.hi, c2.lo:c2.hi] = _ubig(c1, "U") @ t.B12 @ _ubig(c2, "V").T
        out[c2.lo:c2.hi, c1.lo:c1.hi] = _ubig(c2, "U") @ t.B21 @ _ubig(c1, "V").T
        stack.extend(t.children)
    return out


def relative_error(A, res):
    """||A - A_HSS||_F / ||A||_F."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - reconstruct(res)) / np.linalg.norm(A))
