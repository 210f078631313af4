"""Python layer over the C ABI: device memory and streams come from PyTorch, every
step of every sketch runs in the library's HIP kernels.

Matrices are column-major: a torch tensor of shape (m, n) with stride (1, ld),
e.g. ``colmajor(m, n)`` or ``torch.from_numpy(A_fortran.T).T`` after upload.
"""
import ctypes

import numpy as np
import torch

from . import _abi as abi

KIND = {"gaussian": abi.SK_GAUSSIAN, "sjlt": abi.SK_SJLT, "srht": abi.SK_SRHT}
PREC = {"native": abi.SK_PREC_NATIVE, "bf16": abi.SK_PREC_BF16, "bf16x3": abi.SK_PREC_BF16X3}
CONSTRUCTION = {"block": abi.SK_SJLT_BLOCK, "graph": abi.SK_SJLT_GRAPH}


class SketchError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sketch error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != abi.SK_OK:
        raise SketchError(rc, abi.load().sketch_last_error().decode())


def colmajor(m, n, dtype=torch.float64, device="cuda"):
    """Uninitialised column-major m x n tensor (shape (m, n), stride (1, m))."""
    return torch.empty((n, m), dtype=dtype, device=device).T


def to_device_colmajor(A, device="cuda"):
    """Upload a numpy matrix as a column-major device tensor, values unchanged."""
    A = np.asfortranarray(A)
    return torch.from_numpy(A.T).to(device).T


def _dtype_code(t):
    if t == torch.float64:
        return abi.SK_F64
    if t == torch.float32:
        return abi.SK_F32
    raise ValueError("A must be float64 or float32")


def _ld(t):
    """Leading dimension of a column-major 2-D tensor (size-1 dims have free strides)."""
    if t.dim() != 2 or (t.stride(0) != 1 and t.shape[0] > 1):
        raise ValueError("expected a column-major 2-D tensor (stride(0) == 1)")
    ld = t.stride(1) if t.shape[1] > 1 else t.shape[0]
    if ld < t.shape[0]:
        raise ValueError("leading dimension smaller than the row count")
    return max(ld, 1)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def dense_input(A, symmetric=False):
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    m, n = A.shape
    return abi.SkInput(input=abi.SK_DENSE, dtype=_dtype_code(A.dtype), m=m, n=n, lda=_ld(A),
                       A=A.data_ptr(), symmetric=int(bool(symmetric)))


def points_input(X, h, shift=0.0):
    if not X.is_cuda or X.dtype != torch.float32 or not X.is_contiguous() or X.dim() != 2:
        raise ValueError("X must be a contiguous N x dim float32 device tensor")
    return abi.SkInput(input=abi.SK_POINTS, dtype=abi.SK_F32, dim=X.shape[1], X=X.data_ptr(),
                       N=X.shape[0], h=float(h), shift=float(shift))


def _output(S, St):
    o = abi.SkOutput(S=S.data_ptr(), ldS=_ld(S))
    if St is not None:
        o.St = St.data_ptr()
        o.ldSt = _ld(St)
    return o


class Context:
    """Per-device library context (sketch_init / sketch_finalize)."""

    def __init__(self, device=0, profile=False):
        import weakref
        self._lib = abi.load()
        self.ptr = ctypes.c_void_p()
        _check(self._lib.sketch_init(ctypes.byref(self.ptr), device, abi.SK_INIT_PROFILE if profile else 0))
        self.device = device
        self._live = weakref.WeakSet()   # sketches to release before finalize

    def profile(self, on=True):
        _check(self._lib.sketch_profile_enable(self.ptr, int(bool(on))))

    def profile_read(self, name, reset=False):
        """(total ms, launches) recorded for a kernel family since the last reset."""
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        _check(self._lib.sketch_profile_read(self.ptr, name.encode(), ctypes.byref(ms), ctypes.byref(cnt),
                                             int(bool(reset))))
        return ms.value, cnt.value

    def test_hook(self, hook, arg):
        """Failure-injection hooks for tests (sketch_test_hook)."""
        _check(self._lib.sketch_test_hook(self.ptr, hook, int(arg)))

    def poison_lds(self, pattern=0x7fc00000, stream=None):
        """Fill every CU's LDS with ``pattern`` (sketch_test_poison_lds)."""
        _check(self._lib.sketch_test_poison_lds(self.ptr, pattern, _stream(stream)))

    def close(self):
        if self.ptr:
            for sk in list(self._live):
                sk.release()
            _check(self._lib.sketch_finalize(self.ptr))
            self.ptr = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Sketch:
    """One operator R = [R_0 | R_1 | ...] applied to one input.

    ``Sketch(ctx, A, "sjlt", d, seed, alpha=4, transpose=True)`` computes S = A R
    (and S' = A^T R when ``transpose``) into ``self.S`` / ``self.St``.
    """

    def __init__(self, ctx, A, kind, d, seed, alpha=4, prec="native", transpose=False, symmetric=False,
                 points=None, stream=None, construction="block", _handle=None, _widths=None):
        self._lib = abi.load()
        self.ctx = ctx
        self.kind = kind
        self.symmetric = symmetric
        if points is not None:
            X, h, shift = points
            self._in = points_input(X, h, shift)
            rows, dtype, device = X.shape[0], torch.float32, X.device
            self._keep = X
        else:
            self._in = dense_input(A, symmetric)
            rows, dtype, device = A.shape[0], A.dtype, A.device
            self._keep = A
        self.rows = rows
        self.dtype = dtype
        self.device = device
        self.transpose = transpose
        if _handle is not None:        # an existing handle (state import, batched call)
            self.h = _handle
            self.widths = list(_widths)
            self.S = self.St = None
            ctx._live.add(self)
            return
        op = abi.SkOpDesc(kind=KIND[kind], alpha=alpha, construction=CONSTRUCTION[construction],
                          prec=PREC[prec], flags=0)
        self.S = colmajor(rows, d, dtype, device)
        self.St = colmajor(self._in.n, d, dtype, device) if transpose else None
        self.h = ctypes.c_void_p()
        _check(self._lib.sketch_apply(ctx.ptr, ctypes.byref(self._in), ctypes.byref(op), d, seed,
                                      ctypes.byref(_output(self.S, self.St)), ctypes.byref(self.h),
                                      _stream(stream)))
        self.widths = [d]
        ctx._live.add(self)

    # -------------------------------------------------------------- state
    def export_state(self):
        """The operator's state (bytes): sketch_state_export."""
        n = ctypes.c_size_t()
        _check(self._lib.sketch_state_export(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self._lib.sketch_state_export(self.h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    @classmethod
    def import_state(cls, ctx, state, A=None, transpose=False, symmetric=False, points=None, widths=None):
        """A Sketch bound to input A (or points) whose operator comes from
        ``state`` (sketch_state_import).  S / St are None until ``rerun`` or
        ``extend`` computes columns; ``widths`` defaults to the state's blocks."""
        lib = abi.load()
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(state, len(state))
        _check(lib.sketch_state_import(ctx.ptr, buf, len(state), ctypes.byref(h)))
        d, nb = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.sketch_width(h, ctypes.byref(d), ctypes.byref(nb)))
        # the block widths follow the state's 64-byte header as int32 values
        ws = widths if widths is not None else list(np.frombuffer(state, dtype=np.int32, count=nb.value, offset=64))
        return cls(ctx, A, None, d.value, 0, transpose=transpose, symmetric=symmetric, points=points,
                   _handle=h, _widths=ws)

    # -------------------------------------------------------------- growth
    def extend(self, dd, nblocks=1, stream=None):
        """Append nblocks blocks of width dd; computes only the new columns (one
        pass) and returns them (S_new, St_new); self.S / self.St are grown."""
        w = dd * nblocks
        Sn = colmajor(self.rows, w, self.dtype, self.device)
        Stn = colmajor(self._in.n, w, self.dtype, self.device) if self.transpose else None
        _check(self._lib.sketch_extend(self.h, ctypes.byref(self._in), dd, nblocks,
                                       ctypes.byref(_output(Sn, Stn)), _stream(stream)))
        self.widths += [dd] * nblocks
        # a handle resumed from a state (or made by the batched call) has no
        # columns computed yet: S / St stay None until rerun computes all of them
        if self.S is not None:
            self.S = _hcat(self.S, Sn)
            if self.transpose:
                self.St = _hcat(self.St, Stn)
        return Sn, Stn

    def rerun(self, seed, stream=None):
        """Redraw every block from ``seed`` and recompute all columns in place."""
        d = int(sum(self.widths))
        if self.S is None or self.S.shape[1] != d:   # every column of the operator is written
            self.S = colmajor(self.rows, d, self.dtype, self.device)
            self.St = colmajor(self._in.n, d, self.dtype, self.device) if self.transpose else None
        _check(self._lib.sketch_rerun(self.h, ctypes.byref(self._in), seed,
                                      ctypes.byref(_output(self.S, self.St)), _stream(stream)))

    # -------------------------------------------------------------- backward
    def adjoint(self, dS, block0=0, nblocks=None, stream=None):
        """Backward of the sketch for blocks [block0, block0 + nblocks).

        Stored A: returns dA = dS R^T (m x n, column-major).
        Point input: dS is W = dL/dS; returns (dX, dh) for L = sum(W o S)."""
        nb = len(self.widths) - block0 if nblocks is None else nblocks
        if not (0 <= block0 and 1 <= nb and block0 + nb <= len(self.widths)):
            raise ValueError("block range [%d, %d) outside the %d blocks" % (block0, block0 + nb, len(self.widths)))
        wt = sum(self.widths[block0:block0 + nb])
        if tuple(dS.shape) != (self.rows, wt) or dS.dtype != self.dtype or dS.device != self.device:
            raise ValueError("dS must be a %d x %d %s tensor on %s, got %s %s on %s"
                             % (self.rows, wt, self.dtype, self.device, tuple(dS.shape), dS.dtype, dS.device))
        dS = _as_colmajor(dS)
        dS_ld = _ld(dS)
        if self._in.input == abi.SK_POINTS:
            X = self._keep
            dX = torch.empty_like(X)
            dh = torch.empty((), dtype=torch.float64, device=X.device)
            _check(self._lib.sketch_adjoint(self.h, ctypes.byref(self._in), block0, nb, dS.data_ptr(), dS_ld,
                                            None, 0, dX.data_ptr(), dh.data_ptr(), _stream(stream)))
            return dX, dh
        dA = colmajor(self._in.m, self._in.n, self.dtype, self.device)
        _check(self._lib.sketch_adjoint(self.h, ctypes.byref(self._in), block0, nb, dS.data_ptr(), dS_ld,
                                        dA.data_ptr(), _ld(dA), None, None, _stream(stream)))
        return dA

    # -------------------------------------------------------------- queries
    @property
    def width(self):
        d, nb = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.sketch_width(self.h, ctypes.byref(d), ctypes.byref(nb)))
        return d.value, nb.value

    def get_rows(self, i0, i1, j0, j1):
        out = np.zeros((j1 - j0, i1 - i0), dtype=np.float64)  # column-major (i1-i0) x (j1-j0)
        _check(self._lib.sketch_get_rows(self.h, i0, i1, j0, j1, out.ctypes.data, i1 - i0))
        return out.T

    def sjlt_codes(self, block, alpha):
        n = self._in.N if self._in.input == abi.SK_POINTS else self._in.n
        codes = np.zeros((n, alpha), dtype=np.uint32)
        _check(self._lib.sketch_get_sjlt(self.h, block, codes.ctypes.data))
        return codes

    def srht_data(self, j0, j1):
        n = self._in.n
        D = np.zeros(n, dtype=np.int8)
        mu = np.zeros(j1 - j0, dtype=np.uint32)
        _check(self._lib.sketch_get_srht(self.h, D.ctypes.data, mu.ctypes.data, j0, j1))
        return D, mu

    def gaussian_bits(self, block, w):
        n = self._in.N if self._in.input == abi.SK_POINTS else self._in.n
        bits = np.zeros((w, n), dtype=np.uint16)
        _check(self._lib.sketch_get_gaussian(self.h, block, bits.ctypes.data))
        return bits.T

    def release(self):
        if self.h:
            _check(self._lib.sketch_release(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Batch:
    """Batched SJLT sketches of many stored matrices (sketch_batch_*).

    ``Batch(ctx, mats, d, dd, seeds)`` plans S_i = A_i R_i for every device
    matrix ``mats[i]`` (column-major, one dtype) with target width ``d[i]``
    built in blocks of ``dd``; ``run()`` computes all rounds into ``self.S[i]``
    (and ``self.St[i]`` with ``transpose=True``).
    """

    def __init__(self, ctx, mats, d, dd, seeds, alpha=4, transpose=False, graph=True, autotune=False,
                 stream=None):
        self._lib = abi.load()
        self.ctx = ctx
        count = len(mats)
        if not (len(d) == count and len(seeds) == count and count >= 1):
            raise ValueError("mats, d and seeds must have the same positive length")
        self._keep = list(mats)
        ins = (abi.SkInput * count)()
        outs = (abi.SkOutput * count)()
        self.S, self.St = [], []
        for i, A in enumerate(mats):
            ins[i] = dense_input(A, False)
            S = colmajor(A.shape[0], d[i], A.dtype, A.device)
            St = colmajor(A.shape[1], d[i], A.dtype, A.device) if transpose else None
            self.S.append(S)
            self.St.append(St)
            outs[i] = _output(S, St)
        self._ins, self._outs = ins, outs
        self.count = count
        darr = (ctypes.c_int32 * count)(*[int(x) for x in d])
        sarr = (ctypes.c_uint64 * count)(*[int(x) for x in seeds])
        flags = (abi.SK_BATCH_GRAPH if graph else 0) | (abi.SK_BATCH_AUTOTUNE if autotune else 0)
        self.h = ctypes.c_void_p()
        _check(self._lib.sketch_batch_create(ctx.ptr, ins, count, darr, dd, alpha, sarr, outs, flags,
                                             ctypes.byref(self.h), _stream(stream)))
        ctx._live.add(self)

    def run(self, r0=0, r1=None, stream=None):
        if r1 is None:
            r1 = self.info()[0]
        _check(self._lib.sketch_batch_run(self.h, r0, r1, _stream(stream)))

    def reseed(self, seeds, stream=None):
        sarr = (ctypes.c_uint64 * self.count)(*[int(x) for x in seeds])
        _check(self._lib.sketch_batch_reseed(self.h, sarr, _stream(stream)))

    def mode(self, r):
        """How round r runs (abi.SK_ROUND_*)."""
        m = ctypes.c_int32()
        _check(self._lib.sketch_batch_mode(self.h, r, ctypes.byref(m)))
        return m.value

    def info(self):
        """(number of rounds, (chunk, waves, columns per wave, rows per lane))"""
        nr = ctypes.c_int32()
        shape = (ctypes.c_int32 * 4)()
        _check(self._lib.sketch_batch_info(self.h, ctypes.byref(nr), shape))
        return nr.value, tuple(shape)

    def release(self):
        if self.h:
            _check(self._lib.sketch_batch_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def apply_batched(ctx, mats, d, dd, seeds, alpha=4, transpose=False, graph=True, autotune=False, handles=False,
                  stream=None):
    """One call for a whole batch (sketch_apply_batched): returns (S list, St list,
    Sketch list or None).  The Sketch objects hold each matrix's operator (blocks
    of width dd) for later extension; their S / St start as None."""
    lib = abi.load()
    count = len(mats)
    ins = (abi.SkInput * count)()
    outs = (abi.SkOutput * count)()
    S, St = [], []
    for i, A in enumerate(mats):
        ins[i] = dense_input(A, False)
        S.append(colmajor(A.shape[0], d[i], A.dtype, A.device))
        St.append(colmajor(A.shape[1], d[i], A.dtype, A.device) if transpose else None)
        outs[i] = _output(S[i], St[i])
    op = abi.SkOpDesc(kind=abi.SK_SJLT, alpha=alpha, construction=abi.SK_SJLT_BLOCK, prec=0, flags=0)
    darr = (ctypes.c_int32 * count)(*[int(x) for x in d])
    sarr = (ctypes.c_uint64 * count)(*[int(x) for x in seeds])
    hs = (ctypes.c_void_p * count)() if handles else None
    flags = (abi.SK_BATCH_GRAPH if graph else 0) | (abi.SK_BATCH_AUTOTUNE if autotune else 0)
    _check(lib.sketch_apply_batched(ctx.ptr, ins, ctypes.byref(op), darr, dd, sarr, outs, count, flags, hs,
                                    _stream(stream)))
    sks = None
    if handles:
        sks = [Sketch(ctx, mats[i], None, d[i], 0, alpha=alpha, transpose=transpose,
                      _handle=ctypes.c_void_p(hs[i]), _widths=[dd] * (d[i] // dd)) for i in range(count)]
    return S, St, sks


def _as_colmajor(T):
    if T.dim() == 2 and (T.stride(0) == 1 or T.shape[0] == 1):
        return T
    return T.t().contiguous().t()


class DenseSketchFn(torch.autograd.Function):
    """S = A R with a hand-written backward dA = dS R^T (SJLT)."""

    @staticmethod
    def forward(fctx, A, lib_ctx, d, seed, alpha):
        sk = Sketch(lib_ctx, _as_colmajor(A.detach()), "sjlt", d, seed, alpha=alpha)
        fctx.sk = sk
        return sk.S

    @staticmethod
    def backward(fctx, gS):
        dA = fctx.sk.adjoint(gS)
        return dA, None, None, None, None


class KernelSketchFn(torch.autograd.Function):
    """S = K(X, h) R (SJLT R, K never stored) with the hand-written backward
    for dL/dX and dL/dh; the bandwidth h is a 0-dim tensor."""

    @staticmethod
    def forward(fctx, X, h, lib_ctx, d, seed, alpha, shift):
        X = X.detach().contiguous()
        sk = Sketch(lib_ctx, None, "sjlt", d, seed, alpha=alpha, points=(X, float(h), shift))
        fctx.sk = sk
        fctx.h_dtype = h.dtype if torch.is_tensor(h) else None
        return sk.S

    @staticmethod
    def backward(fctx, gS):
        dX, dh = fctx.sk.adjoint(gS)
        dh = dh.to(fctx.h_dtype) if fctx.h_dtype is not None else None
        return dX, dh, None, None, None, None, None


def kernel_sketch(X, h, d, seed, lib_ctx, alpha=4, shift=0.0):
    """Differentiable matrix-free sketch S = K(X, h) R."""
    return KernelSketchFn.apply(X, h, lib_ctx, d, seed, alpha, shift)


def dense_sketch(A, d, seed, lib_ctx, alpha=4):
    """Differentiable SJLT sketch S = A R of a stored matrix."""
    return DenseSketchFn.apply(A, lib_ctx, d, seed, alpha)


def _hcat(X, Y):
    out = colmajor(X.shape[0], X.shape[1] + Y.shape[1], X.dtype, X.device)
    out[:, :X.shape[1]] = X
    out[:, X.shape[1]:] = Y
    return out


def bf16_bits_to_f64(bits):
    """bfloat16 bit patterns -> FP64 values (exact)."""
    u = np.asarray(bits, dtype=np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)
