"""ctypes declarations of the C ABI in include/sketch.h (argument marshalling only).

The shared library is built in-tree by ``paper_2302_01977_amd.build`` (or
``__graft_entry__.build()``).  Loading fails loudly when it is missing: there is
no fallback implementation of any sketch.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhsketch.so")

SK_OK, SK_EINVAL, SK_EUNSUPPORTED, SK_ENOMEM, SK_EHIP, SK_ESTATE = 0, -1, -2, -3, -4, -5
SK_GAUSSIAN, SK_SJLT, SK_SRHT = 0, 1, 2
SK_F64, SK_F32 = 0, 1
SK_PREC_NATIVE, SK_PREC_BF16, SK_PREC_BF16X3 = 0, 1, 2
SK_DENSE, SK_POINTS = 0, 1
SK_BATCH_GRAPH, SK_BATCH_AUTOTUNE = 1, 2
SK_SJLT_BLOCK, SK_SJLT_GRAPH = 0, 1
SK_INIT_PROFILE = 1
SK_ROUND_EAGER, SK_ROUND_NOT_CAPTURED, SK_ROUND_GRAPH, SK_ROUND_CAPTURE_FAILED = 0, 1, 2, 3
SK_HOOK_FAIL_ALLOC, SK_HOOK_FAIL_GRAPH = 1, 2

c_i32, c_i64, c_u64, c_f32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float, ctypes.c_void_p


class SkInput(ctypes.Structure):
    _fields_ = [("input", c_i32), ("dtype", c_i32), ("m", c_i64), ("n", c_i64), ("lda", c_i64),
                ("A", c_vp), ("symmetric", c_i32), ("dim", c_i32), ("X", c_vp), ("N", c_i64),
                ("h", c_f32), ("shift", c_f32)]


class SkOpDesc(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("alpha", c_i32), ("construction", c_i32), ("prec", c_i32), ("flags", c_i32)]


class SkOutput(ctypes.Structure):
    _fields_ = [("S", c_vp), ("ldS", c_i64), ("St", c_vp), ("ldSt", c_i64)]


c_f64 = ctypes.c_double


class SkGemmDesc(ctypes.Structure):
    _fields_ = [("m", c_i32), ("n", c_i32), ("k", c_i32), ("transA", c_i32), ("transB", c_i32),
                ("alpha", c_f64), ("beta", c_f64), ("A", c_vp), ("lda", c_i64), ("B", c_vp), ("ldb", c_i64),
                ("C", c_vp), ("ldc", c_i64)]


class SkQrDesc(ctypes.Structure):
    _fields_ = [("m", c_i32), ("n", c_i32), ("A", c_vp), ("lda", c_i64), ("rdiag", c_vp), ("Q", c_vp),
                ("ldq", c_i64)]


class SkIdDesc(ctypes.Structure):
    _fields_ = [("p", c_i32), ("q", c_i32), ("M", c_vp), ("ldm", c_i64), ("eps_r", c_f64), ("eps_a", c_f64),
                ("perm", c_vp), ("rank", c_vp), ("Y", c_vp), ("ldy", c_i64)]


class SkNormDesc(ctypes.Structure):
    _fields_ = [("m", c_i32), ("n", c_i32), ("A", c_vp), ("lda", c_i64), ("out", c_vp)]


class SkGatherDesc(ctypes.Structure):
    _fields_ = [("m", c_i32), ("n", c_i32), ("trans", c_i32), ("src", c_vp), ("lds", c_i64), ("rows", c_vp),
                ("cols", c_vp), ("row0", c_i64), ("col0", c_i64), ("dst", c_vp), ("ldd", c_i64)]


P = ctypes.POINTER
_SIGS = {
    "sketch_init": (c_i32, [P(c_vp), c_i32, ctypes.c_uint32]),
    "sketch_finalize": (c_i32, [c_vp]),
    "sketch_last_error": (ctypes.c_char_p, []),
    "sketch_apply": (c_i32, [c_vp, P(SkInput), P(SkOpDesc), c_i32, c_u64, P(SkOutput), P(c_vp), c_vp]),
    "sketch_extend": (c_i32, [c_vp, P(SkInput), c_i32, c_i32, P(SkOutput), c_vp]),
    "sketch_rerun": (c_i32, [c_vp, P(SkInput), c_u64, P(SkOutput), c_vp]),
    "sketch_rerun_static": (c_i32, [c_vp, P(SkInput), c_u64, P(SkOutput), c_vp]),
    "sketch_adjoint": (c_i32, [c_vp, P(SkInput), c_i32, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "sketch_width": (c_i32, [c_vp, P(c_i32), P(c_i32)]),
    "sketch_release": (c_i32, [c_vp]),
    "sketch_get_rows": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_i64, c_vp, c_i64]),
    "sketch_get_sjlt": (c_i32, [c_vp, c_i32, c_vp]),
    "sketch_get_srht": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32]),
    "sketch_get_gaussian": (c_i32, [c_vp, c_i32, c_vp]),
    "sketch_batch_create": (c_i32, [c_vp, P(SkInput), c_i32, c_vp, c_i32, c_i32, c_vp, P(SkOutput), c_i32,
                                    P(c_vp), c_vp]),
    "sketch_batch_run": (c_i32, [c_vp, c_i32, c_i32, c_vp]),
    "sketch_batch_reseed": (c_i32, [c_vp, c_vp, c_vp]),
    "sketch_batch_info": (c_i32, [c_vp, P(c_i32), c_vp]),
    "sketch_batch_destroy": (c_i32, [c_vp]),
    "sketch_batch_mode": (c_i32, [c_vp, c_i32, P(c_i32)]),
    "sketch_apply_batched": (c_i32, [c_vp, P(SkInput), P(SkOpDesc), c_vp, c_i32, c_vp, P(SkOutput), c_i32, c_i32,
                                     c_vp, c_vp]),
    "sketch_state_export": (c_i32, [c_vp, c_vp, P(ctypes.c_size_t)]),
    "sketch_state_import": (c_i32, [c_vp, c_vp, ctypes.c_size_t, P(c_vp)]),
    "sketch_test_hook": (c_i32, [c_vp, c_i32, c_i64]),
    "sketch_batched_gemm": (c_i32, [c_vp, c_vp, c_i32, c_vp]),
    "sketch_batched_qr": (c_i32, [c_vp, c_vp, c_i32, c_vp]),
    "sketch_batched_id": (c_i32, [c_vp, c_vp, c_i32, c_vp]),
    "sketch_batched_norm": (c_i32, [c_vp, c_vp, c_i32, c_vp]),
    "sketch_batched_gather": (c_i32, [c_vp, c_vp, c_i32, c_vp]),
    "sketch_get_rows_device": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp]),
    "sketch_test_poison_lds": (c_i32, [c_vp, ctypes.c_uint32, c_vp]),
    "sketch_profile_enable": (c_i32, [c_vp, c_i32]),
    "sketch_profile_read": (c_i32, [c_vp, ctypes.c_char_p, P(ctypes.c_double), P(c_i64), c_i32]),
}

_lib = None


def load():
    """Load libhsketch.so once and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhsketch.so is not built (expected at %s); run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_names():
    return list(_SIGS)
