"""ctypes binding of libglasma.so (argument marshalling only).

The library is loaded from this package directory; a missing or unloadable library
raises at import of the binding so that no caller can silently fall back to another
implementation.
"""
import ctypes as C
import os

# torch first: its bundled HIP runtime then carries the soname libglasma.so asks for, so
# both use one runtime.  Loaded the other way round, the process would hold two HIP
# runtimes, and device memory from one is invalid in the other.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglasma.so")

GLASMA_OK = 0
ERRORS = {-1: "GLASMA_E_ARG", -2: "GLASMA_E_HIP", -3: "GLASMA_E_NONFINITE",
          -4: "GLASMA_E_CONSTRAINT", -5: "GLASMA_E_NOCONV", -6: "GLASMA_E_STATE"}
OBS_NSCALARS = 8
OBS = {"energy": 0, "gauss_l2": 1, "rho_l2": 2, "gauss_max": 3, "unitarity": 4,
       "nonfinite": 5, "gauss_rel": 6}


class Params(C.Structure):
    _fields_ = [("nc", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32),
                ("a_T", C.c_double), ("a_L", C.c_double), ("dt", C.c_double),
                ("fp", C.c_int32), ("scheme", C.c_int32), ("reunit_every", C.c_int32),
                ("max_iter", C.c_int32), ("tol", C.c_double)]


class Buffers(C.Structure):
    _fields_ = [("U", C.c_void_p), ("U_alt", C.c_void_p), ("E", C.c_void_p),
                ("rhoA", C.c_void_p), ("rhoB", C.c_void_p), ("work", C.c_void_p)]


class MV(C.Structure):
    _fields_ = [("m_ir", C.c_double), ("uv_cut", C.c_double), ("sigma", C.c_double),
                ("zA", C.c_double), ("zB", C.c_double)]


class GlasmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2009_02044_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, D, I32, I64, V = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_void_p
    sig = {
        "glasma_version": ([], C.c_char_p),
        "glasma_last_error": ([P], C.c_char_p),
        "glasma_layout": ([C.POINTER(Params), C.POINTER(C.c_size_t)], C.c_int),
        "glasma_create": ([C.POINTER(Params), C.POINTER(Buffers), V, C.POINTER(P)], C.c_int),
        "glasma_destroy": ([P], C.c_int),
        "glasma_init_state": ([P, D, D, D, D, I64], C.c_int),
        "glasma_init_mv": ([P, C.POINTER(MV), D, D], C.c_int),
        "glasma_init_mv_sheets": ([P, C.POINTER(MV), I32, D, D], C.c_int),
        "glasma_bi_work_bytes": ([C.POINTER(Params), C.POINTER(C.c_size_t)], C.c_int),
        "glasma_bi_fields": ([C.POINTER(Params), C.POINTER(MV), I32, D, D, V, V, V, V, V], C.c_int),
        "glasma_step": ([P, I32], C.c_int),
        "glasma_deposit_current": ([P, V], C.c_int),
        "glasma_observe": ([P, V], C.c_int),
        "glasma_observe_noalloc": ([P, V], C.c_int),
        "glasma_rest_frame": ([P, V, V], C.c_int),
        "glasma_step_observe": ([P, I32, V], C.c_int),
        "glasma_observables": ([P, D, D, D, D, D], C.c_int),
        "glasma_get_state": ([P, D, D, D, D, C.POINTER(I64)], C.c_int),
        "glasma_reunitarize": ([P], C.c_int),
        "glasma_get_step": ([P, C.POINTER(I64)], C.c_int),
        "glasma_last_iterations": ([P, C.POINTER(I32)], C.c_int),
        "glasma_host_group_op": ([I32, I32, I32, I64, D, D], C.c_int),
        "glasma_set_state_device": ([P, V, V, V, V, V, V, I64], C.c_int),
        "glasma_get_state_device": ([P, V, V, V, V], C.c_int),
        "glasma_adjoint_layout": ([C.POINTER(Params), I32, I32, C.POINTER(C.c_size_t)], C.c_int),
        "glasma_adjoint_forward": ([P, I32, I32, V, C.c_size_t], C.c_int),
        "glasma_adjoint_backward": ([P, I32, I32, C.c_double, V, C.c_size_t, V, V, D, V, V, V, V, V], C.c_int),
        "glasma_slab_energy": ([P, I32, I32, D], C.c_int),
        "glasma_adjoint_backward_cotangent": ([P, V, C.c_size_t, V, V, V, V, V, V, V, V, V, V, V, V], C.c_int),
        "glasma_batch_layout": ([C.POINTER(Params), I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(C.c_size_t)], C.c_int),
        "glasma_batch_create": ([C.POINTER(Params), I32, C.POINTER(I32), C.POINTER(I32), V, V, C.POINTER(P)], C.c_int),
        "glasma_batch_destroy": ([P], C.c_int),
        "glasma_batch_last_error": ([P], C.c_char_p),
        "glasma_batch_event": ([P, I32, C.POINTER(P)], C.c_int),
        "glasma_batch_run": ([P, I32, I32], C.c_int),
        "glasma_batch_set_tiling": ([P, I32, I32], C.c_int),
        "glasma_batch_classes": ([P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)], C.c_int),
        "glasma_batch_observe": ([P, I32, V, V, V], C.c_int),
        "glasma_batch_autotune": ([P, I32, C.c_char_p, C.c_size_t], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def check(rc, ctx=None):
    if rc != GLASMA_OK:
        msg = lib.glasma_last_error(ctx)
        raise GlasmaError(rc, msg.decode() if msg else "")
    return rc


def check_batch(rc, b=None):
    if rc != GLASMA_OK:
        msg = lib.glasma_batch_last_error(b)
        raise GlasmaError(rc, msg.decode() if msg else "")
    return rc


def dptr(a):
    """double* of a C-contiguous float64 numpy array (or None)."""
    if a is None:
        return None
    assert a.dtype.name == "float64" and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))
