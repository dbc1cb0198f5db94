"""ctypes binding of libplhr.so (argument marshalling only).

Every numerical step runs in the HIP library; this module only mirrors the
C structs of include/plhr.h and loads the shared object.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplhr.so")

# status codes
OK, ERR_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NOT_HPD, ERR_BREAKDOWN, ERR_NOT_CONVERGED, ERR_STATE = range(8)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_UNSUPPORTED", 3: "ERR_HIP", 4: "ERR_NOT_HPD",
                5: "ERR_BREAKDOWN", 6: "ERR_NOT_CONVERGED", 7: "ERR_STATE"}

OP_IDENTITY, OP_FD5_2D, OP_FD7_3D, OP_DIAG, OP_Q1_2D, OP_Q1_3D, OP_Q1_MASS, OP_CSR = 0, 1, 2, 3, 4, 5, 6, 7
OP_BLOCH7_3D = 8
F64, C128 = 0, 1
PREC_IDENTITY, PREC_MG_VCYCLE, PREC_AV_MG, PREC_INV_MG, PREC_DENSE = 0, 1, 2, 3, 4
EXTRACT_T_HARMONIC, EXTRACT_HARMONIC = 0, 1
ALG_BLOCK, ALG_SINGLE, ALG_PLMR = 0, 1, 2
PRECISION_FP64, PRECISION_MIXED = 0, 1


class OpDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("reserved0", C.c_int32), ("h", C.c_double),
                ("scale", C.c_double), ("potential", C.c_void_p), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("values", C.c_void_p), ("nnz", C.c_int64),
                ("theta", C.c_double * 3)]


class PrecDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("levels", C.c_int32), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("omega", C.c_double), ("delta", C.c_double),
                ("degree", C.c_int32), ("reserved0", C.c_int32), ("matrix", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int32), ("k_extra", C.c_int32),
                ("precision", C.c_int32), ("lock", C.c_int32), ("check_every", C.c_int32),
                ("ortho_passes", C.c_int32), ("drop_tol", C.c_double),
                ("extraction", C.c_int32), ("use_graph", C.c_int32),
                ("algorithm", C.c_int32), ("reserved0", C.c_int32)]


class IterInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("n_active", C.c_int32),
                ("status", C.c_int32), ("max_rel_res", C.c_double),
                ("n_excluded", C.c_int32), ("reserved0", C.c_int32)]


KC_COUNT = 16


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int32 * KC_COUNT), ("total_ms", C.c_double * KC_COUNT),
                ("bytes", C.c_double * KC_COUNT), ("flops", C.c_double * KC_COUNT),
                ("truncated", C.c_int32), ("reserved0", C.c_int32)]


KCAT_NAMES = ["stencil", "jacobi", "mg_residual", "restrict", "prolong", "coarse_solve", "gram",
              "gram_reduce", "transform", "update", "tharm_reduce", "tharm_qr", "tharm_vectors",
              "ortho", "small_other", "vec"]
# the HIP kernel each category times
KCAT_KERNELS = ["k_fd_apply", "k_jacobi", "k_residual", "k_restrict", "k_prolong_add",
                "k_dense_apply", "k_gram_mfma", "k_gram_reduce8", "k_rowmul_mfma (transform)",
                "k_rowmul_mfma (update)", "k_tharm_reduce", "k_tharm_qr", "k_tharm_vectors",
                "k_ortho_small", "k_rq_small, k_conv_check", "k_resid_prep, k_xdots, k_copy"]


class BatchTuning(C.Structure):
    _fields_ = [("chunk_points", C.c_int32), ("row_threads", C.c_int32), ("use_graph", C.c_int32),
                ("nchunks", C.c_int32), ("tuned_ms", C.c_double * 8)]


class PLHRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load libplhr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libplhr.so not found at {LIB_PATH}; run "
                           "`python -m paper_1408_0042_amd.build` first")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "plhr_version": (C.c_char_p, []),
        "plhr_last_error": (C.c_char_p, []),
        "plhr_options_default": (C.c_int, [C.POINTER(Options)]),
        "plhr_workspace_size": (C.c_int, [C.POINTER(OpDesc), C.POINTER(OpDesc), C.POINTER(PrecDesc),
                                          C.c_double, C.c_int32, C.POINTER(Options),
                                          C.POINTER(C.c_size_t)]),
        "plhr_create": (C.c_int, [C.POINTER(OpDesc), C.POINTER(OpDesc), C.POINTER(PrecDesc),
                                  C.c_double, C.c_int32, C.POINTER(Options), P, P, C.c_size_t,
                                  C.POINTER(P)]),
        "plhr_start": (C.c_int, [P, P]),
        "plhr_iterate": (C.c_int, [P, C.c_int32, C.POINTER(IterInfo)]),
        "plhr_finish": (C.c_int, [P, P, P, C.POINTER(C.c_double)]),
        "plhr_solve": (C.c_int, [P, P, P, P, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "plhr_eigvals_backward": (C.c_int, [P, P, P, C.c_int32]),
        "plhr_apply": (C.c_int, [P, C.c_int32, P, P, C.c_int32]),
        "plhr_op_apply": (C.c_int, [C.POINTER(OpDesc), C.c_double, P, P, C.c_int32, P]),
        "plhr_bloch_prec_create": (C.c_int, [C.POINTER(OpDesc), C.POINTER(PrecDesc), C.c_int32,
                                             P, P, C.c_size_t, C.POINTER(P)]),
        "plhr_bloch_prec_workspace_size": (C.c_int, [C.POINTER(OpDesc), C.POINTER(PrecDesc),
                                                     C.c_int32, C.POINTER(C.c_size_t)]),
        "plhr_bloch_prec_apply": (C.c_int, [P, P, P, C.c_int32]),
        "plhr_bloch_prec_destroy": (None, [P]),
        "plhr_gram_c128_workspace": (C.c_int, [C.c_int64, C.c_int32, C.c_int32,
                                               C.POINTER(C.c_size_t)]),
        "plhr_gram_c128": (C.c_int, [C.c_int64, P, C.c_int32, P, C.c_int32, P, P, C.c_size_t,
                                     P]),
        "plhr_cholqr_c128_workspace": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
        "plhr_cholqr_c128": (C.c_int, [C.c_int64, P, C.c_int32, P, P, P, C.c_size_t, P]),
        "plhr_rowmul_c128": (C.c_int, [C.c_int64, P, C.c_int32, P, C.c_int32, P, P]),
        "plhr_projected_workspace": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
        "plhr_projected_solve": (C.c_int, [C.c_int32, C.c_int32, P, P, P, P, P, P, P,
                                           C.POINTER(C.c_int32), P, C.c_size_t, P]),
        "plhr_projected_noalloc_scratch_bytes": (C.c_size_t, []),
        "plhr_projected_solve_noalloc": (C.c_int, [C.c_int32, C.c_int32, P, P, P, P, P, P, P, P,
                                                   P]),
        "plhr_get_state": (C.c_int, [P, C.POINTER(C.c_double), P]),
        "plhr_debug_read": (C.c_int, [P, C.c_int32, C.POINTER(C.c_double), C.c_size_t]),
        "plhr_profile_start": (C.c_int, [P, C.c_int32, C.c_int32]),
        "plhr_profile_stop": (C.c_int, [P, C.POINTER(Profile)]),
        "plhr_destroy": (None, [P]),
        "plhr_batch_create": (C.c_int, [C.c_int32, C.POINTER(OpDesc), C.POINTER(PrecDesc),
                                        C.POINTER(C.c_double), C.c_int32, C.POINTER(Options), P,
                                        P, C.c_size_t, C.POINTER(P)]),
        "plhr_batch_workspace_size": (C.c_int, [C.c_int32, C.POINTER(OpDesc),
                                                C.POINTER(PrecDesc), C.POINTER(C.c_double),
                                                C.c_int32, C.POINTER(Options),
                                                C.POINTER(C.c_size_t)]),
        "plhr_batch_solve": (C.c_int, [P, C.POINTER(P), P, C.POINTER(P), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "plhr_batch_eigvals_backward": (C.c_int, [P, P, C.POINTER(P), C.c_int32]),
        "plhr_batch_tuning_info": (C.c_int, [P, C.POINTER(BatchTuning)]),
        "plhr_batch_apply": (C.c_int, [P, C.c_int32, C.POINTER(P), C.POINTER(P), C.c_int32]),
        "plhr_batch_set_graph": (C.c_int, [P, C.c_int32]),
        "plhr_batch_profile_start": (C.c_int, [P, C.c_int32, C.c_int32]),
        "plhr_batch_profile_stop": (C.c_int, [P, C.POINTER(Profile)]),
        "plhr_batch_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != OK:
        msg = load().plhr_last_error().decode(errors="replace")
        raise PLHRError(code, msg)


def default_options() -> Options:
    o = Options()
    check(load().plhr_options_default(C.byref(o)))
    return o
