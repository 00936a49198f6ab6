"""ctypes view of the C ABI in include/tt_kernel.h.

torch is imported before the library is opened so that libttk.so binds to
the HIP runtime torch already loaded (same soname): one runtime per process.
Loading fails loudly when the library has not been built.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttk.so")

# tt_kernel_kind
KINDS = {
    "se": 1, "exp": 2, "matern32": 3, "matern52": 4, "matern_nu": 5, "matern": 6,
    "mq": 7, "tps": 8, "laplace3d": 9, "laplace2d": 10, "biharmonic": 11, "thinplate": 12,
    "poly": 13, "sep": 14,
}
KIND_DTHETA = {"se": 1, "exp": 1, "matern32": 1, "matern52": 1, "matern_nu": 1, "matern": 2,
               "mq": 1, "tps": 1, "laplace3d": 0, "laplace2d": 0, "biharmonic": 0, "thinplate": 0,
               "poly": 1, "sep": 1}
TTK_FP64, TTK_FP32 = 0, 1
STATUS = {0: "OK", 1: "WARN_NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_HIP", -3: "ERR_OOM",
          -4: "ERR_SINGULAR_CROSS", -5: "ERR_UNSUPPORTED"}


class Params(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int), ("d_theta", ctypes.c_int), ("n_spatial", ctypes.c_int),
        ("n_param", ctypes.c_int), ("kind", ctypes.c_int), ("kernel_const", ctypes.c_double),
        ("box_s", ctypes.c_double * 6), ("box_t", ctypes.c_double * 6),
        ("box_theta", ctypes.c_double * 4), ("tol", ctypes.c_double),
        ("max_rank", ctypes.c_int), ("max_sweeps", ctypes.c_int), ("init_card", ctypes.c_int),
        ("init_max_it", ctypes.c_int), ("n_test", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("dtype", ctypes.c_int), ("symmetric_psd", ctypes.c_int), ("theta_fixed", ctypes.c_double * 2),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int), ("r_s", ctypes.c_int), ("r_t", ctypes.c_int),
        ("ranks", ctypes.c_int * 9), ("cross_ranks", ctypes.c_int * 9),
        ("kernel_evals", ctypes.c_int64), ("sweeps", ctypes.c_int), ("n_decisions", ctypes.c_int),
        ("sampled_error", ctypes.c_double), ("init_max_cond", ctypes.c_double),
        ("min_margin", ctypes.c_double), ("t_cross_ms", ctypes.c_double),
        ("t_round_ms", ctypes.c_double), ("t_factor_ms", ctypes.c_double),
        ("n_src", ctypes.c_int64), ("n_tgt", ctypes.c_int64), ("dtype", ctypes.c_int),
    ]


class Decision(ctypes.Structure):
    _fields_ = [
        ("sweep", ctypes.c_int), ("k", ctypes.c_int), ("rank_before", ctypes.c_int),
        ("sample_pos", ctypes.c_int64), ("bit", ctypes.c_int), ("pivot_row", ctypes.c_int),
        ("pivot_col", ctypes.c_int), ("added", ctypes.c_int), ("sample_max", ctypes.c_double),
        ("sample_margin", ctypes.c_double), ("pivot_abs", ctypes.c_double),
        ("search_margin", ctypes.c_double), ("tau", ctypes.c_double),
    ]


class Pair(ctypes.Structure):
    _fields_ = [
        ("box_s", ctypes.c_double * 6), ("box_t", ctypes.c_double * 6),
        ("src_off", ctypes.c_int64), ("n_src", ctypes.c_int64),
        ("tgt_off", ctypes.c_int64), ("n_tgt", ctypes.c_int64),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("num_pairs", ctypes.c_int), ("num_classes", ctypes.c_int), ("kernel_evals", ctypes.c_int64),
        ("factor_rows", ctypes.c_int64), ("t_cross_ms", ctypes.c_double), ("t_round_ms", ctypes.c_double),
        ("t_factor_ms", ctypes.c_double), ("factor_grid", ctypes.c_int), ("reduce_rows", ctypes.c_int),
        ("graph", ctypes.c_int),
    ]


class HmatInfo(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int), ("num_classes", ctypes.c_int), ("leaves", ctypes.c_int64),
        ("nonempty_leaves", ctypes.c_int64), ("far_pairs", ctypes.c_int64), ("near_pairs", ctypes.c_int64),
        ("kernel_evals", ctypes.c_int64), ("t_tree_ms", ctypes.c_double), ("t_build_ms", ctypes.c_double),
    ]


EXPORTS = [
    "tt_kernel_build_offline", "tt_kernel_build_from_cores", "tt_kernel_factor_rows", "tt_kernel_online_core",
    "tt_kernel_apply", "tt_kernel_apply_noalloc", "tt_kernel_project", "tt_kernel_apply_plain",
    "tt_kernel_apply_backward",
    "tt_kernel_global_online", "tt_kernel_global_apply", "tt_kernel_global_factors",
    "tt_kernel_global2_online", "tt_kernel_global2_apply", "tt_kernel_phase4_round",
    "tt_kernel_batch_build", "tt_kernel_batch_configure", "tt_kernel_batch_factor", "tt_kernel_batch_get_info",
    "tt_kernel_batch_get_class", "tt_kernel_batch_get_factors", "tt_kernel_batch_apply", "tt_kernel_batch_destroy",
    "tt_kernel_hmat_build", "tt_kernel_hmat_apply", "tt_kernel_hmat_get_info", "tt_kernel_hmat_get_lists",
    "tt_kernel_hmat_get_batch", "tt_kernel_hmat_destroy",
    "tt_kernel_eval_entries", "tt_kernel_eval_dense", "tt_kernel_get_info",
    "tt_kernel_get_factors", "tt_kernel_get_cores", "tt_kernel_get_coeff_cores", "tt_kernel_get_cross",
    "tt_kernel_destroy", "tt_kernel_last_error",
]

_lib = None


def load():
    """Open libttk.so and declare the signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2406_06344_amd/build.py "
                           "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, c_int, P = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER
    lib.tt_kernel_build_offline.argtypes = [P(Params), vp, i64, vp, i64, vp, P(vp)]
    lib.tt_kernel_build_from_cores.argtypes = [P(Params), P(c_int), P(ctypes.c_double), vp, i64, vp, i64, vp,
                                               P(vp)]
    lib.tt_kernel_factor_rows.argtypes = [vp, c_int, vp, i64, vp, vp]
    lib.tt_kernel_online_core.argtypes = [vp, vp, c_int, vp, vp, vp]
    lib.tt_kernel_apply.argtypes = [vp, vp, c_int, vp, i64, vp, i64, vp, vp]
    lib.tt_kernel_apply_noalloc.argtypes = [vp, vp, c_int, vp, i64, vp, i64, vp, vp]
    lib.tt_kernel_project.argtypes = [vp, c_int, vp, i64, c_int, vp, vp]
    lib.tt_kernel_apply_plain.argtypes = [vp, vp, c_int, vp, i64, vp, i64, vp]
    lib.tt_kernel_apply_backward.argtypes = [vp, vp, c_int, vp, i64, vp, vp, i64, vp, i64, vp, vp]
    lib.tt_kernel_global_online.argtypes = [vp, vp, c_int, vp, vp]
    lib.tt_kernel_global_apply.argtypes = [vp, vp, vp, c_int, vp, i64, vp, i64, vp]
    lib.tt_kernel_global_factors.argtypes = [vp, P(c_int), vp, P(ctypes.c_double), vp]
    lib.tt_kernel_global2_online.argtypes = [vp, vp, ctypes.c_double, vp, i64, vp, P(c_int), vp]
    lib.tt_kernel_global2_apply.argtypes = [vp, vp, i64, vp, c_int, c_int, vp, i64, vp, i64, vp]
    lib.tt_kernel_phase4_round.argtypes = [vp, ctypes.c_double, vp]
    lib.tt_kernel_batch_build.argtypes = [P(Params), P(Pair), c_int, vp, i64, vp, i64, vp, P(vp)]
    lib.tt_kernel_batch_configure.argtypes = [vp, c_int, c_int, c_int]
    lib.tt_kernel_batch_factor.argtypes = [vp, vp, vp, vp]
    lib.tt_kernel_batch_get_info.argtypes = [vp, P(BatchInfo), P(c_int), P(c_int)]
    lib.tt_kernel_hmat_build.argtypes = [P(Params), vp, i64, c_int, vp, P(vp)]
    lib.tt_kernel_hmat_apply.argtypes = [vp, vp, c_int, vp, i64, vp, i64, vp]
    lib.tt_kernel_hmat_get_info.argtypes = [vp, P(HmatInfo)]
    lib.tt_kernel_hmat_get_lists.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.tt_kernel_hmat_get_batch.argtypes = [vp, P(vp)]
    lib.tt_kernel_hmat_destroy.argtypes = [vp]
    lib.tt_kernel_batch_get_class.argtypes = [vp, c_int, P(vp)]
    lib.tt_kernel_batch_get_factors.argtypes = [vp, c_int, vp, vp, vp]
    lib.tt_kernel_batch_apply.argtypes = [vp, vp, c_int, vp, i64, vp, i64, vp, i64, vp, i64, vp, vp]
    lib.tt_kernel_batch_destroy.argtypes = [vp]
    lib.tt_kernel_eval_entries.argtypes = [P(Params), vp, i64, vp, vp]
    lib.tt_kernel_eval_dense.argtypes = [P(Params), vp, i64, vp, i64, P(ctypes.c_double), vp, i64, vp]
    lib.tt_kernel_get_info.argtypes = [vp, P(Info)]
    lib.tt_kernel_get_factors.argtypes = [vp, vp, vp, vp]
    lib.tt_kernel_get_cores.argtypes = [vp, P(ctypes.c_double), i64]
    lib.tt_kernel_get_coeff_cores.argtypes = [vp, P(ctypes.c_double), i64]
    lib.tt_kernel_get_cross.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int32), P(Decision), c_int]
    lib.tt_kernel_destroy.argtypes = [vp]
    lib.tt_kernel_last_error.argtypes = []
    lib.tt_kernel_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "tt_kernel_last_error":
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


class TTKError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status < 0:
        raise TTKError(status, load().tt_kernel_last_error().decode())
    return status
