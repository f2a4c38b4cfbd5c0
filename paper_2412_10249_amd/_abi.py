"""ctypes declarations of the libimask C ABI (include/imask.h).

Argument marshalling only: every computation happens in libimask's HIP
kernels.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libimask.so")

MAX_LEVELS = 8
MAX_LOG2F = 7
MAX_TV_INNER = 12

OK, EINVAL, ENOTSUP, EHIP, ESIZE, ENONFINITE = 0, -1, -2, -3, -4, -5
FULL_PAPER, FULL_UNBIASED = 0, 1
REG_TIKHONOV, REG_SMOOTH_TV, REG_TV = 0, 1, 2
RESTRICT, PROLONG, RESTRICT_ADJ, PROJECT, COMPENSATE = 0, 1, 2, 3, 4
BUDGET_ITERS, BUDGET_EPOCHS = 0, 1
SCHEDULE_PARALLEL, SCHEDULE_SEQUENTIAL = 0, 1
DRAW_COMMON, DRAW_INDEPENDENT = 0, 1

EXPORTS = ["imask_workspace_bytes", "imask_phi_floats", "imask_prepare", "imask_project",
           "imask_backproject", "imask_resample", "imask_sketch_apply", "imask_draws",
           "imask_step", "imask_solve", "imask_time_kernel", "imask_constants_scratch_bytes",
           "imask_step_constants", "imask_sigma_thm3", "imask_sigma_balamurugan", "imask_block_draws",
           "imask_backproject_noalloc", "imask_batch_bytes", "imask_batch_prepare", "imask_batch_step",
           "imask_batch_state", "imask_set_tiles", "imask_get_tiles", "imask_batch_step_part",
           "imask_step_timed"]
BATCH_PLAN, BATCH_FORWARD, BATCH_TRANSPOSE, BATCH_ADVANCE = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 48 << 20
KERNEL_FORWARD, KERNEL_TRANSPOSE, KERNEL_TRANSPOSE_SUM = 0, 1, 2


class Geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_det", ctypes.c_int32),
                ("det_spacing", ctypes.c_double), ("det_offset", ctypes.c_double), ("extent", ctypes.c_double),
                ("angles", ctypes.POINTER(ctypes.c_double)), ("src_dist", ctypes.c_double),
                ("det_dist", ctypes.c_double)]


class Levels(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("log2f", ctypes.c_int32 * MAX_LEVELS),
                ("p", ctypes.c_double * MAX_LEVELS), ("full_mode", ctypes.c_int32), ("n_blocks", ctypes.c_int32)]


class Reg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lam", ctypes.c_double), ("tv_weight", ctypes.c_double),
                ("tv_eps", ctypes.c_double), ("tv_inner", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
                ("schedule", ctypes.c_int32), ("theta", ctypes.c_double), ("draw_mode", ctypes.c_int32),
                ("dual_stream_id", ctypes.c_uint32), ("check_finite", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p * 2), ("y", ctypes.c_void_p * 2), ("phi", ctypes.c_void_p),
                ("psi", ctypes.c_void_p), ("work", ctypes.c_void_p), ("k", ctypes.c_uint64),
                ("epochs", ctypes.c_double), ("cur", ctypes.c_int32), ("xbar", ctypes.c_void_p),
                ("tvd", ctypes.c_void_p * 2), ("ztab", ctypes.c_void_p)]


class Tiles(ctypes.Structure):
    _fields_ = [("bp_rows", ctypes.c_int32), ("bp_waves", ctypes.c_int32), ("bp_wg", ctypes.c_int32),
                ("fwd_lds_kb", ctypes.c_int32)]


class ImaskError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImaskError("libimask.so is not built (run __graft_entry__.build() or "
                             "python -m paper_2412_10249_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz, P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER
        L.imask_workspace_bytes.argtypes = [P(Geometry)]
        L.imask_workspace_bytes.restype = sz
        L.imask_phi_floats.argtypes = [P(Geometry), P(Levels)]
        L.imask_phi_floats.restype = sz
        L.imask_prepare.argtypes = [P(Geometry), vp, sz, vp]
        L.imask_project.argtypes = [P(Geometry), i32, vp, vp, vp, vp]
        L.imask_backproject.argtypes = [P(Geometry), i32, vp, vp, vp, vp]
        L.imask_backproject_noalloc.argtypes = [P(Geometry), i32, vp, vp, vp]
        L.imask_resample.argtypes = [i32, i32, i32, P(Levels), vp, vp, vp]
        L.imask_sketch_apply.argtypes = [P(Geometry), P(Levels), i32, i32, vp, vp, vp, vp]
        L.imask_draws.argtypes = [P(Params), P(Levels), ctypes.c_uint64, i32, P(i32)]
        L.imask_block_draws.argtypes = [P(Params), P(Levels), ctypes.c_uint64, i32, P(i32)]
        L.imask_time_kernel.argtypes = [P(Geometry), i32, i32, vp, vp, vp, i32, vp, P(ctypes.c_double)]
        L.imask_constants_scratch_bytes.argtypes = [P(Geometry)]
        L.imask_constants_scratch_bytes.restype = sz
        L.imask_step_constants.argtypes = [P(Geometry), P(Levels), ctypes.c_double, i32, ctypes.c_uint64, vp, vp,
                                           P(ctypes.c_double), vp]
        L.imask_sigma_thm3.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, i32,
                                       P(ctypes.c_double), P(ctypes.c_double)]
        L.imask_sigma_balamurugan.argtypes = [ctypes.c_double, ctypes.c_double, P(ctypes.c_double)]
        L.imask_step.argtypes = [i32, P(Geometry), P(Levels), P(Reg), P(Params), P(vp), P(State), i32, vp]
        L.imask_step_timed.argtypes = [P(Geometry), P(Levels), P(Reg), P(Params), vp, P(State), i32,
                                       P(ctypes.c_float), vp]
        L.imask_solve.argtypes = [i32, P(Geometry), P(Levels), P(Reg), P(Params), P(vp), P(State),
                                  ctypes.c_double, i32, vp]
        L.imask_batch_bytes.argtypes = [i32, P(Geometry), P(Levels)]
        L.imask_batch_bytes.restype = sz
        L.imask_batch_prepare.argtypes = [i32, P(Geometry), P(Levels), P(Reg), P(Params), P(vp), P(State),
                                          ctypes.c_double, i32, vp, sz, P(ctypes.c_int64), vp]
        L.imask_batch_step.argtypes = [i32, P(Geometry), P(Levels), vp, i32, vp]
        L.imask_batch_step_part.argtypes = [i32, P(Geometry), P(Levels), vp, i32, vp]
        L.imask_batch_state.argtypes = [i32, P(Levels), vp, P(State), vp]
        L.imask_set_tiles.argtypes = [i32, i32, i32, P(Tiles)]
        L.imask_get_tiles.argtypes = [i32, i32, i32, P(Tiles)]
        for name in EXPORTS:
            if getattr(L, name).restype is ctypes.c_int:  # default
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc: int, what: str) -> None:
    if rc != OK:
        names = {EINVAL: "EINVAL", ENOTSUP: "ENOTSUP", EHIP: "EHIP", ESIZE: "ESIZE", ENONFINITE: "ENONFINITE"}
        raise ImaskError(f"{what} failed: {names.get(rc, rc)}")
