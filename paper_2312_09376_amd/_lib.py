"""ctypes loader for librbt.so: the C ABI of include/rbt.h, nothing else.

The library is loaded from this package directory. There is no fallback:
if it is missing, load() raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbt.so")

RBT_ERR_HIP = -100
RBT_ERR_WORKSPACE = -101
RBT_ERR_UNSUPPORTED = -102
RBT_ERR_SYNC = -103
RBT_MAX_DEPTH = 16
RBT_NOALLOC_SCRATCH_MB = 96
RBT_FP64, RBT_FP32, RBT_BF16 = 0, 1, 2
RBT_OP_T, RBT_OP_N = 0, 1
RBT_IR_CLASSIC, RBT_IR_GMRES = 0, 1

i64, i32, u64, dbl, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
vp = ctypes.c_void_p

# name -> (restype, argtypes); keep in the order of include/rbt.h
SIGNATURES = {
    "rbt_version": (i32, []),
    "rbt_structure": (i32, [i64, i32, vp]),
    "rbt_reference_size": (i64, [i64, i32, i64]),
    "rbt_comm_free_granule": (i64, [i64, i64, i64]),
    "rbt_structure_ex": (i32, [i64, i32, i64, vp]),
    "rbt_generate": (i32, [i64, i32, u64, vp, vp]),
    "rbt_generate_rotations": (i32, [i64, i32, u64, i64, vp, vp]),
    "rbt_generate_device": (i32, [i64, i32, u64, vp, vp, vp]),
    "rbt_transform2": (i32, [i64, vp, i64, vp, i64, i32, vp, vp, i32, vp]),
    "rbt_transform_vec": (i32, [i64, i64, vp, i64, vp, i32, i32, vp]),
    "rbt_workspace_size": (sz, [i64, i64, i32, i32]),
    "rbt_genp": (i32, [i64, vp, i64, vp, vp]),
    "rbt_getrs": (i32, [i64, i64, vp, i64, vp, i64, i32, vp, sz, vp]),
    "rbt_solve_ex": (i32, [i64, i64, vp, i64, vp, i64, i32, u64, vp, vp, sz, vp]),
    "rbt_solve_ex_noalloc": (i32, [i64, i64, vp, i64, vp, i64, i32, u64, vp, vp]),
    "rbt_solve": (i32, [i64, i64, vp, i64, vp, i64, i32, u64, vp]),
    "rbt_solve_refine": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, i32, u64, dbl, i32,
                               vp, vp, vp, vp, sz, vp]),
    "rbt_solve_mixed": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, i32, u64, i32, i32,
                              dbl, i32, vp, vp, vp, vp, sz, vp]),
    "rbt_solve_mixed_guarded": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64, i32,
                                      u64, i32, i32, dbl, i32, i32, vp, vp, vp, vp, vp, sz, vp]),
    "rbt_gepp": (i32, [i64, vp, i64, vp, vp, vp, sz, vp]),
    "rbt_gepp_solve": (i32, [i64, i64, vp, i64, vp, vp, i64, vp, sz, vp]),
    "rbt_solve_guarded": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, i32, u64, dbl, i32,
                                vp, vp, vp, vp, vp, sz, vp]),
    "rbt_batched_workspace_size": (sz, [i64, vp, vp, i32, i32]),
    "rbt_batched_plan": (i32, [i64, vp, vp, i32, i32, vp, sz, vp]),
    "rbt_solve_batched": (i32, [i64, vp, vp, vp, vp, vp, vp, i32, u64, i32, dbl, i32, vp, vp, vp,
                                vp, vp, sz, vp]),
    "rbt_backward_error": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, vp, vp, sz, vp]),
    "rbt_solve_backward": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64, i32, u64,
                                 vp, sz, vp]),
    "rbt_solve_backward_mixed": (i32, [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                                       i64, i32, u64, dbl, i32, vp, vp, vp, sz, vp]),
    "rbt_set_option": (i32, [i32, i64]),
    "rbt_get_option": (i64, [i32]),
    "rbt_timing_enable": (i32, [i32]),
    "rbt_timing_read": (i32, [i32, vp, vp, vp]),
}
RBT_STAGE_COUNT = 10
RBT_OPT_OUTER_NB = 1
RBT_OPT_BATCH_TILE_COLS = 2
RBT_OPT_BATCH_WGS_PER_CU = 3
RBT_OPT_LOOKAHEAD = 4
RBT_OPT_BF16_STAGED = 5
RBT_OPT_SWEEP_SPIN_LIMIT = 6
RBT_OPT_MIXED_FP64_INNER = 7
RBT_OPT_GRANULE = 8
RBT_OPT_BUTTERFLY = 9
RBT_OPT_SIDES = 10
RBT_OPT_CAPTURABLE = 11
RBT_OPT_BATCH_TILE_COLS2_MIN_N = 12
RBT_OPT_TIMING_STAGES = 13
RBT_OPT_PANEL_SPLIT = 14
STAGES = ["generate", "transform2", "transform_vec", "diag", "panel", "trailing", "solve",
          "residual", "pivoted", "outer"]

_lib = None


class RBTError(RuntimeError):
    pass


def load(path=None):
    """Load librbt.so and declare every exported symbol's signature."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RBTError(f"librbt.so not built at {p}: run `python -m paper_2312_09376_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(rc, name):
    if rc != 0:
        what = {RBT_ERR_HIP: "HIP runtime error", RBT_ERR_WORKSPACE: "workspace too small",
                RBT_ERR_UNSUPPORTED: "unsupported configuration",
                RBT_ERR_SYNC: "a triangular sweep's bounded wait expired (result is NaN)"}.get(
                    rc, f"invalid argument {-rc}")
        raise RBTError(f"{name} failed ({rc}): {what}")
