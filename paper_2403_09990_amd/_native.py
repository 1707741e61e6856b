"""ctypes view of the C ABI declared in include/purse.h."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpurse.so")

PURSE_OK = 0
PURSE_E_NULL = -1
PURSE_E_BAD_ARG = -2
PURSE_E_WORKSPACE = -3
PURSE_E_NO_DEVICE = -4
PURSE_E_HIP = -5

PURSE_INST_OK = 0
PURSE_INST_EMPTY = 1
PURSE_INST_BAD_SHAPE = 2
PURSE_INST_FIT_FAILED = 3
PURSE_INST_BAD_SIZE = 4
PURSE_INST_NO_ANCHOR = 1 << 8
PURSE_INST_ANCHOR_ITERATED = 1 << 9

PURSE_BWD_OK = 0
PURSE_BWD_EMPTY = 1
PURSE_BWD_OVERFLOW = 2
PURSE_BWD_BAD_TRACE = 3
PURSE_BWD_STALE = 4
PURSE_BWD_NON_FINITE = 5

PURSE_MASK_FEASIBLE = 1
PURSE_MASK_PULLED_IN = 2
PURSE_MASK_FAILED = 4

PURSE_KIND_3D3D = 0
PURSE_KIND_2D3D = 1
PURSE_KIND_REG = 2

PURSE_FLAG_FORCE_FP64_POLAR = 1
PURSE_FLAG_NO_PRUNING = 2
PURSE_FLAG_REUSE_PROLOGUE = 4
PURSE_FLAG_INSTANCE_ORDER = 8
PURSE_FLAG_GENERIC_LOOP = 16
PURSE_FLAG_PAIR_LANES = 32
PURSE_FLAG_REPLAY_DESCENT = 64
PURSE_FLAG_QUAD_LANES = 128
PURSE_FLAG_MATRIX_COTANGENT = 256
PURSE_FLAG_EXACT_MEB = 512
PURSE_FLAG_FORWARD_TANGENTS = 1024
PURSE_FLAG_WORK_QUEUE = 2048
PURSE_FLAG_SERIAL_GROUPS = 4096

EXPORTED = ("purse_default_params", "purse_workspace_size", "purse_sample", "purse_sample_noalloc",
            "purse_megb", "purse_megb_backward", "purse_walk_default_params", "purse_walk_workspace_size",
            "purse_walk", "purse_init", "purse_status_string", "purse_last_error")


class PurseBatch(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int32),
        ("max_kp", ctypes.c_int32),
        ("total_kp", ctypes.c_int64),
        ("total_samples", ctypes.c_int64),
        ("max_samples", ctypes.c_int64),
        ("kind", ctypes.c_void_p),
        ("n_kp", ctypes.c_void_p),
        ("kp_off", ctypes.c_void_p),
        ("sample_off", ctypes.c_void_p),
        ("model_pts", ctypes.c_void_p),
        ("centres", ctypes.c_void_p),
        ("shapes", ctypes.c_void_p),
        ("bounds", ctypes.c_void_p),
        ("intrinsics", ctypes.c_void_p),
        ("seed", ctypes.c_void_p),
    ]


class PurseParams(ctypes.Structure):
    _fields_ = [
        ("n_iters", ctypes.c_int32),
        ("n_gn", ctypes.c_int32),
        ("n_bis", ctypes.c_int32),
        ("megb_iters", ctypes.c_int32),
        ("megb_avg", ctypes.c_int32),
        ("omega0", ctypes.c_float),
        ("v0", ctypes.c_float),
        ("kappa", ctypes.c_float),
        ("tau_abs_3d", ctypes.c_float),
        ("tau_abs_2d", ctypes.c_float),
        ("z_min", ctypes.c_float),
        ("ckpt_every", ctypes.c_int32),
        ("centre_gn", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("waves_per_simd", ctypes.c_int32),
    ]


class PurseWalkParams(ctypes.Structure):
    _fields_ = [
        ("n_walks", ctypes.c_int32),
        ("n_iters", ctypes.c_int32),
        ("n_perturb", ctypes.c_int32),
        ("n_keep", ctypes.c_int32),
        ("n_scales", ctypes.c_int32),
        ("gamma", ctypes.c_float),
        ("omega0", ctypes.c_float),
        ("v0", ctypes.c_float),
        ("t_pert", ctypes.c_float),
        ("r_pert", ctypes.c_float),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpurse.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpurse.so is not built (run __graft_entry__.build() or "
                           "python -m paper_2403_09990_amd.build): %s" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.purse_default_params.argtypes = [P(PurseParams)]
    lib.purse_workspace_size.argtypes = [P(PurseBatch), P(PurseParams), P(ctypes.c_size_t)]
    lib.purse_sample.argtypes = [P(PurseBatch), P(PurseParams), vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.purse_sample_noalloc.argtypes = [P(PurseBatch), P(PurseParams), vp, vp, vp, vp]
    lib.purse_megb.argtypes = [P(PurseBatch), P(PurseParams), vp, vp, vp, vp, vp, vp, vp, vp,
                               ctypes.c_size_t, vp]
    lib.purse_megb_backward.argtypes = [P(PurseBatch), P(PurseParams), vp, vp, vp, vp, vp, vp, vp, vp,
                                        vp, vp, ctypes.c_size_t, vp]
    lib.purse_init.argtypes = [P(PurseBatch), P(PurseParams), vp, vp, vp]
    lib.purse_walk_default_params.argtypes = [P(PurseWalkParams)]
    lib.purse_walk_workspace_size.argtypes = [P(PurseBatch), P(ctypes.c_size_t)]
    lib.purse_walk.argtypes = [P(PurseBatch), P(PurseParams), P(PurseWalkParams), vp, vp, ctypes.c_int64, vp, vp,
                               vp, vp, ctypes.c_size_t, vp]
    for f in ("purse_default_params", "purse_workspace_size", "purse_sample", "purse_sample_noalloc",
              "purse_megb", "purse_megb_backward", "purse_walk_default_params", "purse_walk_workspace_size",
              "purse_walk", "purse_init"):
        getattr(lib, f).restype = ctypes.c_int32
    lib.purse_status_string.argtypes = [ctypes.c_int32]
    lib.purse_status_string.restype = ctypes.c_char_p
    lib.purse_last_error.argtypes = []
    lib.purse_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib
