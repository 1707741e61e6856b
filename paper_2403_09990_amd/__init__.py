"""PURSE boundary sampling and MEGB on MI355X (gfx950).

Thin Python binding of the C ABI in include/purse.h: the functions below carry
the same names as the C entry points and only marshal torch device tensors into
pointers; every step of the computation runs in the HIP kernels of
libpurse.so.  PyTorch provides device memory and streams.

The library is loaded on first use and its absence is an error.
"""
import ctypes
from typing import Optional

from . import _native
from ._native import (PURSE_FLAG_EXACT_MEB, PURSE_FLAG_FORCE_FP64_POLAR, PURSE_FLAG_FORWARD_TANGENTS,
                      PURSE_FLAG_WORK_QUEUE, PURSE_FLAG_SERIAL_GROUPS, PURSE_FLAG_GENERIC_LOOP, PURSE_FLAG_NO_PRUNING,  # noqa: F401
                      PURSE_FLAG_INSTANCE_ORDER, PURSE_FLAG_MATRIX_COTANGENT, PURSE_FLAG_PAIR_LANES,
                      PURSE_FLAG_QUAD_LANES, PURSE_BWD_BAD_TRACE, PURSE_BWD_EMPTY, PURSE_BWD_NON_FINITE,
                      PURSE_BWD_OK, PURSE_BWD_OVERFLOW, PURSE_BWD_STALE,
                      PURSE_FLAG_REPLAY_DESCENT,
                      PURSE_FLAG_REUSE_PROLOGUE,
                      PURSE_INST_ANCHOR_ITERATED, PURSE_INST_BAD_SHAPE, PURSE_INST_BAD_SIZE,
                      PURSE_INST_EMPTY, PURSE_INST_FIT_FAILED, PURSE_INST_NO_ANCHOR, PURSE_INST_OK,
                      PURSE_MASK_FAILED, PURSE_MASK_FEASIBLE, PURSE_MASK_PULLED_IN, PurseBatch,
                      PurseParams, PurseWalkParams)

__all__ = ["PurseError", "DeviceBatch", "purse_default_params", "purse_workspace_size",
           "purse_sample", "purse_sample_noalloc", "purse_megb", "purse_megb_backward", "purse_walk_default_params", "purse_walk_workspace_size",
           "purse_walk", "purse_init", "init", "sample", "megb", "walk", "workspace"]


class PurseError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _native.load()
        msg = "%s: %s (%d)" % (where, lib.purse_status_string(code).decode(), code)
        detail = lib.purse_last_error().decode()
        if detail:
            msg += ": " + detail
        super().__init__(msg)
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise PurseError(code, where)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class DeviceBatch:
    """A workloads.Batch copied to device tensors in the ABI's layout, with the
    purse_batch struct that points at them."""

    def __init__(self, batch, device="cuda"):
        import torch
        a = batch.arrays()
        self.n_inst = batch.n_inst
        self.kind = torch.as_tensor(a["kind"], dtype=torch.int32, device=device)
        self.n_kp = torch.as_tensor(a["n_kp"], dtype=torch.int32, device=device)
        self.kp_off = torch.as_tensor(a["kp_off"], dtype=torch.int64, device=device)
        self.sample_off = torch.as_tensor(a["sample_off"], dtype=torch.int64, device=device)
        self.model_pts = torch.as_tensor(a["model_pts"], dtype=torch.float32, device=device).contiguous()
        self.centres = torch.as_tensor(a["centres"], dtype=torch.float32, device=device).contiguous()
        self.shapes = torch.as_tensor(a["shapes"], dtype=torch.float32, device=device).contiguous()
        self.bounds = torch.as_tensor(a["bounds"], dtype=torch.float32, device=device).contiguous()
        self.intrinsics = torch.as_tensor(a["intrinsics"], dtype=torch.float32, device=device).contiguous()
        self.seed = torch.as_tensor(a["seed"].view("int64"), dtype=torch.int64, device=device)
        self.total_kp = int(a["kp_off"][-1])
        self.total_samples = int(a["sample_off"][-1])
        self.max_samples = int((a["sample_off"][1:] - a["sample_off"][:-1]).max())
        self.max_kp = int(a["n_kp"].max())
        self.sample_off_host = a["sample_off"]
        self.kp_off_host = a["kp_off"]
        self.struct = PurseBatch(
            n_inst=self.n_inst, max_kp=max(3, self.max_kp), total_kp=self.total_kp,
            total_samples=self.total_samples, max_samples=self.max_samples,
            kind=_ptr(self.kind), n_kp=_ptr(self.n_kp), kp_off=_ptr(self.kp_off),
            sample_off=_ptr(self.sample_off), model_pts=_ptr(self.model_pts),
            centres=_ptr(self.centres), shapes=_ptr(self.shapes), bounds=_ptr(self.bounds),
            intrinsics=_ptr(self.intrinsics), seed=_ptr(self.seed))


def purse_default_params(**overrides) -> PurseParams:
    p = PurseParams()
    _check(_native.load().purse_default_params(ctypes.byref(p)), "purse_default_params")
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def purse_workspace_size(db: DeviceBatch, params: PurseParams) -> int:
    n = ctypes.c_size_t(0)
    _check(_native.load().purse_workspace_size(ctypes.byref(db.struct), ctypes.byref(params),
                                               ctypes.byref(n)), "purse_workspace_size")
    return int(n.value)


def workspace(db: DeviceBatch, params: PurseParams, device="cuda"):
    import torch
    return torch.empty(max(1, purse_workspace_size(db, params)), dtype=torch.uint8, device=device)


def purse_sample(db, params, poses, mask, inst_status, ws, stream=None):
    _check(_native.load().purse_sample(ctypes.byref(db.struct), ctypes.byref(params), _ptr(poses),
                                       _ptr(mask), _ptr(inst_status), _ptr(ws), ws.numel(),
                                       _stream(stream)), "purse_sample")


def purse_sample_noalloc(db, params, poses, mask, inst_status, stream=None):
    _check(_native.load().purse_sample_noalloc(ctypes.byref(db.struct), ctypes.byref(params), _ptr(poses),
                                               _ptr(mask), _ptr(inst_status), _stream(stream)),
           "purse_sample_noalloc")


def purse_megb(db, params, poses, mask, centre, radii, n_feasible, trace, inst_status, ws, stream=None):
    _check(_native.load().purse_megb(ctypes.byref(db.struct), ctypes.byref(params), _ptr(poses),
                                     _ptr(mask), _ptr(centre), _ptr(radii), _ptr(n_feasible),
                                     _ptr(trace), _ptr(inst_status), _ptr(ws), ws.numel(),
                                     _stream(stream)), "purse_megb")


def purse_megb_backward(db, params, poses, mask, trace, g_radii, g_centre, g_centres, g_shapes,
                        g_bounds, ws, stream=None, bwd_status=None):
    _check(_native.load().purse_megb_backward(
        ctypes.byref(db.struct), ctypes.byref(params), _ptr(poses), _ptr(mask), _ptr(trace),
        _ptr(g_radii), _ptr(g_centre), _ptr(g_centres), _ptr(g_shapes), _ptr(g_bounds), _ptr(bwd_status),
        _ptr(ws), ws.numel(), _stream(stream)), "purse_megb_backward")


# ----------------------------------------------------------------------------
# conveniences that allocate outputs with torch and call the entry points

def sample(db: DeviceBatch, params: PurseParams, ws=None, stream=None) -> dict:
    import torch
    dev = db.kind.device
    if ws is None:
        ws = workspace(db, params, dev)
    poses = torch.empty(db.total_samples, 12, dtype=torch.float32, device=dev)
    mask = torch.empty(db.total_samples, dtype=torch.uint8, device=dev)
    status = torch.empty(db.n_inst, dtype=torch.int32, device=dev)
    purse_sample(db, params, poses, mask, status, ws, stream)
    return dict(poses=poses, mask=mask, inst_status=status, ws=ws)


def megb(db: DeviceBatch, params: PurseParams, poses, mask, inst_status, ws=None, stream=None) -> dict:
    import torch
    dev = db.kind.device
    if ws is None:
        ws = workspace(db, params, dev)
    centre = torch.empty(db.n_inst, 12, dtype=torch.float32, device=dev)
    radii = torch.empty(db.n_inst, 2, dtype=torch.float64, device=dev)
    nf = torch.empty(db.n_inst, dtype=torch.int64, device=dev)
    trace = torch.empty(db.n_inst, params.megb_iters, 2, dtype=torch.int32, device=dev)
    purse_megb(db, params, poses, mask, centre, radii, nf, trace, inst_status, ws, stream)
    return dict(centre=centre, radii=radii, n_feasible=nf, trace=trace, inst_status=inst_status)


# ----------------------------------------------------------------------------
# the strategic random walk (second sampler mode)

def purse_walk_default_params(**overrides) -> PurseWalkParams:
    w = PurseWalkParams()
    _check(_native.load().purse_walk_default_params(ctypes.byref(w)), "purse_walk_default_params")
    for k, v in overrides.items():
        if not hasattr(w, k):
            raise KeyError(k)
        setattr(w, k, v)
    return w


def purse_walk_workspace_size(db: DeviceBatch) -> int:
    n = ctypes.c_size_t(0)
    _check(_native.load().purse_walk_workspace_size(ctypes.byref(db.struct), ctypes.byref(n)),
           "purse_walk_workspace_size")
    return int(n.value)


def purse_walk(db, params, wparams, start_off, starts, poses, mask, decisions, ws, stream=None):
    _check(_native.load().purse_walk(ctypes.byref(db.struct), ctypes.byref(params), ctypes.byref(wparams),
                                     _ptr(start_off), _ptr(starts), int(starts.shape[0]), _ptr(poses), _ptr(mask),
                                     _ptr(decisions), _ptr(ws), ws.numel(), _stream(stream)), "purse_walk")


def walk(db: DeviceBatch, params: PurseParams, wparams: PurseWalkParams, start_off, starts, ws=None,
         with_decisions=False, stream=None) -> dict:
    """Allocates the outputs and runs purse_walk: poses (2, W, 12) and mask
    (2, W) for the rotation-mode and translation-mode walks (W = starts x
    n_walks), and the per-iteration decisions if asked."""
    import torch
    dev = db.kind.device
    if ws is None:
        ws = torch.empty(max(1, purse_walk_workspace_size(db)), dtype=torch.uint8, device=dev)
    nw = int(starts.shape[0]) * wparams.n_walks
    poses = torch.empty(2, nw, 12, dtype=torch.float32, device=dev)
    mask = torch.empty(2, nw, dtype=torch.uint8, device=dev)
    dec = torch.empty(2, nw, max(1, wparams.n_iters), dtype=torch.int32, device=dev) if with_decisions else None
    purse_walk(db, params, wparams, start_off, starts, poses, mask, dec, ws, stream)
    return dict(poses=poses, mask=mask, decisions=dec, ws=ws)


# ----------------------------------------------------------------------------
# Step I candidates

def purse_init(db, params, poses, mask, stream=None):
    _check(_native.load().purse_init(ctypes.byref(db.struct), ctypes.byref(params), _ptr(poses), _ptr(mask),
                                     _stream(stream)), "purse_init")


def init(db: DeviceBatch, params: PurseParams, stream=None) -> dict:
    """Allocates the outputs and runs purse_init: one trial per sample slot."""
    import torch
    dev = db.kind.device
    poses = torch.empty(db.total_samples, 12, dtype=torch.float32, device=dev)
    mask = torch.empty(db.total_samples, dtype=torch.uint8, device=dev)
    purse_init(db, params, poses, mask, stream)
    return dict(poses=poses, mask=mask)
