"""torch.autograd.Function around purse_sample + purse_megb and
purse_megb_backward: the MEGB centre and radii as differentiable functions of
the ellipse / ball centres, shape matrices and bounds.  Marshalling only;
both passes run in the HIP library."""
import copy

import torch

from . import DeviceBatch, PurseBatch, PurseParams, megb, purse_megb_backward, sample, workspace
from ._native import PURSE_FLAG_MATRIX_COTANGENT


def _bound(db: DeviceBatch, centres, shapes, bounds) -> DeviceBatch:
    """A view of db whose measurements are this call's (detached, float32)
    centres, shapes and bounds, with its own purse_batch struct.  The caller's
    db is left untouched, so every forward keeps the batch its backward must
    see, however many forwards run on db before it."""
    out = copy.copy(db)
    out.centres = centres.detach().to(torch.float32).contiguous()
    out.shapes = shapes.detach().to(torch.float32).contiguous()
    out.bounds = bounds.detach().to(torch.float32).contiguous()
    s = db.struct
    out.struct = PurseBatch(
        n_inst=s.n_inst, max_kp=s.max_kp, total_kp=s.total_kp, total_samples=s.total_samples,
        max_samples=s.max_samples, kind=s.kind, n_kp=s.n_kp, kp_off=s.kp_off, sample_off=s.sample_off,
        model_pts=s.model_pts, centres=out.centres.data_ptr(), shapes=out.shapes.data_ptr(),
        bounds=out.bounds.data_ptr(), intrinsics=s.intrinsics, seed=s.seed)
    return out


class PurseMEGB(torch.autograd.Function):
    """centre (n_inst,12) float32 [R row-major | t] and radii (n_inst,2) float64
    of the MEGB of the PURSE boundary samples."""

    @staticmethod
    def forward(ctx, centres, shapes, bounds, db, params):
        db = _bound(db, centres, shapes, bounds)
        ws = workspace(db, params)
        out = sample(db, params, ws=ws)
        mg = megb(db, params, out["poses"], out["mask"], out["inst_status"], ws=ws)
        ctx.db, ctx.params, ctx.ws = db, PurseParams.from_buffer_copy(params), ws
        ctx.save_for_backward(out["poses"], out["mask"], mg["trace"])
        ctx.mark_non_differentiable(mg["trace"])
        return mg["centre"], mg["radii"]

    @staticmethod
    def backward(ctx, g_centre_out, g_radii):
        poses, mask, trace = ctx.saved_tensors
        db = ctx.db
        n = db.n_inst
        dev = poses.device
        if g_centre_out is None:
            g_centre_out = torch.zeros(n, 12, dtype=torch.float32, device=dev)
        if g_radii is None:
            g_radii = torch.zeros(n, 2, dtype=torch.float64, device=dev)
        # the centre's cotangent as given (12 entries per instance); the library
        # takes its rotation part along SO(3)
        g_c = g_centre_out.to(torch.float32).contiguous()
        params = PurseParams.from_buffer_copy(ctx.params)
        params.flags |= PURSE_FLAG_MATRIX_COTANGENT
        g_centres = torch.empty(db.total_kp, 3, dtype=torch.float32, device=dev)
        g_shapes = torch.empty(db.total_kp, 4, dtype=torch.float32, device=dev)
        g_bounds = torch.empty(db.total_kp, dtype=torch.float32, device=dev)
        purse_megb_backward(db, params, poses, mask, trace, g_radii.double().contiguous(), g_c,
                            g_centres, g_shapes, g_bounds, ctx.ws)
        return g_centres, g_shapes, g_bounds, None, None
