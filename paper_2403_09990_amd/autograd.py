"""torch.autograd.Function around purse_sample + purse_megb and
purse_megb_backward: the MEGB centre and radii as differentiable functions of
the ellipse / ball centres, shape matrices and bounds.  Marshalling only;
both passes run in the HIP library."""
import torch

from . import DeviceBatch, PurseBatch, megb, purse_megb_backward, sample, workspace
from ._native import PurseBatch as _PB  # noqa: F401


def _rebind(db: DeviceBatch, centres, shapes, bounds):
    db.centres = centres.detach().to(torch.float32).contiguous()
    db.shapes = shapes.detach().to(torch.float32).contiguous()
    db.bounds = bounds.detach().to(torch.float32).contiguous()
    s = db.struct
    db.struct = PurseBatch(
        n_inst=s.n_inst, max_kp=s.max_kp, total_kp=s.total_kp, total_samples=s.total_samples,
        max_samples=s.max_samples, kind=s.kind, n_kp=s.n_kp, kp_off=s.kp_off, sample_off=s.sample_off,
        model_pts=s.model_pts, centres=db.centres.data_ptr(), shapes=db.shapes.data_ptr(),
        bounds=db.bounds.data_ptr(), intrinsics=s.intrinsics, seed=s.seed)


def left_cotangent(Rstar, G):
    """Matrix cotangent G of R* (n,3,3) -> left so(3) cotangent v(G R*^T)."""
    X = G @ Rstar.transpose(-1, -2)
    return torch.stack([X[..., 2, 1] - X[..., 1, 2], X[..., 0, 2] - X[..., 2, 0],
                        X[..., 1, 0] - X[..., 0, 1]], -1)


class PurseMEGB(torch.autograd.Function):
    """centre (n_inst,12) float32 [R row-major | t] and radii (n_inst,2) float64
    of the MEGB of the PURSE boundary samples."""

    @staticmethod
    def forward(ctx, centres, shapes, bounds, db, params):
        _rebind(db, centres, shapes, bounds)
        ws = workspace(db, params)
        out = sample(db, params, ws=ws)
        mg = megb(db, params, out["poses"], out["mask"], out["inst_status"], ws=ws)
        ctx.db, ctx.params, ctx.ws = db, params, ws
        ctx.save_for_backward(out["poses"], out["mask"], mg["trace"], mg["centre"])
        ctx.mark_non_differentiable(mg["trace"])
        return mg["centre"], mg["radii"]

    @staticmethod
    def backward(ctx, g_centre_out, g_radii):
        poses, mask, trace, centre = ctx.saved_tensors
        db = ctx.db
        n = db.n_inst
        dev = poses.device
        if g_centre_out is None:
            g_centre_out = torch.zeros(n, 12, dtype=torch.float32, device=dev)
        if g_radii is None:
            g_radii = torch.zeros(n, 2, dtype=torch.float64, device=dev)
        R = centre[:, :9].reshape(n, 3, 3).double()
        gw = left_cotangent(R, g_centre_out[:, :9].reshape(n, 3, 3).double())
        g_c = torch.cat([gw, g_centre_out[:, 9:].double()], 1).to(torch.float32).contiguous()
        g_centres = torch.empty(db.total_kp, 3, dtype=torch.float32, device=dev)
        g_shapes = torch.empty(db.total_kp, 4, dtype=torch.float32, device=dev)
        g_bounds = torch.empty(db.total_kp, dtype=torch.float32, device=dev)
        purse_megb_backward(db, ctx.params, poses, mask, trace, g_radii.double().contiguous(), g_c,
                            g_centres, g_shapes, g_bounds, ctx.ws)
        return g_centres, g_shapes, g_bounds, None, None
