"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same float32 inputs, and compare them."""
import dataclasses
import math

import numpy as np
import torch

from oracle.megb import megb as oracle_megb_fn
from oracle.params import OracleParams
from oracle.purse import Problem, sample as oracle_sample

ROT_TOL = 1e-4      # rad, per sample
TRANS_TOL = 1e-4    # m (3D-3D) or m (2D-3D translation), per sample
RADIUS_RTOL = 1e-3  # MEGB radii, relative
CENTRE_TOL = 1e-4   # MEGB centre, rad and m


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def as_f32_instance(inst):
    """The instance as the device sees it: every float rounded to float32."""
    return dataclasses.replace(inst, model_pts=f32(inst.model_pts), centres=f32(inst.centres),
                               shapes=f32(inst.shapes), bounds=f32(inst.bounds),
                               intrinsics=f32(inst.intrinsics))


def oracle_params(gp) -> OracleParams:
    """The oracle's parameters with the same (float32) values the device uses."""
    return OracleParams(n_iters=gp.n_iters, n_gn=gp.n_gn, n_bis=gp.n_bis,
                        megb_iters=gp.megb_iters, megb_avg=gp.megb_avg,
                        omega0=float(np.float32(gp.omega0)), v0=float(np.float32(gp.v0)),
                        kappa=float(np.float32(gp.kappa)),
                        tau_abs_3d=float(np.float32(gp.tau_abs_3d)),
                        tau_abs_2d=float(np.float32(gp.tau_abs_2d)),
                        z_min=float(np.float32(gp.z_min)), centre_gn=gp.centre_gn)


def run_gpu(batch, params, with_megb=True):
    import paper_2403_09990_amd as P
    db = P.DeviceBatch(batch)
    ws = P.workspace(db, params)
    out = P.sample(db, params, ws=ws)
    res = dict(db=db, ws=ws, poses=out["poses"], mask=out["mask"], inst_status=out["inst_status"])
    if with_megb:
        m = P.megb(db, params, out["poses"], out["mask"], out["inst_status"], ws=ws)
        res.update(m)
    torch.cuda.synchronize()
    return res


def rot_angle(Ra, Rb):
    """2 asin(||Ra - Rb||_F / (2 sqrt 2)), elementwise over (M,3,3)."""
    f = np.sqrt(((Ra - Rb) ** 2).sum((-1, -2)))
    return 2 * np.arcsin(np.minimum(1.0, f / (2 * math.sqrt(2))))


# A decision (a final in_purse test or a bisection step) counts as a hazard
# when the oracle's ratio max_i r_i / (beta_i + tau) is within this band of 1.
# Float32 poses differ from the float64 ones by a few 1e-6 rad (measured),
# which moves a 2D-3D residual by up to f * 3e-6 / a = 600 * 3e-6 / 5 = 4e-4
# of an ellipse's semi-axis a; the band stays below the 1e-3 gap the shrink
# factor kappa = 0.999 leaves between converged trajectories (ratio about
# kappa) and the boundary, so a converged sample never counts as a hazard.
HAZARD_BAND = 5e-4


def compare_samples(gpu_poses, gpu_mask, ora_poses, ora_mask, end_margin=None, bis_margin=None,
                    max_flip_frac=0.0):
    """Per-sample agreement.  Returns stats; asserts the bar: every mask equal
    and every pose within ROT_TOL / TRANS_TOL, except where the oracle shows a
    decision hazard (end_margin / bis_margin within HAZARD_BAND): a mask
    mismatch needs a hazardous final test, a pose outside tolerance a
    hazardous final test or bisection step.  Without margins (two GPU runs
    compared) at most max_flip_frac of the samples may differ."""
    gp = np.asarray(gpu_poses, dtype=np.float64)
    op = np.asarray(ora_poses, dtype=np.float64)
    gm = np.asarray(gpu_mask).astype(np.int64)
    om = np.asarray(ora_mask).astype(np.int64)
    same = gm == om
    ang = rot_angle(gp[:, :9].reshape(-1, 3, 3), op[:, :9].reshape(-1, 3, 3))
    dt = np.linalg.norm(gp[:, 9:] - op[:, 9:], axis=1)
    bad = same & ((ang > ROT_TOL) | (dt > TRANS_TOL))
    stats = dict(n=len(gm), mask_flips=int((~same).sum()), pose_out=int(bad.sum()),
                 max_rot=float(ang[same].max()) if same.any() else 0.0,
                 max_trans=float(dt[same].max()) if same.any() else 0.0,
                 median_rot=float(np.median(ang[same])) if same.any() else 0.0,
                 pulled=int(((om & 2) != 0).sum()))
    n = len(gm)
    if end_margin is None:
        allowed = int(max_flip_frac * n)
        assert stats["mask_flips"] <= allowed, stats
        assert stats["pose_out"] <= allowed, stats
        return stats
    em = np.asarray(end_margin, dtype=np.float64)
    bm = np.full(n, np.inf) if bis_margin is None else np.asarray(bis_margin, dtype=np.float64)
    end_hz = em <= HAZARD_BAND
    bis_hz = bm <= HAZARD_BAND
    flip_bad = ~same & ~end_hz
    out_bad = bad & ~(end_hz | bis_hz)
    stats.update(hazard_end=int(end_hz.sum()), hazard_bis=int(bis_hz.sum()),
                 forgiven=int((~same | bad).sum() - flip_bad.sum() - out_bad.sum()),
                 min_end_margin=float(em.min()) if n else float("inf"))
    assert not flip_bad.any(), dict(stats, ids=np.nonzero(flip_bad)[0][:10].tolist())
    assert not out_bad.any(), dict(stats, ids=np.nonzero(out_bad)[0][:10].tolist(),
                                   rot=ang[out_bad][:10].tolist(), trans=dt[out_bad][:10].tolist())
    return stats


def compare_with_oracle(gpu_poses, gpu_mask, ora):
    """compare_samples against an oracle result computed with diagnostics."""
    return compare_samples(gpu_poses, gpu_mask, ora["poses"].numpy(), ora["mask"].numpy(),
                           ora.get("end_margin"), ora.get("bis_margin"))


def oracle_for_instance(inst, gp, sample_ids):
    prob = Problem.from_instance(as_f32_instance(inst))
    ora = oracle_sample(prob, oracle_params(gp), inst.seed, len(sample_ids), sample_ids=sample_ids,
                        diagnostics=True)
    if "end_margin" not in ora:  # an instance the prologue rejects: no trajectory ran
        ora["end_margin"] = torch.full((len(sample_ids),), float("inf"), dtype=torch.float64)
        ora["bis_margin"] = torch.full((len(sample_ids),), float("inf"), dtype=torch.float64)
    return ora


def oracle_megb(poses, mask, T, avg):
    P = torch.as_tensor(np.asarray(poses, dtype=np.float64))
    sel = torch.nonzero(torch.as_tensor((np.asarray(mask) & 1) != 0))[:, 0]
    R = P[sel, :9].reshape(-1, 3, 3)
    t = P[sel, 9:]
    return oracle_megb_fn(R, t, sel, T, avg)
