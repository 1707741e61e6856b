"""Pins of the oracle's sampler: properties the paper's set definition and the
method's construction fix (no GPU)."""
import dataclasses

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import so3
from oracle.params import OracleParams
from oracle.purse import (MASK_FEASIBLE, MASK_PULLED_IN, STATUS_BAD_SHAPE,
                          STATUS_BAD_SIZE, Problem, feasible, initial_poses,
                          prologue, residual, sample, transform)
from oracle.megb import megb_from_poses
from paper_2403_09990_amd import workloads as W

DT = torch.float64


def _pose(out):
    P = out["poses"]
    return P[:, :9].reshape(-1, 3, 3), P[:, 9:]


def _zero_radius(inst):
    """Noise-free centres and beta = 0: the set is the single true pose."""
    prob = Problem.from_instance(inst)
    P = transform(prob, torch.as_tensor(inst.R_gt)[None], torch.as_tensor(inst.t_gt)[None])[0]
    if prob.kind == 0:
        prob.centres = P.clone()
    else:
        fx, fy, cx, cy = inst.intrinsics
        prob.centres = torch.stack([fx * P[:, 0] / P[:, 2] + cx, fy * P[:, 1] / P[:, 2] + cy], 1)
    prob.beta = torch.zeros_like(prob.beta)
    return prob


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_zero_radius_collapse(cfg):
    """eq. PURSE with beta_i = 0 and exact measurements: S = {x_gt} (unique for
    3D-3D with >= 3 non-collinear points and for generic 2D-3D with >= 6), so
    every feasible sample is x_gt and both MEGB radii are 0."""
    b = W.config_c1(0) if cfg == "c1" else W.config_c2(0, n_samples=256)
    inst = b.instances[0]
    prob = _zero_radius(inst)
    p = OracleParams(n_iters=30)
    out = sample(prob, p, inst.seed, 256)
    assert bool((out["mask"] & MASK_FEASIBLE).all())
    R, t = _pose(out)
    Rg = torch.as_tensor(inst.R_gt)
    assert float(so3.angle(R, Rg).max()) < 1e-9
    assert float((t - torch.as_tensor(inst.t_gt)).abs().max()) < 1e-9
    mg = megb_from_poses(out["poses"], out["mask"], 64, 10)
    assert mg["D"] < 1e-8 and mg["d"] < 1e-9


@pytest.mark.parametrize("cfg,iters", [("c1", 50), ("c1", 8), ("c2", 100), ("c2", 12)])
def test_every_kept_sample_is_in_the_set(cfg, iters):
    """Every mask-1 sample satisfies every constraint of eq. PURSE (with the
    feasibility tolerance), including samples pulled back by bisection (few
    iterations force many pull-ins)."""
    b = W.config_c1(1) if cfg == "c1" else W.config_c2(1, n_samples=512)
    inst = b.instances[0]
    prob = Problem.from_instance(inst)
    p = OracleParams(n_iters=iters)
    out = sample(prob, p, inst.seed, 512)
    m = out["mask"]
    R, t = _pose(out)
    keep = (m & MASK_FEASIBLE) != 0
    assert bool(keep.all())
    assert bool(feasible(prob, R, t, p).all())
    if iters < 20:
        assert int(((m & MASK_PULLED_IN) != 0).sum()) > 50


def test_pull_in_lands_on_the_boundary():
    """Bisection keeps the feasible end: x(lo) is in S and x(lo + 2^-n_bis) is
    not, so pulled-in samples sit on the boundary of S within the bisection
    resolution."""
    inst = W.config_c2(2, n_samples=256).instances[0]
    prob = Problem.from_instance(inst)
    p = OracleParams(n_iters=10)
    out = sample(prob, p, inst.seed, 256)
    pulled = torch.nonzero((out["mask"] & MASK_PULLED_IN) != 0)[:, 0]
    assert len(pulled) > 20
    R, t = _pose(out)
    e, r, _ = residual(prob, R[pulled], t[pulled])
    ratio = ((r - p.tau_abs_2d) / prob.beta).max(1).values
    assert float(ratio.max()) <= 1.0 + 1e-12
    assert float(ratio.min()) > 0.99


def test_initial_offsets():
    """Even trajectories rotate the object about its own centroid by omega0
    (the centroid stays put); odd ones shift it by v0 without rotating."""
    inst = W.config_c1(3).instances[0]
    prob = Problem.from_instance(inst)
    p = OracleParams()
    pro = prologue(prob, p)
    ids = np.arange(400)
    R0, t0 = initial_poses(pro, p, inst.seed, ids)
    cen = R0 @ prob.model.mean(0) + t0
    even = torch.as_tensor(ids % 2 == 0)
    ang = so3.angle(R0, pro["R_c"])
    assert float((ang[even] - p.omega0).abs().max()) < 1e-12
    assert float((cen[even] - pro["o_c"]).abs().max()) < 1e-12
    assert float(ang[~even].max()) < 1e-12
    sh = torch.linalg.norm(cen[~even] - pro["o_c"], dim=1)
    assert float((sh - p.v0).abs().max()) < 1e-12
    # directions are uniform on the sphere: mean ~ 0, second moment ~ I/3
    d = (cen[~even] - pro["o_c"]) / p.v0
    u = torch.cat([so3.log_so3(R0[even] @ pro["R_c"].T) / p.omega0, d])
    assert float(u.mean(0).abs().max()) < 0.1
    np.testing.assert_allclose((u.T @ u / len(u)).numpy(), np.eye(3) / 3, atol=0.06)


def test_interior_starts_are_fixed_points():
    """With no offset every trajectory starts at x_c; when x_c is strictly
    inside the kappa-shrunk set the projection leaves every keypoint where it
    is and the refit returns the same pose."""
    for b in (W.config_c1(4), W.config_c2(4, n_samples=16)):
        inst = b.instances[0]
        prob = Problem.from_instance(inst)
        p = OracleParams(n_iters=5, omega0=0.0, v0=0.0)
        pro = prologue(prob, p)
        assert pro["status"] == 0  # x_c itself is the anchor
        out = sample(prob, p, inst.seed, 16, pro=pro)
        R, t = _pose(out)
        assert float(so3.angle(R, pro["R_c"]).max()) < 1e-10
        assert float((t - pro["t_c"]).abs().max()) < 1e-10


def _transform_model(inst, H, h):
    return dataclasses.replace(inst, model_pts=inst.model_pts @ H.T + h)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_model_frame_equivariance(cfg):
    """Replacing the model points m_i by H m_i + h maps every sample x_s to
    (R_s H^T, t_s - R_s H^T h); D_hat is invariant and d_hat too when h = 0."""
    b = W.config_c1(5) if cfg == "c1" else W.config_c2(5, n_samples=128)
    inst = b.instances[0]
    H = Rotation.from_rotvec([0.3, -0.8, 0.5]).as_matrix()
    h = np.array([0.05, -0.02, 0.04])
    p = OracleParams(n_iters=40)
    o1 = sample(Problem.from_instance(inst), p, inst.seed, 128)
    o2 = sample(Problem.from_instance(_transform_model(inst, H, h)), p, inst.seed, 128)
    R1, t1 = _pose(o1)
    R2, t2 = _pose(o2)
    Ht = torch.as_tensor(H)
    tol = 1e-9 if cfg == "c1" else 1e-7   # DLT is not equivariant; GN removes it
    assert float(so3.angle(R2, R1 @ Ht.T).max()) < tol
    assert float((t2 - (t1 - torch.einsum("mij,j->mi", R1 @ Ht.T, torch.as_tensor(h)))).abs().max()) < tol
    assert torch.equal(o1["mask"], o2["mask"])
    m1 = megb_from_poses(o1["poses"], o1["mask"], 256, 10)
    m2 = megb_from_poses(o2["poses"], o2["mask"], 256, 10)
    assert abs(m1["D"] - m2["D"]) < 1e-6
    o3 = sample(Problem.from_instance(_transform_model(inst, H, 0 * h)), p, inst.seed, 128)
    m3 = megb_from_poses(o3["poses"], o3["mask"], 256, 10)
    assert abs(m1["d"] - m3["d"]) < 1e-6


def test_split_sample_ranges_reproduce():
    """Counter-based randomness: [0, M) equals [0, M/2) followed by [M/2, M)
    (to rounding: torch's batched CPU kernels may round differently for
    different batch sizes)."""
    inst = W.config_c2(6, n_samples=64).instances[0]
    prob = Problem.from_instance(inst)
    p = OracleParams(n_iters=20)
    full = sample(prob, p, inst.seed, 64)
    a = sample(prob, p, inst.seed, 32, sample_ids=np.arange(32))
    b = sample(prob, p, inst.seed, 32, sample_ids=np.arange(32, 64))
    assert float((full["poses"] - torch.cat([a["poses"], b["poses"]])).abs().max()) < 1e-12
    assert torch.equal(full["mask"], torch.cat([a["mask"], b["mask"]]))


def test_bad_instances_are_flagged():
    inst = W.config_c2(7, n_samples=8).instances[0]
    p = OracleParams(n_iters=2)
    bad = dataclasses.replace(inst, shapes=inst.shapes * np.array([1, 1, 1, -1.0]))
    assert prologue(Problem.from_instance(bad), p)["status"] == STATUS_BAD_SHAPE
    small = dataclasses.replace(inst, model_pts=inst.model_pts[:5], centres=inst.centres[:5],
                                shapes=inst.shapes[:5], bounds=inst.bounds[:5])
    assert prologue(Problem.from_instance(small), p)["status"] == STATUS_BAD_SIZE
    neg = dataclasses.replace(inst, bounds=-inst.bounds)
    out = sample(Problem.from_instance(neg), p, inst.seed, 8)
    assert out["status"] == STATUS_BAD_SHAPE and int(out["mask"].sum()) == 0
