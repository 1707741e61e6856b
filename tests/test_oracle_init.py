"""Pins of the oracle's Step I samplers (oracle/ransag.py: RANSAG with Arun's
method and with P3P; oracle/reg.py: the pose-regression set and its
convex-combination sampler) against what geometry fixes (no GPU)."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import ransag, reg
from oracle.params import OracleParams
from oracle.purse import KIND_3D3D, Problem
from paper_2403_09990_amd import workloads as W

DT = torch.float64


def test_pick_three_distinct_and_uniform():
    idx = ransag.pick_three(5, np.arange(6000), 7)
    assert idx.min() >= 0 and idx.max() < 7
    assert all(len(set(r)) == 3 for r in idx.tolist())
    counts = np.bincount(idx.ravel(), minlength=7)
    assert np.abs(counts / counts.sum() - 1 / 7).max() < 0.02


def test_points_inside_their_constraints():
    d = ransag.ball_points(3, np.arange(2000), 1)
    assert (np.linalg.norm(d, axis=1) <= 1 + 1e-12).all()
    assert np.abs(d.mean(0)).max() < 0.05
    rng = np.random.default_rng(0)
    L = []
    for _ in range(50):
        phi = rng.uniform(0, math.pi)
        Q = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
        L.append(Q @ np.diag(rng.uniform(5, 20, 2) ** -2.0) @ Q.T)
    L = np.array(L)
    beta = rng.uniform(0.5, 2.0, 50)
    e = ransag.ellipse_points(4, np.arange(50), 2, L, beta)
    r = np.sqrt(np.einsum("ti,tij,tj->t", e, L, e))
    assert (r <= beta * (1 + 1e-12)).all()


def _exact_3d(rng, n):
    inst = W.make_3d3d(rng, n, 0.01, 0.05, 8)
    b = inst.model_pts @ inst.R_gt.T + inst.t_gt
    prob = Problem(KIND_3D3D, inst.model_pts, b, inst.shapes, np.zeros(n), np.zeros(4))
    return inst, prob


def test_ransag_3d_on_exact_data_returns_the_true_pose():
    """beta = 0: the random points are the ball centres, which the true pose
    maps the model points onto; Arun's method on any three recovers it, and
    it is in S."""
    rng = np.random.default_rng(1)
    inst, prob = _exact_3d(rng, 9)
    poses, mask, idx = ransag.ransag_3d(prob, OracleParams(), 11, 40)
    R = poses[:, :9].reshape(-1, 3, 3).numpy()
    assert np.abs(R - inst.R_gt).max() < 1e-10
    assert np.abs(poses[:, 9:].numpy() - inst.t_gt).max() < 1e-10
    assert bool((mask == 1).all())


def _project(inst, X):
    fx, fy, cx, cy = inst.intrinsics
    return np.stack([fx * X[:, 0] / X[:, 2] + cx, fy * X[:, 1] / X[:, 2] + cy], 1)


@pytest.mark.parametrize("seed", [2, 3, 4, 5])
def test_p3p_recovers_the_true_pose_and_reprojects_exactly(seed):
    """Noise-free projections of three model points: one P3P solution is the
    true pose (the problem is ill-conditioned for a 0.2 m object at 1 m, hence
    1e-5), and every solution maps the three model points onto their rays."""
    rng = np.random.default_rng(seed)
    inst = W.make_2d3d(rng, 8, 2.0, (5.0, 20.0), 8)
    prob = Problem.from_instance(inst)
    Pc = inst.model_pts @ inst.R_gt.T + inst.t_gt
    pix = _project(inst, Pc)
    sols = ransag.p3p(ransag.bearings(prob, pix[:3]), inst.model_pts[:3])
    assert 1 <= len(sols) <= 4
    err = [max(np.abs(R.numpy() - inst.R_gt).max(), np.abs(t.numpy() - inst.t_gt).max()) for _, R, t in sols]
    assert min(err) < 1e-5
    for v, R, t in sols:
        X = inst.model_pts[:3] @ R.numpy().T + t.numpy()
        assert (X[:, 2] > 0).all()
        assert np.abs(_project(inst, X) - pix[:3]).max() < 1e-5
    assert [s[0] for s in sols] == sorted(s[0] for s in sols)


def test_ransag_2d_keeps_a_pose_in_s():
    rng = np.random.default_rng(6)
    inst = W.make_2d3d(rng, 10, 2.0, (5.0, 20.0), 8)
    prob = Problem.from_instance(inst)
    p = OracleParams()
    poses, mask, idx, sols, pix = ransag.ransag_2d(prob, p, 21, 300)
    assert int(mask.sum()) > 0
    from oracle.purse import feasible
    keep = mask == 1
    R = poses[keep, :9].reshape(-1, 3, 3)
    assert bool(feasible(prob, R, poses[keep, 9:], p).all())
    # the kept pose is the first in-S solution of its trial
    for r in np.nonzero(keep.numpy())[0][:20]:
        first = next(s for s in sols[r] if s[3])
        assert torch.equal(poses[r, :9].reshape(3, 3), first[1])


def _reg_problem(rng, n, spread_R=0.05, spread_t=0.01):
    R0 = Rotation.random(random_state=rng.integers(1 << 30)).as_matrix()
    t0 = rng.normal(size=3)
    Ri = np.stack([Rotation.from_rotvec(rng.normal(size=3) * spread_R).as_matrix() @ R0 for _ in range(n)])
    ti = t0 + rng.normal(size=(n, 3)) * spread_t
    return reg.RegProblem(torch.as_tensor(Ri), torch.as_tensor(ti), torch.full((n,), 0.3, dtype=DT),
                          torch.full((n,), 0.05, dtype=DT))


def test_reg_residuals_are_chordal_distances():
    """||R - R_i||_F = 2 sqrt(2) sin(theta / 2) for rotations theta apart."""
    rng = np.random.default_rng(7)
    prob = _reg_problem(rng, 5)
    R = torch.as_tensor(Rotation.random(random_state=3).as_matrix())[None]
    t = torch.zeros(1, 3, dtype=DT)
    rR, rt = reg.residuals(prob, R, t)
    th = Rotation.from_matrix(prob.R_i.numpy() @ R[0].numpy().T).magnitude()
    assert np.abs(rR[0].numpy() - 2 * math.sqrt(2) * np.sin(th / 2)).max() < 1e-12
    assert np.abs(rt[0].numpy() - np.linalg.norm(prob.t_i.numpy(), axis=1)).max() < 1e-12


def test_convex_samples():
    """Weights on the simplex; equal hypotheses give that pose exactly; two
    hypotheses give translations on their segment."""
    w = reg.convex_weights(9, np.arange(500), 10).numpy()
    assert (w >= 0).all() and np.abs(w.sum(1) - 1).max() < 1e-14
    assert np.abs(w.mean(0) - 0.1).max() < 0.01
    rng = np.random.default_rng(8)
    prob = _reg_problem(rng, 6, 0.0, 0.0)
    poses, mask = reg.convex_samples(prob, 5, 50, 1e-5)
    assert np.abs(poses[:, :9].numpy() - prob.R_i[0].numpy().ravel()).max() < 1e-12
    assert np.abs(poses[:, 9:].numpy() - prob.t_i[0].numpy()).max() < 1e-12
    assert bool((mask == 1).all())
    prob = _reg_problem(rng, 2)
    poses, mask = reg.convex_samples(prob, 6, 50, 1e-5)
    a, b = prob.t_i[0].numpy(), prob.t_i[1].numpy()
    lam = (poses[:, 9:].numpy() - a) @ (b - a) / ((b - a) @ (b - a))
    assert np.abs(a + lam[:, None] * (b - a) - poses[:, 9:].numpy()).max() < 1e-12
    assert (lam >= -1e-12).all() and (lam <= 1 + 1e-12).all()
