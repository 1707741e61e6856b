"""Pins of the oracle's building blocks against independent implementations
and closed forms (no GPU)."""
import math

import numpy as np
import pytest
import scipy.optimize
import torch
from scipy.spatial.transform import Rotation

from oracle import philox, so3
from oracle.params import OracleParams
from oracle.purse import (KIND_2D3D, Problem, centre_fit, dlt_2d, gn_step_2d,
                          kabsch, transform)
from paper_2403_09990_amd import workloads as W

DT = torch.float64


# --------------------------------------------------------------------------- Philox

def test_philox_matches_numpy():
    """numpy's Philox (a C implementation of the same published generator)
    advances its counter before producing a block, so its first block for
    counter c is ours for c + 1."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, size=2)]
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4)]
        g = np.random.Philox(counter=np.array(ctr, np.uint64), key=np.array(key, np.uint64))
        ref = g.random_raw(4)
        c1 = list(ctr)
        c1[0] += 1
        out = philox.philox4x64_10([np.uint64(c) for c in c1], [np.uint64(k) for k in key])
        assert [int(o) for o in out] == [int(r) for r in ref]


def test_philox_vectorised_equals_scalar():
    ids = np.arange(1000, dtype=np.uint64)
    z = np.zeros_like(ids)
    vec = philox.philox4x64_10((ids, z, z, z), (np.uint64(99), np.uint64(0)))
    for s in (0, 1, 517, 999):
        sc = philox.philox4x64_10((np.uint64(s), np.uint64(0), np.uint64(0), np.uint64(0)),
                                  (np.uint64(99), np.uint64(0)))
        assert [int(v[s]) for v in vec] == [int(x) for x in sc]


def test_uniforms_are_24bit_and_uniform():
    u1, u2 = philox.trajectory_uniforms(12345, np.arange(200000))
    for u in (u1, u2):
        assert np.all(u >= 0) and np.all(u < 1)
        assert np.all(u * 2**24 == np.floor(u * 2**24))
        assert abs(u.mean() - 0.5) < 3e-3
        assert abs(u.var() - 1 / 12) < 2e-3
    assert abs(np.corrcoef(u1, u2)[0, 1]) < 0.01


# --------------------------------------------------------------------------- SO(3)

def test_exp_log_against_scipy():
    rng = np.random.default_rng(0)
    w = rng.normal(size=(200, 3)) * rng.uniform(0, 3.0, size=(200, 1))
    w = np.concatenate([w, rng.normal(size=(20, 3)) * 1e-7])
    R = so3.exp_so3(torch.as_tensor(w)).numpy()
    np.testing.assert_allclose(R, Rotation.from_rotvec(w).as_matrix(), atol=1e-12)
    back = so3.log_so3(torch.as_tensor(R)).numpy()
    np.testing.assert_allclose(back, Rotation.from_matrix(R).as_rotvec(), atol=1e-10)


def test_angle_matches_arccos_and_scipy():
    rng = np.random.default_rng(1)
    A = Rotation.random(100, random_state=2).as_matrix()
    B = Rotation.random(100, random_state=3).as_matrix()
    got = so3.angle(torch.as_tensor(A), torch.as_tensor(B)).numpy()
    ref = (Rotation.from_matrix(A).inv() * Rotation.from_matrix(B)).magnitude()
    np.testing.assert_allclose(got, ref, atol=1e-10)
    tr = np.einsum("nij,nij->n", A, B)
    np.testing.assert_allclose(got, np.arccos(np.clip((tr - 1) / 2, -1, 1)), atol=1e-7)
    del rng


def test_proj_so3_is_nearest_rotation():
    rng = np.random.default_rng(4)
    for _ in range(50):
        M = rng.normal(size=(3, 3))
        R = so3.proj_so3(torch.as_tensor(M)).numpy()
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1) < 1e-12
        # maximises tr(R^T M) over SO(3): compare with many random rotations
        Q = Rotation.random(2000, random_state=int(rng.integers(1 << 30))).as_matrix()
        assert np.einsum("ij,ij", R, M) >= np.einsum("nij,ij->n", Q, M).max() - 1e-12
        # and against a local optimum found by Nelder-Mead
        f = lambda w: -np.einsum("ij,ij", R @ Rotation.from_rotvec(w).as_matrix(), M)  # noqa: E731
        res = scipy.optimize.minimize(f, np.zeros(3), method="Nelder-Mead",
                                      options=dict(xatol=1e-10, fatol=1e-14))
        assert -res.fun <= np.einsum("ij,ij", R, M) + 1e-9


def test_cosine_rule_on_so3():
    """Cosine rule on SO(3) (appendix "Geodesic Gradient Descent", lemma
    "Cosine rule in SO(3)"): with A3 = I, A1 = Exp(x), A2 = Exp(y),
    cos(a3/2) = cos(a1/2)cos(a2/2) + sin(a1/2)sin(a2/2)cos(angle between x, y)."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        x = rng.normal(size=3) * 0.8
        y = rng.normal(size=3) * 0.8
        A1 = so3.exp_so3(torch.as_tensor(x))
        A2 = so3.exp_so3(torch.as_tensor(y))
        a1, a2 = np.linalg.norm(x), np.linalg.norm(y)
        a3 = float(so3.angle(A1, A2))
        cosang = x @ y / (a1 * a2)
        lhs = math.cos(a3 / 2)
        rhs = math.cos(a1 / 2) * math.cos(a2 / 2) + math.sin(a1 / 2) * math.sin(a2 / 2) * cosang
        assert abs(lhs - rhs) < 1e-12


def _d2(C, s, x):
    return float(so3.angle(C @ so3.exp_so3(torch.as_tensor(x)), s)) ** 2


def test_gradient_and_hessian_of_squared_distance():
    """Derivatives of dist^2(C Exp(x), s) at x = 0, (w, gamma) the axis-angle
    of C^T s (appendix "Geodesic Gradient Descent").  The gradient is
    -2 gamma w: the printed eq. gradientdsquare drops the factor 2 that its own
    derivation (grad a3 = -w, grad a3^2 = 2 a3 grad a3) and the Hessian line
    keep.  The Hessian has eigenvalue 2 along w and gamma cot(gamma/2) across."""
    rng = np.random.default_rng(6)
    h = 1e-5
    for _ in range(20):
        C = torch.as_tensor(Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix())
        rel = rng.normal(size=3)
        rel *= rng.uniform(0.1, 2.5) / np.linalg.norm(rel)
        s = C @ so3.exp_so3(torch.as_tensor(rel))
        gamma = np.linalg.norm(rel)
        w = rel / gamma
        g = np.array([(_d2(C, s, h * e) - _d2(C, s, -h * e)) / (2 * h) for e in np.eye(3)])
        np.testing.assert_allclose(g, -2 * gamma * w, atol=1e-6)
        H = np.zeros((3, 3))
        for i, ei in enumerate(np.eye(3)):
            for j, ej in enumerate(np.eye(3)):
                H[i, j] = (_d2(C, s, h * (ei + ej)) - _d2(C, s, h * (ei - ej))
                           - _d2(C, s, h * (ej - ei)) + _d2(C, s, -h * (ei + ej))) / (4 * h * h)
        Href = 2 * np.outer(w, w) + gamma / math.tan(gamma / 2) * (np.eye(3) - np.outer(w, w))
        np.testing.assert_allclose(H, Href, atol=2e-3)


# --------------------------------------------------------------------------- refits

def test_kabsch_against_scipy_align_vectors():
    rng = np.random.default_rng(8)
    for _ in range(20):
        n = int(rng.integers(3, 30))
        a = rng.uniform(-1, 1, size=(n, 3))
        q = a @ Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix().T \
            + rng.normal(size=3) + rng.normal(scale=0.1, size=(n, 3))
        R, t = kabsch(torch.as_tensor(a), torch.as_tensor(q)[None])
        Rs, _ = Rotation.align_vectors(q - q.mean(0), a - a.mean(0))
        np.testing.assert_allclose(R[0].numpy(), Rs.as_matrix(), atol=1e-10)
        np.testing.assert_allclose(t[0].numpy(), q.mean(0) - Rs.as_matrix() @ a.mean(0), atol=1e-10)


def test_kabsch_reflection_case():
    """Targets that are a mirror image: the fit must still be a rotation and
    beat every other rotation in least squares."""
    rng = np.random.default_rng(9)
    a = rng.uniform(-1, 1, size=(10, 3))
    q = a * np.array([1, 1, -1])
    R, t = kabsch(torch.as_tensor(a), torch.as_tensor(q)[None])
    R = R[0].numpy()
    assert abs(np.linalg.det(R) - 1) < 1e-12
    cost = ((a @ R.T + t[0].numpy() - q) ** 2).sum()
    for Q in Rotation.random(500, random_state=1).as_matrix():
        tt = q.mean(0) - Q @ a.mean(0)
        assert cost <= ((a @ Q.T + tt - q) ** 2).sum() + 1e-9


def _whitened_residual(prob, x):
    R = Rotation.from_rotvec(x[:3]).as_matrix()
    t = x[3:]
    P = prob.model.numpy() @ R.T + t
    fx, fy, cx, cy = prob.K.numpy()
    u = np.stack([fx * P[:, 0] / P[:, 2] + cx, fy * P[:, 1] / P[:, 2] + cy], 1)
    out = []
    for i in range(prob.n):
        L = np.linalg.cholesky(prob.shapes[i].numpy())
        out.append(L.T @ (u[i] - prob.centres[i].numpy()))
    return np.concatenate(out)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_centre_fit_2d_against_scipy_least_squares(seed):
    inst = W.config_c2(seed, n_samples=1).instances[0]
    prob = Problem.from_instance(inst)
    R, t, ok = centre_fit(prob, OracleParams())
    assert ok
    x0 = np.concatenate([Rotation.from_matrix(inst.R_gt).as_rotvec(), inst.t_gt])
    res = scipy.optimize.least_squares(lambda x: _whitened_residual(prob, x), x0,
                                       xtol=1e-15, ftol=1e-15, gtol=1e-15)
    Rs = Rotation.from_rotvec(res.x[:3]).as_matrix()
    np.testing.assert_allclose(R.numpy(), Rs, atol=1e-8)
    np.testing.assert_allclose(t.numpy(), res.x[3:], atol=1e-8)


def test_dlt_exact_on_noise_free_data():
    inst = W.config_c2(3, n_samples=1).instances[0]
    prob = Problem.from_instance(inst)
    P = transform(prob, torch.as_tensor(inst.R_gt)[None], torch.as_tensor(inst.t_gt)[None])[0]
    fx, fy, cx, cy = inst.intrinsics
    prob.centres = torch.stack([fx * P[:, 0] / P[:, 2] + cx, fy * P[:, 1] / P[:, 2] + cy], 1)
    R, t = dlt_2d(prob)
    np.testing.assert_allclose(R.numpy(), inst.R_gt, atol=1e-9)
    np.testing.assert_allclose(t.numpy(), inst.t_gt, atol=1e-9)


def test_gn_step_reaches_exact_targets():
    """Targets that are exact projections of a nearby pose: GN converges to that
    pose (quadratically), which pins the Jacobian and the update's sign."""
    inst = W.config_c2(4, n_samples=1).instances[0]
    prob = Problem.from_instance(inst)
    assert prob.kind == KIND_2D3D
    Rt = torch.as_tensor(inst.R_gt)[None]
    tt = torch.as_tensor(inst.t_gt)[None]
    from oracle.purse import project
    q = project(prob, transform(prob, Rt, tt))
    R = so3.exp_so3(torch.tensor([[0.05, -0.03, 0.02]], dtype=DT)) @ Rt
    t = tt + torch.tensor([[0.01, -0.02, 0.03]], dtype=DT)
    o = torch.tensor([[0.0, 0.0, 1.0]], dtype=DT)
    errs = []
    for _ in range(6):
        R, t, ok = gn_step_2d(prob, R, t, q, o, 1e-3)
        assert bool(ok.all())
        errs.append(float(so3.angle(R, Rt)) + float(torch.linalg.norm(t - tt)))
    assert errs[-1] < 1e-12
    assert errs[2] < errs[1] ** 1.5  # superlinear
