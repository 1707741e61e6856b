"""Pins of the oracle's Lambda-norm residual, its feasibility test and the
iterated-anchor branch of the prologue against values that geometry fixes,
not against the oracle's own formulas (no GPU).

- eq. unknown-but-bounded: ||g||_Lambda = sqrt(g^T Lambda g).  An ellipse
  Lambda = Q(phi) diag(a^-2, b^-2) Q(phi)^T has semi-axes a and b along the
  columns of Q(phi), so a point s * a * Q e1 (or s * b * Q e2) from the centre
  has norm exactly s.  Values of s other than 1 and bounds beta other than 1
  separate r from r^2 and Lambda from its inverse.
- eq. PURSE with unreachable bounds: a regular tetrahedron inflated by
  (1 + eps) cannot be matched by any rigid pose to within eps (the sum of
  squared residuals is at least 4 eps^2), so with beta < eps the set is empty.
- The prologue's anchor when the centre fit is not inside (Section "The
  CLOSURE Algorithm", Step II: the kept pose must be one still in S): on an
  axis-symmetric 3D-3D instance where only one ball is tight, the alternating
  iteration from the centre fit is a scalar affine recurrence with a closed
  form.
"""
import math

import numpy as np
import pytest
import torch

from oracle.params import OracleParams
from oracle.purse import (FLAG_ANCHOR_ITERATED, FLAG_NO_ANCHOR, KIND_2D3D, KIND_3D3D,
                          MASK_FEASIBLE, Problem, feasible, prologue, residual, sample)

DT = torch.float64
K = np.array([600.0, 600.0, 320.0, 240.0])
# model points on the plane Z = 0 seen by the pose (I, (0, 0, 1)) at depth 1:
# pixel u = (600 X + 320, 600 Y + 240), worked out by hand
MODEL_2D = np.array([[0.10, 0.05, 0.0], [-0.10, 0.05, 0.0], [0.05, -0.10, 0.0],
                     [-0.05, -0.05, 0.0], [0.00, 0.10, 0.0], [0.08, 0.00, 0.0]])
PIXELS_2D = np.array([[380.0, 270.0], [260.0, 270.0], [350.0, 180.0],
                      [290.0, 210.0], [320.0, 300.0], [368.0, 240.0]])
R_ID = torch.eye(3, dtype=DT)[None]
T_DEPTH1 = torch.tensor([[0.0, 0.0, 1.0]], dtype=DT)


def _ellipse(phi, a, b):
    c, s = math.cos(phi), math.sin(phi)
    Q = np.array([[c, -s], [s, c]])
    return Q @ np.diag([a ** -2, b ** -2]) @ Q.T, Q


def _problem_2d(scales, axes, beta):
    """Ellipses whose centres sit so that each predicted pixel is s_i semi-axes
    away along the ellipse's first (axes[i] = 0) or second (1) axis."""
    rng = np.random.default_rng(11)
    shapes, centres = [], []
    for i, (s, ax) in enumerate(zip(scales, axes)):
        phi = rng.uniform(0, math.pi)
        a, b = rng.uniform(5, 20), rng.uniform(5, 20)
        L, Q = _ellipse(phi, a, b)
        step = s * (a * Q[:, 0] if ax == 0 else b * Q[:, 1])
        centres.append(PIXELS_2D[i] - step)
        shapes.append(L.reshape(4))
    return Problem(KIND_2D3D, MODEL_2D, np.array(centres), np.array(shapes),
                   np.full(len(scales), beta), K)


def test_pixels_of_the_construction():
    """The hand-worked pixels are the pinhole images (checked once here so the
    pins below rest on them)."""
    u = 600.0 * MODEL_2D[:, :2] + np.array([320.0, 240.0])
    assert np.allclose(u, PIXELS_2D, atol=1e-12)


@pytest.mark.parametrize("axes", [[0] * 6, [1] * 6, [0, 1, 0, 1, 1, 0]])
def test_lambda_norm_along_the_semi_axes(axes):
    """r_i = s_i exactly for points s_i semi-axes away along either axis."""
    scales = [0.25, 0.5, 1.0, 1.5, 2.0, 0.75]
    prob = _problem_2d(scales, axes, 1.0)
    e, r, depth = residual(prob, R_ID, T_DEPTH1)
    assert np.allclose(r[0].numpy(), scales, rtol=0, atol=1e-12)
    assert np.allclose(depth[0].numpy(), 1.0, atol=1e-15)
    # the residual points from the measured centre to the prediction
    assert np.allclose((prob.centres + e[0]).numpy(), PIXELS_2D, atol=1e-9)


@pytest.mark.parametrize("beta", [0.7, 1.3])
def test_feasibility_with_bounds_other_than_one(beta):
    """in_purse: feasible iff every r_i <= beta + tau.  Points just inside and
    just outside beta (a relative 1% either side, far beyond tau = 1e-4)
    decide it, whichever keypoint is outside; r^2 or Lambda^-1 in place of r or
    Lambda would move the decision."""
    p = OracleParams()
    inside = [0.99 * beta] * 6
    prob = _problem_2d(inside, [0, 1, 0, 1, 0, 1], beta)
    assert bool(feasible(prob, R_ID, T_DEPTH1, p)[0])
    for k in range(6):
        sc = list(inside)
        sc[k] = 1.01 * beta
        prob = _problem_2d(sc, [0, 1, 0, 1, 0, 1], beta)
        assert not bool(feasible(prob, R_ID, T_DEPTH1, p)[0]), k


def test_feasibility_tolerance_and_margin():
    """The tolerance is absolute (beta + tau) and the prologue's margin scales
    beta only (margin beta + tau)."""
    p = OracleParams()
    beta = 0.5
    prob = _problem_2d([beta + 0.5 * p.tau_abs_2d] * 6, [0] * 6, beta)
    assert bool(feasible(prob, R_ID, T_DEPTH1, p)[0])
    prob = _problem_2d([beta + 2.0 * p.tau_abs_2d] * 6, [0] * 6, beta)
    assert not bool(feasible(prob, R_ID, T_DEPTH1, p)[0])
    prob = _problem_2d([0.9 * beta] * 6, [1] * 6, beta)
    assert bool(feasible(prob, R_ID, T_DEPTH1, p, margin=0.95)[0])
    assert not bool(feasible(prob, R_ID, T_DEPTH1, p, margin=0.85)[0])


def test_depth_decides_feasibility():
    """A keypoint at or behind z_min is infeasible whatever its pixel."""
    p = OracleParams()
    prob = _problem_2d([0.1] * 6, [0] * 6, 1.0)
    t = torch.tensor([[0.0, 0.0, 0.5 * p.z_min]], dtype=DT)
    assert not bool(feasible(prob, R_ID, t, p)[0])


def test_3d_residual_is_the_euclidean_distance():
    """3D-3D: Lambda = I, r_i = ||R a_i + t - b_i||; with beta other than 1 a
    point at 0.6 beta is inside and one at 1.2 beta is not (r^2 would keep
    both inside for beta = 0.05)."""
    rng = np.random.default_rng(5)
    a = rng.uniform(-1, 1, size=(5, 3))
    d = rng.normal(size=(5, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    beta = 0.05
    dist = np.array([0.6, 0.3, 0.9, 0.1, 0.5]) * beta
    prob = Problem(KIND_3D3D, a, a + dist[:, None] * d, np.tile([1.0, 0, 0, 1.0], (5, 1)),
                   np.full(5, beta), np.zeros(4))
    p = OracleParams()
    e, r, _ = residual(prob, R_ID, torch.zeros(1, 3, dtype=DT))
    assert np.allclose(r[0].numpy(), dist, atol=1e-15)
    assert bool(feasible(prob, R_ID, torch.zeros(1, 3, dtype=DT), p)[0])
    dist[2] = 1.2 * beta
    prob.centres = torch.as_tensor(a + dist[:, None] * d)
    assert not bool(feasible(prob, R_ID, torch.zeros(1, 3, dtype=DT), p)[0])


def _tetrahedron():
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    return v / math.sqrt(3.0)


def test_empty_set_has_no_anchor_and_no_sample():
    """A regular tetrahedron inflated by 1 + eps: for any rigid pose, the sum
    over the four vertices of ||R a_i + t - (1 + eps) a_i||^2 is at least
    4 eps^2 (the vertices sum to zero and ||R a_i|| = 1), so some residual is
    at least eps and beta = eps / 2 leaves S empty.  The prologue finds no
    anchor and no trajectory ends feasible (a dropped square root, r^2 =
    eps^2 < beta, would admit the centre fit)."""
    eps = 0.1
    a = _tetrahedron()
    prob = Problem(KIND_3D3D, a, (1 + eps) * a, np.tile([1.0, 0, 0, 1.0], (4, 1)),
                   np.full(4, 0.5 * eps), np.zeros(4))
    p = OracleParams(n_iters=30)
    pro = prologue(prob, p)
    assert pro["status"] & FLAG_ANCHOR_ITERATED
    assert pro["status"] & FLAG_NO_ANCHOR
    # the centre fit is the identity (the inflation is symmetric)
    assert float((pro["R_c"] - torch.eye(3, dtype=DT)).abs().max()) < 1e-12
    assert float(pro["t_c"].abs().max()) < 1e-12
    out = sample(prob, p, 3, 64, pro=pro)
    assert int((out["mask"] & MASK_FEASIBLE).sum()) == 0


def test_iterated_anchor_closed_form():
    """Six model points at +-e_x, +-e_y, +-e_z; every ball centred on its
    point except b_1 = a_1 + delta e_x, whose ball (radius beta_1) is the only
    tight one.  The centre fit is (I, delta/6 e_x), which leaves keypoint 1 at
    5 delta / 6 > kappa beta_1, so the anchor is iterated.  Each iteration
    clamps keypoint 1 to q_1 = a_1 + (delta - kappa beta_1) e_x and leaves the
    others unclamped; the refit then has H = 2 I + c e_x e_x^T (a rotation of
    I) and translation t_{k+1} = (5 t_k + delta - kappa beta_1) / 6, so
    t_n = t* + (t_0 - t*) (5/6)^n with t* = delta - kappa beta_1 and t_0 =
    delta / 6.  The anchor is (I, t_n e_x) after n_iters iterations."""
    delta, beta1 = 0.1, 0.02
    a = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
    b = a.copy()
    b[0, 0] += delta
    beta = np.array([beta1, 0.5, 0.5, 0.5, 0.5, 0.5])
    prob = Problem(KIND_3D3D, a, b, np.tile([1.0, 0, 0, 1.0], (6, 1)), beta, np.zeros(4))
    p = OracleParams(n_iters=60)
    pro = prologue(prob, p)
    assert pro["status"] & FLAG_ANCHOR_ITERATED
    assert not pro["status"] & FLAG_NO_ANCHOR
    assert np.allclose(pro["t_c"].numpy(), [delta / 6, 0, 0], atol=1e-15)
    ts = delta - p.kappa * beta1
    tn = ts + (delta / 6 - ts) * (5.0 / 6.0) ** p.n_iters
    assert float((pro["R_a"] - torch.eye(3, dtype=DT)).abs().max()) < 1e-12
    assert np.allclose(pro["t_a"].numpy(), [tn, 0, 0], rtol=0, atol=1e-13)
    # fewer iterations leave keypoint 1 outside the shrunk ball by more than
    # tau (though inside the unshrunk one, with 45 iterations): then there is
    # no anchor, the test of the iterated end using the margin kappa as the
    # test of the centre fit does
    for n in (5, 45):
        p_short = OracleParams(n_iters=n)
        tn = ts + (delta / 6 - ts) * (5.0 / 6.0) ** n
        assert (delta - tn) > p_short.kappa * beta1 + p_short.tau_abs_3d
        if n == 45:
            assert (delta - tn) < beta1 + p_short.tau_abs_3d
        pro_n = prologue(prob, p_short)
        assert pro_n["status"] & FLAG_NO_ANCHOR, n
