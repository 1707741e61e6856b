"""Seeded synthetic PURSE workloads (inputs only).

This module produces problem instances: model keypoints, measured centres,
shape matrices, bounds, intrinsics and per-instance Philox keys.  It holds
none of the sampler's or the MEGB's arithmetic; it only synthesises
measurements with the generative models of the paper's two keypoint examples
(2D-3D reprojection residual and 3D-3D Euclidean residual, Section 1,
Examples 1 and 2) and the bounded-noise model (eq. "unknown-but-bounded").

The real datasets the paper evaluates on (LM-O for 2D-3D, 3DMatch for 3D-3D)
are not available; the generators below stand in for them with the shapes,
sizes and noise levels of those workloads.  Ground truth is made feasible by
redrawing each keypoint's noise until its Lambda-norm is at most 0.9 beta, the
role conformal calibration plays in the paper (the true pose lies in the set
with high probability).

Everything is numpy float64 on the host; the device ABI takes float32 copies.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

KIND_3D3D = 0
KIND_2D3D = 1


@dataclasses.dataclass
class Instance:
    kind: int
    model_pts: np.ndarray      # (N,3) a_i or Z_i, metres
    centres: np.ndarray        # (N,3) b_i (m) | (z_i.x, z_i.y, 0) (px)
    shapes: np.ndarray         # (N,4) Lambda_i row-major 2x2 (2D-3D); identity marker for 3D-3D
    bounds: np.ndarray         # (N,)  beta_i
    intrinsics: np.ndarray     # (4,)  fx, fy, cx, cy (2D-3D), zeros for 3D-3D
    seed: int                  # Philox key word 0 for this instance
    n_samples: int
    R_gt: np.ndarray           # (3,3) ground-truth rotation (for checks only)
    t_gt: np.ndarray           # (3,)

    @property
    def n_kp(self) -> int:
        return int(self.model_pts.shape[0])


@dataclasses.dataclass
class Batch:
    """Ragged batch in the layout the C ABI expects (host copies)."""
    instances: List[Instance]

    @property
    def n_inst(self) -> int:
        return len(self.instances)

    def arrays(self):
        ins = self.instances
        n = len(ins)
        kind = np.array([i.kind for i in ins], dtype=np.int32)
        n_kp = np.array([i.n_kp for i in ins], dtype=np.int32)
        kp_off = np.zeros(n + 1, dtype=np.int64)
        kp_off[1:] = np.cumsum(n_kp)
        ms = np.array([i.n_samples for i in ins], dtype=np.int64)
        sample_off = np.zeros(n + 1, dtype=np.int64)
        sample_off[1:] = np.cumsum(ms)
        model = np.concatenate([i.model_pts for i in ins]).astype(np.float64)
        centres = np.concatenate([i.centres for i in ins]).astype(np.float64)
        shapes = np.concatenate([i.shapes for i in ins]).astype(np.float64)
        bounds = np.concatenate([i.bounds for i in ins]).astype(np.float64)
        intr = np.stack([i.intrinsics for i in ins]).astype(np.float64)
        seed = np.array([i.seed for i in ins], dtype=np.uint64)
        return dict(kind=kind, n_kp=n_kp, kp_off=kp_off, sample_off=sample_off,
                    model_pts=model, centres=centres, shapes=shapes,
                    bounds=bounds, intrinsics=intr, seed=seed)


def haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation from a uniform unit quaternion
    (Shoemake's subgroup algorithm)."""
    u1, u2, u3 = rng.random(3)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    w, x, y, z = (a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _seed64(rng: np.random.Generator) -> int:
    return int(rng.integers(0, 2**63 - 1, dtype=np.int64))


def make_3d3d(rng: np.random.Generator, n_kp: int = 8, sigma: float = 0.01,
              radius=0.05, n_samples: int = 1024) -> Instance:
    """Point-cloud registration instance (Example 2, eq. PURSE3D3D with
    Lambda_i = I): a_i ~ U[-1,1]^3, Haar rotation, t ~ N(0, I3),
    b_i = R a_i + t + n_i, n_i ~ N(0, sigma^2 I) redrawn until
    ||n_i|| <= 0.9 beta_i.  `radius` is a scalar or a (lo, hi) range drawn
    per keypoint."""
    a = rng.uniform(-1.0, 1.0, size=(n_kp, 3))
    R = haar_rotation(rng)
    t = rng.normal(0.0, 1.0, size=3)
    if np.isscalar(radius):
        beta = np.full(n_kp, float(radius))
    else:
        beta = rng.uniform(radius[0], radius[1], size=n_kp)
    noise = np.empty((n_kp, 3))
    for i in range(n_kp):
        while True:
            n = rng.normal(0.0, sigma, size=3)
            if np.linalg.norm(n) <= 0.9 * beta[i]:
                break
        noise[i] = n
    b = a @ R.T + t + noise
    shapes = np.tile(np.array([1.0, 0.0, 0.0, 1.0]), (n_kp, 1))
    return Instance(KIND_3D3D, a, b, shapes, beta, np.zeros(4), _seed64(rng),
                    n_samples, R, t)


def make_2d3d(rng: np.random.Generator, n_kp: int = 12, sigma_px: float = 2.0,
              semi_axes=(5.0, 20.0), n_samples: int = 65536,
              K=(600.0, 600.0, 320.0, 240.0)) -> Instance:
    """Object pose instance (Example 1, eq. PURSE2D3D): Z_i ~ U[-0.1,0.1]^3
    (a 0.2 m cube), Haar rotation, t = (U[-.05,.05], U[-.05,.05], U[0.9,1.1]),
    pinhole K; ellipse i has Lambda_i = Q(phi) diag(a^-2, b^-2) Q(phi)^T with
    phi ~ U[0,pi), semi-axes a, b ~ U[semi_axes], beta_i = 1; the ellipse centre
    is the true projection plus N(0, sigma_px^2 I) pixel noise, redrawn until
    its Lambda-norm is <= 0.9."""
    fx, fy, cx, cy = K
    Z = rng.uniform(-0.1, 0.1, size=(n_kp, 3))
    R = haar_rotation(rng)
    t = np.array([rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05),
                  rng.uniform(0.9, 1.1)])
    P = Z @ R.T + t
    proj = np.stack([fx * P[:, 0] / P[:, 2] + cx, fy * P[:, 1] / P[:, 2] + cy], 1)
    shapes = np.empty((n_kp, 4))
    centres = np.zeros((n_kp, 3))
    for i in range(n_kp):
        phi = rng.uniform(0.0, np.pi)
        sa, sb = rng.uniform(semi_axes[0], semi_axes[1], size=2)
        Q = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
        Lam = Q @ np.diag([sa ** -2, sb ** -2]) @ Q.T
        Lam = 0.5 * (Lam + Lam.T)
        shapes[i] = Lam.reshape(-1)
        while True:
            n = rng.normal(0.0, sigma_px, size=2)
            if np.sqrt(n @ Lam @ n) <= 0.9:
                break
        centres[i, :2] = proj[i] + n
    beta = np.ones(n_kp)
    return Instance(KIND_2D3D, Z, centres, shapes, beta, np.array(K, float),
                    _seed64(rng), n_samples, R, t)


KIND_REG = 2


def _quat_of(R: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z), w >= 0, of a rotation matrix."""
    from scipy.spatial.transform import Rotation
    q = Rotation.from_matrix(R).as_quat()          # (x, y, z, w)
    q = np.array([q[3], q[0], q[1], q[2]])
    return q if q[0] >= 0 else -q


def make_reg(rng: np.random.Generator, n_hyp: int = 10, sigma_rot: float = 0.05,
             sigma_t: float = 0.01, n_samples: int = 1500) -> Instance:
    """Pose-regression instance (Example 3, eq. PURSEregression with
    Frobenius and Euclidean balls), shaped like the top pose hypotheses of a
    regression network: a Haar rotation and t = (U[-.05,.05], U[-.05,.05],
    U[0.9,1.1]); hypothesis i has R_i = Exp(w_i) R, w_i ~ N(0, sigma_rot^2 I)
    and t_i = t + N(0, sigma_t^2 I); its bounds are beta_i^R = 2 sqrt(2)
    sin(theta_i / 2), theta_i ~ U[2, 4] sigma_rot, and beta_i^t ~ U[2, 4]
    sigma_t, each hypothesis redrawn until the true pose lies within 0.9 of
    both bounds.  Keypoint i of the batch arrays is hypothesis i: centres =
    t_i, shapes = the quaternion of R_i, model_pts[:, 0] = beta^R, bounds =
    beta^t."""
    from scipy.spatial.transform import Rotation
    R = haar_rotation(rng)
    t = np.array([rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), rng.uniform(0.9, 1.1)])
    model = np.zeros((n_hyp, 3))
    centres = np.zeros((n_hyp, 3))
    shapes = np.zeros((n_hyp, 4))
    beta = np.zeros(n_hyp)
    for i in range(n_hyp):
        th = rng.uniform(2.0, 4.0) * sigma_rot
        bR = 2.0 * np.sqrt(2.0) * np.sin(th / 2.0)
        bt = rng.uniform(2.0, 4.0) * sigma_t
        while True:
            Ri = Rotation.from_rotvec(rng.normal(0.0, sigma_rot, size=3)).as_matrix() @ R
            ti = t + rng.normal(0.0, sigma_t, size=3)
            if np.linalg.norm(R - Ri) <= 0.9 * bR and np.linalg.norm(t - ti) <= 0.9 * bt:
                break
        model[i, 0] = bR
        centres[i] = ti
        shapes[i] = _quat_of(Ri)
        beta[i] = bt
    return Instance(KIND_REG, model, centres, shapes, beta, np.zeros(4), _seed64(rng), n_samples, R, t)


# ---------------------------------------------------------------------------
# The five workloads.  Each takes a seed; instances are reproducible.

def config_c1(seed: int = 0, n_samples: int = 1024) -> Batch:
    rng = np.random.default_rng([1, seed])
    return Batch([make_3d3d(rng, 8, 0.01, 0.05, n_samples)])


def config_c2(seed: int = 0, n_samples: int = 65536, n_kp: int = 12) -> Batch:
    rng = np.random.default_rng([2, seed])
    return Batch([make_2d3d(rng, n_kp, 2.0, (5.0, 20.0), n_samples)])


def config_c3(seed: int = 0, n_inst: int = 512, m_range=(1024, 16384),
              n_range=(6, 48)) -> Batch:
    rng = np.random.default_rng([3, seed])
    ins = []
    for j in range(n_inst):
        n_kp = int(rng.integers(n_range[0], n_range[1] + 1))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        if j % 2 == 0:
            ins.append(make_3d3d(rng, n_kp, 0.01, (0.02, 0.1), m))
        else:
            ins.append(make_2d3d(rng, n_kp, 2.0, (3.0, 25.0), m))
    return Batch(ins)


def config_c4(seed: int = 0, n_samples: int = 262144) -> Batch:
    rng = np.random.default_rng([4, seed])
    return Batch([make_2d3d(rng, 24, 2.0, (5.0, 20.0), n_samples)])


def config_c5(seed: int = 0, n_inst: int = 64, n_samples: int = 1 << 20) -> Batch:
    rng = np.random.default_rng([5, seed])
    return Batch([make_2d3d(rng, 48, 2.0, (5.0, 20.0), n_samples)
                  for _ in range(n_inst)])


CONFIG_ITERS = {"c1": 50, "c2": 100, "c3": 50, "c4": 20, "c5": 50}


def sub_batch(batch: Batch, idx: Sequence[int], n_samples: Optional[int] = None) -> Batch:
    """Instances `idx` of `batch`, optionally with their sample budget reset."""
    out = []
    for j in idx:
        ins = batch.instances[j]
        if n_samples is not None:
            ins = dataclasses.replace(ins, n_samples=n_samples)
        out.append(ins)
    return Batch(out)
