"""Rotation-group helpers in float64 torch (batched over leading dims).

Definitions used by the paper: the geodesic distance on SO(3) is the rotation
angle of C^T R (Section "Minimum Enclosing Geodesic Ball", eq. megb-rot);
the exponential map Exp(x) = exp(x^) and the axis-angle representation appear
in the appendix "Geodesic Gradient Descent".  The angle is evaluated as
2 asin(||C - R||_F / (2 sqrt 2)), which equals the arccos form for exact
rotations but stays accurate at small angles.
"""
import math

import torch

_SMALL = 1e-8


def hat(w: torch.Tensor) -> torch.Tensor:
    z = torch.zeros_like(w[..., 0])
    return torch.stack([
        torch.stack([z, -w[..., 2], w[..., 1]], -1),
        torch.stack([w[..., 2], z, -w[..., 0]], -1),
        torch.stack([-w[..., 1], w[..., 0], z], -1),
    ], -2)


def vee_skew(M: torch.Tensor) -> torch.Tensor:
    """vee of the antisymmetric part (M - M^T)/2."""
    return 0.5 * torch.stack([M[..., 2, 1] - M[..., 1, 2],
                              M[..., 0, 2] - M[..., 2, 0],
                              M[..., 1, 0] - M[..., 0, 1]], -1)


def exp_so3(w: torch.Tensor) -> torch.Tensor:
    """Rodrigues' formula I + (sin th/th) W + ((1 - cos th)/th^2) W^2, with its
    Taylor series below th = 1e-4."""
    th2 = (w * w).sum(-1)
    small = th2 < 1e-8
    th2s = torch.where(small, torch.ones_like(th2), th2)
    th = torch.sqrt(th2s)
    A = torch.where(small, 1.0 - th2 / 6.0 + th2 * th2 / 120.0, torch.sin(th) / th)
    B = torch.where(small, 0.5 - th2 / 24.0 + th2 * th2 / 720.0, (1.0 - torch.cos(th)) / th2s)
    W = hat(w)
    eye = torch.eye(3, dtype=w.dtype).expand(W.shape)
    return eye + A[..., None, None] * W + B[..., None, None] * (W @ W)


def log_so3(R: torch.Tensor) -> torch.Tensor:
    """Axis-angle vector of R (angle < pi): theta = atan2(|s|, (tr R - 1)/2)
    with s = vee((R - R^T)/2) = sin(theta) * axis."""
    s = vee_skew(R)
    c = 0.5 * (R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2] - 1.0)
    sn2 = (s * s).sum(-1)
    small = sn2 < 1e-16
    sn = torch.sqrt(torch.where(small, torch.ones_like(sn2), sn2))
    th = torch.atan2(sn, c)
    f = torch.where(small, 1.0 + sn2 / 6.0, th / sn)
    return f[..., None] * s


def proj_so3(M: torch.Tensor) -> torch.Tensor:
    """Nearest rotation in Frobenius norm: U diag(1, 1, det(U V^T)) V^T for
    M = U S V^T."""
    U, S, Vh = torch.linalg.svd(M)
    d = torch.sign(torch.linalg.det(U @ Vh))
    d = torch.where(d == 0, torch.ones_like(d), d)
    D = torch.ones(M.shape[:-2] + (3,), dtype=M.dtype)
    D = torch.cat([D[..., :2], d[..., None]], -1)
    return U @ (D[..., :, None] * Vh)


def proj_so3_newton(M: torch.Tensor, iters: int = 12) -> torch.Tensor:
    """The same nearest rotation for det(M) > 0 by the Newton iteration
    X <- (X + X^-T)/2 on the polar factor (scaled to unit determinant first).
    Used where derivatives are needed and M is close to a multiple of a
    rotation: there the singular values are nearly equal and the SVD's own
    derivative is ill-conditioned, while this iteration's is not."""
    X = M / torch.linalg.det(M).abs().pow(1.0 / 3.0)
    for _ in range(iters):
        X = 0.5 * (X + torch.linalg.inv(X).transpose(-1, -2))
    return X


def angle(C: torch.Tensor, R: torch.Tensor) -> torch.Tensor:
    """Geodesic distance on SO(3), 2 asin(||C - R||_F / (2 sqrt 2))."""
    f = torch.sqrt(((C - R) ** 2).sum((-1, -2)))
    return 2.0 * torch.asin(torch.clamp(f / (2.0 * math.sqrt(2.0)), max=1.0))


def rot_to_quat(R: torch.Tensor) -> torch.Tensor:
    """Unit quaternion (w, x, y, z) with w >= 0 (Shepperd's branch choice)."""
    tr = R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2]
    out = []
    for i in range(R.reshape(-1, 3, 3).shape[0]):
        m = R.reshape(-1, 3, 3)[i]
        t = float(tr.reshape(-1)[i])
        if t > 0:
            s = math.sqrt(t + 1.0) * 2
            q = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif m[0, 0] > m[1, 1] and m[0, 0] > m[2, 2]:
            s = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2
            q = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif m[1, 1] > m[2, 2]:
            s = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2
            q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2
            q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
        q = torch.stack([torch.as_tensor(v, dtype=R.dtype) for v in q])
        q = q / torch.linalg.norm(q)
        if q[0] < 0:
            q = -q
        out.append(q)
    return torch.stack(out).reshape(R.shape[:-2] + (4,))


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
