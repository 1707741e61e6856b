"""Exact and brute-force enclosing balls, used only to pin the MEGB.

* `welzl`: smallest enclosing ball in R^d by Welzl's randomised recursion in
  Gaertner's move-to-front form (Gaertner 1999 is the miniball the paper's
  Step III uses, Section "The CLOSURE Algorithm").
* `brute_force_meb`: the same ball by enumerating every support set of at most
  d+1 points (textbook definition; tiny inputs only).
* `so3_minimax`: min over C in SO(3) of the max geodesic angle to a rotation
  set, by a derivative-free local search from several starts; the objective is
  geodesically convex for sets inside a ball of radius pi/2 (appendix
  "Geodesic Gradient Descent", Proposition on convexity), so local = global.
* `quaternion_meb`: the R^4 ball of sign-aligned unit quaternions, the embedding
  Step III applies to rotations.
"""
import itertools

import numpy as np
import scipy.optimize

from . import so3
import torch


def circumsphere(P: np.ndarray):
    """Centre and radius of the smallest sphere through the points P (k,d),
    centre in their affine hull."""
    p0 = P[0]
    if len(P) == 1:
        return p0.copy(), 0.0
    A = P[1:] - p0
    G = A @ A.T
    rhs = 0.5 * (A * A).sum(1)
    lam = np.linalg.lstsq(G, rhs, rcond=None)[0]
    c = p0 + lam @ A
    return c, float(np.linalg.norm(c - p0))


def _inside(c, r, p, eps):
    return np.linalg.norm(p - c) <= r * (1 + eps) + eps


def welzl(P: np.ndarray, eps: float = 1e-12, seed: int = 0):
    P = np.asarray(P, dtype=np.float64)
    d = P.shape[1]
    order = list(np.random.default_rng(seed).permutation(len(P)))
    L = [P[i] for i in order]

    def mtf(n, B):
        if B:
            c, r = circumsphere(np.array(B))
        else:
            c, r = L[0].copy(), -1.0
        if len(B) == d + 1:
            return c, r
        i = 0
        while i < n:
            p = L[i]
            if r < 0 or not _inside(c, r, p, eps):
                c, r = mtf(i, B + [p])
                L.insert(0, L.pop(i))
            i += 1
        return c, r

    c, r = mtf(len(L), [])
    return c, max(r, 0.0)


def brute_force_meb(P: np.ndarray, eps: float = 1e-10):
    P = np.asarray(P, dtype=np.float64)
    d = P.shape[1]
    best = (None, np.inf)
    for k in range(1, min(d + 1, len(P)) + 1):
        for S in itertools.combinations(range(len(P)), k):
            c, r = circumsphere(P[list(S)])
            if r < best[1] and np.all(np.linalg.norm(P - c, axis=1) <= r * (1 + eps) + eps):
                best = (c, r)
    return best


def quaternion_meb(R: np.ndarray):
    """R^4 ball of the unit quaternions of R (K,3,3), all put on the
    hemisphere of the first; returns the rotation of the normalised centre."""
    q = so3.rot_to_quat(torch.as_tensor(R, dtype=torch.float64)).numpy()
    q = q * np.sign(q @ q[0])[:, None]
    c, r = welzl(q)
    C = so3.quat_to_rot(torch.as_tensor(c / np.linalg.norm(c))).numpy()
    return C, r


def max_angle(C: np.ndarray, R: np.ndarray) -> float:
    return float(so3.angle(torch.as_tensor(C)[None], torch.as_tensor(R)).max())


def so3_minimax(R: np.ndarray, starts=None, n_restarts: int = 4, seed: int = 0):
    """min_C max_s angle(C, R_s) by Nelder-Mead on C0 Exp(w)."""
    R = np.asarray(R, dtype=np.float64)
    Rt = torch.as_tensor(R)
    rng = np.random.default_rng(seed)
    if starts is None:
        starts = [R[0]]
    starts = list(starts) + [R[int(rng.integers(len(R)))] for _ in range(n_restarts)]
    best = (None, np.inf)
    for C0 in starts:
        C0t = torch.as_tensor(C0)

        def f(w):
            C = C0t @ so3.exp_so3(torch.as_tensor(w))
            return float(so3.angle(C[None], Rt).max())

        w = np.zeros(3)
        for scale in (0.2, 0.02, 0.002):
            res = scipy.optimize.minimize(
                f, w, method="Nelder-Mead",
                options=dict(xatol=1e-12, fatol=1e-14, maxiter=20000,
                             initial_simplex=np.vstack([w, w + scale * np.eye(3)])))
            w = res.x
        if res.fun < best[1]:
            best = ((C0t @ so3.exp_so3(torch.as_tensor(w))).numpy(), float(res.fun))
    return best


def exact_megb(poses: np.ndarray, mask: np.ndarray):
    """Step III on a sample set: the exact minimum enclosing ball of the
    feasible translations (R^3) and of their rotations as unit quaternions in
    R^4 on the hemisphere of the first feasible sample; the rotation centre is
    the normalised quaternion centre.  Returns (R*, t*, D, d) with D the
    largest geodesic angle and d the largest distance from that centre."""
    P = np.asarray(poses, dtype=np.float64)[(np.asarray(mask) & 1) != 0]
    R = P[:, :9].reshape(-1, 3, 3)
    t = P[:, 9:]
    from scipy.spatial.transform import Rotation
    q = Rotation.from_matrix(R).as_quat()[:, [3, 0, 1, 2]]   # (w, x, y, z)
    q = q * np.where(q @ q[0] < 0, -1.0, 1.0)[:, None]
    c, _ = welzl(q)
    C = so3.quat_to_rot(torch.as_tensor(c / np.linalg.norm(c))).numpy()
    ct, d = welzl(t)
    return C, ct, max_angle(C, R), float(np.linalg.norm(t - ct, axis=1).max())
