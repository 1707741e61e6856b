"""Minimum enclosing geodesic ball of a sample set by geodesic (sub)gradient
descent.

The MEGB of the rotation and translation projections is the pair of minimax
problems of Section "Minimum Enclosing Geodesic Ball" (eqs. megb-rot,
megb-tran); on a finite sample set they give the inner approximation of
Proposition 1.  The recipe is the geodesic gradient descent of the same
section: from the current centre, find the sample at maximum distance and move
a fraction of the way along the geodesic towards it.  The appendix "Geodesic
Gradient Descent" fixes the details used here: the step fraction 1/i of the
SLERP in the SDP-based algorithm (read as SLERP from the previous iterate), the
centre as the projection onto SO(3) of the sum of the last 10 iterates, and
the argmax taken by Frobenius distance, which orders samples exactly as the
geodesic distance does (the remark after the Riemannian Danskin theorem).
The translation ball mirrors this in R^3 (the Badoiu-Clarkson step).

Ties in the argmax go to the lowest sample index.  The final radii are the
maximum geodesic angle and Euclidean distance from the centre to the samples.
"""
import math

import torch

from .so3 import angle, exp_so3, log_so3, proj_so3

DT = torch.float64


def megb(R_s: torch.Tensor, t_s: torch.Tensor, ids: torch.Tensor, T: int, avg: int) -> dict:
    """R_s (K,3,3), t_s (K,3): the feasible samples in increasing sample index
    `ids` (K,).  Returns the centre (R*, t*), the radii (D_hat rad, d_hat m),
    and the argmax trace as sample indices, shape (T, 2) (rotation,
    translation)."""
    K = R_s.shape[0]
    if K == 0:
        nan = float("nan")
        return dict(R=torch.full((3, 3), nan, dtype=DT), t=torch.full((3,), nan, dtype=DT),
                    D=nan, d=nan, trace=torch.full((T, 2), -1, dtype=torch.int64), n=0)
    C = R_s[0].clone()
    c = t_s[0].clone()
    trace = torch.empty(T, 2, dtype=torch.int64)
    keep_C, keep_c = [], []
    for i in range(1, T + 1):
        kr = ((C - R_s) ** 2).sum((-1, -2))
        sr = int(torch.argmax(kr))
        C = C @ exp_so3(log_so3(C.T @ R_s[sr]) / i)
        kt = ((c - t_s) ** 2).sum(-1)
        st = int(torch.argmax(kt))
        c = c + (t_s[st] - c) / i
        trace[i - 1, 0] = ids[sr]
        trace[i - 1, 1] = ids[st]
        if i > T - avg:
            keep_C.append(C)
            keep_c.append(c)
    Rstar = proj_so3(torch.stack(keep_C).sum(0))
    tstar = torch.stack(keep_c).mean(0)
    D = float(angle(Rstar[None], R_s).max())
    d = float(torch.sqrt(((tstar - t_s) ** 2).sum(-1)).max())
    return dict(R=Rstar, t=tstar, D=D, d=d, trace=trace, n=K)


def megb_from_poses(poses: torch.Tensor, mask: torch.Tensor, T: int, avg: int) -> dict:
    """MEGB of the mask-feasible rows of a (M,12) pose array."""
    sel = torch.nonzero((mask.to(torch.int64) & 1) != 0)[:, 0]
    P = poses[sel].to(DT)
    return megb(P[:, :9].reshape(-1, 3, 3), P[:, 9:], sel, T, avg)


def radii_at(Rc: torch.Tensor, tc: torch.Tensor, R_s: torch.Tensor, t_s: torch.Tensor):
    """Enclosing radii of the samples about a given centre."""
    return (float(angle(Rc[None], R_s).max()),
            float(torch.sqrt(((tc - t_s) ** 2).sum(-1)).max()))


def frobenius_to_angle(f: float) -> float:
    return 2.0 * math.asin(min(1.0, f / (2.0 * math.sqrt(2.0))))
