"""The pose-regression PURSE (eq. PURSEregression): the intersection of balls
around N pose hypotheses, ||vec(R) - vec(R_i)||_{Lambda_i^R} <= beta_i^R and
||t - t_i||_{Lambda_i^t} <= beta_i^t, read with Lambda^R = I_9 (the Frobenius
distance) and Lambda^t = I_3 (Section "Geometric Structures": the set is
simply the intersection of N balls around R_i and t_i), and its Step I
initial sampler: a random convex combination of the hypotheses, kept when it
lies in S (Section "The CLOSURE Algorithm", Step I, third item).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings: the rotation of a convex combination is proj_SO3(sum_i w_i R_i)
and its translation sum_i w_i t_i; the weights are uniform on the simplex,
w_i = e_i / sum_k e_k with e_i = -ln(1 - U_i) for uniforms U_i from
Philox4x64-10, key (seed, 3), counter (trial, i, 0, 0), top 24 bits of word 0;
membership uses the sampler's tolerance tau (metres and Frobenius units
alike).
"""
import dataclasses

import numpy as np
import torch

from .philox import philox4x64_10
from .so3 import proj_so3

DT = torch.float64
KIND_REG = 2


@dataclasses.dataclass
class RegProblem:
    R_i: torch.Tensor       # (N, 3, 3)
    t_i: torch.Tensor       # (N, 3)
    beta_R: torch.Tensor    # (N,)  Frobenius radius
    beta_t: torch.Tensor    # (N,)  metres
    kind: int = KIND_REG

    @property
    def n(self) -> int:
        return self.R_i.shape[0]

    @property
    def beta(self):
        return torch.cat([self.beta_R, self.beta_t])


def residuals(prob: RegProblem, R, t):
    """||R - R_i||_F and ||t - t_i|| for every hypothesis: (..., N) each."""
    lead = R.shape[:-2]
    Rf = R.reshape(-1, 1, 9)
    rR = torch.sqrt(((Rf - prob.R_i.reshape(1, -1, 9)) ** 2).sum(-1))
    rt = torch.sqrt(((t.reshape(-1, 1, 3) - prob.t_i[None]) ** 2).sum(-1))
    return rR.reshape(lead + (prob.n,)), rt.reshape(lead + (prob.n,))


def boundary_distance(prob: RegProblem, R, t):
    """eq. partial-s-dist over both families of constraints."""
    rR, rt = residuals(prob, R, t)
    return torch.minimum((prob.beta_R - rR).min(-1).values, (prob.beta_t - rt).min(-1).values)


def in_purse(prob: RegProblem, R, t, tau: float):
    rR, rt = residuals(prob, R, t)
    return (rR <= prob.beta_R + tau).all(-1) & (rt <= prob.beta_t + tau).all(-1)


def feasibility_ratio(prob: RegProblem, R, t, tau: float):
    rR, rt = residuals(prob, R, t)
    return torch.maximum((rR / (prob.beta_R + tau)).max(-1).values, (rt / (prob.beta_t + tau)).max(-1).values)


def convex_weights(seed: int, trials: np.ndarray, n: int):
    """(T, N) weights uniform on the simplex."""
    tr = np.repeat(np.asarray(trials, dtype=np.uint64), n)
    i = np.tile(np.arange(n, dtype=np.uint64), len(trials))
    z = np.zeros_like(tr)
    out = philox4x64_10((tr, i, z, z), (np.uint64(seed), np.uint64(3)))
    u = (out[0] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    e = -np.log1p(-u).reshape(len(trials), n)
    return torch.as_tensor(e / e.sum(1, keepdims=True), dtype=DT)


def convex_samples(prob: RegProblem, seed: int, n_trials: int, tau: float):
    """Step I for the pose-regression set: n_trials convex combinations of the
    hypotheses; returns poses (T, 12) and the in_purse mask."""
    w = convex_weights(seed, np.arange(n_trials), prob.n)
    R = proj_so3(torch.einsum("tn,nij->tij", w, prob.R_i))
    t = w @ prob.t_i
    ok = in_purse(prob, R, t, tau)
    return torch.cat([R.reshape(-1, 9), t], 1), ok.to(torch.uint8)


def from_instance(inst) -> RegProblem:
    """The pose-regression set of a batch instance (keypoint i = hypothesis
    i: centres = t_i, shapes = quaternion (w, x, y, z) of R_i, model_pts x =
    beta_i^R, bounds = beta_i^t)."""
    from .so3 import quat_to_rot
    q = torch.as_tensor(np.asarray(inst.shapes, dtype=np.float64)).reshape(-1, 4)
    return RegProblem(quat_to_rot(q), torch.as_tensor(np.asarray(inst.centres, dtype=np.float64)).reshape(-1, 3),
                      torch.as_tensor(np.asarray(inst.model_pts, dtype=np.float64)).reshape(-1, 3)[:, 0].clone(),
                      torch.as_tensor(np.asarray(inst.bounds, dtype=np.float64)).reshape(-1))
