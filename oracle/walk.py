"""The paper's own Step II: the strategic random walk that samples the
rotation boundary and the translation boundary of a PURSE separately
(Section "The CLOSURE Algorithm", Step II; Alg. "d S_R sampler" and
"d S_R parallel sampler"; appendix "Boundary Sampler Algorithms",
Alg. "d S_t sampler" and "d S_t parallel sampler").

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

From each start pose (R0, t0) of S0, N_W walks per mode run N_I iterations:

- rotation mode: the angular velocity w = omega0 (u + u~), u the axis of the
  start's rotation relative to the average rotation R_bar = proj_SO3(sum R0)
  (pointing away from it), u~ a random unit vector.  Each iteration draws N_P
  translation perturbations t_j = t* + delta_j, ranks them by the distance
  to the boundary dist(R*, t_j) = min_i (beta_i - ||g_i||_Lambda_i) (eq.
  partial-s-dist), keeps the N_P* largest, and tries every kept t_j with the
  rotation stepped by each scale gamma^(m-1), m = 1..N_T:
  R_km = Exp(w gamma^(m-1)) R*.  The largest step (smallest m) at which some
  kept perturbation is in S wins, among those the highest ranked (smallest
  k); the walk moves there.  No move if nothing is in S.
- translation mode: the centre velocity v = v0 ((t0 - t_bar) / |t0 - t_bar|
  + v~); the perturbations are rotations R_j = Exp(theta_p e_j) R*, ranked by
  dist(R_j, t*), and the kept ones are tried with t_km = t* + v gamma^(m-1).

The walks are vectorised across walks and perturbations only; each walk's
iterations run in order.  Readings (the paper leaves them open): a
perturbation is a random direction times a uniform magnitude in [0, scale);
the rotation step is a left increment about the camera frame with t fixed,
the translation step leaves R fixed; the translation-mode ranking uses the
perturbed rotation (the printed dist(R*, t_j) there is read as
dist(R_j, t*)); in_purse is the sampler's test r_i <= beta_i + tau (and depth
> z_min for 2D-3D; for the pose-regression set both families of balls of
oracle/reg.py, with the 3D-3D tau); the velocity's radial part is dropped when the start is
at the centre; the PCA rescaling of the translation velocity is omitted.

Random numbers: Philox4x64-10 with key (seed, 1 + mode) and counter
(walk, iteration, perturbation, 0) (iteration 2^32 - 1 for the initial
velocity); the top 24 bits of output words 0, 1, 2 give three uniforms U1,
U2, U3, the direction (sqrt(1 - z^2) cos phi, sqrt(1 - z^2) sin phi, z) with
z = 1 - 2 U1, phi = 2 pi U2, and U3 the magnitude fraction.
"""
import dataclasses
import math
from typing import Optional

import numpy as np
import torch

from . import reg
from .philox import philox4x64_10
from .purse import KIND_2D3D, Problem, residual
from .so3 import exp_so3, log_so3, proj_so3

DT = torch.float64
MODE_R = 0
MODE_T = 1
INIT_ITER = 0xFFFFFFFF


@dataclasses.dataclass
class WalkParams:
    n_walks: int = 2          # N_W walks per start and mode
    n_iters: int = 5          # N_I
    n_perturb: int = 150      # N_P
    n_keep: int = 10          # N_P*
    n_scales: int = 15        # N_T
    gamma: float = 0.5        # step decay
    omega0: float = 0.5       # angular velocity magnitude (rad per unit step)
    v0: float = 0.05          # centre velocity magnitude (m per unit step)
    t_pert: float = 0.005     # translation perturbation scale t_p (m), rotation mode
    r_pert: float = 0.02      # rotation perturbation scale theta_p (rad), translation mode
    tau_abs_3d: float = 1e-5
    tau_abs_2d: float = 1e-4
    z_min: float = 1e-3


def walk_uniforms(seed: int, mode: int, walks, iteration, perturb):
    """Three 24-bit uniforms per (walk, iteration, perturbation) (float64,
    exact in float32)."""
    w = np.asarray(walks, dtype=np.uint64)
    it = np.broadcast_to(np.asarray(iteration, dtype=np.uint64), w.shape)
    j = np.broadcast_to(np.asarray(perturb, dtype=np.uint64), w.shape)
    z = np.zeros_like(w)
    out = philox4x64_10((w, it, j, z), (np.uint64(seed), np.uint64(1 + mode)))
    return [(out[k] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24 for k in range(3)]


def _direction(u1, u2):
    z = 1.0 - 2.0 * u1
    phi = 2.0 * math.pi * u2
    rho = np.sqrt(np.maximum(1.0 - z * z, 0.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], -1)


def perturbations(seed, mode, walks, iteration, n_perturb, scale):
    """(W, N_P, 3): direction times a uniform fraction of scale."""
    W = len(walks)
    wv = np.repeat(np.asarray(walks, dtype=np.uint64), n_perturb)
    jv = np.tile(np.arange(n_perturb, dtype=np.uint64), W)
    u1, u2, u3 = walk_uniforms(seed, mode, wv, iteration, jv)
    d = _direction(u1, u2) * (scale * u3)[:, None]
    return torch.as_tensor(d.reshape(W, n_perturb, 3), dtype=DT)


def boundary_distance(prob: Problem, R, t):
    """eq. partial-s-dist: min_i (beta_i - ||g_i||_Lambda_i), batched over
    leading pose dims (R: (..., 3, 3), t: (..., 3))."""
    if isinstance(prob, reg.RegProblem):
        return reg.boundary_distance(prob, R, t)
    lead = R.shape[:-2]
    e, r, depth = residual(prob, R.reshape(-1, 3, 3), t.reshape(-1, 3))
    d = (prob.beta - r).min(-1).values
    return d.reshape(lead)


def in_purse(prob: Problem, R, t, wp: WalkParams):
    if isinstance(prob, reg.RegProblem):
        return reg.in_purse(prob, R, t, wp.tau_abs_3d)
    lead = R.shape[:-2]
    e, r, depth = residual(prob, R.reshape(-1, 3, 3), t.reshape(-1, 3))
    tau = wp.tau_abs_2d if prob.kind == KIND_2D3D else wp.tau_abs_3d
    ok = (r <= prob.beta + tau).all(-1)
    if depth is not None:
        ok = ok & (depth > wp.z_min).all(-1)
    return ok.reshape(lead)


def feasibility_ratio(prob: Problem, R, t, wp: WalkParams):
    """Diagnostic: max_i r_i / (beta_i + tau) (inf behind z_min)."""
    if isinstance(prob, reg.RegProblem):
        return reg.feasibility_ratio(prob, R, t, wp.tau_abs_3d)
    lead = R.shape[:-2]
    e, r, depth = residual(prob, R.reshape(-1, 3, 3), t.reshape(-1, 3))
    tau = wp.tau_abs_2d if prob.kind == KIND_2D3D else wp.tau_abs_3d
    ratio = (r / (prob.beta + tau)).max(-1).values
    if depth is not None:
        ratio = torch.where((depth > wp.z_min).all(-1), ratio, torch.full_like(ratio, math.inf))
    return ratio.reshape(lead)


def top_k(d: torch.Tensor, k: int):
    """Indices of the k largest entries of each row, largest first; equal
    values in increasing index order (a stable sort on -d)."""
    order = np.argsort(-d.numpy(), axis=-1, kind="stable")
    return torch.as_tensor(order[..., :k].copy())


def centre_of_starts(R0, t0):
    """R_bar = proj_SO3(sum R_j), t_bar = mean t_j (the parallel samplers'
    first lines)."""
    return proj_so3(R0.sum(0)), t0.mean(0)


def initial_velocity(mode, R0, t0, Rbar, tbar, walks, seed, wp: WalkParams):
    """Rotation mode: omega0 (u + u~), u the unit axis of R0 R_bar^T (zero at
    the centre); translation mode: v0 ((t0 - t_bar)/|t0 - t_bar| + v~)."""
    u1, u2, _ = walk_uniforms(seed, mode, walks, INIT_ITER, 0)
    rnd = torch.as_tensor(_direction(u1, u2), dtype=DT)
    if mode == MODE_R:
        a = log_so3(R0 @ Rbar.T)
        n = a.norm(dim=-1, keepdim=True)
        u = torch.where(n > 0, a / torch.where(n > 0, n, torch.ones_like(n)), torch.zeros_like(a))
        return wp.omega0 * (u + rnd)
    dv = t0 - tbar
    n = dv.norm(dim=-1, keepdim=True)
    u = torch.where(n > 0, dv / torch.where(n > 0, n, torch.ones_like(n)), torch.zeros_like(dv))
    return wp.v0 * (u + rnd)


def walk(prob: Problem, starts_R, starts_t, seed: int, mode: int, wp: WalkParams,
         diagnostics: bool = False) -> dict:
    """All N_W walks of every start in one mode.  Walk w = s N_W + n starts
    from start s.  Returns the final poses (W, 12), the in_purse bit of each,
    the per-iteration decision k0 N_T + (m0 - 1) (-1: no move), the step sum
    of each walk, and with diagnostics the decision margins."""
    R0 = torch.as_tensor(starts_R, dtype=DT).reshape(-1, 3, 3)
    t0 = torch.as_tensor(starts_t, dtype=DT).reshape(-1, 3)
    S = R0.shape[0]
    Rbar, tbar = centre_of_starts(R0, t0)
    W = S * wp.n_walks
    walks = np.arange(W, dtype=np.uint64)
    Rs = R0.repeat_interleave(wp.n_walks, 0)
    ts = t0.repeat_interleave(wp.n_walks, 0)
    vel = initial_velocity(mode, Rs, ts, Rbar, tbar, walks, seed, wp)
    K, NT = wp.n_keep, wp.n_scales
    scales = torch.as_tensor([wp.gamma ** m for m in range(NT)], dtype=DT)      # gamma^(m-1), m = 1..N_T
    decisions = torch.full((W, wp.n_iters), -1, dtype=torch.int64)
    steps = torch.zeros(W, dtype=DT)
    rank_gap = torch.full((W, wp.n_iters), math.inf, dtype=DT)
    feas_margin = torch.full((W, wp.n_iters), math.inf, dtype=DT)
    ar = torch.arange(W)
    for i in range(wp.n_iters):
        if mode == MODE_R:
            delta = perturbations(seed, mode, walks, i, wp.n_perturb, wp.t_pert)
            Rp = Rs[:, None].expand(W, wp.n_perturb, 3, 3)
            tp = ts[:, None, :] + delta
        else:
            delta = perturbations(seed, mode, walks, i, wp.n_perturb, wp.r_pert)
            Rp = exp_so3(delta) @ Rs[:, None]
            tp = ts[:, None, :].expand(W, wp.n_perturb, 3)
        d = boundary_distance(prob, Rp, tp)                           # (W, N_P)
        keep = top_k(d, K)                                            # (W, K)
        Rk = Rp[ar[:, None], keep]                                    # (W, K, 3, 3)
        tk = tp[ar[:, None], keep]                                    # (W, K, 3)
        if mode == MODE_R:
            E = exp_so3(vel[:, None, :] * scales[None, :, None])      # (W, N_T, 3, 3)
            Rc = (E @ Rs[:, None])[:, :, None].expand(W, NT, K, 3, 3)
            tc = tk[:, None].expand(W, NT, K, 3)
        else:
            Rc = Rk[:, None].expand(W, NT, K, 3, 3)
            tc = (ts[:, None, :] + vel[:, None, :] * scales[None, :, None])[:, :, None].expand(W, NT, K, 3)
        ok = in_purse(prob, Rc, tc, wp)                               # (W, N_T, K)
        flat = ok.reshape(W, NT * K)
        any_ok = flat.any(-1)
        first = torch.argmax(flat.to(torch.int64), -1)                # smallest m, then smallest k
        m0 = first // K
        k0 = first % K
        newR = Rc[ar, m0, k0]
        newt = tc[ar, m0, k0]
        Rs = torch.where(any_ok[:, None, None], newR, Rs)
        ts = torch.where(any_ok[:, None], newt, ts)
        decisions[:, i] = torch.where(any_ok, k0 * NT + m0, torch.full_like(k0, -1))
        steps = steps + torch.where(any_ok, scales[m0], torch.zeros_like(steps))
        if diagnostics:
            ds = torch.sort(d, dim=-1, descending=True).values[:, :K + 1]
            rank_gap[:, i] = (ds[:, :-1] - ds[:, 1:]).min(-1).values
            ratio = feasibility_ratio(prob, Rc, tc, wp)               # (W, N_T, K)
            upto = torch.arange(NT)[None, :, None] <= torch.where(any_ok, m0, torch.full_like(m0, NT - 1))[:, None, None]
            feas_margin[:, i] = torch.where(upto, (ratio - 1.0).abs(), torch.full_like(ratio, math.inf)) \
                .reshape(W, -1).min(-1).values
    poses = torch.cat([Rs.reshape(W, 9), ts], 1)
    out = dict(poses=poses, mask=in_purse(prob, Rs, ts, wp).to(torch.uint8), decisions=decisions,
               steps=steps, velocity=vel, start_R=R0.repeat_interleave(wp.n_walks, 0),
               start_t=t0.repeat_interleave(wp.n_walks, 0))
    if diagnostics:
        out.update(rank_gap=rank_gap, feas_margin=feas_margin)
    return out
