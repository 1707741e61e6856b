"""Reverse pass of the sampler + MEGB in float64, by autograd over the oracle's
own forward with every discrete decision frozen.

The map differentiated is (measurements) -> (D_hat, d_hat, R*, t*) as the
forward computes it: the centre fit at its converged Gauss-Newton solution,
the trajectories of the samples the MEGB actually touched (the first feasible
sample, every argmax of the descent, and the two samples that realise the
final radii), with their projection clamps, feasibility outcome and bisection
step held as computed, and the geodesic descent replayed along the given
argmax trace.  The paper states no gradient; this is the frozen-decision
reading (derivatives of the computed map away from switching surfaces).  The
projection clamp of a constraint within a relative 1e-5 inside its shrunk
ball is taken on its projected side (converged trajectories end on that kink;
see project_targets).

Cotangents: g_radii = (dL/dD_hat, dL/dd_hat); g_centre = (g_w, g_t) with g_w
paired with the left so(3) perturbation of R* (R* -> Exp(e) R*) and g_t with
t*.  Gradients are returned for the ellipse / ball centres (N,3; the third
column is zero for 2D-3D), the shape matrices (N,4, symmetrised, zero for
3D-3D) and the bounds (N,).
"""
import numpy as np
import torch

from .params import OracleParams
from .purse import (KIND_2D3D, MASK_FEASIBLE, Problem, feasibility_ratio, feasible, initial_poses, prologue,
                    pull_in, run_trajectories)
from .so3 import angle, exp_so3, log_so3, proj_so3, proj_so3_newton, vee_skew

DT = torch.float64


def _leaves(inst):
    c = torch.tensor(np.asarray(inst.centres, dtype=np.float64), requires_grad=True)
    L = torch.tensor(np.asarray(inst.shapes, dtype=np.float64).reshape(-1, 2, 2), requires_grad=True)
    b = torch.tensor(np.asarray(inst.bounds, dtype=np.float64), requires_grad=True)
    return c, L, b


def frozen_forward(inst, p: OracleParams, trace, s0, sD, sd, centres=None, shapes=None, bounds=None,
                   lo=None):
    """(D_hat, d_hat, R*, t*) of the frozen-decision map.  trace (T,2) holds the
    argmax sample of every descent step (rotation, translation); s0 the first
    feasible sample; sD, sd the samples realising the radii; lo (optional,
    indexed by sample) the bisection outcome of pulled-in samples, else it is
    recomputed."""
    centres = torch.as_tensor(np.asarray(inst.centres), dtype=DT) if centres is None else centres
    shapes = torch.as_tensor(np.asarray(inst.shapes), dtype=DT) if shapes is None else shapes
    bounds = torch.as_tensor(np.asarray(inst.bounds), dtype=DT) if bounds is None else bounds
    prob = Problem(inst.kind, inst.model_pts, centres, shapes, bounds, inst.intrinsics)
    pro = prologue(prob, p)
    trace = np.asarray(trace, dtype=np.int64)
    active = sorted(set(trace[:, 0].tolist()) | set(trace[:, 1].tolist()) | {int(s0), int(sD), int(sd)})
    ids = np.asarray(active, dtype=np.uint64)
    R0, t0 = initial_poses(pro, p, inst.seed, ids)
    R, t, failed = run_trajectories(prob, R0, t0, pro["o_c"], p, deriv_convention=True)
    with torch.no_grad():
        feas = feasible(prob, R, t, p) & ~failed
    need = torch.nonzero(~feas & ~failed)[:, 0]
    if len(need):
        lo_fixed = None if lo is None else np.asarray(lo)[ids[need.numpy()].astype(np.int64)]
        Rb, tb, _ = pull_in(prob, pro["R_a"], pro["t_a"], R[need], t[need], p, lo_fixed)
        Rl, tl = list(R.unbind(0)), list(t.unbind(0))
        for k, j in enumerate(need.tolist()):
            Rl[j], tl[j] = Rb[k], tb[k]
        R, t = torch.stack(Rl), torch.stack(tl)
    pos = {s: k for k, s in enumerate(active)}
    C = R[pos[int(s0)]]
    c = t[pos[int(s0)]]
    T = len(trace)
    keep_C, keep_c = [], []
    for i in range(1, T + 1):
        C = C @ exp_so3(log_so3(C.T @ R[pos[int(trace[i - 1, 0])]]) / i)
        c = c + (t[pos[int(trace[i - 1, 1])]] - c) / i
        if i > T - p.megb_avg:
            keep_C.append(C)
            keep_c.append(c)
    Rstar = proj_so3_newton(torch.stack(keep_C).sum(0))  # same value as proj_so3, stable derivative
    tstar = torch.stack(keep_c).mean(0)
    D = angle(Rstar[None], R[pos[int(sD)]][None])[0]
    d = torch.sqrt(((tstar - t[pos[int(sd)]]) ** 2).sum())
    return D, d, Rstar, tstar


def objective(D, d, Rs, ts, g_radii, g_centre, Rref=None):
    """g_radii . (D, d) + g_w . e(R*) + g_t . t*, e the left so(3) offset of R*
    from Rref (R* itself when not given)."""
    g_radii = torch.as_tensor(np.asarray(g_radii, dtype=np.float64))
    g_centre = torch.as_tensor(np.asarray(g_centre, dtype=np.float64))
    Rref = Rs.detach() if Rref is None else torch.as_tensor(Rref, dtype=DT)
    return (g_radii[0] * D + g_radii[1] * d + (g_centre[:3] * vee_skew(Rs @ Rref.T)).sum()
            + (g_centre[3:] * ts).sum())


def backward(inst, p: OracleParams, trace, s0, sD, sd, g_radii, g_centre, lo=None):
    """Gradients (centres (N,3), shapes (N,4), bounds (N,)) of
    g_radii . (D, d) + g_w . e(R*) + g_t . t*."""
    cen, L, b = _leaves(inst)
    D, d, Rs, ts = frozen_forward(inst, p, trace, s0, sD, sd, cen, L, b, lo)
    loss = objective(D, d, Rs, ts, g_radii, g_centre)
    gc, gL, gb = torch.autograd.grad(loss, [cen, L, b], allow_unused=True)
    gc = torch.zeros_like(cen) if gc is None else gc
    gL = torch.zeros_like(L) if gL is None else gL
    gb = torch.zeros_like(b) if gb is None else gb
    gL = 0.5 * (gL + gL.transpose(-1, -2))
    if inst.kind == KIND_2D3D:
        gc = gc.clone()
        gc[:, 2] = 0.0
    else:
        gL = torch.zeros_like(gL)
    return gc.detach().numpy(), gL.reshape(-1, 4).detach().numpy(), gb.detach().numpy()


def decision_margins(inst, p: OracleParams, sample_ids, bis_steps: int = 8):
    """Per sample, the smallest relative margin of the decisions the frozen-
    decision map holds fixed: the projection clamps of every iteration (at
    the derivative convention's threshold), the final in_purse test
    (|max_i r_i / (beta_i + tau) - 1|) and, for samples pulled in, the
    bisection's first bis_steps tests (a later step's outcome moves the
    pulled-in pose by at most 2^-bis_steps of the segment).  A margin near
    float32 rounding marks a decision that a float32 recomputation may take
    the other way, and with it a different (equally valid) frozen-decision
    derivative (diagnostic)."""
    prob = Problem(inst.kind, inst.model_pts, torch.as_tensor(np.asarray(inst.centres), dtype=DT),
                   torch.as_tensor(np.asarray(inst.shapes), dtype=DT),
                   torch.as_tensor(np.asarray(inst.bounds), dtype=DT), inst.intrinsics)
    pro = prologue(prob, p)
    ids = np.asarray(sample_ids, dtype=np.uint64)
    R0, t0 = initial_poses(pro, p, inst.seed, ids)
    m_cl = []
    with torch.no_grad():
        R, t, failed = run_trajectories(prob, R0, t0, pro["o_c"], p, deriv_convention=True, margins=m_cl)
        out = torch.minimum(m_cl[0], (feasibility_ratio(prob, R, t, p) - 1.0).abs())
        need = torch.nonzero(~feasible(prob, R, t, p) & ~failed)[:, 0]
        if len(need) and pro.get("R_a") is not None:
            mb = []
            pull_in(prob, pro["R_a"], pro["t_a"], R[need], t[need], p, margins=mb, margin_steps=bis_steps)
            out[need] = torch.minimum(out[need], mb[0])
    return out.numpy()


def radius_argmax(poses, mask, Rstar, tstar):
    """Samples realising the radii about a centre (lowest index on ties)."""
    P = torch.as_tensor(np.asarray(poses, dtype=np.float64))
    sel = torch.nonzero(torch.as_tensor((np.asarray(mask) & MASK_FEASIBLE) != 0))[:, 0]
    R = P[sel, :9].reshape(-1, 3, 3)
    t = P[sel, 9:]
    kr = ((torch.as_tensor(Rstar, dtype=DT) - R) ** 2).sum((-1, -2))
    kt = ((torch.as_tensor(tstar, dtype=DT) - t) ** 2).sum(-1)
    return int(sel[int(torch.argmax(kr))]), int(sel[int(torch.argmax(kt))])
