"""PURSE boundary sampler: prologue, trajectories, feasibility, pull-in.

The set sampled is the pose uncertainty set of eq. PURSE,
    S = { x = (R, t) : ||g(x, y_i)||_{Lambda_i} <= beta_i for every i },
with the 2D-3D residual g = z_i - Pi(R Z_i + t) (eq. g-2D3D, Example 1) and
the 3D-3D residual g = b_i - (R a_i + t) (eq. g-3D3D, Example 2); the set
forms are eqs. PURSE2D3D and PURSE3D3D (Section "Geometric Structures").

The sampler is the alternating scheme built from the paper's geometric reading
of those sets (Section "Geometric Structures": the keypoints form a rigid body
that must keep each keypoint inside its ball, or each bearing line through its
ellipse) together with the ingredients of Step I and Step II of the CLOSURE
algorithm (Section "The CLOSURE Algorithm"): a pose is fitted in closed form
to one point per constraint (Arun's method for 3D-3D), trajectories start
with random angular or centre velocities pointing away from the centre
(Step II, "Walk away from the center"), rotation-seeking and
translation-seeking walks are kept separate (Alg. 1), and each pose is tested
with in_purse (Alg. 2 and Alg. 3).  Each iteration moves every predicted
keypoint onto its ball or ellipse (radial projection in the Lambda metric)
and refits the pose; a final feasibility test keeps the sample, or pulls it
back towards a feasible anchor by bisection so that the kept pose is the one
still in S (Step II, last bullet).

Units: 3D-3D in metres with Lambda = I; 2D-3D residuals in pixels through the
pinhole K, Lambda in px^-2, beta dimensionless.
"""
import math
from typing import Optional

import numpy as np
import torch

from .params import OracleParams
from .philox import trajectory_uniforms
from .so3 import exp_so3, hat, log_so3, proj_so3

DT = torch.float64

KIND_3D3D = 0
KIND_2D3D = 1

STATUS_OK = 0
STATUS_EMPTY = 1
STATUS_BAD_SHAPE = 2
STATUS_FIT_FAILED = 3
STATUS_BAD_SIZE = 4
FLAG_NO_ANCHOR = 1 << 8
FLAG_ANCHOR_ITERATED = 1 << 9

MASK_FEASIBLE = 1
MASK_PULLED_IN = 2
MASK_FAILED = 4


def _t(x) -> torch.Tensor:
    """float64 tensor; torch inputs keep their autograd graph."""
    if isinstance(x, torch.Tensor):
        return x.to(DT)
    return torch.as_tensor(np.asarray(x), dtype=DT)


class Problem:
    """One PURSE instance as float64 tensors."""

    def __init__(self, kind, model_pts, centres, shapes, bounds, intrinsics):
        self.kind = int(kind)
        self.model = _t(model_pts).reshape(-1, 3)
        c = _t(centres)
        if c.shape[-1] == 3 and self.kind == KIND_2D3D:
            c = c[:, :2]
        self.centres = c.reshape(-1, 3) if self.kind == KIND_3D3D else c.reshape(-1, 2)
        self.shapes = _t(shapes).reshape(-1, 2, 2)
        self.beta = _t(bounds).reshape(-1)
        self.K = _t(intrinsics).reshape(4)

    @classmethod
    def from_instance(cls, inst):
        return cls(inst.kind, inst.model_pts, inst.centres, inst.shapes,
                   inst.bounds, inst.intrinsics)

    @property
    def n(self) -> int:
        return self.model.shape[0]

    def tau(self, p: OracleParams) -> float:
        return p.tau_abs_3d if self.kind == KIND_3D3D else p.tau_abs_2d


# ---------------------------------------------------------------------------
# residuals and feasibility (eqs. g-2D3D, g-3D3D, unknown-but-bounded, PURSE)

def transform(prob: Problem, R: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """Model points mapped by each pose: (M, N, 3)."""
    return torch.einsum("mij,nj->mni", R, prob.model) + t[:, None, :]


def project(prob: Problem, P: torch.Tensor) -> torch.Tensor:
    """Pinhole projection in pixels, Pi_K(v) = (fx v1/v3 + cx, fy v2/v3 + cy)."""
    fx, fy, cx, cy = prob.K
    return torch.stack([fx * P[..., 0] / P[..., 2] + cx,
                        fy * P[..., 1] / P[..., 2] + cy], -1)


def residual(prob: Problem, R, t):
    """Prediction minus measurement e_i (the negative of g) and its
    Lambda-norm r_i = sqrt(e_i^T Lambda_i e_i); also the depths (2D-3D)."""
    P = transform(prob, R, t)
    if prob.kind == KIND_3D3D:
        e = P - prob.centres
        r = torch.sqrt((e * e).sum(-1))
        return e, r, None
    u = project(prob, P)
    e = u - prob.centres
    r2 = torch.einsum("mni,nij,mnj->mn", e, prob.shapes, e)
    return e, torch.sqrt(torch.clamp(r2, min=0.0)), P[..., 2]


def feasible(prob: Problem, R, t, p: OracleParams, margin: float = 1.0):
    """in_purse with tolerance: every r_i <= margin * beta_i + tau_abs, and for
    2D-3D every keypoint in front of the camera (depth > z_min)."""
    e, r, depth = residual(prob, R, t)
    ok = (r <= margin * prob.beta + prob.tau(p)).all(-1)
    if depth is not None:
        ok = ok & (depth > p.z_min).all(-1)
    return ok


def feasibility_ratio(prob: Problem, R, t, p: OracleParams):
    """Diagnostic only (no decision uses it): max_i r_i / (beta_i + tau_abs),
    +inf where a 2D-3D depth is <= z_min.  The in_purse decision is ratio <= 1;
    how close the ratio is to 1 says how near a pose is to flipping it."""
    e, r, depth = residual(prob, R, t)
    ratio = (r / (prob.beta + prob.tau(p))).max(-1).values
    if depth is not None:
        ratio = torch.where((depth > p.z_min).all(-1), ratio, torch.full_like(ratio, math.inf))
    return ratio


DERIV_EPS = 1e-5


def project_targets(prob: Problem, e, r, kappa: float, deriv_convention: bool = False):
    """Move every predicted keypoint onto its ball/ellipse shrunk by kappa:
    q_i = centre_i + s_i e_i with s_i = 1 if r_i <= kappa beta_i else
    kappa beta_i / r_i (the nearest point of the set in the Lambda metric).

    deriv_convention: the map used for derivatives, where a constraint within
    DERIV_EPS (relative) inside its shrunk ball counts as projected.  Converged
    trajectories end on that boundary, approaching it from outside, so their
    clamp sits on its kink to rounding; this side is the one the limit takes."""
    kb = kappa * prob.beta
    inside = r <= kb
    if deriv_convention:
        inside = r <= kb * (1.0 - DERIV_EPS)
    s = torch.where(inside, torch.ones_like(r), kb / torch.where(inside, torch.ones_like(r), r))
    return prob.centres + s[..., None] * e


# ---------------------------------------------------------------------------
# closed-form refit (3D-3D) and Gauss-Newton refit (2D-3D)

def kabsch(a: torch.Tensor, q: torch.Tensor):
    """Arun's least-squares rigid fit of model points a (N,3) to targets
    q (M,N,3): R = proj_SO3(sum (q_i - q_bar)(a_i - a_bar)^T), t = q_bar - R a_bar."""
    abar = a.mean(0)
    qbar = q.mean(1)
    H = torch.einsum("mni,nj->mij", q - qbar[:, None, :], a - abar)
    R = proj_so3(H)
    t = qbar - torch.einsum("mij,j->mi", R, abar)
    return R, t


def gn_step_2d(prob: Problem, R, t, q, o, z_min: float, return_delta: bool = False):
    """One undamped Gauss-Newton step on sum_i ||q_i - Pi_K(R Z_i + t)||^2_Lambda_i
    with the left update about the pivot o:
      R <- Exp(dw) R,  t <- Exp(dw)(t - o) + o + dv,
    J_i = dPi/dP * [ -[P_i - o]_x | I ], A = sum J^T Lambda J, g = sum J^T Lambda (q - u),
    A delta = g by Cholesky.  Returns (R, t, ok) (and delta if asked); ok is
    False where a depth is <= z_min or A is not positive definite."""
    fx, fy = prob.K[0], prob.K[1]
    P = transform(prob, R, t)
    X, Y, Z = P[..., 0], P[..., 1], P[..., 2]
    ok = (Z > z_min).all(-1)
    Zs = torch.where(Z > z_min, Z, torch.ones_like(Z))
    u = project(prob, torch.stack([X, Y, Zs], -1))
    res = q - u
    zero = torch.zeros_like(X)
    D = torch.stack([torch.stack([fx / Zs, zero, -fx * X / (Zs * Zs)], -1),
                     torch.stack([zero, fy / Zs, -fy * Y / (Zs * Zs)], -1)], -2)
    G = torch.cat([-hat(P - o[:, None, :]),
                   torch.eye(3, dtype=DT).expand(P.shape[:-1] + (3, 3))], -1)
    J = D @ G                                               # (M,N,2,6)
    LJ = prob.shapes @ J                                    # Lambda J
    A = torch.einsum("mnki,mnkj->mij", J, LJ)
    g = torch.einsum("mnki,mnk->mi", LJ, res)
    L, info = torch.linalg.cholesky_ex(A)
    ok = ok & (info == 0)
    eye6 = torch.eye(6, dtype=DT).expand(A.shape)
    L = torch.where((info == 0)[:, None, None], L, eye6)
    delta = torch.cholesky_solve(g[..., None], L)[..., 0]
    E = exp_so3(delta[:, :3])
    Rn = E @ R
    tn = torch.einsum("mij,mj->mi", E, t - o) + o + delta[:, 3:]
    if return_delta:
        return Rn, tn, ok, delta
    return Rn, tn, ok


# ---------------------------------------------------------------------------
# per-instance prologue: centre fit, pivot, anchor

def dlt_2d(prob: Problem):
    """Direct linear transform in normalised coordinates: the null vector of
    the 2N x 12 system x_i (p3 . Zh_i) - p1 . Zh_i = 0, y_i (p3 . Zh_i) -
    p2 . Zh_i = 0; sign fixed so det(P[:, :3]) > 0, then R = proj_SO3 and
    t = P[:, 3] / scale with scale the mean singular value of P[:, :3]."""
    fx, fy, cx, cy = prob.K
    xn = (prob.centres[:, 0] - cx) / fx
    yn = (prob.centres[:, 1] - cy) / fy
    Zh = torch.cat([prob.model, torch.ones(prob.n, 1, dtype=DT)], 1)
    zero = torch.zeros_like(Zh)
    A = torch.cat([torch.cat([-Zh, zero, xn[:, None] * Zh], 1),
                   torch.cat([zero, -Zh, yn[:, None] * Zh], 1)], 0)
    _, _, Vh = torch.linalg.svd(A)
    Pm = Vh[-1].reshape(3, 4)
    if torch.linalg.det(Pm[:, :3]) < 0:
        Pm = -Pm
    s = torch.linalg.svdvals(Pm[:, :3]).mean()
    return proj_so3(Pm[:, :3]), Pm[:, 3] / s


def affine_2d(prob: Problem):
    """Weak-perspective initialisation: least-squares fit of the normalised
    image points by x_n = A Z + b (a scaled orthographic camera, which the
    object's small depth range makes a good model); s = mean row norm of A,
    R = proj_SO3 of the rows of A/s and their cross product, t = (b/s, 1/s)."""
    fx, fy, cx, cy = prob.K
    xn = torch.stack([(prob.centres[:, 0] - cx) / fx, (prob.centres[:, 1] - cy) / fy], 1)
    X = torch.cat([prob.model, torch.ones(prob.n, 1, dtype=DT)], 1)
    sol = torch.linalg.lstsq(X, xn).solution            # (4, 2)
    A = sol[:3].T
    b = sol[3]
    s = 0.5 * (torch.linalg.norm(A[0]) + torch.linalg.norm(A[1]))
    r3 = torch.linalg.cross(A[0], A[1]) / (s * s)
    R = proj_so3(torch.stack([A[0] / s, A[1] / s, r3]))
    t = torch.cat([b / s, (1.0 / s).reshape(1)])
    return R, t


def gn_cost_2d(prob: Problem, R, t) -> float:
    e, r, depth = residual(prob, R[None], t[None])
    return float((r * r).sum().detach())


def centre_fit(prob: Problem, p: OracleParams):
    """Maximum-likelihood centre x_c (eq. MLE with rho = ||.||^2_Lambda).
    3D-3D: Arun's method on all N pairs.  2D-3D: Gauss-Newton steps towards
    the ellipse centres, each about the pivot R Zbar + t of the current pose,
    run to convergence (until the step has |dw|_inf <= centre_tol and
    |dv|_inf <= centre_tol (1 + |t|_inf), at most `centre_gn` steps), from two
    initialisations, the DLT and the weak-perspective fit; the successful fit
    with the lower cost is kept (ties: the DLT one).  Returns (R, t, ok)."""
    if prob.kind == KIND_3D3D:
        R, t = kabsch(prob.model, prob.centres[None])
        return R[0], t[0], True
    best = None
    zbar = prob.model.mean(0)
    # the initialisations only start the fit; their influence is below rounding
    # after the Gauss-Newton steps, and derivatives are taken at the converged fit
    for init in (dlt_2d, affine_2d):
        R, t = init(prob)
        R, t = R.detach()[None], t.detach()[None]
        ok = True
        for _ in range(p.centre_gn):
            o = R @ zbar + t
            R, t, okk, delta = gn_step_2d(prob, R, t, prob.centres[None], o, p.z_min, return_delta=True)
            ok = ok and bool(okk.all())
            if not ok:
                break
            dw = float(delta[0, :3].detach().abs().max())
            dv = float(delta[0, 3:].detach().abs().max())
            if dw <= p.centre_tol and dv <= p.centre_tol * (1.0 + float(t.detach().abs().max())):
                break
        P = transform(prob, R, t)
        ok = ok and bool((P[..., 2] > p.z_min).all())
        if ok:
            cost = gn_cost_2d(prob, R[0], t[0])
            if best is None or cost < best[2]:
                best = (R[0], t[0], cost)
    if best is None:
        return R[0], t[0], False
    return best[0], best[1], True


def check_instance(prob: Problem) -> int:
    n_min = 3 if prob.kind == KIND_3D3D else 6
    if prob.n < n_min:
        return STATUS_BAD_SIZE
    vals = [prob.model, prob.centres, prob.beta]
    if prob.kind == KIND_2D3D:
        vals += [prob.shapes, prob.K]
    if not all(bool(torch.isfinite(v).all()) for v in vals):
        return STATUS_BAD_SHAPE
    if bool((prob.beta < 0).any()):
        return STATUS_BAD_SHAPE
    if prob.kind == KIND_2D3D:
        L = prob.shapes
        if bool((L[:, 0, 1] != L[:, 1, 0]).any()):
            return STATUS_BAD_SHAPE
        det = L[:, 0, 0] * L[:, 1, 1] - L[:, 0, 1] * L[:, 1, 0]
        if bool((L[:, 0, 0] <= 0).any() or (det <= 0).any()):
            return STATUS_BAD_SHAPE
        if bool(prob.K[0] <= 0) or bool(prob.K[1] <= 0):
            return STATUS_BAD_SHAPE
    return STATUS_OK


def prologue(prob: Problem, p: OracleParams) -> dict:
    """Centre x_c, pivot o_c = R_c mean(model) + t_c, and the anchor: x_c
    itself if every r_i(x_c) <= kappa beta_i + tau, else the end of one
    trajectory run from x_c with no offset if it passes the same test, else
    none."""
    st = check_instance(prob)
    if st != STATUS_OK:
        return dict(status=st)
    Rc, tc, ok = centre_fit(prob, p)
    if not ok:
        return dict(status=STATUS_FIT_FAILED, R_c=Rc, t_c=tc)
    oc = Rc @ prob.model.mean(0) + tc
    status = STATUS_OK
    if bool(feasible(prob, Rc[None], tc[None], p, margin=p.kappa)[0]):
        Ra, ta = Rc, tc
    else:
        status |= FLAG_ANCHOR_ITERATED
        Ri, ti, failed = run_trajectories(prob, Rc[None], tc[None], oc, p)
        if (not bool(failed[0])) and bool(feasible(prob, Ri, ti, p, margin=p.kappa)[0]):
            Ra, ta = Ri[0], ti[0]
        else:
            Ra, ta = None, None
            status |= FLAG_NO_ANCHOR
    return dict(status=status, R_c=Rc, t_c=tc, o_c=oc, R_a=Ra, t_a=ta)


# ---------------------------------------------------------------------------
# trajectories

def initial_poses(pro: dict, p: OracleParams, seed: int, ids: np.ndarray):
    """Random start of each trajectory ("Walk away from the center", Step II):
    a direction u on S^2 from two Philox uniforms (z = 1 - 2 U1,
    phi = 2 pi U2); even trajectories rotate the object about its centroid by
    omega0 u (rotation-seeking), odd ones shift it by v0 u (translation-
    seeking): x0 = (Exp(w) R_c, Exp(w)(t_c - o_c) + o_c + v)."""
    u1, u2 = trajectory_uniforms(seed, ids)
    z = torch.as_tensor(1.0 - 2.0 * u1, dtype=DT)
    phi = torch.as_tensor(2.0 * math.pi * u2, dtype=DT)
    rho = torch.sqrt(torch.clamp(1.0 - z * z, min=0.0))
    d = torch.stack([rho * torch.cos(phi), rho * torch.sin(phi), z], -1)
    even = torch.as_tensor(np.asarray(ids) % 2 == 0)[:, None]
    w = torch.where(even, p.omega0 * d, torch.zeros_like(d))
    v = torch.where(even, torch.zeros_like(d), p.v0 * d)
    E = exp_so3(w)
    R0 = E @ pro["R_c"]
    t0 = torch.einsum("mij,j->mi", E, pro["t_c"] - pro["o_c"]) + pro["o_c"] + v
    return R0, t0


def run_trajectories(prob: Problem, R, t, o_c, p: OracleParams, deriv_convention: bool = False,
                     margins=None):
    """n_iters alternating iterations from (R, t): project every keypoint onto
    its constraint (shrunk by kappa), then refit the pose (Arun for 3D-3D,
    n_gn Gauss-Newton steps about o_c for 2D-3D).  A 2D-3D trajectory whose
    Gauss-Newton step fails is frozen and flagged.
    margins (a list): receives, per trajectory, the smallest relative margin
    |r_i / threshold_i - 1| of the projection decisions over all iterations
    and keypoints (the threshold of project_targets under the same
    convention; diagnostic)."""
    M = R.shape[0]
    failed = torch.zeros(M, dtype=torch.bool)
    o = o_c.expand(M, 3)
    closest = torch.full((M,), math.inf, dtype=DT)
    for _ in range(p.n_iters):
        e, r, _ = residual(prob, R, t)
        if margins is not None:
            thr = p.kappa * prob.beta * ((1.0 - DERIV_EPS) if deriv_convention else 1.0)
            with torch.no_grad():
                closest = torch.minimum(closest, (r / thr - 1.0).abs().min(-1).values)
        q = project_targets(prob, e, r, p.kappa, deriv_convention)
        if prob.kind == KIND_3D3D:
            R, t = kabsch(prob.model, q)
        else:
            for _g in range(p.n_gn):
                Rn, tn, ok = gn_step_2d(prob, R, t, q, o, p.z_min)
                failed = failed | ~ok
                R = torch.where(failed[:, None, None], R, Rn)
                t = torch.where(failed[:, None], t, tn)
    if margins is not None:
        margins.append(closest)
    return R, t, failed


def pull_in(prob: Problem, Ra, ta, R, t, p: OracleParams, lo_fixed=None, margins=None, margin_steps=None):
    """Bisection on the geodesic segment x(l) = (R_a Exp(l Log(R_a^T R)),
    t_a + l (t - t_a)) from the feasible anchor (l = 0) to the infeasible end
    (l = 1); returns x(lo) after n_bis steps, which is in S, and lo.  With
    lo_fixed the bisection's outcome is taken as given (frozen decisions).
    margins (a list): receives, per trajectory, the smallest |ratio - 1| of
    the bisection's feasibility tests, or of its first margin_steps tests
    when given (diagnostic)."""
    w = log_so3(Ra.transpose(-1, -2) @ R)
    M = R.shape[0]
    if lo_fixed is None:
        lo = torch.zeros(M, dtype=DT)
        hi = torch.ones(M, dtype=DT)
        closest = torch.full((M,), math.inf, dtype=DT)
        with torch.no_grad():
            for step in range(p.n_bis):
                mid = 0.5 * (lo + hi)
                Rm = Ra @ exp_so3(mid[:, None] * w)
                tm = ta + mid[:, None] * (t - ta)
                f = feasible(prob, Rm, tm, p)
                if margins is not None and (margin_steps is None or step < margin_steps):
                    closest = torch.minimum(closest, (feasibility_ratio(prob, Rm, tm, p) - 1.0).abs())
                lo = torch.where(f, mid, lo)
                hi = torch.where(f, hi, mid)
        if margins is not None:
            margins.append(closest)
    else:
        lo = torch.as_tensor(np.asarray(lo_fixed), dtype=DT)
    return Ra @ exp_so3(lo[:, None] * w), ta + lo[:, None] * (t - ta), lo


def sample(prob: Problem, p: OracleParams, seed: int, n_samples: int,
           sample_ids: Optional[np.ndarray] = None, pro: Optional[dict] = None,
           diagnostics: bool = False) -> dict:
    """All trajectories of one instance.  Returns poses (M,12) as
    [R row-major | t], mask bits (feasible 1, pulled-in 2, failed 4) and the
    prologue record.  With diagnostics, also how close each trajectory's
    decisions were to flipping: end_margin = |ratio - 1| of the final in_purse
    test and bis_margin = the smallest |ratio - 1| of its bisection tests
    (inf where it was not pulled in), ratio being max_i r_i / (beta_i + tau)."""
    ids = np.arange(n_samples, dtype=np.uint64) if sample_ids is None else \
        np.asarray(sample_ids, dtype=np.uint64)
    M = len(ids)
    if pro is None:
        pro = prologue(prob, p)
    st = pro["status"] & 0xFF
    if st != STATUS_OK:
        return dict(poses=torch.zeros(M, 12, dtype=DT), mask=torch.zeros(M, dtype=torch.uint8),
                    prologue=pro, status=pro["status"])
    R0, t0 = initial_poses(pro, p, seed, ids)
    R, t, failed = run_trajectories(prob, R0, t0, pro["o_c"], p)
    feas = feasible(prob, R, t, p) & ~failed
    diag = {}
    if diagnostics:
        diag["end_margin"] = (feasibility_ratio(prob, R, t, p) - 1.0).abs()
        diag["bis_margin"] = torch.full((M,), math.inf, dtype=DT)
    mask = torch.where(feas, MASK_FEASIBLE, 0)
    mask = torch.where(failed, MASK_FAILED, mask)
    need = ~feas & ~failed
    lo_out = torch.full((M,), -1.0, dtype=DT)
    if pro["R_a"] is not None and bool(need.any()):
        idx = torch.nonzero(need)[:, 0]
        margins = [] if diagnostics else None
        Rb, tb, lo = pull_in(prob, pro["R_a"], pro["t_a"], R[idx], t[idx], p, margins=margins)
        if diagnostics:
            diag["bis_margin"][idx] = margins[0]
        R = R.clone()
        t = t.clone()
        R[idx] = Rb
        t[idx] = tb
        lo_out[idx] = lo
        mask[idx] = MASK_FEASIBLE | MASK_PULLED_IN
    poses = torch.cat([R.reshape(M, 9), t], 1)
    return dict(poses=poses, mask=mask.to(torch.uint8), prologue=pro,
                status=pro["status"], lo=lo_out, **diag)
