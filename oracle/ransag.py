"""Step I of the paper ("The CLOSURE Algorithm"): candidate start poses, kept
when they lie in S (random sample averaging, RANSAG, for the keypoint sets;
the convex-combination sampler for the pose-regression set, oracle/reg.py).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

3D-3D: each trial picks 3 distinct correspondences, a random point inside
each of their balls, and fits the pose to the three pairs by Arun's method
(the least-squares rigid fit, oracle/purse.py kabsch); the candidate is kept
if it satisfies eq. PURSE3D3D (with the sampler's tolerance).

2D-3D: each trial picks 3 distinct correspondences and a random point inside
each of their ellipses, and solves the perspective-3-point problem for the
three bearing rays (oracle p3p); every real solution in front of the camera is
a candidate (so a trial gives up to four), kept if it satisfies eq.
PURSE2D3D.  The GPU keeps the first in-S solution per trial in the solver's
order; the oracle returns all of them.

Random numbers (readings): Philox4x64-10, key (seed, 4), counter
(trial, k, 0, 0); k = 0 picks the correspondences (i1 = floor(U1 N),
i2 = floor(U2 (N - 1)), i3 = floor(U3 (N - 2)), each skipping the indices
already taken, in increasing order), k = 1, 2, 3 the point in the k-th
constraint: a direction (z = 1 - 2 U1, phi = 2 pi U2) and a radius fraction
U3^(1/3) (uniform in the 3D ball); in an ellipse e^T Lambda e <= beta^2 the
point is z + beta sqrt(U3) U^-1 (cos 2 pi U2, sin 2 pi U2) with U^T U =
Lambda (uniform in the ellipse).  Uniforms are the top 24 bits of output
words 0, 1, 2.

P3P (the minimal solver the paper names for 2D-3D): with bearing unit
vectors f_k, model points P_k, side lengths a = |P2 - P3|, b = |P1 - P3|,
c = |P1 - P2| and cosines ca = f2.f3, cb = f1.f3, cg = f1.f2, the depths
s_k along the rays satisfy the law of cosines for each pair; with s2 = u s1,
s3 = v s1, dividing pairs of them gives
u = N(v) / D(v), N = K (1 + v^2 - 2 v cb) + 1 - v^2, D = 2 (cg - v ca),
K = (a^2 - c^2) / b^2, and the quartic
D^2 + N^2 - 2 cg N D - (c^2 / b^2)(1 + v^2 - 2 v cb) D^2 = 0 in v
(derived here; the classical three-point formulation).  Each real root with
u, v > 0 gives s1 = b / sqrt(1 + v^2 - 2 v cb), the camera points s_k f_k,
and the pose by Arun's method on the three pairs.  Candidates are taken in
increasing v; the GPU keeps the first that lies in S.
"""
import math

import numpy as np
import torch

from .philox import philox4x64_10
from .purse import KIND_3D3D, Problem, feasible, kabsch
from .params import OracleParams

DT = torch.float64


def trial_uniforms(seed: int, trials, k: int):
    t = np.asarray(trials, dtype=np.uint64)
    kk = np.full_like(t, k)
    z = np.zeros_like(t)
    out = philox4x64_10((t, kk, z, z), (np.uint64(seed), np.uint64(4)))
    return [(out[q] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24 for q in range(3)]


def pick_three(seed: int, trials, n: int):
    """(T, 3) distinct correspondence indices."""
    u1, u2, u3 = trial_uniforms(seed, trials, 0)
    out = np.zeros((len(u1), 3), dtype=np.int64)
    for r in range(len(u1)):
        taken = []
        for q, u in enumerate((u1[r], u2[r], u3[r])):
            x = int(math.floor(u * (n - q)))
            for t_ in sorted(taken):
                if x >= t_:
                    x += 1
            taken.append(x)
        out[r] = taken
    return out


def ball_points(seed: int, trials, k: int):
    """Offsets of a random point in the unit ball, for the k-th constraint."""
    u1, u2, u3 = trial_uniforms(seed, trials, k)
    z = 1.0 - 2.0 * u1
    phi = 2.0 * math.pi * u2
    rho = np.sqrt(np.maximum(1.0 - z * z, 0.0))
    d = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], -1)
    return d * np.cbrt(u3)[:, None]


def ransag_3d(prob: Problem, p: OracleParams, seed: int, n_trials: int):
    """3D-3D trials: poses (T, 12) and the in-S mask."""
    assert prob.kind == KIND_3D3D
    T = n_trials
    trials = np.arange(T)
    idx = pick_three(seed, trials, prob.n)
    q = torch.zeros(T, 3, 3, dtype=DT)
    a = torch.zeros(T, 3, 3, dtype=DT)
    for k in range(3):
        off = torch.as_tensor(ball_points(seed, trials, k + 1), dtype=DT)
        ii = torch.as_tensor(idx[:, k])
        q[:, k] = prob.centres[ii] + prob.beta[ii][:, None] * off
        a[:, k] = prob.model[ii]
    R = torch.zeros(T, 3, 3, dtype=DT)
    t = torch.zeros(T, 3, dtype=DT)
    for r in range(T):
        Rr, tr = kabsch(a[r], q[r][None])
        R[r], t[r] = Rr[0], tr[0]
    ok = feasible(prob, R, t, p)
    return torch.cat([R.reshape(T, 9), t], 1), ok.to(torch.uint8), idx


def ellipse_points(seed: int, trials, k: int, shapes, beta):
    """Offsets (pixels) of a random point in the ellipse e^T Lambda e <= beta^2
    of the k-th picked constraint; shapes (T, 2, 2), beta (T,)."""
    _, u2, u3 = trial_uniforms(seed, trials, k)
    y = np.stack([np.cos(2 * math.pi * u2), np.sin(2 * math.pi * u2)], -1) * (np.sqrt(u3) * beta)[:, None]
    out = np.zeros_like(y)
    for r in range(len(y)):
        U = np.linalg.cholesky(shapes[r]).T          # U^T U = Lambda, U upper triangular
        out[r] = np.linalg.solve(U, y[r])
    return out


def _pmul(a, b):
    return np.convolve(a, b)


def _padd(*ps):
    n = max(len(p) for p in ps)
    out = np.zeros(n)
    for p in ps:
        out[n - len(p):] += p
    return out


def p3p(f, P):
    """Solutions of the perspective-3-point problem: bearing unit vectors f
    (3, 3) (rows) and model points P (3, 3); returns [(v, R, t)] for the real
    roots with positive depths, in increasing v."""
    a = np.linalg.norm(P[1] - P[2])
    b = np.linalg.norm(P[0] - P[2])
    c = np.linalg.norm(P[0] - P[1])
    ca, cb, cg = f[1] @ f[2], f[0] @ f[2], f[0] @ f[1]
    K = (a * a - c * c) / (b * b)
    # polynomials in v, highest degree first
    q = np.array([1.0, -2.0 * cb, 1.0])                   # 1 + v^2 - 2 v cb
    N = _padd(K * q, np.array([-1.0, 0.0, 1.0]))          # K q + 1 - v^2
    D = np.array([-2.0 * ca, 2.0 * cg])                   # 2 (cg - v ca)
    quartic = _padd(_pmul(D, D), _pmul(N, N), -2.0 * cg * _pmul(N, D), -(c * c) / (b * b) * _pmul(q, _pmul(D, D)))
    dq = np.polyder(quartic)
    out = []
    for v in sorted(r.real for r in np.roots(quartic) if abs(r.imag) <= 1e-9 * max(1.0, abs(r))):
        for _ in range(4):  # Newton polish of the eigenvalue root
            dv = np.polyval(dq, v)
            if dv != 0:
                v = v - np.polyval(quartic, v) / dv
        if v <= 0:
            continue
        Dv = np.polyval(D, v)
        if abs(Dv) < 1e-14:
            continue
        u = np.polyval(N, v) / Dv
        qv = np.polyval(q, v)
        if u <= 0 or qv <= 0:
            continue
        s1 = b / math.sqrt(qv)
        X = np.stack([s1 * f[0], u * s1 * f[1], v * s1 * f[2]])
        R, t = kabsch(torch.as_tensor(P, dtype=DT), torch.as_tensor(X, dtype=DT)[None])
        out.append((float(v), R[0], t[0]))
    return out


def bearings(prob: Problem, pix):
    """Unit bearing vectors of pixel points (T, 2) through the pinhole K."""
    fx, fy, cx, cy = [float(x) for x in prob.K]
    d = np.stack([(pix[:, 0] - cx) / fx, (pix[:, 1] - cy) / fy, np.ones(len(pix))], -1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def ransag_2d(prob: Problem, p: OracleParams, seed: int, n_trials: int):
    """2D-3D trials: for each, every P3P solution in increasing v with its
    in-S bit; also the pose the GPU keeps (the first in S) and its mask."""
    T = n_trials
    trials = np.arange(T)
    idx = pick_three(seed, trials, prob.n)
    z = prob.centres.numpy()
    L = prob.shapes.numpy()
    beta = prob.beta.numpy()
    pix = np.zeros((T, 3, 2))
    for k in range(3):
        ii = idx[:, k]
        pix[:, k] = z[ii] + ellipse_points(seed, trials, k + 1, L[ii], beta[ii])
    poses = torch.zeros(T, 12, dtype=DT)
    mask = torch.zeros(T, dtype=torch.uint8)
    sols = []
    for r in range(T):
        f = bearings(prob, pix[r])
        cand = p3p(f, prob.model.numpy()[idx[r]])
        row = []
        for v, R, t in cand:
            ok = bool(feasible(prob, R[None], t[None], p)[0])
            row.append((v, R, t, ok))
            if ok and mask[r] == 0:
                poses[r] = torch.cat([R.reshape(9), t])
                mask[r] = 1
        sols.append(row)
    return poses, mask, idx, sols, pix
