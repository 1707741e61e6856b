"""Pins of the oracle's strategic random walk (oracle/walk.py, the paper's
Step II samplers) against properties the algorithm fixes (no GPU):

- the ranking keeps the N_P* largest boundary distances, ties in index order;
- the boundary distance is min_i (beta_i - r_i) on constructed geometry;
- a rotation-mode walk only ever turns about its velocity's axis, so its end
  is Exp(w s) R0 with s the sum of the accepted step scales, at geodesic
  angle |w| s from the start; a translation-mode walk ends at t0 + v s;
- every end pose is in S, re-checked from the residual definition;
- the walk equals a literal per-walk, per-perturbation, per-scale loop of
  the sequential samplers (brute force on a tiny instance): same decisions
  and poses.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import walk as WK
from oracle.philox import philox4x64_10
from oracle.purse import KIND_2D3D, KIND_3D3D, Problem, feasible, prologue, sample
from oracle.params import OracleParams
from paper_2403_09990_amd import workloads as W

DT = torch.float64


def test_top_k_keeps_the_largest_in_rank_order():
    rng = np.random.default_rng(0)
    for _ in range(50):
        n, k = int(rng.integers(5, 40)), int(rng.integers(1, 5))
        d = rng.integers(0, 6, size=(3, n)).astype(np.float64)   # many ties
        got = WK.top_k(torch.as_tensor(d), k).numpy()
        for row in range(3):
            ref = sorted(range(n), key=lambda j: (-d[row, j], j))[:k]
            assert got[row].tolist() == ref


def test_boundary_distance_on_constructed_balls():
    """3D-3D: keypoints at known distances s_i beta_i from their ball
    centres give dist = min_i beta_i (1 - s_i)."""
    rng = np.random.default_rng(1)
    a = rng.uniform(-1, 1, size=(6, 3))
    u = rng.normal(size=(6, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    beta = rng.uniform(0.02, 0.1, size=6)
    s = np.array([0.2, 0.9, 0.5, 1.3, 0.1, 0.7])
    prob = Problem(KIND_3D3D, a, a + (s * beta)[:, None] * u, np.tile([1.0, 0, 0, 1.0], (6, 1)), beta, np.zeros(4))
    d = WK.boundary_distance(prob, torch.eye(3, dtype=DT)[None], torch.zeros(1, 3, dtype=DT))
    assert abs(float(d[0]) - float((beta * (1 - s)).min())) < 1e-14


def test_walk_uniforms_follow_the_counter_layout():
    """Key (seed, 1 + mode), counter (walk, iteration, perturbation, 0); the
    three uniforms are the top 24 bits of words 0..2."""
    u = WK.walk_uniforms(7, WK.MODE_T, np.array([3, 4]), 2, np.array([9, 9]))
    out = philox4x64_10((np.array([3, 4], dtype=np.uint64), np.array([2, 2], dtype=np.uint64),
                         np.array([9, 9], dtype=np.uint64), np.zeros(2, dtype=np.uint64)),
                        (np.uint64(7), np.uint64(2)))
    for k in range(3):
        assert np.array_equal(u[k], (out[k] >> np.uint64(40)).astype(np.float64) / 2 ** 24)
        assert (u[k] >= 0).all() and (u[k] < 1).all()


def _starts(inst, n, iters=40):
    """Feasible start poses: ends of the alternating sampler (any points of S
    serve as S0)."""
    prob = Problem.from_instance(inst)
    out = sample(prob, OracleParams(n_iters=iters), inst.seed, n)
    keep = (out["mask"] & 1) != 0
    P = out["poses"][keep]
    return prob, P[:, :9].reshape(-1, 3, 3), P[:, 9:]


def _angle(A, B):
    return Rotation.from_matrix((A @ B.transpose(-1, -2)).numpy()).magnitude()


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_rotation_walk_turns_about_its_velocity_axis(kind):
    rng = np.random.default_rng(2)
    inst = W.make_2d3d(rng, 10, 2.0, (5.0, 20.0), 64) if kind == "2d" else W.make_3d3d(rng, 8, 0.01, 0.05, 64)
    prob, R0, t0 = _starts(inst, 32)
    wp = WK.WalkParams(n_iters=6, n_perturb=40, n_keep=5, n_scales=12, t_pert=0.002 if kind == "2d" else 0.005)
    out = WK.walk(prob, R0, t0, 11, WK.MODE_R, wp)
    Rend = out["poses"][:, :9].reshape(-1, 3, 3)
    # Exp(w s) R0
    ref = WK.exp_so3(out["velocity"] * out["steps"][:, None]) @ out["start_R"]
    assert float((Rend - ref).abs().max()) < 1e-12
    # at geodesic angle |w| s from the start (all below pi here)
    ang = _angle(Rend, out["start_R"])
    expect = (out["velocity"].norm(dim=-1) * out["steps"]).numpy()
    assert np.all(expect < math.pi)
    assert np.abs(ang - expect).max() < 1e-9
    assert (out["decisions"] >= 0).any()
    # every end pose is in S (residuals from the problem's definition)
    p = OracleParams(tau_abs_2d=wp.tau_abs_2d, tau_abs_3d=wp.tau_abs_3d, z_min=wp.z_min)
    assert bool(feasible(prob, Rend, out["poses"][:, 9:], p).all())
    assert bool((out["mask"] == 1).all())


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_translation_walk_moves_along_its_velocity(kind):
    rng = np.random.default_rng(3)
    inst = W.make_2d3d(rng, 10, 2.0, (5.0, 20.0), 64) if kind == "2d" else W.make_3d3d(rng, 8, 0.01, 0.05, 64)
    prob, R0, t0 = _starts(inst, 32)
    wp = WK.WalkParams(n_iters=6, n_perturb=40, n_keep=5, n_scales=12, v0=0.02)
    out = WK.walk(prob, R0, t0, 12, WK.MODE_T, wp)
    tend = out["poses"][:, 9:]
    ref = out["start_t"] + out["velocity"] * out["steps"][:, None]
    assert float((tend - ref).abs().max()) < 1e-13
    assert (out["steps"] > 0).any()
    p = OracleParams(tau_abs_2d=wp.tau_abs_2d, tau_abs_3d=wp.tau_abs_3d, z_min=wp.z_min)
    assert bool(feasible(prob, out["poses"][:, :9].reshape(-1, 3, 3), tend, p).all())


def _np_exp(w):
    th = np.linalg.norm(w)
    if th < 1e-12:
        return np.eye(3)
    k = w / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx


def _np_radii(kind, a, c, L, K, R, t):
    """r_i and depths of one pose, written out per keypoint."""
    r, z = [], []
    for i in range(len(a)):
        p = R @ a[i] + t
        if kind == KIND_3D3D:
            e = p - c[i]
            r.append(math.sqrt(e @ e))
            z.append(1.0)
        else:
            u = np.array([K[0] * p[0] / p[2] + K[2], K[1] * p[1] / p[2] + K[3]])
            e = u - c[i][:2]
            r.append(math.sqrt(e @ L[i].reshape(2, 2) @ e))
            z.append(p[2])
    return np.array(r), np.array(z)


@pytest.mark.parametrize("kind,mode", [("3d", WK.MODE_R), ("3d", WK.MODE_T), ("2d", WK.MODE_R), ("2d", WK.MODE_T)])
def test_walk_equals_the_sequential_sampler_loops(kind, mode):
    """Brute force: the sequential samplers' loops written out per walk,
    perturbation, kept rank and scale, with the same random draws."""
    rng = np.random.default_rng(4)
    inst = W.make_2d3d(rng, 7, 2.0, (5.0, 20.0), 16) if kind == "2d" else W.make_3d3d(rng, 5, 0.01, 0.05, 16)
    prob, R0, t0 = _starts(inst, 6, iters=30)
    wp = WK.WalkParams(n_walks=2, n_iters=3, n_perturb=9, n_keep=3, n_scales=5, t_pert=0.003, r_pert=0.01,
                       v0=0.02)
    seed = 5
    out = WK.walk(prob, R0, t0, seed, mode, wp)
    a = prob.model.numpy()
    c = prob.centres.numpy()
    L = prob.shapes.numpy().reshape(-1, 4)
    Kc = prob.K.numpy()
    beta = prob.beta.numpy()
    tau = wp.tau_abs_2d if prob.kind == KIND_2D3D else wp.tau_abs_3d
    Rbar = WK.proj_so3(R0.sum(0)).numpy()
    tbar = t0.mean(0).numpy()
    for s in range(R0.shape[0]):
        for n in range(wp.n_walks):
            w = s * wp.n_walks + n
            Rs, ts = R0[s].numpy().copy(), t0[s].numpy().copy()
            u1, u2, _ = WK.walk_uniforms(seed, mode, np.array([w]), WK.INIT_ITER, np.array([0]))
            z = 1 - 2 * u1[0]
            rnd = np.array([math.sqrt(max(0.0, 1 - z * z)) * math.cos(2 * math.pi * u2[0]),
                            math.sqrt(max(0.0, 1 - z * z)) * math.sin(2 * math.pi * u2[0]), z])
            if mode == WK.MODE_R:
                ax = Rotation.from_matrix(Rs @ Rbar.T).as_rotvec()
                vel = wp.omega0 * ((ax / np.linalg.norm(ax) if np.linalg.norm(ax) > 0 else 0 * ax) + rnd)
            else:
                dv = ts - tbar
                vel = wp.v0 * ((dv / np.linalg.norm(dv) if np.linalg.norm(dv) > 0 else 0 * dv) + rnd)
            for i in range(wp.n_iters):
                cand = []
                for j in range(wp.n_perturb):
                    q1, q2, q3 = WK.walk_uniforms(seed, mode, np.array([w]), i, np.array([j]))
                    z = 1 - 2 * q1[0]
                    dirn = np.array([math.sqrt(max(0.0, 1 - z * z)) * math.cos(2 * math.pi * q2[0]),
                                     math.sqrt(max(0.0, 1 - z * z)) * math.sin(2 * math.pi * q2[0]), z])
                    if mode == WK.MODE_R:
                        Rj, tj = Rs, ts + wp.t_pert * q3[0] * dirn
                    else:
                        Rj, tj = _np_exp(wp.r_pert * q3[0] * dirn) @ Rs, ts
                    r, _ = _np_radii(prob.kind, a, c, L, Kc, Rj, tj)
                    cand.append((float((beta - r).min()), j, Rj, tj))
                kept = sorted(cand, key=lambda x: (-x[0], x[1]))[:wp.n_keep]
                moved = None
                for m in range(wp.n_scales):
                    for k in range(wp.n_keep):
                        _, _, Rj, tj = kept[k]
                        if mode == WK.MODE_R:
                            Rc, tc = _np_exp(vel * wp.gamma ** m) @ Rs, tj
                        else:
                            Rc, tc = Rj, ts + vel * wp.gamma ** m
                        r, zz = _np_radii(prob.kind, a, c, L, Kc, Rc, tc)
                        if (r <= beta + tau).all() and (prob.kind == KIND_3D3D or (zz > wp.z_min).all()):
                            moved = (k, m, Rc, tc)
                            break
                    if moved:
                        break
                if moved:
                    k, m, Rs, ts = moved
                    assert int(out["decisions"][w, i]) == k * wp.n_scales + m
                else:
                    assert int(out["decisions"][w, i]) == -1
            assert np.abs(out["poses"][w, :9].numpy() - Rs.ravel()).max() < 1e-12
            assert np.abs(out["poses"][w, 9:].numpy() - ts).max() < 1e-12
