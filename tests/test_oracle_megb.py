"""Pins of the oracle's MEGB: closed forms, exact enclosing balls, Prop. 1
(no GPU)."""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import exact, so3
from oracle.megb import megb, megb_from_poses, radii_at
from oracle.params import OracleParams
from oracle.purse import Problem, sample
from paper_2403_09990_amd import workloads as W

DT = torch.float64
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "megb_closed_forms.json")))


def _run(R, t, T=4096, avg=10):
    R = torch.as_tensor(np.asarray(R), dtype=DT)
    t = torch.as_tensor(np.asarray(t), dtype=DT)
    return megb(R, t, torch.arange(len(R)), T, avg)


def test_two_rotations_midpoint():
    g = GOLD["two_rotations"]
    ax = np.array(g["axis"])
    R = Rotation.from_rotvec([ax * g["angle_a"], ax * g["angle_b"]]).as_matrix()
    out = _run(R, np.zeros((2, 3)))
    C = Rotation.from_rotvec(ax * g["centre_angle"]).as_matrix()
    assert float(so3.angle(out["R"], torch.as_tensor(C))) < 1e-3 * g["radius"]
    assert abs(out["D"] - g["radius"]) < 1e-3 * g["radius"]
    assert out["D"] >= g["radius"] - 1e-12   # a max distance from a valid centre


def test_rectangle_corners_translation_ball():
    g = GOLD["rectangle_corners"]
    P = np.array(g["points"])
    out = _run(np.tile(np.eye(3), (4, 1, 1)), P)
    np.testing.assert_allclose(out["t"].numpy(), g["centre"], atol=1e-3 * g["radius"])
    assert g["radius"] - 1e-12 <= out["d"] <= g["radius"] * (1 + 1e-3)
    assert out["D"] == 0.0


def test_unit_ball_toy():
    g = GOLD["unit_ball_toy"]
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3000, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    disc = np.concatenate([x[:, :2], np.zeros((3000, 1))], 1)
    seg = np.concatenate([np.zeros((3000, 2)), x[:, 2:]], 1)
    I = np.tile(np.eye(3), (3000, 1, 1))
    # samples of the sphere's boundary reach the disc's rim and the segment's
    # ends only approximately; the enclosing radius is within sampling error
    assert abs(_run(I, disc)["d"] - g["radius_R"]) < 5e-3
    assert abs(_run(I, seg)["d"] - g["radius_t"]) < 5e-3


def test_rotations_about_one_axis():
    """Rotations about one axis with angles in [a, b]: centre at (a+b)/2,
    radius (b-a)/2."""
    rng = np.random.default_rng(1)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    ang = rng.uniform(-0.3, 0.7, size=200)
    ang[:2] = [-0.3, 0.7]
    out = _run(Rotation.from_rotvec(ang[:, None] * ax).as_matrix(), np.zeros((200, 3)))
    assert abs(out["D"] - 0.5) < 1e-3 * 0.5
    C = Rotation.from_rotvec(0.2 * ax).as_matrix()
    assert float(so3.angle(out["R"], torch.as_tensor(C))) < 1e-3


def test_welzl_against_brute_force():
    rng = np.random.default_rng(2)
    for d in (3, 4):
        for _ in range(10):
            P = rng.normal(size=(int(rng.integers(2, 11)), d))
            c1, r1 = exact.welzl(P)
            c2, r2 = exact.brute_force_meb(P)
            assert abs(r1 - r2) < 1e-9
            np.testing.assert_allclose(c1, c2, atol=1e-8)


def test_proposition_1_subset_monotone():
    """Prop. 1 (Inner Approximation): the MEB of a subset is no larger."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        P = rng.normal(size=(200, 3))
        _, r = exact.welzl(P)
        sub = P[rng.random(200) < 0.3]
        _, rs = exact.welzl(sub)
        assert rs <= r + 1e-12


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_gd_sandwich_on_sampler_output(cfg):
    """r* <= r_hat <= r*(1 + eps): the GD radius is a max distance from a valid
    centre, so it never undercuts the exact minimax radius; the gap after
    T steps is small.  r* for translations is Welzl's ball; for rotations the
    min over SO(3) of the max angle by local search (convex objective)."""
    b = W.config_c1(0) if cfg == "c1" else W.config_c2(0, n_samples=512)
    inst = b.instances[0]
    p = OracleParams(n_iters=50 if cfg == "c1" else 100)
    out = sample(Problem.from_instance(inst), p, inst.seed, 512)
    mg = megb_from_poses(out["poses"], out["mask"], 4096, 10)
    sel = (out["mask"] & 1) != 0
    R = out["poses"][sel, :9].reshape(-1, 3, 3).numpy()
    t = out["poses"][sel, 9:].numpy()
    _, d_star = exact.welzl(t)
    assert d_star - 1e-12 <= mg["d"] <= d_star * (1 + 2e-3)
    C, D_star = exact.so3_minimax(R, starts=[mg["R"].numpy()])
    assert D_star - 1e-9 <= mg["D"] <= D_star * (1 + 5e-3)
    Cq, _ = exact.quaternion_meb(R)
    assert abs(exact.max_angle(Cq, R) - D_star) < 1e-3 * D_star


def test_gd_convergence_slope():
    """The distance of the iterates to the final centre falls roughly like
    1/i (appendix "Geodesic Gradient Descent", subgradient convergence)."""
    rng = np.random.default_rng(4)
    R = Rotation.from_rotvec(rng.normal(size=(300, 3)) * 0.2).as_matrix()
    Rt = torch.as_tensor(R)
    final = _run(R, np.zeros((300, 3)), T=2048)["R"]
    errs = []
    for T in (32, 128, 512):
        errs.append(float(so3.angle(_run(R, np.zeros((300, 3)), T=T, avg=1)["R"], final)))
    slope = np.polyfit(np.log([32, 128, 512]), np.log(errs), 1)[0]
    assert -1.6 < slope < -0.4
    del Rt


def test_empty_and_single_sample():
    out = megb(torch.zeros(0, 3, 3, dtype=DT), torch.zeros(0, 3, dtype=DT),
               torch.zeros(0, dtype=torch.int64), 16, 10)
    assert math.isnan(out["D"]) and out["n"] == 0
    R = torch.as_tensor(Rotation.from_rotvec([0.1, 0.2, 0.3]).as_matrix())[None]
    out = megb(R, torch.ones(1, 3, dtype=DT), torch.tensor([7]), 16, 10)
    assert out["D"] < 1e-12 and out["d"] == 0.0 and bool((out["trace"] == 7).all())


def test_trace_ties_go_to_lowest_index():
    """Duplicate samples: the argmax picks the first of equal keys."""
    R = np.tile(np.eye(3), (4, 1, 1))
    t = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0], [0.0, 0, 0]])
    out = megb(torch.as_tensor(R), torch.as_tensor(t), torch.tensor([10, 11, 12, 13]), 3, 1)
    assert int(out["trace"][0, 1]) == 11          # from (0,0,0): samples 11 and 12 tie
    assert int(out["trace"][1, 1]) == 10          # from (1,0,0): samples 10 and 13 tie
    rad = radii_at(out["R"], out["t"], torch.as_tensor(R), torch.as_tensor(t))
    assert rad[0] == 0.0


def test_exact_megb_of_rotations_about_one_axis_and_two_points():
    """Step III's ball: rotations about one axis through angles in [a, b]
    have the centre at angle (a + b)/2 and radius (b - a)/2; two translations
    have their midpoint and half their distance."""
    ax = np.array([0.3, -0.4, 0.866])
    ax /= np.linalg.norm(ax)
    angs = np.array([0.1, 0.35, 0.22, 0.6, 0.45])
    R = Rotation.from_rotvec(angs[:, None] * ax).as_matrix()
    t = np.zeros((5, 3))
    t[0] = [0.1, 0.2, 0.3]
    t[3] = [0.5, -0.2, 0.1]
    t[1:3] = 0.5 * (t[0] + t[3])
    t[4] = 0.5 * (t[0] + t[3]) + 0.01
    poses = np.concatenate([R.reshape(5, 9), t], 1)
    C, ct, D, d = exact.exact_megb(poses, np.ones(5, dtype=np.uint8))
    mid = Rotation.from_rotvec(0.35 * ax).as_matrix()
    assert np.abs(C - mid).max() < 1e-9
    assert abs(D - 0.25) < 1e-9
    assert np.abs(ct - 0.5 * (t[0] + t[3])).max() < 1e-9
    assert abs(d - 0.5 * np.linalg.norm(t[0] - t[3])) < 1e-9
