"""GPU parity of the strategic random walk (purse_walk through the C ABI)
against the oracle's walk (oracle/walk.py) on the same float32 inputs and
start poses (drawn by the oracle's sampler, rounded to float32).

A walk is a chain of discrete decisions (the ranking of perturbations, the
feasibility of each candidate), so float32 and float64 can part ways where a
decision is a near-tie.  Per walk: if the GPU's decisions equal the oracle's
at every iteration, the end pose must agree within 1e-4 rad / 1e-4 m and the
masks must be equal; otherwise the oracle must show a hazard at the first
iteration that differs (a gap between ranked boundary distances within
1e-4 of the largest bound, or a candidate's max r_i / (beta_i + tau) within
1e-4 of 1).  Every end pose the GPU marks as in S is re-checked in float64.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import walk as WK
from oracle.params import OracleParams
from oracle.purse import Problem, feasible, sample as oracle_sample
from paper_2403_09990_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

RANK_BAND = 1e-4     # times max beta
RATIO_BAND = 1e-4


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _starts(inst, n, iters):
    """Start poses in S from the oracle's alternating sampler, in float32."""
    prob = Problem.from_instance(PT.as_f32_instance(inst))
    out = oracle_sample(prob, OracleParams(n_iters=iters), inst.seed, 4 * n)
    P = out["poses"][(out["mask"] & 1) != 0][:n]
    return P.numpy().astype(np.float32)


def _run(batch, starts_per_inst, wp_kw, decisions=True):
    import paper_2403_09990_amd as P
    db = P.DeviceBatch(batch)
    gp = P.purse_default_params()
    wp = P.purse_walk_default_params(**wp_kw)
    counts = [len(s) for s in starts_per_inst]
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    starts = torch.as_tensor(np.concatenate(starts_per_inst), device="cuda")
    res = P.walk(db, gp, wp, torch.as_tensor(off, device="cuda"), starts, with_decisions=decisions)
    torch.cuda.synchronize()
    return db, gp, wp, off, res


def _oracle_params(gp, wp):
    return WK.WalkParams(n_walks=wp.n_walks, n_iters=wp.n_iters, n_perturb=wp.n_perturb, n_keep=wp.n_keep,
                         n_scales=wp.n_scales, gamma=float(np.float32(wp.gamma)),
                         omega0=float(np.float32(wp.omega0)), v0=float(np.float32(wp.v0)),
                         t_pert=float(np.float32(wp.t_pert)), r_pert=float(np.float32(wp.r_pert)),
                         tau_abs_3d=float(np.float32(gp.tau_abs_3d)), tau_abs_2d=float(np.float32(gp.tau_abs_2d)),
                         z_min=float(np.float32(gp.z_min)))


def _compare(inst, starts, res, j, off, gp, wp):
    prob = Problem.from_instance(PT.as_f32_instance(inst))
    owp = _oracle_params(gp, wp)
    nw_all = res["poses"].shape[1]
    a, b = int(off[j]) * wp.n_walks, int(off[j + 1]) * wp.n_walks
    stats = dict(walks=0, same=0, hazard=0, moves=0)
    band_d = RANK_BAND * float(prob.beta.max())
    for mode in (WK.MODE_R, WK.MODE_T):
        ora = WK.walk(prob, starts[:, :9].astype(np.float64), starts[:, 9:].astype(np.float64), inst.seed, mode,
                      owp, diagnostics=True)
        gpose = res["poses"][mode, a:b].cpu().numpy().astype(np.float64)
        gmask = res["mask"][mode, a:b].cpu().numpy()
        gdec = res["decisions"][mode, a:b].cpu().numpy()
        odec = ora["decisions"].numpy()
        assert gdec.shape == odec.shape
        same = (gdec == odec).all(1)
        stats["walks"] += len(same)
        stats["same"] += int(same.sum())
        stats["moves"] += int((odec >= 0).sum())
        # walks that took the same decisions: same end pose, same mask
        op = ora["poses"].numpy()
        ang = PT.rot_angle(gpose[same, :9].reshape(-1, 3, 3), op[same, :9].reshape(-1, 3, 3))
        dt = np.linalg.norm(gpose[same, 9:] - op[same, 9:], axis=1)
        assert (ang <= PT.ROT_TOL).all() and (dt <= PT.TRANS_TOL).all(), (ang.max(), dt.max())
        assert np.array_equal(gmask[same], ora["mask"].numpy()[same])
        # walks that parted: a hazard at the first differing iteration
        for w in np.nonzero(~same)[0]:
            i = int(np.nonzero(gdec[w] != odec[w])[0][0])
            hz = float(ora["rank_gap"][w, i]) <= band_d or float(ora["feas_margin"][w, i]) <= RATIO_BAND
            assert hz, dict(walk=int(w), mode=mode, iteration=i, gpu=gdec[w].tolist(), oracle=odec[w].tolist(),
                            rank_gap=float(ora["rank_gap"][w, i]), feas_margin=float(ora["feas_margin"][w, i]))
            stats["hazard"] += 1
        # the GPU's end poses in S are in S (float64 re-check)
        keep = gmask == 1
        p64 = OracleParams(tau_abs_2d=owp.tau_abs_2d, tau_abs_3d=owp.tau_abs_3d, z_min=owp.z_min)
        R = torch.as_tensor(gpose[keep, :9].reshape(-1, 3, 3))
        t = torch.as_tensor(gpose[keep, 9:])
        ratio = WK.feasibility_ratio(prob, R, t, owp).numpy()
        assert (ratio <= 1.0 + 1e-5).all(), ratio.max()
    return stats


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_walk_matches_oracle(kind):
    """LM-O-shaped 2D-3D (N = 10) or 3DMatch-shaped 3D-3D (N = 50) instance,
    100 starts, the paper's CLOSURE walk parameters (N_W 2, N_I 5, N_P 150,
    N_P* 10, N_T 15, gamma 0.5)."""
    _log("case: walk parity", kind)
    rng = np.random.default_rng(500 if kind == "2d" else 501)
    if kind == "2d":
        inst = W.make_2d3d(rng, 10, 2.0, (5.0, 20.0), 64)
        kw = dict(omega0=0.5, v0=0.05, t_pert=0.005, r_pert=0.02)
    else:
        inst = W.make_3d3d(rng, 50, 0.01, 0.05, 64)
        kw = dict(omega0=0.5, v0=0.05, t_pert=0.02, r_pert=0.02)
    starts = _starts(inst, 100, 30)
    db, gp, wp, off, res = _run(W.Batch([inst]), [starts], kw)
    st = _compare(inst, starts, res, 0, off, gp, wp)
    _log(st)
    assert st["moves"] > 0
    assert st["same"] >= 0.9 * st["walks"]


def test_walk_batch_of_both_kinds_and_ragged_starts():
    """Three instances (2D-3D, 3D-3D, 2D-3D) with 37, 0 and 64 starts in one
    call: each instance's walks equal those of the instance alone (the
    counters are instance-local), and agree with the oracle."""
    _log("case: walk batch")
    rng = np.random.default_rng(502)
    ins = [W.make_2d3d(rng, 12, 2.0, (5.0, 20.0), 64), W.make_3d3d(rng, 8, 0.01, 0.05, 64),
           W.make_2d3d(rng, 8, 2.0, (3.0, 25.0), 64)]
    st = [_starts(ins[0], 37, 30), np.zeros((0, 12), dtype=np.float32), _starts(ins[2], 64, 30)]
    kw = dict(n_iters=4, n_perturb=100, n_keep=8, n_scales=12)
    db, gp, wp, off, res = _run(W.Batch(ins), st, kw)
    for j in (0, 2):
        s = _compare(ins[j], st[j], res, j, off, gp, wp)
        _log(j, s)
        db1, gp1, wp1, off1, r1 = _run(W.Batch([ins[j]]), [st[j]], kw)
        a, b = int(off[j]) * wp.n_walks, int(off[j + 1]) * wp.n_walks
        assert torch.equal(res["poses"][:, a:b], r1["poses"])
        assert torch.equal(res["decisions"][:, a:b], r1["decisions"])


def test_walk_without_perturbations_is_a_line_search():
    """t_pert = r_pert = 0: every kept perturbation is the walk's own pose,
    so the rank is always 0 and the walk is a line search along its
    velocity; the GPU takes the oracle's decisions."""
    _log("case: walk line search")
    rng = np.random.default_rng(503)
    inst = W.make_3d3d(rng, 8, 0.01, 0.05, 64)
    starts = _starts(inst, 20, 30)
    db, gp, wp, off, res = _run(W.Batch([inst]), [starts], dict(t_pert=0.0, r_pert=0.0, n_iters=6))
    dec = res["decisions"].cpu().numpy()
    moved = dec[dec >= 0]
    assert len(moved) > 0 and ((moved // wp.n_scales) == 0).all()
    _compare(inst, starts, res, 0, off, gp, wp)
