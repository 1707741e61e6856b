"""GPU parity of Step I (purse_init through the C ABI: RANSAG with Arun's
method for 3D-3D, with P3P for 2D-3D, and the convex-combination sampler of
the pose-regression set) against the oracle's samplers on the same float32
inputs and Philox draws, and of the strategic random walk on the
pose-regression set.  Both sides solve in float64; a mask may differ only
where the oracle's max r_i / (beta_i + tau) of a candidate is within 1e-6 of
1 (3D-3D and pose regression) or 1e-3 (2D-3D, whose P3P quartic is
ill-conditioned for a small object at 1 m: two float64 root finders agree to
about 1e-6 rad there), and poses kept by both must agree within 1e-5 (rad and
m; 1e-4 for 2D-3D)."""
import sys

import numpy as np
import pytest
import torch

from oracle import ransag, reg
from oracle import walk as WK
from oracle.params import OracleParams
from oracle.purse import Problem
from paper_2403_09990_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu
BAND = 1e-6
TOL = 1e-5


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu_init(batch):
    import paper_2403_09990_amd as P
    db = P.DeviceBatch(batch)
    gp = P.purse_default_params()
    out = P.init(db, gp)
    torch.cuda.synchronize()
    return db, gp, out["poses"].cpu().numpy().astype(np.float64), out["mask"].cpu().numpy()


def _check(gpose, gmask, opose, omask, ratio_near, tol=TOL):
    same = gmask == omask
    assert (~same <= ratio_near).all(), np.nonzero(~same & ~ratio_near)[0][:10]
    both = same & (gmask == 1) & ~ratio_near
    ang = PT.rot_angle(gpose[both, :9].reshape(-1, 3, 3), opose[both, :9].reshape(-1, 3, 3))
    dt = np.linalg.norm(gpose[both, 9:] - opose[both, 9:], axis=1)
    assert (ang <= tol).all() and (dt <= tol).all(), (ang.max(), dt.max())
    return dict(n=len(gmask), kept=int(gmask.sum()), differ=int((~same).sum()))


def test_ransag_3d_matches_oracle():
    _log("case: ransag 3d")
    rng = np.random.default_rng(600)
    inst = W.make_3d3d(rng, 8, 0.01, 0.05, 3000)
    db, gp, gpose, gmask = _gpu_init(W.Batch([inst]))
    prob = Problem.from_instance(PT.as_f32_instance(inst))
    p = PT.oracle_params(gp)
    opose, omask, idx = ransag.ransag_3d(prob, p, inst.seed, inst.n_samples)
    R = opose[:, :9].reshape(-1, 3, 3)
    near = np.abs(WK.feasibility_ratio(prob, R, opose[:, 9:], WK.WalkParams(tau_abs_3d=p.tau_abs_3d)).numpy() - 1) <= BAND
    st = _check(gpose, gmask, opose.numpy(), omask.numpy(), near)
    _log(st)
    assert st["kept"] > 0


def test_ransag_2d_matches_oracle():
    _log("case: ransag 2d (P3P)")
    rng = np.random.default_rng(601)
    inst = W.make_2d3d(rng, 10, 2.0, (5.0, 20.0), 1000)
    db, gp, gpose, gmask = _gpu_init(W.Batch([inst]))
    prob = Problem.from_instance(PT.as_f32_instance(inst))
    p = PT.oracle_params(gp)
    opose, omask, idx, sols, pix = ransag.ransag_2d(prob, p, inst.seed, inst.n_samples)
    wpp = WK.WalkParams(tau_abs_2d=p.tau_abs_2d, z_min=p.z_min)
    near = np.zeros(len(sols), dtype=bool)
    for r, row in enumerate(sols):
        for k, (v, R, t, ok) in enumerate(row):
            ratio = float(WK.feasibility_ratio(prob, R[None], t[None], wpp)[0])
            close_root = k > 0 and abs(v - row[k - 1][0]) <= 1e-4 * max(1.0, abs(v))
            near[r] |= abs(ratio - 1) <= 1e-3 or close_root
    st = _check(gpose, gmask, opose.numpy(), omask.numpy(), near, tol=PT.ROT_TOL)
    _log(st)
    assert st["kept"] > 0


def test_convex_sampler_matches_oracle():
    _log("case: convex sampler (pose regression)")
    rng = np.random.default_rng(602)
    inst = W.make_reg(rng, 10, 0.05, 0.01, 1500)
    db, gp, gpose, gmask = _gpu_init(W.Batch([inst]))
    prob = reg.from_instance(PT.as_f32_instance(inst))
    tau = float(np.float32(gp.tau_abs_3d))
    opose, omask = reg.convex_samples(prob, inst.seed, inst.n_samples, tau)
    R = opose[:, :9].reshape(-1, 3, 3)
    near = np.abs(reg.feasibility_ratio(prob, R, opose[:, 9:], tau).numpy() - 1) <= BAND
    # every trial's pose (kept or not) is the same convex combination
    ang = PT.rot_angle(gpose[:, :9].reshape(-1, 3, 3), opose.numpy()[:, :9].reshape(-1, 3, 3))
    assert ang.max() <= TOL and np.abs(gpose[:, 9:] - opose.numpy()[:, 9:]).max() <= TOL
    st = _check(gpose, gmask, opose.numpy(), omask.numpy(), near)
    _log(st)
    assert st["kept"] > 100


def test_walk_on_the_pose_regression_set_matches_oracle():
    """The strategic random walk on a pose-regression set (LM-shaped: 10
    hypotheses), from the oracle's convex-combination starts."""
    import paper_2403_09990_amd as P
    from tests.test_gpu_walk import _oracle_params, RANK_BAND, RATIO_BAND
    _log("case: walk on pose regression")
    rng = np.random.default_rng(603)
    inst = W.make_reg(rng, 10, 0.05, 0.01, 64)
    prob = reg.from_instance(PT.as_f32_instance(inst))
    tau = float(np.float32(P.purse_default_params().tau_abs_3d))
    sp, sm = reg.convex_samples(prob, 77, 400, tau)
    starts = sp[sm == 1][:100].numpy().astype(np.float32)
    db = P.DeviceBatch(W.Batch([inst]))
    gp = P.purse_default_params()
    wp = P.purse_walk_default_params(omega0=0.3, v0=0.03, t_pert=0.005, r_pert=0.02)
    off = torch.as_tensor([0, len(starts)], dtype=torch.int64, device="cuda")
    res = P.walk(db, gp, wp, off, torch.as_tensor(starts, device="cuda"), with_decisions=True)
    torch.cuda.synchronize()
    owp = _oracle_params(gp, wp)
    same_tot = walks = 0
    for mode in (WK.MODE_R, WK.MODE_T):
        ora = WK.walk(prob, starts[:, :9].astype(np.float64), starts[:, 9:].astype(np.float64), inst.seed, mode,
                      owp, diagnostics=True)
        gdec = res["decisions"][mode].cpu().numpy()
        odec = ora["decisions"].numpy()
        same = (gdec == odec).all(1)
        walks += len(same)
        same_tot += int(same.sum())
        gp_ = res["poses"][mode].cpu().numpy().astype(np.float64)
        op_ = ora["poses"].numpy()
        ang = PT.rot_angle(gp_[same, :9].reshape(-1, 3, 3), op_[same, :9].reshape(-1, 3, 3))
        assert (ang <= PT.ROT_TOL).all() and (np.linalg.norm(gp_[same, 9:] - op_[same, 9:], axis=1) <= PT.TRANS_TOL).all()
        band_d = RANK_BAND * float(prob.beta.max())
        for w in np.nonzero(~same)[0]:
            i = int(np.nonzero(gdec[w] != odec[w])[0][0])
            assert float(ora["rank_gap"][w, i]) <= band_d or float(ora["feas_margin"][w, i]) <= RATIO_BAND
        assert (res["mask"][mode].cpu().numpy() == 1).all()
        assert (odec >= 0).any()
    _log(dict(walks=walks, same=same_tot))
    assert same_tot >= 0.9 * walks


@pytest.mark.parametrize("kind", ["2d", "3d", "reg"])
def test_closure_pipeline_on_the_gpu(kind):
    """The paper's three steps in one pass on the GPU: Step I candidates,
    Step II walks from the first 100 in S, Step III exact balls of the walks'
    end poses; every end pose is in S and the balls enclose them."""
    import paper_2403_09990_amd as P
    _log("case: closure pipeline", kind)
    rng = np.random.default_rng(610)
    inst = {"2d": lambda: W.make_2d3d(rng, 10, 2.0, (5.0, 20.0), 3000),
            "3d": lambda: W.make_3d3d(rng, 50, 0.01, 0.05, 3000),
            "reg": lambda: W.make_reg(rng, 10, 0.05, 0.01, 1500)}[kind]()
    b = W.Batch([inst])
    db, gp, gpose, gmask = _gpu_init(b)
    keep = np.nonzero(gmask == 1)[0][:100]
    assert len(keep) >= 10
    starts = torch.as_tensor(gpose[keep].astype(np.float32), device="cuda")
    wp = P.purse_walk_default_params()
    off = torch.as_tensor([0, len(keep)], dtype=torch.int64, device="cuda")
    res = P.walk(db, gp, wp, off, starts)
    ends = res["poses"].reshape(-1, 12).contiguous()
    emask = res["mask"].reshape(-1).contiguous()
    assert bool((emask == 1).all())
    # Step III on the walks' end poses (an instance whose samples are the ends)
    b2 = W.Batch([W.sub_batch(b, [0], n_samples=ends.shape[0]).instances[0]])
    db2 = P.DeviceBatch(b2)
    gx = P.purse_default_params(megb_iters=1024, flags=P.PURSE_FLAG_EXACT_MEB)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    m = P.megb(db2, gx, ends, emask, st)
    torch.cuda.synchronize()
    rad = m["radii"][0].cpu().numpy()
    C = m["centre"][0].cpu().numpy().astype(np.float64)
    E = ends.cpu().numpy().astype(np.float64)
    D = PT.rot_angle(E[:, :9].reshape(-1, 3, 3), np.broadcast_to(C[:9].reshape(3, 3), (len(E), 3, 3))).max()
    d = np.linalg.norm(E[:, 9:] - C[9:], axis=1).max()
    _log("radii", rad, "check", D, d)
    # radii against the float32 centre handed back: 1e-5 rad / m of slack
    assert abs(rad[0] - D) <= 1e-5 and abs(rad[1] - d) <= 1e-5
    assert rad[0] > 0 and rad[1] > 0
