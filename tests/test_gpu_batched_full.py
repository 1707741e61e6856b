"""The batched workloads at their full sizes, in the launch configuration the
benchmark times.

- 512 uneven instances (half 3D-3D, half 2D-3D, N ~ U{6..48}, M ~
  U{1024..16384}, 50 iterations): per-instance status, sampled trajectories
  of 64 instances against the oracle one by one, and the MEGB of three
  instances against the oracle's MEGB on the GPU's samples.
- 64 x 2D-3D instances with N = 48 and 2^20 trajectories each (67,108,864
  trajectories, 50 iterations): sampled trajectories of 8 instances against
  the oracle, the MEGB radii against a float64 reduction over every sample
  about the returned centre, and the gradients of two instances against the
  oracle's reverse pass, all instances differentiated in one call.
"""
import sys

import numpy as np
import pytest
import torch

from oracle.adjoint import backward as oracle_backward
from oracle.adjoint import radius_argmax
from paper_2403_09990_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _sampled(batch, res, j, gp, ids):
    inst = batch.instances[j]
    off = int(res["db"].sample_off_host[j])
    ora = PT.oracle_for_instance(inst, gp, ids)
    tid = torch.as_tensor(off + np.asarray(ids), device=res["poses"].device)
    gpu_poses = res["poses"][tid].cpu().numpy()
    gpu_mask = res["mask"][tid].cpu().numpy()
    assert int(res["inst_status"][j]) & 0xFF == ora["status"] & 0xFF
    return PT.compare_with_oracle(gpu_poses, gpu_mask, ora)


def _ids(rng, M, k):
    return np.unique(np.concatenate([[0, 1, M - 1], rng.integers(0, M, size=k)]))


def test_c3_full_size():
    import paper_2403_09990_amd as P
    _log("case: c3 full size")
    b = W.config_c3(0)
    gp = P.purse_default_params(n_iters=50)
    res = PT.run_gpu(b, gp)
    st = res["inst_status"].cpu().numpy() & 0xFF
    assert (st == P.PURSE_INST_OK).all()
    rng = np.random.default_rng(3)
    tot = dict(n=0, mask_flips=0, pose_out=0, forgiven=0, max_rot=0.0, max_trans=0.0)
    for j in range(0, 512, 8):
        s = _sampled(b, res, j, gp, _ids(rng, b.instances[j].n_samples, 3))
        for k in ("n", "mask_flips", "pose_out", "forgiven"):
            tot[k] += s[k]
        tot["max_rot"] = max(tot["max_rot"], s["max_rot"])
        tot["max_trans"] = max(tot["max_trans"], s["max_trans"])
    _log(tot)
    for j in (0, 1, 257):
        off, end = res["db"].sample_off_host[j], res["db"].sample_off_host[j + 1]
        ora = PT.oracle_megb(res["poses"][off:end].cpu().numpy(), res["mask"][off:end].cpu().numpy(),
                             gp.megb_iters, gp.megb_avg)
        rad = res["radii"][j].cpu().numpy()
        _log("instance", j, "gpu radii", rad, "oracle", ora["D"], ora["d"])
        assert abs(rad[0] - ora["D"]) <= PT.RADIUS_RTOL * ora["D"]
        assert abs(rad[1] - ora["d"]) <= PT.RADIUS_RTOL * ora["d"]
        assert int(res["n_feasible"][j]) == ora["n"]


def _radii_f64(poses, mask, centre):
    """max over feasible samples of the geodesic angle and the translation
    distance to the centre, in float64 (plain torch on the device)."""
    P = poses.double()
    sel = (mask & 1) != 0
    C = centre.double()
    fr = ((P[:, :9] - C[:9]) ** 2).sum(1)
    ft = ((P[:, 9:] - C[9:]) ** 2).sum(1)
    fr = torch.where(sel, fr, torch.zeros_like(fr)).max()
    ft = torch.where(sel, ft, torch.zeros_like(ft)).max()
    x = torch.clamp(torch.sqrt(fr) / (2.0 * np.sqrt(2.0)), max=1.0)
    return float(2.0 * torch.asin(x)), float(torch.sqrt(ft))


def test_c5_full_size_forward_and_backward():
    """(An earlier backward that linearised the descent at iterates stored by
    purse_megb faulted the GPU on this case.  The backward now checks every
    workspace record against the batch and stops an instance, with NaN
    gradients, before a data-derived id outside the instance can index poses:
    a non-finite centre used to leave the radius search's sentinel INT32_MAX
    in the active set, about 100 GB past the poses; see
    tests/native/bwd_check_test.cpp.)"""
    import paper_2403_09990_amd as P
    _log("case: c5 full size")
    b = W.config_c5(0)
    gp = P.purse_default_params(n_iters=50)
    res = PT.run_gpu(b, gp)
    assert res["db"].total_samples == 64 << 20
    st = res["inst_status"].cpu().numpy() & 0xFF
    assert (st == P.PURSE_INST_OK).all()
    rng = np.random.default_rng(5)
    for j in (0, 9, 18, 27, 36, 45, 54, 63):
        s = _sampled(b, res, j, gp, _ids(rng, 1 << 20, 20))
        _log("instance", j, s)
    for j in (0, 31, 63):
        off, end = int(res["db"].sample_off_host[j]), int(res["db"].sample_off_host[j + 1])
        D, d = _radii_f64(res["poses"][off:end], res["mask"][off:end], res["centre"][j])
        rad = res["radii"][j].cpu().numpy()
        _log("instance", j, "radii", rad, "f64 reduction", D, d)
        assert abs(rad[0] - D) <= 1e-9 * max(1.0, D) and abs(rad[1] - d) <= 1e-9 * max(1.0, d)
        R = res["centre"][j, :9].double().reshape(3, 3).cpu().numpy()
        assert np.abs(R @ R.T - np.eye(3)).max() < 1e-5 and np.linalg.det(R) > 0
    # gradients of every instance in one call; two of them against the oracle
    dev = res["poses"].device
    g_radii = rng.normal(size=(64, 2))
    g_centre = rng.normal(size=(64, 6))
    db = res["db"]
    _log("c5: backward of all 64 instances in one call")
    g_c = torch.empty(db.total_kp, 3, dtype=torch.float32, device=dev)
    g_L = torch.empty(db.total_kp, 4, dtype=torch.float32, device=dev)
    g_b = torch.empty(db.total_kp, dtype=torch.float32, device=dev)
    bst = torch.full((64,), -1, dtype=torch.int32, device=dev)
    P.purse_megb_backward(db, gp, res["poses"], res["mask"], res["trace"],
                          torch.as_tensor(g_radii, dtype=torch.float64, device=dev),
                          torch.as_tensor(g_centre, dtype=torch.float32, device=dev),
                          g_c, g_L, g_b, res["ws"], bwd_status=bst)
    torch.cuda.synchronize()
    bst = bst.cpu().numpy()
    _log("backward status per instance", (bst & 0xFF).tolist())
    _log("active-set sizes", (bst >> 8).tolist())
    assert ((bst & 0xFF) == P.PURSE_BWD_OK).all()
    gpu = (g_c.cpu().numpy(), g_L.cpu().numpy(), g_b.cpu().numpy())
    assert all(np.isfinite(x).all() for x in gpu)
    for j in (0, 63):
        inst = b.instances[j]
        off, end = int(db.sample_off_host[j]), int(db.sample_off_host[j + 1])
        kof, kend = int(db.kp_off_host[j]), int(db.kp_off_host[j + 1])
        mask = res["mask"][off:end].cpu().numpy()
        poses = res["poses"][off:end].cpu().numpy()
        C = res["centre"][j].cpu().numpy().astype(np.float64)
        s0 = int(np.nonzero(mask & 1)[0][0])
        sD, sd = radius_argmax(poses, mask, C[:9].reshape(3, 3), C[9:])
        ora = oracle_backward(PT.as_f32_instance(inst), PT.oracle_params(gp), res["trace"][j].cpu().numpy(),
                              s0, sD, sd, g_radii[j], g_centre[j])
        g = np.concatenate([x[kof:kend].ravel() for x in gpu])
        o = np.concatenate([x.ravel() for x in ora])
        rel = np.linalg.norm(g - o) / max(1e-12, np.linalg.norm(o))
        _log("instance", j, "gradient rel err", rel)
        assert rel <= 1e-3
