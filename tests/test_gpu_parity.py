"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded float32 inputs.  Per sample: rotation within 1e-4 rad and
translation within 1e-4 m; MEGB radii within 1e-3 relative and centres within
1e-4.  Decision flips (feasibility bits, bisection steps decided by float32
vs float64 rounding at the boundary) are counted and bounded."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from paper_2403_09990_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _params(**kw):
    import paper_2403_09990_amd as P
    return P.purse_default_params(**kw)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _check_instance(batch, res, j, gp, ids=None):
    inst = batch.instances[j]
    off = int(res["db"].sample_off_host[j])
    M = inst.n_samples
    ids = np.arange(M) if ids is None else np.asarray(ids)
    ora = PT.oracle_for_instance(inst, gp, ids)
    gpu_poses = res["poses"][off:off + M].cpu().numpy()[ids]
    gpu_mask = res["mask"][off:off + M].cpu().numpy()[ids]
    st = PT.compare_with_oracle(gpu_poses, gpu_mask, ora)
    assert int(res["inst_status"][j]) & 0xFF == ora["status"] & 0xFF
    return st


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_c1_all_samples(seed):
    _log("case: c1 seed", seed)
    b = W.config_c1(seed)
    gp = _params(n_iters=50)
    res = PT.run_gpu(b, gp)
    st = _check_instance(b, res, 0, gp)
    _log(st)


def _tuned(batch, gp):
    """The schedule the benchmark times for this batch: the autotuner's
    choice of tile size, tile order and keypoint loop (pair or quad lanes
    for small 2D-3D instances)."""
    import paper_2403_09990_amd as P
    from paper_2403_09990_amd import autotune
    db = P.DeviceBatch(batch)
    ws = P.workspace(db, gp)
    out = P.sample(db, gp, ws=ws)
    gp2, rep = autotune.tune(db, gp, ws, out["poses"], out["mask"], out["inst_status"])
    _log("schedule", rep.get("choice"), "flags", gp2.flags, "tile", gp2.tile)
    return gp2


def _sampled_ids(M, rng, k=400):
    return np.unique(np.concatenate([np.arange(8), np.arange(M - 8, M), rng.integers(0, M, size=k)]))


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_c2_full_size_sampled(seed):
    """The 2D-3D workload at its full size (65,536 trajectories, 100
    iterations) in the launch configuration the benchmark times (the
    autotuned schedule); outputs checked on a sample of trajectories the
    oracle recomputes one by one."""
    _log("case: c2 full size, seed", seed)
    b = W.config_c2(seed)
    gp = _tuned(b, _params(n_iters=100))
    res = PT.run_gpu(b, gp, with_megb=False)
    st = _check_instance(b, res, 0, gp, _sampled_ids(65536, np.random.default_rng(seed)))
    _log(st)
    m = res["mask"].cpu().numpy()
    assert (m & 1).mean() > 0.99


def test_c4_full_size_sampled():
    """The differentiation workload's forward at its full size (2D-3D, N = 24,
    262,144 trajectories, 20 iterations) in the benchmark's schedule, checked
    on sampled trajectories against the oracle."""
    _log("case: c4 full size forward")
    b = W.config_c4(0)
    gp = _tuned(b, _params(n_iters=20))
    res = PT.run_gpu(b, gp, with_megb=False)
    st = _check_instance(b, res, 0, gp, _sampled_ids(262144, np.random.default_rng(44)))
    _log(st)


def test_ragged_batch_mixed_kinds():
    """Several instances in one batch: both kinds, N from 3 to 64, sample
    counts that leave ragged tails (1, 255, 257, 700)."""
    _log("case: ragged batch")
    rng = np.random.default_rng(11)
    ins = [W.make_3d3d(rng, 3, 0.01, 0.05, 257),
           W.make_2d3d(rng, 6, 2.0, (5.0, 20.0), 255),
           W.make_3d3d(rng, 33, 0.01, (0.02, 0.1), 1),
           W.make_2d3d(rng, 64, 2.0, (3.0, 25.0), 700),
           W.make_3d3d(rng, 64, 0.01, (0.02, 0.1), 300)]
    b = W.Batch(ins)
    gp = _params(n_iters=30)
    res = PT.run_gpu(b, gp)
    for j in range(len(ins)):
        st = _check_instance(b, res, j, gp)
        _log(j, st)


def test_centre_fit_needs_weak_perspective_start():
    """A small 2D-3D instance whose DLT start lands behind the camera (weak
    perspective): the fit started from the scaled-orthographic solution wins."""
    _log("case: weak-perspective start")
    rng = np.random.default_rng(100)
    b = W.Batch([W.make_2d3d(rng, 8, 2.0, (5.0, 20.0), 512)])
    gp = _params(n_iters=40)
    res = PT.run_gpu(b, gp, with_megb=False)
    assert int(res["inst_status"][0]) & 0xFF == 0
    _check_instance(b, res, 0, gp)


def test_pull_in_path():
    """Few iterations leave many trajectories outside the set; they are pulled
    back by bisection towards the anchor."""
    _log("case: pull-in")
    b = W.config_c2(3, n_samples=2048)
    gp = _params(n_iters=8)
    res = PT.run_gpu(b, gp, with_megb=False)
    st = _check_instance(b, res, 0, gp)
    _log(st)
    assert st["pulled"] > 200


def test_no_iterations():
    _log("case: n_iters = 0")
    b = W.config_c1(2, n_samples=300)
    gp = _params(n_iters=0)
    res = PT.run_gpu(b, gp, with_megb=False)
    _check_instance(b, res, 0, gp)


def test_zero_radius_collapse_on_gpu():
    """beta = 0 and exact measurements: every feasible sample is the true pose
    and both radii are 0 (to float32 resolution)."""
    _log("case: zero radius")
    out = []
    for b in (W.config_c1(0, n_samples=512), W.config_c2(0, n_samples=512)):
        inst = b.instances[0]
        P = inst.model_pts @ inst.R_gt.T + inst.t_gt
        if inst.kind == W.KIND_3D3D:
            c = P
        else:
            fx, fy, cx, cy = inst.intrinsics
            c = np.stack([fx * P[:, 0] / P[:, 2] + cx, fy * P[:, 1] / P[:, 2] + cy, 0 * P[:, 0]], 1)
        out.append(dataclasses.replace(inst, centres=c, bounds=0 * inst.bounds))
    b = W.Batch(out)
    gp = _params(n_iters=30, megb_iters=256)
    res = PT.run_gpu(b, gp)
    poses = res["poses"].cpu().numpy().astype(np.float64)
    mask = res["mask"].cpu().numpy()
    for j, inst in enumerate(out):
        sl = slice(int(res["db"].sample_off_host[j]), int(res["db"].sample_off_host[j + 1]))
        m = mask[sl]
        assert (m & 1).all()
        R = poses[sl, :9].reshape(-1, 3, 3)
        t = poses[sl, 9:]
        assert PT.rot_angle(R, inst.R_gt[None]).max() < 2e-5
        assert np.abs(t - inst.t_gt).max() < 2e-5
        rad = res["radii"][j].cpu().numpy()
        assert rad[0] < 2e-5 and rad[1] < 2e-5


def test_bad_instances_flagged():
    _log("case: bad instances")
    rng = np.random.default_rng(5)
    good = W.make_2d3d(rng, 8, 2.0, (5.0, 20.0), 64)
    bad_shape = dataclasses.replace(good, shapes=good.shapes * np.array([1, 1, 1, -1.0]))
    neg_beta = dataclasses.replace(good, bounds=-good.bounds)
    small = W.make_2d3d(rng, 5, 2.0, (5.0, 20.0), 64)
    b = W.Batch([good, bad_shape, neg_beta, small])
    gp = _params(n_iters=10, megb_iters=64)
    res = PT.run_gpu(b, gp)
    st = res["inst_status"].cpu().numpy() & 0xFF
    assert list(st) == [0, 2, 2, 4]
    m = res["mask"].cpu().numpy()
    off = res["db"].sample_off_host
    for j in (1, 2, 3):
        assert (m[off[j]:off[j + 1]] == 0).all()
    nf = res["n_feasible"].cpu().numpy()
    assert nf[0] == 64 and (nf[1:] == 0).all()
    assert np.isnan(res["radii"][1:].cpu().numpy()).all()


def test_deterministic_and_batch_independent():
    """Two runs are bitwise equal, and an instance gives bitwise the same
    samples alone as inside a batch (counter-based randomness)."""
    _log("case: determinism")
    b = W.config_c3(0, n_inst=6, m_range=(100, 400), n_range=(6, 20))
    gp = _params(n_iters=20, megb_iters=128)
    r1 = PT.run_gpu(b, gp)
    r2 = PT.run_gpu(b, gp)
    assert torch.equal(r1["poses"], r2["poses"]) and torch.equal(r1["mask"], r2["mask"])
    assert torch.equal(r1["trace"], r2["trace"]) and torch.equal(r1["radii"], r2["radii"])
    for j in (0, 3):
        single = PT.run_gpu(W.sub_batch(b, [j]), gp)
        off = r1["db"].sample_off_host
        assert torch.equal(single["poses"], r1["poses"][off[j]:off[j + 1]])
        assert torch.equal(single["trace"][0], r1["trace"][j])


@pytest.mark.parametrize("cfg", ["c1", "c2", "c2-full"])
def test_megb_against_oracle_on_gpu_samples(cfg):
    """The GPU's MEGB against the oracle's MEGB on the GPU's own samples (read
    back exactly), which isolates the MEGB arithmetic from sampler rounding.
    At the full 65,536 samples the first steps run in the multi-workgroup
    first phase."""
    _log("case: megb", cfg)
    b = {"c1": W.config_c1(0), "c2": W.config_c2(0, n_samples=8192), "c2-full": W.config_c2(0)}[cfg]
    gp = _params(n_iters=50 if cfg == "c1" else 100)
    res = PT.run_gpu(b, gp)
    ora = PT.oracle_megb(res["poses"].cpu().numpy(), res["mask"].cpu().numpy(), gp.megb_iters, gp.megb_avg)
    rad = res["radii"][0].cpu().numpy()
    _log("gpu radii", rad, "oracle", ora["D"], ora["d"])
    assert abs(rad[0] - ora["D"]) <= PT.RADIUS_RTOL * ora["D"]
    assert abs(rad[1] - ora["d"]) <= PT.RADIUS_RTOL * ora["d"]
    C = res["centre"][0].cpu().numpy().astype(np.float64)
    assert PT.rot_angle(C[:9].reshape(3, 3), ora["R"].numpy()) <= PT.CENTRE_TOL
    assert np.linalg.norm(C[9:] - ora["t"].numpy()) <= PT.CENTRE_TOL
    tr = res["trace"][0].cpu().numpy()
    agree = (tr == ora["trace"].numpy()).mean(0)
    _log("trace agreement (rot, trans)", agree)
    assert int(res["n_feasible"][0]) == ora["n"]


@pytest.mark.parametrize("m", [12000, 40000, 131072])
def test_megb_pruning_is_exact(m):
    """The LDS shell with triangle-inequality checks (and, from 32,768
    samples, the first steps spread over many workgroups and rescans that
    stream the global shell of the farthest sixteenth) gives bitwise the same
    argmax trace and centre as scanning every sample at every step in one
    workgroup."""
    _log("case: pruning", m)
    b = W.config_c2(1, n_samples=m)
    gp = _params(n_iters=40, megb_iters=1024)
    res = PT.run_gpu(b, gp)
    import paper_2403_09990_amd as P
    gp2 = _params(n_iters=40, megb_iters=1024, flags=P.PURSE_FLAG_NO_PRUNING)
    full = P.megb(res["db"], gp2, res["poses"], res["mask"], res["inst_status"].clone())
    torch.cuda.synchronize()
    assert torch.equal(full["trace"], res["trace"])
    assert torch.equal(full["centre"], res["centre"])
    assert torch.equal(full["radii"], res["radii"])


@pytest.mark.parametrize("cfg", ["c1", "c2-16k", "c3-8"])
def test_megb_full_descent_is_exact(cfg):
    """Over the whole descent (T = 4096, where most steps run in pipelined
    segments with predicted winners), the shell path gives bitwise the trace,
    centre and radii of scanning every sample at every step."""
    _log("case: full descent", cfg)
    import paper_2403_09990_amd as P
    b = {"c1": W.config_c1(0), "c2-16k": W.config_c2(0, n_samples=16384),
         "c3-8": W.config_c3(2, n_inst=8, m_range=(1024, 16384), n_range=(6, 48))}[cfg]
    gp = _params(n_iters=50)
    res = PT.run_gpu(b, gp)
    gp2 = _params(n_iters=50, flags=P.PURSE_FLAG_NO_PRUNING)
    full = P.megb(res["db"], gp2, res["poses"], res["mask"], res["inst_status"].clone())
    torch.cuda.synchronize()
    assert torch.equal(full["trace"], res["trace"])
    assert torch.equal(full["centre"], res["centre"])
    assert torch.equal(full["radii"], res["radii"])


def test_megb_ties_take_the_lowest_id():
    """Every sample of a 40,000-sample instance copied to id + 20,000 (another
    workgroup of the first phase): each step's farthest sample is tied with
    its copy, and the first phase (packed maximum), the shell steps and the
    full scan all take the lower id, with bitwise the same trace, centre and
    radii."""
    _log("case: ties, 40000 samples")
    import paper_2403_09990_amd as P
    m, h = 40000, 20000
    b = W.config_c2(1, n_samples=m)
    gp = _params(n_iters=40, megb_iters=1024)
    res = PT.run_gpu(b, gp, with_megb=False)
    poses, mask = res["poses"].clone(), res["mask"].clone()
    poses[h:] = poses[:h]
    mask[h:] = mask[:h]
    assert int((mask[:h] & 1).sum()) > 2 * 3072  # the first phase applies
    pr = P.megb(res["db"], gp, poses, mask, res["inst_status"].clone())
    gp2 = _params(n_iters=40, megb_iters=1024, flags=P.PURSE_FLAG_NO_PRUNING)
    full = P.megb(res["db"], gp2, poses, mask, res["inst_status"].clone())
    torch.cuda.synchronize()
    tr = pr["trace"][0].cpu().numpy()
    assert (tr >= 0).all() and (tr < h).all()
    assert torch.equal(full["trace"], pr["trace"])
    assert torch.equal(full["centre"], pr["centre"])
    assert torch.equal(full["radii"], pr["radii"])


@pytest.mark.parametrize("n_inst,m_range", [(160, (1024, 4096)), (600, (1024, 2048)), (140, (32768, 40000))])
def test_megb_shared_cu_variants_are_exact(n_inst, m_range):
    """Batches with more chains than compute units run the narrow pipelined
    chain workgroups, four per compute unit: 160 instances (320 chains, all
    resident), 600 instances (1,200 chains, more than fit at once), and 140
    instances of at least 32,768 samples (the first phase and the global
    shell, which the narrow variant never rebuilds).  Each gives bitwise the
    trace, centre and radii of scanning every sample at every step."""
    _log("case: shared compute units,", n_inst, "instances, M in", m_range)
    import paper_2403_09990_amd as P
    b = W.config_c3(4, n_inst=n_inst, m_range=m_range, n_range=(6, 16))
    gp = _params(n_iters=20)
    res = PT.run_gpu(b, gp)
    gp2 = _params(n_iters=20, flags=P.PURSE_FLAG_NO_PRUNING)
    full = P.megb(res["db"], gp2, res["poses"], res["mask"], res["inst_status"].clone())
    torch.cuda.synchronize()
    assert torch.equal(full["trace"], res["trace"])
    assert torch.equal(full["centre"], res["centre"])
    assert torch.equal(full["radii"], res["radii"])


def test_fp64_polar_path_agrees():
    """Forcing the float64 polar step changes 3D-3D samples by rounding only."""
    _log("case: fp64 polar")
    import paper_2403_09990_amd as P
    b = W.config_c1(1, n_samples=512)
    r32 = PT.run_gpu(b, _params(n_iters=50), with_megb=False)
    r64 = PT.run_gpu(b, _params(n_iters=50, flags=P.PURSE_FLAG_FORCE_FP64_POLAR), with_megb=False)
    st = PT.compare_samples(r32["poses"].cpu().numpy(), r32["mask"].cpu().numpy(),
                            r64["poses"].cpu().numpy(), r64["mask"].cpu().numpy(), max_flip_frac=2e-3)
    _log(st)


@pytest.mark.parametrize("cfg", ["c1", "c2-16k", "batch"])
def test_exact_meb_against_oracle(cfg):
    """Step III (PURSE_FLAG_EXACT_MEB): the GPU's exact ball of its own
    samples against the oracle's (Welzl on the translations and on the
    hemisphere-aligned quaternions) of the same samples, to float32 input
    rounding; the exact radii never exceed the descent's."""
    import paper_2403_09990_amd as P
    from oracle.exact import exact_megb
    _log("case: exact meb", cfg)
    if cfg == "c1":
        b = W.config_c1(0)
        gp = _params(n_iters=50)
    elif cfg == "c2-16k":
        b = W.config_c2(1, n_samples=16384)
        gp = _params(n_iters=100)
    else:
        b = W.config_c3(6, n_inst=6, m_range=(2000, 40000), n_range=(6, 20))
        gp = _params(n_iters=30)
    res = PT.run_gpu(b, gp)
    gx = _params(**{f: getattr(gp, f) for f, _ in type(gp)._fields_})
    gx.flags = gp.flags | P.PURSE_FLAG_EXACT_MEB
    ex = P.megb(res["db"], gx, res["poses"], res["mask"], res["inst_status"].clone(), ws=res["ws"])
    torch.cuda.synchronize()
    assert torch.equal(ex["trace"], res["trace"])
    for j in range(b.n_inst):
        off, end = int(res["db"].sample_off_host[j]), int(res["db"].sample_off_host[j + 1])
        C, ct, D, d = exact_megb(res["poses"][off:end].cpu().numpy(), res["mask"][off:end].cpu().numpy())
        rad = ex["radii"][j].cpu().numpy()
        gd = res["radii"][j].cpu().numpy()
        cen = ex["centre"][j].cpu().numpy().astype(np.float64)
        _log(j, "exact", rad, "oracle", D, d, "descent", gd)
        assert abs(rad[0] - D) <= 1e-5 * D and abs(rad[1] - d) <= 1e-5 * d
        assert float(PT.rot_angle(cen[:9].reshape(1, 3, 3), C.reshape(1, 3, 3))[0]) <= PT.CENTRE_TOL
        assert np.linalg.norm(cen[9:] - ct) <= PT.CENTRE_TOL
        assert rad[0] <= gd[0] * (1 + 1e-6) and rad[1] <= gd[1] * (1 + 1e-6)
