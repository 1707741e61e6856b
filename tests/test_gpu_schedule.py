"""The sampler's tile schedule: every sample of a ragged mixed batch is written
exactly as in the plain per-instance order, whatever the workgroup size and
tile order, and the autotuner picks among those candidates and caches them."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from paper_2403_09990_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _batch():
    rng = np.random.default_rng(77)
    ins = []
    for j, (m, n) in enumerate([(1, 6), (300, 40), (64, 7), (1000, 12), (65, 48), (129, 9), (257, 30)]):
        if j % 2 == 0:
            ins.append(W.make_2d3d(rng, n, 2.0, (3.0, 25.0), m))
        else:
            ins.append(W.make_3d3d(rng, n, 0.01, (0.02, 0.1), m))
    # an instance of an unknown kind: flagged, outputs zero
    ins.append(dataclasses.replace(W.make_3d3d(rng, 8, 0.01, 0.05, 70), kind=7))
    return W.Batch(ins)


def _run(P, db, gp):
    dev = db.kind.device
    ws = P.workspace(db, gp)
    ws.fill_(0xCD)
    poses = torch.full((db.total_samples, 12), float("nan"), dtype=torch.float32, device=dev)
    mask = torch.full((db.total_samples,), 0xEE, dtype=torch.uint8, device=dev)
    status = torch.full((db.n_inst,), -99, dtype=torch.int32, device=dev)
    P.purse_sample(db, gp, poses, mask, status, ws)
    torch.cuda.synchronize()
    return poses.cpu(), mask.cpu(), status.cpu()


def test_every_schedule_writes_every_sample_identically():
    import paper_2403_09990_amd as P
    b = _batch()
    db = P.DeviceBatch(b)
    ref = None
    for tile in (64, 128, 256):
        for order in (0, P.PURSE_FLAG_INSTANCE_ORDER):
            _log("case: schedule tile", tile, "order", order)
            gp = P.purse_default_params(n_iters=15, tile=tile, flags=order)
            poses, mask, status = _run(P, db, gp)
            assert not torch.isnan(poses).any()
            assert not (mask == 0xEE).any()
            if ref is None:
                ref = (poses, mask, status)
                st = status.numpy() & 0xFF
                assert (st[:-1] == P.PURSE_INST_OK).all() and st[-1] == P.PURSE_INST_BAD_SIZE
                off = db.sample_off_host
                assert (poses[off[-2]:off[-1]] == 0).all() and (mask[off[-2]:off[-1]] == 0).all()
            else:
                assert torch.equal(poses, ref[0]) and torch.equal(mask, ref[1]) and torch.equal(status, ref[2])
    # persistent work-queue kernels, residency caps and the launch groups one
    # after the other on the caller's stream: the same samples
    for tile in (64, 256):
        for flags, waves in ((P.PURSE_FLAG_WORK_QUEUE, 0), (0, 2), (P.PURSE_FLAG_WORK_QUEUE, 4),
                             (P.PURSE_FLAG_WORK_QUEUE | P.PURSE_FLAG_INSTANCE_ORDER, 1),
                             (P.PURSE_FLAG_SERIAL_GROUPS, 0),
                             (P.PURSE_FLAG_SERIAL_GROUPS | P.PURSE_FLAG_WORK_QUEUE, 0)):
            _log("case: schedule tile", tile, "flags", flags, "waves", waves)
            gp = P.purse_default_params(n_iters=15, tile=tile, flags=flags, waves_per_simd=waves)
            poses, mask, status = _run(P, db, gp)
            assert torch.equal(poses, ref[0]) and torch.equal(mask, ref[1]) and torch.equal(status, ref[2])


def test_unrolled_and_generic_keypoint_loops_agree():
    """2D-3D instances of at most 16 keypoints run an unrolled keypoint loop
    that keeps the iteration's projection targets in registers; the general
    loop recomputes them; pair mode splits the keypoints of each trajectory
    over two lanes.  All compute the same values to float32 rounding."""
    import paper_2403_09990_amd as P
    _log("case: unrolled vs generic loop")
    rng = np.random.default_rng(8)
    b = W.Batch([W.make_2d3d(rng, n, 2.0, (5.0, 20.0), m) for n, m in ((6, 300), (12, 1000), (16, 257))])
    db = P.DeviceBatch(b)
    a = _run(P, db, P.purse_default_params(n_iters=40))
    g = _run(P, db, P.purse_default_params(n_iters=40, flags=P.PURSE_FLAG_GENERIC_LOOP))
    assert torch.equal(a[1], g[1]) and torch.equal(a[2], g[2])
    diff = (a[0] - g[0]).abs().max().item()
    _log("max pose difference", diff)
    assert diff <= 1e-5
    # two or four lanes per trajectory: every sample written, the same values to rounding
    for flag, name in ((P.PURSE_FLAG_PAIR_LANES, "pair"), (P.PURSE_FLAG_QUAD_LANES, "quad")):
        for tile in (64, 256):
            pr = _run(P, db, P.purse_default_params(n_iters=40, tile=tile, flags=flag))
            assert not torch.isnan(pr[0]).any() and not (pr[1] == 0xEE).any()
            assert torch.equal(a[1], pr[1]) and torch.equal(a[2], pr[2])
            diff = (a[0] - pr[0]).abs().max().item()
            _log(name, "lanes, tile", tile, "max pose difference", diff)
            assert diff <= 1e-5
            # the same lane groups from the work queue: bitwise the same
            pq = _run(P, db, P.purse_default_params(n_iters=40, tile=tile, flags=flag | P.PURSE_FLAG_WORK_QUEUE,
                                                    waves_per_simd=2 if tile == 64 else 0))
            assert torch.equal(pq[0], pr[0]) and torch.equal(pq[1], pr[1]) and torch.equal(pq[2], pr[2])


def test_autotune_picks_and_caches(tmp_path):
    import paper_2403_09990_amd as P
    from paper_2403_09990_amd import autotune
    _log("case: autotune")
    b = W.config_c3(3, n_inst=16, m_range=(256, 2048), n_range=(6, 24))
    db = P.DeviceBatch(b)
    gp = P.purse_default_params(n_iters=10)
    ws = P.workspace(db, gp)
    out = P.sample(db, gp, ws=ws)
    cache = str(tmp_path / "tune.json")
    best, rep = autotune.tune(db, gp, ws, out["poses"], out["mask"], out["inst_status"], cache=cache, reps=1)
    assert not rep["cached"] and best.tile in autotune.TILES
    assert len(rep["candidates_ms"]) >= len(autotune.TILES) * len(autotune.ORDERS) + len(autotune.STAGE2)
    best2, rep2 = autotune.tune(db, gp, ws, out["poses"], out["mask"], out["inst_status"], cache=cache)
    assert rep2["cached"] and best2.tile == best.tile and best2.flags == best.flags
    assert best2.waves_per_simd == best.waves_per_simd
    # the tuned schedule gives the default schedule's results
    ref = P.sample(db, gp)
    got = P.sample(db, best)
    torch.cuda.synchronize()
    assert torch.equal(ref["mask"], got["mask"])
    if best.flags & (P.PURSE_FLAG_GENERIC_LOOP | P.PURSE_FLAG_PAIR_LANES | P.PURSE_FLAG_QUAD_LANES):
        assert (ref["poses"] - got["poses"]).abs().max().item() <= 1e-5
    else:
        assert torch.equal(ref["poses"], got["poses"])
