"""purse_sample_noalloc (static device scratch, no workspace) against
purse_sample with a workspace, through the C ABI: bitwise the same poses,
masks and statuses on two calls in a row, the second with a smaller batch."""
import sys

import numpy as np
import pytest
import torch

from paper_2403_09990_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _both(batch, gp):
    import paper_2403_09990_amd as P
    db = P.DeviceBatch(batch)
    ref = P.sample(db, gp)
    dev = db.kind.device
    poses = torch.full((db.total_samples, 12), float("nan"), dtype=torch.float32, device=dev)
    mask = torch.full((db.total_samples,), 255, dtype=torch.uint8, device=dev)
    st = torch.full((db.n_inst,), -7, dtype=torch.int32, device=dev)
    P.purse_sample_noalloc(db, gp, poses, mask, st)
    torch.cuda.synchronize()
    return ref, dict(poses=poses, mask=mask, inst_status=st)


def test_noalloc_equals_workspace_sampler():
    import paper_2403_09990_amd as P
    rng = np.random.default_rng(70)
    big = W.Batch([W.make_2d3d(rng, 12, 2.0, (5.0, 20.0), 3000), W.make_3d3d(rng, 20, 0.01, (0.02, 0.1), 1500),
                   W.make_2d3d(rng, 40, 2.0, (3.0, 25.0), 777), W.make_3d3d(rng, 8, 0.01, 0.05, 64)])
    small = W.Batch([W.make_3d3d(rng, 6, 0.01, 0.05, 300)])
    gp = P.purse_default_params(n_iters=20)
    for name, b in (("4 instances", big), ("1 smaller instance", small)):
        _log("case: noalloc vs workspace,", name)
        ref, got = _both(b, gp)
        assert torch.equal(ref["inst_status"], got["inst_status"])
        assert torch.equal(ref["mask"], got["mask"])
        assert torch.equal(ref["poses"], got["poses"])
        assert int((got["mask"] & 1).sum()) > 0
