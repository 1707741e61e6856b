"""The forward hot path (purse_sample then purse_megb) and the backward captured
in one HIP graph: every replay reproduces the eager results bitwise, the graph
re-reads its inputs on each replay, and it can be replayed with eager work and
synchronisations in between."""
import sys

import numpy as np
import pytest
import torch

from paper_2403_09990_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


class _Run:
    """Output buffers of one forward + backward pass, allocated once."""

    def __init__(self, P, db, gp):
        dev = db.kind.device
        self.P, self.db, self.gp = P, db, gp
        self.ws = P.workspace(db, gp)
        self.poses = torch.empty(db.total_samples, 12, dtype=torch.float32, device=dev)
        self.mask = torch.empty(db.total_samples, dtype=torch.uint8, device=dev)
        self.status = torch.empty(db.n_inst, dtype=torch.int32, device=dev)
        self.centre = torch.empty(db.n_inst, 12, dtype=torch.float32, device=dev)
        self.radii = torch.empty(db.n_inst, 2, dtype=torch.float64, device=dev)
        self.nf = torch.empty(db.n_inst, dtype=torch.int64, device=dev)
        self.trace = torch.empty(db.n_inst, gp.megb_iters, 2, dtype=torch.int32, device=dev)
        rng = np.random.default_rng(9)
        self.g_radii = torch.as_tensor(rng.normal(size=(db.n_inst, 2)), dtype=torch.float64, device=dev)
        self.g_centre = torch.as_tensor(rng.normal(size=(db.n_inst, 6)), dtype=torch.float32, device=dev)
        self.g_c = torch.empty(db.total_kp, 3, dtype=torch.float32, device=dev)
        self.g_L = torch.empty(db.total_kp, 4, dtype=torch.float32, device=dev)
        self.g_b = torch.empty(db.total_kp, dtype=torch.float32, device=dev)

    def __call__(self, stream=None):
        P, db, gp = self.P, self.db, self.gp
        P.purse_sample(db, gp, self.poses, self.mask, self.status, self.ws, stream)
        P.purse_megb(db, gp, self.poses, self.mask, self.centre, self.radii, self.nf, self.trace,
                     self.status, self.ws, stream)
        P.purse_megb_backward(db, gp, self.poses, self.mask, self.trace, self.g_radii, self.g_centre,
                              self.g_c, self.g_L, self.g_b, self.ws, stream)

    def outputs(self):
        return [x.clone() for x in (self.poses, self.mask, self.status, self.centre, self.radii,
                                    self.nf, self.trace, self.g_c, self.g_L, self.g_b)]

    def scramble(self):
        for x in (self.poses, self.centre, self.g_c, self.g_L, self.g_b):
            x.fill_(float("nan"))
        for x in (self.mask, self.status, self.nf, self.trace):
            x.fill_(77)
        self.radii.fill_(float("nan"))
        self.ws.fill_(0xAB)


def _same(x, y):
    """Bitwise equality with NaN equal to NaN (an empty instance's centre and
    radii are NaN by contract)."""
    if x.is_floating_point():
        return torch.equal(torch.isnan(x), torch.isnan(y)) and torch.equal(torch.nan_to_num(x), torch.nan_to_num(y))
    return torch.equal(x, y)


def _equal(a, b):
    for x, y in zip(a, b):
        assert _same(x, y)


_CASES = {
    # 12 mixed instances, every MEGB in its chain's workgroup
    "mixed-12": (lambda: W.config_c3(2, n_inst=12, m_range=(256, 2048), n_range=(6, 24)), 20, 256),
    # the 512-instance batch (both kinds, N in 6..48, M in 1,024..16,384)
    "c3-512": (lambda: W.config_c3(0), 20, 512),
    # instances of 2^17 samples: the multi-workgroup first phase (35 launches
    # whose buffers alternate between steps) and rescans of the global shell
    "big-4": (lambda: W.config_c5(1, n_inst=4, n_samples=1 << 17), 20, 1024),
}


@pytest.mark.parametrize("case", sorted(_CASES))
def test_graph_replay_matches_eager(case):
    import paper_2403_09990_amd as P
    _log("case: graph replay,", case)
    make, iters, T = _CASES[case]
    b = make()
    gp = P.purse_default_params(n_iters=iters, megb_iters=T)
    db = P.DeviceBatch(b)
    run = _Run(P, db, gp)
    run()
    torch.cuda.synchronize()
    eager = run.outputs()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    torch.cuda.synchronize()
    for rep in range(3):
        run.scramble()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _log("replay", rep)
        _equal(run.outputs(), eager)
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()

    # the graph reads the inputs at replay time: new seeds give the eager
    # results for those seeds
    db.seed.add_(1000)
    run.scramble()
    g.replay()
    torch.cuda.synchronize()
    replayed = run.outputs()
    run()
    torch.cuda.synchronize()
    _equal(replayed, run.outputs())
    assert not torch.equal(replayed[0], eager[0])
