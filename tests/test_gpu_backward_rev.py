"""The backward's reverse sweep over 2D-3D trajectories (one per active
sample) against its forward mode (one re-run per input direction,
PURSE_FLAG_FORWARD_TANGENTS): the same derivative of the same float32
computation, so the gradients agree to float32 rounding of two summation
orders (relative 2e-3 of each array's largest entry).  The forward mode is
itself checked against the oracle's reverse pass (test_gpu_backward.py)."""
import sys

import numpy as np
import pytest
import torch

from paper_2403_09990_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu
RTOL = 2e-3


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _grads(P, res, gp, flags, g_radii, g_centre):
    db = res["db"]
    dev = res["poses"].device
    gpf = P.purse_default_params(**{f: getattr(gp, f) for f, _ in type(gp)._fields_})
    gpf.flags = gp.flags | flags
    g = [torch.full((db.total_kp, k), float("nan"), dtype=torch.float32, device=dev) for k in (3, 4)]
    g.append(torch.full((db.total_kp,), float("nan"), dtype=torch.float32, device=dev))
    st = torch.full((db.n_inst,), -1, dtype=torch.int32, device=dev)
    P.purse_megb_backward(db, gpf, res["poses"], res["mask"], res["trace"],
                          torch.as_tensor(g_radii, dtype=torch.float64, device=dev),
                          torch.as_tensor(g_centre, dtype=torch.float32, device=dev), g[0], g[1], g[2], res["ws"],
                          bwd_status=st)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in g], st.cpu().numpy()


_CASES = {
    # 2D-3D, N = 12, 65,536 samples, 40 iterations (80 passes on the tape)
    "c2": (lambda: W.config_c2(0), 40),
    # 2D-3D, N = 24, 20 iterations: most samples pulled in by bisection
    "c4-64k": (lambda: W.config_c4(0, n_samples=65536), 20),
    # the headline instances (N = 48) at 2^16 samples, 50 iterations
    "c5-4": (lambda: W.config_c5(0, n_inst=4, n_samples=1 << 16), 50),
    # both kinds in one batch (3D-3D stays in forward mode)
    "mixed-10": (lambda: W.config_c3(3, n_inst=10, m_range=(2000, 8000), n_range=(6, 48)), 30),
    # 160 iterations (320 passes): the largest tape
    "c1-2d-160": (lambda: W.Batch([W.make_2d3d(np.random.default_rng(9), 10, 2.0, (5.0, 20.0), 4096)]), 160),
}


@pytest.mark.parametrize("case", sorted(_CASES))
def test_reverse_sweep_equals_forward_mode(case):
    import paper_2403_09990_amd as P
    _log("case: reverse vs forward tangents", case)
    make, iters = _CASES[case]
    b = make()
    gp = P.purse_default_params(n_iters=iters)
    res = PT.run_gpu(b, gp)
    rng = np.random.default_rng(11)
    g_radii = rng.normal(size=(b.n_inst, 2))
    g_centre = rng.normal(size=(b.n_inst, 6))
    rev, st_r = _grads(P, res, gp, 0, g_radii, g_centre)
    fwd, st_f = _grads(P, res, gp, P.PURSE_FLAG_FORWARD_TANGENTS, g_radii, g_centre)
    assert np.array_equal(st_r, st_f)
    ok = (st_r & 0xFF) == P.PURSE_BWD_OK
    assert ok.any()
    for name, a, c in zip(("g_centres", "g_shapes", "g_bounds"), rev, fwd):
        assert np.array_equal(np.isnan(a), np.isnan(c)), name
        a, c = np.nan_to_num(a), np.nan_to_num(c)
        scale = max(np.abs(c).max(), 1e-12)
        err = np.abs(a - c).max() / scale
        _log(name, "max |rev - fwd| / max |fwd| =", err, "scale", scale)
        assert err <= RTOL, (name, err)
