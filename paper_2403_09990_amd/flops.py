"""Algorithmic float32 operation counts of the sampler, per trajectory.

Counted from the arithmetic the method performs in the formulation the kernels
use (fused multiply-add = 2, add / multiply / compare / reciprocal / square
root / reciprocal square root / sin / cos = 1; selects, moves and integer work
= 0).  The counts follow the kernels' source on the common path (no float64
polar fallback, no pull-in).

2D-3D, per alternating iteration with N keypoints and n_gn Gauss-Newton steps:
  first step, per keypoint   164  (transform + projection 25, projection
                                   target and whitened residual 15, pivot
                                   offset 3, whitened Jacobian rows and the
                                   normal-equation update 121)
  each later step, per kp    196  (targets recomputed from the projection
                                   pose 37 + residual 10, transform +
                                   projection 25, pivot 3, Jacobian and
                                   update 121)
  per step                   282  (6x6 Cholesky and two solves 169, Exp and
                                   the left update 113)
3D-3D, per iteration: per keypoint 56 (transform and residual 21, squared
  norm 5, clamp 3, target 6, accumulation of M 18 and qbar 3), plus 889 (the
  centroid offset 18, the polar step 850: M^T M 45, four Jacobi sweeps
  12 x 40, the normalised images and cross products 80, R assembly 45, Newton
  polish 185, det 14; and the translation 21).
Per trajectory: the start (Philox draw and offset, 150) and the final
feasibility test (2D-3D 40 N + Bjorck step 90; 3D-3D 30 N).
"""

PER_KP_GN_FIRST = 164
PER_KP_GN_LATER = 196
PER_GN_STEP = 282
PER_KP_3D = 56
PER_ITER_3D = 889
START = 150


def per_trajectory(kind: int, n_kp: int, n_iters: int, n_gn: int = 2) -> int:
    if kind == 1:
        it = n_kp * (PER_KP_GN_FIRST + (n_gn - 1) * PER_KP_GN_LATER) + n_gn * PER_GN_STEP
        return START + n_iters * it + 40 * n_kp + 90
    it = n_kp * PER_KP_3D + PER_ITER_3D
    return START + n_iters * it + 30 * n_kp


def batch_flops(batch, n_iters: int, n_gn: int = 2) -> int:
    return sum(ins.n_samples * per_trajectory(ins.kind, ins.n_kp, n_iters, n_gn)
               for ins in batch.instances)


# ---------------------------------------------------------------------------
# The method's algorithmic count by the rough per-keypoint model of the
# method's arithmetic (fused multiply-add = 2, other operations = 1): per
# sample-iteration 56 N + 650 (3D-3D: transform, projection onto the ball,
# accumulation; polar step about 550 and composition about 100) and
# 40 N + n_gn (190 N + 400) (2D-3D: projection onto the ellipse, then per
# Gauss-Newton step the Jacobian, whitening and normal equations per keypoint
# and the 6x6 Cholesky, solves, Exp and composition); per sample a final
# feasibility pass of 25 N, and n_bis (25 N + 60) for each sample pulled in by
# bisection.  This is the count the roofline fraction is reported against;
# per_trajectory above is the count of the kernels' own formulation.

def model_per_iteration(kind: int, n_kp: int, n_gn: int = 2) -> int:
    if kind == 1:
        return 40 * n_kp + n_gn * (190 * n_kp + 400)
    return 56 * n_kp + 650


def model_batch_flops(batch, n_iters: int, n_gn: int = 2, n_bis: int = 16, pulled=None) -> int:
    """pulled: per instance, the number of samples pulled in (None: 0)."""
    tot = 0
    for j, ins in enumerate(batch.instances):
        n = ins.n_kp
        tot += ins.n_samples * (n_iters * model_per_iteration(ins.kind, n, n_gn) + 25 * n)
        if pulled is not None:
            tot += int(pulled[j]) * n_bis * (25 * n + 60)
    return tot
