"""Benchmark of the PURSE hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c5]

A step is one pass of the whole hot path over one batch: the sampler
(prologue + trajectories, purse_sample), the MEGB (purse_megb) and the
backward of the radii and centre (purse_megb_backward of fixed random
cotangents), through the C ABI, on inputs already resident in HBM.  The
default workload is the largest one that fits one GPU: 64 instances of
2D-3D with N = 48 keypoints and 2^20 trajectories each (67,108,864
trajectories, 50 alternating iterations), every instance differentiated in one
backward call.  Prints one JSON line; `value` is samples/s of the whole step,
the forward alone is reported beside it.

Also reported: the sampler and MEGB times separately, the roofline of the
dominant kernel (the trajectory kernel; algorithmic float32 FLOPs per launch
over its average duration, measured with HIP events on the launch stream) and
the FP64 oracle timed on this host on a bounded sample.  After the timed
region one device copy of COPY_BYTES runs as the calibration kernel for HBM
traffic counters read by rocprofv3 on this same command.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pose samples/sec (alt-projection iters) & per-instance MEGB ms, fwd vs fwd+bwd"
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 28              # calibration copy: reads and writes 256 MiB

CONFIGS = {
    "c1": dict(desc="3D-3D single instance, N=8, M=1024, 50 iterations", iters=50),
    "c2": dict(desc="2D-3D single instance, N=12, M=65536, 100 iterations", iters=100),
    "c3": dict(desc="512 uneven instances (50% 3D-3D / 50% 2D-3D), N~U{6..48}, M~U{1024..16384}, "
                    "50 iterations", iters=50),
    "c4": dict(desc="2D-3D single instance, N=24, M=262144, 20 iterations", iters=20),
    "c5": dict(desc="64 instances 2D-3D, N=48, M=1048576 each, 50 iterations", iters=50),
}


def make_batch(cfg, seed=0, n_inst=None):
    from paper_2403_09990_amd import workloads as W
    make = {"c1": W.config_c1, "c2": W.config_c2, "c3": W.config_c3, "c4": W.config_c4, "c5": W.config_c5}[cfg]
    if n_inst is None:
        return make(seed)
    if cfg not in ("c3", "c5"):
        raise SystemExit("--n-inst applies to the multi-instance workloads (c3, c5)")
    return make(seed, n_inst=n_inst)


def read_traffic(kernel, workload):
    """HBM traffic of the kernel from the committed rocprofv3 PMC summary, or
    None if the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    from paper_2403_09990_amd.profile_summary import source_hash
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


def read_valu(kernel, workload):
    """FP32 operations per launch of the kernel from the committed F32 VALU
    counter summary (rocprofv3 --pmc), or None if the kernel sources changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", "valu_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    from paper_2403_09990_amd.profile_summary import source_hash
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash(kernel):
        return None
    return rec.get("f32_flops_per_dispatch")


def per_instance_bench(P, torch, batch, db, gp, stream, no_backward, poses, mask, status, centre, radii, nfeas,
                       trace, g_radii, g_centre, g_c, g_L, g_b, bwd_status, ref, ms_fwd_batched,
                       ms_step_batched):
    """The batch run as one library call per instance (the plain single-instance
    path, as a caller without batching would): sampler, MEGB and backward of
    each instance in turn on the stream, eager, writing into the batched
    outputs' slices of that instance.  Timed like the batched step, and its
    results compared with the batched call's."""
    from paper_2403_09990_amd.workloads import Batch
    so, ko = db.sample_off_host, db.kp_off_host
    calls = []
    for j, ins in enumerate(batch.instances):
        d1 = P.DeviceBatch(Batch([ins]))
        w1 = P.workspace(d1, gp)
        a, b, ka, kb = int(so[j]), int(so[j + 1]), int(ko[j]), int(ko[j + 1])
        calls.append((d1, w1, poses[a:b], mask[a:b], status[j:j + 1], centre[j:j + 1], radii[j:j + 1],
                      nfeas[j:j + 1], trace[j:j + 1], g_radii[j:j + 1], g_centre[j:j + 1], g_c[ka:kb],
                      g_L[ka:kb], g_b[ka:kb], bwd_status[j:j + 1]))

    def fwd():
        for d1, w1, po, ma, st, ce, ra, nf, tr, *_ in calls:
            P.purse_sample(d1, gp, po, ma, st, w1)
            P.purse_megb(d1, gp, po, ma, ce, ra, nf, tr, st, w1)

    def step():
        for d1, w1, po, ma, st, ce, ra, nf, tr, gr, gce, gc, gl, gb, bs in calls:
            P.purse_sample(d1, gp, po, ma, st, w1)
            P.purse_megb(d1, gp, po, ma, ce, ra, nf, tr, st, w1)
            if not no_backward:
                P.purse_megb_backward(d1, gp, po, ma, tr, gr, gce, gc, gl, gb, w1, bwd_status=bs)

    step()
    torch.cuda.synchronize()
    ms_fwd = time_events(fwd, 1, stream)
    ms_step = time_events(step, 1, stream)
    torch.cuda.synchronize()

    def same(a, b):
        return bool(torch.equal(torch.nan_to_num(a, 7.0), torch.nan_to_num(b, 7.0))) if a.is_floating_point() \
            else bool(torch.equal(a, b))
    res = {"calls": len(calls), "fwd_ms": ms_fwd, "fwd_samples_per_s": db.total_samples / (ms_fwd * 1e-3),
           "batched_fwd_speedup": ms_fwd / ms_fwd_batched,
           "samples_equal_batched": same(poses, ref["poses"]) and same(mask, ref["mask"]),
           "radii_equal_batched": same(radii, ref["radii"])}
    if not no_backward:
        res.update({"fwd_bwd_ms": ms_step, "fwd_bwd_samples_per_s": db.total_samples / (ms_step * 1e-3),
                    "batched_fwd_bwd_speedup_vs_eager_step": ms_step / ms_step_batched,
                    "gradients_equal_batched": same(g_c, ref["g_c"]) and same(g_L, ref["g_L"])})
    return res


def _progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_events(fn, reps, stream):
    import torch
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def cpu_baseline(batch, iters, megb_iters, budget_s=20.0):
    """The FP64 oracle on a bounded sample of the same workload: its first
    trajectories of instance 0 (count chosen to take roughly budget_s) plus
    the MEGB of those samples; scaled to samples/s."""
    import torch

    from oracle.megb import megb_from_poses
    from oracle.params import OracleParams
    from oracle.purse import Problem, prologue, sample
    inst = batch.instances[0]
    prob = Problem.from_instance(inst)
    p = OracleParams(n_iters=iters, megb_iters=megb_iters)
    pro = prologue(prob, p)
    t0 = time.perf_counter()
    sample(prob, p, inst.seed, 64, pro=pro)
    t_probe = (time.perf_counter() - t0) / 64
    m = int(max(256, min(inst.n_samples, budget_s * 0.5 / max(t_probe, 1e-6))))
    m = 1 << int(np.log2(m))
    t0 = time.perf_counter()
    out = sample(prob, p, inst.seed, m, pro=pro)
    t_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    megb_from_poses(out["poses"], out["mask"], megb_iters, 10)
    t_m = time.perf_counter() - t0
    return dict(value=m / (t_s + t_m), unit="samples/s", cores=torch.get_num_threads(),
                host_nproc=os.cpu_count(), kind="oracle",
                sample="first %d of %d trajectories of instance 0 (%d iterations) + MEGB (T=%d) of "
                       "those samples; sampler %.2f s, MEGB %.2f s" % (m, inst.n_samples, iters,
                                                                       megb_iters, t_s, t_m))


def walk_bench(P, torch, reps=5):
    """The paper's Step II (strategic random walk, both modes) on an
    LM-O-shaped 2D-3D instance (N = 10 keypoints, 100 starts in S drawn by
    purse_sample) with the paper's CLOSURE and CLOSURE++ walk parameters;
    the paper's own timing of this step (RTX 3090, CuPy) is context only."""
    from paper_2403_09990_amd import workloads as W
    rng = np.random.default_rng(2024)
    inst = W.make_2d3d(rng, 10, 2.0, (5.0, 20.0), 1500)
    db = P.DeviceBatch(W.Batch([inst]))
    gp = P.purse_default_params(n_iters=30)
    out = P.sample(db, gp)
    torch.cuda.synchronize()
    feas = torch.nonzero((out["mask"] & 1) != 0)[:, 0][:100]
    starts = out["poses"][feas].contiguous()
    off = torch.as_tensor([0, starts.shape[0]], dtype=torch.int64, device=starts.device)
    res = {}
    for name, kw in (("closure", dict(n_walks=2, n_iters=5)), ("closure_pp", dict(n_walks=10, n_iters=10))):
        wp = P.purse_walk_default_params(**kw)
        ws = torch.empty(max(1, P.purse_walk_workspace_size(db)), dtype=torch.uint8, device=starts.device)
        nw = starts.shape[0] * wp.n_walks
        poses = torch.empty(2, nw, 12, dtype=torch.float32, device=starts.device)
        mask = torch.empty(2, nw, dtype=torch.uint8, device=starts.device)

        def run():
            P.purse_walk(db, gp, wp, off, starts, poses, mask, None, ws)

        run()
        ms = time_events(run, reps, torch.cuda.current_stream())
        checks = 2 * nw * wp.n_iters * (wp.n_perturb + wp.n_keep * wp.n_scales)
        res[name] = {"ms": ms, "starts": int(starts.shape[0]), "walks_per_mode": nw,
                     "pose_checks": checks, "pose_checks_per_s": checks / (ms * 1e-3),
                     "end_in_S_fraction": float((mask == 1).float().mean())}
    res["paper_context"] = "RTX 3090 / CuPy, LM-O average: 0.0915 s (CLOSURE), 0.6235 s (CLOSURE++)"
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5", choices=sorted(CONFIGS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-reps", type=int, default=5)
    ap.add_argument("--no-backward", action="store_true", help="time the forward alone as the step")
    ap.add_argument("--no-tune", action="store_true", help="default schedule instead of the autotuned one")
    ap.add_argument("--no-graph", action="store_true", help="time the eager step instead of its graph replay")
    ap.add_argument("--no-walk", action="store_true", help="skip the strategic random walk figures")
    ap.add_argument("--no-per-instance", action="store_true",
                    help="skip timing the batch as one call per instance")
    ap.add_argument("--n-inst", type=int, default=None,
                    help="first N instances of c3/c5 only (profiling runs whose per-dispatch counters must stay "
                         "short); the reported workload names the count")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2403_09990_amd as P
    from paper_2403_09990_amd import flops as F

    torch.cuda.set_device(0)
    cfg = CONFIGS[args.config]
    batch = make_batch(args.config, n_inst=args.n_inst)
    gp = P.purse_default_params(n_iters=cfg["iters"])
    db = P.DeviceBatch(batch)
    ws = P.workspace(db, gp)
    dev = db.kind.device
    poses = torch.empty(db.total_samples, 12, dtype=torch.float32, device=dev)
    mask = torch.empty(db.total_samples, dtype=torch.uint8, device=dev)
    status = torch.empty(db.n_inst, dtype=torch.int32, device=dev)
    schedule = "default"
    candidates_ms = None
    _progress("workload", args.config, "samples", db.total_samples)
    if not args.no_tune:
        # the sampler's launch schedule (tile size, tile order, keypoint loop),
        # picked by timing the candidates on this batch before the timed region
        from paper_2403_09990_amd import autotune
        reps = 1 if db.total_samples > (1 << 23) else 3
        gp, rep = autotune.tune(db, gp, ws, poses, mask, status, reps=reps)
        schedule = rep["choice"] if "choice" in rep else "tuned"
        if isinstance(rep.get("candidates_ms"), dict):
            # every candidate's time (warm, HIP events): the spread says how
            # close the choice was, the level how fast this device runs
            candidates_ms = {k: round(float(v), 3) for k, v in rep["candidates_ms"].items()}
    centre = torch.empty(db.n_inst, 12, dtype=torch.float32, device=dev)
    radii = torch.empty(db.n_inst, 2, dtype=torch.float64, device=dev)
    nfeas = torch.empty(db.n_inst, dtype=torch.int64, device=dev)
    trace = torch.empty(db.n_inst, gp.megb_iters, 2, dtype=torch.int32, device=dev)
    rng = np.random.default_rng(0)
    g_radii = torch.as_tensor(rng.normal(size=(db.n_inst, 2)), dtype=torch.float64, device=dev)
    g_centre = torch.as_tensor(rng.normal(size=(db.n_inst, 6)), dtype=torch.float32, device=dev)
    g_c = torch.empty(db.total_kp, 3, dtype=torch.float32, device=dev)
    g_L = torch.empty(db.total_kp, 4, dtype=torch.float32, device=dev)
    g_b = torch.empty(db.total_kp, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    bwd_status = torch.empty(db.n_inst, dtype=torch.int32, device=dev)

    # every call goes to the stream current at call time (the capture stream
    # while the step is being captured into a graph)
    def do_sample(params=gp):
        P.purse_sample(db, params, poses, mask, status, ws)

    def do_megb():
        P.purse_megb(db, gp, poses, mask, centre, radii, nfeas, trace, status, ws)

    def do_backward():
        P.purse_megb_backward(db, gp, poses, mask, trace, g_radii, g_centre, g_c, g_L, g_b, ws,
                              bwd_status=bwd_status)

    def fwd():
        do_sample()
        do_megb()

    def step():
        fwd()
        if not args.no_backward:
            do_backward()

    _progress("schedule", schedule, "; warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the whole step captured once into a HIP graph and replayed in the
    # timed region; the first replay is checked against the eager step
    graph = None
    graph_check = None
    if not args.no_graph:
        ref = [x.clone() for x in (poses, mask, radii, trace, g_c, g_b)]
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
        for x in (poses, g_c, g_b):
            x.fill_(float("nan"))
        radii.fill_(float("nan"))
        trace.fill_(-7)
        graph.replay()
        torch.cuda.synchronize()
        graph_check = all(torch.equal(a, b) if a.dtype not in (torch.float32, torch.float64)
                          else bool(torch.equal(torch.nan_to_num(a, 7.0), torch.nan_to_num(b, 7.0)))
                          for a, b in zip(ref, (poses, mask, radii, trace, g_c, g_b)))
        _progress("graph captured; replay equals the eager step:", graph_check)
    run_step = graph.replay if graph is not None else step
    _progress("timed steps")
    ms_step = time_events(run_step, args.steps, stream)
    ms_step_eager = time_events(step, max(1, args.steps // 2), stream) if graph is not None else ms_step
    _progress("step %.3f ms (eager %.3f ms); breakdown" % (ms_step, ms_step_eager))
    total_m = db.total_samples
    value = total_m / (ms_step * 1e-3)

    # breakdown and roofline of the trajectory kernel (prologue reused so the
    # events bracket the trajectory launches alone)
    ms_fwd = time_events(fwd, args.roofline_reps, stream)
    ms_sample = time_events(do_sample, args.roofline_reps, stream)
    ms_megb = time_events(do_megb, args.roofline_reps, stream)
    ms_bwd = None if args.no_backward else time_events(do_backward, args.roofline_reps, stream)
    gp_reuse = P.purse_default_params(n_iters=cfg["iters"], tile=gp.tile, flags=gp.flags | P.PURSE_FLAG_REUSE_PROLOGUE,
                                      waves_per_simd=gp.waves_per_simd)
    ms_traj = time_events(lambda: do_sample(gp_reuse), args.roofline_reps, stream)
    torch.cuda.synchronize()
    m = mask.cpu().numpy()
    st = status.cpu().numpy()
    rad = radii.cpu().numpy()
    grads_finite = bool(torch.isfinite(g_c).all() and torch.isfinite(g_L).all() and torch.isfinite(g_b).all()) \
        if not args.no_backward else None
    pulled = [int(((m[a:b] & 2) != 0).sum()) for a, b in zip(db.sample_off_host[:-1], db.sample_off_host[1:])]
    bst = None if args.no_backward else bwd_status.cpu().numpy()
    # the method's algorithmic count (per-keypoint model) and the count of the
    # kernels' own formulation, both per trajectory launch
    flops = F.model_batch_flops(batch, cfg["iters"], gp.n_gn, gp.n_bis, pulled)
    flops_kernel = F.batch_flops(batch, cfg["iters"], gp.n_gn)
    achieved = flops / (ms_traj * 1e-3) / 1e12
    # the trajectory kernel that carries the workload: the lane-group variant
    # when the schedule runs 2D-3D trajectories on two or four lanes each
    traj_kernel = ("k_sample2d_lanes" if gp.flags & (P.PURSE_FLAG_PAIR_LANES | P.PURSE_FLAG_QUAD_LANES)
                   else "k_sample")
    wl_key = args.config if args.n_inst is None else "%s_n%d" % (args.config, db.n_inst)
    traffic = read_traffic(traj_kernel, wl_key)
    flops_counted = read_valu(traj_kernel, wl_key)

    # calibration kernel for the traffic counters: a copy of known size
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator shaped like the paper's 2D-3D / 3D-3D workloads)",
        "config": {"workload": "%s: %s" % (args.config, cfg["desc"]) +
                   ("" if args.n_inst is None else " (first %d instances only)" % db.n_inst), "n_inst": db.n_inst,
                   "samples": total_m, "megb_iters": gp.megb_iters,
                   "step": "sample + MEGB" + ("" if args.no_backward else " + backward (all instances, one call)"),
                   "parallelism": "single GPU"},
        "sampler_schedule": schedule,
        "sampler_candidates_ms": candidates_ms,
        "timed_as": "graph replay" if graph is not None else "eager launches",
        "graph_replay_equals_eager": graph_check,
        "ms_per_step_eager": ms_step_eager,
        "fwd_ms": ms_fwd,
        "fwd_samples_per_s": total_m / (ms_fwd * 1e-3),
        "fwd_bwd_ms": None if args.no_backward else ms_step,
        "backward_ms": ms_bwd,
        "gradients_finite": grads_finite,
        **({} if bst is None else {
            "backward_status_counts": {str(k): int(v) for k, v in zip(*np.unique(bst & 0xFF, return_counts=True))},
            "active_set_max": int((bst >> 8).max()), "active_set_mean": float((bst >> 8).mean())}),
        "sampler_ms": ms_sample,
        "trajectory_kernel_ms": ms_traj,
        "megb_ms": ms_megb,
        "megb_ms_per_instance": ms_megb / db.n_inst,
        "megb_us_per_descent_step": ms_megb * 1e3 / gp.megb_iters,
        "sampler_samples_per_s": total_m / (ms_sample * 1e-3),
        "sample_iters_per_s": total_m * cfg["iters"] / (ms_sample * 1e-3),
        "feasible_fraction": float((m & 1).mean()),
        "pulled_in_fraction": float(((m & 2) != 0).mean()),
        "inst_status_nonzero": int((st & 0xFF != 0).sum()),
        "radii_first_instance": [float(rad[0, 0]), float(rad[0, 1])],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic, "kernel": traj_kernel + " (trajectory kernels of the launch)",
                     "flops_per_launch": flops,
                     "frac_nonpacked_ceiling": achieved / (FP32_VECTOR_PEAK_TFLOPS / 2),
                     "flops_per_launch_kernel_formulation": flops_kernel,
                     "frac_kernel_formulation": flops_kernel / (ms_traj * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                     "flops_per_launch_f32_counters": flops_counted,
                     "frac_f32_counters": None if flops_counted is None else
                     flops_counted / (ms_traj * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS},
        # write-out: 12 float32 of pose and one mask byte per sample
        "hbm_write_gbs": total_m * 49 / (ms_traj * 1e-3) / 1e9,
    }
    if db.n_inst > 1 and not args.no_per_instance:
        _progress("the same batch as one call per instance")
        ref = dict(poses=poses.clone(), mask=mask.clone(), radii=radii.clone(), g_c=g_c.clone(), g_L=g_L.clone())
        out["per_instance_calls"] = per_instance_bench(
            P, torch, batch, db, gp, stream, args.no_backward, poses, mask, status, centre, radii, nfeas, trace,
            g_radii, g_centre, g_c, g_L, g_b, bwd_status, ref, ms_fwd, None if args.no_backward else ms_step_eager)
    if not args.no_walk:
        _progress("strategic random walk (LM-O-shaped)")
        out["walk_lmo"] = walk_bench(P, torch)
    if not args.no_cpu_baseline:
        _progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(batch, cfg["iters"], gp.megb_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
