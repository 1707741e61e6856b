"""Autotuner of the sampler's launch schedule.

The sampler's results do not depend on the schedule: only the workgroup size
(params.tile: 64, 128 or 256 samples), the tile order (heaviest instances
first, or instance order with PURSE_FLAG_INSTANCE_ORDER) and, for 2D-3D
instances of at most 16 keypoints, the keypoint loop (unrolled; the general
one with PURSE_FLAG_GENERIC_LOOP; two or four lanes per trajectory with
PURSE_FLAG_PAIR_LANES or PURSE_FLAG_QUAD_LANES) change its speed; the last
three change float32 rounding only.  A second stage tries, on the fastest of
those, the persistent work-queue kernels (PURSE_FLAG_WORK_QUEUE), caps of 4
and 2 resident wavefronts per SIMD (params.waves_per_simd) and the launch
groups one after the other on one stream (PURSE_FLAG_SERIAL_GROUPS; by
default they run concurrently, which overlaps their tails on mixed batches
but costs a fork and a join on single-group ones), alone and with either
cap, which change speed only.
tune() times every candidate with HIP events on the given batch and keeps the
fastest; the choice is cached in a JSON file keyed by the workload's
signature (kinds, keypoint counts, sample counts, iteration counts, device
name), so later calls on the same shape skip the timing.
"""
import hashlib
import json
import os
from typing import Optional

from . import (PURSE_FLAG_GENERIC_LOOP, PURSE_FLAG_INSTANCE_ORDER, PURSE_FLAG_PAIR_LANES, PURSE_FLAG_QUAD_LANES,
               PURSE_FLAG_SERIAL_GROUPS, PURSE_FLAG_WORK_QUEUE, purse_default_params, purse_sample)

TILES = (64, 128, 256)
ORDERS = (0, PURSE_FLAG_INSTANCE_ORDER)
LOOPS = (0, PURSE_FLAG_GENERIC_LOOP, PURSE_FLAG_PAIR_LANES, PURSE_FLAG_QUAD_LANES)
SMALL_N = 16
_TUNED = (PURSE_FLAG_INSTANCE_ORDER | PURSE_FLAG_GENERIC_LOOP | PURSE_FLAG_PAIR_LANES | PURSE_FLAG_QUAD_LANES |
          PURSE_FLAG_WORK_QUEUE | PURSE_FLAG_SERIAL_GROUPS)
# second stage, on the fastest tile / order / loop: (flags, waves per SIMD)
STAGE2 = ((PURSE_FLAG_WORK_QUEUE, 0), (0, 4), (0, 2), (PURSE_FLAG_SERIAL_GROUPS, 0),
          (PURSE_FLAG_SERIAL_GROUPS | PURSE_FLAG_WORK_QUEUE, 0), (PURSE_FLAG_SERIAL_GROUPS, 4),
          (PURSE_FLAG_SERIAL_GROUPS, 2))


def default_cache_path() -> str:
    return os.environ.get("PURSE_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "purse_autotune.json"))


def signature(db, params) -> str:
    """Key of a workload: everything the schedule's speed depends on."""
    import numpy as np
    import torch
    kinds = db.kind.cpu().numpy()
    nkp = db.n_kp.cpu().numpy()
    m = np.diff(db.sample_off_host)
    h = hashlib.sha256()
    for a in (kinds, nkp, m):
        h.update(np.ascontiguousarray(a).tobytes())
    dev = torch.cuda.get_device_name(db.kind.device)
    return "%s|n%d|it%d|gn%d|bis%d|%s" % (dev, db.n_inst, params.n_iters, params.n_gn, params.n_bis,
                                          h.hexdigest()[:16])


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    """Writes the cache; an unwritable location only costs the caching."""
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _with(params, tile, flags, waves=0):
    p = purse_default_params()
    for name, _ in type(params)._fields_:
        setattr(p, name, getattr(params, name))
    p.tile = tile
    p.flags = (params.flags & ~_TUNED) | flags
    p.waves_per_simd = waves
    return p


def _name(tile, flags, waves=0):
    loop = ("generic" if flags & PURSE_FLAG_GENERIC_LOOP else
            "quad-lanes" if flags & PURSE_FLAG_QUAD_LANES else
            "pair-lanes" if flags & PURSE_FLAG_PAIR_LANES else "unrolled")
    name = "%d/%s/%s" % (tile, "instance" if flags & PURSE_FLAG_INSTANCE_ORDER else "heaviest-first", loop)
    if flags & PURSE_FLAG_WORK_QUEUE:
        name += "/queue"
    if flags & PURSE_FLAG_SERIAL_GROUPS:
        name += "/serial"
    if waves:
        name += "/%dwaves" % waves
    return name


def tune(db, params, ws, poses, mask, inst_status, stream=None, reps: int = 3,
         cache: Optional[str] = None, force: bool = False):
    """Returns (params with the fastest tile and order, report dict).

    The candidates run on the caller's buffers (poses, mask, inst_status and
    the workspace are overwritten)."""
    import torch
    path = cache or default_cache_path()
    key = signature(db, params)
    table = _load(path)
    rec = table.get(key)
    if not force and isinstance(rec, dict) and "tile" in rec and "flags" in rec:
        return _with(params, rec["tile"], rec["flags"], rec.get("waves", 0)), dict(rec, cached=True)
    if stream is None:
        stream = torch.cuda.current_stream()
    loops = LOOPS if db.max_kp <= SMALL_N and bool((db.kind == 1).any()) else (0,)
    times, cand = {}, {}

    def run(tile, flags, waves):
        p = _with(params, tile, flags, waves)
        purse_sample(db, p, poses, mask, inst_status, ws, stream)  # warm-up
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(reps):
            purse_sample(db, p, poses, mask, inst_status, ws, stream)
        e.record(stream)
        e.synchronize()
        name = _name(tile, flags, waves)
        times[name] = s.elapsed_time(e) / reps
        cand[name] = (tile, flags, waves)

    for tile in TILES:
        for order in ORDERS:
            for loop in loops:
                run(tile, order | loop, 0)
    tile, flags, _ = cand[min(times, key=times.get)]
    for extra, waves in STAGE2:
        run(tile, flags | extra, waves)
    best = min(times, key=times.get)
    tile, flags, waves = cand[best]
    rec = {"tile": tile, "flags": flags, "waves": waves, "choice": best, "ms": times[best], "candidates_ms": times}
    table[key] = rec
    _store(path, table)
    return _with(params, tile, flags, waves), dict(rec, cached=False)
