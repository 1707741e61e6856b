"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2403_09990_amd.profile_summary stats DIR [--title T] [--cmd C]
        Markdown table of the per-kernel statistics (--kernel-trace --stats)
        found under DIR.

    python -m paper_2403_09990_amd.profile_summary shapes DIR [--match NAME]
        Per (kernel, workgroup size, grid size) statistics (rocpd database).

    python -m paper_2403_09990_amd.profile_summary counters DIR --kernel NAME
        Mean per dispatch of every counter of a --pmc run for one kernel, over
        the dispatches that carry the workload.

    python -m paper_2403_09990_amd.profile_summary valu DIR --kernel NAME [--out FILE.json] [--cmd C]
        FP32 operations per dispatch from the F32 VALU instruction counters
        (SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F32), stamped like traffic.

    python -m paper_2403_09990_amd.profile_summary traffic FETCH_DIR WRITE_DIR
            --kernel k_sample --copy-bytes B --out FILE.json [--cmd-fetch C] [--cmd-write C]
        HBM bytes per dispatch of a kernel from two --pmc runs (FETCH_SIZE, then
        WRITE_SIZE, both in KiB per dispatch), each scaled by what the same
        counter reads for the calibration copy of B bytes (the largest copy
        kernel of the run).  Stamped with the hash of the kernel's sources so a
        stale figure is not reported after they change.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sqlite3
import sys

PKG = os.path.dirname(os.path.abspath(__file__))


# Sources each profiled kernel is compiled from (the file that defines it and
# every header it includes); other kernels: all of csrc/.
_SAMPLER_SOURCES = ("csrc/purse_sample.hip", "csrc/purse_launch.hpp", "csrc/purse_traj.hpp", "csrc/purse_device.hpp",
                    "csrc/purse_dual.hpp", "csrc/purse_layout.hpp", "../include/purse.h")
KERNEL_SOURCES = {"k_sample": _SAMPLER_SOURCES, "k_sample2d_lanes": _SAMPLER_SOURCES}


def source_hash(kernel=None) -> str:
    """Hash of the sources the kernel is built from, so that a traffic figure
    is not reported once they have changed."""
    h = hashlib.sha256()
    base = kernel.split("<")[0].strip() if kernel else None
    if base in KERNEL_SOURCES:
        files = [os.path.normpath(os.path.join(PKG, f)) for f in KERNEL_SOURCES[base]]
    else:
        d = os.path.join(PKG, "csrc")
        files = [os.path.join(d, f) for f in sorted(os.listdir(d))]
    for f in files:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _find(dirname, suffix, required=True):
    hits = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    if not hits and required:
        raise FileNotFoundError("no *%s under %s" % (suffix, dirname))
    return hits


def _db_rows(dirname, query):
    """Rows of a query over every rocpd database (*_results.db) under dirname."""
    rows = []
    for path in _find(dirname, "results.db"):
        con = sqlite3.connect(path)
        try:
            cur = con.execute(query)
            names = [d[0] for d in cur.description]
            rows += [dict(zip(names, r), _path=path) for r in cur.fetchall()]
        finally:
            con.close()
    return rows


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name if len(name) <= 90 else name[:87] + "..."


def _kernel_rows(dirname):
    """Per-kernel statistics, from the CSV output or the rocpd database."""
    rows = []
    for path in _find(dirname, "kernel_stats.csv", required=False):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    if rows:
        return rows
    disp = _db_rows(dirname, "select name, duration from kernels")
    by = {}
    for r in disp:
        by.setdefault(r["name"], []).append(float(r["duration"]))
    total = sum(sum(v) for v in by.values()) or 1.0
    for name, v in by.items():
        rows.append({"Name": name, "Calls": str(len(v)), "TotalDurationNs": sum(v),
                     "AverageNs": sum(v) / len(v), "MinNs": min(v), "MaxNs": max(v),
                     "Percentage": 100.0 * sum(v) / total})
    return rows


def stats(dirname, title=None, cmd=None):
    rows = _kernel_rows(dirname)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = []
    if title:
        out.append("# " + title)
        out.append("")
    if cmd:
        out.append("Command: `%s`" % cmd)
        out.append("")
    out.append("| kernel | calls | avg us | min us | max us | total ms | % |")
    out.append("|---|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        out.append("| %s | %s | %.2f | %.2f | %.2f | %.3f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    return "\n".join(out) + "\n"


def shapes(dirname, match=None):
    """Per (kernel, workgroup size, grid size) statistics from the rocpd
    database: the autotuner's candidates and the timed launches of one kernel
    show up as separate rows."""
    q = ("select name, workgroup_x, grid_x, count(*) as n, avg(duration) as a, min(duration) as lo, "
         "max(duration) as hi, vgpr_count, sgpr_count from kernels group by name, workgroup_x, grid_x")
    rows = [r for r in _db_rows(dirname, q) if match is None or match in r["name"]]
    rows.sort(key=lambda r: (r["name"], r["workgroup_x"]))
    out = ["| kernel | workgroup | grid (threads) | calls | avg us | min us | max us | VGPRs | SGPRs |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| %s | %d | %d | %d | %.2f | %.2f | %.2f | %d | %d |" % (
            _short(r["name"]), r["workgroup_x"], r["grid_x"], r["n"], r["a"] / 1e3, r["lo"] / 1e3, r["hi"] / 1e3,
            r["vgpr_count"], r["sgpr_count"]))
    return "\n".join(out) + "\n"


def _per_dispatch(dirname, counter):
    """[(kernel name, value)] of one counter, one entry per dispatch (values
    of the counter's instances summed)."""
    vals = {}
    for path in _find(dirname, "counter_collection.csv", required=False):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                key = (path, r["Dispatch_Id"])
                prev = vals.get(key, (r["Kernel_Name"], 0.0))[1]
                vals[key] = (r["Kernel_Name"], prev + float(r["Counter_Value"]))
    if not vals:
        q = ("select dispatch_id, kernel_name, value from counters_collection where counter_name = '%s'"
             % counter)
        for r in _db_rows(dirname, q):
            key = (r["_path"], r["dispatch_id"])
            prev = vals.get(key, (r["kernel_name"], 0.0))[1]
            vals[key] = (r["kernel_name"], prev + float(r["value"]))
    return list(vals.values())


def _counter_dispatches(dirname, kernel):
    """{dispatch: {counter: value}} of every dispatch of the matching kernels
    (values of a counter's instances summed)."""
    q = "select dispatch_id, kernel_name, counter_name, value from counters_collection"
    acc = {}
    for r in _db_rows(dirname, q):
        if kernel not in r["kernel_name"]:
            continue
        d = acc.setdefault((r["_path"], r["dispatch_id"]), {})
        d[r["counter_name"]] = d.get(r["counter_name"], 0.0) + float(r["value"])
    return acc


def counters(dirname, kernel):
    """Mean per dispatch of every counter collected for the dispatches of
    kernel that carry the workload: those whose VALU instruction count (or,
    without it, the sum of all counters) is within half of the largest.  A
    warm-up launch of a few iterations or a launch group with no instances
    (whose workgroups exit at once) would otherwise pull the mean down."""
    acc = _counter_dispatches(dirname, kernel)
    if not acc:
        return {}

    def weight(d):
        return d["SQ_INSTS_VALU"] if "SQ_INSTS_VALU" in d else sum(d.values())

    top = max(weight(d) for d in acc.values())
    keep = [d for d in acc.values() if weight(d) >= 0.5 * top]
    names = sorted(set().union(*keep))
    res = {c: sum(d.get(c, 0.0) for d in keep) / len(keep) for c in names}
    res["dispatches"] = len(keep)
    res["dispatches_dropped"] = len(acc) - len(keep)
    return res


# FP32 VALU counters and the operations each instruction counts for
_F32_OPS = {"SQ_INSTS_VALU_FMA_F32": 2, "SQ_INSTS_VALU_MUL_F32": 1, "SQ_INSTS_VALU_ADD_F32": 1,
            "SQ_INSTS_VALU_TRANS_F32": 1}


def valu(dirname, kernel, out=None, cmd=None):
    """FP32 operations per dispatch of a kernel from the F32 VALU instruction
    counters: 64 lanes x (2 FMA + MUL + ADD + TRANS) wave instructions (the
    library is compiled with packed FP32 instructions disabled), stamped with the hash
    of the kernel's sources."""
    c = counters(dirname, kernel)
    missing = [k for k in _F32_OPS if k not in c]
    if missing:
        raise RuntimeError("counters %s not collected for %s in %s" % (missing, kernel, dirname))
    res = {"kernel": kernel, "source_hash": source_hash(kernel), "cmd": cmd, "counters": c,
           "f32_flops_per_dispatch": 64.0 * sum(w * c[k] for k, w in _F32_OPS.items())}
    if "SQ_ACTIVE_INST_VALU" in c and c.get("SQ_WAVE_CYCLES"):
        res["valu_active_per_wave_cycle"] = c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"]
    if out:
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
    return res


def _mean_for(disp, pred):
    """Mean over the dispatches of the matching kernels that carry the
    workload: those within half of the largest (a launch group with no
    instances, whose workgroups exit at once, would otherwise pull the mean
    down)."""
    v = [x for n, x in disp if pred(n)]
    if not v:
        return None, 0
    top = max(v)
    v = [x for x in v if x >= 0.5 * top]
    return sum(v) / len(v), len(v)


def traffic(fetch_dir, write_dir, kernel, copy_bytes, out, cmd_fetch=None, cmd_write=None):
    res = {"kernel": kernel, "copy_bytes": copy_bytes, "source_hash": source_hash(kernel),
           "cmd_fetch": cmd_fetch, "cmd_write": cmd_write}
    total = 0.0
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        disp = _per_dispatch(d, counter)
        k_kib, nk = _mean_for(disp, lambda n: kernel in n)
        copies = [x for n, x in disp if "copy" in n.lower() or "elementwise" in n.lower()]
        if k_kib is None or not copies:
            raise RuntimeError("%s: kernel or calibration copy not found in %s" % (counter, d))
        c_kib = max(copies)
        factor = c_kib * 1024.0 / copy_bytes
        res[tag] = {"counter": counter, "kernel_kib_per_dispatch": k_kib, "dispatches": nk,
                    "copy_kib": c_kib, "factor": factor, "bytes_per_dispatch": k_kib * 1024.0 / factor}
        total += k_kib * 1024.0 / factor
    res["bytes_per_launch"] = total
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--title")
    a.add_argument("--cmd")
    a.add_argument("--out")
    sh = sub.add_parser("shapes")
    sh.add_argument("dir")
    sh.add_argument("--match")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", required=True)
    v = sub.add_parser("valu")
    v.add_argument("dir")
    v.add_argument("--kernel", required=True)
    v.add_argument("--out")
    v.add_argument("--cmd")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--cmd-fetch")
    b.add_argument("--cmd-write")
    args = ap.parse_args(argv)
    if args.mode == "shapes":
        sys.stdout.write(shapes(args.dir, args.match))
        return
    if args.mode == "counters":
        print(json.dumps(counters(args.dir, args.kernel), indent=1))
        return
    if args.mode == "valu":
        print(json.dumps(valu(args.dir, args.kernel, args.out, args.cmd), indent=1))
        return
    if args.mode == "stats":
        text = stats(args.dir, args.title, args.cmd)
        if args.out:
            open(args.out, "w").write(text)
        sys.stdout.write(text)
    else:
        print(json.dumps(traffic(args.fetch_dir, args.write_dir, args.kernel, args.copy_bytes, args.out,
                                 args.cmd_fetch, args.cmd_write), indent=1))


if __name__ == "__main__":
    main()
