"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2403_09990_amd.profile_summary stats DIR [--title T] [--cmd C]
        Markdown table of the per-kernel statistics (--kernel-trace --stats)
        found under DIR.

    python -m paper_2403_09990_amd.profile_summary traffic FETCH_DIR WRITE_DIR
            --kernel k_sample --copy-bytes B --out FILE.json [--cmd-fetch C] [--cmd-write C]
        HBM bytes per dispatch of a kernel from two --pmc runs (FETCH_SIZE, then
        WRITE_SIZE, both in KiB per dispatch), each scaled by what the same
        counter reads for the calibration copy of B bytes (the largest copy
        kernel of the run).  Stamped with the hash of the kernel sources so a
        stale figure is not reported after the kernels change.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(PKG, "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _find(dirname, suffix):
    hits = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, dirname))
    return hits


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name if len(name) <= 90 else name[:87] + "..."


def stats(dirname, title=None, cmd=None):
    rows = []
    for path in _find(dirname, "kernel_stats.csv"):
        with open(path) as f:
            rows += list(csv.DictReader(f))
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


def _per_dispatch(dirname, counter):
    """{dispatch id: (kernel name, value)} of one counter."""
    vals = {}
    for path in _find(dirname, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                key = (path, r["Dispatch_Id"])
                name = r["Kernel_Name"]
                v = float(r["Counter_Value"])
                prev = vals.get(key, (name, 0.0))[1]
                vals[key] = (name, prev + v)
    return list(vals.values())


def _mean_for(disp, pred):
    v = [x for n, x in disp if pred(n)]
    return (sum(v) / len(v), len(v)) if v else (None, 0)


def traffic(fetch_dir, write_dir, kernel, copy_bytes, out, cmd_fetch=None, cmd_write=None):
    res = {"kernel": kernel, "copy_bytes": copy_bytes, "source_hash": source_hash(),
           "cmd_fetch": cmd_fetch, "cmd_write": cmd_write}
    total = 0.0
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        disp = _per_dispatch(d, counter)
        k_kib, nk = _mean_for(disp, lambda n: kernel in n)
        copies = [x for n, x in disp if "copy" in n.lower()]
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
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--cmd-fetch")
    b.add_argument("--cmd-write")
    args = ap.parse_args(argv)
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
