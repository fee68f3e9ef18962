"""Short text summaries of rocprofv3 CSV output (kernel statistics and
per-dispatch counters), and the calibrated HBM traffic of one kernel.

    python -m paper_1611_01034_amd.profsum stats DIR OUT --cmd "..."
    python -m paper_1611_01034_amd.profsum pmc DIR OUT --cmd "..."
    python -m paper_1611_01034_amd.profsum traffic --fetch F.json --write W.json
        --kernel REGEX --copy REGEX --copy-bytes N --site-bytes B --sites V
        --source FILE[,FILE...] --out OUT.json

`stats` reads *kernel_stats.csv, `pmc` reads *counter_collection.csv found
under DIR (recursively); each writes a text table and a JSON twin (OUT with
.json).  `traffic` scales the FETCH_SIZE and WRITE_SIZE readings of a kernel
by those of a plain copy kernel that moves a known number of bytes each way.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict


def sources_sha256(paths):
    """SHA-256 over the concatenated contents of the given source files (the
    kernel and the headers it is built from)."""
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _find(d, suffix):
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def _col(row, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {list(row)}")


def short(name, n=90):
    s = name.split("(")[0] if not name.startswith("void ") else name[5:].split("(")[0]
    return s if len(s) <= n else s[: n - 3] + "..."


def stats(d, out, cmd, top=25):
    rows = defaultdict(lambda: [0, 0.0])
    for f in _find(d, "kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = short(_col(r, "Name", "KernelName"))
                rows[k][0] += int(_col(r, "Calls"))
                rows[k][1] += float(_col(r, "TotalDurationNs"))
    tot = sum(v[1] for v in rows.values()) or 1.0
    items = sorted(rows.items(), key=lambda kv: -kv[1][1])
    data = [{"kernel": k, "calls": c, "total_ms": t / 1e6, "avg_us": t / c / 1e3, "pct": 100 * t / tot}
            for k, (c, t) in items]
    with open(out, "w") as fh:
        fh.write(f"command: {cmd}\n\n")
        fh.write(f"{'kernel':<92}{'calls':>9}{'total ms':>12}{'avg us':>12}{'%':>7}\n")
        for r in data[:top]:
            fh.write(f"{r['kernel']:<92}{r['calls']:>9}{r['total_ms']:>12.2f}{r['avg_us']:>12.2f}{r['pct']:>7.2f}\n")
        fh.write(f"\n{len(data)} kernels, total GPU kernel time {tot / 1e6:.1f} ms\n")
    with open(os.path.splitext(out)[0] + ".json", "w") as fh:
        json.dump({"command": cmd, "kernels": data}, fh, indent=1)


def pmc(d, out, cmd):
    acc = defaultdict(lambda: defaultdict(list))
    for f in _find(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = short(_col(r, "Kernel_Name", "KernelName"))
                acc[k][_col(r, "Counter_Name", "CounterName")].append(float(_col(r, "Counter_Value", "CounterValue")))
    data = []
    for k, cs in acc.items():
        for c, vals in cs.items():
            data.append({"kernel": k, "counter": c, "dispatches": len(vals), "mean": sum(vals) / len(vals),
                         "min": min(vals), "max": max(vals)})
    with open(out, "w") as fh:
        fh.write(f"command: {cmd}\n\n")
        fh.write(f"{'kernel':<92}{'counter':>14}{'n':>5}{'mean/dispatch':>16}{'min':>14}{'max':>14}\n")
        for r in data:
            fh.write(f"{r['kernel']:<92}{r['counter']:>14}{r['dispatches']:>5}{r['mean']:>16.1f}"
                     f"{r['min']:>14.1f}{r['max']:>14.1f}\n")
        fh.write("\nFETCH_SIZE and WRITE_SIZE are in KiB per dispatch.\n")
    with open(os.path.splitext(out)[0] + ".json", "w") as fh:
        json.dump({"command": cmd, "rows": data}, fh, indent=1)


def _mean_for(rows, kernel_re, counter):
    vals = [r["mean"] for r in rows if re.search(kernel_re, r["kernel"]) and r["counter"] == counter]
    if len(vals) != 1:
        raise SystemExit(f"expected one row for /{kernel_re}/ {counter}, got {len(vals)}")
    return vals[0]


def traffic(a):
    with open(a.fetch) as fh:
        fr = json.load(fh)["rows"]
    with open(a.write) as fh:
        wr = json.load(fh)["rows"]
    f_k = _mean_for(fr, a.kernel, "FETCH_SIZE")
    w_k = _mean_for(wr, a.kernel, "WRITE_SIZE")
    f_c = _mean_for(fr, a.copy, "FETCH_SIZE")
    w_c = _mean_for(wr, a.copy, "WRITE_SIZE")
    sf = a.copy_bytes / f_c
    sw = a.copy_bytes / w_c
    fetch_b = f_k * sf
    write_b = w_k * sw
    alg = a.site_bytes * a.sites
    src = sources_sha256(a.source.split(","))
    res = {"kernel": a.kernel, "copy_kernel": a.copy, "fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k,
           "copy_fetch_kib": f_c, "copy_write_kib": w_c, "copy_bytes_each_way": a.copy_bytes,
           "scale_fetch": sf, "scale_write": sw, "fetch_bytes": fetch_b, "write_bytes": write_b,
           "bytes_per_launch": fetch_b + write_b, "algorithmic_bytes_per_launch": alg,
           "traffic_over_algorithmic": (fetch_b + write_b) / alg,
           "source": [os.path.relpath(x) for x in a.source.split(",")], "source_sha256": src,
           "commands": {"fetch": json.load(open(a.fetch))["command"], "write": json.load(open(a.write))["command"]}}
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sp = ap.add_subparsers(dest="mode", required=True)
    for m in ("stats", "pmc"):
        p = sp.add_parser(m)
        p.add_argument("dir")
        p.add_argument("out")
        p.add_argument("--cmd", required=True)
    p = sp.add_parser("traffic")
    for k in ("--fetch", "--write", "--kernel", "--copy", "--source", "--out"):
        p.add_argument(k, required=True)
    p.add_argument("--copy-bytes", type=float, required=True)
    p.add_argument("--site-bytes", type=float, required=True)
    p.add_argument("--sites", type=float, required=True)
    a = ap.parse_args(argv)
    if a.mode == "stats":
        stats(a.dir, a.out, a.cmd)
    elif a.mode == "pmc":
        pmc(a.dir, a.out, a.cmd)
    else:
        traffic(a)


if __name__ == "__main__":
    sys.exit(main())
