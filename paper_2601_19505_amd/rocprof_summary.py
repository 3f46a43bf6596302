"""Per-kernel summary of rocprofv3 results for the step kernels.

    python -m paper_2601_19505_amd.rocprof_summary DIR [--last K] [--copy-bytes B]
                                                    [--copy-kernel SUBSTR] [--title T]

Reads what rocprofv3 wrote under DIR (CSV files from `--output-format csv`,
or rocpd SQLite databases) and prints, per kernel name, statistics over the
last K dispatches of that kernel (the steady-state steps at the end of a
run): mean / min / max duration in milliseconds from the kernel trace, and
the mean per dispatch of every collected counter.

HBM traffic calibration: with --copy-bytes B, the dispatches whose kernel
name contains SUBSTR (default "neg") are taken as a streaming kernel that
reads B bytes and writes B bytes.  FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) of that kernel give the factors f = counter * 1024 / B, and each
kernel's counters are also printed divided by f, as calibrated bytes per
dispatch.
"""
import argparse
import collections
import csv
import glob
import os
import sqlite3


def _rows_csv(d):
    trace, ctr = [], []
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                r = {k.lower(): v for k, v in r.items()}
                trace.append((r["kernel_name"], int(r["dispatch_id"]), int(r["start_timestamp"]),
                              int(r["end_timestamp"])))
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                r = {k.lower(): v for k, v in r.items()}
                ctr.append((r["kernel_name"], int(r["dispatch_id"]), r["counter_name"],
                            float(r["counter_value"])))
    return trace, ctr


def _rows_db(d):
    trace, ctr = [], []
    for f in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
        c = sqlite3.connect(f)
        views = {r[0] for r in c.execute("select name from sqlite_master where type in ('view','table')")}
        if "kernels" in views:
            trace += list(c.execute("select name, dispatch_id, start, end from kernels"))
        if "counters_collection" in views:
            ctr += list(c.execute("select kernel_name, dispatch_id, counter_name, value "
                                  "from counters_collection"))
        c.close()
    return trace, ctr


def summarize(d, last=100, copy_bytes=None, copy_kernel="neg"):
    trace, ctr = _rows_csv(d)
    if not trace and not ctr:
        trace, ctr = _rows_db(d)
    out = {}
    by_k = collections.defaultdict(list)
    for name, disp, t0, t1 in trace:
        by_k[name].append((disp, (t1 - t0) * 1e-6))
    for name, lst in by_k.items():
        lst.sort()
        sel = [x[1] for x in lst[-last:]]
        out.setdefault(name, {})["duration_ms"] = (sum(sel) / len(sel), min(sel), max(sel), len(sel),
                                                   len(lst))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for name, disp, cname, v in ctr:
        per[(name, disp)][cname] += v
    by_kc = collections.defaultdict(list)
    for (name, disp), cv in per.items():
        by_kc[name].append((disp, cv))
    for name, lst in by_kc.items():
        lst.sort()
        sel = lst[-last:]
        keys = sorted({k for _, cv in sel for k in cv})
        out.setdefault(name, {})["counters"] = {k: sum(cv.get(k, 0.0) for _, cv in sel) / len(sel)
                                                for k in keys}
        out[name]["counter_dispatches"] = len(sel)
    factors = {}
    if copy_bytes:
        for name, v in out.items():
            if copy_kernel in name and "counters" in v:
                for k in ("FETCH_SIZE", "WRITE_SIZE"):
                    if k in v["counters"]:
                        factors[k] = v["counters"][k] * 1024.0 / copy_bytes
    return out, factors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--last", type=int, default=100)
    ap.add_argument("--copy-bytes", type=float, default=None)
    ap.add_argument("--copy-kernel", default="neg")
    ap.add_argument("--title", default="")
    a = ap.parse_args()
    out, factors = summarize(a.dir, a.last, a.copy_bytes, a.copy_kernel)
    if a.title:
        print(f"# {a.title}")
    from paper_2601_19505_amd import source_digest
    print(f"# kernel source sha256: {source_digest()}")
    if factors:
        print("# calibration factors (counter KiB * 1024 / bytes of the copy kernel): " +
              ", ".join(f"{k} {v:.4f}" for k, v in factors.items()))
    for name in sorted(out, key=lambda n: -out[n].get("duration_ms", (0,))[0]):
        v = out[name]
        print(name[:160])
        if "duration_ms" in v:
            m, lo, hi, n, tot = v["duration_ms"]
            print(f"    duration_ms mean {m:.4f} min {lo:.4f} max {hi:.4f} "
                  f"(last {n} of {tot} dispatches)")
        for k, x in v.get("counters", {}).items():
            line = f"    {k:24s} {x:.6g} per dispatch (last {v['counter_dispatches']})"
            if k in factors and factors[k] > 0:
                line += f"  -> calibrated {x * 1024.0 / factors[k] / 1e9:.4f} GB"
            print(line)


if __name__ == "__main__":
    main()
