"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2201_04269_amd.prof_summary trace DIR            # --kernel-trace --stats
    python -m paper_2201_04269_amd.prof_summary counters DIR [DIR..] # --pmc runs (any counters)
    python -m paper_2201_04269_amd.prof_summary traffic FETCH WRITE CAL_FETCH CAL_WRITE CAL_BYTES

`traffic` scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what the same
counters read for a plain elementwise kernel of known traffic (CAL_BYTES read
and CAL_BYTES written per dispatch), and prints HBM bytes per dispatch per
kernel, with the hash of the kernel sources the numbers belong to.
"""
import collections
import csv
import os
import re
import sys

from paper_2201_04269_amd.build import source_hash


def _short(name):
    m = re.search(r"::(\w+)(<[^(]*>)?\(", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    m = re.search(r"(\w+)(<.*>)?$", name.split("(")[0])
    return (m.group(0) if m else name)[:80]


def _csv(dirname, suffix):
    for f in sorted(os.listdir(dirname)):
        if f.endswith(suffix):
            with open(os.path.join(dirname, f)) as fh:
                return list(csv.DictReader(fh))
    raise SystemExit(f"no *{suffix} in {dirname}")


def trace(dirname):
    rows = _csv(dirname, "kernel_stats.csv")
    print(f"{'kernel':58s} {'calls':>6s} {'avg ms':>10s} {'total ms':>10s} {'%':>6s}")
    for r in rows:
        print(f"{_short(r['Name']):58s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:10.3f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")


def _per_dispatch(dirname):
    """{kernel: [ {counter: value} per dispatch ]} and durations (ns) per dispatch."""
    rows = _csv(dirname, "counter_collection.csv")
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    dur = {}
    for r in rows:
        k = (int(r["Dispatch_Id"]), _short(r["Kernel_Name"]))
        agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
        dur[k] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = collections.defaultdict(list)
    for (d, name), v in sorted(agg.items()):
        out[name].append((dict(v), dur[(d, name)]))
    return out


def counters(dirs):
    for dirname in dirs:
        print(f"# {dirname}")
        for name, lst in _per_dispatch(dirname).items():
            keys = sorted(lst[0][0])
            avg = {k: sum(x[0][k] for x in lst) / len(lst) for k in keys}
            print(f"{name}  dispatches={len(lst)}  avg_ms={sum(x[1] for x in lst) / len(lst) / 1e6:.3f}")
            for k in keys:
                print(f"    {k:28s} {avg[k]:.6e}")


def traffic(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, cal_bytes):
    cal_bytes = float(cal_bytes)

    def cal(dirname, counter):
        vals = [x[0][counter] for name, lst in _per_dispatch(dirname).items() if "add" in name for x in lst]
        if not vals:
            raise SystemExit(f"no calibration dispatch in {dirname}")
        return cal_bytes / (1024.0 * sum(vals) / len(vals))

    ff = cal(cal_fetch_dir, "FETCH_SIZE")
    fw = cal(cal_write_dir, "WRITE_SIZE")
    print(f"source_hash {source_hash()}")
    print(f"calibration fetch_factor {ff:.4f} write_factor {fw:.4f} (bytes per counted byte, "
          f"elementwise kernel reading and writing {cal_bytes:.0f} B)")
    fetch = _per_dispatch(fetch_dir)
    write = _per_dispatch(write_dir)
    print(f"{'#':8s}{'kernel':50s} {'disp':>4s} {'fetch B':>12s} {'write B':>12s} {'total B':>12s}")
    for name in fetch:
        if name not in write:
            continue
        fb = ff * 1024.0 * sum(x[0]["FETCH_SIZE"] for x in fetch[name]) / len(fetch[name])
        wb = fw * 1024.0 * sum(x[0]["WRITE_SIZE"] for x in write[name]) / len(write[name])
        print(f"traffic {name.replace(' ', ''):50s} {len(fetch[name]):4d} {fb:12.4e} {wb:12.4e} {fb + wb:12.4e}")


def main(argv):
    if not argv:
        raise SystemExit(__doc__)
    cmd, args = argv[0], argv[1:]
    if cmd == "trace":
        trace(args[0])
    elif cmd == "counters":
        counters(args)
    elif cmd == "traffic":
        traffic(*args)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
