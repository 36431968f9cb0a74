"""Summaries of rocprofv3 runs of bench.py, for bench.py's measured fields.

The benchmark reports, beside each kernel's launch time, figures that only
hardware counters give: the bytes a kernel moved across the L2 / fabric
boundary (HBM traffic), its float-atomic requests, and the MFMA activity of
the bfloat16 deferred MLP.  This script turns the CSV files that rocprofv3
writes into

* ``profiles/traffic.json``: per (kernel, workload) the per-launch figures
  with the hash of the kernel family's source files at the time the
  counters were taken -- bench.py uses a figure only while that hash still
  matches the current source;
* a short markdown table of the same figures (printed; the committed
  summaries under ``profiles/`` are made from it).

Subcommands (``DIR`` = a rocprofv3 ``-d`` output directory, searched
recursively for ``*_counter_collection.csv`` / ``*_kernel_stats.csv``):

    python bench_counters.py traffic --fetch DIR --write DIR --workload W [--slice A:B] KEY=PATTERN ...
    python bench_counters.py counters --dir DIR --workload W KEY=PATTERN ...
    python bench_counters.py stats --dir DIR

``KEY=PATTERN``: KEY is the kernel key bench.py looks up (e.g.
``k_march_fwd_lane<GatherBF16>``), PATTERN a substring of the demangled
kernel name (e.g. ``k_march_fwd_lane<omerf::GatherBF16, false, false, false>``).

HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) each scaled by what
the same counter reads for a device-to-device copy of 1 GiB in the same
process (``bench.py --calib-copy`` issues it first): the copy reads and
writes 2^30 bytes, so scale = 2^30 / (counter KiB x 1024).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
COPY_KERNEL = "copyBuffer"  # the HIP runtime's device-to-device copy kernel
COPY_BYTES = 1 << 30


def _csvs(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def counter_values(d: str):
    """{kernel name: {counter: [value per dispatch, in dispatch order]}}."""
    out: dict = {}
    rows = _csvs(d, "_counter_collection.csv")
    rows.sort(key=lambda r: int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)) or 0))
    for r in rows:
        name = r.get("Kernel_Name", "")
        out.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def _match(values: dict, pattern: str):
    hits = [k for k in values if pattern in k]
    if not hits:
        raise SystemExit(f"no kernel matches {pattern!r}")
    if len(hits) > 1:
        raise SystemExit(f"{pattern!r} matches several kernels: {hits}")
    return hits[0], values[hits[0]]


def _median(v):
    return float(statistics.median(v))


def source_hash(family: str) -> str:
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash

    return kernel_source_hash(family)


def family_of(key: str) -> str:
    if key.startswith("k_march_bwd"):
        return "bwd"
    if key.startswith("k_mlp"):
        return "mlp"
    return "fwd"


def _load():
    if os.path.exists(TRAFFIC):
        with open(TRAFFIC) as fh:
            return json.load(fh)
    return {}


def _save(rec):
    with open(TRAFFIC, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
        fh.write("\n")


def cmd_traffic(a):
    fetch = counter_values(a.fetch)
    write = counter_values(a.write)
    cf = _match(fetch, COPY_KERNEL)[1]["FETCH_SIZE"]
    cw = _match(write, COPY_KERNEL)[1]["WRITE_SIZE"]
    fs = COPY_BYTES / (cf[0] * 1024.0)
    ws = COPY_BYTES / (cw[0] * 1024.0)
    rec = _load()
    print(f"calibration: 1 GiB copy FETCH_SIZE {cf[0]:.1f} KiB (x {fs:.4f}), WRITE_SIZE {cw[0]:.1f} KiB (x {ws:.4f})")
    print("| kernel | workload | dispatches | FETCH_SIZE KiB (median) | WRITE_SIZE KiB (median) | HBM bytes per launch |")
    print("|---|---|---|---|---|---|")
    sl = slice(*[int(x) if x else None for x in a.slice.split(":")]) if a.slice else slice(None)
    for spec in a.kernels:
        key, pat = spec.split("=", 1)
        name, fv = _match(fetch, pat)
        _, wv = _match(write, pat)
        fv = {"FETCH_SIZE": fv["FETCH_SIZE"][sl]}
        wv = {"WRITE_SIZE": wv["WRITE_SIZE"][sl]}
        f, w = _median(fv["FETCH_SIZE"]), _median(wv["WRITE_SIZE"])
        hbm = int(round(f * 1024.0 * fs + w * 1024.0 * ws))
        fam = family_of(key)
        e = rec.setdefault(key, {}).setdefault(a.workload, {})
        e.update({"family": fam, "source_hash": source_hash(fam), "kernel_name": name.split("(")[0],
                  "fetch_size_kib_raw": round(f, 1), "write_size_kib_raw": round(w, 1),
                  "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                  "calibration": f"1 GiB device-to-device copy in the same process: FETCH_SIZE {cf[0]:.2f} KiB, "
                                 f"WRITE_SIZE {cw[0]:.2f} KiB",
                  "hbm_bytes_per_launch": hbm, "dispatches": len(fv["FETCH_SIZE"])})
        print(f"| {name.split('(')[0]} | {a.workload} | {len(fv['FETCH_SIZE'])} | {f:,.1f} | {w:,.1f} | {hbm:,} |")
    _save(rec)


def cmd_counters(a):
    vals = counter_values(a.dir)
    rec = _load()
    for spec in a.kernels:
        key, pat = spec.split("=", 1)
        name, cv = _match(vals, pat)
        fam = family_of(key)
        e = rec.setdefault(key, {}).setdefault(a.workload, {})
        med = {c: _median(v) for c, v in cv.items()}
        e.setdefault("counters", {}).update({c: round(v, 1) for c, v in med.items()})
        e.update({"family": fam, "kernel_name": name.split("(")[0]})
        e["counter_source_hash"] = source_hash(fam)
        print(f"{name.split('(')[0]} [{a.workload}], median of {len(next(iter(cv.values())))} dispatches:")
        for c, v in sorted(med.items()):
            print(f"  {c:40s} {v:,.1f}")
        if "MfmaUtil" in med:  # rocprofv3's derived metric, in percent
            e["mfma_busy_frac"] = round(med["MfmaUtil"] / 100.0, 5)
            e["source_hash"] = source_hash(fam)
            print(f"  mfma_busy_frac = MfmaUtil / 100 = {e['mfma_busy_frac']}")
    _save(rec)


def cmd_stats(a):
    rows = _csvs(a.dir, "_kernel_stats.csv")
    print("| kernel | calls | average ms | min ms | max ms | share |")
    print("|---|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        if float(r["Percentage"]) < a.min_pct:
            continue
        print(f"| {r['Name'].split('(')[0]} | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
              f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | {float(r['Percentage']):.1f} % |")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--slice", default="", help="START:STOP of each kernel's dispatches (in dispatch order), "
                                               "when one run holds several workloads of one kernel")
    t.add_argument("kernels", nargs="+")
    c = sub.add_parser("counters")
    c.add_argument("--dir", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("kernels", nargs="+")
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--min-pct", type=float, default=0.0)
    a = ap.parse_args()
    {"traffic": cmd_traffic, "counters": cmd_counters, "stats": cmd_stats}[a.cmd](a)


if __name__ == "__main__":
    main()
