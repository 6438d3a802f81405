"""HBM traffic of a kernel from rocprofv3 counter runs.

rocprofv3 reports FETCH_SIZE and WRITE_SIZE in KiB per dispatch.  Their scale
against bytes actually moved is fixed by a plain device copy of known size
(``python bench.py --copy-calibration`` copies 1 GiB three times): the
calibrated HBM bytes of a kernel are its FETCH_SIZE times (1 GiB / the copy's
FETCH_SIZE) plus its WRITE_SIZE times (1 GiB / the copy's WRITE_SIZE).

    python -m paper_2102_06611_amd.counters --kernel k_sweep_msc64 \\
        --match 'k_sweep<1, 2, 1, 0, 0>' --fetch F.csv --write W.csv \\
        --copy-fetch CF.csv --copy-write CW.csv [--command '...'] [--out profiles/traffic.json]

writes (or updates) the kernel's entry in the JSON file, keyed by a hash of
the kernel sources, and prints a short markdown table.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict
from typing import Dict, List

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 30
SOURCES = ("pa_kernels.hip", "pa_device.hpp", "pa_block.hpp")


def source_hash() -> str:
    """Hash of the sources of the population kernels (the key of a measurement)."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def per_dispatch(path: str, counter: str) -> Dict[str, List[float]]:
    """Counter value of every dispatch, by kernel name (summed over its instances)."""
    acc: Dict[tuple, float] = defaultdict(float)
    names: Dict[tuple, str] = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            key = (row.get("Dispatch_Id") or row.get("Correlation_Id"), row["Kernel_Name"])
            acc[key] += float(row["Counter_Value"])
            names[key] = row["Kernel_Name"]
    out: Dict[str, List[float]] = defaultdict(list)
    for key, v in acc.items():
        out[names[key]].append(v)
    return out


def mean_for(path: str, counter: str, match: str) -> tuple:
    vals = [v for name, vs in per_dispatch(path, counter).items() if match in name for v in vs]
    if not vals:
        raise SystemExit("no dispatch of a kernel matching %r with %s in %s" % (match, counter, path))
    return sum(vals) / len(vals), len(vals)


def copy_kib(path: str, counter: str) -> float:
    """The copy kernel's counter (the largest dispatch of the calibration run)."""
    best = 0.0
    for vs in per_dispatch(path, counter).values():
        best = max(best, max(vs))
    if best <= 0:
        raise SystemExit("no copy dispatch with %s in %s" % (counter, path))
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True, help="entry name in the JSON file")
    ap.add_argument("--match", required=True, help="substring of the kernel's name in the CSVs")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args(argv)
    fetch, nf = mean_for(args.fetch, "FETCH_SIZE", args.match)
    write, nw = mean_for(args.write, "WRITE_SIZE", args.match)
    cf = copy_kib(args.copy_fetch, "FETCH_SIZE")
    cw = copy_kib(args.copy_write, "WRITE_SIZE")
    kf = COPY_BYTES / (cf * 1024.0)
    kw = COPY_BYTES / (cw * 1024.0)
    entry = {
        "source_hash": source_hash(),
        "fetch_kib_per_launch": fetch, "write_kib_per_launch": write,
        "launches": [nf, nw],
        "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_factor": kf, "write_factor": kw,
        "hbm_read_bytes_per_launch": fetch * 1024.0 * kf,
        "hbm_write_bytes_per_launch": write * 1024.0 * kw,
        "hbm_bytes_per_launch": fetch * 1024.0 * kf + write * 1024.0 * kw,
        "command": args.command,
    }
    try:
        with open(args.out) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[args.kernel] = entry
    tmp = args.out + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, args.out)
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | factors | HBM read MB | HBM write MB |")
    print("|---|---:|---:|---|---:|---:|")
    print("| `%s` | %.0f | %.0f | x%.3f / x%.3f | %.1f | %.1f |" % (
        args.match, fetch, write, kf, kw, entry["hbm_read_bytes_per_launch"] / 1e6,
        entry["hbm_write_bytes_per_launch"] / 1e6))


if __name__ == "__main__":
    main()
