"""Writes profiles/traffic.json: HBM bytes per launch of the forward and gather kernels on
the 256^3 circular cone, from two rocprofv3 counter runs of the benchmark.

    cd /tmp && export TMPDIR=/tmp
    B="python3 <repo>/bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-learned --no-batched --no-2d \
       --no-tune --launch PC,XR --copy-reference"   # PC,XR: the shape bench.py's autotuner picks
    rocprofv3 --pmc FETCH_SIZE -d <out>/fetch -o run -- $B
    rocprofv3 --pmc WRITE_SIZE -d <out>/write -o run -- $B
    python -m paper_2006_00686_amd.traffic <out>/fetch/run_results.db <out>/write/run_results.db

FETCH_SIZE and WRITE_SIZE are KiB per dispatch as the counters report them.  Each is
scaled by the factor that maps the same counter's reading for a plain device-to-device
copy of known size (the benchmark's --copy-reference, in the same run) onto the bytes
that copy moves.  The file records the source hash of the kernels it was measured on;
bench.py reports the traffic only while that hash matches the sources.
"""
from __future__ import annotations

import json
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "profiles", "traffic.json")
COPY_BYTES = 256 << 20          # bench.py --copy-reference
# the 3D forward (the workload's) and the cone gather; 2D forwards, if a run has any, and
# the attenuated and batched forwards are other kernels
KERNELS = {"k_forward": r"::k_forward<3, ", "k_cone_gather": r"::k_cone_gather<"}
COPY = r"copyBuffer"


def _averages(db: str, counter: str) -> dict:
    """Mean per-dispatch value of `counter` for the tracked kernels; for the copy, the
    largest copy dispatch of the run (the 256 MiB reference; the runtime's other copies
    move a few KiB)."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, avg(value), max(value) from counters_collection "
                       "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    out = {}
    for name, mean, peak in rows:
        for key, pat in KERNELS.items():
            if re.search(pat, name):
                out[key] = float(mean)
        if re.search(COPY, name):
            out["copy"] = max(out.get("copy", 0.0), float(peak))
    return out


def build(fetch_db: str, write_db: str) -> dict:
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash
    fetch, write = _averages(fetch_db, "FETCH_SIZE"), _averages(write_db, "WRITE_SIZE")
    if "copy" not in fetch or "copy" not in write:
        raise SystemExit("no copy-reference dispatch in the counter runs (bench.py --copy-reference)")
    # the reference writes exactly its 256 MiB: another large copy in the run would be
    # taken for it and scale every figure wrongly
    if abs(write["copy"] * 1024.0 - COPY_BYTES) > 0.01 * COPY_BYTES:
        raise SystemExit(f"largest copy wrote {write['copy']:.0f} KiB, not the 256 MiB reference")
    fs = COPY_BYTES / 1024.0 / fetch["copy"]
    ws = COPY_BYTES / 1024.0 / write["copy"]
    kernels = {}
    for k in KERNELS:
        if k in fetch and k in write:
            fb, wb = fetch[k] * 1024.0 * fs, write[k] * 1024.0 * ws
            kernels[k] = {"bytes_per_launch": int(round(fb + wb)), "fetch_bytes": int(round(fb)),
                          "write_bytes": int(round(wb)), "fetch_kib_raw": round(fetch[k], 1),
                          "write_kib_raw": round(write[k], 1)}
    return {"source_hash": kernel_source_hash(),
            "workload": "cone_256^3_360x384x512 (forward + voxel-driven adjoint)",
            "method": "rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, KiB per dispatch, each scaled by "
                      "the same counter's reading for a 256 MiB device-to-device copy in the same run "
                      "(bench.py --copy-reference)",
            "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
            "copy_reference": {"bytes": COPY_BYTES, "fetch_kib": round(fetch["copy"], 1),
                               "write_kib": round(write["copy"], 1)},
            "kernels": kernels}


if __name__ == "__main__":
    if len(sys.argv) != 3:
        raise SystemExit(__doc__)
    t = build(sys.argv[1], sys.argv[2])
    with open(OUT, "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps(t, indent=1))
