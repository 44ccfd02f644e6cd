"""HBM traffic per launch of one kernel from two rocprofv3 counter passes.

    python -m paper_2511_06407_amd.pmc_traffic FETCH_CSV WRITE_CSV --kernel NAME
        --calib-bytes B --source FILE [--out JSON]

FETCH_CSV / WRITE_CSV are the run_counter_collection.csv files of a
``rocprofv3 --pmc FETCH_SIZE`` and a ``--pmc WRITE_SIZE`` pass over the same
program (values in KiB per dispatch).  The program also ran one device copy of
B bytes; the counters' readings for that copy give the factors that turn each
counter into bytes (read and write separately).  The result records the
per-launch bytes of every dispatch of the kernel, their average, and a hash
of the kernel's source file, so a consumer can tell when it is stale.
"""
import argparse
import csv
import hashlib
import json
import sys
from collections import defaultdict


def read(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def calibration(rows, calib_bytes):
    """Counter KiB of the calibration copy: the largest dispatch of the
    runtime's device-to-device copy kernel (the program's own copy kernels,
    such as the chain's accept copy, are not of known size)."""
    copies = [r for r in rows if "__amd_rocclr_copyBuffer" in r["Kernel_Name"]]
    if not copies:
        raise SystemExit("no __amd_rocclr_copyBuffer dispatch: run the program with its calibration copy")
    best = max(copies, key=lambda r: float(r["Counter_Value"]))
    kib = float(best["Counter_Value"])
    return calib_bytes / (kib * 1024.0), kib


def per_dispatch(rows, kernel):
    return {int(r["Dispatch_Id"]): (int(r["Grid_Size"]), float(r["Counter_Value"]))
            for r in rows if kernel in r["Kernel_Name"]}


def summarise(fetch_rows, write_rows, kernel, calib_bytes, source):
    ff, fkib = calibration(fetch_rows, calib_bytes)
    wf, wkib = calibration(write_rows, calib_bytes)
    fd, wd = per_dispatch(fetch_rows, kernel), per_dispatch(write_rows, kernel)
    by_grid = defaultdict(lambda: [0, 0.0, 0.0])
    total = 0.0
    n = 0
    for grid, fk in fd.values():
        by_grid[grid][0] += 1
        by_grid[grid][1] += fk * 1024.0 * ff
    for grid, wk in wd.values():
        by_grid[grid][2] += wk * 1024.0 * wf
    for grid, (cnt, fb, wb) in by_grid.items():
        total += fb + wb
        n += cnt
    with open(source, "rb") as f:
        src_hash = hashlib.sha256(f.read()).hexdigest()[:16]
    return {
        "kernel": kernel,
        "bytes_per_launch": total / max(n, 1),
        "launches": n,
        "by_grid": {str(g): {"launches": c, "fetch_bytes_per_launch": fb / c,
                             "write_bytes_per_launch": wb / c}
                    for g, (c, fb, wb) in sorted(by_grid.items())},
        "calibration": {"copy_bytes": calib_bytes, "fetch_kib": fkib, "write_kib": wkib,
                        "fetch_factor": ff, "write_factor": wf},
        "kernel_source": source,
        "kernel_source_hash": src_hash,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--calib-bytes", type=float, required=True)
    ap.add_argument("--source", required=True)
    ap.add_argument("--cmd", default="")
    ap.add_argument("--out")
    a = ap.parse_args(argv)
    d = summarise(read(a.fetch_csv), read(a.write_csv), a.kernel, a.calib_bytes, a.source)
    if a.cmd:
        d["command"] = a.cmd
    text = json.dumps(d, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    sys.stdout.write(text + "\n")


if __name__ == "__main__":
    main()
