"""HBM traffic of a kernel from rocprofv3 hardware counters.

Two subcommands, both run from the repository root:

  python -m paper_2312_02891_amd.pmc copy [--mib N]
      A plain device-to-device copy of N MiB (five times), the calibration
      kernel: it reads and writes exactly N MiB per dispatch.

  python -m paper_2312_02891_amd.pmc summarize --fetch F.csv --write W.csv
         --calib-fetch CF.csv --calib-write CW.csv --kernel REGEX --mib N
         [--source FILE ...] [--json OUT]
      Reads the per-dispatch counter files that `rocprofv3 --pmc FETCH_SIZE`
      and `rocprofv3 --pmc WRITE_SIZE` wrote for the workload and for the
      copy, scales each counter by (known bytes / counted bytes) of the copy,
      and prints the average HBM bytes per dispatch of the kernels whose name
      matches REGEX.  --source files are hashed into the JSON so that a
      consumer can tell whether the kernel changed since the counters were
      taken.

FETCH_SIZE and WRITE_SIZE are reported by rocprofv3 in KiB per dispatch.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys


def source_digest(paths):
    h = hashlib.sha256()
    for p in sorted(paths):
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode())
            h.update(fh.read())
    return h.hexdigest()


def _per_dispatch(path, counter, kernel_re):
    """{dispatch id: (kernel name, value)} for one counter."""
    pat = re.compile(kernel_re)
    out = {}
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            if not pat.search(name):
                continue
            key = row.get("Dispatch_Id") or row.get("Correlation_Id")
            val = float(row["Counter_Value"])
            prev = out.get(key)
            # counters of one dispatch can come split per hardware instance
            out[key] = (name, val + (prev[1] if prev else 0.0))
    return out


def _avg(d):
    if not d:
        raise SystemExit("no matching dispatches")
    return sum(v for _, v in d.values()) / len(d), len(d)


def summarize(a):
    known_kib = a.mib * 1024.0
    cf, ncf = _avg(_per_dispatch(a.calib_fetch, "FETCH_SIZE", a.calib_kernel))
    cw, ncw = _avg(_per_dispatch(a.calib_write, "WRITE_SIZE", a.calib_kernel))
    kf, nkf = _avg(_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel))
    kw, nkw = _avg(_per_dispatch(a.write, "WRITE_SIZE", a.kernel))
    sf, sw = known_kib / cf, known_kib / cw
    fetch_b = kf * sf * 1024.0
    write_b = kw * sw * 1024.0
    res = {
        "kernel_regex": a.kernel,
        "dispatches": {"fetch": nkf, "write": nkw, "calib_fetch": ncf, "calib_write": ncw},
        "calib_copy_mib": a.mib,
        "calib_counted_kib": {"fetch": round(cf, 1), "write": round(cw, 1)},
        "scale": {"fetch": round(sf, 5), "write": round(sw, 5)},
        "avg_counted_kib": {"fetch": round(kf, 1), "write": round(kw, 1)},
        "traffic_bytes_per_dispatch": round(fetch_b + write_b),
        "fetch_bytes_per_dispatch": round(fetch_b),
        "write_bytes_per_dispatch": round(write_b),
    }
    if a.source:
        res["source_sha256"] = source_digest(a.source)
        res["source_files"] = [os.path.relpath(p) for p in a.source]
    text = json.dumps(res, indent=2)
    print(text)
    if a.json:
        with open(a.json, "w") as fh:
            fh.write(text + "\n")


def copy(a):
    import torch
    n = a.mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB five times", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2312_02891_amd.pmc")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--calib-fetch", required=True)
    s.add_argument("--calib-write", required=True)
    s.add_argument("--kernel", required=True)
    # the copies only: the fill that creates the source buffer reads nothing
    s.add_argument("--calib-kernel", default="copyBuffer")
    s.add_argument("--mib", type=int, default=512)
    s.add_argument("--source", nargs="*", default=[])
    s.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy(a)
    else:
        summarize(a)


if __name__ == "__main__":
    sys.exit(main())
