"""HBM traffic of the filter kernel from rocprofv3 counters, scaled by a plain copy of known size.

Two subcommands:

``python -m paper_1206_3768_amd.traffic copy [--mib N]``
    runs a plain device-to-device copy of N MiB (default 1024) three times; profiled with
    ``rocprofv3 --pmc FETCH_SIZE`` and, in another run, ``--pmc WRITE_SIZE``, it gives the counter
    reading of a kernel whose HBM traffic is known (N MiB read, N MiB written).

``python -m paper_1206_3768_amd.traffic summarize --fetch DIR --write DIR --copy-fetch DIR
--copy-write DIR --kernel NAME --mib N --out FILE``
    reads the four ``*_counter_collection.csv`` files, averages FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) over the dispatches of the named kernel, scales each by the ratio of the copy's known
    bytes to its counter reading and writes the per-launch HBM bytes, with the source hash of the
    GEMM kernel, to FILE (JSON).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("gemm.hip", "gemm_tile.h")


def kernel_source_hash() -> str:
    """Hash of the sources of the filter GEMM kernel; a counter summary is valid for this hash only."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1206_3768_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _copy(mib: int) -> int:
    import torch
    if not torch.cuda.is_available():
        print("traffic copy needs a GPU", file=sys.stderr)
        return 1
    n = mib * (1 << 20) // 16
    src = torch.ones(n, dtype=torch.complex128, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "elements": n}), flush=True)
    return 0


def _read(d: str, counter: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") == counter:
                    out.append((row["Kernel_Name"], float(row["Counter_Value"])))
    return out


def _per_dispatch(rows, match):
    vals = [v for name, v in rows if match(name)]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def _summarize(a) -> int:
    copy_bytes = a.mib * (1 << 20)
    is_copy = lambda name: "copy" in name.lower()   # noqa: E731
    # the copy dispatch of the full size is the largest reading of its run
    cf = max(v for name, v in _read(a.copy_fetch, "FETCH_SIZE") if is_copy(name))
    cw = max(v for name, v in _read(a.copy_write, "WRITE_SIZE") if is_copy(name))
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    match = lambda name: name.replace(" ", "").startswith(a.kernel.replace(" ", "")) or \
        a.kernel.replace(" ", "") in name.replace(" ", "")   # noqa: E731
    kf, nf = _per_dispatch(_read(a.fetch, "FETCH_SIZE"), match)
    kw, nw = _per_dispatch(_read(a.write, "WRITE_SIZE"), match)
    if kf is None or kw is None:
        print(f"kernel {a.kernel} not found in the counter runs", file=sys.stderr)
        return 1
    fetch_b = kf * 1024.0 * f_scale
    write_b = kw * 1024.0 * w_scale
    res = {
        "kernel": a.kernel,
        "kernel_source_sha256_16": kernel_source_hash(),
        "dispatches": {"fetch_run": nf, "write_run": nw},
        "fetch_kib_per_dispatch_raw": kf, "write_kib_per_dispatch_raw": kw,
        "copy_calibration": {"bytes": copy_bytes, "fetch_kib_raw": cf, "write_kib_raw": cw,
                             "fetch_scale": f_scale, "write_scale": w_scale},
        "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
        "bytes_per_launch": fetch_b + write_b,
        "commands": a.commands,
    }
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    s = sub.add_parser("summarize")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernel", "out"):
        s.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    s.add_argument("--mib", type=int, default=1024)
    s.add_argument("--commands", default="")
    a = ap.parse_args()
    return _copy(a.mib) if a.cmd == "copy" else _summarize(a)


if __name__ == "__main__":
    sys.exit(main())
