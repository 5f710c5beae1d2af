"""HBM traffic of a tile-kernel launch from rocprofv3 counter runs.

The TCC counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what
the same counters read for a plain device-to-device copy of known size, so the
reported bytes are in the units of the bytes a copy really moves.

  # calibration copy of MIB mebibytes (reads MIB, writes MIB)
  python -m paper_2204_01133_amd.traffic copy --mib 512

  # combine counter runs (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE --output-format csv)
  python -m paper_2204_01133_amd.traffic summarize --mib 512 \\
      --kernel-fetch K_F.csv --kernel-write K_W.csv --copy-fetch C_F.csv --copy-write C_W.csv \\
      --kernel-name at_tile_kernel --out profiles/c3_fp32c_traffic.json --hash HASH
"""
from __future__ import annotations

import argparse
import csv
import json
import statistics
import sys


def _rows(path, counter):
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                yield r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])


def kernel_kib(path, counter, name):
    """Median per-dispatch value (KiB) of `counter` over the dispatches of kernel `name`."""
    vals = [v for k, _, v in _rows(path, counter) if name in k]
    if not vals:
        raise SystemExit(f"no dispatch of {name} with {counter} in {path}")
    return statistics.median(vals), len(vals)


def copy_kib(path, counter, name="copyBuffer"):
    """Median value over the copy kernel's dispatches of the calibration run (the
    run's fill kernel, which initialises the source, is not one of them)."""
    vals = [v for k, _, v in _rows(path, counter) if name in k]
    if not vals:
        raise SystemExit(f"no {name} dispatch with {counter} in {path}")
    return statistics.median(vals), len(vals)


def do_copy(mib: int, reps: int = 3):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "reps": reps}))


def summarize(a):
    kf, nkf = kernel_kib(a.kernel_fetch, "FETCH_SIZE", a.kernel_name)
    kw, nkw = kernel_kib(a.kernel_write, "WRITE_SIZE", a.kernel_name)
    cf, ncf = copy_kib(a.copy_fetch, "FETCH_SIZE")
    cw, ncw = copy_kib(a.copy_write, "WRITE_SIZE")
    nbytes = a.mib * (1 << 20)
    f_fetch = nbytes / (cf * 1024.0)
    f_write = nbytes / (cw * 1024.0)
    fetch = kf * 1024.0 * f_fetch
    write = kw * 1024.0 * f_write
    out = {
        "kernel": a.kernel_name,
        "kernel_hash": a.hash,
        "bytes_per_launch": fetch + write,
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "raw_fetch_kib": kf, "raw_write_kib": kw, "dispatches": [nkf, nkw],
        "copy_mib": a.mib, "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_dispatches": [ncf, ncw],
        "scale_fetch": f_fetch, "scale_write": f_write,
    }
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    s = sub.add_parser("summarize")
    s.add_argument("--mib", type=int, required=True)
    for k in ("kernel-fetch", "kernel-write", "copy-fetch", "copy-write"):
        s.add_argument("--" + k, required=True)
    s.add_argument("--kernel-name", default="at_tile_kernel")
    s.add_argument("--hash", required=True)
    s.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        do_copy(a.mib)
    else:
        summarize(a)


if __name__ == "__main__":
    sys.exit(main())
