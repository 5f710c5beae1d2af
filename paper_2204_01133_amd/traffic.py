"""Memory traffic of a tile-kernel launch from rocprofv3 counter runs.

The bytes are counted where the L2 (TCC) talks to the memory fabric (EA), from the
numbers of requests of each size:

  read  = 32 TCC_EA0_RDREQ_32B + 64 TCC_EA0_RDREQ_64B + 128 TCC_EA0_RDREQ_128B
  write = 64 TCC_EA0_WRREQ_64B + 32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B)

and, beside them, the part the L2 sends towards DRAM (TCC_EA0_RDREQ_DRAM_32B and
TCC_EA0_WRREQ_WRITE_DRAM_32B, in 32-byte units).  Requests towards DRAM are served
by the 256 MB last-level cache (MALL) when it holds the line, so the DRAM-side
counts bound HBM traffic from above.  A device copy of known size checks the counts
and gives the achievable copy bandwidth.

  # copy of MIB mebibytes (reads MIB, writes MIB), timed with HIP events
  python -m paper_2204_01133_amd.traffic copy --mib 512

  # combine counter runs (rocprofv3 --pmc ... --output-format csv)
  python -m paper_2204_01133_amd.traffic summarize --kernel K1.csv K2.csv --copy C1.csv C2.csv \\
      --kernel-name at_tile_kernel --mib 512 --hash HASH --out profiles/c3_fp32c_traffic.json
"""
from __future__ import annotations

import argparse
import csv
import json
import statistics
import sys

READ = {"TCC_EA0_RDREQ_32B_sum": 32, "TCC_EA0_RDREQ_64B_sum": 64, "TCC_EA0_RDREQ_128B_sum": 128}
DRAM = {"TCC_EA0_RDREQ_DRAM_32B_sum": ("read", 32), "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum": ("write", 32)}


def medians(paths, name):
    """Per-dispatch median of every counter over the dispatches of kernels whose name
    contains `name` (values of one dispatch summed over its rows)."""
    per = {}
    for path in paths:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if name not in r["Kernel_Name"]:
                    continue
                key = (path, r["Dispatch_Id"])
                per.setdefault(r["Counter_Name"], {}).setdefault(key, 0.0)
                per[r["Counter_Name"]][key] += float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no dispatch of {name} in {paths}")
    return {c: (statistics.median(v.values()), len(v)) for c, v in per.items()}


def bytes_of(m):
    rd = sum(w * m[c][0] for c, w in READ.items())
    wr_all, wr64 = m["TCC_EA0_WRREQ_sum"][0], m["TCC_EA0_WRREQ_64B_sum"][0]
    wr = 64 * wr64 + 32 * (wr_all - wr64)
    out = {"read": rd, "write": wr, "total": rd + wr}
    for c, (k, w) in DRAM.items():
        if c in m:
            out["dram_" + k] = w * m[c][0]
    if "dram_read" in out and "dram_write" in out:
        out["dram_total"] = out["dram_read"] + out["dram_write"]
    return out


def do_copy(mib: int, reps: int = 5):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1000.0 / reps
    gbs = 2 * mib * (1 << 20) / s / 1e9
    print(json.dumps({"copy_mib": mib, "reps": reps, "us_per_copy": s * 1e6, "read_plus_write_gbs": gbs}))


def summarize(a):
    k = medians(a.kernel, a.kernel_name)
    c = medians(a.copy, a.copy_name)
    kb, cb = bytes_of(k), bytes_of(c)
    nbytes = a.mib * (1 << 20)
    out = {
        "kernel": a.kernel_name,
        "kernel_hash": a.hash,
        "bytes_per_launch": kb["total"],
        "read_bytes_per_launch": kb["read"],
        "write_bytes_per_launch": kb["write"],
        "dram_side_bytes_per_launch": kb.get("dram_total"),
        "dram_side_read": kb.get("dram_read"), "dram_side_write": kb.get("dram_write"),
        "dispatches": {cn: v[1] for cn, v in k.items()},
        "counters_median": {cn: v[0] for cn, v in k.items()},
        "copy_check": {"mib": a.mib, "read_vs_known": cb["read"] / nbytes, "write_vs_known": cb["write"] / nbytes,
                       "dram_read_vs_known": cb.get("dram_read", 0.0) / nbytes,
                       "dram_write_vs_known": cb.get("dram_write", 0.0) / nbytes},
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
    s.add_argument("--kernel", nargs="+", required=True)
    s.add_argument("--copy", nargs="+", required=True)
    s.add_argument("--kernel-name", default="at_tile_kernel")
    s.add_argument("--copy-name", default="copyBuffer")
    s.add_argument("--hash", required=True)
    s.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        do_copy(a.mib)
    else:
        summarize(a)


if __name__ == "__main__":
    sys.exit(main())
