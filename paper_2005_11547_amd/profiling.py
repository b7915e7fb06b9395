"""Turn rocprofv3 result databases into the short text summaries kept under
profiles/, and read them back.

    python -m paper_2005_11547_amd.profiling trace  <run_results.db> <out.md> "<command>"
    python -m paper_2005_11547_amd.profiling pmc    <run_results.db> <out.md> "<command>"
    python -m paper_2005_11547_amd.profiling traffic <fetch.db> <write.db> <kernel> <out.txt> "<commands>"

The traffic summary scales the FETCH_SIZE / WRITE_SIZE counters (KiB per
dispatch) by what the same counters read for the calibration copy kernel,
whose bytes are known, and records a hash of the kernel sources it was taken
with; a reader treats it as stale once those sources change.
"""
from __future__ import annotations

import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/dms_sketch.hip", "csrc/dms_device.h", "csrc/dms_internal.h"]
COPY_KERNEL = "calib_copy_kernel"


def source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("dms::", "")


def kernel_stats(db_path: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    return [(n, int(c), float(t), float(a), float(p)) for n, c, t, a, p in rows]


def pmc_per_dispatch(db_path: str):
    """{kernel short name: {counter: (sum over dispatches, dispatches)}}"""
    db = sqlite3.connect(db_path)
    out = {}
    q = ("select kernel_name, counter_name, sum(value), count(distinct dispatch_id) "
         "from counters_collection group by kernel_name, counter_name")
    for kname, cname, total, n in db.execute(q):
        out.setdefault(_short(kname), {})[cname] = (float(total), int(n))
    return out


def write_trace(db_path: str, out: str, command: str):
    rows = kernel_stats(db_path)
    with open(out, "w") as f:
        f.write("# rocprofv3 kernel trace summary\n\n")
        f.write(f"Command (from the repository root):\n\n    {command}\n\n")
        # the top_kernels view reports microseconds
        f.write("| kernel | calls | total ms | average ms | % |\n|---|---|---|---|---|\n")
        for n, c, t, a, p in rows:
            f.write(f"| {_short(n)} | {c} | {t / 1e3:.3f} | {a / 1e3:.3f} | {p:.2f} |\n")
        f.write(f"\nKernel sources hash: {source_hash()}\n")


def write_pmc(db_path: str, out: str, command: str):
    data = pmc_per_dispatch(db_path)
    with open(out, "w") as f:
        f.write("# rocprofv3 counters (sum over the dispatches of each kernel)\n\n")
        f.write(f"Command (from the repository root):\n\n    {command}\n\n")
        for k, cs in sorted(data.items()):
            f.write(f"## {k}\n\n| counter | sum | dispatches | per dispatch |\n|---|---|---|---|\n")
            for c, (tot, n) in sorted(cs.items()):
                f.write(f"| {c} | {tot:.6g} | {n} | {tot / max(n, 1):.6g} |\n")
            f.write("\n")
        f.write(f"Kernel sources hash: {source_hash()}\n")


def write_traffic(fetch_db: str, write_db: str, kernel: str, copy_bytes: int, out: str, command: str):
    """HBM bytes per launch of `kernel`, scaled by the copy kernel's counters."""
    fe = pmc_per_dispatch(fetch_db)
    wr = pmc_per_dispatch(write_db)

    def per(d, k, c):
        tot, n = d[k][c]
        return tot / max(n, 1)

    copy_fetch_kib = per(fe, COPY_KERNEL, "FETCH_SIZE")
    copy_write_kib = per(wr, COPY_KERNEL, "WRITE_SIZE")
    f_scale = copy_bytes / (copy_fetch_kib * 1024.0)
    w_scale = copy_bytes / (copy_write_kib * 1024.0)
    k_fetch = per(fe, kernel, "FETCH_SIZE") * 1024.0 * f_scale
    k_write = per(wr, kernel, "WRITE_SIZE") * 1024.0 * w_scale
    with open(out, "w") as f:
        f.write("# HBM traffic per launch from FETCH_SIZE / WRITE_SIZE\n\n")
        f.write(f"Commands (from the repository root):\n\n    {command}\n\n")
        f.write(f"kernel: {kernel}\n")
        f.write(f"copy_bytes: {copy_bytes}\n")
        f.write(f"copy_fetch_kib: {copy_fetch_kib:.1f}\n")
        f.write(f"copy_write_kib: {copy_write_kib:.1f}\n")
        f.write(f"fetch_scale: {f_scale:.4f}\n")
        f.write(f"write_scale: {w_scale:.4f}\n")
        f.write(f"kernel_fetch_bytes: {k_fetch:.0f}\n")
        f.write(f"kernel_write_bytes: {k_write:.0f}\n")
        f.write(f"traffic_bytes: {k_fetch + k_write:.0f}\n")
        f.write(f"source_hash: {source_hash()}\n")


def read_traffic(path: str):
    """Bytes per launch from a traffic summary, or None if missing or stale."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#") and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["traffic_bytes"])
    except (KeyError, ValueError):
        return None


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        write_trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif mode == "pmc":
        write_pmc(sys.argv[2], sys.argv[3], sys.argv[4])
    elif mode == "traffic":
        write_traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6], sys.argv[7])
    else:
        raise SystemExit(__doc__)
