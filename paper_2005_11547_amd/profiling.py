"""Turn rocprofv3 result databases into the short text summaries kept under
profiles/, and read them back.

    python -m paper_2005_11547_amd.profiling trace  <run_results.db> <out.md> "<command>"
    python -m paper_2005_11547_amd.profiling pmc    <run_results.db or -d dir> <out.md> "<command>" ["<note>"]
    python -m paper_2005_11547_amd.profiling schema <dir>
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


def code_text(text: str) -> str:
    """The code of a C++/HIP source without // comments, blank lines and
    indentation (the kernel sources hold no block comments and no string
    literal with two slashes), so that comment edits keep a profile valid."""
    lines = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].strip()
        if code:
            lines.append(code)
    return "\n".join(lines)


def source_hash() -> str:
    """Hash of the code of the sketch kernel's sources (comments excluded)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("dms::", "")


def kernel_stats(db_path: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    return [(n, int(c), float(t), float(a), float(p)) for n, c, t, a, p in rows]


def schema(db_path: str) -> str:
    """Tables and views of a result database with their columns."""
    db = sqlite3.connect(db_path)
    out = []
    for name, kind in db.execute("select name, type from sqlite_master where type in ('table', 'view') order by name"):
        try:
            cols = [r[1] for r in db.execute(f"pragma table_info('{name}')")]
        except sqlite3.Error:
            cols = []
        out.append(f"{kind} {name}: {', '.join(cols)}")
    return "\n".join(out)


def dispatch_values(db_path: str):
    """[(dispatch id, kernel short name, {counter: value})] in dispatch order."""
    db = sqlite3.connect(db_path)
    rows = {}
    q = "select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection group by dispatch_id, counter_name"
    for did, kname, cname, v in db.execute(q):
        rows.setdefault(int(did), (_short(kname), {}))[1][cname] = float(v)
    return [(d, rows[d][0], rows[d][1]) for d in sorted(rows)]


def pmc_per_dispatch(db_path: str):
    """{kernel short name: {counter: (sum over dispatches, dispatches)}}"""
    db = sqlite3.connect(db_path)
    out = {}
    q = ("select kernel_name, counter_name, sum(value), count(distinct dispatch_id) "
         "from counters_collection group by kernel_name, counter_name")
    for kname, cname, total, n in db.execute(q):
        out.setdefault(_short(kname), {})[cname] = (float(total), int(n))
    return out


OURS = ("fast_kernel", "pair_vec", "jaccard", "bbit", "unary", "calib", "hamming", "plan_", "repeated_ids",
        "sketch_plain", "lsh_plain", "index_", "order_keys")


def kernel_dispatches(db_path: str):
    """[(kernel short name, duration ns, {extra column: value})] of every
    dispatch of the library's kernels, from the first kernel table or view of
    the database that has a name and either a duration or start and end."""
    db = sqlite3.connect(db_path)
    cands = [n for (n,) in db.execute("select name from sqlite_master where type in ('table', 'view')")
             if "kernel" in n.lower() and "top" not in n.lower() and "summary" not in n.lower()]
    for name in cands:
        cols = [r[1] for r in db.execute(f"pragma table_info('{name}')")]
        ncol = next((c for c in ("kernel_name", "name") if c in cols), None)
        if ncol is None:
            continue
        if "duration" in cols:
            dur = "duration"
        elif "start" in cols and "end" in cols:
            dur = '"end" - start'
        else:
            continue
        extra = [c for c in ("grid_size", "grid_size_x", "workgroup_size", "workgroup_size_x", "lds_size",
                             "group_segment_size", "dispatch_id", "start") if c in cols]
        q = f"select {ncol}, {dur}{''.join(', ' + e for e in extra)} from '{name}'"
        try:
            rows = db.execute(q).fetchall()
        except sqlite3.Error:
            continue
        out = []
        for r in rows:
            k = _short(str(r[0]))
            if any(t in k for t in OURS):
                out.append((k, float(r[1]), dict(zip(extra, r[2:]))))
        if "start" in extra:
            out.sort(key=lambda x: x[2]["start"])
        return out
    return []


def write_trace(db_path: str, out: str, command: str, note: str = ""):
    rows = kernel_stats(db_path)
    with open(out, "w") as f:
        f.write("# rocprofv3 kernel trace summary\n\n")
        f.write(f"Command (from the repository root):\n\n    {command}\n\n")
        if note:
            f.write(note.rstrip() + "\n\n")
        # the top_kernels view reports microseconds
        f.write("| kernel | calls | total ms | average ms | % |\n|---|---|---|---|---|\n")
        for n, c, t, a, p in rows[:25]:
            f.write(f"| {_short(n)[:120]} | {c} | {t / 1e3:.3f} | {a / 1e3:.3f} | {p:.2f} |\n")
        disp = kernel_dispatches(db_path)
        if disp:
            f.write("\nDispatches of the library's kernels, in order (duration ms; launch geometry):\n\n")
            f.write("| # | kernel | ms | geometry |\n|---|---|---|---|\n")
            for i, (k, d, ex) in enumerate(disp):
                geo = ", ".join(f"{a}={b}" for a, b in ex.items() if a not in ("start", "dispatch_id"))
                f.write(f"| {i} | {k[:90]} | {d / 1e6:.4f} | {geo} |\n")
        f.write(f"\nKernel sources hash: {source_hash()}\n")


def write_pmc(db_path: str, out: str, command: str, note: str = ""):
    """Counters of every dispatch of the library's kernels (in dispatch order,
    so launches of one kernel on different workloads stay apart), then the
    sums per kernel name of everything else."""
    per = dispatch_values(db_path)
    ours = OURS
    with open(out, "w") as f:
        f.write("# rocprofv3 counters per dispatch\n\n")
        f.write(f"Command (from the repository root):\n\n    {command}\n\n")
        if note:
            f.write(note.rstrip() + "\n\n")
        names = sorted({c for _, _, cs in per for c in cs})
        f.write("| dispatch | kernel | " + " | ".join(names) + " |\n|" + "---|" * (len(names) + 2) + "\n")
        for did, k, cs in per:
            if any(t in k for t in ours):
                f.write(f"| {did} | {k} | " + " | ".join(f"{cs.get(c, 0):.6g}" for c in names) + " |\n")
        f.write(f"\nKernel sources hash: {source_hash()}\n")


def write_traffic(fetch_db: str, write_db: str, kernel: str, copy_bytes: int, out: str, command: str):
    """HBM bytes of every dispatch of the library's kernels, FETCH_SIZE and
    WRITE_SIZE (KiB) scaled by what they read for the plain copy kernel of
    copy_bytes; `traffic_bytes` is the first dispatch named `kernel`.  The two
    runs execute the same program, so their dispatches pair up in order."""
    fe = [d for d in dispatch_values(fetch_db) if any(t in d[1] for t in OURS)]
    wr = [d for d in dispatch_values(write_db) if any(t in d[1] for t in OURS)]
    cf = [cs["FETCH_SIZE"] for _, k, cs in fe if k == COPY_KERNEL]
    cw = [cs["WRITE_SIZE"] for _, k, cs in wr if k == COPY_KERNEL]
    copy_fetch_kib, copy_write_kib = sum(cf) / len(cf), sum(cw) / len(cw)
    f_scale = copy_bytes / (copy_fetch_kib * 1024.0)
    w_scale = copy_bytes / (copy_write_kib * 1024.0)
    rows = []
    for (_, k1, c1), (_, k2, c2) in zip(fe, wr):
        if k1 != k2:
            raise ValueError(f"dispatch order differs between the runs: {k1} / {k2}")
        rows.append((k1, c1["FETCH_SIZE"] * 1024.0 * f_scale, c2["WRITE_SIZE"] * 1024.0 * w_scale))
    head = next(r for r in rows if r[0] == kernel)
    with open(out, "w") as f:
        f.write("# HBM traffic per launch from FETCH_SIZE / WRITE_SIZE\n\n")
        f.write(f"Commands (from the repository root):\n\n    {command}\n\n")
        f.write("| # | kernel | fetch bytes | write bytes | traffic bytes |\n|---|---|---|---|---|\n")
        for i, (k, a, b) in enumerate(rows):
            f.write(f"| {i} | {k[:90]} | {a:.4g} | {b:.4g} | {a + b:.4g} |\n")
        f.write("\n")
        f.write(f"kernel: {kernel} (its first dispatch)\n")
        f.write(f"copy_bytes: {copy_bytes}\n")
        f.write(f"copy_fetch_kib: {copy_fetch_kib:.1f}\n")
        f.write(f"copy_write_kib: {copy_write_kib:.1f}\n")
        f.write(f"fetch_scale: {f_scale:.4f}\n")
        f.write(f"write_scale: {w_scale:.4f}\n")
        f.write(f"kernel_fetch_bytes: {head[1]:.0f}\n")
        f.write(f"kernel_write_bytes: {head[2]:.0f}\n")
        f.write(f"traffic_bytes: {head[1] + head[2]:.0f}\n")
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


def find_db(directory: str) -> str:
    """The result database rocprofv3 wrote under a -d directory."""
    for root, _, files in os.walk(directory):
        for f in files:
            if f.endswith("_results.db"):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *_results.db under {directory}")


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "schema":
        print(schema(find_db(sys.argv[2])))
    elif mode == "trace":
        write_trace(find_db(sys.argv[2]) if os.path.isdir(sys.argv[2]) else sys.argv[2], sys.argv[3], sys.argv[4],
                    sys.argv[5] if len(sys.argv) > 5 else "")
    elif mode == "pmc":
        write_pmc(find_db(sys.argv[2]) if os.path.isdir(sys.argv[2]) else sys.argv[2], sys.argv[3], sys.argv[4],
                  sys.argv[5] if len(sys.argv) > 5 else "")
    elif mode == "traffic":
        fe = find_db(sys.argv[2]) if os.path.isdir(sys.argv[2]) else sys.argv[2]
        wr = find_db(sys.argv[3]) if os.path.isdir(sys.argv[3]) else sys.argv[3]
        write_traffic(fe, wr, sys.argv[4], int(sys.argv[5]), sys.argv[6], sys.argv[7])
    else:
        raise SystemExit(__doc__)
