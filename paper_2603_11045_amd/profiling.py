"""Summaries of rocprofv3 results for the step kernels (measurement tooling).

rocprofv3 writes a SQLite database per run (``<name>_results.db``). This
module turns one into the short text summaries kept with the benchmark:

``python -m paper_2603_11045_amd.profiling kernels DB [--kernel K --last N]``
    per-kernel dispatch statistics (the ``--stats`` table), and for kernel K
    the average duration over its last N dispatches (the timed region).

``python -m paper_2603_11045_amd.profiling markers DB``
    the library's roctx ranges (forward, adjoint, checkpoint segments,
    serving ticks) of a ``--marker-trace`` run: count and host-side duration
    per range name.

``python -m paper_2603_11045_amd.profiling traffic --fetch DB1 --write DB2 --kernel K --last N --out F``
    HBM bytes per dispatch of kernel K from a ``--pmc FETCH_SIZE`` run and a
    ``--pmc WRITE_SIZE`` run, each scaled by what the same counter reads for
    the calibration copy kernel (``nh::copy_kernel<float>``, 2^28 elements:
    1 GiB read and 1 GiB written per dispatch). Writes a JSON record with the
    hash of the kernel sources it was measured on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys
from typing import Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
# every source under csrc/ (one translation unit includes all the headers)
KERNEL_SOURCES = sorted("csrc/" + f for f in os.listdir(os.path.join(HERE, "csrc"))
                        if f.endswith((".hip", ".hpp", ".h")))
CALIB_KERNEL = "nh::copy_kernel<float>"
CALIB_BYTES = 4 << 28          # bytes read (and, separately, written) per calibration dispatch


def kernel_source_hash() -> str:
    """SHA-256 over the HIP sources that define and launch the kernels."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def _short(name: str) -> str:
    # display names carry the return type and the argument list; keep the
    # template-qualified name
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def dispatches(db: str) -> List[tuple]:
    """(short kernel name, start ns, end ns) of every dispatch, in order."""
    con = sqlite3.connect(db)
    rows = con.execute("SELECT name, start, end FROM kernels ORDER BY start").fetchall()
    con.close()
    return [(_short(n), int(s), int(e)) for n, s, e in rows]


def kernel_table(db: str) -> str:
    rows = dispatches(db)
    agg: Dict[str, list] = {}
    for n, s, e in rows:
        agg.setdefault(n, []).append((e - s) / 1e3)
    total = sum(sum(v) for v in agg.values()) or 1.0
    out = ["| kernel | calls | total us | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for n, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{n}` | {len(v)} | {sum(v):.0f} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} | "
                   f"{100 * sum(v) / total:.2f} |")
    return "\n".join(out)


def marker_table(db: str) -> str:
    """Count, total and mean duration (ms) of the roctx ranges, by range message."""
    con = sqlite3.connect(db)
    rows = con.execute("SELECT extdata, start, end FROM regions WHERE category LIKE 'MARKER%'").fetchall()
    con.close()
    agg: Dict[str, list] = {}
    for ext, s, e in rows:
        try:
            name = json.loads(ext).get("message", "?") if ext else "?"
        except ValueError:
            name = "?"
        agg.setdefault(name, []).append((int(e) - int(s)) / 1e6)
    out = ["| range | count | total ms | mean ms | min ms | max ms |", "|---|---|---|---|---|---|"]
    for n, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{n}` | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} |")
    return "\n".join(out)


def last_average_us(db: str, kernel: str, last: int) -> dict:
    d = [(e - s) / 1e3 for n, s, e in dispatches(db) if n == kernel]
    if not d:
        raise SystemExit(f"no dispatches of {kernel} in {db}")
    sel = d[-last:] if last > 0 else d
    return {"kernel": kernel, "dispatches": len(sel), "avg_us": sum(sel) / len(sel), "total_us": sum(sel)}


def counter_per_dispatch(db: str, counter: str) -> Dict[str, List[float]]:
    """Counter value (summed over its instances) of every dispatch, by kernel, in dispatch order."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "SELECT kernel_name, dispatch_id, SUM(value) FROM counters_collection WHERE counter_name = ? "
        "GROUP BY dispatch_id ORDER BY dispatch_id", (counter,)).fetchall()
    con.close()
    out: Dict[str, List[float]] = {}
    for name, _, v in rows:
        out.setdefault(_short(name), []).append(float(v))
    return out


def traffic(fetch_db: str, write_db: str, kernel: str, last: int) -> dict:
    f = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    w = counter_per_dispatch(write_db, "WRITE_SIZE")
    for name, m in ((CALIB_KERNEL, f), (CALIB_KERNEL, w), (kernel, f), (kernel, w)):
        if name not in m:
            raise SystemExit(f"{name} has no counter rows (kernels seen: {sorted(m)})")
    # counters are in KiB; the calibration copy moves CALIB_BYTES each way
    f_cal = sum(f[CALIB_KERNEL]) / len(f[CALIB_KERNEL]) * 1024.0
    w_cal = sum(w[CALIB_KERNEL]) / len(w[CALIB_KERNEL]) * 1024.0
    kf = f[kernel][-last:] if last > 0 else f[kernel]
    kw = w[kernel][-last:] if last > 0 else w[kernel]
    fetch = sum(kf) / len(kf) * 1024.0 * (CALIB_BYTES / f_cal)
    write = sum(kw) / len(kw) * 1024.0 * (CALIB_BYTES / w_cal)
    return {
        "kernel": kernel,
        "dispatches": [len(kf), len(kw)],
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "traffic_bytes_per_launch": fetch + write,
        "calibration": {"kernel": CALIB_KERNEL, "bytes_each_way": CALIB_BYTES,
                        "fetch_factor": CALIB_BYTES / f_cal, "write_factor": CALIB_BYTES / w_cal},
        "source_sha256": kernel_source_hash(),
    }


def load_traffic(path: str, kernel: str) -> Optional[dict]:
    """The stored traffic record if it was measured on this kernel and these
    sources, else None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel") != kernel or rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--kernel", default=None)
    k.add_argument("--last", type=int, default=0)
    m = sub.add_parser("markers")
    m.add_argument("db")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--last", type=int, default=0)
    t.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        print(kernel_table(a.db))
        if a.kernel:
            print()
            print(json.dumps(last_average_us(a.db, a.kernel, a.last)))
    elif a.cmd == "markers":
        print(marker_table(a.db))
    else:
        rec = traffic(a.fetch, a.write, a.kernel, a.last)
        txt = json.dumps(rec, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(txt + "\n")
        print(txt)


if __name__ == "__main__":
    sys.exit(main())
