"""Summaries of rocprofv3 output databases for the committed profiles.

    python -m paper_1805_06019_amd.prof_summary trace <kernel_trace.db> [command]
    python -m paper_1805_06019_amd.prof_summary traffic <fetch.db> <write.db> <out.json> [command [tile_blocks [staged]]]
    python -m paper_1805_06019_amd.prof_summary counters <counters.db>... [--kernel NAME]...
    python -m paper_1805_06019_amd.prof_summary kernel_traffic <fetch.db> <write.db> NAME...

``trace`` prints a markdown table of per-kernel dispatch counts and durations.
``traffic`` reads one FETCH_SIZE run and one WRITE_SIZE run (KiB per
dispatch), scales each by what the same counter reads for a device-to-device
copy of 256 MiB in the same run (the copy moves exactly 256 MiB each way),
and writes the per-launch HBM bytes of the whole-field decode kernel,
together with a hash of the kernel source it was measured on and the decode
tile capacity and staging of the run.
``counters`` prints, for the whole-field decode kernel (or the kernels named
with --kernel, short names as ``k_interp_rgb<0>``), the mean per dispatch
of every counter in the given runs.  ``kernel_traffic`` prints the
copy-calibrated FETCH and WRITE bytes per dispatch of the named kernels.
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 << 20
DECODE_KERNEL = "k_decode_lf<4>"


def _code_only(src: str) -> str:
    """C++ source without comments and blank-line or indentation changes."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(" ".join(line.split()) for line in src.splitlines() if line.strip())


def kernel_source_hash() -> str:
    """Hash of the code of the whole-field decode kernel, comments left out:
    the device code of kernels.hip up to the random-access section, its host
    launcher, and internal.h (a change elsewhere, e.g. in the render kernels,
    or in a comment, keeps it)."""
    with open(os.path.join(HERE, "csrc", "kernels.hip")) as fh:
        src = fh.read()
    device = src[:src.index("// random access: one (view, block) at a time")]
    i = src.index("lfc_status decode_images(")
    launcher = src[i:src.index("\n}\n", i)]
    h = hashlib.sha256()
    h.update(_code_only(device).encode())
    h.update(_code_only(launcher).encode())
    with open(os.path.join(HERE, "csrc", "internal.h")) as fh:
        h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """A kernel's name with its template arguments (k_decode_lf<4>,
    k_decode_rgb<4, true>, k_interp_rgb<false>), else the first 60 characters."""
    m = re.search(r"(k_\w+)ILi(\d)E", name)
    if m:
        return f"{m.group(1)}<{m.group(2)}>"
    m = re.search(r"(k_\w+)(<[^()]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name[:60]


def trace_rows(db: str):
    con = sqlite3.connect(db)
    q = ("select name, count(*), avg(duration), min(duration), max(duration), grid_x, grid_y, grid_z, "
         "workgroup_x, lds_size, vgpr_count, sgpr_count from kernels group by name order by sum(duration) desc")
    return list(con.execute(q))


def counter_per_dispatch(db: str, counter: str):
    """{kernel short name: [value per dispatch]} for one counter."""
    return {n: d[counter] for n, d in counters_per_dispatch(db).items() if counter in d}


def counters_per_dispatch(db: str):
    """{kernel name: {counter: [value per dispatch]}} (a counter's instances summed)."""
    con = sqlite3.connect(db)
    table = [r[0] for r in con.execute("select name from sqlite_master where type in ('table','view')")
             if "counters_collection" in r[0]][0]
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    for name, disp, cname, val in con.execute(
            f"select kernel_name, dispatch_id, counter_name, value from {table}"):
        per[name][cname][disp] += val
    return {n: {c: list(v.values()) for c, v in d.items()} for n, d in per.items()}


def copy_kernel_value(per: dict) -> float:
    """The counter for the 256 MiB device-to-device copy: the largest
    dispatch of a copy kernel."""
    best = 0.0
    for name, vals in per.items():
        if "copy" in name.lower():
            best = max(best, max(vals))
    if best <= 0:
        raise SystemExit("no copy kernel in the counter run (run bench.py with --calib-copy)")
    return best


def decode_values(per: dict):
    vals = []
    for name, v in per.items():
        if short_name(name) == DECODE_KERNEL:
            vals += v
    if not vals:
        raise SystemExit(f"no {DECODE_KERNEL} dispatch in the counter run")
    return vals


def main(argv):
    if len(argv) < 3:
        raise SystemExit(__doc__)
    mode = argv[1]
    if mode == "trace":
        print("| kernel | calls | avg us | min us | max us | grid | wg | lds B | vgpr | sgpr |")
        print("|---|---|---|---|---|---|---|---|---|---|")
        for r in trace_rows(argv[2]):
            print(f"| {short_name(r[0])} | {r[1]} | {r[2] / 1e3:.2f} | {r[3] / 1e3:.2f} | {r[4] / 1e3:.2f} | "
                  f"{r[5]}x{r[6]}x{r[7]} | {r[8]} | {r[9]} | {r[10]} | {r[11]} |")
    elif mode == "traffic":
        fetch = counter_per_dispatch(argv[2], "FETCH_SIZE")
        write = counter_per_dispatch(argv[3], "WRITE_SIZE")
        f_copy, w_copy = copy_kernel_value(fetch), copy_kernel_value(write)
        f_scale, w_scale = f_copy * 1024 / COPY_BYTES, w_copy * 1024 / COPY_BYTES
        fv, wv = decode_values(fetch), decode_values(write)
        f_bytes = sum(fv) / len(fv) * 1024 / f_scale
        w_bytes = sum(wv) / len(wv) * 1024 / w_scale
        rec = dict(kernel=DECODE_KERNEL, kernel_source_hash=kernel_source_hash(),
                   bytes_per_launch=round(f_bytes + w_bytes), fetch_bytes_per_launch=round(f_bytes),
                   write_bytes_per_launch=round(w_bytes), dispatches=[len(fv), len(wv)],
                   fetch_kib_per_dispatch=round(sum(fv) / len(fv), 1), write_kib_per_dispatch=round(sum(wv) / len(wv), 1),
                   copy_fetch_kib=round(f_copy, 1), copy_write_kib=round(w_copy, 1),
                   copy_fetch_factor=round(f_scale, 4), copy_write_factor=round(w_scale, 4),
                   command=argv[5] if len(argv) > 5 else "",
                   tile_blocks=int(argv[6]) if len(argv) > 6 else None,
                   staged=len(argv) > 7 and argv[7] in ("1", "staged", "true"))
        with open(argv[4], "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        print(json.dumps(rec, indent=1))
    elif mode == "counters":
        dbs, kernels, rest = [], [], argv[2:]
        while rest:
            if rest[0] == "--kernel":
                kernels.append(rest[1])
                rest = rest[2:]
            else:
                dbs.append(rest[0])
                rest = rest[1:]
        kernels = kernels or [DECODE_KERNEL]
        print("| kernel | counter | dispatches | mean per dispatch |")
        print("|---|---|---|---|")
        for k in kernels:
            for db in dbs:
                for name, d in counters_per_dispatch(db).items():
                    if short_name(name) != k:
                        continue
                    for c in sorted(d):
                        print(f"| {k} | {c} | {len(d[c])} | {sum(d[c]) / len(d[c]):,.0f} |")
    elif mode == "kernel_traffic":
        fetch = counter_per_dispatch(argv[2], "FETCH_SIZE")
        write = counter_per_dispatch(argv[3], "WRITE_SIZE")
        f_scale = copy_kernel_value(fetch) * 1024 / COPY_BYTES
        w_scale = copy_kernel_value(write) * 1024 / COPY_BYTES
        print(f"copy calibration: FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x {w_scale:.4f} of the bytes moved")
        print()
        print("| kernel | dispatches | HBM read MB | HBM write MB |")
        print("|---|---|---|---|")
        by_short = lambda per: {short_name(n): v for n, v in per.items()}
        fetch_s, write_s = by_short(fetch), by_short(write)
        for k in argv[4:]:
            fv, wv = fetch_s.get(k, []), write_s.get(k, [])
            if not fv or not wv:
                print(f"| {k} | 0 | - | - |")
                continue
            print(f"| {k} | {len(fv)} | {sum(fv) / len(fv) * 1024 / f_scale / 1e6:.1f} | "
                  f"{sum(wv) / len(wv) * 1024 / w_scale / 1e6:.1f} |")
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
