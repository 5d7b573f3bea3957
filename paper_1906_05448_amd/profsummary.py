"""Summarise rocprofv3 results databases as text tables.

    python -m paper_1906_05448_amd.profsummary <run_results.db> [title]
    python -m paper_1906_05448_amd.profsummary --pmc <fetch_results.db> <write_results.db> [title]
    python -m paper_1906_05448_amd.profsummary --counters <results.db> [title]

The first form (kernel trace) prints one row per kernel: calls, total (ms)
and average (us) duration, share. The second (one FETCH_SIZE run, one
WRITE_SIZE run of the same program) prints per kernel and grid the median
KiB per dispatch of each counter and the bytes after scaling each counter by
what it reads for the runtime's device-to-device copy kernel in the same run
(a copy of known size: bench.py copies 2 GiB). The third prints, per kernel
and grid, the median per dispatch of every counter the run collected.
"""
import sqlite3
import sys


def summary(db: str) -> list:
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    con.close()
    return rows


def _demangle_lbm(name: str) -> str:
    """Names the profiler leaves mangled (the _Float16 kernels): namespace
    path and integer template arguments, e.g. lbm::k_stream_collide_seg<0>."""
    import re
    rest = name[len("_ZN"):]
    parts = []
    while rest and rest[0].isdigit():
        m = re.match(r"(\d+)", rest)
        n = int(m.group(1))
        ident = rest[len(m.group(1)):len(m.group(1)) + n]
        rest = rest[len(m.group(1)) + n:]
        if ident != "_GLOBAL__N_1":
            parts.append(ident)
    args = re.match(r"I((?:Li-?\d+E|Lb[01]E)+)E", rest)
    targs = ""
    if args:
        targs = "<" + ", ".join(re.findall(r"L[ib](-?\d+)E", args.group(1))) + ">"
    return "::".join(parts) + targs


def short(name: str) -> str:
    if name.startswith("_ZN"):
        return _demangle_lbm(name)
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def main(argv):
    rows = summary(argv[1])
    title = argv[2] if len(argv) > 2 else argv[1]
    print(f"# {title}\n")
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---:|---:|---:|---:|")
    for name, calls, total, avg, pct in rows:
        print(f"| `{short(name)}` | {calls} | {total / 1e3:.2f} | {avg:.1f} | {pct:.2f} |")


def _pmc(db: str, counter: str) -> dict:
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, grid_size, value from counters_collection where counter_name = ?",
                       (counter,)).fetchall()
    con.close()
    out = {}
    for name, grid, v in rows:
        out.setdefault((short(name), grid), []).append(v)
    return out


def _median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


COPY_BYTES = 2 * 1024 ** 3  # bench.py's calibration copy, read and written


def pmc_main(argv):
    fetch, write = _pmc(argv[2], "FETCH_SIZE"), _pmc(argv[3], "WRITE_SIZE")
    title = argv[4] if len(argv) > 4 else argv[2]
    copy_key = [k for k in fetch if "copyBuffer" in k[0]]
    scale_f = scale_w = 1.0
    if copy_key:
        k = max(copy_key, key=lambda t: _median(fetch[t]))
        scale_f = COPY_BYTES / (_median(fetch[k]) * 1024)
        if k in write:
            scale_w = COPY_BYTES / (_median(write[k]) * 1024)
    print(f"# {title}\n")
    print(f"Counter scale from the 2 GiB copy: FETCH_SIZE x {scale_f:.4f}, WRITE_SIZE x {scale_w:.4f}.\n")
    print("| kernel | grid | dispatches | FETCH KiB | WRITE KiB | read GB | write GB |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    keys = sorted(fetch, key=lambda t: -_median(fetch[t]) - _median(write.get(t, [0])))
    for k in keys:
        if "copyBuffer" in k[0] or "fillBuffer" in k[0]:
            continue
        f = _median(fetch[k])
        w = _median(write.get(k, [0]))
        print(f"| `{k[0]}` | {k[1]} | {len(fetch[k])} | {f:.0f} | {w:.0f} | {f * 1024 * scale_f / 1e9:.3f} | "
              f"{w * 1024 * scale_w / 1e9:.3f} |")


def counters_main(argv):
    con = sqlite3.connect(argv[2])
    rows = con.execute("select kernel_name, grid_size, counter_name, dispatch_id, sum(value) from counters_collection "
                       "group by kernel_name, grid_size, counter_name, dispatch_id").fetchall()
    con.close()
    title = argv[3] if len(argv) > 3 else argv[2]
    vals, names = {}, []
    for name, grid, cn, _, v in rows:
        vals.setdefault((short(name), grid), {}).setdefault(cn, []).append(v)
        if cn not in names:
            names.append(cn)
    names.sort()
    print(f"# {title}\n")
    print("Median per dispatch.\n")
    print("| kernel | grid | dispatches | " + " | ".join(names) + " |")
    print("|---|---:|---:|" + "---:|" * len(names))
    for (k, g), cs in sorted(vals.items()):
        n = max(len(v) for v in cs.values())
        cells = [f"{_median(cs[c]):.0f}" if c in cs else "" for c in names]
        print(f"| `{k}` | {g} | {n} | " + " | ".join(cells) + " |")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--pmc":
        pmc_main(sys.argv)
    elif len(sys.argv) > 1 and sys.argv[1] == "--counters":
        counters_main(sys.argv)
    else:
        main(sys.argv)
