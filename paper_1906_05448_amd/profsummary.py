"""Summarise a rocprofv3 results database (kernel trace) as a text table.

    python -m paper_1906_05448_amd.profsummary <run_results.db> [title]

Prints one row per kernel: calls, total (ms) and average (us) duration, share.
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


if __name__ == "__main__":
    main(sys.argv)
