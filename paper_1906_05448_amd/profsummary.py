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


def short(name: str) -> str:
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
