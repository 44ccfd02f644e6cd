"""Summarise a rocprofv3 kernel-stats CSV into a short Markdown table.

    python -m paper_2511_06407_amd.profile_summary STATS_CSV [--title T] [--cmd CMD] [--top N]

rocprofv3 --kernel-trace --stats writes *_kernel_stats.csv with one row per
kernel name (calls, total / average / min / max duration in ns, percentage).
"""
import argparse
import csv
import re
import sys


def short_name(name):
    n = name.replace("(anonymous namespace)::", "").replace("rmhmc::", "")
    n = re.sub(r"^void ", "", n)
    # drop the parameter list (the last balanced parenthesis group)
    if n.endswith(")"):
        depth = 0
        for i in range(len(n) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(n[i], 0)
            if depth == 0:
                n = n[:i]
                break
    return n


def load(path):
    with open(path) as f:
        rows = list(csv.DictReader(f))
    out = []
    for r in rows:
        out.append({"name": r.get("Name") or r.get("KernelName"),
                    "calls": int(r.get("Calls", 0)),
                    "total_ns": float(r.get("TotalDurationNs", 0)),
                    "avg_ns": float(r.get("AverageNs", 0)),
                    "pct": float(r.get("Percentage", 0))})
    out.sort(key=lambda r: -r["total_ns"])
    return out


def to_markdown(rows, title, cmd, top):
    lines = [f"# {title}", "", f"Command: `{cmd}`", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append(f"| `{short_name(r['name'])}` | {r['calls']} | {r['total_ns'] / 1e6:.2f} | "
                     f"{r['avg_ns'] / 1e3:.2f} | {r['pct']:.1f} |")
    tot = sum(r["total_ns"] for r in rows)
    lines += ["", f"All kernels: {sum(r['calls'] for r in rows)} launches, {tot / 1e6:.2f} ms."]
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("csv")
    ap.add_argument("--title", default="rocprofv3 kernel statistics")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--top", type=int, default=20)
    a = ap.parse_args(argv)
    sys.stdout.write(to_markdown(load(a.csv), a.title, a.cmd, a.top))


if __name__ == "__main__":
    main()
