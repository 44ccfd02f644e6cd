"""Render the parity records of a GPU test run (the JSON lines that
tests.parity_util.record appends to $RMHMC_PARITY_LOG) as a Markdown table:
one row per recorded case with its errors, floor and bar.

    python -m tests.parity_report RECORDS.jsonl "COMMAND" > SUMMARY.md
"""
import json
import sys


def fmt(v):
    if isinstance(v, float):
        return f"{v:.3g}"
    return str(v)


def main(path, command):
    rows = [json.loads(line) for line in open(path) if line.strip()]
    print("# GPU parity records: error, floor and bar of every recorded case\n")
    print(f"Command: `{command}`\n")
    print("Errors are norm-wise relative (scalars: |x - y| / max(|y|, 1)); `floor` is the FP64 "
          "reference's disagreement with itself on the same problem with the data points "
          "reordered, `bar` the threshold the test asserted.\n")
    by_case = {}
    for r in rows:
        by_case.setdefault(r["case"], []).append(r)
    for case, rs in by_case.items():
        keys = []
        for r in rs:
            for k in r:
                if k != "case" and k not in keys:
                    keys.append(k)
        print(f"## {case}\n")
        print("| " + " | ".join(keys) + " |")
        print("|" + "---|" * len(keys))
        for r in rs:
            print("| " + " | ".join(fmt(r.get(k, "")) for k in keys) + " |")
        print()


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else "")
