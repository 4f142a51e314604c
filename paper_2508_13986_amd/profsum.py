"""Summaries of rocprofv3 output for the GBEES kernels.

  python -m paper_2508_13986_amd.profsum stats KERNEL_STATS_CSV --command CMD [--note TEXT]
      Markdown table of per-kernel time from a `rocprofv3 --kernel-trace --stats
      --output-format csv` run.

  python -m paper_2508_13986_amd.profsum pmc --kernel NAME --bench-log LOG --copy-bytes B
          --csv COUNTER_CSV [--csv ...] --command CMD [--command ...] --out JSON
      Per-launch averages of the counters in one or more `rocprofv3 --pmc` runs
      for the kernels whose name contains NAME.  FETCH_SIZE and WRITE_SIZE (KiB
      per dispatch) are turned into bytes and divided by what the same counter
      reads per byte for the largest plain device copy in the same run (B bytes
      read and B bytes written), so that the result is in HBM bytes.  The
      bench's JSON line in LOG gives the bricks per launch.
"""
import argparse
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_KERNELS = ("copyBuffer", "elementwise_kernel", "copy_kernel")
N_XCD, N_CU = 8, 256  # MI355X


def kernel_source_hash():
    """Hash of the device sources that the counters describe."""
    h = hashlib.sha256()
    for f in ("gbees_dev.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2508_13986_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    s = name[5:] if name.startswith("void ") else name
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return s[:i]
    return s


def stats_table(path, command, note):
    rows = list(csv.DictReader(open(path)))
    total = sum(int(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -int(r["TotalDurationNs"])):
        t = int(r["TotalDurationNs"])
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {t / 1e6:.1f} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{100.0 * t / total:.1f} |")
    text = ["Command (MI355X, one GPU):", "", "```", command, "```", ""] + out + ["", f"Total kernel time {total / 1e6:.1f} ms."]
    if note:
        text += ["", note]
    return "\n".join(text)


def bench_line(log):
    for line in open(log):
        line = line.strip()
        if line.startswith("{") and '"metric"' in line:
            return json.loads(line)
    raise SystemExit(f"no bench JSON line in {log}")


def pmc_summary(args):
    per = defaultdict(lambda: defaultdict(list))  # counter -> dispatch -> values (summed over dims)
    names = {}
    for path in args.csv:
        for r in csv.DictReader(open(path)):
            key = (path, r["Dispatch_Id"])
            names[key] = r["Kernel_Name"]
            per[r["Counter_Name"]][key].append(float(r["Counter_Value"]))
    result = {"kernel": args.kernel, "kernel_source_hash": kernel_source_hash(), "commands": args.command,
              "copy_bytes": args.copy_bytes}
    bl = bench_line(args.bench_log)
    result["bricks_per_launch"] = bl["config"]["bricks_per_step_mean"]
    result["workload"] = bl["config"]["workload"]
    for counter, disp in per.items():
        vals = {k: sum(v) for k, v in disp.items()}
        mine = [v for k, v in vals.items() if args.kernel in names[k]]
        if not mine:
            continue
        mean = sum(mine) / len(mine)
        entry = {"launches": len(mine), "mean_per_launch": mean}
        if counter in ("FETCH_SIZE", "WRITE_SIZE"):
            copies = [v for k, v in vals.items() if any(c in names[k] for c in COPY_KERNELS)]
            if not copies:
                raise SystemExit(f"no copy kernel in the {counter} run to calibrate against")
            factor = max(copies) * 1024.0 / args.copy_bytes
            entry["copy_kib"] = max(copies)
            entry["calibration_factor"] = factor
            entry["hbm_bytes_per_launch"] = mean * 1024.0 / factor
            key = "fetch_bytes_per_launch" if counter == "FETCH_SIZE" else "write_bytes_per_launch"
            result[key] = entry["hbm_bytes_per_launch"]
        result.setdefault("counters", {})[counter] = entry
    c = {k: v["mean_per_launch"] for k, v in result.get("counters", {}).items()}
    if "SQ_ACTIVE_INST_VALU" in c and "GRBM_GUI_ACTIVE" in c:
        # GRBM_GUI_ACTIVE is summed over the XCDs; SQ_ACTIVE_INST_VALU counts
        # quad-cycles (one per wave64 VALU instruction issue) over all CUs.
        per_xcd = c["GRBM_GUI_ACTIVE"] / N_XCD
        result["derived"] = {"valu_busy_pct": 100.0 * c["SQ_ACTIVE_INST_VALU"] / N_CU / per_xcd}
        if "SQ_WAVE_CYCLES" in c:
            for k in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY"):
                if k in c:
                    result["derived"][k.lower() + "_frac_of_wave_cycles"] = c[k] / c["SQ_WAVE_CYCLES"]
        if "SQ_INSTS_VALU" in c and "SQ_WAVES" in c:
            result["derived"]["valu_insts_per_wave"] = c["SQ_INSTS_VALU"] / c["SQ_WAVES"]
    return result


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    p = sub.add_parser("pmc")
    p.add_argument("--kernel", required=True)
    p.add_argument("--bench-log", required=True)
    p.add_argument("--copy-bytes", type=int, required=True)
    p.add_argument("--csv", action="append", required=True)
    p.add_argument("--command", action="append", required=True)
    p.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats_table(args.csv, args.command, args.note))
    else:
        res = pmc_summary(args)
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)
            fh.write("\n")
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    sys.exit(main())
