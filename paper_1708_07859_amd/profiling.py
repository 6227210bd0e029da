"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1708_07859_amd.profiling stats <kernel_stats.csv> <out.md> --command "..." --title "..."
    python -m paper_1708_07859_amd.profiling traffic <fetch_dir> <write_dir> <kernel> <out.txt> \
        --copy-fetch <dir> --copy-write <dir> --command "..."

``stats`` turns a ``--kernel-trace --stats`` kernel table into a short
markdown table.  ``traffic`` averages FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) of one kernel over two ``--pmc`` runs and scales each by what the
same counter reads for a plain 1 GiB device copy; the summary records the
hash of the kernel's source file so that a benchmark can tell whether the
counters still describe the code it runs.
"""
import argparse
import csv
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = {  # kernel -> source file whose hash stamps its counters
    "k_leaf2_count": os.path.join(HERE, "csrc", "join.hip"),
    "k_elem": os.path.join(HERE, "csrc", "join.hip"),
    "k_lr_cols": os.path.join(HERE, "csrc", "ml.hip"),
    "k_lr_cols_blocked": os.path.join(HERE, "csrc", "ml.hip"),
    "k_lr_rows": os.path.join(HERE, "csrc", "ml.hip"),
}
COPY_BYTES = 1 << 30


def short_name(k):
    k = k.replace("lh::(anonymous namespace)::", "").replace("lh::", "")
    return re.sub(r"\(.*", "", k).strip()


def source_hash(kernel):
    path = KERNEL_SOURCE.get(kernel)
    if not path or not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stats_md(stats_csv, out, command, title, top=14):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 kernel stats: {title}", "", "Command (from the repository root, on an MI355X):", "",
             "    " + command, "", "| kernel | calls | total ms | avg ms | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(run_dir, kernel, counter):
    path = os.path.join(run_dir, "run_counter_collection.csv")
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter and short_name(r["Kernel_Name"]).endswith(kernel)]
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel} in {path}")
    return sum(vals) / len(vals), len(vals)


def traffic_txt(fetch_dir, write_dir, kernel, out, copy_fetch, copy_write, command):
    fk, nf = _per_dispatch(fetch_dir, kernel, "FETCH_SIZE")
    wk, nw = _per_dispatch(write_dir, kernel, "WRITE_SIZE")
    cf, _ = _per_dispatch(copy_fetch, "copyBuffer", "FETCH_SIZE")
    cw, _ = _per_dispatch(copy_write, "copyBuffer", "WRITE_SIZE")
    ff = COPY_BYTES / 1024 / cf
    wf = COPY_BYTES / 1024 / cw
    total = (fk * ff + wk * wf) * 1024
    lines = [
        f"kernel: {kernel}",
        f"source_sha256_16: {source_hash(kernel)}",
        f"fetch_kib_per_dispatch: {fk:.1f}  ({nf} dispatches)",
        f"write_kib_per_dispatch: {wk:.1f}  ({nw} dispatches)",
        f"copy_1gib_fetch_kib: {cf:.1f}  -> fetch_factor: {ff:.4f}",
        f"copy_1gib_write_kib: {cw:.1f}  -> write_factor: {wf:.4f}",
        f"hbm_bytes_per_dispatch: {total:.0f}",
        "command: " + command,
    ]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_traffic(path, kernel):
    """HBM bytes per dispatch of `kernel` from a traffic summary, or None
    when the summary is missing or was taken on a different source."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if kv.get("kernel") != kernel or kv.get("source_sha256_16") != source_hash(kernel):
        return None
    return float(kv["hbm_bytes_per_dispatch"])


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--title", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("kernel")
    t.add_argument("out")
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--command", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        stats_md(a.csv, a.out, a.command, a.title)
    else:
        traffic_txt(a.fetch_dir, a.write_dir, a.kernel, a.out, a.copy_fetch, a.copy_write, a.command)


if __name__ == "__main__":
    main()
