"""Hardware-counter byte counts of the library's kernels, read back by the
benchmark.

A traffic summary (profiles/*_traffic.txt) holds, for one kernel, the bytes
its dispatches moved between the L2 caches and memory according to
rocprofv3 counters, and the hash of the kernel's source file when the
counters were taken.  `read_traffic` returns the bytes per dispatch, or None
once the source has changed (the counters then describe other code).
"""
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = {  # kernel -> source file whose hash stamps its counters
    "k_leaf2_count": os.path.join(HERE, "csrc", "join.hip"),
    "k_leaf2_count_top": os.path.join(HERE, "csrc", "join.hip"),
    "k_leaf2_merge": os.path.join(HERE, "csrc", "join.hip"),
    "k_elem": os.path.join(HERE, "csrc", "join.hip"),
    "k_lr_cols": os.path.join(HERE, "csrc", "ml.hip"),
    "k_lr_cols_blocked": os.path.join(HERE, "csrc", "ml.hip"),
    "k_lr_rows": os.path.join(HERE, "csrc", "ml.hip"),
}


def source_hash(kernel):
    path = KERNEL_SOURCE.get(kernel)
    if not path or not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(path, kernel):
    """HBM bytes per dispatch of `kernel` from a traffic summary, or None
    when the summary is missing, has no block for the kernel, or was taken
    on a different source.  A summary holds one block per kernel, each
    opened by its `kernel:` line."""
    if not os.path.exists(path):
        return None
    blocks, kv = [], None
    for line in open(path):
        if ":" not in line:
            continue
        k, v = line.split(":", 1)
        k, v = k.strip(), v.strip()
        if k == "kernel":
            kv = {}
            blocks.append(kv)
        if kv is not None:
            kv[k] = v.split()[0] if v else ""
    for kv in blocks:
        if kv.get("kernel") == kernel and kv.get("source_sha256_16") == source_hash(kernel):
            return float(kv["hbm_bytes_per_dispatch"])
    return None
