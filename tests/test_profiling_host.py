"""The traffic-summary reader the benchmark uses for its `traffic` field:
one block per kernel, and a block counts only while the kernel's source
file hashes as it did when the counters were taken."""
from paper_1708_07859_amd import profiling


def test_blocks_by_kernel_and_source_hash(tmp_path):
    h = profiling.source_hash("k_leaf2_count")
    assert h and h == profiling.source_hash("k_leaf2_merge")   # one source file
    f = tmp_path / "t.txt"
    f.write_text(f"kernel: k_leaf2_count\nsource_sha256_16: {h}\nhbm_bytes_per_dispatch: 1000\n"
                 f"command: x\n\nkernel: k_leaf2_merge\nsource_sha256_16: {h}\nhbm_bytes_per_dispatch: 250.5\n"
                 f"kernel: k_leaf2_count_top\nsource_sha256_16: 0000000000000000\nhbm_bytes_per_dispatch: 7\n")
    assert profiling.read_traffic(str(f), "k_leaf2_count") == 1000.0
    assert profiling.read_traffic(str(f), "k_leaf2_merge") == 250.5
    assert profiling.read_traffic(str(f), "k_leaf2_count_top") is None      # stale source
    assert profiling.read_traffic(str(f), "k_elem") is None                 # no block
    assert profiling.read_traffic(str(tmp_path / "missing.txt"), "k_leaf2_count") is None


def test_committed_summaries_describe_the_committed_kernels():
    """The benchmark's `traffic` field reads these summaries; each must
    have been taken on the kernel source in the tree (else the field goes
    null), so an edit to a kernel's source calls for new counters."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for name, kernels in (("triangle_rmat22_learned_leaf_traffic.txt", ("k_leaf2_count", "k_leaf2_count_top")),
                          ("triangle_rmat22_plain_leaf_traffic.txt", ("k_leaf2_count", "k_leaf2_count_top")),
                          ("voter_lr_cols_blocked_traffic.txt", ("k_lr_cols_blocked",)),
                          ("voter_lr_rows_traffic.txt", ("k_lr_rows",))):
        path = os.path.join(root, "profiles", name)
        for k in kernels:
            b = profiling.read_traffic(path, k)
            assert b is not None and b > 0, (name, k)
