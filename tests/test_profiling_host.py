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
