"""Trie builds over key widths that take every form of the build's radix
sort: one pass, an odd and an even number of passes, a column of zeros
(no bits), a full 64-bit packed key, and keys wider than one word (the
multi-word sort).  Bag relations carry an annotation, so the row
permutation that the sort produces is checked too: the SUM of every key
tuple must equal the oracle's, bit for bit (section 2.2's trie build;
section 3's SUM over a bag)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh as binding
    return binding


# (case, key domains per column, bag): the packed key's bits decide the passes
CASES = [
    ("1 pass", [2], True),                          # 1 bit
    ("3 passes", [1 << 20], True),                  # 20 bits
    ("3 passes, 2 columns", [1 << 10, 1 << 12], True),
    ("zero column", [1, 1000], True),               # 0 + 10 bits, 2 passes
    ("3 passes, set", [256, 256, 256], False),      # 24 bits
    ("8 passes", [1 << 16] * 4, True),              # 64 bits
    ("wider than a word", [1 << 22] * 3, True),     # 66 bits: two sorts of 6 and 3 passes
    ("wider than a word, set", [1 << 22] * 3, False),
]


@pytest.mark.parametrize("case,doms,bag", CASES, ids=[c[0] for c in CASES])
def test_sort_paths(lh, case, doms, bag):
    print(f"sort path: {case}", file=sys.stderr, flush=True)
    rng = synth.rng_for(41 + len(doms))
    n = 150_001
    cols = [rng.integers(0, d, n).astype(np.uint32) for d in doms]
    # the largest value of each domain occurs, so each column has its bits
    for c, d in zip(cols, doms):
        c[rng.integers(0, n)] = d - 1
    v = synth.uniform_pm1(rng, n) if bag else None
    t = lh.trie_build(cols, [v] if bag else [], bag=bag)
    nk = len(doms)
    try:
        uniq = np.unique(np.stack(cols, 1), axis=0)
        info = t.info()
        assert info["level_size"][-1] == len(uniq)
        assert info["n_rows"] == (n if bag else len(uniq))
        keys0, _ = t.read_level(0)
        assert np.array_equal(keys0, np.unique(cols[0]))
        p = lh.plan(nk, [(t, list(range(nk)), 0 if bag else -1)], out=list(range(nk)),
                    agg="sum" if bag else "count")
        got = lh.join_aggregate([p])[0].to_host()
        p.free()
    finally:
        t.free()
    q = {"n_attrs": nk, "out": list(range(nk)), "agg": "sum" if bag else "count",
         "atoms": [{"keys": cols, "attrs": list(range(nk)), "annos": [v] if bag else [],
                    "anno": 0 if bag else -1, "bag": bag}]}
    want = oracle.join_aggregate(q)
    assert np.array_equal(got["keys"], want["keys"])
    assert np.array_equal(got["counts"], want["counts"])
    if bag:
        assert np.array_equal(got["sums"].view(np.uint64), want["sums"].view(np.uint64))
