"""lh_trie_build on input that is already (partly) in trie order: one pass
finds the sorted trailing levels, and the sort skips them.  The tries must
equal those built from the same rows shuffled, level by level, and queries
over them must give the oracle's result."""
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


def levels(t):
    return [t.read_level(l) for l in range(t.info()["n_levels"])]


def rows3(rng, n, dup):
    a = rng.integers(0, 300, n).astype(np.uint32)
    b = rng.integers(0, 50, n).astype(np.uint32)
    c = rng.integers(0, 5000, n).astype(np.uint32)
    if not dup:
        key = np.unique(np.stack([a, b, c], 1), axis=0)
        a, b, c = key[:, 0].copy(), key[:, 1].copy(), key[:, 2].copy()
    return [a, b, c]


@pytest.mark.parametrize("bag", [False, True])
@pytest.mark.parametrize("order", ["sorted", "tail1", "tail2", "reverse", "shuffled"])
def test_presorted_input_builds_the_same_trie(lh, bag, order):
    print(f"presorted bag={bag} order={order}", file=sys.stderr, flush=True)
    rng = synth.rng_for(31)
    cols = rows3(rng, 200_000, dup=True)
    if not bag:
        cols = [np.ascontiguousarray(c) for c in cols]
    v = synth.uniform_pm1(rng, len(cols[0]))
    if order == "sorted":
        perm = np.lexsort((cols[2], cols[1], cols[0]))
    elif order == "tail1":          # last level sorted, the rest not
        perm = np.argsort(cols[2], kind="stable")
    elif order == "tail2":          # last two levels sorted
        perm = np.lexsort((cols[2], cols[1]))
    elif order == "reverse":        # descending: no tail
        perm = np.lexsort((cols[2], cols[1], cols[0]))[::-1]
    else:
        perm = rng.permutation(len(cols[0]))
    ordered = [c[perm] for c in cols]
    shuffled_perm = rng.permutation(len(cols[0]))
    shuffled = [c[shuffled_perm] for c in cols]
    annos_o = [v[perm]] if bag else []
    annos_s = [v[shuffled_perm]] if bag else []
    t1 = lh.trie_build(ordered, annos_o, bag=bag)
    t2 = lh.trie_build(shuffled, annos_s, bag=bag)
    try:
        for (k1, o1), (k2, o2) in zip(levels(t1), levels(t2)):
            assert np.array_equal(k1, k2) and np.array_equal(o1, o2)
        q_atoms = [(t1, [0, 1, 2], 0 if bag else -1)]
        p = lh.plan(3, q_atoms, out=[1], agg="sum" if bag else "count")
        got = lh.join_aggregate([p])[0].to_host()
        p.free()
    finally:
        t1.free()
        t2.free()
    q = {"n_attrs": 3, "out": [1], "agg": "sum" if bag else "count",
         "atoms": [{"keys": cols, "attrs": [0, 1, 2], "annos": [v] if bag else [], "anno": 0 if bag else -1,
                    "bag": bag}]}
    want = oracle.join_aggregate(q)
    assert np.array_equal(got["keys"], want["keys"]) and np.array_equal(got["counts"], want["counts"])
    if bag:
        assert np.array_equal(got["sums"], want["sums"])


def test_sorted_design_matrix_trie(lh):
    """(row, feature) triples in row-major order build both tries of a
    design matrix; the transposed one from a one-level tail."""
    rng = synth.rng_for(32)
    rows = np.repeat(np.arange(0, 40000, 2, dtype=np.uint32), 9)
    feats = np.tile(np.array([0, 3, 7, 12, 20, 44, 90, 101, 139], np.uint32), 20000)
    vals = synth.uniform_pm1(rng, len(rows))
    xr = lh.trie_build([rows, feats], [vals], bag=True)
    xc = lh.trie_build([rows, feats], [vals], level_order=[1, 0], bag=True)
    try:
        k0, o0 = xr.read_level(0)
        assert np.array_equal(k0, np.arange(0, 40000, 2)) and np.all(np.diff(o0) == 9)
        f0, fo = xc.read_level(0)
        assert list(f0) == [0, 3, 7, 12, 20, 44, 90, 101, 139] and np.all(np.diff(fo) == 20000)
        r1, _ = xc.read_level(1)
        assert np.array_equal(r1, np.tile(np.arange(0, 40000, 2, dtype=np.uint32), 9))
    finally:
        xr.free()
        xc.free()
