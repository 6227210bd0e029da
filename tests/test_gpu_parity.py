"""GPU parity: every result of the HIP path (through the C ABI) equals the
oracle's -- keys, counts and group sets bit-exact, FP64 sums bit-exact
(the library sums exactly and rounds once, as the oracle does; the 1e-9
relative bound is never needed)."""
import itertools
import sys
from math import comb

import numpy as np
import pytest

import oracle
import synth
from tests import queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh as binding
    return binding


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def assert_same(got, want):
    assert got["keys"].shape == want["keys"].shape, (got["keys"].shape, want["keys"].shape)
    assert np.array_equal(got["keys"], want["keys"])
    assert np.array_equal(got["counts"], want["counts"])
    if want["sums"] is not None:
        g, w = got["sums"], want["sums"]
        assert np.array_equal(g.view(np.uint64), w.view(np.uint64)), \
            f"sums differ at {np.nonzero(g != w)[0][:5]}: {g[g != w][:5]} vs {w[g != w][:5]}"


# --------------------------------------------------------------------------
# trie construction
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,nk,dom,bag", [(1, 1, 5, False), (2047, 2, 50, False), (4099, 3, 9, True),
                                          (100_003, 2, 3000, False), (65_537, 4, 7, True)])
def test_trie_levels_match_unique(lh, n, nk, dom, bag):
    say("trie", n, nk, dom, bag)
    rng = synth.rng_for(n + nk)
    cols = [rng.integers(0, dom, n).astype(np.uint32) for _ in range(nk)]
    t = lh.trie_build(cols, bag=bag)
    info = t.info()
    tup = np.stack(cols, 1)
    uniq = np.unique(tup, axis=0)
    assert info["level_size"][-1] == len(uniq)
    assert info["n_rows"] == (n if bag else len(uniq))
    # rebuild the tuple list from the levels and compare with np.unique
    prefix = [np.zeros((1, 0), np.uint32)]
    rows = np.zeros((1, 0), np.uint32)
    starts = np.array([0], np.int64)
    ends = np.array([info["level_size"][0]], np.int64)
    for l in range(nk):
        keys, offs = t.read_level(l)
        rep = ends - starts
        assert np.all(rep >= 1)
        parent = np.repeat(np.arange(len(starts)), rep)
        idx = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)])
        assert np.array_equal(idx, np.arange(len(keys)))
        # every set strictly increasing
        seg_first = np.zeros(len(keys), bool)
        seg_first[np.cumsum(np.concatenate([[0], rep[:-1]]))] = True
        assert np.all((np.diff(keys.astype(np.int64)) > 0) | seg_first[1:])
        rows = np.concatenate([rows[parent], keys[:, None]], axis=1)
        if l + 1 < nk:
            assert np.all(np.diff(offs.astype(np.int64)) >= 1) and offs[-1] == info["level_size"][l + 1]
            starts, ends = offs[:-1].astype(np.int64), offs[1:].astype(np.int64)
        elif bag:
            run = offs.astype(np.int64)
            assert run[0] == 0 and run[-1] == n and np.all(np.diff(run) >= 1)
            _, counts = np.unique(tup, axis=0, return_counts=True)
            assert np.array_equal(np.diff(run), counts)
    assert np.array_equal(rows, uniq)
    t.free()


def test_trie_layout_census(lh):
    # a dense first level becomes one bitset; sparse second levels stay uint
    lo, hi = synth.rmat_edges(14, 16 << 14, seed=5)
    t = lh.trie_build([lo, hi])
    inf = t.info()
    assert inf["level_sets"][0] == 1 and inf["level_bitsets"][0] == 1
    assert inf["level_bitsets"][1] < inf["level_sets"][1]
    tu = lh.trie_build([lo, hi], layout="uint")
    assert tu.info()["level_bitsets"] == [0, 0]


# --------------------------------------------------------------------------
# triangle COUNT
# --------------------------------------------------------------------------

def _tri_gpu(lh, lo, hi, **kw):
    return int(lh.run_query(queries.triangle(lo, hi), **kw)["counts"][0])


@pytest.mark.parametrize("n", [3, 4, 17, 64, 130])
def test_triangle_complete_graph(lh, n):
    lo, hi = synth.complete_graph(n)
    assert _tri_gpu(lh, lo, hi) == comb(n, 3)


def test_triangle_families(lh):
    assert _tri_gpu(lh, *synth.complete_tripartite(5, 7, 9)) == 5 * 7 * 9
    assert _tri_gpu(lh, *synth.wheel(100)) == 100
    assert _tri_gpu(lh, *synth.cycle(1000)) == 0
    assert _tri_gpu(lh, *synth.random_bipartite(60, 70, 0.3, seed=2)) == 0


@pytest.mark.parametrize("layout", ["plain", "uint", "bitset"])
def test_triangle_rmat_all_orders_and_layouts(lh, layout):
    lo, hi = synth.rmat_edges(13, 16 << 13, seed=11)
    want = int(oracle.join_aggregate(queries.triangle(lo, hi))["counts"][0])
    say("rmat13 triangles", want, layout)
    for order in itertools.permutations(range(3)):
        assert _tri_gpu(lh, lo, hi, attr_order=list(order), layout=layout) == want


def test_triangle_count_grouped_by_vertex(lh):
    lo, hi = synth.rmat_edges(12, 16 << 12, seed=12)
    q = queries.triangle(lo, hi)
    q["out"] = [0]
    got = lh.run_query(q)
    assert_same(got, oracle.join_aggregate(q))


# --------------------------------------------------------------------------
# SUM: sparse matrix products
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,deg", [(300, 7), (4096, 10)])
def test_spgemm_bit_exact(lh, n, deg):
    a = synth.sparse_matrix(n, deg, seed=1)
    b = synth.sparse_matrix(n, deg, seed=11)
    q = queries.spgemm(a, b)
    want = oracle.join_aggregate(q)
    got = lh.run_query(q, return_plan_info=True)
    assert got["plan"]["attr_order"] == [0, 1, 2]      # the relaxed order
    assert_same(got, want)
    for layout in ("uint", "bitset"):
        assert_same(lh.run_query(q, layout=layout), want)
    # the materialized-first order gives the same bits
    assert_same(lh.run_query(q, attr_order=[0, 2, 1]), want)


def test_spgemm_zipf_rows(lh):
    rng = synth.rng_for(44)
    a = synth.zipf_degree_matrix(3000, 1.1, 16, rng)
    q = queries.spgemm(a, a)
    assert_same(lh.run_query(q), oracle.join_aggregate(q))


def test_spmv_bit_exact(lh):
    rng = synth.rng_for(8)
    a = synth.zipf_degree_matrix(5000, 1.1, 16, rng)
    x = synth.uniform_pm1(rng, 5000)
    q = queries.spmv(a, x)
    got = lh.run_query(q, return_plan_info=True)
    assert got["plan"]["case_prefix"] == 1
    assert_same(got, oracle.join_aggregate(q))


def test_total_sum_exact(lh):
    a = synth.sparse_matrix(2000, 10, seed=3)
    b = synth.sparse_matrix(2000, 10, seed=4)
    q = queries.spgemm(a, b)
    q["out"] = []
    assert_same(lh.run_query(q), oracle.join_aggregate(q))


# --------------------------------------------------------------------------
# star schema: filters, bag relations, GROUP BY a meta column
# --------------------------------------------------------------------------

def test_star_group_by(lh):
    s = synth.star_schema(n_fact=300_000, dims=(20_000, 5000, 1000, 100), seed=3)
    q = queries.star(s, u_hi=0.5, m2=0, m3=3)
    want = oracle.join_aggregate(q)
    say("star groups", len(want["keys"]))
    got = lh.run_query(q, return_plan_info=True)
    assert_same(got, want)
    assert_same(lh.run_query(q, attr_order=[3, 2, 1, 0]), want)


def test_star_empty_filter(lh):
    s = synth.star_schema(n_fact=5000, dims=(100, 50, 20, 10), seed=9)
    q = queries.star(s, u_hi=-1.0)
    got = lh.run_query(q)
    assert got["keys"].shape == (0, 1)


# --------------------------------------------------------------------------
# random tiny hypergraph queries
# --------------------------------------------------------------------------

@pytest.mark.parametrize("block", range(8))
def test_random_queries(lh, block):
    for seed in range(block * 40, block * 40 + 40):
        q = queries.random_query(seed)
        try:
            want = oracle.join_aggregate(q)
        except oracle.OracleError:
            continue
        got = lh.run_query(q)
        try:
            assert_same(got, want)
        except AssertionError:
            say("random query seed", seed)
            raise


@pytest.mark.parametrize("policy", ["plain", "learned"])
def test_materialized_joins(lh, policy):
    """COUNT with every attribute an output (the join materialized) in a
    random output order: bag runs multiply, filters apply, rows come out
    sorted by the declared columns."""
    n = 0
    for seed in range(3000, 3120):
        q = queries.random_query(seed, max_atoms=3, max_attrs=4, domain=12, max_rows=60)
        rng = synth.rng_for(seed + 7)
        q["out"] = rng.permutation(q["n_attrs"]).tolist()
        q["agg"] = "count"
        q["group"] = []
        for a in q["atoms"]:
            a["anno"] = -1
        want = oracle.join_aggregate(q)
        got = lh.run_query(q, policy=policy)
        try:
            assert_same(got, want)
        except AssertionError:
            say("materialized join seed", seed, "policy", policy)
            raise
        n += len(want["counts"])
    assert n > 100


def test_random_queries_larger_domains(lh):
    for seed in range(1000, 1030):
        q = queries.random_query(seed, max_atoms=3, max_attrs=4, domain=40, max_rows=300)
        want = oracle.join_aggregate(q)
        got = lh.run_query(q)
        assert_same(got, want)


def test_ungrouped_empty_join_has_one_zero_row(lh):
    lo = np.array([0, 1], np.uint32)
    hi = np.array([1, 2], np.uint32)
    got = lh.run_query(queries.triangle(lo, hi))
    assert got["counts"].tolist() == [0] and got["keys"].shape == (1, 0)


def test_no_device_memory_leaks(lh):
    before = lh.live_allocations()
    lo, hi = synth.complete_graph(30)
    for _ in range(3):
        _tri_gpu(lh, lo, hi)
    a = synth.sparse_matrix(100, 5, seed=1)
    lh.run_query(queries.spgemm(a, a))
    assert lh.live_allocations() == before


def _mixed_pairs():
    rng = synth.rng_for(7)
    pairs = list(synth.set_pairs(30000, 60000, 6, seed=100))         # density 1/2
    pairs += synth.set_pairs(5000, 64 * 5000, 3, seed=101)           # sparse
    big = np.sort(rng.choice(1 << 20, 40000, replace=False)).astype(np.uint32)
    small = np.sort(rng.choice(1 << 20, 400, replace=False)).astype(np.uint32)
    pairs.append((big, small))                                       # size ratio 100
    pairs.append((small, big))
    pairs.append((np.arange(0, 1000, dtype=np.uint32), np.arange(5000, 7000, dtype=np.uint32)))  # disjoint
    pairs.append((np.arange(1, 4000, 3, dtype=np.uint32), np.arange(2, 4000, 2, dtype=np.uint32)))
    pairs.append((np.array([7], np.uint32), np.array([7], np.uint32)))
    return pairs


def _merge_pairs():
    """Pairs for the merge path (two sorted sets of 4096 elements or more,
    sizes within a factor of 4): the bounds of that rule on both sides,
    identical sets (a common value on every tile boundary that falls
    between a set-0 element and its equal set-1 element), disjoint sets in
    both orders, tiles made of one set only, and values near 2^32."""
    rng = synth.rng_for(11)

    def draw(n, universe, base=0):
        return (np.sort(rng.choice(universe, n, replace=False)) + base).astype(np.uint32)

    pairs = [(draw(4096, 8192), draw(4096, 8192)),                # both at the size bound
             (draw(4095, 8192), draw(9000, 20000)),               # one below it: probed
             (draw(4096, 40000), draw(16384, 40000)),             # ratio exactly 4
             (draw(4096, 40000), draw(16385, 40000)),             # ratio above 4: probed
             (draw(12345, 50000), draw(23456, 50000))]
    same = draw(20000, 1 << 20)
    pairs.append((same, same.copy()))
    pairs.append((np.arange(0, 10000, dtype=np.uint32), np.arange(10000, 20000, dtype=np.uint32)))
    pairs.append((np.arange(10000, 20000, dtype=np.uint32), np.arange(0, 10000, dtype=np.uint32)))
    pairs.append((np.arange(0, 40000, 2, dtype=np.uint32), np.arange(0, 60000, 3, dtype=np.uint32)))
    top = np.uint32(0xFFFFFFFE)
    pairs.append((top - np.arange(9000, dtype=np.uint32)[::-1] * 2, top - np.arange(9000, dtype=np.uint32)[::-1] * 3))
    pairs.append((draw(6000, 1 << 31, base=1 << 31), draw(7000, 1 << 31, base=1 << 31)))
    return pairs


@pytest.mark.parametrize("grouped", [True, False])
def test_merge_path_intersections(lh, grouped):
    """Rows that take the merge path, per pair (COUNT GROUP BY pair) and in
    total (COUNT): equal to numpy's intersect1d and to the oracle."""
    pairs = _merge_pairs()
    q = queries.set_pairs(pairs)
    if not grouped:
        q["out"] = []
    say(f"merge pairs grouped={grouped}: {len(pairs)} pairs")
    ta = lh.trie_build(q["atoms"][0]["keys"], layout="uint")
    tb = lh.trie_build(q["atoms"][1]["keys"], layout="uint")
    p = lh.plan(2, [(ta, [0, 1], -1), (tb, [0, 1], -1)], out=q["out"], agg="count", attr_order=[0, 1],
                policy="fixed")
    lh.profile_reset()
    lh.profile_enable(True)
    r = lh.join_aggregate([p])[0]
    got = r.to_host()
    lh.profile_enable(False)
    prof = lh.profile_read()
    r.free(); p.free(); ta.free(); tb.free()
    assert prof.get("leaf_merge", {"launches": 0})["launches"] == 1
    sizes = np.array([len(np.intersect1d(a, b)) for a, b in pairs])
    if grouped:
        nz = np.nonzero(sizes)[0]
        assert np.array_equal(got["keys"][:, 0], nz) and np.array_equal(got["counts"], sizes[nz])
    else:
        assert int(got["counts"][0]) == int(sizes.sum())
    assert_same(got, oracle.join_aggregate(q))


@pytest.mark.parametrize("la,lb", [("uint", "uint"), ("uint", "bitset"), ("bitset", "uint"),
                                   ("bitset", "bitset"), ("plain", "plain")])
def test_set_pair_intersections(lh, la, lb):
    """Intersections of set pairs (the intersection micro-benchmark's shape)
    in every layout combination, including the word-AND path of two
    bitsets: equal to the oracle and to numpy's intersect1d."""
    pairs = _mixed_pairs()
    q = queries.set_pairs(pairs)
    say(f"set pairs {la}/{lb}: {len(pairs)} pairs")
    ta = lh.trie_build(q["atoms"][0]["keys"], layout=la)
    tb = lh.trie_build(q["atoms"][1]["keys"], layout=lb)
    p = lh.plan(2, [(ta, [0, 1], -1), (tb, [0, 1], -1)], out=[0], agg="count")
    r = lh.join_aggregate([p])[0]
    got = r.to_host()
    r.free(); p.free(); ta.free(); tb.free()
    want = oracle.join_aggregate(q)
    assert_same(got, want)
    sizes = np.array([len(np.intersect1d(a, b)) for a, b in pairs])
    nz = np.nonzero(sizes)[0]
    assert np.array_equal(got["keys"][:, 0], nz) and np.array_equal(got["counts"], sizes[nz])


@pytest.mark.parametrize("bag,nk", [(False, 2), (True, 2), (False, 3), (True, 3)])
def test_column_stats(lh, bag, nk):
    """Per-column statistics behind the learned order features: distinct
    values and the largest number of the trie's rows sharing one value,
    against numpy on the rows the trie keeps (all rows for a bag, distinct
    key tuples for a set)."""
    rng = synth.rng_for(60 + nk + 10 * bag)
    n = 50_000
    cols = [rng.integers(0, d, n).astype(np.uint32) for d in (300, 2000, 70)[:nk]]
    t = lh.trie_build(cols, bag=bag)
    inf = t.info()
    t.free()
    rows = np.stack(cols, 1)
    if not bag:
        rows = np.unique(rows, axis=0)
    for l in range(nk):
        vals, cnt = np.unique(rows[:, l], return_counts=True)
        assert inf["col_distinct"][l] == len(vals)
        assert inf["col_freq_max"][l] == cnt.max()


@pytest.mark.parametrize("case", ["one value", "all distinct", "one row", "hub"])
def test_column_stats_edge_runs(lh, case):
    """Column statistics where the runs of a column are extreme: one run
    over every row, runs of one row, a single row, and one hub value over
    most rows (a run far longer than the rest)."""
    rng = synth.rng_for(70)
    n = 1 if case == "one row" else 40_000
    a = rng.integers(0, 500, n).astype(np.uint32)
    if case == "one value":
        b = np.full(n, 7, np.uint32)
    elif case == "all distinct":
        b = rng.permutation(n).astype(np.uint32)
    elif case == "hub":
        b = np.where(rng.random(n) < 0.9, 12345, rng.integers(0, 1 << 20, n)).astype(np.uint32)
    else:
        b = np.array([3], np.uint32)
    for bag in (False, True):
        t = lh.trie_build([a, b], bag=bag)
        inf = t.info()
        t.free()
        rows = np.stack([a, b], 1)
        if not bag:
            rows = np.unique(rows, axis=0)
        for l in range(2):
            vals, cnt = np.unique(rows[:, l], return_counts=True)
            assert inf["col_distinct"][l] == len(vals), (case, bag, l)
            assert inf["col_freq_max"][l] == cnt.max(), (case, bag, l)
