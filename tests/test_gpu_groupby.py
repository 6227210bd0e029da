"""GROUP BY outside the attribute order's prefix (section 5): the key union
of a projected-away attribute placed before a materialized one, and GROUP BY
on meta columns, under the three implementations (sort, device-wide hash
table, dense array) and the automatic choice.  Every implementation must
give the oracle's result bit for bit (sums are exact whichever runs)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import queries

pytestmark = pytest.mark.gpu

IMPLS = ["sort", "hash", "dense", "auto"]


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
        assert np.array_equal(got["sums"].view(np.uint64), want["sums"].view(np.uint64))


def key_union(n_rows, x_dom, y_dom, z_dom, seed, agg="sum"):
    """R(x,y) |x| S(y,z), SUM(R.v * S.w) GROUP BY z with the order x,y,z:
    the output z comes after the projected-away x and y, so the leaf's
    values are unioned by a GROUP BY.  Attributes x=0, y=1, z=2."""
    rng = synth.rng_for(seed)
    r = [rng.integers(0, x_dom, n_rows).astype(np.uint32), rng.integers(0, y_dom, n_rows).astype(np.uint32)]
    s = [rng.integers(0, y_dom, n_rows).astype(np.uint32), rng.integers(0, z_dom, n_rows).astype(np.uint32)]
    rv = rng.integers(-8, 9, n_rows) / 8.0
    sw = synth.uniform_pm1(rng, n_rows)
    return {"n_attrs": 3, "agg": agg, "out": [2],
            "atoms": [{"keys": r, "attrs": [0, 1], "annos": [rv], "anno": 0 if agg == "sum" else -1, "bag": True},
                      {"keys": s, "attrs": [1, 2], "annos": [sw], "anno": 0 if agg == "sum" else -1, "bag": True}]}


@pytest.mark.parametrize("z_dom,n_rows", [(64, 3000), (20_000, 3000), (1_000_000, 20_000), (5, 50_000)])
@pytest.mark.parametrize("impl", IMPLS)
def test_key_union(lh, z_dom, n_rows, impl):
    say("key union", z_dom, n_rows, impl)
    q = key_union(n_rows, 300, 200, z_dom, seed=z_dom + n_rows)
    want = oracle.join_aggregate(q)
    got = lh.run_query(q, attr_order=[0, 1, 2], policy="fixed", group_impl=impl)
    assert got["group_impl"] == ({"sort": "sort", "hash": "hash", "dense": "dense"}.get(impl) or got["group_impl"])
    assert_same(got, want)


def test_auto_choice_follows_density(lh):
    # a dense output range picks the dense array, a sparse one the hash table
    q = key_union(20_000, 300, 200, 1000, seed=3)
    assert lh.run_query(q, attr_order=[0, 1, 2], policy="fixed")["group_impl"] == "dense"
    q = key_union(20_000, 300, 200, 200_000_000, seed=3)
    got = lh.run_query(q, attr_order=[0, 1, 2], policy="fixed")
    assert got["group_impl"] == "hash"
    assert_same(got, oracle.join_aggregate(q))


@pytest.mark.parametrize("impl", IMPLS)
def test_wide_group_key(lh, impl):
    """GROUP BY five values (two keys and three meta columns), high
    cardinality: the wide-key case of section 5."""
    rng = synth.rng_for(21)
    n = 30_000
    a = [rng.integers(0, 50, n).astype(np.uint32), rng.integers(0, 400, n).astype(np.uint32)]
    b = [rng.integers(0, 400, n).astype(np.uint32), rng.integers(0, 30, n).astype(np.uint32)]
    q = {"n_attrs": 3, "agg": "sum", "out": [0, 2],
         "atoms": [{"keys": a, "attrs": [0, 1], "annos": [synth.uniform_pm1(rng, n)], "anno": 0, "bag": True,
                    "meta": [rng.integers(0, 7, n).astype(np.uint32), rng.integers(0, 1000, n).astype(np.uint32)]},
                   {"keys": b, "attrs": [1, 2], "annos": [rng.integers(-4, 5, n) / 4.0], "anno": 0, "bag": True,
                    "meta": [rng.integers(0, 3, n).astype(np.uint32)]}],
         "group": [(0, 0), (0, 1), (1, 0)]}
    want = oracle.join_aggregate(q)
    assert len(want["counts"]) > 10_000
    got = lh.run_query(q, group_impl=impl)
    assert_same(got, want)


def test_hash_table_grows(lh):
    # few distinct keys but many bag rows with distinct meta values: the
    # table sized from the leaf's work is too small and is grown
    n = 200_000
    rng = synth.rng_for(5)
    x = rng.integers(0, 10, n).astype(np.uint32)
    q = {"n_attrs": 1, "agg": "count", "out": [],
         "atoms": [{"keys": [x], "attrs": [0], "bag": True, "annos": [np.zeros(n)],
                    "meta": [rng.permutation(n).astype(np.uint32)]}],
         "group": [(0, 0)]}
    want = oracle.join_aggregate(q)
    assert len(want["counts"]) == n
    for impl in ["hash", "auto", "sort"]:
        assert_same(lh.run_query(q, group_impl=impl), want)


@pytest.mark.parametrize("impl", IMPLS)
def test_random_queries_every_group_impl(lh, impl):
    for seed in range(200, 320):
        q = queries.random_query(seed)
        try:
            want = oracle.join_aggregate(q)
        except oracle.OracleError:
            continue
        try:
            assert_same(lh.run_query(q, group_impl=impl), want)
        except AssertionError:
            say("random query seed", seed, impl)
            raise


def test_star_group_by_every_impl(lh):
    s = synth.star_schema(n_fact=400_000, dims=(20_000, 5_000, 1_000, 100), seed=7)
    q = queries.star(s)
    want = oracle.join_aggregate(q)
    for impl in IMPLS:
        got = lh.run_query(q, group_impl=impl)
        assert_same(got, want)


@pytest.mark.parametrize("impl", IMPLS)
def test_empty_key_union(lh, impl):
    q = key_union(100, 10, 10, 50, seed=9)
    q["atoms"][1]["keys"][0] = q["atoms"][1]["keys"][0] + 100   # no y in common
    want = oracle.join_aggregate(q)
    assert len(want["counts"]) == 0
    assert_same(lh.run_query(q, attr_order=[0, 1, 2], policy="fixed", group_impl=impl), want)


def test_dense_refuses_a_huge_key_space(lh):
    q = key_union(1000, 30, 20, 1 << 31, seed=4)
    with pytest.raises(lh.LHError):
        lh.run_query(q, attr_order=[0, 1, 2], policy="fixed", group_impl="dense")


def test_no_device_memory_leaks(lh):
    before = lh.live_allocations()
    q = key_union(5000, 100, 100, 100_000, seed=2)
    for impl in IMPLS:
        lh.run_query(q, attr_order=[0, 1, 2], policy="fixed", group_impl=impl)
    assert lh.live_allocations() == before


@pytest.mark.parametrize("impl", ["hash", "auto", "sort"])
def test_group_key_wider_than_64_bits(lh, impl):
    # x and z take values up to 2^30 and a meta column up to 2^20: an 80-bit
    # key, kept column by column in the table (claim, write, publish)
    rng = synth.rng_for(44)
    n = 20_000
    xs = rng.integers(0, 1 << 30, 300).astype(np.uint32)
    zs = rng.integers(0, 1 << 30, 500).astype(np.uint32)
    a = [xs[rng.integers(0, 300, n)], rng.integers(0, 200, n).astype(np.uint32)]
    b = [rng.integers(0, 200, n).astype(np.uint32), zs[rng.integers(0, 500, n)]]
    q = {"n_attrs": 3, "agg": "sum", "out": [0, 2],
         "atoms": [{"keys": a, "attrs": [0, 1], "annos": [synth.uniform_pm1(rng, n)], "anno": 0, "bag": True},
                   {"keys": b, "attrs": [1, 2], "annos": [rng.integers(-4, 5, n) / 4.0], "anno": 0, "bag": True,
                    "meta": [rng.integers(0, 1 << 20, n).astype(np.uint32)]}],
         "group": [(1, 0)]}
    want = oracle.join_aggregate(q)
    assert len(want["counts"]) > 100_000
    got = lh.run_query(q, attr_order=[0, 1, 2], policy="fixed", group_impl=impl)
    if impl != "sort":
        assert got["group_impl"] == "hash"
    assert_same(got, want)
