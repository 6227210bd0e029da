"""Multi-node plans on the GPU: queries run under generalized hypertree
decompositions (sections 2.3 and 3.2) against the oracle.  Keys and counts
must be identical whatever the decomposition.  A child node hands each
group's sum to its parent as exact parts, so with at most two annotated
atoms in the query every node sums exact products and the result is
bit-identical to the oracle's and flagged exact; with more annotated atoms
the per-node products are rounded differently from the single plan's and
sums agree to 1e-9 relative."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import queries
from tests.test_ghd import rooted_trees, set_partitions

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


def n_annotated(q):
    return sum(1 for a in q["atoms"] if a.get("anno", -1) >= 0) if q.get("agg") == "sum" else 0


def assert_close(got, want, exact_sums=None, q=None):
    assert got["keys"].shape == want["keys"].shape, (got["keys"].shape, want["keys"].shape)
    assert np.array_equal(got["keys"], want["keys"])
    assert np.array_equal(got["counts"], want["counts"])
    assert got["n_join"] == want["n_join"]
    if want["sums"] is not None:
        g, w = got["sums"], want["sums"]
        if exact_sums is None:
            exact_sums = q is not None and n_annotated(q) <= 2
            if exact_sums:
                assert got["exact"] == 1
        if exact_sums:
            assert np.array_equal(g.view(np.uint64), w.view(np.uint64)), (g, w)
        else:
            assert np.all(np.abs(g - w) <= 1e-9 * np.abs(w) + 1e-12), (g, w)


def query_masks(q):
    edges = [sum(1 << v for v in a["attrs"]) for a in q["atoms"]]
    sel = sum(1 << f["atom"] for f in q.get("filters", []))
    root = sum(1 << ga for ga, _ in q.get("group", []))
    out = sum(1 << v for v in q.get("out", []))
    return edges, sel, root, out


def all_decompositions(q, limit=None, max_nodes=4):
    """Every decomposition of q's hypergraph (each edge in one node, running
    intersection, children sharing an attribute with their parent, outputs
    and GROUP BY relations in the root), parents numbered before children."""
    edges, sel, root_edges, out = query_masks(q)
    n_attrs = q["n_attrs"]
    found = []
    for part in set_partitions(list(range(len(edges)))):
        if len(part) > max_nodes:
            continue
        bags = [sum(1 << e for e in p) for p in part]
        chis = []
        for p in part:
            c = 0
            for e in p:
                c |= edges[e]
            chis.append(c)
        k = len(bags)
        for parent in rooted_trees(k):
            r = parent.index(-1)
            if (bags[r] & root_edges) != root_edges or (chis[r] & out) != out:
                continue
            if any(parent[t] >= 0 and not (chis[t] & chis[parent[t]]) for t in range(k)):
                continue
            ok = True
            for v in range(n_attrs):
                holders = [t for t in range(k) if chis[t] >> v & 1]
                tops = [t for t in holders if parent[t] < 0 or not (chis[parent[t]] >> v & 1)]
                if holders and len(tops) != 1:
                    ok = False
                    break
            if not ok:
                continue
            order = [r]
            for h in order:
                order += [t for t in range(k) if parent[t] == h]
            pos = {t: i for i, t in enumerate(order)}
            found.append({"edges": [bags[t] for t in order],
                          "parent": [-1 if parent[t] < 0 else pos[parent[t]] for t in order],
                          "pushed": [0] * k})
            if limit and len(found) >= limit:
                return found
    return found


def add_selection_nodes(d, q):
    """The same decomposition with every filtered edge pushed below its node."""
    d = {k: list(v) for k, v in d.items()}
    for f in sorted({f["atom"] for f in q.get("filters", [])}):
        t = next(i for i, b in enumerate(d["edges"]) if b >> f & 1 and not d["pushed"][i])
        d["edges"].append(1 << f)
        d["parent"].append(t)
        d["pushed"].append(1)
    return d


# --------------------------------------------------------------- Q5 shape

@pytest.fixture(scope="module")
def q5s():
    return synth.q5_schema(0.02, seed=5)


@pytest.mark.parametrize("agg", ["sum", "count"])
def test_q5_shape_chosen_decomposition(lh, q5s, agg):
    say("q5 shape", agg)
    q = queries.q5(q5s, agg=agg)
    want = oracle.join_aggregate(q)
    assert len(want["counts"]) == 5
    got = lh.run_query(q, ghd=None)
    assert_close(got, want, q=q)
    # the single plan gives the same keys and counts, and exact sums
    assert_close(lh.run_query(q), want, exact_sums=True)


def test_q5_shape_every_decomposition(lh, q5s):
    q = queries.q5(q5s)
    want = oracle.join_aggregate(q)
    decs = all_decompositions(q)
    say("q5 decompositions", len(decs))
    assert len(decs) > 10
    for i, d in enumerate(decs[:: max(1, len(decs) // 12)]):
        say("q5 decomposition", d)
        assert_close(lh.run_query(q, ghd=d), want, q=q)
        assert_close(lh.run_query(q, ghd=add_selection_nodes(d, q)), want, q=q)


def test_q5_shape_choice(lh, q5s):
    q = queries.q5(q5s)
    tries = [lh.trie_build(a["keys"], a.get("annos", []), a.get("meta", []), bag=a.get("bag", False))
             for a in q["atoms"]]
    atoms = [(t, a["attrs"], a.get("anno", -1)) for t, a in zip(tries, q["atoms"])]
    g = lh.ghd_for_query(q["n_attrs"], atoms, out=q["out"], agg="sum", filters=q["filters"])
    bags = sorted(g["edges"][t] for t in range(g["n_nodes"]) if not g["pushed"][t])
    assert bags == sorted([0b001111, 0b110000]) and g["fhw"] == pytest.approx(2.0)
    for t in tries:
        t.free()


def test_q5_shape_empty_child(lh, q5s):
    # no order in the date window: the cycle node hands up nothing
    q = queries.q5(q5s, date_lo=5000, date_hi=6000)
    want = oracle.join_aggregate(q)
    assert len(want["counts"]) == 0
    assert_close(lh.run_query(q, ghd=None), want, q=q)


def test_q5_shape_ungrouped(lh, q5s):
    q = queries.q5(q5s)
    q["out"] = []
    want = oracle.join_aggregate(q)
    assert_close(lh.run_query(q, ghd=None), want, q=q)


# ------------------------------------------------------ cycles and random

def test_five_cycle_count(lh):
    # C5 over a random graph: width 2 under two nodes, 5/2 as one node
    lo, hi = synth.gnp(60, 0.15, seed=7)
    e = {"keys": [np.concatenate([lo, hi]), np.concatenate([hi, lo])], "bag": False}
    q = {"n_attrs": 5, "agg": "count", "out": [],
         "atoms": [dict(e, attrs=[i, (i + 1) % 5]) for i in range(5)]}
    want = oracle.join_aggregate(q)
    assert want["counts"][0] > 0
    got = lh.run_query(q, ghd=None)
    assert_close(got, want)


def test_two_triangles_sum_grouped(lh):
    rng = synth.rng_for(11)
    atoms = []
    for a, b in [(0, 1), (1, 2), (0, 2), (0, 3), (3, 4), (0, 4)]:
        n = 400
        keys = [rng.integers(0, 12, n).astype(np.uint32), rng.integers(0, 12, n).astype(np.uint32)]
        atoms.append({"keys": keys, "attrs": [a, b], "bag": True, "annos": [rng.integers(-8, 9, n) / 8.0],
                      "anno": 0 if a == 3 or b == 2 else -1})
    q = {"n_attrs": 5, "agg": "sum", "out": [0], "atoms": atoms}
    want = oracle.join_aggregate(q)
    # dyadic values with small sums: every node's sum is exact
    assert_close(lh.run_query(q, ghd=None), want, exact_sums=True)
    for d in all_decompositions(q, limit=40)[::5]:
        assert_close(lh.run_query(q, ghd=d), want, exact_sums=True)


@pytest.mark.parametrize("block", range(4))
def test_random_queries_under_decompositions(lh, block):
    multi = 0
    for seed in range(5000 + block * 30, 5000 + block * 30 + 30):
        q = queries.random_query(seed, max_atoms=5, max_attrs=5, domain=5, max_rows=9)
        try:
            want = oracle.join_aggregate(q)
        except oracle.OracleError:
            continue
        decs = all_decompositions(q, limit=200, max_nodes=3)
        try:
            got = lh.run_query(q, ghd=None)
            assert_close(got, want, q=q)
            for d in decs[:: max(1, len(decs) // 4)]:
                multi += len(d["edges"]) > 1
                assert_close(lh.run_query(q, ghd=d), want, q=q)
                if q.get("filters"):
                    assert_close(lh.run_query(q, ghd=add_selection_nodes(d, q)), want, q=q)
        except AssertionError:
            say("random query seed", seed)
            raise
    assert multi > 0


# ------------------------------------------------------------------ errors

def test_invalid_decompositions_rejected(lh, q5s):
    q = queries.q5(q5s)
    bad = [
        {"edges": [0b001111, 0b110000, 0b000001], "parent": [-1, 0, 0], "pushed": [0, 0, 0]},  # edge twice
        {"edges": [0b001111], "parent": [-1], "pushed": [0]},                                   # edge in no node
        {"edges": [0b110000, 0b001111], "parent": [-1, -1], "pushed": [0, 0]},                  # two roots
        {"edges": [0b110001, 0b000010, 0b001100], "parent": [-1, 0, 0], "pushed": [0, 0, 0]},   # o in two subtrees
        {"edges": [0b100000, 0b011111], "parent": [-1, 0], "pushed": [0, 0]},                   # output not in root
        {"edges": [0b001111, 0b110000, 0b000100], "parent": [-1, 1, 0],
         "pushed": [0, 0, 1]},                                                                  # parent after child
        {"edges": [0b001111, 0b110000, 0b000100], "parent": [-1, 0, 0], "pushed": [0, 0, 1]},  # pushed unfiltered
    ]
    before = lh.live_allocations()
    for d in bad:
        with pytest.raises(lh.LHError):
            lh.run_query(q, ghd=d)
    assert lh.live_allocations() == before


def test_no_device_memory_leaks(lh, q5s):
    before = lh.live_allocations()
    q = queries.q5(q5s)
    for _ in range(2):
        lh.run_query(q, ghd=None)
    assert lh.live_allocations() == before
