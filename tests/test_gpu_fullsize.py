"""Parity at the benchmark's full size: triangle COUNT on the R-MAT graph
with 2^22 vertices and 2^26 sampled edges, in both configurations bench.py
times (plain rules; the learned cost model with its committed weights,
learned layouts and the order it picks), and on the held-out R-MAT graph
with 2^24 vertices and 2^28 samples.

The total has no closed form, so it is pinned through sampled outputs:
the GPU computes the count grouped by the first attribute of the order
(one output row per vertex), and
  * the grouped counts sum to the ungrouped count, which is the same under
    every configuration,
  * for sampled vertices with a moderate wedge count the oracle evaluates
    the same query restricted to that vertex,
  * for the hubs (wedge counts too large for the oracle's pairwise join)
    the count is taken from its definition with numpy.
"""
import sys
from contextlib import contextmanager

import numpy as np
import pytest

import oracle
import synth
from tests import queries

pytestmark = pytest.mark.gpu

SCALE, SAMPLES_LOG2 = 22, 26
# the order the learned model picks for the triangle with the committed
# weights: c, b, a (the plan re-sorts the edges into (high, low) order)
LEARNED_TRIANGLE_ORDER = [2, 1, 0]
# and for the star: k0, k1, k2, k3
LEARNED_STAR_ORDER = [0, 1, 2, 3]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@contextmanager
def committed_model(lh):
    from paper_1708_07859_amd import learned as L
    lm, om, _ = L.load(L.DEFAULT_WEIGHTS)
    L.register(lm, om)
    try:
        yield
    finally:
        lh.use_model(lh.LH_MODEL_LAYOUT, None)
        lh.use_model(lh.LH_MODEL_ORDER, None)
        lm.free()
        om.free()


def unique_edges(lo, hi):
    key = np.unique(lo.astype(np.uint64) << np.uint64(32) | hi.astype(np.uint64))
    return (key >> np.uint64(32)).astype(np.uint32), (key & np.uint64(0xffffffff)).astype(np.uint32)


@pytest.fixture(scope="module")
def graph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi = synth.rmat_edges(SCALE, 1 << SAMPLES_LOG2, seed=2)
    ulo, uhi = unique_edges(lo, hi)
    say("edges", len(ulo))
    return lo, hi, ulo, uhi


def _gpu(lh, lo_d, hi_d, out, policy, layout, order=None):
    t = lh.trie_build([lo_d, hi_d], layout=layout)
    p = lh.plan(3, [(t, [0, 1], -1), (t, [1, 2], -1), (t, [0, 2], -1)], agg="count", out=out,
                attr_order=order, policy=policy)
    info = p.info()
    r = lh.join_aggregate([p])[0]
    res = r.to_host()
    res["order"] = info["attr_order"]
    r.free()
    p.free()
    t.free()
    return res


def check_triangles(lh, lo, hi, ulo, uhi, scale, policy, n_moderate=4, n_random=2):
    """Total, grouped and sampled checks of one configuration; returns the
    total.  The grouped run groups by the first attribute of the order the
    configuration uses (a for the plain rule; for the learned order, its own
    first attribute, with that order fixed and learned layouts)."""
    lo_d, hi_d = lh.to_device(lo), lh.to_device(hi)
    layout = "learned" if policy == "learned" else "plain"
    full = _gpu(lh, lo_d, hi_d, [], policy, layout)
    total = int(full["counts"][0])
    say(policy, "order", full["order"], "triangles", total)
    if policy == "learned":
        assert full["order"] == LEARNED_TRIANGLE_ORDER
        g = _gpu(lh, lo_d, hi_d, [full["order"][0]], "fixed", layout, order=full["order"])
    else:
        g = _gpu(lh, lo_d, hi_d, [0], policy, layout)
    first = g["order"][0]
    say("grouped by attribute", first, "rows", len(g["keys"]))
    assert int(g["counts"].sum()) == total
    per_v = dict(zip(g["keys"][:, 0].tolist(), g["counts"].tolist()))

    n = 1 << scale
    # grouped by a: triangles (v, b, c) with v < b < c take v's out-edges;
    # grouped by c: triangles (a, b, v) take v's in-edges
    own, other = (ulo, uhi) if first == 0 else (uhi, ulo)
    order = np.argsort(own, kind="stable")
    own_s, other_s = own[order], other[order]
    deg = np.bincount(own, minlength=n).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(deg)])
    # wedges through v: the degrees (same direction) of its neighbours
    wedge = np.bincount(own, weights=deg[other].astype(np.float64), minlength=n)

    def by_definition(v0):
        nb = other_s[start[v0]:start[v0 + 1]]
        mask = np.zeros(n, bool)
        mask[nb] = True
        return int(np.count_nonzero(mask[ulo] & mask[uhi]))

    for v0 in list(np.argsort(-deg)[:3]):
        want = by_definition(int(v0))
        say("hub", int(v0), "degree", int(deg[v0]), "triangles", want)
        assert per_v.get(int(v0), 0) == want

    rng = synth.rng_for(77 + scale)
    moderate = np.nonzero((wedge > 1000) & (wedge < 3_000_000))[0]
    picks = list(rng.choice(moderate, n_moderate, replace=False)) + list(rng.integers(0, n, n_random))
    for v0 in picks:
        v0 = int(v0)
        nb = other_s[start[v0]:start[v0 + 1]]
        mask = np.zeros(n, bool)
        mask[nb] = True
        q = queries.triangle(lo, hi)
        if first == 0:
            # rows of S whose b is not an out-neighbour of v0 cannot join R(v0, b)
            keep = mask[lo]
            q["atoms"][1] = dict(q["atoms"][1], keys=[lo[keep], hi[keep]])
            q["filters"] = [{"atom": 0, "kind": "eq_key", "col": 0, "eq": v0},
                            {"atom": 2, "kind": "eq_key", "col": 0, "eq": v0}]
        else:
            # triangles (a, b, v0): R(a, b) with both ends in-neighbours of v0
            keep = mask[lo] & mask[hi]
            q["atoms"][0] = dict(q["atoms"][0], keys=[lo[keep], hi[keep]])
            q["filters"] = [{"atom": 1, "kind": "eq_key", "col": 1, "eq": v0},
                            {"atom": 2, "kind": "eq_key", "col": 1, "eq": v0}]
        want = int(oracle.join_aggregate(q)["counts"][0])
        say("vertex", v0, "wedges", int(wedge[v0]), "triangles", want)
        assert per_v.get(v0, 0) == want
    return total


@pytest.mark.parametrize("policy", ["plain", "learned"])
def test_fullsize_triangles_sampled(graph, policy):
    from paper_1708_07859_amd import lh
    lo, hi, ulo, uhi = graph
    if policy == "learned":
        with committed_model(lh):
            check_triangles(lh, lo, hi, ulo, uhi, SCALE, policy)
    else:
        check_triangles(lh, lo, hi, ulo, uhi, SCALE, policy)


def test_heldout_rmat24_triangles():
    """The held-out graph of the learned model's evaluation (2^24 vertices,
    2^28 samples, seed 5): equal totals under both policies, each pinned by
    sampled vertices."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh
    say("generating R-MAT 24")
    lo, hi = synth.rmat_edges(24, 1 << 28, seed=5)
    ulo, uhi = unique_edges(lo, hi)
    say("edges", len(ulo))
    t_plain = check_triangles(lh, lo, hi, ulo, uhi, 24, "plain", n_moderate=2, n_random=1)
    with committed_model(lh):
        t_learn = check_triangles(lh, lo, hi, ulo, uhi, 24, "learned", n_moderate=2, n_random=1)
    assert t_plain == t_learn


@pytest.fixture(scope="module")
def star_schema():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("generating the star schema (60M fact rows)")
    return synth.star_schema(seed=3)


@pytest.mark.parametrize("policy", ["plain", "learned"])
def test_fullsize_star_group_by(star_schema, policy):
    """The star-schema query at full size (60M fact rows, dimensions of
    2M / 500k / 100k / 10k rows, filters of 20% / 10% / 1%): GROUP BY a
    dimension attribute of SUM(price * (1 - discount)), checked against a
    direct denormalized scan (each fact row looks up its dimension rows by
    dense id) whose per-group sums are exact (math.fsum rounds once); under
    the plain rules and under the learned model with its committed weights
    and learned layouts."""
    import math

    from paper_1708_07859_amd import lh
    s = star_schema
    q = queries.star(s, u_hi=0.20, m2=0, m3=0)
    if policy == "learned":
        with committed_model(lh):
            got = lh.run_query(q, policy="learned", layout="learned", return_plan_info=True)
        say("learned star order", got["plan"]["attr_order"])
        assert got["plan"]["attr_order"] == LEARNED_STAR_ORDER
    else:
        got = lh.run_query(q)
    k0, k1, k2, k3 = s["fact"]["k"]
    d = s["dims"]
    keep = (d[0]["u"][k0] < 0.20) & (d[2]["m"][k2] == 0) & (d[3]["m"][k3] == 0)
    g = d[1]["g"][k1][keep]
    ann = s["fact"]["ann"][keep]
    groups = np.unique(g)
    say("surviving fact rows", int(keep.sum()), "groups", len(groups))
    assert got["keys"][:, 0].tolist() == groups.tolist()
    order = np.argsort(g, kind="stable")
    bounds = np.searchsorted(g[order], groups, side="left").tolist() + [len(g)]
    for i, gv in enumerate(groups):
        sel = ann[order[bounds[i]:bounds[i + 1]]]
        assert got["counts"][i] == len(sel)
        assert got["sums"][i] == math.fsum(sel.tolist()), (int(gv), got["sums"][i], math.fsum(sel.tolist()))


def test_fullsize_batch(tmp_path, monkeypatch):
    """The 512 SpMV / SpGEMM instances of the batched benchmark (n
    log-uniform in [1k, 64k], Zipf(1.1) degrees with mean 16): the batched,
    graph-captured run gives every instance bit for bit the result of its
    own single-plan run, on two replays; the smallest instances also match
    the oracle."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh
    from tests.test_gpu_batch import make_plans, same
    monkeypatch.setenv("LH_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    insts = synth.batched_instances(count=512)
    keep, plans, qs = make_plans(lh, insts)
    say("instances", len(plans), "rows", sum(i["n"] for i in insts))
    import hashlib
    digests = []
    for rnd in range(2):                       # the second round replays the captured graph
        rs = lh.join_aggregate(plans)
        say("batched round", rnd, "output rows", sum(r.n_rows for r in rs))
        for i, (p, r) in enumerate(zip(plans, rs)):
            got = r.to_host()
            r.free()
            d = hashlib.sha256(got["keys"].tobytes() + got["counts"].tobytes() + got["sums"].tobytes()).hexdigest()
            if rnd == 0:
                alone = lh.join_aggregate([p])[0]
                same(got, alone.to_host())
                alone.free()
                digests.append(d)
            else:
                assert d == digests[i]
    smallest = np.argsort([i["n"] for i in insts])[:3]
    for i in smallest:
        got = lh.join_aggregate([plans[i]])[0]
        same(got.to_host(), oracle.join_aggregate(qs[i]))
        got.free()
    for p in plans:
        p.free()
    for ts in keep:
        for t in ts:
            t.free()
