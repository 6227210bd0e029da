"""Parity at the benchmark's full size: triangle COUNT on the R-MAT graph
with 2^22 vertices and 2^26 sampled edges, in the configuration bench.py
times (plain layout, optimizer-chosen order).

The total has no closed form, so it is pinned through sampled outputs:
the GPU computes the count grouped by the smallest vertex a (one output row
per a), and
  * the grouped counts sum to the ungrouped count,
  * for sampled vertices with a moderate wedge count the oracle evaluates
    the same query restricted to a = a0,
  * for the hubs (wedge counts too large for the oracle's pairwise join)
    the count is taken from its definition with numpy: the number of edges
    (b, c) with both endpoints out-neighbours of a0.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import queries

pytestmark = pytest.mark.gpu

SCALE, SAMPLES_LOG2 = 22, 26


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def graph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi = synth.rmat_edges(SCALE, 1 << SAMPLES_LOG2, seed=2)
    key = np.unique(lo.astype(np.uint64) << np.uint64(32) | hi.astype(np.uint64))
    ulo = (key >> np.uint64(32)).astype(np.uint32)
    uhi = (key & np.uint64(0xffffffff)).astype(np.uint32)
    say("edges", len(ulo))
    return lo, hi, ulo, uhi


def _gpu(lh, lo_d, hi_d, grouped):
    t = lh.trie_build([lo_d, hi_d])
    p = lh.plan(3, [(t, [0, 1], -1), (t, [1, 2], -1), (t, [0, 2], -1)], agg="count",
                out=[0] if grouped else [])
    r = lh.join_aggregate([p])[0]
    res = r.to_host()
    r.free()
    p.free()
    t.free()
    return res


def test_fullsize_triangles_sampled(graph):
    from paper_1708_07859_amd import lh
    lo, hi, ulo, uhi = graph
    lo_d, hi_d = lh.to_device(lo), lh.to_device(hi)
    total = int(_gpu(lh, lo_d, hi_d, grouped=False)["counts"][0])
    g = _gpu(lh, lo_d, hi_d, grouped=True)
    say("triangles", total, "vertices with triangles", len(g["keys"]))
    assert int(g["counts"].sum()) == total
    per_a = dict(zip(g["keys"][:, 0].tolist(), g["counts"].tolist()))

    n = 1 << SCALE
    deg = np.bincount(ulo, minlength=n).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(deg)])
    # wedges through a0: sum of out-degrees of its out-neighbours
    wedge = np.zeros(n, np.int64)
    np.add.at(wedge, ulo, deg[uhi])

    def by_definition(a0):
        nb = uhi[start[a0]:start[a0 + 1]]
        mask = np.zeros(n, bool)
        mask[nb] = True
        return int(np.count_nonzero(mask[ulo] & mask[uhi]))

    hubs = list(np.argsort(-deg)[:3])
    for a0 in hubs:
        want = by_definition(int(a0))
        say("hub", int(a0), "out-degree", int(deg[a0]), "triangles", want)
        assert per_a.get(int(a0), 0) == want

    rng = synth.rng_for(77)
    moderate = np.nonzero((wedge > 1000) & (wedge < 3_000_000))[0]
    picks = list(rng.choice(moderate, 4, replace=False)) + list(rng.integers(0, n, 2))
    for a0 in picks:
        a0 = int(a0)
        nb = uhi[start[a0]:start[a0 + 1]]
        # rows of S whose b is not an out-neighbour of a0 cannot join R(a0, b):
        # drop them before the pairwise join (the result is unchanged)
        keep = np.isin(lo, nb)
        q = queries.triangle(lo, hi)
        q["atoms"][1] = dict(q["atoms"][1], keys=[lo[keep], hi[keep]])
        q["filters"] = [{"atom": 0, "kind": "eq_key", "col": 0, "eq": a0},
                        {"atom": 2, "kind": "eq_key", "col": 0, "eq": a0}]
        want = int(oracle.join_aggregate(q)["counts"][0])
        say("vertex", a0, "wedges", int(wedge[a0]), "triangles", want)
        assert per_a.get(a0, 0) == want


def test_fullsize_star_group_by():
    """The star-schema query at full size (60M fact rows, dimensions of
    2M / 500k / 100k / 10k rows, filters of 20% / 10% / 1%): GROUP BY a
    dimension attribute of SUM(price * (1 - discount)), checked against a
    direct denormalized scan (each fact row looks up its dimension rows by
    dense id) whose per-group sums are exact (math.fsum rounds once)."""
    import math

    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh
    say("generating the star schema (60M fact rows)")
    s = synth.star_schema(seed=3)
    q = queries.star(s, u_hi=0.20, m2=0, m3=0)
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
