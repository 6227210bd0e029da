"""Batched execution: many SpMV / SpGEMM instances in one persistent,
graph-captured launch give, instance by instance, exactly the result of
running each plan alone (and of the oracle)."""
import sys

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


def make_plans(lh, insts):
    keep, plans, qs = [], [], []
    for inst in insts:
        a = (inst["rows"], inst["cols"], inst["vals"])
        q = queries.spmv(a, inst["x"]) if inst["kind"] == "spmv" else queries.spgemm(a, a)
        tries = []
        atoms = []
        for at in q["atoms"]:
            t = lh.trie_build(at["keys"], at.get("annos", []), bag=True)
            tries.append(t)
            atoms.append((t, at["attrs"], at["anno"]))
        p = lh.plan(q["n_attrs"], atoms, out=q["out"], agg="sum")
        keep.append(tries)
        plans.append(p)
        qs.append(q)
    return keep, plans, qs


def same(a, b):
    assert np.array_equal(a["keys"], b["keys"])
    assert np.array_equal(a["counts"], b["counts"])
    assert np.array_equal(a["sums"].view(np.uint64), b["sums"].view(np.uint64))
    assert a["n_join"] == b["n_join"]


@pytest.mark.parametrize("seed", [4, 5])
def test_batched_equals_sequential_and_oracle(lh, seed, tmp_path, monkeypatch):
    monkeypatch.setenv("LH_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    insts = synth.batched_instances(count=24, n_lo=64, n_hi=3000, seed=seed)
    keep, plans, qs = make_plans(lh, insts)
    say("instances", len(plans), "rows", sum(i["n"] for i in insts))
    for rnd in range(2):                       # second round replays the graph
        batched = [r.to_host() for r in lh.join_aggregate(plans)]
        for i, p in enumerate(plans):
            alone = lh.join_aggregate([p])[0].to_host()
            same(batched[i], alone)
    for i in range(0, len(plans), 5):
        want = oracle.join_aggregate(qs[i])
        got = batched[i]
        assert np.array_equal(got["keys"], want["keys"])
        assert np.array_equal(got["counts"], want["counts"])
        assert np.array_equal(got["sums"].view(np.uint64), want["sums"].view(np.uint64))


def test_batch_cache_follows_plans(lh, tmp_path, monkeypatch):
    monkeypatch.setenv("LH_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    insts = synth.batched_instances(count=6, n_lo=64, n_hi=500, seed=9)
    keep, plans, qs = make_plans(lh, insts)
    first = [r.to_host() for r in lh.join_aggregate(plans)]
    # free the plans, build different ones (addresses may be reused)
    for p in plans:
        p.free()
    insts2 = synth.batched_instances(count=6, n_lo=64, n_hi=500, seed=10)
    keep2, plans2, qs2 = make_plans(lh, insts2)
    second = [r.to_host() for r in lh.join_aggregate(plans2)]
    for i, q in enumerate(qs2):
        want = oracle.join_aggregate(q)
        assert np.array_equal(second[i]["keys"], want["keys"])
        assert np.array_equal(second[i]["sums"].view(np.uint64), want["sums"].view(np.uint64))
    assert len(first) == 6


def test_mixed_batch_falls_back(lh):
    # a triangle plan is not a row-union instance: the batch runs plan by plan
    lo, hi = synth.complete_graph(12)
    t = lh.trie_build([lo, hi])
    p1 = lh.plan(3, [(t, [0, 1], -1), (t, [1, 2], -1), (t, [0, 2], -1)], agg="count")
    a = synth.sparse_matrix(50, 4, seed=1)
    q = queries.spgemm(a, a)
    ta = lh.trie_build(q["atoms"][0]["keys"], q["atoms"][0]["annos"], bag=True)
    p2 = lh.plan(3, [(ta, [0, 1], 0), (ta, [1, 2], 0)], out=[0, 2], agg="sum")
    r = lh.join_aggregate([p1, p2])
    assert int(r[0].to_host()["counts"][0]) == 220
    same(r[1].to_host(), lh.join_aggregate([p2])[0].to_host())


def test_batch_wide_k_range(lh, tmp_path, monkeypatch):
    """SpGEMM instances whose k range exceeds one bitmap window of the heavy
    path (n = 100,000 > 65,536), with heavy and dense rows, next to small
    instances: the batched result equals each plan run alone, and the
    oracle on the small ones."""
    monkeypatch.setenv("LH_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    rng = synth.rng_for(31)
    insts = synth.batched_instances(count=6, n_lo=64, n_hi=500, seed=12)
    r, c, v = synth.zipf_degree_matrix(100_000, 1.1, 4, rng)
    insts.append({"kind": "spgemm", "n": 100_000, "rows": r, "cols": c, "vals": v})
    keep, plans, qs = make_plans(lh, insts)
    batched = [x.to_host() for x in lh.join_aggregate(plans)]
    for i, p in enumerate(plans):
        same(batched[i], lh.join_aggregate([p])[0].to_host())
    for i in range(6):
        want = oracle.join_aggregate(qs[i])
        assert np.array_equal(batched[i]["keys"], want["keys"])
        assert np.array_equal(batched[i]["sums"].view(np.uint64), want["sums"].view(np.uint64))
