"""The join that allocates no device memory (lh_join_aggregate_noalloc)
against lh_join_aggregate on the same plans: identical rows, counts and
sums, on two calls in a row whose second input is smaller (the static
scratch keeps the first call's contents), for a COUNT and a SUM plan."""
import sys

import numpy as np
import pytest

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


def tries_and_plan(lh, q, policy="plain"):
    tries, atoms = {}, []
    for a in q["atoms"]:
        ident = (tuple(id(k) for k in a["keys"]), tuple(id(x) for x in a.get("annos", [])), a.get("bag", False))
        if ident not in tries:
            tries[ident] = lh.trie_build(a["keys"], a.get("annos", []), a.get("meta", []), bag=a.get("bag", False))
        atoms.append((tries[ident], list(a["attrs"]), int(a.get("anno", -1))))
    p = lh.plan(q["n_attrs"], atoms, out=q.get("out", []), group=q.get("group", []), agg=q.get("agg", "count"),
                policy=policy)
    return list(tries.values()), p


def run_both(lh, q, cap):
    import torch
    tries, p = tries_and_plan(lh, q)
    r = lh.join_aggregate([p])[0]
    want = r.to_host()
    r.free()
    n_cols = len(q.get("out", [])) + len(q.get("group", []))
    keys = [torch.full((cap,), -1, dtype=torch.int32, device="cuda") for _ in range(n_cols)]
    counts = torch.zeros(cap, dtype=torch.int64, device="cuda")
    sums = torch.zeros(cap, dtype=torch.float64, device="cuda") if q.get("agg") == "sum" else None
    live = lh.live_allocations()
    n = lh.join_aggregate_noalloc(p, keys, counts, sums)
    torch.cuda.synchronize()
    assert lh.live_allocations() == live
    got_keys = np.stack([k[:n].cpu().numpy().view(np.uint32) for k in keys], axis=1) if n_cols else \
        np.zeros((n, 0), np.uint32)
    assert n == len(want["counts"])
    assert np.array_equal(got_keys, want["keys"])
    assert np.array_equal(counts[:n].cpu().numpy().view(np.uint64), want["counts"])
    if sums is not None:
        assert np.array_equal(sums[:n].cpu().numpy().view(np.uint64), want["sums"].view(np.uint64))
    p.free()
    for t in tries:
        t.free()
    return n


def test_noalloc_matches_join_aggregate_twice(lh):
    # triangle COUNT: the two-set leaf with its unit descriptors
    for scale in (13, 11):
        say("noalloc triangle, R-MAT scale", scale)
        lo, hi = synth.rmat_edges(scale, 16 << scale, seed=2)
        assert run_both(lh, queries.triangle(lo, hi), cap=1) == 1
    # SpGEMM SUM: a grouped result with exact sums, larger then smaller
    for n in (1024, 300):
        say("noalloc spgemm, n =", n)
        a = synth.sparse_matrix(n, 10, seed=1)
        b = synth.sparse_matrix(n, 10, seed=11)
        rows = run_both(lh, queries.spgemm(a, b), cap=n * 100)
        assert rows > 0


def test_noalloc_limits(lh):
    import torch
    a = synth.sparse_matrix(512, 10, seed=1)
    tries, p = tries_and_plan(lh, queries.spgemm(a, a))
    # output buffers too small: a clear overflow error
    keys = [torch.zeros(4, dtype=torch.int32, device="cuda") for _ in range(2)]
    with pytest.raises(lh.LHError) as ei:
        lh.join_aggregate_noalloc(p, keys, torch.zeros(4, dtype=torch.int64, device="cuda"),
                                  torch.zeros(4, dtype=torch.float64, device="cuda"))
    assert ei.value.status == 5
    p.free()
    for t in tries:
        t.free()
    # temporaries beyond the scratch: rejected when the allocation is asked
    # for, before any kernel would use it
    lo, hi = synth.rmat_edges(20, 16 << 20, seed=2)
    tries, p = tries_and_plan(lh, queries.triangle(lo, hi))
    with pytest.raises(lh.LHError) as ei:
        lh.join_aggregate_noalloc(p, [], torch.zeros(1, dtype=torch.int64, device="cuda"))
    assert ei.value.status == 5
    assert "scratch" in str(ei.value)
    p.free()
    for t in tries:
        t.free()
    # the scratch is whole again for the next call
    lo, hi = synth.rmat_edges(10, 16 << 10, seed=3)
    assert run_both(lh, queries.triangle(lo, hi), cap=1) == 1
