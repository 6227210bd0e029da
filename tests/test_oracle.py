"""Pins for the oracle: closed forms, library routines, brute force and the
exact-sum definition.  CPU only."""
import math
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle
import synth
from tests import queries
from tests.brute import brute


# --------------------------------------------------------------------------
# exact summation
# --------------------------------------------------------------------------

def _fraction_dot(a, b=None):
    if b is None:
        return float(sum(Fraction(x) for x in a))
    return float(sum(Fraction(x) * Fraction(y) for x, y in zip(a, b)))


@pytest.mark.parametrize("seed", range(6))
def test_exact_dot_matches_fraction(seed):
    rng = synth.rng_for(100 + seed)
    n = 300
    a = synth.uniform_pm1(rng, n) * 2.0 ** rng.integers(-40, 40, n)
    b = synth.uniform_pm1(rng, n) * 2.0 ** rng.integers(-40, 40, n)
    # heavy cancellation: append the negated products of a prefix
    a2 = np.concatenate([a, -a[:100], [1e30, -1e30, 3.0]])
    b2 = np.concatenate([b, b[:100], [1.0, 1.0, 2.0 ** -60]])
    assert oracle.exact_dot(a2, b2) == _fraction_dot(a2, b2)
    assert oracle.exact_dot(a2) == _fraction_dot(a2)
    perm = rng.permutation(len(a2))
    assert oracle.exact_dot(a2[perm], b2[perm]) == oracle.exact_dot(a2, b2)


def test_exact_dot_ties_round_to_even():
    # 1 + 2^-53 is a tie between 1 and 1+2^-52: rounds to even (1.0)
    assert oracle.exact_dot([1.0, 2.0 ** -53]) == 1.0
    # 1 + 2^-52 + 2^-53 ties to 1 + 2^-51 (even mantissa)
    assert oracle.exact_dot([1.0, 2.0 ** -52, 2.0 ** -53]) == 1.0 + 2.0 ** -51
    # a sticky bit below the tie breaks it upward
    assert oracle.exact_dot([1.0, 2.0 ** -53, 2.0 ** -200]) == 1.0 + 2.0 ** -52
    assert oracle.exact_dot([-1.0, -(2.0 ** -53), -(2.0 ** -200)]) == -(1.0 + 2.0 ** -52)
    assert oracle.exact_dot([]) == 0.0
    assert oracle.exact_dot([0.1, -0.1]) == 0.0


def test_exact_dot_out_of_window_raises():
    with pytest.raises(oracle.OracleError):
        oracle.exact_dot([2.0 ** -300])
    with pytest.raises(oracle.OracleError):
        oracle.exact_dot([np.nan])


# --------------------------------------------------------------------------
# triangle counting: closed forms and a textbook identity
# --------------------------------------------------------------------------

def _tri(lo, hi):
    return int(oracle.join_aggregate(queries.triangle(lo, hi))["counts"][0])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 17, 40])
def test_triangle_complete_graph(n):
    lo, hi = synth.complete_graph(n)
    assert _tri(lo, hi) == comb(n, 3)


@pytest.mark.parametrize("abc", [(1, 1, 1), (2, 3, 4), (5, 1, 7)])
def test_triangle_complete_tripartite(abc):
    lo, hi = synth.complete_tripartite(*abc)
    assert _tri(lo, hi) == abc[0] * abc[1] * abc[2]


@pytest.mark.parametrize("n", [4, 5, 11])
def test_triangle_wheel_cycle_bipartite(n):
    assert _tri(*synth.wheel(n)) == n
    assert _tri(*synth.cycle(n)) == 0
    assert _tri(*synth.random_bipartite(n, n + 3, 0.5, seed=n)) == 0


def _trace_a3_over_6(lo, hi, n):
    a = np.zeros((n, n), dtype=np.int64)
    a[lo, hi] = 1
    a[hi, lo] = 1
    return int(np.trace(a @ a @ a)) // 6


@pytest.mark.parametrize("seed", [0, 1])
def test_triangle_trace_identity_gnp(seed):
    lo, hi = synth.gnp(200, 0.08, seed)
    assert _tri(lo, hi) == _trace_a3_over_6(lo, hi, 200)


def test_triangle_trace_identity_small_rmat_with_duplicates():
    lo, hi = synth.rmat_edges(10, 16 << 10, seed=7)
    # duplicates are in the input: a set relation removes them
    assert len(set(zip(lo.tolist(), hi.tolist()))) < len(lo)
    assert _tri(lo, hi) == _trace_a3_over_6(lo, hi, 1 << 10)


def test_triangle_brute_force_tiny():
    lo, hi = synth.gnp(24, 0.3, 3)
    n = 24
    adj = set(zip(lo.tolist(), hi.tolist()))
    want = sum(1 for a in range(n) for b in range(a + 1, n) for c in range(b + 1, n)
               if (a, b) in adj and (b, c) in adj and (a, c) in adj)
    assert _tri(lo, hi) == want


# --------------------------------------------------------------------------
# sparse matrix products against the definition of the matrix product
# --------------------------------------------------------------------------

def _exact_dense_product(a, b, n):
    """C = A B with every value scaled to an integer on the 2^-53 grid."""
    A = [[0] * n for _ in range(n)]
    B = [[0] * n for _ in range(n)]
    for r, c, v in zip(*a):
        A[int(r)][int(c)] = int(v * 2 ** 53)
    for r, c, v in zip(*b):
        B[int(r)][int(c)] = int(v * 2 ** 53)
    out = {}
    for i in range(n):
        for j in range(n):
            if A[i][j] == 0:
                continue
            for k in range(n):
                if B[j][k] != 0:
                    out[(i, k)] = out.get((i, k), 0) + A[i][j] * B[j][k]
    return out


def test_spgemm_exact_small():
    n = 24
    a = synth.sparse_matrix(n, 5, seed=1)
    b = synth.sparse_matrix(n, 5, seed=11)
    res = oracle.join_aggregate(queries.spgemm(a, b))
    want = _exact_dense_product(a, b, n)
    keys = [tuple(map(int, k)) for k in res["keys"]]
    assert keys == sorted(want)
    for k, s in zip(keys, res["sums"]):
        assert s == float(Fraction(want[k], 2 ** 106))


def test_spgemm_dense_product_full_size_shape():
    """n = 4096, 10 nonzeros per row: structure equals the boolean product,
    values equal numpy's dense A @ B within a scale-aware bound, and the
    checksum 1'C1 = (1'A)(B1) holds exactly."""
    n = 4096
    a = synth.sparse_matrix(n, 10, seed=1)
    b = synth.sparse_matrix(n, 10, seed=11)
    res = oracle.join_aggregate(queries.spgemm(a, b))
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    A[a[0], a[1]] = a[2]
    B[b[0], b[1]] = b[2]
    structure = (A != 0).astype(np.float32) @ (B != 0).astype(np.float32)
    nz = np.nonzero(structure)
    assert res["keys"].shape[0] == len(nz[0])
    assert np.array_equal(res["keys"][:, 0], nz[0]) and np.array_equal(res["keys"][:, 1], nz[1])
    C = A @ B
    absC = np.abs(A) @ np.abs(B)
    got = res["sums"]
    want = C[nz]
    assert np.all(np.abs(got - want) <= 1e-12 * absC[nz] + 1e-300)
    # exact checksum with integers on the 2^-106 grid
    colsum_a = {}
    for c, v in zip(a[1].tolist(), a[2].tolist()):
        colsum_a[c] = colsum_a.get(c, 0) + int(v * 2 ** 53)
    rowsum_b = {}
    for r, v in zip(b[0].tolist(), b[2].tolist()):
        rowsum_b[r] = rowsum_b.get(r, 0) + int(v * 2 ** 53)
    exact_total = sum(colsum_a.get(j, 0) * rowsum_b.get(j, 0) for j in range(n))
    q = queries.spgemm(a, b)
    q["out"] = []                            # ungrouped: one exactly rounded total
    total = oracle.join_aggregate(q)["sums"][0]
    assert total == float(Fraction(exact_total, 2 ** 106))


def test_spmv_dense():
    n = 300
    rng = synth.rng_for(9)
    a = synth.sparse_matrix(n, 7, seed=5)
    x = synth.uniform_pm1(rng, n)
    res = oracle.join_aggregate(queries.spmv(a, x))
    A = np.zeros((n, n))
    A[a[0], a[1]] = a[2]
    rows = sorted(set(a[0].tolist()))
    assert res["keys"][:, 0].tolist() == rows
    for (i,), s in zip(res["keys"], res["sums"]):
        want = sum(Fraction(A[i, j]) * Fraction(x[j]) for j in np.nonzero(A[i])[0])
        assert s == float(want)


# --------------------------------------------------------------------------
# star schema against a denormalized scan
# --------------------------------------------------------------------------

def test_star_denormalized_scan():
    s = synth.star_schema(n_fact=20000, dims=(2000, 500, 100, 40), seed=3)
    res = oracle.join_aggregate(queries.star(s, u_hi=0.5, m2=0, m3=1))
    k0, k1, k2, k3 = s["fact"]["k"]
    d = s["dims"]
    keep = (d[0]["u"][k0] < 0.5) & (d[2]["m"][k2] == 0) & (d[3]["m"][k3] == 1)
    g = d[1]["g"][k1][keep]
    ann = s["fact"]["ann"][keep]
    groups = sorted(set(g.tolist()))
    assert res["keys"][:, 0].tolist() == groups
    for gv, cnt, sm in zip(res["keys"][:, 0], res["counts"], res["sums"]):
        sel = ann[g == gv]
        assert cnt == len(sel)
        assert sm == math.fsum(sel.tolist())


def test_star_no_filter_single_group_and_empty():
    s = synth.star_schema(n_fact=5000, dims=(100, 50, 20, 10), seed=8)
    s["dims"][1]["g"][:] = 7
    q = queries.star(s, u_hi=2.0, m2=0, m3=0)
    q["filters"] = []
    res = oracle.join_aggregate(q)
    assert res["keys"].tolist() == [[7]]
    assert res["sums"][0] == math.fsum(s["fact"]["ann"].tolist())
    q = queries.star(s, u_hi=-1.0)
    res = oracle.join_aggregate(q)
    assert res["keys"].shape == (0, 1)


# --------------------------------------------------------------------------
# brute force on random tiny queries
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(150))
def test_random_queries_match_brute_force(seed):
    q = queries.random_query(seed)
    got = oracle.join_aggregate(q)
    want = brute(q)
    assert [tuple(map(int, k)) for k in got["keys"]] == want["keys"]
    assert got["counts"].tolist() == want["counts"]
    assert got["n_join"] == want["n_join"]
    if want["sums"] is not None:
        assert got["sums"].tolist() == want["sums"]


def test_ungrouped_empty_is_one_zero_row():
    lo = np.zeros(0, np.uint32)
    q = queries.triangle(lo, lo)
    res = oracle.join_aggregate(q)
    assert res["counts"].tolist() == [0] and res["keys"].shape == (1, 0)


def test_invalid_queries_rejected():
    lo, hi = synth.complete_graph(4)
    bad = queries.triangle(lo, hi)
    bad["atoms"][0]["attrs"] = [0, 0]
    with pytest.raises(oracle.OracleError):
        oracle.join_aggregate(bad)
    bad = queries.triangle(lo, hi)
    bad["agg"] = "sum"                       # SUM without an annotated atom
    with pytest.raises(oracle.OracleError):
        oracle.join_aggregate(bad)
    bad = queries.triangle(lo, hi)
    bad["n_attrs"] = 4                       # attribute 3 in no atom
    with pytest.raises(oracle.OracleError):
        oracle.join_aggregate(bad)


def test_too_many_group_columns_rejected():
    # the aggregation key holds at most 128 columns (outputs + GROUP BY)
    n = 5
    rel = {"keys": [np.arange(n, dtype=np.uint32)], "attrs": [0], "bag": True, "anno": -1,
           "meta": [np.zeros(n, np.uint32)]}
    q = {"n_attrs": 1, "agg": "count", "out": [0], "atoms": [rel], "group": [(0, 0)] * 127}
    res = oracle.join_aggregate(q)                   # 1 + 127 columns: accepted
    assert res["keys"].shape == (n, 128)
    q["group"] = [(0, 0)] * 128                      # 129 columns
    with pytest.raises(oracle.OracleError) as ei:
        oracle.join_aggregate(q)
    assert ei.value.code == oracle.ORC_E_INVALID


@pytest.mark.parametrize("seed", range(40))
def test_thread_count_does_not_change_results(seed):
    # thread-local tables merged exactly: every thread count gives the same bits
    q = queries.random_query(seed, max_rows=40, domain=5)
    outs = []
    for t in (1, 3, 8):
        oracle.set_threads(t)
        try:
            outs.append(oracle.join_aggregate(q))
        finally:
            oracle.set_threads(0)
    for o in outs[1:]:
        assert np.array_equal(o["keys"], outs[0]["keys"])
        assert np.array_equal(o["counts"], outs[0]["counts"])
        assert o["n_join"] == outs[0]["n_join"]
        if o["sums"] is not None:
            assert np.array_equal(o["sums"].view(np.uint64), outs[0]["sums"].view(np.uint64))
