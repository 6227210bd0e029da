"""Host-side checks of the C ABI: the library loads and exports every entry
point include/lh.h declares, validation paths fail cleanly without touching
a GPU, and the section 4 cost estimate reproduces the paper's worked
examples.  CPU only."""
import ctypes as C
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lh.h")


@pytest.fixture(scope="module")
def lh():
    from paper_1708_07859_amd import lh as binding
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lh_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("lh_trie_build", "lh_plan", "lh_join_aggregate", "lh_free"):
        assert n in names


def test_library_exports_every_declared_symbol(lh):
    for name in declared_functions():
        assert hasattr(lh.lib, name), name
        assert name in lh.SIGNATURES, name


def test_null_arguments_are_invalid_without_a_gpu(lh):
    out = C.c_void_p(123)
    assert lh.lib.lh_trie_build(None, None, C.byref(out)) == lh.LH_ERR_INVALID
    assert out.value is None
    assert lh.lib.lh_last_error()
    assert lh.lib.lh_plan(None, None, C.byref(out)) == lh.LH_ERR_INVALID
    assert lh.lib.lh_join_aggregate(None, 0, None, None) == lh.LH_ERR_INVALID
    lh.lib.lh_free(None)          # no-op
    lh.lib.lh_free(C.c_void_p(0x1234))  # unknown handle: ignored


def test_relation_validation(lh):
    d = lh.RelationDesc()
    out = C.c_void_p()
    d.n_keys = 0
    assert lh.lib.lh_trie_build(C.byref(d), None, C.byref(out)) == lh.LH_ERR_INVALID
    d.n_keys = 9
    assert lh.lib.lh_trie_build(C.byref(d), None, C.byref(out)) == lh.LH_ERR_INVALID
    d.n_keys = 2
    ptrs = (C.c_void_p * 2)(0, 0)
    d.keys = C.cast(ptrs, C.POINTER(C.c_void_p))
    d.n_rows = 0
    lo = (C.c_uint32 * 2)(0, 0)          # not a permutation
    d.level_order = C.cast(lo, C.POINTER(C.c_uint32))
    assert lh.lib.lh_trie_build(C.byref(d), None, C.byref(out)) == lh.LH_ERR_INVALID
    d.level_order = None
    d.n_annos = 1                        # a set relation carries no annotation
    aptr = (C.c_void_p * 1)(0)
    d.annos = C.cast(aptr, C.POINTER(C.c_void_p))
    assert lh.lib.lh_trie_build(C.byref(d), None, C.byref(out)) == lh.LH_ERR_INVALID
    d.n_annos = 0
    d.n_rows = 1 << 32                   # too many rows for uint32 positions
    assert lh.lib.lh_trie_build(C.byref(d), None, C.byref(out)) == lh.LH_ERR_OVERFLOW


def test_plan_rejects_foreign_trie(lh):
    q = lh.Query()
    q.n_attrs = 1
    q.n_atoms = 1
    atoms = (lh.Atom * 1)()
    atoms[0].trie = 0xdead
    q.atoms = atoms
    out = C.c_void_p()
    assert lh.lib.lh_plan(C.byref(q), None, C.byref(out)) == lh.LH_ERR_INVALID
    q.agg = 7
    assert lh.lib.lh_plan(C.byref(q), None, C.byref(out)) == lh.LH_ERR_INVALID


def test_encode_and_logreg_validate_without_a_gpu(lh):
    nf = C.c_uint32(7)
    ids = (C.c_void_p * 1)(0)
    # NULL id array, n_id_cols 0, row_col out of range, no feature at all
    assert lh.lib.lh_encode(0, 1, None, 0, 0, None, 1, None, None, None, C.byref(nf), None) == lh.LH_ERR_INVALID
    assert lh.lib.lh_encode(0, 0, ids, 0, 0, None, 1, None, None, None, C.byref(nf), None) == lh.LH_ERR_INVALID
    assert lh.lib.lh_encode(0, 1, ids, 1, 0, None, 1, None, None, None, C.byref(nf), None) == lh.LH_ERR_INVALID
    assert lh.lib.lh_encode(0, 1, ids, 0, 0, None, 0, None, None, None, C.byref(nf), None) == lh.LH_ERR_INVALID
    cols = (lh.FeatureCol * 2)()
    cols[0].codes, cols[0].values, cols[0].card = 0x10, 0x20, 3   # both codes and values
    assert lh.lib.lh_encode(0, 1, ids, 0, 1, cols, 1, None, None, None, C.byref(nf), None) == lh.LH_ERR_INVALID
    cols[0].values = None
    cols[0].by = 1                                                  # no id column 1
    assert lh.lib.lh_encode(0, 1, ids, 0, 1, cols, 1, None, None, None, C.byref(nf), None) == lh.LH_ERR_INVALID
    cols[0].by = 0
    cols[0].card = 0                                                # empty category
    assert lh.lib.lh_encode(0, 1, ids, 0, 1, cols, 1, None, None, None, C.byref(nf), None) == lh.LH_ERR_INVALID
    # zero rows: only the feature count is produced
    cols[0].card = 3
    cols[1].values, cols[1].by = 0x30, 0
    assert lh.lib.lh_encode(0, 1, ids, 0, 2, cols, 1, None, None, None, C.byref(nf), None) == lh.LH_OK
    assert nf.value == 1 + 3 + 1
    assert lh.lib.lh_logreg_fit(C.c_void_p(0xdead), C.c_void_p(0xbeef), 0, None, 0, 0, 1, 0.5, None, None,
                                None) == lh.LH_ERR_INVALID
    assert b"live" in lh.lib.lh_last_error()


# --------------------------------------------------------------------------
# section 4 worked examples
# --------------------------------------------------------------------------

def _golden():
    return json.load(open(os.path.join(ROOT, "tests", "golden", "cost_examples.json")))


def test_icost_worked_example(lh):
    g = _golden()
    edges = [dict(e) for e in g["edges"] if e["name"] in g["icost_edges"]]
    # the example's node holds the four attributes orderkey..suppkey
    for e in edges:
        e["attrs"] = [v for v in e["attrs"] if v < 4]
    icost, _, _ = lh.order_cost(4, edges, g["icost_order"])
    assert icost == g["expected_icost"]


def test_weight_worked_example(lh):
    g = _golden()
    order = list(range(5))
    _, w, _ = lh.order_cost(5, g["edges"], order)
    names = g["attrs"]
    assert {names[i]: w[i] for i in range(5)} == g["expected_weights"]


def test_weighted_cost_of_the_example(lh):
    g = _golden()
    edges = [dict(e) for e in g["edges"] if e["name"] in g["icost_edges"]]
    for e in edges:
        e["attrs"] = [v for v in e["attrs"] if v < 4]
    icost, w, cost = lh.order_cost(4, edges, g["icost_order"])
    assert cost == sum(i * x for i, x in zip(icost, w))


def test_spgemm_order_relaxation(lh):
    # C(i,k) = SUM_j A(i,j) B(j,k): materialized-first [i,k,j] costs 50 at j
    # (uint & uint); the relaxation swaps to [i,j,k], 10 at j (uint & bs)
    edges = [{"attrs": [0, 1], "card": 40960}, {"attrs": [1, 2], "card": 40960}]
    ic, _, _ = lh.order_cost(3, edges, [0, 2, 1])
    assert ic == [0, 0, 50]
    ic, _, _ = lh.order_cost(3, edges, [0, 1, 2])
    assert ic == [0, 10, 0]
    order, cost = lh.choose_order(3, edges, out=[0, 2])
    assert order == [0, 1, 2] and cost == 10 * 100


def test_triangle_orders_tie_to_lexicographic(lh):
    edges = [{"attrs": [0, 1], "card": 100}, {"attrs": [1, 2], "card": 100}, {"attrs": [0, 2], "card": 100}]
    for o in ([0, 1, 2], [2, 1, 0], [1, 0, 2]):
        ic, _, cost = lh.order_cost(3, edges, o)
        assert ic == [1, 10, 50] and cost == 61 * 100
    order, _ = lh.choose_order(3, edges)
    assert order == [0, 1, 2]


def test_dense_relation_adds_no_intersection(lh):
    # SpMV y(i) = SUM_j A(i,j) x(j) with x completely dense
    edges = [{"attrs": [0, 1], "card": 1000}, {"attrs": [1], "card": 100, "dense": True}]
    ic, _, cost = lh.order_cost(2, edges, [0, 1])
    assert ic == [0, 0] and cost == 0
    edges[1]["dense"] = False
    ic, _, _ = lh.order_cost(2, edges, [0, 1])
    assert ic == [0, 10]


def test_star_order_prefers_equality_selected_heavy_attributes(lh):
    fact = {"attrs": [0, 1, 2, 3], "card": 60_000_000}
    dims = [{"attrs": [0], "card": 2_000_000}, {"attrs": [1], "card": 500_000},
            {"attrs": [2], "card": 100_000, "eq": True}, {"attrs": [3], "card": 10_000, "eq": True}]
    _, w, _ = lh.order_cost(4, [fact] + dims, [0, 1, 2, 3])
    assert w == [4, 1, 100, 100]
    order, cost = lh.choose_order(4, [fact] + dims)
    assert order[0] == 2 and cost == 1 * 100 + 10 * (100 + 4 + 1)


def test_invalid_orders_rejected(lh):
    edges = [{"attrs": [0, 1], "card": 10}]
    with pytest.raises(lh.LHError):
        lh.order_cost(2, edges, [0, 0])
    with pytest.raises(lh.LHError):
        lh.order_cost(2, [{"attrs": [0, 5], "card": 1}], [0, 1])
