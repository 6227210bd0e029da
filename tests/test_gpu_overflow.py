"""Large multiplicities in the exact SUM and in tuple counts.

A join of bag relations that carry no annotation multiplies the term of
every surviving combination by the product of their run lengths (section
2.3: each duplicate row is its own tuple).  These inputs are tiny but make
that multiplicity 2^32 and more, the case where 32-bit digits times the
multiplicity leave int64, where a block's row count leaves 32 bits, and
where a count leaves 64 bits.  Expected values are closed forms: the join of
relations that all hold one key value is their cross product, so
COUNT = prod |R_e| and SUM = v * prod of the unannotated |R_e|, rounded once.
"""
import sys
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KEY = 7
V = 0.7853981633974483 - 2.0 ** -53 * 3     # a full 53-bit mantissa


@pytest.fixture(scope="module")
def lh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh as binding
    return binding


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dup_relation(n, anno=None, meta=False):
    keys = [np.full(n, KEY, np.uint32)]
    rel = {"keys": keys, "attrs": [0], "bag": True, "anno": -1}
    if anno is not None:
        rel["annos"] = [np.full(n, anno, np.float64)]
        rel["anno"] = 0
    if meta:
        rel["meta"] = [np.full(n, 3, np.uint32)]
    return rel


def star_query(sizes, annotated_last=True, out=(), group=(), agg="sum"):
    """sizes[i] duplicate rows of KEY in relation i, all joined on one
    attribute; the last relation carries the annotation V when asked."""
    atoms = []
    for i, n in enumerate(sizes):
        last = i == len(sizes) - 1
        atoms.append(dup_relation(n, anno=V if (last and annotated_last) else None, meta=last))
    return {"n_attrs": 1, "agg": agg, "out": list(out), "group": list(group), "atoms": atoms}


def expect_sum(sizes):
    mult = 1
    for n in sizes[:-1]:
        mult *= n
    return float(Fraction(V) * mult * sizes[-1])


CASES = [
    # (sizes, out, group, group_impl)
    ([65536, 65536, 1], [], [], "auto"),          # one group: the register accumulator
    ([65536, 65536, 1], [0], [], "sort"),         # emitted tuples, sorted and reduced
    ([65536, 65536, 1], [0], [], "hash"),
    ([65536, 65536, 1], [0], [], "dense"),
    ([65536, 65536, 1], [], [(2, 0)], "sort"),    # GROUP BY a meta column of the annotated relation
    ([65536, 65537, 3], [0], [], "sort"),         # multiplicity 65536 * 65537, not a power of two
    ([65536, 65537, 3], [], [], "auto"),
    ([65536, 65536, 65536, 1], [], [], "auto"),   # multiplicity 2^48
]


@pytest.mark.parametrize("sizes,out,group,impl", CASES)
def test_sum_with_large_multiplicity(lh, sizes, out, group, impl):
    say("large multiplicity", sizes, out, group, impl)
    q = star_query(sizes, out=out, group=group)
    got = lh.run_query(q, group_impl=impl)
    count = 1
    for n in sizes:
        count *= n
    assert got["counts"].tolist() == [count]
    want = expect_sum(sizes)
    assert got["sums"].view(np.uint64).tolist() == np.array([want]).view(np.uint64).tolist(), (got["sums"], want)
    if out:
        assert got["keys"].tolist() == [[KEY]]
    if group:
        assert got["keys"].tolist() == [[3]]


def test_count_beyond_2_64_is_an_error(lh):
    # four unannotated relations of 65536 duplicate rows: 2^64 tuples
    say("count 2^64")
    q = star_query([65536] * 4, annotated_last=False, agg="count")
    with pytest.raises(lh.LHError) as ei:
        lh.run_query(q)
    assert ei.value.status == 5      # LH_ERR_OVERFLOW
    # one fewer relation: 2^48 tuples, counted exactly
    q = star_query([65536] * 3, annotated_last=False, agg="count")
    assert lh.run_query(q)["counts"].tolist() == [1 << 48]


def test_emitted_rows_beyond_2_32_rejected_by_count_pass(lh):
    # two annotated relations of 65536 rows: one hit stands for 2^32 row
    # combinations, more than the sorted GROUP BY can materialize; the
    # count pass alone must reject it (no fill runs)
    say("emit 2^32")
    atoms = [dup_relation(65536, anno=0.5), dup_relation(65536, anno=0.25)]
    q = {"n_attrs": 1, "agg": "sum", "out": [0], "atoms": atoms}
    with pytest.raises(lh.LHError) as ei:
        lh.run_query(q, group_impl="sort")
    assert ei.value.status == 5      # LH_ERR_OVERFLOW
