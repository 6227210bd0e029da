"""Join-aggregate oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it and
shares no code with it.

``join_aggregate(query)`` evaluates an aggregate-join query over annotated
relations (paper, section 2.3, "Capturing Aggregate-Join Queries"; filters
per section 2.1; GROUP BY per section 5) with a pairwise hash join in atom
declaration order followed by hash aggregation, summing exactly and rounding
once to the nearest double (see ``oracle.h``).

Query format (plain Python data; numpy arrays for columns)::

    {"n_attrs": 3,
     "atoms": [{"keys": [u32, ...], "attrs": [0, 1], "annos": [f64, ...],
                "meta": [u32, ...], "anno": -1 | i, "bag": bool}, ...],
     "out": [attr, ...], "group": [(atom, meta_col), ...],
     "agg": "count" | "sum",
     "filters": [{"atom": a, "kind": "eq_key"|"eq_meta"|"range_anno"|"range_meta",
                  "col": c, "eq": v, "lo": x, "hi": y}, ...]}

The result is ``{"keys": (n, n_out+n_group) uint32, "counts": uint64[n],
"sums": float64[n] | None, "n_join": int, "n_intermediate": int}``, rows
sorted ascending by key.  An ungrouped query returns exactly one row.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_KIND = {"eq_key": 0, "eq_meta": 1, "range_anno": 2, "range_meta": 3}
_AGG = {"count": 0, "sum": 1}
ORC_OK, ORC_E_INVALID, ORC_E_NOMEM, ORC_E_RANGE = 0, 1, 2, 3


class _Atom(C.Structure):
    _fields_ = [
        ("n_rows", C.c_uint64),
        ("n_keys", C.c_uint32),
        ("keys", C.POINTER(C.POINTER(C.c_uint32))),
        ("attr_of_key", C.POINTER(C.c_uint32)),
        ("n_annos", C.c_uint32),
        ("annos", C.POINTER(C.POINTER(C.c_double))),
        ("n_meta", C.c_uint32),
        ("meta", C.POINTER(C.POINTER(C.c_uint32))),
        ("anno", C.c_int32),
        ("bag", C.c_uint32),
    ]


class _Filter(C.Structure):
    _fields_ = [("atom", C.c_uint32), ("kind", C.c_uint32), ("col", C.c_uint32),
                ("eq", C.c_uint32), ("lo", C.c_double), ("hi", C.c_double)]


class _Group(C.Structure):
    _fields_ = [("atom", C.c_uint32), ("meta_col", C.c_uint32)]


class _Query(C.Structure):
    _fields_ = [
        ("n_attrs", C.c_uint32),
        ("n_atoms", C.c_uint32),
        ("atoms", C.POINTER(_Atom)),
        ("n_out", C.c_uint32),
        ("out_attrs", C.POINTER(C.c_uint32)),
        ("n_group", C.c_uint32),
        ("groups", C.POINTER(_Group)),
        ("agg", C.c_uint32),
        ("n_filters", C.c_uint32),
        ("filters", C.POINTER(_Filter)),
    ]


class _Result(C.Structure):
    _fields_ = [
        ("n_rows", C.c_uint64),
        ("n_cols", C.c_uint32),
        ("keys", C.POINTER(C.c_uint32)),
        ("counts", C.POINTER(C.c_uint64)),
        ("sums", C.POINTER(C.c_double)),
        ("n_join_tuples", C.c_uint64),
        ("n_intermediate", C.c_uint64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = C.CDLL(path)
        lib.orc_join_aggregate.argtypes = [C.POINTER(_Query), C.POINTER(_Result)]
        lib.orc_join_aggregate.restype = C.c_int
        lib.orc_result_free.argtypes = [C.POINTER(_Result)]
        lib.orc_result_free.restype = None
        lib.orc_exact_dot.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]
        lib.orc_exact_dot.restype = C.c_double
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_set_threads.restype = None
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = C.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__({1: "invalid query", 2: "out of memory",
                          3: "a term does not fit the exact accumulator"}.get(code, str(code)))
        self.code = code


def _ptr_array(arrays, ctype, dtype, keep):
    arr = (C.POINTER(ctype) * max(1, len(arrays)))()
    for i, a in enumerate(arrays):
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        arr[i] = a.ctypes.data_as(C.POINTER(ctype))
    keep.append(arr)
    return arr


def join_aggregate(query):
    lib = _load()
    keep = []
    atoms = query["atoms"]
    catoms = (_Atom * len(atoms))()
    for i, a in enumerate(atoms):
        keys = a["keys"]
        n = len(keys[0]) if keys else 0
        attrs = np.ascontiguousarray(a["attrs"], dtype=np.uint32)
        keep.append(attrs)
        annos = a.get("annos", [])
        meta = a.get("meta", [])
        catoms[i].n_rows = n
        catoms[i].n_keys = len(keys)
        catoms[i].keys = _ptr_array(keys, C.c_uint32, np.uint32, keep)
        catoms[i].attr_of_key = attrs.ctypes.data_as(C.POINTER(C.c_uint32))
        catoms[i].n_annos = len(annos)
        catoms[i].annos = _ptr_array(annos, C.c_double, np.float64, keep)
        catoms[i].n_meta = len(meta)
        catoms[i].meta = _ptr_array(meta, C.c_uint32, np.uint32, keep)
        catoms[i].anno = int(a.get("anno", -1))
        catoms[i].bag = 1 if a.get("bag", False) else 0
    out = np.ascontiguousarray(query.get("out", []), dtype=np.uint32)
    groups = query.get("group", [])
    cgroups = (_Group * max(1, len(groups)))()
    for i, (ga, gc) in enumerate(groups):
        cgroups[i].atom, cgroups[i].meta_col = ga, gc
    filters = query.get("filters", [])
    cfilt = (_Filter * max(1, len(filters)))()
    for i, f in enumerate(filters):
        cfilt[i].atom = f["atom"]
        cfilt[i].kind = _KIND[f["kind"]]
        cfilt[i].col = f.get("col", 0)
        cfilt[i].eq = f.get("eq", 0)
        cfilt[i].lo = f.get("lo", 0.0)
        cfilt[i].hi = f.get("hi", 0.0)
    q = _Query()
    q.n_attrs = query["n_attrs"]
    q.n_atoms = len(atoms)
    q.atoms = catoms
    q.n_out = len(out)
    q.out_attrs = out.ctypes.data_as(C.POINTER(C.c_uint32))
    q.n_group = len(groups)
    q.groups = cgroups
    q.agg = _AGG[query.get("agg", "count")]
    q.n_filters = len(filters)
    q.filters = cfilt
    res = _Result()
    st = lib.orc_join_aggregate(C.byref(q), C.byref(res))
    if st != ORC_OK:
        raise OracleError(st)
    try:
        n, w = res.n_rows, res.n_cols
        keys = np.ctypeslib.as_array(res.keys, shape=(n * w,)).copy().reshape(n, w) if n * w else np.zeros((n, w), np.uint32)
        counts = np.ctypeslib.as_array(res.counts, shape=(n,)).copy() if n else np.zeros(0, np.uint64)
        sums = None
        if query.get("agg", "count") == "sum":
            sums = np.ctypeslib.as_array(res.sums, shape=(n,)).copy() if n else np.zeros(0, np.float64)
        return {"keys": keys, "counts": counts, "sums": sums,
                "n_join": int(res.n_join_tuples), "n_intermediate": int(res.n_intermediate)}
    finally:
        lib.orc_result_free(C.byref(res))


def set_threads(n):
    """Threads of the probe side (OpenMP); 0 restores the default."""
    _load().orc_set_threads(int(n))


def threads():
    """Threads the next join_aggregate call will use."""
    return int(_load().orc_threads())


def exact_dot(a, b=None):
    """Exact SUM a[i]*b[i] (or SUM a[i]) rounded once to the nearest double."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    bp = None
    if b is not None:
        b = np.ascontiguousarray(b, dtype=np.float64)
        assert b.shape == a.shape
        bp = b.ctypes.data
    st = C.c_int(0)
    v = lib.orc_exact_dot(a.ctypes.data, bp, a.size, C.byref(st))
    if st.value != ORC_OK:
        raise OracleError(st.value)
    return v


def lib_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboracle.so")
