"""ctypes binding of the C ABI in include/lh.h (argument marshalling only).

Every step of the join runs in liblh.so's HIP kernels; this module only
lays out descriptors, hands device pointers across and copies results back.
torch supplies device memory and the current stream.  If liblh.so is not
built, importing the binding raises: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblh.so")

LH_OK, LH_ERR_INVALID, LH_ERR_OOM, LH_ERR_DEVICE, LH_ERR_UNSUPPORTED, LH_ERR_OVERFLOW = range(6)
LH_SET, LH_BAG = 0x0, 0x1
LAYOUT = {"plain": 0x00, "uint": 0x10, "bitset": 0x20, "learned": 0x30}
LH_AGG_COUNT, LH_AGG_SUM = 0, 1
FILTER_KIND = {"eq_key": 0, "eq_meta": 1, "range_anno": 2, "range_meta": 3}
POLICY = {"plain": 0, "learned": 1, "fixed": 2}
GROUP_IMPL = {"auto": 0x00, "sort": 0x10, "hash": 0x20, "dense": 0x30}
GROUP_IMPL_NAME = {0: "streamed", 1: "sort", 2: "hash", 3: "dense"}
LH_MAX_KEYS = 8


class RelationDesc(C.Structure):
    _fields_ = [
        ("n_rows", C.c_uint64),
        ("n_keys", C.c_uint32),
        ("keys", C.POINTER(C.c_void_p)),
        ("n_annos", C.c_uint32),
        ("annos", C.POINTER(C.c_void_p)),
        ("n_meta", C.c_uint32),
        ("meta", C.POINTER(C.c_void_p)),
        ("level_order", C.POINTER(C.c_uint32)),
        ("flags", C.c_uint32),
    ]


class Atom(C.Structure):
    _fields_ = [("trie", C.c_void_p), ("attr_of_key", C.POINTER(C.c_uint32)), ("anno", C.c_int32)]


class Filter(C.Structure):
    _fields_ = [("atom", C.c_uint32), ("kind", C.c_uint32), ("col", C.c_uint32), ("eq", C.c_uint32),
                ("lo", C.c_double), ("hi", C.c_double)]


class GroupCol(C.Structure):
    _fields_ = [("atom", C.c_uint32), ("meta_col", C.c_uint32)]


class Query(C.Structure):
    _fields_ = [
        ("n_attrs", C.c_uint32),
        ("n_atoms", C.c_uint32),
        ("atoms", C.POINTER(Atom)),
        ("n_out", C.c_uint32),
        ("out_attrs", C.POINTER(C.c_uint32)),
        ("n_group", C.c_uint32),
        ("group_cols", C.POINTER(GroupCol)),
        ("agg", C.c_uint32),
        ("n_filters", C.c_uint32),
        ("filters", C.POINTER(Filter)),
        ("attr_order", C.POINTER(C.c_uint32)),
        ("policy", C.c_uint32),
    ]


class Result(C.Structure):
    _fields_ = [
        ("n_rows", C.c_uint64),
        ("n_cols", C.c_uint32),
        ("out_keys", C.POINTER(C.c_void_p)),
        ("counts", C.c_void_p),
        ("sums", C.c_void_p),
        ("exact", C.c_uint32),
        ("n_join_tuples", C.c_uint64),
        ("group_impl", C.c_uint32),
    ]


class TrieInfo(C.Structure):
    _fields_ = [
        ("n_levels", C.c_uint32),
        ("n_rows", C.c_uint64),
        ("level_size", C.c_uint64 * LH_MAX_KEYS),
        ("level_sets", C.c_uint64 * LH_MAX_KEYS),
        ("level_bitsets", C.c_uint64 * LH_MAX_KEYS),
        ("level_words", C.c_uint64 * LH_MAX_KEYS),
        ("level_order", C.c_uint32 * LH_MAX_KEYS),
        ("col_distinct", C.c_uint64 * LH_MAX_KEYS),
        ("col_freq_max", C.c_uint64 * LH_MAX_KEYS),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("n_attrs", C.c_uint32),
        ("attr_order", C.c_uint32 * 16),
        ("cost", C.c_double),
        ("case_prefix", C.c_uint32),
        ("exact_digits", C.c_uint32),
        ("exact_lsb", C.c_int32),
        ("level_alg", C.c_uint32 * 16),
        ("blas", C.c_uint32),
    ]


class Hypergraph(C.Structure):
    _fields_ = [
        ("n_attrs", C.c_uint32),
        ("n_edges", C.c_uint32),
        ("edge_attr_count", C.POINTER(C.c_uint32)),
        ("edge_attrs", C.POINTER(C.c_uint32)),
        ("edge_card", C.POINTER(C.c_uint64)),
        ("edge_eq", C.POINTER(C.c_uint32)),
        ("edge_dense", C.POINTER(C.c_uint32)),
        ("edge_attr_lf_mean", C.POINTER(C.c_float)),
        ("edge_attr_lf_max", C.POINTER(C.c_float)),
    ]


LH_GHD_MAX_NODES = 16


class Ghd(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_uint32),
        ("parent", C.c_int32 * LH_GHD_MAX_NODES),
        ("edges", C.c_uint32 * LH_GHD_MAX_NODES),
        ("attrs", C.c_uint32 * LH_GHD_MAX_NODES),
        ("pushed", C.c_uint32 * LH_GHD_MAX_NODES),
        ("node_fhw", C.c_double * LH_GHD_MAX_NODES),
        ("fhw", C.c_double),
        ("depth", C.c_uint32),
        ("shared", C.c_uint32),
        ("sel_depth", C.c_uint32),
    ]


class FeatureCol(C.Structure):
    _fields_ = [
        ("codes", C.c_void_p),
        ("values", C.c_void_p),
        ("card", C.c_uint32),
        ("by", C.c_uint32),
        ("n_ids", C.c_uint64),
    ]


# Every entry point declared in include/lh.h, with its ctypes signature.
SIGNATURES = {
    "lh_trie_build": ([C.POINTER(RelationDesc), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "lh_plan": ([C.POINTER(Query), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "lh_join_aggregate": ([C.POINTER(C.c_void_p), C.c_uint32, C.c_void_p, C.POINTER(C.POINTER(Result))], C.c_int),
    "lh_join_aggregate_noalloc": ([C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_void_p), C.c_void_p,
                                   C.c_void_p, C.POINTER(C.c_uint64)], C.c_int),
    "lh_free": ([C.c_void_p], None),
    "lh_last_error": ([], C.c_char_p),
    "lh_trie_get_info": ([C.c_void_p, C.POINTER(TrieInfo)], C.c_int),
    "lh_trie_read_level": ([C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p], C.c_int),
    "lh_result_read": ([C.POINTER(Result), C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p], C.c_int),
    "lh_plan_get_info": ([C.c_void_p, C.POINTER(PlanInfo)], C.c_int),
    "lh_order_cost": ([C.POINTER(Hypergraph), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                       C.POINTER(C.c_uint32), C.POINTER(C.c_double)], C.c_int),
    "lh_choose_order": ([C.POINTER(Hypergraph), C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                         C.POINTER(C.c_double)], C.c_int),
    "lh_live_allocations": ([], C.c_long),
    "lh_mlp_create": ([C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(C.c_void_p)], C.c_int),
    "lh_mlp_free": ([C.c_void_p], None),
    "lh_mlp_num_params": ([C.c_void_p], C.c_uint64),
    "lh_mlp_get_params": ([C.c_void_p, C.c_void_p], C.c_int),
    "lh_mlp_set_params": ([C.c_void_p, C.c_void_p], C.c_int),
    "lh_mlp_loss_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.POINTER(C.c_float),
                          C.c_void_p], C.c_int),
    "lh_mlp_train": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_float,
                      C.c_uint64, C.c_void_p, C.POINTER(C.c_float)], C.c_int),
    "lh_mlp_predict": ([C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p, C.c_void_p], C.c_int),
    "lh_use_model": ([C.c_uint32, C.c_void_p], C.c_int),
    "lh_order_features": ([C.POINTER(Hypergraph), C.POINTER(C.c_uint32), C.c_void_p], C.c_int),
    "lh_profile_enable": ([C.c_int], None),
    "lh_profile_reset": ([], None),
    "lh_profile_read": ([C.c_void_p, C.c_uint32], C.c_uint32),
    "lh_ghd_fhw": ([C.POINTER(Hypergraph), C.c_uint32, C.POINTER(C.c_double)], C.c_int),
    "lh_ghd_choose": ([C.POINTER(Hypergraph), C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(C.c_uint32),
                       C.POINTER(Ghd)], C.c_int),
    "lh_ghd_for_query": ([C.POINTER(Query), C.POINTER(Ghd)], C.c_int),
    "lh_ghd_join_aggregate": ([C.POINTER(Query), C.POINTER(Ghd), C.c_void_p, C.POINTER(C.POINTER(Result))],
                              C.c_int),
    "lh_encode": ([C.c_uint64, C.c_uint32, C.POINTER(C.c_void_p), C.c_uint32, C.c_uint32, C.POINTER(FeatureCol),
                   C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32), C.c_void_p], C.c_int),
    "lh_logreg_fit": ([C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32,
                       C.c_double, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
}


def _load():
    # torch brings its own HIP runtime (same soname as the one liblh.so
    # links); loading torch first makes the process use exactly one.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run paper_1708_07859_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


class LHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lh status {status}: {msg}")
        self.status = status


def _check(st):
    if st != LH_OK:
        raise LHError(st, lib.lh_last_error().decode())


# --------------------------------------------------------------------------
# device columns
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def current_stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_device(a, dtype=None):
    """numpy array -> contiguous device tensor with the same bytes
    (uint32 is carried as int32 storage)."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.contiguous()
    a = np.ascontiguousarray(a, dtype=dtype) if dtype is not None else np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to("cuda")


def _ptr_array(tensors):
    arr = (C.c_void_p * max(1, len(tensors)))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


class Trie:
    """Owning handle of an lh_trie."""

    def __init__(self, handle, n_keys):
        self.handle = handle
        self.n_keys = n_keys

    def info(self):
        inf = TrieInfo()
        _check(lib.lh_trie_get_info(self.handle, C.byref(inf)))
        L = inf.n_levels
        return {"n_levels": L, "n_rows": inf.n_rows,
                "level_size": list(inf.level_size[:L]), "level_sets": list(inf.level_sets[:L]),
                "level_bitsets": list(inf.level_bitsets[:L]), "level_words": list(inf.level_words[:L]),
                "level_order": list(inf.level_order[:L]),
                "col_distinct": list(inf.col_distinct[:L]), "col_freq_max": list(inf.col_freq_max[:L])}

    def read_level(self, level):
        inf = self.info()
        n = inf["level_size"][level]
        keys = np.zeros(n, np.uint32)
        offs = np.zeros(n + 1, np.uint32)
        _check(lib.lh_trie_read_level(self.handle, level, keys.ctypes.data, offs.ctypes.data))
        return keys, offs

    def free(self):
        if self.handle:
            lib.lh_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def trie_build(keys, annos=(), meta=(), level_order=None, bag=False, layout="plain", stream=None):
    """lh_trie_build over device columns (torch tensors or numpy arrays)."""
    kt = [to_device(k, np.uint32) for k in keys]
    at = [to_device(a, np.float64) for a in annos]
    mt = [to_device(m, np.uint32) for m in meta]
    n = int(kt[0].numel()) if kt else 0
    d = RelationDesc()
    d.n_rows = n
    d.n_keys = len(kt)
    ka, aa, ma = _ptr_array(kt), _ptr_array(at), _ptr_array(mt)
    d.keys = C.cast(ka, C.POINTER(C.c_void_p))
    d.n_annos = len(at)
    d.annos = C.cast(aa, C.POINTER(C.c_void_p))
    d.n_meta = len(mt)
    d.meta = C.cast(ma, C.POINTER(C.c_void_p))
    lo = None
    if level_order is not None:
        lo = (C.c_uint32 * len(level_order))(*level_order)
        d.level_order = C.cast(lo, C.POINTER(C.c_uint32))
    d.flags = (LH_BAG if bag else LH_SET) | LAYOUT[layout]
    out = C.c_void_p()
    _check(lib.lh_trie_build(C.byref(d), stream if stream is not None else current_stream(), C.byref(out)))
    return Trie(out.value, len(kt))


class Plan:
    def __init__(self, handle, tries):
        self.handle = handle
        self._tries = tries  # a plan borrows its tries

    def info(self):
        inf = PlanInfo()
        _check(lib.lh_plan_get_info(self.handle, C.byref(inf)))
        n = inf.n_attrs
        return {"attr_order": list(inf.attr_order[:n]), "cost": inf.cost, "case_prefix": inf.case_prefix,
                "exact_digits": inf.exact_digits, "exact_lsb": inf.exact_lsb,
                "level_alg": list(inf.level_alg[:n]), "blas": inf.blas}

    def free(self):
        if self.handle:
            lib.lh_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


LH_DENSE_BLAS = 0x40


def _query(n_attrs, atoms, out=(), group=(), agg="count", filters=(), attr_order=None, policy="plain",
           group_impl="auto", dense_blas=False):
    """An lh_query and the ctypes arrays it points into (keep them alive)."""
    catoms = (Atom * len(atoms))()
    keep = [catoms]
    for i, (t, attrs, anno) in enumerate(atoms):
        am = (C.c_uint32 * len(attrs))(*attrs)
        keep.append(am)
        catoms[i].trie = t.handle
        catoms[i].attr_of_key = C.cast(am, C.POINTER(C.c_uint32))
        catoms[i].anno = anno
    q = Query()
    q.n_attrs = n_attrs
    q.n_atoms = len(atoms)
    q.atoms = catoms
    oa = (C.c_uint32 * max(1, len(out)))(*out)
    keep.append(oa)
    q.n_out = len(out)
    q.out_attrs = C.cast(oa, C.POINTER(C.c_uint32))
    ga = (GroupCol * max(1, len(group)))()
    keep.append(ga)
    for i, (a, c) in enumerate(group):
        ga[i].atom, ga[i].meta_col = a, c
    q.n_group = len(group)
    q.group_cols = ga
    q.agg = LH_AGG_SUM if agg == "sum" else LH_AGG_COUNT
    fa = (Filter * max(1, len(filters)))()
    keep.append(fa)
    for i, f in enumerate(filters):
        fa[i].atom = f["atom"]
        fa[i].kind = FILTER_KIND[f["kind"]]
        fa[i].col = f.get("col", 0)
        fa[i].eq = f.get("eq", 0)
        fa[i].lo = f.get("lo", 0.0)
        fa[i].hi = f.get("hi", 0.0)
    q.n_filters = len(filters)
    q.filters = fa
    if attr_order is not None:
        ao = (C.c_uint32 * len(attr_order))(*attr_order)
        keep.append(ao)
        q.attr_order = C.cast(ao, C.POINTER(C.c_uint32))
    q.policy = POLICY[policy] | GROUP_IMPL[group_impl] | (LH_DENSE_BLAS if dense_blas else 0)
    return q, keep


def plan(n_attrs, atoms, out=(), group=(), agg="count", filters=(), attr_order=None, policy="plain",
         stream=None, group_impl="auto", dense_blas=False):
    """lh_plan.  atoms: [(Trie, attr_of_key list, anno index or -1)]."""
    q, keep = _query(n_attrs, atoms, out, group, agg, filters, attr_order, policy, group_impl, dense_blas)
    out_h = C.c_void_p()
    _check(lib.lh_plan(C.byref(q), stream if stream is not None else current_stream(), C.byref(out_h)))
    return Plan(out_h.value, [a[0] for a in atoms])


class _DevCol:
    """A device column owned by someone else (a result's key column)."""

    def __init__(self, ptr, n):
        self.ptr, self.n = ptr, n

    def data_ptr(self):
        return self.ptr or 0

    def numel(self):
        return self.n


class JoinResult:
    def __init__(self, ptr):
        self.ptr = ptr

    @property
    def n_rows(self):
        return self.ptr.contents.n_rows

    def key_columns(self):
        """The result's output columns as device pointers wrapped for
        lh_encode (objects with data_ptr() and numel())."""
        r = self.ptr.contents
        return [_DevCol(r.out_keys[c], r.n_rows) for c in range(r.n_cols)]

    def to_host(self):
        r = self.ptr.contents
        n, w = r.n_rows, r.n_cols
        cols = [np.zeros(n, np.uint32) for _ in range(w)]
        counts = np.zeros(n, np.uint64)
        # a SUM result is flagged exact even when it has no rows
        sums = np.zeros(n, np.float64) if (r.sums or r.exact) else None
        kp = (C.c_void_p * max(1, w))(*[c.ctypes.data for c in cols])
        _check(lib.lh_result_read(self.ptr, kp, counts.ctypes.data,
                                  sums.ctypes.data if (sums is not None and n) else None))
        keys = np.stack(cols, axis=1) if w else np.zeros((n, 0), np.uint32)
        return {"keys": keys, "counts": counts, "sums": sums, "n_join": int(r.n_join_tuples), "exact": r.exact,
                "group_impl": GROUP_IMPL_NAME.get(r.group_impl, r.group_impl)}

    def free(self):
        if self.ptr:
            lib.lh_free(C.cast(self.ptr, C.c_void_p))
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def join_aggregate(plans, stream=None):
    """lh_join_aggregate over one or more plans (more than one = batched)."""
    n = len(plans)
    arr = (C.c_void_p * n)(*[p.handle for p in plans])
    outs = (C.POINTER(Result) * n)()
    _check(lib.lh_join_aggregate(arr, n, stream if stream is not None else current_stream(), outs))
    return [JoinResult(outs[i]) for i in range(n)]


def join_aggregate_noalloc(plan, out_keys, counts, sums=None, stream=None):
    """lh_join_aggregate_noalloc: run one plan with no device allocation,
    writing into caller-owned device tensors (out_keys: one uint32/int32
    tensor per output column, counts: uint64/int64, sums: float64 or None),
    all with the same capacity.  Returns the number of rows written."""
    cap = counts.numel()
    for t in list(out_keys) + ([sums] if sums is not None else []):
        if t.numel() < cap:
            raise ValueError("every output buffer needs the capacity of counts")
    keys = (C.c_void_p * max(1, len(out_keys)))(*[t.data_ptr() for t in out_keys])
    n = C.c_uint64(0)
    _check(lib.lh_join_aggregate_noalloc(plan.handle, stream if stream is not None else current_stream(), cap,
                                         keys, counts.data_ptr(), sums.data_ptr() if sums is not None else None,
                                         C.byref(n)))
    return n.value


def live_allocations():
    return lib.lh_live_allocations()


LH_MODEL_LAYOUT, LH_MODEL_ORDER = 0, 1
LH_LAYOUT_FEATURES, LH_ORDER_FEATURES = 4, 24


class Mlp:
    """Owning handle of an lh_mlp (the learned cost model's network)."""

    def __init__(self, d_in, width=64, seed=0):
        h = C.c_void_p()
        _check(lib.lh_mlp_create(d_in, width, seed, C.byref(h)))
        self.handle = h.value
        self.d_in = d_in

    @property
    def n_params(self):
        return int(lib.lh_mlp_num_params(self.handle))

    def get_params(self):
        p = np.zeros(self.n_params, np.float32)
        _check(lib.lh_mlp_get_params(self.handle, p.ctypes.data))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.n_params
        _check(lib.lh_mlp_set_params(self.handle, p.ctypes.data))

    def loss_grad(self, X, y):
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_float()
        _check(lib.lh_mlp_loss_grad(self.handle, X.ctypes.data, y.ctypes.data, len(y), current_stream(),
                                    C.byref(loss), g.ctypes.data))
        return loss.value, g

    def train(self, X, y, epochs=200, batch=256, lr=1e-3, seed=0):
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        loss = C.c_float()
        _check(lib.lh_mlp_train(self.handle, X.ctypes.data, y.ctypes.data, len(y), epochs, batch, lr, seed,
                                current_stream(), C.byref(loss)))
        return loss.value

    def predict(self, X, bf16=True):
        X = np.ascontiguousarray(X, np.float32)
        y = np.zeros(len(X), np.float32)
        _check(lib.lh_mlp_predict(self.handle, X.ctypes.data, len(X), 1 if bf16 else 0, current_stream(),
                                  y.ctypes.data))
        return y

    def free(self):
        if self.handle:
            lib.lh_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def use_model(slot, mlp):
    _check(lib.lh_use_model(slot, mlp.handle if mlp is not None else None))


def order_features(n_attrs, edges, order):
    h, keep = _hypergraph(n_attrs, edges)
    o = (C.c_uint32 * n_attrs)(*order)
    f = np.zeros(LH_ORDER_FEATURES, np.float32)
    _check(lib.lh_order_features(C.byref(h), o, f.ctypes.data))
    return f


class ProfileEntry(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_uint64), ("total_ms", C.c_double),
                ("rows", C.c_uint64), ("elements", C.c_uint64)]


def profile_enable(on=True):
    lib.lh_profile_enable(1 if on else 0)


def profile_reset():
    lib.lh_profile_reset()


def profile_read():
    """{kernel: {launches, total_ms, rows, elements}} since the last reset."""
    n = lib.lh_profile_read(None, 0)
    arr = (ProfileEntry * max(1, n))()
    n = lib.lh_profile_read(arr, n)
    return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                   "rows": arr[i].rows, "elements": arr[i].elements} for i in range(n)}


# --------------------------------------------------------------------------
# the section 4 cost estimate on a bare hypergraph
# --------------------------------------------------------------------------

def _hypergraph(n_attrs, edges):
    """edges: [{"attrs": [...], "card": int, "eq": bool, "dense": bool}]"""
    cnt = (C.c_uint32 * len(edges))(*[len(e["attrs"]) for e in edges])
    flat = [v for e in edges for v in e["attrs"]]
    attrs = (C.c_uint32 * max(1, len(flat)))(*flat)
    card = (C.c_uint64 * len(edges))(*[int(e["card"]) for e in edges])
    eq = (C.c_uint32 * len(edges))(*[1 if e.get("eq") else 0 for e in edges])
    dense = (C.c_uint32 * len(edges))(*[1 if e.get("dense") else 0 for e in edges])
    has_lf = all("lf_mean" in e for e in edges) and edges
    lfm = (C.c_float * max(1, len(flat)))(*([v for e in edges for v in e["lf_mean"]] if has_lf else []))
    lfx = (C.c_float * max(1, len(flat)))(*([v for e in edges for v in e["lf_max"]] if has_lf else []))
    h = Hypergraph(n_attrs, len(edges), cnt, attrs, card, eq, dense, lfm if has_lf else None, lfx if has_lf else None)
    return h, (cnt, attrs, card, eq, dense, lfm, lfx)


def order_cost(n_attrs, edges, order):
    h, keep = _hypergraph(n_attrs, edges)
    o = (C.c_uint32 * n_attrs)(*order)
    ic = (C.c_uint32 * n_attrs)()
    w = (C.c_uint32 * n_attrs)()
    cost = C.c_double()
    _check(lib.lh_order_cost(C.byref(h), o, ic, w, C.byref(cost)))
    return list(ic), list(w), cost.value


def choose_order(n_attrs, edges, out=()):
    h, keep = _hypergraph(n_attrs, edges)
    oa = (C.c_uint32 * max(1, len(out)))(*out)
    o = (C.c_uint32 * n_attrs)()
    cost = C.c_double()
    _check(lib.lh_choose_order(C.byref(h), len(out), oa, o, C.byref(cost)))
    return list(o), cost.value


# --------------------------------------------------------------------------
# multi-node plans (generalized hypertree decompositions)
# --------------------------------------------------------------------------

def _ghd_dict(g):
    n = g.n_nodes
    return {"n_nodes": n, "parent": list(g.parent[:n]), "edges": list(g.edges[:n]), "attrs": list(g.attrs[:n]),
            "pushed": list(g.pushed[:n]), "node_fhw": list(g.node_fhw[:n]), "fhw": g.fhw, "depth": g.depth,
            "shared": g.shared, "sel_depth": g.sel_depth}


def _ghd_struct(d):
    g = Ghd()
    g.n_nodes = len(d["edges"])
    for t in range(g.n_nodes):
        g.parent[t] = d["parent"][t]
        g.edges[t] = d["edges"][t]
        g.pushed[t] = 1 if d.get("pushed", [0] * g.n_nodes)[t] else 0
    return g


def _edges_only(n_attrs, edges):
    return _hypergraph(n_attrs, [dict(e, card=e.get("card", 1)) for e in edges])


def ghd_fhw(n_attrs, edges, edge_mask):
    """lh_ghd_fhw: edges [{"attrs": [...]}]."""
    h, keep = _edges_only(n_attrs, edges)
    f = C.c_double()
    _check(lib.lh_ghd_fhw(C.byref(h), edge_mask, C.byref(f)))
    return f.value


def ghd_choose(n_attrs, edges, out=()):
    """lh_ghd_choose: edges [{"attrs": [...], "sel": bool, "root": bool}]."""
    h, keep = _edges_only(n_attrs, edges)
    sel = (C.c_uint32 * len(edges))(*[1 if e.get("sel") else 0 for e in edges])
    root = (C.c_uint32 * len(edges))(*[1 if e.get("root") else 0 for e in edges])
    oa = (C.c_uint32 * max(1, len(out)))(*out)
    g = Ghd()
    _check(lib.lh_ghd_choose(C.byref(h), sel, root, len(out), oa, C.byref(g)))
    return _ghd_dict(g)


def ghd_for_query(n_attrs, atoms, out=(), group=(), agg="count", filters=()):
    q, keep = _query(n_attrs, atoms, out, group, agg, filters)
    g = Ghd()
    _check(lib.lh_ghd_for_query(C.byref(q), C.byref(g)))
    return _ghd_dict(g)


def ghd_join_aggregate(n_attrs, atoms, out=(), group=(), agg="count", filters=(), attr_order=None,
                       policy="plain", ghd=None, stream=None, group_impl="auto"):
    """lh_ghd_join_aggregate; ghd: a dict with parent/edges/pushed lists, or
    None for the library's choice."""
    q, keep = _query(n_attrs, atoms, out, group, agg, filters, attr_order, policy, group_impl)
    gp = C.byref(_ghd_struct(ghd)) if ghd is not None else None
    res = C.POINTER(Result)()
    _check(lib.lh_ghd_join_aggregate(C.byref(q), gp, stream if stream is not None else current_stream(),
                                     C.byref(res)))
    return JoinResult(res)


# --------------------------------------------------------------------------
# query dictionaries (the format documented in tests/queries.py)
# --------------------------------------------------------------------------

def run_query(query, attr_order=None, policy="plain", layout="plain", return_plan_info=False, ghd=False,
              group_impl="auto", dense_blas=False):
    """Build one trie per distinct relation of the query, plan, run, and
    copy the result to host in the format {keys, counts, sums, n_join}.
    ghd=False runs one plan; ghd=None runs the library's decomposition, a
    dict (parent/edges/pushed lists) runs that one."""
    tries = {}
    atoms = []
    for a in query["atoms"]:
        ident = (tuple(id(k) for k in a["keys"]), tuple(id(x) for x in a.get("annos", [])),
                 tuple(id(m) for m in a.get("meta", [])), bool(a.get("bag", False)))
        if ident not in tries:
            tries[ident] = trie_build(a["keys"], a.get("annos", []), a.get("meta", []), bag=a.get("bag", False),
                                      layout=layout)
        atoms.append((tries[ident], list(a["attrs"]), int(a.get("anno", -1))))
    args = dict(out=query.get("out", []), group=query.get("group", []), agg=query.get("agg", "count"),
                filters=query.get("filters", []), attr_order=attr_order, policy=policy, group_impl=group_impl)
    p = None
    try:
        if ghd is False:
            p = plan(query["n_attrs"], atoms, dense_blas=dense_blas, **args)
            r = join_aggregate([p])[0]
        else:
            r = ghd_join_aggregate(query["n_attrs"], atoms, ghd=ghd, **args)
        out = r.to_host()
        r.free()
        if return_plan_info and p is not None:
            out["plan"] = p.info()
    finally:
        if p is not None:
            p.free()
        for t in tries.values():
            t.free()
    return out


# --------------------------------------------------------------------------
# the SQL + ML pipeline (section 7): encoding and logistic regression
# --------------------------------------------------------------------------

def encode(ids, row_col, cols, bias=True, stream=None):
    """lh_encode.  ids: device id columns (e.g. JoinResult.key_columns());
    cols: dicts {"codes": column, "card": c, "by": i} or {"values": column,
    "by": i} with device (or numpy) columns indexed by ids[by].  Returns
    (rows, feats, vals, n_feat) as device tensors of n * slots entries."""
    torch = _torch()
    n = int(ids[0].numel()) if ids else 0
    keep = []
    fc = (FeatureCol * max(1, len(cols)))()
    for i, c in enumerate(cols):
        if "codes" in c:
            t = to_device(c["codes"], np.uint32)
            fc[i].codes = t.data_ptr()
            fc[i].card = int(c["card"])
        else:
            t = to_device(c["values"], np.float64)
            fc[i].values = t.data_ptr()
        keep.append(t)
        fc[i].by = int(c["by"])
        fc[i].n_ids = int(t.numel())
    slots = len(cols) + (1 if bias else 0)
    rows = torch.empty(n * slots, dtype=torch.int32, device="cuda")
    feats = torch.empty(n * slots, dtype=torch.int32, device="cuda")
    vals = torch.empty(n * slots, dtype=torch.float64, device="cuda")
    ia = (C.c_void_p * max(1, len(ids)))(*[t.data_ptr() for t in ids])
    nf = C.c_uint32()
    _check(lib.lh_encode(n, len(ids), ia, row_col, len(cols), fc, 1 if bias else 0, rows.data_ptr(),
                         feats.data_ptr(), vals.data_ptr(), C.byref(nf),
                         stream if stream is not None else current_stream()))
    return rows, feats, vals, nf.value


def logreg_fit(x_rows, x_cols, y, w, iters, step, anno=0, loss=True, stream=None):
    """lh_logreg_fit on two Trie handles; y and w are device float64
    tensors (w is updated in place).  Returns the per-iteration mean
    log-loss as a device tensor (or None)."""
    torch = _torch()
    lt = torch.empty(max(1, iters), dtype=torch.float64, device="cuda") if loss else None
    _check(lib.lh_logreg_fit(x_rows.handle, x_cols.handle, anno, y.data_ptr(), int(y.numel()), int(w.numel()),
                             iters, float(step), w.data_ptr(), lt.data_ptr() if loss else None,
                             stream if stream is not None else current_stream()))
    return lt[:iters] if loss else None
