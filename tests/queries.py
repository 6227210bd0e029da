"""Query specifications shared by the tests (plain data, no arithmetic).

A query is a dict in the format documented in ``oracle/__init__.py``; the
GPU-side tests translate the same dict into C-ABI calls.
"""
import numpy as np

import synth


def triangle(lo, hi):
    """R(a,b) |x| S(b,c) |x| T(a,c), COUNT(*), R = S = T = the oriented edges."""
    e = {"keys": [lo, hi], "bag": False}
    return {"n_attrs": 3, "agg": "count", "out": [],
            "atoms": [dict(e, attrs=[0, 1]), dict(e, attrs=[1, 2]), dict(e, attrs=[0, 2])]}


def spgemm(a, b):
    """C(i,k) = SUM_j A(i,j) * B(j,k); attributes i=0, j=1, k=2."""
    (ar, ac, av), (br, bc, bv) = a, b
    return {"n_attrs": 3, "agg": "sum", "out": [0, 2],
            "atoms": [{"keys": [ar, ac], "attrs": [0, 1], "annos": [av], "anno": 0, "bag": True},
                      {"keys": [br, bc], "attrs": [1, 2], "annos": [bv], "anno": 0, "bag": True}]}


def spmv(a, x):
    """y(i) = SUM_j A(i,j) * x(j); attributes i=0, j=1."""
    ar, ac, av = a
    n = len(x)
    return {"n_attrs": 2, "agg": "sum", "out": [0],
            "atoms": [{"keys": [ar, ac], "attrs": [0, 1], "annos": [av], "anno": 0, "bag": True},
                      {"keys": [np.arange(n, dtype=np.uint32)], "attrs": [1], "annos": [x],
                       "anno": 0, "bag": True}]}


def set_pairs(pairs):
    """R(p,x) |x| S(p,x), COUNT(*) GROUP BY p: row p of the result is
    |A_p intersect B_p| for the p-th pair (A_p, B_p); attributes p=0, x=1."""
    pr = np.concatenate([np.full(len(a), i, np.uint32) for i, (a, _) in enumerate(pairs)])
    ps = np.concatenate([np.full(len(b), i, np.uint32) for i, (_, b) in enumerate(pairs)])
    xr = np.concatenate([a for a, _ in pairs]).astype(np.uint32)
    xs = np.concatenate([b for _, b in pairs]).astype(np.uint32)
    return {"n_attrs": 2, "agg": "count", "out": [0],
            "atoms": [{"keys": [pr, xr], "attrs": [0, 1], "bag": False},
                      {"keys": [ps, xs], "attrs": [0, 1], "bag": False}]}


def star(s, u_hi=0.20, m2=0, m3=0):
    """SUM(fact.ann) GROUP BY D1.g over fact |x| D0..D3 with D0.u < u_hi,
    D2.m == m2 and D3.m == m3.  Attributes k0..k3 = 0..3."""
    f = s["fact"]
    d = s["dims"]
    atoms = [
        {"keys": list(f["k"]), "attrs": [0, 1, 2, 3], "annos": [f["ann"]], "anno": 0, "bag": True},
        {"keys": [d[0]["key"]], "attrs": [0], "annos": [d[0]["u"]], "anno": -1, "bag": True},
        {"keys": [d[1]["key"]], "attrs": [1], "meta": [d[1]["g"]], "anno": -1, "bag": True},
        {"keys": [d[2]["key"]], "attrs": [2], "meta": [d[2]["m"]], "anno": -1, "bag": True},
        {"keys": [d[3]["key"]], "attrs": [3], "meta": [d[3]["m"]], "anno": -1, "bag": True},
    ]
    filters = [
        {"atom": 1, "kind": "range_anno", "col": 0, "lo": -np.inf, "hi": u_hi},
        {"atom": 3, "kind": "eq_meta", "col": 0, "eq": m2},
        {"atom": 4, "kind": "eq_meta", "col": 0, "eq": m3},
    ]
    return {"n_attrs": 4, "agg": "sum", "out": [], "group": [(2, 0)], "atoms": atoms, "filters": filters}


def q5(s, region=2, date_lo=730, date_hi=1095, agg="sum"):
    """SUM(lineitem.ann) (or COUNT) GROUP BY n over customer(c,n),
    orders(o,c), lineitem(o,s), supplier(s,n), nation(n,r), region(r) with
    region.name == region and date_lo <= orders.date < date_hi.
    Attributes c=0, o=1, s=2, n=3, r=4."""
    atoms = [
        {"keys": [s["customer"]["c"], s["customer"]["n"]], "attrs": [0, 3], "bag": False},
        {"keys": [s["orders"]["o"], s["orders"]["c"]], "attrs": [1, 0], "meta": [s["orders"]["date"]],
         "bag": True},
        {"keys": [s["lineitem"]["o"], s["lineitem"]["s"]], "attrs": [1, 2], "annos": [s["lineitem"]["ann"]],
         "anno": 0 if agg == "sum" else -1, "bag": True},
        {"keys": [s["supplier"]["s"], s["supplier"]["n"]], "attrs": [2, 3], "bag": False},
        {"keys": [s["nation"]["n"], s["nation"]["r"]], "attrs": [3, 4], "bag": False},
        {"keys": [s["region"]["r"]], "attrs": [4], "meta": [s["region"]["name"]], "bag": True},
    ]
    filters = [{"atom": 5, "kind": "eq_meta", "col": 0, "eq": region},
               {"atom": 1, "kind": "range_meta", "col": 0, "lo": float(date_lo), "hi": float(date_hi)}]
    return {"n_attrs": 5, "agg": agg, "out": [3], "atoms": atoms, "filters": filters}


def random_query(seed, max_atoms=4, max_attrs=4, domain=6, max_rows=7):
    """A tiny random hypergraph query with filters, group columns, bag or
    set relations, COUNT or SUM.  Values are small multiples of 2^-3 and
    random doubles, so sums exercise both exact and rounded cases."""
    rng = synth.rng_for(seed)
    n_attrs = int(rng.integers(1, max_attrs + 1))
    n_atoms = int(rng.integers(1, max_atoms + 1))
    agg = "sum" if rng.random() < 0.6 else "count"
    atoms = []
    for e in range(n_atoms):
        k = int(rng.integers(1, n_attrs + 1))
        attrs = sorted(rng.choice(n_attrs, k, replace=False).tolist())
        rng.shuffle(attrs)
        n = int(rng.integers(0, max_rows + 1))
        keys = [rng.integers(0, domain, n).astype(np.uint32) for _ in range(k)]
        bag = bool(rng.random() < 0.7)
        atom = {"keys": keys, "attrs": attrs, "bag": bag, "anno": -1}
        if bag:
            vals = synth.uniform_pm1(rng, n) if rng.random() < 0.5 else rng.integers(-8, 9, n) / 8.0
            atom["annos"] = [vals]
            atom["meta"] = [rng.integers(0, 3, n).astype(np.uint32)]
            if agg == "sum" and rng.random() < 0.7:
                atom["anno"] = 0
        atoms.append(atom)
    # every attribute must be covered
    covered = set(v for a in atoms for v in a["attrs"])
    for v in range(n_attrs):
        if v not in covered:
            a = atoms[int(rng.integers(0, n_atoms))]
            a["attrs"].append(v)
            a["keys"].append(rng.integers(0, domain, len(a["keys"][0])).astype(np.uint32))
    if agg == "sum" and all(a["anno"] < 0 for a in atoms):
        bags = [a for a in atoms if a["bag"]]
        if bags:
            bags[0]["anno"] = 0
        else:
            agg = "count"
    n_out = int(rng.integers(0, n_attrs + 1))
    out = rng.choice(n_attrs, n_out, replace=False).tolist()
    groups = []
    for e, a in enumerate(atoms):
        if a["bag"] and rng.random() < 0.2:
            groups.append((e, 0))
    filters = []
    for e, a in enumerate(atoms):
        if rng.random() < 0.3:
            filters.append({"atom": e, "kind": "eq_key", "col": int(rng.integers(0, len(a["keys"]))),
                            "eq": int(rng.integers(0, domain))})
        if a["bag"] and rng.random() < 0.3:
            filters.append({"atom": e, "kind": "range_anno", "col": 0, "lo": -0.5, "hi": 0.75})
        if a["bag"] and rng.random() < 0.2:
            filters.append({"atom": e, "kind": "eq_meta", "col": 0, "eq": int(rng.integers(0, 3))})
    return {"n_attrs": n_attrs, "atoms": atoms, "out": out, "group": groups, "agg": agg, "filters": filters}
