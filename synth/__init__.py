"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers (numpy ``Generator(PCG64(seed))``) and
lays them out as columns.  It holds none of the join or aggregation
arithmetic; both the GPU library's tests and the oracle consume its output.

Workloads (paper section 6 evaluates LA and BI queries; the datasets it
uses are not available, so these stand in for them by shape):

* ``rmat_edges``      R-MAT graph, edges oriented (low, high), self-loops
                      dropped, duplicates KEPT (a set-mode trie removes them).
* ``sparse_matrix``   exactly ``nnz_per_row`` distinct uniform columns per row,
                      values ``2*random()-1`` (multiples of 2^-53 in [-1, 1)).
* ``zipf_degree_matrix`` power-law row degrees (rank law r^-s scaled to a
                      target mean, clamped to [1, n], rows permuted).
* ``batched_instances`` the mixed SpMV / SpGEMM batch.
* ``star_schema``     fact table with Zipf foreign keys and four dimensions.
* small graph families for closed-form tests.
"""
import math

import numpy as np


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_pm1(rng, n):
    """Uniform(-1, 1) as 2*random()-1: every value is a multiple of 2^-53."""
    return 2.0 * rng.random(n) - 1.0


# --------------------------------------------------------------------------
# Graphs
# --------------------------------------------------------------------------

def rmat_edges(scale, n_samples, a=0.57, b=0.19, c=0.19, seed=2, chunk=1 << 22):
    """R-MAT samples: at each of ``scale`` levels pick a quadrant with
    probabilities (a, b, c, 1-a-b-c).  Returns (lo, hi) uint32 columns with
    lo < hi; self-loops are dropped, duplicates are kept, no vertex
    permutation is applied."""
    rng = rng_for(seed)
    t1 = np.uint32(round(a * 2**32))
    t2 = np.uint32(min(round((a + b) * 2**32), 2**32 - 1))
    t3 = np.uint32(min(round((a + b + c) * 2**32), 2**32 - 1))
    los, his = [], []
    done = 0
    while done < n_samples:
        m = min(chunk, n_samples - done)
        u = np.zeros(m, dtype=np.uint32)
        v = np.zeros(m, dtype=np.uint32)
        for _ in range(scale):
            r = rng.integers(0, 2**32, size=m, dtype=np.uint32)
            bu = r >= t2               # quadrants c, d: source bit 1
            bv = ((r >= t1) & (r < t2)) | (r >= t3)   # quadrants b, d: target bit 1
            u = (u << np.uint32(1)) | bu.astype(np.uint32)
            v = (v << np.uint32(1)) | bv.astype(np.uint32)
        keep = u != v
        u, v = u[keep], v[keep]
        los.append(np.minimum(u, v))
        his.append(np.maximum(u, v))
        done += m
    return np.concatenate(los), np.concatenate(his)


def complete_graph(n):
    i, j = np.triu_indices(n, 1)
    return i.astype(np.uint32), j.astype(np.uint32)


def complete_tripartite(a, b, c):
    """K_{a,b,c}: parts [0,a), [a,a+b), [a+b,a+b+c); every cross-part pair."""
    parts = [np.arange(0, a), np.arange(a, a + b), np.arange(a + b, a + b + c)]
    lo, hi = [], []
    for x in range(3):
        for y in range(x + 1, 3):
            p, q = np.meshgrid(parts[x], parts[y], indexing="ij")
            lo.append(p.ravel())
            hi.append(q.ravel())
    lo = np.concatenate(lo)
    hi = np.concatenate(hi)
    return np.minimum(lo, hi).astype(np.uint32), np.maximum(lo, hi).astype(np.uint32)


def wheel(n):
    """Hub 0 joined to an n-cycle on vertices 1..n."""
    rim = np.arange(1, n + 1)
    nxt = np.roll(rim, -1)
    lo = np.concatenate([np.zeros(n, dtype=np.int64), np.minimum(rim, nxt)])
    hi = np.concatenate([rim, np.maximum(rim, nxt)])
    return lo.astype(np.uint32), hi.astype(np.uint32)


def cycle(n):
    v = np.arange(n)
    w = np.roll(v, -1)
    return np.minimum(v, w).astype(np.uint32), np.maximum(v, w).astype(np.uint32)


def random_bipartite(n_left, n_right, p, seed):
    rng = rng_for(seed)
    m = rng.random((n_left, n_right)) < p
    i, j = np.nonzero(m)
    return i.astype(np.uint32), (j + n_left).astype(np.uint32)


def gnp(n, p, seed):
    rng = rng_for(seed)
    m = np.triu(rng.random((n, n)) < p, 1)
    i, j = np.nonzero(m)
    return i.astype(np.uint32), j.astype(np.uint32)


# --------------------------------------------------------------------------
# Sparse matrices
# --------------------------------------------------------------------------

def _distinct_columns(rng, deg, n):
    """For each row r draw deg[r] distinct uniform columns in [0, n)."""
    deg = np.asarray(deg, dtype=np.int64)
    rows = np.repeat(np.arange(len(deg), dtype=np.int64), deg)
    cols = np.empty(len(rows), dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(deg)])
    dense = deg * 2 > n
    sparse_mask = np.repeat(~dense, deg)
    # dense rows: a random subset via a permutation
    for r in np.nonzero(dense)[0]:
        cols[start[r]:start[r + 1]] = rng.permutation(n)[: deg[r]]
    idx = np.nonzero(sparse_mask)[0]
    cols[idx] = rng.integers(0, n, size=len(idx))
    while len(idx):
        key = rows[idx] * n + cols[idx]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(len(ks), dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        # also collide with entries already fixed in the same row
        redo = idx[order[dup]]
        if len(redo) == 0:
            break
        cols[redo] = rng.integers(0, n, size=len(redo))
        # re-check every sparse entry of the affected rows
        bad_rows = np.unique(rows[redo])
        idx = idx[np.isin(rows[idx], bad_rows)]
    return rows.astype(np.uint32), cols.astype(np.uint32)


def sparse_matrix(n, nnz_per_row, seed):
    """n x n, exactly nnz_per_row distinct uniform columns in every row."""
    rng = rng_for(seed)
    rows, cols = _distinct_columns(rng, np.full(n, nnz_per_row), n)
    vals = uniform_pm1(rng, len(rows))
    return rows, cols, vals


def zipf_degrees(n, s, mean, rng):
    """deg(r) = clamp(round(c * r^-s), 1, n) for ranks r = 1..n with c chosen
    by bisection so that the mean degree is ``mean``; rows permuted."""
    r = np.arange(1, n + 1, dtype=np.float64) ** (-s)

    def mean_for(c):
        return np.clip(np.round(c * r), 1, n).mean()

    lo, hi = 0.0, float(mean) * n
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if mean_for(mid) < mean:
            lo = mid
        else:
            hi = mid
    deg = np.clip(np.round(hi * r), 1, n).astype(np.int64)
    return rng.permutation(deg)


def zipf_degree_matrix(n, s, mean, rng):
    deg = zipf_degrees(n, s, mean, rng)
    rows, cols = _distinct_columns(rng, deg, n)
    vals = uniform_pm1(rng, len(rows))
    return rows, cols, vals


def batched_instances(count=512, n_lo=1024, n_hi=65536, s=1.1, mean=16, seed=4):
    """Half SpMV (y = A x, x dense) and half SpGEMM (C = A A), interleaved
    by a seeded shuffle; n log-uniform in [n_lo, n_hi]."""
    rng = rng_for(seed)
    kinds = np.array(["spmv"] * (count // 2) + ["spgemm"] * (count - count // 2))
    rng.shuffle(kinds)
    out = []
    for k in kinds:
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        rows, cols, vals = zipf_degree_matrix(n, s, mean, rng)
        inst = {"kind": str(k), "n": n, "rows": rows, "cols": cols, "vals": vals}
        if k == "spmv":
            inst["x"] = uniform_pm1(rng, n)
        out.append(inst)
    return out


# --------------------------------------------------------------------------
# Star schema
# --------------------------------------------------------------------------

def zipf_keys(rng, n_keys, s, size, chunk=1 << 23):
    """P(rank r) proportional to r^-s over n_keys ranks; rank -> key through
    a seeded permutation."""
    w = np.arange(1, n_keys + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = rng.permutation(n_keys).astype(np.uint32)
    out = np.empty(size, dtype=np.uint32)
    for i in range(0, size, chunk):
        m = min(chunk, size - i)
        u = rng.random(m)
        rank = np.minimum(np.searchsorted(cdf, u, side="right"), n_keys - 1)
        out[i:i + m] = perm[rank]
    return out


def star_schema(n_fact=60_000_000, dims=(2_000_000, 500_000, 100_000, 10_000), s=1.0, seed=3):
    """Fact(k0..k3, ann) with ann = price * (1 - discount) computed once per
    row (an expression over one relation becomes its annotation); four
    dimensions keyed by dense ids:
      D0: anno u ~ U[0,1)          (filter: u < 0.20)
      D1: meta g in [0, 100)       (GROUP BY g)
      D2: meta m in [0, 10)        (filter: m == 0)
      D3: meta m in [0, 100)       (filter: m == 0)
    """
    rng = rng_for(seed)
    fk = [zipf_keys(rng, d, s, n_fact) for d in dims]
    price = rng.random(n_fact)
    discount = rng.random(n_fact)
    ann = price * (1.0 - discount)
    d0 = {"key": np.arange(dims[0], dtype=np.uint32), "u": rng.random(dims[0])}
    d1 = {"key": np.arange(dims[1], dtype=np.uint32), "g": rng.integers(0, 100, dims[1]).astype(np.uint32)}
    d2 = {"key": np.arange(dims[2], dtype=np.uint32), "m": rng.integers(0, 10, dims[2]).astype(np.uint32)}
    d3 = {"key": np.arange(dims[3], dtype=np.uint32), "m": rng.integers(0, 100, dims[3]).astype(np.uint32)}
    return {"fact": {"k": fk, "ann": ann}, "dims": [d0, d1, d2, d3]}


def q5_schema(sf=1.0, seed=5):
    """Six relations with the join shape of a five-way TPC-H-style query
    around a cycle (customer, orders, lineitem, supplier sharing the nation
    key) with a nation/region tail, at TPC-H-like sizes per scale factor:
      region(r)          5 rows,   meta name = r
      nation(n, r)       25 rows,  r = n // 5
      supplier(s, n)     10,000 sf rows, n uniform
      customer(c, n)     150,000 sf rows, n uniform
      orders(o, c)       1,500,000 sf rows, c uniform, meta date in [0, 2557) days
      lineitem(o, s)     1..7 rows per order (mean 4), s uniform, bag,
                         annotation price * (1 - discount)
    Keys are dense ids; an expression over one relation inside the
    aggregate is that relation's annotation."""
    rng = rng_for(seed)
    n_s = max(1, int(10_000 * sf))
    n_c = max(1, int(150_000 * sf))
    n_o = max(1, int(1_500_000 * sf))
    region = {"r": np.arange(5, dtype=np.uint32), "name": np.arange(5, dtype=np.uint32)}
    nation = {"n": np.arange(25, dtype=np.uint32), "r": (np.arange(25) // 5).astype(np.uint32)}
    supplier = {"s": np.arange(n_s, dtype=np.uint32), "n": rng.integers(0, 25, n_s).astype(np.uint32)}
    customer = {"c": np.arange(n_c, dtype=np.uint32), "n": rng.integers(0, 25, n_c).astype(np.uint32)}
    orders = {"o": np.arange(n_o, dtype=np.uint32), "c": rng.integers(0, n_c, n_o).astype(np.uint32),
              "date": rng.integers(0, 2557, n_o).astype(np.uint32)}
    per = rng.integers(1, 8, n_o)
    lo = np.repeat(np.arange(n_o, dtype=np.uint32), per)
    n_l = len(lo)
    price = rng.random(n_l)
    discount = rng.integers(0, 11, n_l) / 100.0
    lineitem = {"o": lo, "s": rng.integers(0, n_s, n_l).astype(np.uint32), "ann": price * (1.0 - discount)}
    return {"region": region, "nation": nation, "supplier": supplier, "customer": customer,
            "orders": orders, "lineitem": lineitem}


# --------------------------------------------------------------------------
# Voter classification (section 7)
# --------------------------------------------------------------------------

def voter_schema(n_voters=7_503_555, n_precincts=2_751, seed=7):
    """Two tables shaped like the voter classification application of
    section 7 (its dataset is not available): voters keyed by a dense id,
    each registered in a precinct (Zipf s = 0.6 over precincts), and the
    precincts keyed by a dense id.
      voters:    precinct, sex (3 codes), race (7), age in [18, 100),
                 age_group = (age - 18) // 10 (9 codes), party (4),
                 age_std = (age - 50) / 20 (a numeric feature),
                 voted (label 0/1)
      precincts: county (100 codes), district (13), urban (2)
    The label is a Bernoulli draw whose probability adds per-code offsets
    of age group, party and the precinct's urban flag (clipped to
    [0.02, 0.98]), so the classes depend on the features."""
    rng = rng_for(seed)
    n = n_voters
    precinct = zipf_keys(rng, n_precincts, 0.6, n)
    sex = rng.choice(3, n, p=[0.52, 0.46, 0.02]).astype(np.uint32)
    race = rng.choice(7, n, p=[0.62, 0.17, 0.09, 0.06, 0.03, 0.02, 0.01]).astype(np.uint32)
    age = rng.integers(18, 100, n).astype(np.uint32)
    age_group = ((age - 18) // 10).astype(np.uint32)
    party = rng.choice(4, n, p=[0.38, 0.33, 0.25, 0.04]).astype(np.uint32)
    age_std = (age.astype(np.float64) - 50.0) / 20.0
    county = rng.integers(0, 100, n_precincts).astype(np.uint32)
    district = rng.integers(0, 13, n_precincts).astype(np.uint32)
    urban = rng.integers(0, 2, n_precincts).astype(np.uint32)
    t_age = rng.random(9) * 0.4
    t_party = rng.random(4) * 0.3
    t_urban = np.array([0.0, 0.15])
    prob = np.clip(0.1 + t_age[age_group] + t_party[party] + t_urban[urban[precinct]], 0.02, 0.98)
    voted = (rng.random(n) < prob).astype(np.float64)
    voters = {"id": np.arange(n, dtype=np.uint32), "precinct": precinct, "sex": sex, "race": race, "age": age,
              "age_group": age_group, "party": party, "age_std": age_std, "voted": voted}
    precincts = {"id": np.arange(n_precincts, dtype=np.uint32), "county": county, "district": district,
                 "urban": urban}
    return {"voters": voters, "precincts": precincts}


# The voter pipeline's selections and encoded columns: id column 0 is the
# voter id, 1 the precinct id of a result row.
VOTER_FILTER = {"age_lo": 21, "age_hi": 200, "district_lo": 0, "district_hi": 10}


def voter_features(schema):
    """The source columns of the encoding, in feature order."""
    v, p = schema["voters"], schema["precincts"]
    return [{"codes": v["sex"], "card": 3, "by": 0},
            {"codes": v["race"], "card": 7, "by": 0},
            {"codes": v["age_group"], "card": 9, "by": 0},
            {"codes": v["party"], "card": 4, "by": 0},
            {"codes": p["county"], "card": 100, "by": 1},
            {"codes": p["district"], "card": 13, "by": 1},
            {"codes": p["urban"], "card": 2, "by": 1},
            {"values": v["age_std"], "by": 0}]


# --------------------------------------------------------------------------
# Intersection micro-benchmark sets
# --------------------------------------------------------------------------

def set_pairs(card, universe, n_pairs, seed):
    """n_pairs pairs of sorted distinct uint32 sets, each of size ``card``
    drawn uniformly without replacement from [0, universe)."""
    rng = rng_for(seed)

    def one():
        # the sorted draw, read off a mask (no sort of the sample needed)
        mask = np.zeros(universe, dtype=bool)
        mask[rng.choice(universe, card, replace=False)] = True
        return np.flatnonzero(mask).astype(np.uint32)

    out = []
    for _ in range(n_pairs):
        a = one()
        b = one()
        out.append((a, b))
    return out
