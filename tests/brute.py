"""Nested-loop brute force for tiny aggregate-join queries (test pin).

Enumerates every combination of one row per atom, keeps the combinations
whose rows agree on every shared attribute and pass the filters, and sums
the annotation products with ``fractions.Fraction`` before one correctly
rounded conversion to float.  Written from the definition of the
annotated join (paper, section 2.3): a join multiplies the annotations of
the joined tuples and the aggregation sums them over the projected-away
attributes.  It shares nothing with the hash-join oracle it checks.
"""
import itertools
from fractions import Fraction


def _passes(atom_idx, atom, r, filters):
    for f in filters:
        if f["atom"] != atom_idx:
            continue
        k = f["kind"]
        if k == "eq_key" and int(atom["keys"][f["col"]][r]) != f["eq"]:
            return False
        if k == "eq_meta" and int(atom["meta"][f["col"]][r]) != f["eq"]:
            return False
        if k == "range_anno" and not (f["lo"] <= float(atom["annos"][f["col"]][r]) < f["hi"]):
            return False
        if k == "range_meta" and not (f["lo"] <= float(atom["meta"][f["col"]][r]) < f["hi"]):
            return False
    return True


def _rows(i, atom, filters):
    n = len(atom["keys"][0])
    rows = [r for r in range(n) if _passes(i, atom, r, filters)]
    if not atom.get("bag", False):
        seen, keep = set(), []
        for r in rows:
            t = tuple(int(c[r]) for c in atom["keys"])
            if t not in seen:
                seen.add(t)
                keep.append(r)
        rows = keep
    return rows


def _term(factors):
    if len(factors) == 1:
        return Fraction(factors[0])
    p = factors[0]
    for x in factors[1:-1]:
        p = p * x                     # rounded double multiply, left to right
    return Fraction(p) * Fraction(factors[-1])


def brute(query):
    atoms = query["atoms"]
    filters = query.get("filters", [])
    out = list(query.get("out", []))
    groups = list(query.get("group", []))
    is_sum = query.get("agg", "count") == "sum"
    rows = [_rows(i, a, filters) for i, a in enumerate(atoms)]
    acc = {}
    n_join = 0
    for combo in itertools.product(*rows):
        binding = {}
        ok = True
        for a, r in zip(atoms, combo):
            for col, attr in zip(a["keys"], a["attrs"]):
                v = int(col[r])
                if binding.setdefault(attr, v) != v:
                    ok = False
                    break
            if not ok:
                break
        if not ok:
            continue
        key = tuple(binding[v] for v in out) + tuple(
            int(atoms[ga]["meta"][gc][combo[ga]]) for ga, gc in groups)
        cnt, s = acc.get(key, (0, Fraction(0)))
        if is_sum:
            f = [float(a["annos"][a["anno"]][r]) for a, r in zip(atoms, combo) if a.get("anno", -1) >= 0]
            s += _term(f)
        acc[key] = (cnt + 1, s)
        n_join += 1
    if not out and not groups and not acc:
        acc[()] = (0, Fraction(0))
    keys = sorted(acc)
    return {"keys": keys, "counts": [acc[k][0] for k in keys],
            "sums": [float(acc[k][1]) for k in keys] if is_sum else None, "n_join": n_join}
