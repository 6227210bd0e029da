"""The voter classification application of section 7 on the library: a SQL
phase (a filtered two-table join), categorical feature encoding of its
result, and logistic regression trained on the design matrix's tries.

Argument marshalling only: every step is a library call (lh_plan and
lh_join_aggregate, lh_encode, lh_trie_build, lh_logreg_fit) running HIP
kernels on the current stream.
"""
from . import lh


class VoterTables:
    """The two tables resident on the device: the voters trie over (id,
    precinct) with age as a meta column, the precincts trie over (id) with
    the district, and the columns the encoding reads."""

    def __init__(self, schema, features):
        """schema: {"voters": columns, "precincts": columns}; features: the
        encoded source columns in feature order, as lh.encode takes them
        (codes or values indexed by id column 0, the voter, or 1, the
        precinct)."""
        v, p = schema["voters"], schema["precincts"]
        self.voters = lh.trie_build([v["id"], v["precinct"]], meta=[v["age"]], bag=True)
        self.precincts = lh.trie_build([p["id"]], meta=[p["district"]], bag=True)
        self.y = lh.to_device(v["voted"], "float64")
        self.n_voters = len(v["id"])
        self.features = []
        for c in features:
            d = dict(c)
            key = "codes" if "codes" in c else "values"
            d[key] = lh.to_device(c[key])
            self.features.append(d)

    def free(self):
        self.voters.free()
        self.precincts.free()


def sql_phase(t, age_lo, age_hi, district_lo, district_hi, policy="plain"):
    """Voters of the age range in precincts of the district range: the
    join result with (voter id, precinct id) per row, ascending."""
    atoms = [(t.voters, [0, 1], -1), (t.precincts, [1], -1)]
    filters = [{"atom": 0, "kind": "range_meta", "col": 0, "lo": age_lo, "hi": age_hi},
               {"atom": 1, "kind": "range_meta", "col": 0, "lo": district_lo, "hi": district_hi}]
    p = lh.plan(2, atoms, out=[0, 1], agg="count", filters=filters, policy=policy)
    try:
        return lh.join_aggregate([p])[0]
    finally:
        p.free()


def design_tries(rows, feats, vals):
    """The (row, feature) and (feature, row) tries of the triples.  The
    training kernels read the sets' keys only, so every set keeps the uint
    layout (no bitsets are built)."""
    xr = lh.trie_build([rows, feats], annos=[vals], bag=True, layout="uint")
    xc = lh.trie_build([rows, feats], annos=[vals], level_order=[1, 0], bag=True, layout="uint")
    return xr, xc


def run(t, iters=5, step=0.5, age_lo=21, age_hi=200, district_lo=0, district_hi=10, w0=None):
    """The whole application; returns {"w", "loss", "n_rows", "n_feat"}
    with w and loss as device tensors."""
    torch = lh._torch()
    res = sql_phase(t, age_lo, age_hi, district_lo, district_hi)
    try:
        rows, feats, vals, nf = lh.encode(res.key_columns(), 0, t.features, bias=True)
        n_rows = res.n_rows
    finally:
        res.free()
    xr, xc = design_tries(rows, feats, vals)
    del rows, feats, vals
    try:
        w = torch.zeros(nf, dtype=torch.float64, device="cuda") if w0 is None else w0.clone()
        loss = lh.logreg_fit(xr, xc, t.y, w, iters, step)
    finally:
        xr.free()
        xc.free()
    return {"w": w, "loss": loss, "n_rows": n_rows, "n_feat": nf}
