"""FP64 reference of the mixed SQL + ML pipeline of section 7 -- TEST
INFRASTRUCTURE ONLY (tests, the smoke check and the CPU-baseline leg of the
benchmark call it; the GPU library never does).

The application of section 7 joins and filters two tables into one feature
set, encodes its categorical variables, and trains a logistic regression
model for five iterations.  The paper fixes none of the details; the
readings taken here:

* SQL phase: the natural join voters(id, precinct) |x| precincts(id) on the
  precinct id, with half-open range selections on the voter's age and the
  precinct's district; the result is the set of (voter id, precinct id)
  pairs, ascending.
* Encoding: a bias feature 0 with value 1, then for each source column in
  order either one indicator feature per code (categorical; value 1) or
  one feature carrying the value (numeric).  A result row yields one
  (row, feature, value) triple per slot, in slot order.
* Training: full-batch gradient descent on the mean log-loss
  L(w) = mean_i [log(1 + exp(z_i)) - y_i z_i], z = X w, whose gradient is
  X^T (sigmoid(z) - y) / n; each iteration sets w = w - step * gradient.
  The loss reported for an iteration is L at its starting w.

Pins (tests/test_oracle_ml.py): the join against nested loops, the
indicator blocks against scikit-learn's OneHotEncoder, the loss against
scikit-learn's log_loss, the gradient against central finite differences
of the loss, and long runs against scikit-learn's unpenalized
LogisticRegression optimum.
"""
import numpy as np


def sql_phase(voters, precincts, age_lo, age_hi, district_lo, district_hi):
    """(voter ids, precinct ids) of the filtered join, ascending, distinct."""
    keep_p = (precincts["district"] >= district_lo) & (precincts["district"] < district_hi)
    good_precincts = np.asarray(precincts["id"])[keep_p]
    keep_v = (voters["age"] >= age_lo) & (voters["age"] < age_hi)
    keep_v &= np.isin(voters["precinct"], good_precincts)
    pairs = np.stack([np.asarray(voters["id"])[keep_v], np.asarray(voters["precinct"])[keep_v]], axis=1)
    pairs = np.unique(pairs.astype(np.uint64), axis=0).astype(np.uint32)  # sorted by (voter, precinct)
    return pairs[:, 0].copy(), pairs[:, 1].copy()


def feature_bases(cols, bias=True):
    """First feature id of each column's block, and the feature count."""
    bases = []
    nf = 1 if bias else 0
    for c in cols:
        bases.append(nf)
        nf += int(c["card"]) if "codes" in c else 1
    return bases, nf


def encode(ids, row_col, cols, bias=True):
    """Triples (rows, feats, vals) of n * slots entries, row-major, and the
    feature count.  cols: {"codes", "card", "by"} or {"values", "by"}."""
    n = len(ids[row_col]) if ids else 0
    slots = len(cols) + (1 if bias else 0)
    bases, nf = feature_bases(cols, bias)
    rows = np.repeat(np.asarray(ids[row_col], dtype=np.uint32), slots)
    feats = np.zeros(n * slots, dtype=np.uint32)
    vals = np.ones(n * slots, dtype=np.float64)
    first = 1 if bias else 0
    for k, c in enumerate(cols):
        idx = np.asarray(ids[c["by"]], dtype=np.int64)
        slot = first + k
        if "codes" in c:
            codes = np.asarray(c["codes"])[idx]
            assert np.all(codes < c["card"]), "a code is not below its card"
            feats[slot::slots] = bases[k] + codes
        else:
            feats[slot::slots] = bases[k]
            vals[slot::slots] = np.asarray(c["values"], dtype=np.float64)[idx]
    return rows, feats, vals, nf


def design_matrix(rows, feats, vals, n_feat):
    """Dense X over the distinct row ids (ascending); repeated (row,
    feature) triples add up.  Returns (row ids, X)."""
    row_ids = np.unique(rows)
    X = np.zeros((len(row_ids), n_feat), dtype=np.float64)
    np.add.at(X, (np.searchsorted(row_ids, rows), feats.astype(np.int64)), vals)
    return row_ids, X


def loss(X, y, w):
    z = X @ w
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def gradient(X, y, w):
    z = X @ w
    p = 1.0 / (1.0 + np.exp(-z))
    return X.T @ (p - y) / X.shape[0]


def logreg(X, y, w0, iters, step):
    """Weights after `iters` gradient steps and the loss at each step's
    start."""
    w = np.array(w0, dtype=np.float64, copy=True)
    losses = []
    for _ in range(iters):
        losses.append(loss(X, y, w))
        w = w - step * gradient(X, y, w)
    return w, np.array(losses)
