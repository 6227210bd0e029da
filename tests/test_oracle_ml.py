"""Pins for the oracle of the SQL + ML pipeline (section 7): nested-loop
joins, scikit-learn's one-hot encoder, log-loss and unpenalized logistic
regression, and finite differences.  CPU only."""
import numpy as np
import pytest
from scipy.special import expit
from sklearn.linear_model import LogisticRegression
from sklearn.metrics import log_loss
from sklearn.preprocessing import OneHotEncoder

import synth
from oracle import ml


def _schema(n=300, m=7, seed=11):
    return synth.voter_schema(n, m, seed)


def test_sql_phase_matches_nested_loops():
    d = _schema()
    v, p = d["voters"], d["precincts"]
    f = dict(age_lo=30, age_hi=70, district_lo=2, district_hi=9)
    got = ml.sql_phase(v, p, **f)
    want = []
    for i in range(len(v["id"])):
        for j in range(len(p["id"])):
            if (v["precinct"][i] == p["id"][j] and f["age_lo"] <= v["age"][i] < f["age_hi"]
                    and f["district_lo"] <= p["district"][j] < f["district_hi"]):
                want.append((int(v["id"][i]), int(p["id"][j])))
    want.sort()
    assert len(want) > 20
    assert [tuple(map(int, t)) for t in zip(*got)] == want


def test_sql_phase_empty_selection():
    d = _schema()
    vid, pid = ml.sql_phase(d["voters"], d["precincts"], 0, 0, 0, 13)
    assert len(vid) == 0 and len(pid) == 0


def test_encoding_matches_one_hot_encoder():
    d = _schema(500, 9, 3)
    vid, pid = ml.sql_phase(d["voters"], d["precincts"], **synth.VOTER_FILTER)
    cols = synth.voter_features(d)
    rows, feats, vals, nf = ml.encode([vid, pid], 0, cols, bias=True)
    assert nf == 1 + 3 + 7 + 9 + 4 + 100 + 13 + 2 + 1
    row_ids, X = ml.design_matrix(rows, feats, vals, nf)
    assert np.array_equal(row_ids, vid)
    ids = [vid, pid]
    assert np.all(X[:, 0] == 1.0)  # bias
    col = 1
    for c in cols:
        src = np.asarray(ids[c["by"]], dtype=np.int64)
        if "codes" in c:
            enc = OneHotEncoder(categories=[np.arange(c["card"])], sparse_output=False)
            want = enc.fit_transform(np.asarray(c["codes"])[src].reshape(-1, 1))
            assert np.array_equal(X[:, col:col + c["card"]], want)
            col += c["card"]
        else:
            assert np.array_equal(X[:, col], np.asarray(c["values"])[src])
            col += 1
    assert col == nf


def test_design_matrix_adds_repeated_entries():
    rows = np.array([5, 5, 9, 5], np.uint32)
    feats = np.array([1, 1, 0, 2], np.uint32)
    vals = np.array([0.5, 0.25, 2.0, -1.0])
    ids, X = ml.design_matrix(rows, feats, vals, 3)
    assert list(ids) == [5, 9]
    assert np.array_equal(X, np.array([[0.0, 0.75, -1.0], [2.0, 0.0, 0.0]]))


def _random_problem(n=400, f=3, seed=5):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, f))
    w_true = np.array([1.5, -2.0, 0.5])[:f]
    y = (rng.random(n) < expit(X @ w_true)).astype(np.float64)
    return X, y


def test_loss_matches_log_loss():
    X, y = _random_problem()
    rng = np.random.default_rng(1)
    for _ in range(3):
        w = rng.standard_normal(X.shape[1])
        assert ml.loss(X, y, w) == pytest.approx(log_loss(y, expit(X @ w)), rel=1e-12)


def test_gradient_matches_finite_differences():
    X, y = _random_problem(200, 3, 9)
    w = np.array([0.3, -0.7, 1.1])
    g = ml.gradient(X, y, w)
    h = 1e-6
    fd = np.array([(ml.loss(X, y, w + h * e) - ml.loss(X, y, w - h * e)) / (2 * h) for e in np.eye(3)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)
    # one step of logreg moves along -step * gradient
    w1, losses = ml.logreg(X, y, w, 1, 0.25)
    assert np.allclose(w1, w - 0.25 * fd, rtol=1e-6, atol=1e-9)
    assert losses[0] == ml.loss(X, y, w)


def test_long_run_reaches_the_unpenalized_optimum():
    X, y = _random_problem()
    w, losses = ml.logreg(X, y, np.zeros(3), 3000, 1.0)
    ref = LogisticRegression(penalty=None, fit_intercept=False, tol=1e-12, max_iter=10000).fit(X, y)
    assert np.allclose(w, ref.coef_[0], rtol=1e-6, atol=1e-8)
    assert np.all(np.diff(losses) <= 1e-15)


def test_loss_decreases_on_voter_features():
    d = _schema(2000, 40, 4)
    vid, pid = ml.sql_phase(d["voters"], d["precincts"], **synth.VOTER_FILTER)
    rows, feats, vals, nf = ml.encode([vid, pid], 0, synth.voter_features(d))
    row_ids, X = ml.design_matrix(rows, feats, vals, nf)
    y = d["voters"]["voted"][row_ids]
    w, losses = ml.logreg(X, y, np.zeros(nf), 20, 0.5)
    assert losses[0] == pytest.approx(np.log(2.0))
    assert np.all(np.diff(losses) < 0)
