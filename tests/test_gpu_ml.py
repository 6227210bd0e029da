"""The SQL + ML pipeline of section 7 on the GPU against the oracle: the
filtered join and the encoding bit for bit, logistic regression on the
design matrix's tries within 1e-9 of the FP64 oracle (relative to
max(1, |w|)), on voter-shaped tables and on random sparse matrices whose
rows and feature lists span the kernels' staged and unstaged paths, runs
of repeated entries, and empty input."""
import sys

import numpy as np
import pytest

import synth
from oracle import ml

pytestmark = pytest.mark.gpu

# The FP64 sums of the GPU and of numpy differ in order only: the
# gradient's error is below n * eps * max|x|, far inside this bound for
# the sizes here, and five damped steps do not amplify it past it.
W_TOL = 1e-9
LOSS_RTOL = 1e-12


@pytest.fixture(scope="module")
def lh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh as binding
    return binding


@pytest.fixture(scope="module")
def pipeline(lh):
    from paper_1708_07859_amd import pipeline as p
    return p


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check_w(w_gpu, w_ref):
    err = np.abs(w_gpu - w_ref) / np.maximum(1.0, np.abs(w_ref))
    assert np.all(err <= W_TOL), float(err.max())


def oracle_pipeline(schema, iters, step, f=synth.VOTER_FILTER):
    vid, pid = ml.sql_phase(schema["voters"], schema["precincts"], **f)
    rows, feats, vals, nf = ml.encode([vid, pid], 0, synth.voter_features(schema))
    row_ids, X = ml.design_matrix(rows, feats, vals, nf)
    y = schema["voters"]["voted"][row_ids]
    w, losses = ml.logreg(X, y, np.zeros(nf), iters, step)
    return vid, pid, (rows, feats, vals, nf), w, losses


@pytest.mark.parametrize("n,m,seed", [(3000, 40, 1), (60000, 2751, 2)])
def test_sql_phase_and_encoding_bit_exact(lh, pipeline, n, m, seed):
    say(f"voter sql+encode n={n} precincts={m} seed={seed}")
    d = synth.voter_schema(n, m, seed)
    t = pipeline.VoterTables(d, synth.voter_features(d))
    try:
        res = pipeline.sql_phase(t, **synth.VOTER_FILTER)
        host = res.to_host()
        vid, pid = ml.sql_phase(d["voters"], d["precincts"], **synth.VOTER_FILTER)
        assert np.array_equal(host["keys"][:, 0], vid) and np.array_equal(host["keys"][:, 1], pid)
        assert np.all(host["counts"] == 1)
        rows, feats, vals, nf = lh.encode(res.key_columns(), 0, t.features)
        res.free()
        want = ml.encode([vid, pid], 0, synth.voter_features(d))
        assert nf == want[3]
        assert np.array_equal(rows.cpu().numpy().view(np.uint32), want[0])
        assert np.array_equal(feats.cpu().numpy().view(np.uint32), want[1])
        assert np.array_equal(vals.cpu().numpy(), want[2])
    finally:
        t.free()


@pytest.mark.parametrize("n,m,seed,iters,step", [(5000, 60, 3, 5, 0.5), (100000, 2751, 4, 5, 0.5),
                                                 (20000, 300, 5, 12, 1.0)])
def test_voter_pipeline_matches_oracle(lh, pipeline, n, m, seed, iters, step):
    say(f"voter pipeline n={n} precincts={m} seed={seed} iters={iters}")
    d = synth.voter_schema(n, m, seed)
    t = pipeline.VoterTables(d, synth.voter_features(d))
    try:
        out = pipeline.run(t, iters=iters, step=step, **synth.VOTER_FILTER)
    finally:
        t.free()
    vid, _, _, w_ref, loss_ref = oracle_pipeline(d, iters, step)
    assert out["n_rows"] == len(vid)
    check_w(out["w"].cpu().numpy(), w_ref)
    np.testing.assert_allclose(out["loss"].cpu().numpy(), loss_ref, rtol=LOSS_RTOL)


def random_sparse(rng, n_rows, id_space, n_feat, long_rows=3, long_len=3000, dup=False):
    """Triples of a random sparse matrix over sparse row ids: most rows
    hold 1..20 entries, a few hold long_len, feature 0 is in every row
    (a list longer than one chunk); dup repeats some triples."""
    ids = np.sort(rng.choice(id_space, n_rows, replace=False)).astype(np.uint32)
    lens = rng.integers(1, 21, n_rows)
    lens[rng.choice(n_rows, long_rows, replace=False)] = long_len
    rows, feats = [], []
    for r, k in zip(ids, lens):
        f = rng.choice(np.arange(1, n_feat), min(k, n_feat - 1), replace=False)
        rows.append(np.full(len(f) + 1, r, np.uint32))
        feats.append(np.concatenate([[0], f]).astype(np.uint32))
    rows, feats = np.concatenate(rows), np.concatenate(feats)
    if dup:
        extra = rng.choice(len(rows), len(rows) // 5, replace=False)
        rows, feats = np.concatenate([rows, rows[extra]]), np.concatenate([feats, feats[extra]])
    vals = synth.uniform_pm1(rng, len(rows))
    perm = rng.permutation(len(rows))
    return rows[perm], feats[perm], vals[perm]


# many features over a wide row-id space take the chunked column pass; few
# features over a narrow one take the pass blocked by row id
@pytest.mark.parametrize("dup,n_feat,id_space", [(False, 4000, 1 << 20), (True, 4000, 1 << 20),
                                                 (False, 64, 1 << 16), (True, 64, 1 << 16)])
def test_logreg_on_random_sparse_tries(lh, pipeline, dup, n_feat, id_space):
    import torch
    rng = synth.rng_for(21 + dup + n_feat)
    rows, feats, vals = random_sparse(rng, 3000, id_space, n_feat, dup=dup)
    say(f"random sparse logreg dup={dup} n_feat={n_feat} nnz={len(rows)}")
    y_all = (rng.random(id_space) < 0.4).astype(np.float64)
    w0 = synth.uniform_pm1(rng, n_feat) * 0.1
    xr, xc = pipeline.design_tries(lh.to_device(rows), lh.to_device(feats), lh.to_device(vals))
    try:
        if not dup:
            assert xr.info()["level_size"][1] == len(rows)
        w = lh.to_device(w0)
        y = lh.to_device(y_all)
        loss = lh.logreg_fit(xr, xc, y, w, 5, 0.8).cpu().numpy()
        w_gpu = w.cpu().numpy()
        # the same call again repeats every bit
        w2 = lh.to_device(w0)
        loss2 = lh.logreg_fit(xr, xc, y, w2, 5, 0.8).cpu().numpy()
        assert np.array_equal(w2.cpu().numpy(), w_gpu) and np.array_equal(loss2, loss)
        # without the loss output the weights are the same
        w3 = lh.to_device(w0)
        assert lh.logreg_fit(xr, xc, y, w3, 5, 0.8, loss=False) is None
        assert np.array_equal(w3.cpu().numpy(), w_gpu)
    finally:
        xr.free()
        xc.free()
    row_ids, X = ml.design_matrix(rows, feats, vals, n_feat)
    w_ref, loss_ref = ml.logreg(X, y_all[row_ids], w0, 5, 0.8)
    check_w(w_gpu, w_ref)
    np.testing.assert_allclose(loss, loss_ref, rtol=LOSS_RTOL)
    del torch


def test_empty_selection_keeps_the_weights(lh, pipeline):
    import torch
    d = synth.voter_schema(2000, 30, 6)
    t = pipeline.VoterTables(d, synth.voter_features(d))
    try:
        w0 = torch.full((140,), 0.25, dtype=torch.float64, device="cuda")
        out = pipeline.run(t, iters=3, step=0.5, age_lo=0, age_hi=0, district_lo=0, district_hi=13, w0=w0)
    finally:
        t.free()
    assert out["n_rows"] == 0 and out["n_feat"] == 140
    assert np.all(out["w"].cpu().numpy() == 0.25)
    assert np.all(out["loss"].cpu().numpy() == 0.0)


def test_errors_are_reported(lh, pipeline):
    import torch
    rows = np.array([0, 0, 1, 2], np.uint32)
    feats = np.array([0, 3, 1, 2], np.uint32)
    vals = np.array([1.0, 0.5, -1.0, 2.0])
    xr, xc = pipeline.design_tries(lh.to_device(rows), lh.to_device(feats), lh.to_device(vals))
    same = lh.trie_build([rows, feats], annos=[vals], bag=True)
    try:
        y = torch.zeros(3, dtype=torch.float64, device="cuda")
        w = torch.zeros(4, dtype=torch.float64, device="cuda")
        with pytest.raises(lh.LHError):   # feature id 3 is not below n_feat = 3
            lh.logreg_fit(xr, xc, y, w[:3], 1, 0.5)
        with pytest.raises(lh.LHError):   # row id 2 is not below n_y = 2
            lh.logreg_fit(xr, xc, y[:2], w, 1, 0.5)
        with pytest.raises(lh.LHError):   # level orders are not swapped
            lh.logreg_fit(xr, same, y, w, 1, 0.5)
        with pytest.raises(lh.LHError):   # no annotation column 1
            lh.logreg_fit(xr, xc, y, w, 1, 0.5, anno=1)
        lh.logreg_fit(xr, xc, y, w, 1, 0.5)   # the valid call still works
    finally:
        xr.free()
        xc.free()
        same.free()
    ids = [lh.to_device(np.array([0, 1, 2], np.uint32))]
    with pytest.raises(lh.LHError):       # code 5 is not below card 3
        lh.encode(ids, 0, [{"codes": np.array([0, 5, 1], np.uint32), "card": 3, "by": 0}])
    with pytest.raises(lh.LHError):       # id 2 is not below the column's 2 entries
        lh.encode(ids, 0, [{"values": np.array([0.5, 1.5]), "by": 0}])
    lh.encode(ids, 0, [{"codes": np.array([0, 2, 1], np.uint32), "card": 3, "by": 0}])


def test_no_device_memory_leaks(lh, pipeline):
    before = lh.live_allocations()
    d = synth.voter_schema(3000, 40, 8)
    t = pipeline.VoterTables(d, synth.voter_features(d))
    out = pipeline.run(t, iters=2)
    t.free()
    del out
    assert lh.live_allocations() == before


def test_voter_pipeline_full_size(lh, pipeline):
    """The benchmark's workload (7,503,555 voters, 2,751 precincts, five
    iterations, step 0.5) against the oracle.  At this size the bound on
    the gradient's rounding error, n * eps * max|x| per iteration, is
    carried over the iterations: |dw| <= iters * step * n * eps * max|x|."""
    say("voter pipeline full size")
    d = synth.voter_schema(7_503_555, 2751, 7)
    t = pipeline.VoterTables(d, synth.voter_features(d))
    try:
        out = pipeline.run(t, iters=5, step=0.5, **synth.VOTER_FILTER)
    finally:
        t.free()
    vid, _, (rows, feats, vals, nf), w_ref, loss_ref = oracle_pipeline(d, 5, 0.5)
    assert out["n_rows"] == len(vid) and out["n_feat"] == nf
    bound = 5 * 0.5 * len(vid) * np.finfo(np.float64).eps * float(np.max(np.abs(vals)))
    err = np.abs(out["w"].cpu().numpy() - w_ref)
    assert np.all(err <= max(bound, W_TOL)), (float(err.max()), bound)
    np.testing.assert_allclose(out["loss"].cpu().numpy(), loss_ref, rtol=1e-10)
