"""The learned cost model on the GPU: FP32 gradients against the FP64
reference, BF16 inference against the reference's bf16 arithmetic,
training, and decisions that change plans but never results."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as ref
from tests import queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh as binding
    return binding


@pytest.fixture(autouse=True)
def no_models(lh):
    yield
    lh.use_model(lh.LH_MODEL_LAYOUT, None)
    lh.use_model(lh.LH_MODEL_ORDER, None)


@pytest.mark.parametrize("d,n", [(4, 33), (24, 200)])
def test_gradients_match_fp64_reference(lh, d, n):
    m = lh.Mlp(d, 64, seed=3)
    rng = synth.rng_for(d + n)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    y = rng.normal(0, 2, n).astype(np.float32)
    loss, g = m.loss_grad(X, y)
    p = m.get_params().astype(np.float64)
    want_loss, want_g = ref.loss_grad(p, X.astype(np.float64), y.astype(np.float64))
    assert abs(loss - want_loss) <= 1e-4 * max(1.0, want_loss)
    scale = np.abs(want_g).max()
    assert np.abs(g - want_g).max() <= 1e-4 * scale


def test_bf16_inference(lh):
    d = 24
    m = lh.Mlp(d, 64, seed=5)
    rng = synth.rng_for(6)
    X = rng.normal(0, 1, (500, d)).astype(np.float32)
    y16 = m.predict(X, bf16=True)
    y32 = m.predict(X, bf16=False)
    p = m.get_params()
    want16 = ref.forward_bf16(p, X)
    want64 = ref.forward(p.astype(np.float64), X.astype(np.float64))
    scale = np.abs(want64).max()
    assert np.abs(y32 - want64).max() <= 1e-4 * scale
    # same bf16 roundings, fp32 sums in a different order: a few bf16 ulps
    assert np.abs(y16 - want16).max() <= 2 ** -6 * scale
    # against full precision: three bf16 roundings of ~2^-8 relative each
    assert np.abs(y16 - want64).max() <= 2 ** -4 * scale


@pytest.mark.parametrize("d,n,steps,lr", [(4, 64, 10, 1e-3), (24, 96, 25, 3e-3)])
def test_adam_training_matches_fp64_reference(lh, d, n, steps, lr):
    # one batch holding every sample: each epoch is one Adam step on the
    # full-batch gradient, so the GPU's FP32 forward, backward and Adam
    # kernels follow the reference's FP64 trajectory step for step
    rng = synth.rng_for(100 + d)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    y = (X[:, 0] - 0.5 * X[:, 1] + 0.25 * rng.normal(0, 1, n)).astype(np.float32)
    m = lh.Mlp(d, 64, seed=7)
    p0 = m.get_params().astype(np.float64)
    m.train(X, y, epochs=steps, batch=n, lr=lr, seed=1)
    got = m.get_params().astype(np.float64)
    want, losses = ref.train_full_batch(p0, X.astype(np.float64), y.astype(np.float64), steps, lr)
    dg, dw = got - p0, want - p0
    # Adam's bound on one step: lr * (1 - b1) / sqrt(1 - b2) < 3.2 lr
    assert np.abs(dg).max() <= 3.2 * steps * lr
    # the update agrees with the reference's to FP32 accuracy, in norm; a
    # parameter whose gradient is near zero may differ by its whole step
    # (Adam normalizes the gradient's sign), so those are bounded apart
    err = np.linalg.norm(dg - dw) / np.linalg.norm(dw)
    print(f"adam d={d} n={n} steps={steps}: relative update error {err:.2e}, "
          f"max |diff| {np.abs(dg - dw).max():.2e} (lr {lr})")
    assert err <= 1e-3
    assert ref.loss(got, X, y) < losses[0]


def test_training_fits_a_cost_surface(lh):
    rng = synth.rng_for(9)
    X = rng.uniform(0, 1, (2000, 4)).astype(np.float32) * np.array([17, 22, 1, 1], np.float32)
    X[:, 3] = np.round(X[:, 3])
    # a smooth synthetic log-cost: log-depth search vs constant probe
    y = np.where(X[:, 3] > 0.5, 1.0 + 0.1 * X[:, 1], 2.0 + np.log2(1 + X[:, 0])).astype(np.float32)
    m = lh.Mlp(4, 64, seed=11)
    loss0, _ = m.loss_grad(X, y)
    loss = m.train(X, y, epochs=150, batch=128, lr=3e-3, seed=2)
    assert loss < 0.02 * loss0
    pred = m.predict(X, bf16=True)
    assert np.sqrt(np.mean((pred - y) ** 2)) < 0.25


def test_learned_layout_changes_layouts_not_results(lh):
    # a model that always prefers bitsets: probe cost 0 for bitsets, 10 for uint
    m = lh.Mlp(4, 64, seed=1)
    p = np.zeros(m.n_params, np.float32)
    # output = 10 - 10 * choice: W1 row 0 copies the choice feature, W2 passes it
    H, d = 64, 4
    W1 = np.zeros((H, d), np.float32); W1[0, 3] = 1.0
    W2 = np.zeros((H, H), np.float32); W2[0, 0] = 1.0
    W3 = np.zeros((1, H), np.float32); W3[0, 0] = -10.0
    p[:] = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), [10.0]])
    m.set_params(p)
    lh.use_model(lh.LH_MODEL_LAYOUT, m)
    lo, hi = synth.rmat_edges(14, 16 << 14, seed=3)
    t_plain = lh.trie_build([lo, hi], layout="plain")
    t_learn = lh.trie_build([lo, hi], layout="learned")
    assert sum(t_learn.info()["level_bitsets"]) > sum(t_plain.info()["level_bitsets"])
    q = queries.triangle(lo, hi)
    want = oracle.join_aggregate(q)["counts"][0]
    assert lh.run_query(q, layout="learned")["counts"][0] == want
    assert lh.run_query(q, layout="plain")["counts"][0] == want


def test_learned_order_is_the_models_argmin_and_exact(lh):
    a = synth.sparse_matrix(500, 8, seed=2)
    b = synth.sparse_matrix(500, 8, seed=3)
    q = queries.spgemm(a, b)
    want = oracle.join_aggregate(q)
    # a model that scores each order by its first position's icost feature
    # (feature 5): any order with icost 0 there is "cheapest"
    def model(scale):
        # prediction = scale x the second position's icost feature (feature 5)
        m = lh.Mlp(24, 64, seed=1)
        H, d = 64, 24
        W1 = np.zeros((H, d), np.float32); W1[0, 5] = 1.0
        W2 = np.zeros((H, H), np.float32); W2[0, 0] = 1.0
        W3 = np.zeros((1, H), np.float32); W3[0, 0] = scale
        m.set_params(np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), [0.0]]))
        return m
    plain = lh.run_query(q, return_plan_info=True)["plan"]["attr_order"]
    assert plain == [0, 1, 2]
    m = model(10.0)
    lh.use_model(lh.LH_MODEL_ORDER, m)
    got = lh.run_query(q, policy="learned", return_plan_info=True)
    # candidates: [0,2,1], [0,1,2] (relaxed), [2,0,1], [2,1,0]; second-position
    # icost is 0 for [0,2,1] and [2,0,1], so the tie goes to [0,2,1], which
    # the model scores well past the plain order's
    assert got["plan"]["attr_order"] == [0, 2, 1]
    assert np.array_equal(got["keys"], want["keys"])
    assert np.array_equal(got["sums"].view(np.uint64), want["sums"].view(np.uint64))
    # the same preference a hundred times weaker is within the model's
    # margin: the plain rule's order stays
    m2 = model(0.1)
    lh.use_model(lh.LH_MODEL_ORDER, m2)
    assert lh.run_query(q, policy="learned", return_plan_info=True)["plan"]["attr_order"] == plain


@pytest.mark.parametrize("kind", ["spmv", "spgemm", "triangle"])
def test_training_features_match_the_plan(lh, kind):
    """The features the training script records for a candidate order are
    the ones the plan scores: with the committed weights, the decision taken
    from the training script's features (the order model's prediction on
    every candidate, the plain order kept unless beaten by the margin of
    2^0.5) is the plan's own, and the plain rule's order computed from those
    features is the plain plan's.  SpMV holds a completely dense vector
    relation, which both sides must leave out of the set features."""
    from paper_1708_07859_amd import learned as L
    rng = synth.rng_for(77)
    if kind == "spmv":
        n = 6000
        q = queries.spmv(synth.zipf_degree_matrix(n, 1.1, 16, rng), synth.uniform_pm1(rng, n))
    elif kind == "spgemm":
        a = synth.zipf_degree_matrix(3000, 1.1, 16, rng)
        q = queries.spgemm(a, a)
    else:
        lo, hi = synth.rmat_edges(14, 16 << 14, seed=77)
        q = queries.triangle(lo, hi)
    lm, om, _ = L.load(L.DEFAULT_WEIGHTS)
    tries, uniq = L.build_tries(q)
    try:
        edges = L._edges_of(q, tries)
        out = q.get("out", [])
        plain, _ = lh.choose_order(q["n_attrs"], edges, out)
        cands = L.candidate_orders(q["n_attrs"], out)
        if plain not in cands:
            cands.append(plain)
        X = np.stack([lh.order_features(q["n_attrs"], edges, o) for o in cands])
        y = om.predict(X, bf16=True)
        best = min(range(len(cands)), key=lambda c: (y[c], cands[c]))
        want = cands[best] if y[cands.index(plain)] - y[best] >= 0.5 else plain
        atoms = [(t, list(a["attrs"]), int(a.get("anno", -1))) for t, a in zip(tries, q["atoms"])]
        p = lh.plan(q["n_attrs"], atoms, out=out, agg=q["agg"], policy="plain")
        assert p.info()["attr_order"] == plain
        p.free()
        L.register(lm, om)
        p = lh.plan(q["n_attrs"], atoms, out=out, agg=q["agg"], policy="learned")
        got = p.info()["attr_order"]
        p.free()
        assert got == want, (kind, got, want, dict(zip(map(tuple, cands), y.tolist())))
    finally:
        lh.use_model(lh.LH_MODEL_LAYOUT, None)
        lh.use_model(lh.LH_MODEL_ORDER, None)
        for t in uniq:
            t.free()
        lm.free()
        om.free()
