"""What the trained cost model gains over the plain rule of section 4 on a
graph it never saw.

Triangle COUNT on an R-MAT graph with 2^20 vertices and 2^24 samples, seed
1020: the model's training set (`learned.training_queries`) holds other
seeds and sizes only.  Each policy runs the whole step (trie build with its
layouts, plan with its order, join, count read back), best of 3.  The counts
must be equal (the choices never change results), and the learned step must
not be slower than the plain one beyond a 5% timing margin.  The regret of
each policy against the best of every candidate (6 attribute orders x plain
or learned layouts, best of 2) is printed.
"""
import itertools
import sys
import time

import pytest

import synth

pytestmark = pytest.mark.gpu

SCALE, SAMPLES_LOG2, SEED = 20, 24, 1020
MARGIN = 1.05


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07859_amd import lh as binding
    return binding


def test_learned_model_gain_on_unseen_graph(lh):
    import torch

    from paper_1708_07859_amd import learned as L
    lm, om, meta = L.load(L.DEFAULT_WEIGHTS)
    trained_on = {r["query"] for r in meta.get("order_rows", [])}
    assert not any(q.startswith("triangle rmat20 seed %d" % SEED) for q in trained_on)
    lo, hi = synth.rmat_edges(SCALE, 1 << SAMPLES_LOG2, seed=SEED)
    lo_d, hi_d = lh.to_device(lo), lh.to_device(hi)

    def step(layout, policy, order=None):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = lh.trie_build([lo_d, hi_d], layout=layout)
        p = lh.plan(3, [(t, [0, 1], -1), (t, [1, 2], -1), (t, [0, 2], -1)], agg="count", attr_order=order,
                    policy=policy)
        r = lh.join_aggregate([p])[0]
        c = int(r.to_host()["counts"][0])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000
        chosen = p.info()["attr_order"]
        r.free()
        p.free()
        t.free()
        return ms, c, chosen

    def best(layout, policy, order=None, reps=3):
        runs = [step(layout, policy, order) for _ in range(reps)]
        assert len({r[1] for r in runs}) == 1
        return min(r[0] for r in runs), runs[0][1], runs[0][2]

    L.register(lm, om)
    try:
        step("plain", "plain")                      # warm-up
        t_plain, c_plain, o_plain = best("plain", "plain")
        t_learn, c_learn, o_learn = best("learned", "learned")
        cands = {}
        for layout in ("plain", "learned"):
            for order in itertools.permutations(range(3)):
                ms, c, _ = best(layout, "fixed", list(order), reps=2)
                assert c == c_plain
                cands[(layout, order)] = ms
    finally:
        lh.use_model(lh.LH_MODEL_LAYOUT, None)
        lh.use_model(lh.LH_MODEL_ORDER, None)
        lm.free()
        om.free()
    t_best = min(cands.values())
    say(f"unseen R-MAT {SCALE} seed {SEED}: {c_plain} triangles; plain {t_plain:.1f} ms (order {o_plain}), "
        f"learned {t_learn:.1f} ms (order {o_learn}); speedup {t_plain / t_learn:.2f}x; "
        f"regret plain {t_plain / t_best - 1:.1%}, learned {t_learn / t_best - 1:.1%} "
        f"(best candidate {t_best:.1f} ms: {min(cands, key=cands.get)})")
    assert c_learn == c_plain
    assert t_learn <= MARGIN * t_plain
