"""The decision-tree selector (Sec. IV-B's model): the CART trainer against
small cases with a known answer and against scikit-learn's CART (an
independent implementation of the same greedy Gini rule), the compiled-in
tree against the trainer's own predictions on every database record, and
its held-out gain over the fixed choices.  Host only."""
import json
import os

import numpy as np
import pytest

from paper_2010_10131_amd.selector import train as T
from paper_2010_10131_amd.selector import tree as TR

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(HERE, "..", "paper_2010_10131_amd", "selector", "data")


def test_stump_splits_a_separable_feature_at_the_gap():
    X = np.array([[1], [2], [3], [4], [5], [6]], dtype=np.float32)
    y = np.array([0, 0, 0, 1, 1, 1])
    t = TR.gini_tree(X, y, np.ones(6), 1)
    assert t["feature"][0] == 0 and t["threshold"][0] == 3.0
    assert t["cls"][t["left"][0]] == 0 and t["cls"][t["right"][0]] == 1
    assert (TR.tree_predict(t, X) == y).all()


def test_depth_two_learns_a_conjunction_depth_one_cannot():
    rng = np.random.default_rng(0)
    X = rng.random((400, 2)).astype(np.float32)
    y = ((X[:, 0] > 0.5) & (X[:, 1] > 0.5)).astype(int)
    acc1 = np.mean(TR.tree_predict(TR.gini_tree(X, y, np.ones(400), 1), X) == y)
    acc2 = np.mean(TR.tree_predict(TR.gini_tree(X, y, np.ones(400), 2), X) == y)
    assert acc2 == 1.0 and acc1 < 0.9


def test_pure_node_and_no_gain_make_leaves():
    X = np.array([[0, 0], [0, 1], [1, 0], [1, 1]], dtype=np.float32)
    t = TR.gini_tree(X, np.array([1, 1, 1, 1]), np.ones(4), 5)
    assert t["feature"] == [-1] and t["cls"] == [1]
    # XOR: no single axis split lowers the Gini impurity, so greedy CART stops
    t = TR.gini_tree(X, np.array([0, 1, 1, 0]), np.ones(4), 5)
    assert t["feature"] == [-1]


def test_balanced_class_weights():
    y = np.array([0, 0, 0, 1])
    w = TR.class_weights(y, "balanced")
    np.testing.assert_allclose(w, [4 / 6, 4 / 6, 4 / 6, 2.0])
    assert w[y == 0].sum() == pytest.approx(w[y == 1].sum())


@pytest.fixture(scope="module")
def db():
    from paper_2010_10131_amd import api
    _, recs = T.load_db(os.path.join(DATA, "timing_db.json"))
    X = T.features(api, recs).T.astype(np.float32)
    y, te, ta = TR.labels(recs)
    return recs, X, y, te, ta


@pytest.mark.parametrize("weights", ["uniform", "balanced"])
def test_cart_matches_scikit_learn_training_accuracy(db, weights):
    sk = pytest.importorskip("sklearn.tree")
    recs, X, y, _, _ = db
    for d in (1, 2, 4, 6, 8):
        ours = TR.tree_predict(TR.gini_tree(X, y, TR.class_weights(y, weights), d), X)
        ref = sk.DecisionTreeClassifier(criterion="gini", max_depth=d, random_state=0,
                                        class_weight=None if weights == "uniform" else "balanced")
        ref.fit(X, y)
        a, b = np.mean(ours == y), np.mean(ref.predict(X) == y)
        # the same greedy rule; only the choice among equally good splits
        # (features with the same order, e.g. I and I^2) may differ
        assert abs(a - b) <= 0.005, (d, a, b)


def test_compiled_in_tree_is_the_trained_one(db):
    from paper_2010_10131_amd import api
    recs, X, _, _, _ = db
    with open(os.path.join(DATA, "tree.json")) as f:
        tree = json.load(f)
    want = TR.apply_limits(TR.tree_predict(tree, X), recs)
    got = np.array([1 if api.selector_tree_choose(r["I"], r["R"], r["J"]) == "als" else 0 for r in recs])
    assert (got == want).all(), int((got != want).sum())


def test_tree_beats_both_fixed_choices_on_heldout(db):
    from paper_2010_10131_amd import api
    recs, _, _, te, ta = db
    with open(os.path.join(DATA, "tree_report.json")) as f:
        rep = json.load(f)
    _, ho = T.split(recs, rep["seed"])
    choice = np.array([1 if api.selector_tree_choose(recs[i]["I"], recs[i]["R"], recs[i]["J"]) == "als" else 0
                       for i in ho])
    ev = T.evaluate(choice, te[ho], ta[ho])
    assert ev["accuracy"] == pytest.approx(rep["heldout"]["accuracy"])
    assert ev["total_ms_selected"] <= min(ev["total_ms_always_eig_feasible"], ev["total_ms_always_als_feasible"])
    assert ev["total_ms_selected"] < 0.5 * ev["total_ms_always_als_feasible"]
    assert ev["regret"] <= 0.02 and ev["accuracy"] >= 0.936


def test_plan_auto_tree_uses_the_tree():
    import torch
    from paper_2010_10131_amd import api
    for dims, ranks in [((64, 64, 64), (8, 8, 8)), ((48,) * 5, (8,) * 5), ((300, 40, 30), (126, 8, 8))]:
        p = api.Plan(dims, ranks, torch.float32, "bf16x6", "bf16x3", "auto_tree")
        cur = list(dims)
        for n in range(len(dims)):
            J = int(np.prod(cur)) // cur[n]
            assert ["eig", "als"][p.solvers[n]] == api.selector_tree_choose(cur[n], ranks[n], J)
            cur[n] = ranks[n]
