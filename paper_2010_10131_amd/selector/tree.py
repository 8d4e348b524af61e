"""The decision-tree solver selector of Sec. IV-B, trained on the same
per-mode timing database as the MLP.

Each mode of the database is a sample: the ten Table I features (taken as
their logarithms, the library's feature vector; a tree depends only on the
order of each feature, so the splits are those of the raw features) and the
label "the faster solver" (the one that ran, where only one did).  The tree
is grown by CART: every node takes the axis-aligned split "feature <=
threshold" of largest decrease of the weighted Gini impurity, until the
depth limit or a pure node.  As in Sec. IV-B, max_depth is searched over
1..10 and the class weights over {uniform, balanced} by cross-validated grid
search (5 folds over the training shapes, accuracy), and the winner is
refitted on the whole 70 % training split.  The tree is written as flat node
arrays for the library's host inference (solver = auto_tree).

  python -m paper_2010_10131_amd.selector.tree --db db.json --out-dir DIR
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

from paper_2010_10131_amd.selector import train as T


def gini_tree(X, y, w, max_depth):
    """CART on features X (n x d, float32), labels y in {0, 1}, sample
    weights w.  Returns node arrays (feature, threshold, left, right, cls);
    a leaf has feature -1.  A split sends x[f] <= threshold left; the
    threshold is the larger training value on the left side, so the
    training partition is reproduced exactly in float32."""
    feat, thr, left, right, cls = [], [], [], [], []

    def leaf_class(idx):
        c1 = w[idx][y[idx] == 1].sum()
        c0 = w[idx][y[idx] == 0].sum()
        return 1 if c1 > c0 else 0

    def best_split(idx):
        ws = w[idx]
        tot = ws.sum()
        tot1 = (ws * y[idx]).sum()
        parent = tot * (1.0 - (tot1 / tot) ** 2 - (1.0 - tot1 / tot) ** 2)
        best = (parent - 1e-12 * tot, -1, 0.0)   # a split must lower the impurity
        for f in range(X.shape[1]):
            xs = X[idx, f]
            order = np.argsort(xs, kind="stable")
            xo, wo, yo = xs[order], ws[order], y[idx][order]
            cw = np.cumsum(wo)[:-1]
            c1 = np.cumsum(wo * yo)[:-1]
            valid = xo[:-1] < xo[1:]   # split only between distinct values
            if not valid.any():
                continue
            rw = tot - cw
            r1 = tot1 - c1
            with np.errstate(divide="ignore", invalid="ignore"):
                gl = cw * (1.0 - (c1 / cw) ** 2 - (1.0 - c1 / cw) ** 2)
                gr = rw * (1.0 - (r1 / rw) ** 2 - (1.0 - r1 / rw) ** 2)
            g = np.where(valid, gl + gr, np.inf)
            k = int(np.argmin(g))
            if g[k] < best[0]:
                best = (g[k], f, float(xo[k]))
        return best

    def grow(idx, depth):
        node = len(feat)
        feat.append(-1)
        thr.append(0.0)
        left.append(-1)
        right.append(-1)
        cls.append(leaf_class(idx))
        if depth >= max_depth or len(np.unique(y[idx])) < 2:
            return node
        _, f, t = best_split(idx)
        if f < 0:
            return node
        go_left = X[idx, f] <= np.float32(t)
        feat[node] = f
        thr[node] = t
        left[node] = grow(idx[go_left], depth + 1)
        right[node] = grow(idx[~go_left], depth + 1)
        return node

    grow(np.arange(len(y)), 0)
    return {"feature": feat, "threshold": thr, "left": left, "right": right, "cls": cls}


def tree_predict(tree, X):
    out = np.empty(len(X), dtype=int)
    thr = np.asarray(tree["threshold"], dtype=np.float32)
    for i, x in enumerate(X):
        k = 0
        while tree["feature"][k] >= 0:
            k = tree["left"][k] if x[tree["feature"][k]] <= thr[k] else tree["right"][k]
        out[i] = tree["cls"][k]
    return out


# The library applies the solvers' limits after either model (selector.h):
# ALS needs R_n <= 128 and R_n <= J_n (the rank bound of the unfolding); EIG
# needs I_n <= 512; above order 128 with R_n in 125..128 the plan takes ALS
# where it can (EIG would run the direct solver on the whole Gram).
def apply_limits(choice, recs):
    out = np.array(choice, dtype=int)
    for i, r in enumerate(recs):
        I, R, J = r["I"], r["R"], r["J"]
        als_ok = R <= 128 and R <= J
        if out[i] == 1 and not als_ok:
            out[i] = 0
        if out[i] == 0 and I > 128 and 124 < R <= 128 and als_ok:
            out[i] = 1
        if out[i] == 0 and I > 512 and als_ok:
            out[i] = 1
    return out


def class_weights(y, mode):
    if mode == "uniform":
        return np.ones(len(y))
    n, n1 = len(y), int(y.sum())
    c = np.array([n / (2.0 * max(n - n1, 1)), n / (2.0 * max(n1, 1))])
    return c[y]


def labels(recs):
    te, ta = T.targets(recs)
    return (ta < te).astype(int), te, ta


def grid_search(X, y, shapes, depths=range(1, 11), weights=("uniform", "balanced"), folds=5, seed=7):
    """Mean 5-fold cross-validated accuracy of every (max_depth, class
    weight); folds are drawn over shapes, so the modes of one tensor stay
    together.  Returns the best pair and the table."""
    us = np.unique(shapes)
    rng = np.random.default_rng(seed)
    fold_of = dict(zip(us[rng.permutation(len(us))], np.arange(len(us)) % folds))
    fid = np.array([fold_of[s] for s in shapes])
    table = {}
    for wm in weights:
        for d in depths:
            acc = []
            for k in range(folds):
                tr, va = fid != k, fid == k
                t = gini_tree(X[tr], y[tr], class_weights(y[tr], wm), d)
                acc.append(float(np.mean(tree_predict(t, X[va]) == y[va])))
            table[f"{wm}/{d}"] = float(np.mean(acc))
    best = max(table, key=lambda k: (table[k], -int(k.split("/")[1])))
    wm, d = best.split("/")
    return wm, int(d), table


def write_inc(path, tree):
    n = len(tree["feature"])
    f32 = [float(np.float32(t)) for t in tree["threshold"]]
    lines = ["// Decision-tree selector written by paper_2010_10131_amd/selector/tree.py from the",
             "// per-mode timing database measured on MI355X (see selector/tree_report.json).",
             "// Node k: leaf when kTreeFeature[k] < 0 (class kTreeClass[k]: 0 = EIG, 1 = ALS),",
             "// otherwise feature <= kTreeThreshold[k] goes to kTreeLeft[k], else kTreeRight[k].",
             f"static const int kTreeNodes = {n};",
             "static const int kTreeFeature[] = {" + ", ".join(str(x) for x in tree["feature"]) + "};",
             "static const float kTreeThreshold[] = {" + ", ".join(f"{x:.9e}f" for x in f32) + "};",
             "static const int kTreeLeft[] = {" + ", ".join(str(x) for x in tree["left"]) + "};",
             "static const int kTreeRight[] = {" + ", ".join(str(x) for x in tree["right"]) + "};",
             "static const int kTreeClass[] = {" + ", ".join(str(x) for x in tree["cls"]) + "};"]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--db", required=True)
    ap.add_argument("--out-dir", required=True)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()
    from paper_2010_10131_amd import api
    meta, recs = T.load_db(args.db)
    X = T.features(api, recs).T.astype(np.float32)   # n x 10
    y, te, ta = labels(recs)
    tr, ho = T.split(recs, args.seed)
    shapes = np.array([r["shape"] for r in recs])
    wm, d, table = grid_search(X[tr], y[tr], shapes[tr], seed=args.seed)
    tree = gini_tree(X[tr], y[tr], class_weights(y[tr], wm), d)
    rep = {"meta": meta, "seed": args.seed, "class_weight": wm, "max_depth": d,
           "nodes": len(tree["feature"]), "cv_accuracy": table,
           "train": T.evaluate(apply_limits(tree_predict(tree, X[tr]), [recs[i] for i in tr]), te[tr], ta[tr]),
           "heldout": T.evaluate(apply_limits(tree_predict(tree, X[ho]), [recs[i] for i in ho]), te[ho], ta[ho])}
    os.makedirs(args.out_dir, exist_ok=True)
    write_inc(os.path.join(args.out_dir, "selector_tree.inc"), tree)
    with open(os.path.join(args.out_dir, "tree.json"), "w") as f:
        json.dump(tree, f)
    with open(os.path.join(args.out_dir, "tree_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    print(json.dumps({k: rep[k] for k in ("class_weight", "max_depth", "nodes", "train", "heldout")}, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
