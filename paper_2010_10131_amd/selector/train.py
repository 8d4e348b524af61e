"""Trains the solver selector's MLP on the timing database with the
library's own device kernels (forward, backward, Adam), and evaluates it on
the held-out 30 % (split 7:3 by shape, as Sec. IV-B splits its samples).

Writes the packed weights (as the C include compiled into the library and
as JSON) and an evaluation report: prediction accuracy, and the total time
of the chosen solvers against the exhaustive per-mode choice (regret),
always-EIG and always-ALS.

  python -m paper_2010_10131_amd.selector.train --db db.json --out-dir DIR
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

NI, NH, NO = 10, 32, 2
BIG = 1e30


def load_db(path):
    with open(path) as f:
        db = json.load(f)
    recs = [r for r in db["records"] if r.get("t_eig") is not None or r.get("t_als") is not None]
    return db["meta"], recs


def features(api, recs):
    return np.stack([api.selector_features(r["I"], r["R"], r["J"]) for r in recs], axis=1)


def targets(recs):
    te = np.array([r["t_eig"] if r.get("t_eig") is not None else BIG for r in recs])
    ta = np.array([r["t_als"] if r.get("t_als") is not None else BIG for r in recs])
    return te, ta


def split(recs, seed):
    shapes = sorted({r["shape"] for r in recs})
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(shapes))
    ntr = int(round(0.7 * len(shapes)))
    train = {shapes[i] for i in perm[:ntr]}
    tr = [i for i, r in enumerate(recs) if r["shape"] in train]
    te = [i for i, r in enumerate(recs) if r["shape"] not in train]
    return np.array(tr), np.array(te)


def init_params(seed, mu, isd):
    rng = np.random.default_rng(seed)

    def glorot(o, i):
        return (rng.standard_normal((o, i)) * np.sqrt(2.0 / (o + i))).astype(np.float32)
    parts = [glorot(NH, NI).T.ravel(), np.zeros(NH, np.float32), glorot(NH, NH).T.ravel(),
             np.zeros(NH, np.float32), glorot(NO, NH).T.ravel(), np.zeros(NO, np.float32),
             mu.astype(np.float32), isd.astype(np.float32)]
    return np.concatenate(parts).astype(np.float32)


def choose(api, recs, w):
    """0 = EIG, 1 = ALS: the library's own choice under solver="auto" (argmin
    of the predicted times, then the solvers' limits)."""
    return np.array([1 if api.selector_choose(r["I"], r["R"], r["J"], weights=w) == "als" else 0
                     for r in recs])


def evaluate(choice, te, ta):
    """Accuracy, totals and regret over the modes where both solvers have a
    time (a missing time is a solver beyond its limits or, for ALS, a
    non-finite result: R_n above the rank of the unfolding, which the shape
    features cannot see); those modes are counted separately."""
    best = np.minimum(te, ta)
    chosen = np.where(choice == 1, ta, te)
    valid = (te < BIG) & (ta < BIG)
    truth = (ta < te).astype(int)
    acc = float(np.mean(choice[valid] == truth[valid]))
    tot_best = float(best[valid].sum())
    tot_chosen = float(chosen[valid].sum())
    eig_ok = te < BIG
    als_ok = ta < BIG
    return {"accuracy": acc, "modes": int(valid.sum()),
            "modes_one_solver_only": int((eig_ok != als_ok).sum()),
            "chose_a_missing_solver": int(((choice == 1) & ~als_ok & eig_ok).sum()
                                          + ((choice == 0) & ~eig_ok & als_ok).sum()),
            "total_ms_exhaustive": tot_best, "total_ms_selected": tot_chosen,
            "regret": tot_chosen / tot_best - 1.0,
            "total_ms_always_eig": float(te[eig_ok].sum()) if eig_ok.all() else None,
            "total_ms_always_als": float(ta[als_ok].sum()) if als_ok.all() else None,
            "total_ms_always_eig_feasible": float(np.where(eig_ok, te, ta)[valid].sum()),
            "total_ms_always_als_feasible": float(np.where(als_ok, ta, te)[valid].sum())}


def report(api, recs, w, seed):
    """Accuracy and total times of the library's choices with weights w on
    the training and held-out records (host inference only)."""
    te_ms, ta_ms = targets(recs)
    tr, ho = split(recs, seed)
    return {"train_modes": int(len(tr)), "heldout_modes": int(len(ho)),
            "train": evaluate(choose(api, [recs[i] for i in tr], w), te_ms[tr], ta_ms[tr]),
            "heldout": evaluate(choose(api, [recs[i] for i in ho], w), te_ms[ho], ta_ms[ho])}


def write_inc(path, w):
    lines = ["// Selector weights written by paper_2010_10131_amd/selector/train.py from the",
             "// per-mode timing database measured on MI355X (see selector/report.json).",
             "static const bool kSelectorTrained = true;",
             "static const float kSelectorWeights[SEL_NPARAM] = {"]
    for i in range(0, len(w), 6):
        lines.append("    " + ", ".join(f"{float(x):.9e}f" for x in w[i:i + 6]) + ",")
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--db", required=True)
    ap.add_argument("--out-dir", required=True)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--eval-only", metavar="WEIGHTS_JSON",
                    help="recompute the evaluation of stored weights on the host (no training)")
    args = ap.parse_args()
    if args.eval_only:
        from paper_2010_10131_amd import api
        meta, recs = load_db(args.db)
        with open(args.eval_only) as f:
            w = np.array(json.load(f)["weights"], dtype=np.float32)
        path = os.path.join(args.out_dir, "report.json")
        old = {}
        if os.path.exists(path):
            with open(path) as f:
                old = json.load(f)
        old.update({"meta": meta, "seed": args.seed})
        old.update(report(api, recs, w, args.seed))
        with open(path, "w") as f:
            json.dump(old, f, indent=1)
        print(json.dumps({"train": old["train"], "heldout": old["heldout"]}, indent=1))
        return 0

    import torch

    from paper_2010_10131_amd import api

    meta, recs = load_db(args.db)
    X = features(api, recs)                       # 10 x n
    te_ms, ta_ms = targets(recs)
    both = (te_ms < BIG) & (ta_ms < BIG)
    Tl = np.stack([np.log(np.where(both, te_ms, 1.0)), np.log(np.where(both, ta_ms, 1.0))])
    tr, ho = split(recs, args.seed)
    # the network is fitted on the modes where both solvers ran: a mode one
    # solver cannot run is decided by the solvers' limits after the network
    # (apply_limits), so a made-up target for it would only cost capacity
    tr_fit = tr[both[tr]]
    mu = X[:, tr_fit].mean(axis=1)
    sd = X[:, tr_fit].std(axis=1)
    isd = 1.0 / np.maximum(sd, 1e-3)
    p = init_params(args.seed, mu, isd)
    dev = torch.device("cuda:0")

    def dcol(a):  # column-major device matrix of shape a.shape
        return torch.from_numpy(np.ascontiguousarray(a.T.astype(np.float32))).to(dev).t()

    Xtr, Ttr = dcol(X[:, tr_fit]), dcol(Tl[:, tr_fit])
    pd = torch.from_numpy(p).to(dev)
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    ntrain = api.selector_num_trainable()
    hist = []
    ws = None
    for step in range(1, args.steps + 1):
        loss, grad = api.mlp_loss_grad(pd, Xtr, Ttr, ws)
        lr = args.lr * (0.1 ** (step / args.steps))
        api.mlp_adam(pd, grad, m, v, ntrain, lr, step)
        if step % 500 == 0 or step == 1:
            hist.append((step, float(loss.item())))
            print(f"[train] step {step} loss {hist[-1][1]:.5f}", flush=True)
    w = pd.cpu().numpy()
    pred_ho = api.mlp_forward(pd, dcol(X[:, ho])).cpu().numpy()
    rep = {"meta": meta, "seed": args.seed, "steps": args.steps, "lr": args.lr,
           "loss_history": hist}
    rep.update(report(api, recs, w, args.seed))
    # host inference (used at plan time) must agree with the device network
    k = int(ho[0])
    host = api.selector_predict(recs[k]["I"], recs[k]["R"], recs[k]["J"], weights=w)
    rep["host_vs_device_max_abs"] = float(np.abs(host - pred_ho[:, 0]).max())
    os.makedirs(args.out_dir, exist_ok=True)
    write_inc(os.path.join(args.out_dir, "selector_weights.inc"), w)
    with open(os.path.join(args.out_dir, "weights.json"), "w") as f:
        json.dump({"weights": [float(x) for x in w]}, f)
    with open(os.path.join(args.out_dir, "report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    print(json.dumps({"train": rep["train"], "heldout": rep["heldout"]}, indent=1))


if __name__ == "__main__":
    sys.exit(main())
