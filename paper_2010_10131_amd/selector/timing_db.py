"""Per-mode timing database for the solver selector (the procedure of
Sec. IV-B, on this GPU): random tensor shapes are decomposed mode by mode and
both the EIG and the ALS step of Alg. 2 are timed on the same working tensor.
One record per (shape, mode): the shape features I_n, R_n, J_n (on the current
working tensor) and the median times of both solvers.

The tensors have the structure Tucker is run on: multilinear rank equal to
the target ranks plus 1e-4 relative Gaussian noise (the workloads' recipe).
The eigensolver's time depends on the Gram's spectrum (how many Jacobi
sweeps it takes), which the shape features cannot see, so the database is
measured on the kind of spectrum the selector will meet; --data gaussian
fills the tensors with plain Gaussian values instead.

  python -m paper_2010_10131_amd.selector.timing_db --count 2000 --out db.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def random_shapes(count: int, seed: int, max_elems: int, dmin=16, dmax=512, rmin=0.05, rmax=0.5):
    """3-5 way shapes, dims log-uniform in [dmin, dmax], rank ratio uniform in
    [rmin, rmax]; shapes above max_elems are redrawn (as the paper drops what
    does not fit)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        N = int(rng.integers(3, 6))
        dims = [int(round(np.exp(rng.uniform(np.log(dmin), np.log(dmax))))) for _ in range(N)]
        if np.prod(dims, dtype=np.float64) > max_elems:
            continue
        ranks = [max(1, int(round(rng.uniform(rmin, rmax) * d))) for d in dims]
        out.append((dims, ranks))
    return out


def time_step(api, torch, Y, n, R, solver, gp, tp, reps, ws_cache, budget_ms=60.0):
    """Median time (ms) of one mode step; a step slower than budget_ms is
    timed once."""
    st = torch.cuda.Event(enable_timing=True)
    en = torch.cuda.Event(enable_timing=True)
    times = []
    for r in range(reps + 1):
        st.record()
        Z, U, ev, ws = api.mode_step(Y, n, R, solver, gp, tp, workspace=ws_cache.get(solver))
        en.record()
        en.synchronize()
        ws_cache[solver] = ws
        t = st.elapsed_time(en)
        if r > 0 or t > budget_ms:
            times.append(t)
        if t > budget_ms:
            break
    return float(np.median(times)), Z


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=20101013 + 10)
    ap.add_argument("--max-elems", type=int, default=1 << 27)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--gram-prec", default="bf16x6")
    ap.add_argument("--ttm-prec", default="bf16x3")
    ap.add_argument("--data", choices=("lowrank", "gaussian"), default="lowrank")
    ap.add_argument("--noise", type=float, default=1e-4)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    import torch

    from paper_2010_10131_amd import api
    from paper_2010_10131_amd._lib import SthError

    dev = torch.device("cuda:0")
    shapes = random_shapes(args.count, args.seed, args.max_elems)
    recs = []
    t0 = time.time()
    ws_cache = {}
    for si, (dims, ranks) in enumerate(shapes):
        if args.data == "lowrank":
            import workloads
            Y = workloads.lowrank_plus_noise_device(dims, ranks, nu=args.noise, seed=args.seed + si, device=dev)
        else:
            g = torch.Generator(device=dev)
            g.manual_seed(args.seed + si)
            Y = torch.randn(tuple(dims[::-1]), generator=g, device=dev, dtype=torch.float32)
            Y = Y.permute(*range(len(dims) - 1, -1, -1))
        cur = list(dims)
        for n in range(len(dims)):
            R = ranks[n]
            I = cur[n]
            J = int(np.prod(cur)) // I
            rec = {"shape": si, "order": len(dims), "mode": n, "I": I, "R": R, "J": J}
            Ynext = None
            for solver in ("eig", "als"):
                try:
                    t, Z = time_step(api, torch, Y, n, R, solver, args.gram_prec, args.ttm_prec,
                                     args.reps, ws_cache)
                    rec["t_" + solver] = t
                except SthError as e:      # e.g. ALS with R_n above its limit
                    rec["t_" + solver] = None
                    rec["err_" + solver] = str(e)
                    Z = None
                if Z is not None and not bool(torch.isfinite(Z).all()):
                    # e.g. ALS with R_n above the rank of the unfolding: its
                    # normal equations are singular; the solver is not an option
                    rec["t_" + solver] = None
                    rec["err_" + solver] = "non-finite result"
                    Z = None
                if Z is not None and Ynext is None:
                    Ynext = Z              # the EIG result when there is one
            recs.append(rec)
            if Ynext is None:
                break
            Y = Ynext
            cur[n] = R
        if si % 100 == 0 or si + 1 == len(shapes):
            print(f"[timing_db] {si + 1}/{len(shapes)} shapes, {time.time() - t0:.0f}s", flush=True)
            ws_cache.clear()
            torch.cuda.empty_cache()
            # written as it goes, so that a run cut short still leaves its records
            meta = {"count": si + 1, "requested": args.count, "seed": args.seed,
                    "data": args.data, "noise": args.noise if args.data == "lowrank" else None,
                    "max_elems": args.max_elems, "gram_prec": args.gram_prec,
                    "ttm_prec": args.ttm_prec, "reps": args.reps,
                    "device": torch.cuda.get_device_name(0), "seconds": time.time() - t0}
            with open(args.out, "w") as f:
                json.dump({"meta": meta, "records": recs}, f)
    print(f"[timing_db] wrote {len(recs)} records in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    sys.exit(main())
