"""Tile autotuner of the batched path.

Times sthosvd_run_batched on the caller's resident batch under candidate
tile choices (sth_batch_tiles) and keeps the fastest.  The search is a
coordinate search: the Gram's split-K depth and tile cap first (with the
default TTM split), then the TTM rows per wave (with the best Gram choice).
Every candidate is run once untimed and checked for numerical flags before
it is timed, so a choice is only kept if its run is valid.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import torch

from .api import BatchPlan

DEFAULT = (4, 4, 4)
GRAM_WG_PER_CU = (2, 4, 8, 16, 32, 64)
GRAM_WT_MAX = (1, 2, 4)
TTM_ROWS_PER_WAVE = (1, 2, 4, 8)


def time_tiles(shapes, xp: torch.Tensor, gram_prec: str, ttm_prec: str, tiles, reps: int = 3,
               device="cuda") -> float:
    """Milliseconds per batched run with the given tiles (events on the current stream)."""
    plan = BatchPlan(shapes, gram_prec, ttm_prec, tiles=tiles)
    G, U, cp, up = plan.outputs(device)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=device)
    plan.run(xp, cp, up, ws)
    plan.check(ws)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.run(xp, cp, up, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    plan.check(ws)
    del plan, G, U, cp, up, ws
    return ms


def tune_batched(shapes: Sequence, xp: torch.Tensor, gram_prec: str = "bf16x6",
                 ttm_prec: str = "bf16x3", reps: int = 3,
                 device="cuda") -> Tuple[Tuple[int, int, int], float, List[dict]]:
    """(best tiles, its ms per run, every timed candidate)."""
    table: List[dict] = []
    seen = {}

    def measure(t):
        t = tuple(int(v) for v in t)
        if t not in seen:
            seen[t] = time_tiles(shapes, xp, gram_prec, ttm_prec, t, reps, device)
            table.append({"gram_wg_per_cu": t[0], "gram_wt_max": t[1], "ttm_rows_per_wave": t[2],
                          "ms": seen[t]})
        return seen[t]

    best = DEFAULT
    best_ms = measure(best)
    for wg in GRAM_WG_PER_CU:
        for wt in GRAM_WT_MAX:
            ms = measure((wg, wt, best[2]))
            if ms < best_ms:
                best, best_ms = (wg, wt, best[2]), ms
    for rpw in TTM_ROWS_PER_WAVE:
        ms = measure((best[0], best[1], rpw))
        if ms < best_ms:
            best, best_ms = (best[0], best[1], rpw), ms
    return best, best_ms, table
