"""Batched path: every tensor of a batch equals its single-tensor run and the
FP64 oracle (T1/T2), and a HIP-graph capture of the batched run replays to
the eager result bit for bit."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

# mixed shapes: first-mode I % 4 != 0, orders <= 128 (matrix in LDS) and
# > 128 (matrix in the workspace), small and large ranks, a mode of size < 32
SHAPES = [((40, 36, 33), (4, 5, 6)), ((37, 60, 50), (6, 8, 5)), ((130, 40, 35), (16, 6, 5)),
          ((200, 150, 33), (30, 20, 5)), ((64, 256, 40), (10, 40, 8)), ((96, 96, 96), (12, 12, 12)),
          ((33, 20, 150), (5, 4, 18)), ((250, 60, 32), (60, 9, 5)),
          ((120, 50, 40), (12, 6, 5)), ((110, 4, 5), (25, 3, 4))]
# ((110, 4, 5), ...): R_1 = 25 exceeds the rank bound 20 of the mode-1 Gram;
# ((33, 20, 150), (5, 4, 18)): the mode-3 Gram has rank <= 5 * 4 = 20 > 18


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    from paper_2010_10131_amd import api as a
    return a


def make_batch(api, shapes, seed=5):
    import torch
    xs = [wl.lowrank_plus_noise(d, r, "none", 1e-4, seed + t, "float32") for t, (d, r) in enumerate(shapes)]
    xd = [api.to_device(x) for x in xs]
    xp = torch.tensor([x.data_ptr() for x in xd], dtype=torch.int64, device="cuda")
    return xs, xd, xp


def recon(api, G, U):
    return oracle.reconstruct(api.to_numpy(G), [api.to_numpy(u) for u in U])


@pytest.mark.parametrize("gp,tp", [("fp64", "fp32"), ("bf16x6", "bf16x3")])
def test_batched_equals_single_and_oracle(api, gp, tp):
    import torch
    xs, xd, xp = make_batch(api, SHAPES)
    plan = api.BatchPlan(SHAPES, gp, tp)
    G, U, cp, up = plan.outputs()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(xp, cp, up, ws)
    plan.check(ws)
    for t, (d, r) in enumerate(SHAPES):
        Xh = recon(api, G[t], U[t])
        Gs, Us, _ = api.sthosvd(xd[t], r, gp, tp)
        Xs = recon(api, Gs, Us)
        Go, Uo, _ = oracle.sthosvd(xs[t], r)
        Xo = oracle.reconstruct(Go, Uo)
        xn = np.linalg.norm(xs[t].astype(np.float64))
        t2_single = np.linalg.norm(Xh - Xs) / xn
        t2_oracle = np.linalg.norm(Xh - Xo) / xn
        t1 = abs(np.linalg.norm(api.to_numpy(G[t])) - np.linalg.norm(Go)) / np.linalg.norm(Go)
        assert t2_single <= 1e-5 and t2_oracle <= 1e-5 and t1 <= 1e-5, (t, d, r, t2_single, t2_oracle, t1)
        for n in range(3):
            u = api.to_numpy(U[t][n])
            np.testing.assert_allclose(u.T @ u, np.eye(r[n]), atol=1e-10)


def test_batched_graph_replay_is_deterministic(api):
    import torch
    shapes = SHAPES[:5]
    xs, xd, xp = make_batch(api, shapes, seed=11)
    plan = api.BatchPlan(shapes, "bf16x6", "bf16x3")
    G, U, cp, up = plan.outputs()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(xp, cp, up, ws)          # eager reference (also warms up kernels)
    torch.cuda.synchronize()
    ref_G = [g.clone() for g in G]
    ref_U = [[u.clone() for u in us] for us in U]
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            plan.run(xp, cp, up, ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for g in G:
            g.zero_()                 # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for t in range(len(shapes)):
            assert torch.equal(G[t], ref_G[t]), (rep, t)
            for n in range(3):
                assert torch.equal(U[t][n], ref_U[t][n]), (rep, t, n)


@pytest.mark.parametrize("tiles", [(2, 1, 1), (16, 2, 8), (64, 4, 64)])
def test_batched_tiles_agree(api, tiles):
    """Other tile choices split the work differently (the Gram's split-K
    depth changes the order of its partial sums): every choice stays within
    the tolerance of the oracle, and the choices agree with each other to it."""
    import torch
    xs, xd, xp = make_batch(api, SHAPES, seed=21)
    outs = []
    for t in [None, tiles]:
        plan = api.BatchPlan(SHAPES, "bf16x6", "bf16x3", tiles=t)
        G, U, cp, up = plan.outputs()
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        plan.run(xp, cp, up, ws)
        plan.check(ws)
        outs.append((G, U))
    for t, (d, r) in enumerate(SHAPES):
        xn = np.linalg.norm(xs[t].astype(np.float64))
        Xa = recon(api, outs[0][0][t], outs[0][1][t])
        Xb = recon(api, outs[1][0][t], outs[1][1][t])
        Go, Uo, _ = oracle.sthosvd(xs[t], r)
        Xo = oracle.reconstruct(Go, Uo)
        assert np.linalg.norm(Xb - Xo) / xn <= 1e-5, (t, d, r, tiles)
        assert np.linalg.norm(Xa - Xb) / xn <= 1e-5, (t, d, r, tiles)


def test_autotuner_picks_a_valid_choice(api):
    import torch
    from paper_2010_10131_amd import autotune
    shapes = SHAPES[:6]
    xs, xd, xp = make_batch(api, shapes, seed=31)
    best, ms, table = autotune.tune_batched(shapes, xp, "bf16x6", "bf16x3", reps=1)
    assert ms > 0 and len(table) >= 12
    assert min(r["ms"] for r in table) == ms
    assert (table[0]["gram_wg_per_cu"], table[0]["gram_wt_max"], table[0]["ttm_rows_per_wave"]) == autotune.DEFAULT
    plan = api.BatchPlan(shapes, "bf16x6", "bf16x3", tiles=best)
    G, U, cp, up = plan.outputs()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(xp, cp, up, ws)
    plan.check(ws)
    for t, (d, r) in enumerate(shapes):
        Go, Uo, _ = oracle.sthosvd(xs[t], r)
        xn = np.linalg.norm(xs[t].astype(np.float64))
        assert np.linalg.norm(recon(api, G[t], U[t]) - oracle.reconstruct(Go, Uo)) / xn <= 1e-5


def test_batched_gapless_and_rank_deficient_match_oracle(api):
    """Gaussian tensors (no gap after R_n in any mode) and a mode whose Gram
    has rank below R_n (mode 3 of (33, 20, 150) with R_3 = 24 > 15) in one
    batch: every tensor against the oracle."""
    import torch
    shapes = [((200, 150, 40), (20, 15, 5)), ((129, 64, 33), (12, 8, 4)), ((64, 64, 64), (8, 8, 8)),
              ((33, 20, 150), (5, 3, 24))]
    rng = np.random.default_rng(41)
    xs = [np.asfortranarray(rng.standard_normal(d).astype(np.float32)) for d, _ in shapes[:3]]
    xs.append(wl.lowrank_plus_noise(*shapes[3], "none", 1e-4, 43, "float32"))
    xd = [api.to_device(x) for x in xs]
    xp = torch.tensor([x.data_ptr() for x in xd], dtype=torch.int64, device="cuda")
    plan = api.BatchPlan(shapes, "fp64", "fp32")
    G, U, cp, up = plan.outputs()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(xp, cp, up, ws)
    plan.check(ws)
    for t, (d, r) in enumerate(shapes):
        Go, Uo, _ = oracle.sthosvd(xs[t], r)
        xn = np.linalg.norm(xs[t].astype(np.float64))
        t2 = np.linalg.norm(recon(api, G[t], U[t]) - oracle.reconstruct(Go, Uo)) / xn
        assert t2 <= 1e-6, (t, d, r, t2)
        for n in range(3):
            u = api.to_numpy(U[t][n])
            np.testing.assert_allclose(u.T @ u, np.eye(r[n]), atol=1e-12)


def test_batched_64_tensors_match_oracle(api):
    """64 tensors of the batched workload's recipe (sides 32..128, ranks
    10-25 %, low rank + 1e-4 noise) against the oracle, default recipe."""
    import torch
    shapes, xs = wl.batch_tensors(64, hi=128, workers=4)
    xd = [api.to_device(x) for x in xs]
    xp = torch.tensor([x.data_ptr() for x in xd], dtype=torch.int64, device="cuda")
    plan = api.BatchPlan(shapes, "bf16x6", "bf16x3")
    G, U, cp, up = plan.outputs()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(xp, cp, up, ws)
    plan.check(ws)
    worst = 0.0
    for t, (d, r) in enumerate(shapes):
        Go, Uo, _ = oracle.sthosvd(xs[t], r)
        xn = np.linalg.norm(xs[t].astype(np.float64))
        t2 = np.linalg.norm(recon(api, G[t], U[t]) - oracle.reconstruct(Go, Uo)) / xn
        worst = max(worst, t2)
        assert t2 <= 1e-5, (t, d, r, t2)
    print(f"64 tensors: worst T2 {worst:.2e}")


def test_batched_full_range_tensors_match_oracle(api):
    """24 tensors of the batched workload's full recipe (sides 32..256, ranks
    10-25 %): orders above 128 take the subspace iteration inside their
    workgroup, which passes its residual test on these spectra (no direct
    solve of S is counted); every tensor against the oracle."""
    import torch
    shapes, xs = wl.batch_tensors(24, seed=wl.BASE_SEED + 17, workers=4)
    assert any(max(d) > 128 for d, _ in shapes)
    xd = [api.to_device(x) for x in xs]
    xp = torch.tensor([x.data_ptr() for x in xd], dtype=torch.int64, device="cuda")
    plan = api.BatchPlan(shapes, "bf16x6", "bf16x3")
    G, U, cp, up = plan.outputs()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(xp, cp, up, ws)
    torch.cuda.synchronize()
    flags = ws[:32].view(dtype=torch.int64).cpu().numpy()
    assert flags[0] == 0 and flags[1] == 0, flags
    plan.check(ws)
    for t, (d, r) in enumerate(shapes):
        Go, Uo, _ = oracle.sthosvd(xs[t], r)
        xn = np.linalg.norm(xs[t].astype(np.float64))
        t2 = np.linalg.norm(recon(api, G[t], U[t]) - oracle.reconstruct(Go, Uo)) / xn
        assert t2 <= 1e-5, (t, d, r, t2)
        for n in range(3):
            u = api.to_numpy(U[t][n])
            np.testing.assert_allclose(u.T @ u, np.eye(r[n]), atol=1e-10)


@pytest.mark.parametrize("shapes", [
    [((150, 90), (12, 8)), ((33, 200), (5, 20)), ((64, 64), (8, 8))],
    [((24, 30, 18, 20), (4, 5, 3, 4)), ((40, 12, 9, 33), (6, 3, 2, 5)), ((150, 10, 8, 6), (15, 3, 2, 2))],
    [((12, 10, 9, 8, 11), (3, 2, 3, 2, 3)), ((20, 6, 7, 5, 9), (4, 2, 2, 2, 3))],
])
def test_batched_orders_2_4_5_match_oracle(api, shapes):
    """The rotated layout for orders other than 3: each step contracts the
    tensor's first index and writes its output transposed, so the core must
    come out in natural order and every factor must belong to its mode;
    checked against the oracle (reconstruction, core norm, and each factor's
    subspace)."""
    import torch
    xs, xd, xp = make_batch(api, shapes, seed=33)
    plan = api.BatchPlan(shapes, "fp64", "fp32")
    G, U, cp, up = plan.outputs()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(xp, cp, up, ws)
    plan.check(ws)
    for t, (d, r) in enumerate(shapes):
        Go, Uo, _ = oracle.sthosvd(xs[t], r)
        xn = np.linalg.norm(xs[t].astype(np.float64))
        t2 = np.linalg.norm(recon(api, G[t], U[t]) - oracle.reconstruct(Go, Uo)) / xn
        t1 = abs(np.linalg.norm(api.to_numpy(G[t])) - np.linalg.norm(Go)) / np.linalg.norm(Go)
        assert t2 <= 1e-5 and t1 <= 1e-5, (t, d, r, t2, t1)
        for n in range(len(d)):
            u = api.to_numpy(U[t][n])
            assert u.shape == (d[n], r[n])
            np.testing.assert_allclose(u.T @ u, np.eye(r[n]), atol=1e-10)
            # the leading vectors are unique up to sign only within the rank
            # of the mode-n unfolding (earlier modes already truncated)
            k = min(r[n], int(np.prod(r[:n])) * int(np.prod(d[n + 1:])))
            np.testing.assert_allclose(u[:, :k] @ u[:, :k].T, Uo[n][:, :k] @ Uo[n][:, :k].T, atol=1e-5)


def test_batched_tiny_sides_match_oracle(api):
    """Sides of 1 to 3 (every loader's quad crosses the last row, skinny
    triangles of one super tile, rank-1 modes) and a long last mode."""
    import torch
    shapes = [((2, 50, 40), (1, 5, 4)), ((64, 3, 1), (6, 2, 1)), ((3, 3, 300), (2, 2, 3)),
              ((1, 70, 33), (1, 7, 4)), ((5, 7, 6), (2, 3, 2))]
    xs, xd, xp = make_batch(api, shapes, seed=61)
    for gp, tp in (("fp64", "fp32"), ("bf16x6", "bf16x3")):
        plan = api.BatchPlan(shapes, gp, tp)
        G, U, cp, up = plan.outputs()
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        plan.run(xp, cp, up, ws)
        plan.check(ws)
        for t, (d, r) in enumerate(shapes):
            Go, Uo, _ = oracle.sthosvd(xs[t], r)
            xn = np.linalg.norm(xs[t].astype(np.float64))
            t2 = np.linalg.norm(recon(api, G[t], U[t]) - oracle.reconstruct(Go, Uo)) / xn
            assert t2 <= 1e-5, (gp, t, d, r, t2)
