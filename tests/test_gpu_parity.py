"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances.  FP64 work is compared at 1e-12 relative or tighter.  For the
reduced-precision contractions every output is checked against an
elementwise error bound built from the same contraction on absolute values,
|got - ref| <= tol * (|A| x |B|), with tol per precision:
  fp32   products exact to 2^-24, summed in FP32 over n_acc terms:
                                        tol = 2^-24 (1 + 2 * n_acc)
  bf16x3 operands carried to 2^-17, the lo*lo cross terms dropped:
                                        tol = 2^-15 + 2^-24 (1 + 2 * n_acc)
  bf16x6 operands to 2^-25:             tol = 2^-21 + 2^-24 (1 + 2 * n_acc)
where n_acc is the length of the FP32 sums: min(K, 128) for the Gram and
the TTT (FP64 across chunks of 128), K for the TTM (FP32 over the whole
contraction of length K).  Whole decompositions are compared by
T1 = | ||G|| - ||G*|| | / ||G*|| and T2 = ||X^ - X^*|| / ||X|| (invariant to
factor signs and to rotations inside degenerate eigenspaces).
"""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


def tol_for(prec, K, ttm=False):
    acc = U24 * (1 + 2 * (K if ttm else min(K, 128)))
    return {"fp64": 64 * K * 2.0 ** -53, "fp32": acc, "bf16x3": 2.0 ** -15 + acc,
            "bf16x6": 2.0 ** -21 + acc}[prec]


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    from paper_2010_10131_amd import api as a
    return a


def randn(shape, seed, dtype="float32"):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape).astype(dtype))


def check_bound(got, ref, bound, tol, what):
    err = np.abs(got - ref)
    lim = tol * bound + 1e-300
    bad = err > lim
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} outside bound; worst ratio "
                           f"{(err / lim).max():.3g}")


# ------------------------------------------------------------------- TTM ----

TTM_CASES = [
    # dims, mode, R  (L = 1; L >= 64; small L; M = 1; ragged K / R / rows)
    ((64, 40, 3), 0, 8),
    ((37, 50, 9), 0, 5),          # ragged K, odd rows
    ((100, 33), 0, 17),           # two r-tiles with a ragged one
    ((64, 64, 64), 1, 16),        # L = 64
    ((96, 20, 7), 1, 64),         # L = 96, R = 64
    ((8, 48, 30), 1, 8),          # small L (C5-like mode 2)
    ((3, 65, 11), 1, 33),         # L = 3, ragged K
    ((16, 160, 5), 1, 16),        # L = 16 (C3-like mode 2)
    ((12, 10, 70), 2, 70),        # M = 1, R = K (rotation), three r-blocks... ragged
    ((5, 7, 130), 2, 130),        # R > 64: several r-blocks
    ((1, 1, 1), 1, 1),            # degenerate
    ((200, 3), 1, 2),             # M = 1, tiny K
    ((512, 300), 0, 64),          # contiguous rows, K = 512: K-split kernel, whole chunks, ragged row block
    ((384, 77), 0, 40),           # K-split with 12 chunks (idle waves), ragged R
    ((300, 50), 0, 20),           # K-split with a ragged last chunk
    ((1024, 40), 0, 16),          # long contractions (FP32 sums over all of K):
    ((3, 1024, 7), 1, 16),        #   K = 1024, L = 1 and L = 3
    ((4096, 20), 0, 8),           #   K = 4096
    ((2, 4096, 3), 1, 12),
    ((30648, 6), 0, 6),           #   K = 30648 (the Air-Quality-like first mode of the ALS case)
    ((2, 30648, 2), 1, 4),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("dims,n,R", TTM_CASES)
def test_ttm_parity(api, dims, n, R, prec):
    dtype = "float64" if prec == "fp64" else "float32"
    Y = randn(dims, 100 + sum(dims) + n, dtype)
    K = dims[n]
    U = np.asfortranarray(np.random.default_rng(7 + K + R).standard_normal((K, R)))
    Z = api.to_numpy(api.ttm_mode_n(api.to_device(Y), api.to_device(U), n, prec))
    ref = oracle.ttm_tensor(Y, U.T, n)
    bound = oracle.ttm_tensor(np.abs(Y), np.abs(U).T, n)
    check_bound(Z, ref, bound, tol_for(prec, K, ttm=True), f"ttm {dims} n={n} R={R} {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ttm_transposed_factor_expands(api, prec):
    dtype = "float64" if prec == "fp64" else "float32"
    Y = randn((6, 5, 7), 3, dtype)
    W = np.asfortranarray(np.random.default_rng(4).standard_normal((40, 5)))  # I x R factor
    Z = api.to_numpy(api.ttm_mode_n(api.to_device(Y), api.to_device(W), 1, prec, transpose_u=True))
    ref = oracle.ttm_tensor(Y, W, 1)
    check_bound(Z, ref, oracle.ttm_tensor(np.abs(Y), np.abs(W), 1), tol_for(prec, 5), "ttm^T")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("dims,n,R", [((40, 520, 3), 1, 64), ((512, 300), 0, 64), ((9, 33, 7), 2, 5)])
def test_ttm_prepared_factor_matches(api, dims, n, R, prec):
    """One prepared factor applied twice gives the bits of ttm_mode_n (same kernel, same split)."""
    dtype = "float64" if prec == "fp64" else "float32"
    Y = api.to_device(randn(dims, 11 + n, dtype))
    U = api.to_device(np.asfortranarray(np.random.default_rng(5 + R).standard_normal((dims[n], R))))
    Up = api.ttm_factor_prepare(U, prec)
    Z0 = api.to_numpy(api.ttm_mode_n(Y, U, n, prec))
    for _ in range(2):
        Z1 = api.to_numpy(api.ttm_mode_n_prepared(Y, Up, n, R, prec))
        assert np.array_equal(Z0, Z1), f"prepared ttm {dims} n={n} {prec}"
    Wt = api.to_device(np.asfortranarray(np.random.default_rng(6).standard_normal((dims[n], R))))
    Z2 = api.to_numpy(api.ttm_mode_n_prepared(api.to_device(api.to_numpy(api.ttm_mode_n_prepared(
        Y, Up, n, R, prec))), api.ttm_factor_prepare(Wt, prec, transpose_u=True), n, dims[n], prec))
    Z3 = api.to_numpy(api.ttm_mode_n(api.to_device(Z0), Wt, n, prec, transpose_u=True))
    assert np.array_equal(Z2, Z3)


# ------------------------------------------------------------ Gram / TTT ----

GRAM_CASES = [
    ((64, 40, 3), 0),
    ((37, 50, 9), 0),
    ((130, 20, 6), 0),            # I > 128: several blocks incl. ragged
    ((64, 64, 20), 1),            # L = 64
    ((8, 48, 300), 1),            # small L, many rows
    ((3, 65, 11), 1),
    ((16, 100, 40), 2),           # M = 1
    ((1, 5, 1), 1),
    ((2, 3, 5000), 0),            # I = 2, long contraction (split-K)
    ((512, 30, 7), 0),            # first mode, 4 x 4 blocks of 128
    ((160, 50, 40), 0),           # first mode, ragged blocks, split-K
    ((100, 999), 0),              # first mode, I % 4 == 0, odd row count
    ((33, 4096), 0),              # first mode, ragged I (scalar loads)
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("dims,n", GRAM_CASES)
def test_gram_parity(api, dims, n, prec):
    dtype = "float64" if prec == "fp64" else "float32"
    Y = randn(dims, 200 + sum(dims) + n, dtype)
    S = api.to_numpy(api.gram_mode_n(api.to_device(Y), n, prec))
    Yn = oracle.unfold(Y, n)
    ref = oracle.gram(Yn)
    bound = oracle.gram(np.abs(Yn))
    assert np.array_equal(S, S.T)
    K = Yn.shape[1]
    check_bound(S, ref, bound, tol_for(prec, K), f"gram {dims} n={n} {prec}")


@pytest.mark.parametrize("dims,n", [((64, 40, 3), 0), ((512, 30, 7), 0), ((37, 50, 9), 0),
                                    ((16, 100, 40), 1)])
def test_gram_fp64_products_of_fp32_data(api, dims, n):
    """STH_PREC_FP64 on FP32 data: products exact, FP64 accumulation."""
    Y = randn(dims, 400 + sum(dims), "float32")
    S = api.to_numpy(api.gram_mode_n(api.to_device(Y), n, "fp64"))
    Yn = oracle.unfold(Y, n)
    check_bound(S, oracle.gram(Yn), oracle.gram(np.abs(Yn)), tol_for("fp64", Yn.shape[1]),
                "gram fp64 of fp32")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("dims,n,R", [((64, 40, 3), 0, 8), ((16, 96, 30), 1, 20),
                                      ((5, 7, 130), 2, 3), ((200, 9), 0, 150)])
def test_ttt_parity(api, dims, n, R, prec):
    dtype = "float64" if prec == "fp64" else "float32"
    Y = randn(dims, 300 + sum(dims), dtype)
    zd = list(dims)
    zd[n] = R
    Z = randn(tuple(zd), 301 + R, dtype)
    P = api.to_numpy(api.ttt_mode_n(api.to_device(Y), api.to_device(Z), n, prec))
    Yn, Zn = oracle.unfold(Y, n), oracle.unfold(Z, n)
    ref = oracle.ttt(Yn, Zn)
    check_bound(P, ref, oracle.ttt(np.abs(Yn), np.abs(Zn)), tol_for(prec, Yn.shape[1]), "ttt")


# ---------------------------------------------------------------- eigen ----

def spd_with_spectrum(lam, seed):
    n = len(lam)
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return np.asfortranarray((Q * lam) @ Q.T)


@pytest.mark.parametrize("n,R", [(1, 1), (2, 1), (5, 3), (16, 16), (33, 7), (64, 8), (90, 30),
                                 (100, 10), (128, 64), (128, 128)])
def test_eig_parity(api, n, R):
    lam = 2.0 ** (-np.arange(n) / 4.0)          # distinct, gaps >> roundoff
    S = spd_with_spectrum(lam, n)
    U, ev, ws = api.eig_leading(api.to_device(S), R)
    U, ev = api.to_numpy(U), ev.cpu().numpy()
    assert int(ws[:8].view(dtype=__import__("torch").int64).item()) == 0
    lo, Vo, _ = oracle.jacobi_eig(S)
    np.testing.assert_allclose(ev, lo[:R], rtol=0, atol=1e-13 * lo[0] * max(1, n / 16))
    # eigenvector i is determined to ~eps ||S|| / gap_i (Davis-Kahan)
    gaps = np.abs(np.diff(np.concatenate([[np.inf], lo, [-np.inf]])))
    gap = np.minimum(gaps[:-1], gaps[1:])[:R]
    tol = np.minimum(1e-10, 0) + 1e-10 + 64 * n * 2.2e-16 * lo[0] / gap
    assert np.all(np.abs(U - Vo[:, :R]) <= tol[None, :])
    np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-12)


@pytest.mark.parametrize("n,R", [(129, 8), (200, 16), (256, 40), (512, 64), (512, 8),
                                 (300, 100), (478, 122)])   # blocks 120 and 128 (guard 6)
def test_eig_subspace_iteration_parity(api, n, R):
    """n > 128: subspace iteration + Rayleigh-Ritz.  The spectrum has the
    structure of a low-rank-plus-noise Gram (a gap after the R leading
    eigenvalues), so the leading eigenvectors are well determined."""
    # the R leading eigenvalues span at most 2^-8, then a gap to the 1e-9 floor
    lam = np.concatenate([2.0 ** (-np.arange(R) * min(0.25, 8.0 / R)), 1e-9 * np.exp(-np.arange(n - R) / n)])
    S = spd_with_spectrum(lam, n + R)
    U, ev, ws = api.eig_leading(api.to_device(S), R)
    U, ev = api.to_numpy(U), ev.cpu().numpy()
    flags = ws[:16].view(dtype=__import__("torch").int64).cpu().numpy()
    assert flags[0] == 0
    assert flags[1] == 0   # the gap after R: the subspace iteration passed its residual test
    lo, Vo, _ = oracle.jacobi_eig(S)
    np.testing.assert_allclose(ev, lo[:R], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(U, Vo[:, :R], rtol=0, atol=1e-9)
    np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-12)


def test_eig_gapless_spectrum_is_exact(api):
    """Without a gap after R (lam_i = 2^(-i/4)) three subspace iterations
    cannot resolve the leading subspace: the residual test fails and the
    direct solver runs on S.  The result is the oracle's leading subspace to
    working accuracy (Davis-Kahan: eps ||S|| / gap ~ 2e-14 here)."""
    import torch
    n, R = 160, 16
    lam = 2.0 ** (-np.arange(n) / 4.0)
    S = spd_with_spectrum(lam, 3)
    U, ev, ws = api.eig_leading(api.to_device(S), R)
    U = api.to_numpy(U)
    flags = ws[:32].view(dtype=torch.int64).cpu().numpy()
    assert flags[0] == 0 and flags[1] == 1 and flags[3] == 1, flags   # both rounds failed
    lo, Vo, _ = oracle.jacobi_eig(S)
    sin_theta = np.linalg.norm(U @ U.T - Vo[:, :R] @ Vo[:, :R].T, 2)
    assert sin_theta <= 1e-11, sin_theta
    # eigenvalues to the backward error of a Householder-based solver (~ n eps ||S||)
    np.testing.assert_allclose(ev.cpu().numpy(), lo[:R], rtol=0, atol=4 * n * 2.2e-16 * lo[0])
    np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-13)
    gaps = lo[:R] - lo[1:R + 1]
    assert np.all(np.abs(U - Vo[:, :R]) <= 1e-12 + 64 * n * 2.2e-16 * lo[0] / np.minimum(gaps, np.r_[np.inf, gaps[:-1]]))


def test_eig_second_round_resolves_a_moderate_gap(api):
    """lam_(p+1) / lam_R ~ 2e-4 (p = 40): three products leave Ritz residuals
    near 1e-12 |theta_1|, above the FP64 test, so the gated second round runs
    (two more products and Rayleigh-Ritz); five products pass it, and the
    direct solver is not needed.  The result is the oracle's leading
    subspace."""
    import torch
    n, R = 300, 20
    lam = np.concatenate([1.0 - np.arange(20) / 40.0, 0.5 * 2.0 ** -np.arange(1.0, 21.0),
                          1e-4 * 0.9 ** np.arange(n - 40)])
    S = spd_with_spectrum(lam, 29)
    U, ev, ws = api.eig_leading(api.to_device(S), R)
    U, ev = api.to_numpy(U), ev.cpu().numpy()
    flags = ws[:32].view(dtype=torch.int64).cpu().numpy()
    assert flags[0] == 0 and flags[3] == 1 and flags[1] == 0, flags
    lo, Vo, _ = oracle.jacobi_eig(S)
    np.testing.assert_allclose(ev, lo[:R], rtol=0, atol=4 * n * 2.2e-16 * lo[0])
    assert np.linalg.norm(U @ U.T - Vo[:, :R] @ Vo[:, :R].T, 2) <= 1e-12
    assert np.linalg.norm(S @ U - U * ev, axis=0).max() <= 16 * np.sqrt(n) * 2.3e-16 * lo[0]
    np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-13)


@pytest.mark.parametrize("n,R", [(129, 8), (300, 40), (512, 64)])
def test_eig_gaussian_gram_matches_oracle(api, n, R):
    """Gram of a Gaussian n x 4n matrix (Marchenko-Pastur spectrum, no gap
    after R): the leading pairs agree with the oracle's Jacobi to the
    accuracy a backward-stable solver allows."""
    import torch
    B = np.random.default_rng(n).standard_normal((n, 4 * n))
    S = np.asfortranarray(B @ B.T)
    U, ev, ws = api.eig_leading(api.to_device(S), R)
    U, ev = api.to_numpy(U), ev.cpu().numpy()
    assert ws[:8].view(dtype=torch.int64).item() == 0
    lo, Vo, _ = oracle.jacobi_eig(S)
    np.testing.assert_allclose(ev, lo[:R], rtol=0, atol=4 * n * 2.2e-16 * lo[0])
    gap = lo[R - 1] - lo[R]
    sin_theta = np.linalg.norm(U @ U.T - Vo[:, :R] @ Vo[:, :R].T, 2)
    assert sin_theta <= 64 * n * 2.2e-16 * lo[0] / gap, (sin_theta, gap / lo[0])
    res = np.linalg.norm(S @ U - U * ev, axis=0).max()
    assert res <= 1e-13 * lo[0], res
    np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-13)


def test_eig_clusters_above_order_128(api):
    """Eigenvalues of multiplicity 3 and 4 at the top of an order-200
    spectrum: a cut between the clusters gives the oracle's subspace; a cut
    through the second cluster gives eigenpairs of S (any basis of the
    cluster is correct) that are orthonormal."""
    n = 200
    lam = np.concatenate([np.full(3, 5.0), np.full(4, 4.0), 2.0 ** (-np.arange(n - 7) / 8.0)])
    S = spd_with_spectrum(lam, 17)
    lo, Vo, _ = oracle.jacobi_eig(S)
    for R in (7, 5):
        U, ev, ws = api.eig_leading(api.to_device(S), R)
        U, ev = api.to_numpy(U), ev.cpu().numpy()
        np.testing.assert_allclose(ev, lam[:R], rtol=0, atol=1e-13 * 5)
        assert np.linalg.norm(S @ U - U * ev, axis=0).max() <= 1e-13 * 5
        np.testing.assert_allclose(U.T @ U, np.eye(R), atol=1e-13)
        if R == 7:
            assert np.linalg.norm(U @ U.T - Vo[:, :7] @ Vo[:, :7].T, 2) <= 1e-12


def test_eig_nan_input_is_contained(api):
    """A NaN on the diagonal (a non-finite Gram, e.g. from a failed ALS step
    upstream) is reported as flag 3 and sorts last, so the selection stays a
    permutation and no column index leaves the matrix; order 110 keeps V in
    the workspace, where a stray column would be a stray global address."""
    import torch
    S = spd_with_spectrum(2.0 ** (-np.arange(110) / 4.0), 110)
    S[5, 5] = np.nan
    U, ev, ws = api.eig_leading(api.to_device(S), 6, max_sweeps=3)
    torch.cuda.synchronize()
    assert int(ws[:8].view(dtype=torch.int64).item()) == 3
    assert U.shape == (110, 6)


def test_eig_degenerate_and_cap(api):
    import torch
    S = np.asfortranarray(np.diag([3.0, 1.0, 3.0, 2.0]))
    U, ev, ws = api.eig_leading(api.to_device(S), 3)
    np.testing.assert_array_equal(ev.cpu().numpy(), [3.0, 3.0, 2.0])
    # ties by index: eigenvectors e0, e2, e3
    np.testing.assert_array_equal(api.to_numpy(U), np.eye(4)[:, [0, 2, 3]])
    A = randn((12, 12), 5, "float64")
    S2 = np.asfortranarray(A @ A.T)
    U, ev, ws = api.eig_leading(api.to_device(S2), 2, max_sweeps=1)
    torch.cuda.synchronize()
    assert int(ws[:8].view(dtype=torch.int64).item()) == 1   # sweep cap reported


# -------------------------------------------------------- decomposition ----

def t1_t2(api, X, G, U, Go, Uo):
    Gn = api.to_numpy(G)
    Un = [api.to_numpy(u) for u in U]
    Xh = oracle.reconstruct(Gn, Un)
    Xho = oracle.reconstruct(Go, Uo)
    t2 = np.linalg.norm(Xh - Xho) / np.linalg.norm(np.asarray(X, dtype=np.float64))
    t1 = abs(np.linalg.norm(Gn) - np.linalg.norm(Go)) / np.linalg.norm(Go)
    return t1, t2, Gn, Un


def test_c1_fp64_matches_oracle(api):
    """The small parity workload: 64^3 FP64, ranks 8, 1e-3 noise, EIG, order 1,2,3."""
    X = wl.make(wl.C1)
    G, U, ev = api.sthosvd(api.to_device(X), wl.C1.ranks, "fp64", "fp64", return_eigvals=True)
    Go, Uo, lo = oracle.sthosvd(X, wl.C1.ranks)
    t1, t2, Gn, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-12 and t2 <= 1e-12, (t1, t2)
    for n in range(3):
        np.testing.assert_allclose(Un[n], Uo[n], rtol=0, atol=1e-10)
        np.testing.assert_allclose(ev[n].cpu().numpy(), lo[n][:8], rtol=1e-12)
    np.testing.assert_allclose(Gn, Go, rtol=0, atol=1e-10 * np.abs(Go).max())


@pytest.mark.parametrize("dims,ranks,order", [
    ((30, 20), (6, 6), None),                          # N = 2: truncated SVD
    ((12, 10, 9, 8), (3, 4, 2, 5), (3, 1, 0, 2)),      # 4-way, permuted order
    ((10, 9, 8, 7, 6), (2, 3, 2, 3, 2), None),         # 5-way
    ((16, 12, 10), (16, 12, 10), None),                # R = I: rotations
    ((20, 15, 10), (1, 1, 1), None),                   # R = 1
    ((1, 17, 5), (1, 4, 2), None),                     # a mode of size 1
])
def test_decomposition_fp64_edge_cases(api, dims, ranks, order):
    X = wl.lowrank_plus_noise(dims, tuple(min(r, d) for r, d in zip(ranks, dims)), "none", 1e-2,
                              sum(dims), "float64")
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp64", mode_order=order)
    Go, Uo, _ = oracle.sthosvd(X, ranks, order=order)
    t1, t2, _, _ = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-11 and t2 <= 1e-11, (t1, t2)


@pytest.mark.parametrize("dims,ranks", [
    ((33, 20, 150), (5, 3, 24)),   # mode 3: rank(Gram) <= 15 < R = 24 (direct solver, n > 128)
    ((33, 20, 150), (5, 4, 18)),   # mode 3: rank(Gram) <= 20 < block 40 (block capped at 20)
    ((120, 50, 40), (12, 6, 5)),   # mode 1, order 120 (direct solver)
    ((110, 4, 5), (25, 3, 4)),     # mode 1, order 110: R above the rank bound 20
    ((24, 100, 9), (6, 40, 3)),    # mode 2, order 100: R near the rank bound 54
])
def test_gram_rank_below_the_subspace_block(api, dims, ranks):
    """Ranks at or above what the earlier truncations leave: only X^ and
    ||G|| are defined (the completing eigenvectors are arbitrary), and the
    factors stay orthonormal."""
    X = wl.lowrank_plus_noise(dims, ranks, "none", 1e-4, 11, "float32")
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp32")
    Go, Uo, _ = oracle.sthosvd(X, ranks)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-5 and t2 <= 1e-5, (t1, t2)
    for n in range(3):
        np.testing.assert_allclose(Un[n].T @ Un[n], np.eye(ranks[n]), atol=1e-12)


@pytest.mark.parametrize("dims,ranks", [
    ((96, 64, 50), (24, 16, 8)),
    ((90, 70, 60), (40, 30, 6)),
    ((49, 81, 33), (8, 17, 4)),
])
def test_fp32_orders_49_to_128(api, dims, ranks):
    """FP32 data, Grams of orders 33..96 with blocks below and above half the
    order (the rule of the former subspace-iteration route): the direct
    solver for every order up to 128."""
    X = wl.lowrank_plus_noise(dims, ranks, "0.9", 1e-4, 23, "float32")
    Go, Uo, _ = oracle.sthosvd(X, ranks)
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp32")
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-5 and t2 <= 1e-5, (t1, t2)
    for n in range(3):
        np.testing.assert_allclose(Un[n].T @ Un[n], np.eye(ranks[n]), atol=1e-12)


@pytest.mark.parametrize("dims,ranks", [
    ((97, 60, 50), (10, 8, 6)),       # order 97: just past the direct range of mode 1
    ((256, 40, 30), (20, 10, 8)),     # order 256: subspace block 40
    ((200, 150, 100), (20, 15, 10)),  # three gapless modes above, at and below 128
    ((512, 24, 20), (16, 8, 6)),      # order 512: the largest Gram
])
def test_gapless_fp64_decomposition_matches_oracle(api, dims, ranks):
    """Gaussian FP64 tensors (no low-rank structure, no gap after R_n in any
    mode): T1 and T2 against the oracle at 1e-12."""
    X = np.asfortranarray(np.random.default_rng(sum(dims)).standard_normal(dims))
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp64")
    Go, Uo, _ = oracle.sthosvd(X, ranks)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-12 and t2 <= 1e-12, (t1, t2)
    for n in range(3):
        np.testing.assert_allclose(Un[n].T @ Un[n], np.eye(ranks[n]), atol=1e-13)


@pytest.mark.parametrize("gp,tp,t2max", [("fp64", "fp32", 1e-6), ("fp32", "fp32", 1e-5),
                                         ("bf16x6", "bf16x3", 1e-5), ("bf16x3", "bf16x3", 1e-5)])
def test_gapless_fp32_decomposition_recipes(api, gp, tp, t2max):
    """A Gaussian 200 x 150 x 100 FP32 tensor, ranks (20, 15, 10): every
    recipe against the FP64 oracle at T2 <= 1e-5 (FP64 Gram products: 1e-6)."""
    X = np.asfortranarray(np.random.default_rng(3).standard_normal((200, 150, 100)).astype(np.float32))
    ranks = (20, 15, 10)
    G, U, _ = api.sthosvd(api.to_device(X), ranks, gp, tp)
    Go, Uo, _ = oracle.sthosvd(X, ranks)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= t2max and t2 <= t2max, (gp, tp, t1, t2)
    for u in Un:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)


def test_rank_above_the_gram_rank_above_order_128(api):
    """Mode 1 of (150, 4, 5) with R_1 = 30: the Gram has rank <= 20, the
    direct solver completes the basis; X^ and ||G|| match the oracle."""
    dims, ranks = (150, 4, 5), (30, 3, 4)
    X = wl.lowrank_plus_noise(dims, (20, 3, 4), "none", 1e-3, 5, "float64")
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp64")
    Go, Uo, _ = oracle.sthosvd(X, ranks)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-12 and t2 <= 1e-12, (t1, t2)
    np.testing.assert_allclose(Un[0].T @ Un[0], np.eye(30), atol=1e-13)


@pytest.mark.parametrize("gp,tp,t2max", [("fp64", "bf16x3", 1e-5), ("fp64", "fp32", 1e-6)])
def test_c3_regime_fp32_eig_recipes(api, gp, tp, t2max):
    """The 4-way workload's regime at 64^4: core 2^-(k1+k2+k3+k4), ranks 16,
    1e-5 noise, so lam_16 / lam_1 = 4^-15 in every mode.  FP32 data: the EIG
    recipes with FP64-product Grams meet the bar (FP32 or bf16 Gram products
    cannot resolve a spectrum 2^-30 deep)."""
    dims, ranks = (64, 64, 64, 64), (16, 16, 16, 16)
    X = wl.lowrank_plus_noise(dims, ranks, "2^-k", 1e-5, 77, "float32")
    G, U, _ = api.sthosvd(api.to_device(X), ranks, gp, tp)
    Go, Uo, _ = oracle.sthosvd(X, ranks)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= t2max and t2 <= t2max, (gp, tp, t1, t2)


@pytest.mark.parametrize("per_mode", [("als", "als", "als", "als"), ("eig", "als", "eig", "als")])
def test_c3_regime_fp64_eig_and_als_per_mode(api, per_mode):
    """The same regime in FP64 with EIG and ALS per mode (5 sweeps from the
    oracle's own initial guesses): parity with the oracle's run of the same
    choices.  After 5 sweeps at a convergence rate of 1/4 the iterate is not
    the leading subspace, and the normal matrix C = R_k^T R_k has condition
    number near lam_1 / lam_16 = 4^15 ~ 1e9: two correct FP64 runs (the oracle
    orthonormalizes with Householder QR, the device with shifted
    Cholesky-QR3) may differ by up to cond(C) eps ~ 2e-7 in X^; measured
    ~2e-10, bar 1e-8.  ||G|| is well conditioned (1e-12)."""
    dims, ranks = (64, 64, 64, 64), (16, 16, 16, 16)
    X = wl.lowrank_plus_noise(dims, ranks, "2^-k", 1e-5, 78, "float64")
    L0 = [wl.gaussian_init(d, r, 9, n) for n, (d, r) in enumerate(zip(dims, ranks))]
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp64", per_mode=per_mode, als_init=L0)
    meth = [0 if m == "eig" else 1 for m in per_mode]
    Go, Uo, _ = oracle.sthosvd(X, ranks, methods=meth, L0=L0, als_variant=1)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-12 and t2 <= 1e-8, (t1, t2)
    for u in Un:
        np.testing.assert_allclose(u.T @ u, np.eye(16), atol=1e-12)


@pytest.mark.parametrize("variant_dims,ranks,per_mode", [
    ((24, 20, 18), (4, 5, 3), ("als", "als", "als")),
    ((24, 20, 18), (4, 5, 3), ("eig", "als", "eig")),
    ((40, 12, 9, 7), (5, 3, 4, 2), ("als", "eig", "als", "als")),
])
def test_als_fp64_matches_oracle(api, variant_dims, ranks, per_mode):
    """ALS branch (Alg. 3 with L_k re-orthonormalized) against the oracle's
    re-orthonormalized variant, same initial guesses: same subspaces, so the
    same X^ and ||G|| (factors may differ by a rotation)."""
    dims = variant_dims
    X = wl.lowrank_plus_noise(dims, ranks, "none", 1e-3, 77, "float64")
    L0 = [wl.gaussian_init(d, r, 9, n) for n, (d, r) in enumerate(zip(dims, ranks))]
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp64", per_mode=per_mode,
                          als_init=L0)
    meth = [0 if m == "eig" else 1 for m in per_mode]
    Go, Uo, _ = oracle.sthosvd(X, ranks, methods=meth, L0=L0, als_variant=1)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-10 and t2 <= 1e-10, (t1, t2)
    for n in range(len(dims)):
        np.testing.assert_allclose(Un[n].T @ Un[n], np.eye(ranks[n]), atol=1e-12)
        np.testing.assert_allclose(Un[n] @ Un[n].T, Uo[n] @ Uo[n].T, atol=1e-9)


def test_exhaustive_selection_keeps_the_faster_step_and_matches_oracle(api):
    """sthosvd_choose_exhaustive (Sec. IV-B): every mode's choice is the
    faster of the two timed steps that counted, X is left untouched, and the
    decomposition planned with those choices matches the oracle run with the
    same per-mode methods and ALS initial guesses."""
    import torch
    dims, ranks = (40, 36, 30, 24), (6, 5, 4, 3)
    X = wl.lowrank_plus_noise(dims, ranks, "none", 1e-3, 91, "float64")
    Xd = api.to_device(X)
    X0 = Xd.clone()
    choice, ms = api.choose_exhaustive(Xd, ranks, "fp64", "fp64")
    assert torch.equal(Xd, X0)
    assert len(choice) == len(dims)
    for c, (te, ta) in zip(choice, ms):
        assert te > 0
        assert c == ("als" if 0 <= ta < te else "eig"), (choice, ms)
    L0 = [wl.gaussian_init(d, r, 9, n) for n, (d, r) in enumerate(zip(dims, ranks))]
    G, U, _ = api.sthosvd(Xd, ranks, "fp64", "fp64", per_mode=choice, als_init=L0)
    Go, Uo, _ = oracle.sthosvd(X, ranks, methods=[0 if c == "eig" else 1 for c in choice], L0=L0,
                               als_variant=1)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-10 and t2 <= 1e-10, (t1, t2)


def test_large_first_mode_takes_als_and_matches_oracle(api):
    """An Air-Quality-like first mode (I_1 = 30648, beyond the eigensolver's
    512): the plan takes ALS there under either selector and EIG for the
    small modes; FP32 data, FP64 products, same initial guess as the oracle."""
    import torch
    dims, ranks = (30648, 12, 10), (6, 5, 4)
    for solver in ("auto", "auto_tree"):
        p = api.Plan(dims, ranks, torch.float32, "fp64", "fp32", solver)
        assert p.solvers[0] == 1
    X = wl.lowrank_plus_noise(dims, ranks, "none", 1e-4, 41, "float32")
    L0 = [wl.gaussian_init(d, r, 9, n) for n, (d, r) in enumerate(zip(dims, ranks))]
    per_mode = ("als", "eig", "eig")
    G, U, _ = api.sthosvd(api.to_device(X), ranks, "fp64", "fp32", per_mode=per_mode, als_init=L0)
    Go, Uo, _ = oracle.sthosvd(X, ranks, methods=[1, 0, 0], L0=L0, als_variant=1)
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t1 <= 1e-5 and t2 <= 1e-5, (t1, t2)
    np.testing.assert_allclose(Un[0].T @ Un[0], np.eye(ranks[0]), atol=1e-10)


def test_als_device_initial_guess_runs(api):
    X = wl.lowrank_plus_noise((30, 20, 10), (3, 3, 3), "none", 0.0, 3, "float64")
    G, U, _ = api.sthosvd(api.to_device(X), (3, 3, 3), "fp64", "fp64", solver="als", seed=5)
    Xh = oracle.reconstruct(api.to_numpy(G), [api.to_numpy(u) for u in U])
    assert np.linalg.norm(Xh - X) / np.linalg.norm(X) <= 1e-11


@pytest.mark.parametrize("gp,tp,t2max", [("fp64", "fp32", 1e-6), ("fp32", "fp32", 1e-5),
                                         ("bf16x6", "bf16x3", 1e-5), ("bf16x3", "bf16x3", 1e-4)])
def test_fp32_data_recipes(api, gp, tp, t2max):
    """FP32 data, 48^3 with ranks 6 and decaying core: every recipe against the FP64 oracle."""
    X = wl.lowrank_plus_noise((48, 40, 36), (6, 6, 6), "0.9", 1e-4, 31, "float32")
    G, U, _ = api.sthosvd(api.to_device(X), (6, 6, 6), gp, tp)
    Go, Uo, _ = oracle.sthosvd(X, (6, 6, 6))
    t1, t2, _, Un = t1_t2(api, X, G, U, Go, Uo)
    assert t2 <= t2max and t1 <= t2max, (gp, tp, t1, t2)
    for u in Un:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)


# -------------------------------------------------------- reconstruction ----

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,ranks", [((20, 14, 9), (5, 4, 3)), ((70, 45, 37), (9, 7, 5)),
                                        ((24, 18, 12, 40), (4, 3, 5, 6))])
def test_reconstruct_and_error(api, prec, dims, ranks):
    """tucker_reconstruct against the oracle's reconstruction; tucker_error
    (the last expansion fused with the sums, X^ never stored) against the
    sums over the oracle's X^: several workgroups and r-blocks, ragged I_N."""
    dtype = "float64" if prec == "fp64" else "float32"
    G = randn(ranks, 1, dtype)
    U = [randn((d, r), 2 + d, "float64") for d, r in zip(dims, ranks)]
    Xh = api.to_numpy(api.tucker_reconstruct(api.to_device(G), [api.to_device(u) for u in U], prec))
    ref = oracle.reconstruct(G, U)
    bound = oracle.reconstruct(np.abs(G), [np.abs(u) for u in U])
    check_bound(Xh, ref, bound, 3 * tol_for(prec, 5), "reconstruct")
    X = randn(dims, 9, dtype)
    out = api.tucker_error(api.to_device(X), api.to_device(G), [api.to_device(u) for u in U], prec)
    e2, x2 = out.cpu().numpy()
    Xf = X.astype(np.float64)
    assert abs(x2 - np.sum(Xf * Xf)) <= 1e-12 * np.sum(Xf * Xf)
    assert abs(e2 - np.sum((Xf - ref) ** 2)) <= 1e-5 * np.sum((Xf - ref) ** 2)


def test_sumsq(api):
    x = randn((1000, 37), 11, "float32")
    got = float(api.sumsq(api.to_device(x)).item())
    ref = oracle.sumsq(x)
    assert abs(got - ref) <= 1e-13 * ref
