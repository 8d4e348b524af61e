"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests calls the HIP library.  Each pin is independent of the
oracle's own code: closed forms, invariants, textbook special cases computed
with LAPACK through numpy, and brute force at tiny sizes.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def rand_tensor(shape, seed):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


def numpy_unfold(X, n):
    """Independent unfolding: move mode n first, column-major reshape."""
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


# ------------------------------------------------------------ Sec. II-A ----

@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 4, 5), (7, 1, 3), (4, 6)])
def test_unfold_matches_kolda_order_and_fold_inverts(orc, shape):
    X = rand_tensor(shape, 1)
    for n in range(len(shape)):
        Yn = orc.unfold(X, n)
        np.testing.assert_array_equal(Yn, numpy_unfold(X, n))
        np.testing.assert_array_equal(orc.fold(Yn, shape, n), X)


def test_frobenius_norm_same_for_every_matricization(orc):
    """Eq. 1: ||X||_F equals the Frobenius norm of every unfolding."""
    X = rand_tensor((5, 6, 7), 2)
    ref = float(np.sum(X * X))
    for n in range(3):
        assert abs(orc.sumsq(orc.unfold(X, n)) - ref) <= 1e-13 * ref
    assert abs(orc.sumsq(X) - ref) <= 1e-13 * ref


def test_gram_trace_symmetry_psd_and_library_product(orc):
    """Gram = TTT(Y, Y): trace S = ||Y||^2, symmetric PSD, equals Yn Yn^T."""
    X = rand_tensor((6, 5, 4), 3)
    for n in range(3):
        Yn = numpy_unfold(X, n)
        S = orc.gram(Yn)
        np.testing.assert_allclose(S, Yn @ Yn.T, rtol=1e-13, atol=1e-13)
        assert np.array_equal(S, S.T)
        assert abs(np.trace(S) - np.sum(X * X)) <= 1e-12 * np.sum(X * X)
        assert np.linalg.eigvalsh(S).min() > -1e-12


def test_ttt_against_einsum_and_gram_identity(orc):
    """Eq. 3 (reading: contraction over every mode but n) and TTT(Y, Y x_n A^T) = S A."""
    X = rand_tensor((4, 5, 6), 4)
    A = rand_tensor((5, 3), 5)
    n = 1
    Y2 = np.einsum("ijk,jr->irk", X, A)            # X x_2 A^T
    Z = orc.ttt(numpy_unfold(X, n), numpy_unfold(Y2, n))
    np.testing.assert_allclose(Z, np.einsum("ijk,irk->jr", X, Y2), rtol=1e-12, atol=1e-12)
    S = orc.gram(numpy_unfold(X, n))
    np.testing.assert_allclose(Z, S @ A, rtol=1e-12, atol=1e-12)


def test_ttm_definition_and_algebra(orc):
    """Eq. 2 and its algebra: identity, composition, commuting modes,
    orthogonal invariance of the norm, first/last mode = plain GEMM."""
    X = rand_tensor((4, 5, 6), 6)
    A = rand_tensor((3, 5), 7)
    B = rand_tensor((2, 3), 8)
    C = rand_tensor((7, 4), 9)
    Y = orc.ttm_tensor(X, A, 1)
    np.testing.assert_allclose(Y, np.einsum("ijk,rj->irk", X, A), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(orc.ttm_tensor(X, np.eye(5), 1), X, rtol=0, atol=0)
    np.testing.assert_allclose(orc.ttm_tensor(Y, B, 1), orc.ttm_tensor(X, B @ A, 1),
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(orc.ttm_tensor(orc.ttm_tensor(X, A, 1), C, 0),
                               orc.ttm_tensor(orc.ttm_tensor(X, C, 0), A, 1),
                               rtol=1e-12, atol=1e-12)
    Q, _ = np.linalg.qr(rand_tensor((6, 6), 10))
    assert abs(np.linalg.norm(orc.ttm_tensor(X, Q.T, 2)) - np.linalg.norm(X)) < 1e-12
    # mode 1 (L = 1) and last mode (M = 1) are single GEMMs
    M0 = orc.ttm_tensor(X, C, 0)
    np.testing.assert_allclose(M0.reshape(7, -1, order="F"), C @ X.reshape(4, -1, order="F"),
                               rtol=1e-12, atol=1e-12)
    D = rand_tensor((3, 6), 11)
    M2 = orc.ttm_tensor(X, D, 2)
    np.testing.assert_allclose(M2.reshape(-1, 3, order="F"), X.reshape(-1, 6, order="F") @ D.T,
                               rtol=1e-12, atol=1e-12)
    # the transposed-factor form used by the core update
    U = rand_tensor((5, 3), 12)
    np.testing.assert_allclose(orc.ttm_t(U, numpy_unfold(X, 1)),
                               numpy_unfold(orc.ttm_tensor(X, U.T, 1), 1), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- eigen ----

@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
def test_jacobi_matches_lapack_and_is_orthonormal(orc, n):
    A = rand_tensor((n, n + 3), 20 + n)
    S = A @ A.T
    lam, V, sweeps = orc.jacobi_eig(S)
    assert sweeps >= 0
    ref = np.sort(np.linalg.eigvalsh(S))[::-1]
    np.testing.assert_allclose(lam, ref, rtol=0, atol=50 * n * EPS * np.abs(ref).max())
    assert np.all(np.diff(lam) <= 0)
    assert np.abs(S @ V - V * lam).max() <= 100 * n * EPS * np.abs(S).max()
    assert np.abs(V.T @ V - np.eye(n)).max() <= 100 * n * EPS
    # sign rule: entry of largest magnitude positive
    for c in range(n):
        assert V[np.argmax(np.abs(V[:, c])), c] > 0


def test_jacobi_diagonal_and_degenerate(orc):
    S = np.diag([1.0, 3.0, 2.0])
    lam, V, sweeps = orc.jacobi_eig(S)
    np.testing.assert_array_equal(lam, [3.0, 2.0, 1.0])
    np.testing.assert_array_equal(np.abs(V), np.eye(3)[:, [1, 2, 0]])
    assert sweeps == 0
    lam, V, _ = orc.jacobi_eig(np.eye(4) * 2.5)
    np.testing.assert_array_equal(lam, [2.5] * 4)


def test_jacobi_sweep_cap_reports_failure(orc):
    A = rand_tensor((8, 8), 30)
    lam, V, sweeps = orc.jacobi_eig(A @ A.T, max_sweeps=0)
    assert sweeps == -1


# ------------------------------------------------------------- small LA ----

@pytest.mark.parametrize("m,n", [(5, 5), (9, 4), (64, 8), (3, 1)])
def test_householder_qr(orc, m, n):
    A = rand_tensor((m, n), 40 + m)
    Q, R = orc.qr(A)
    np.testing.assert_allclose(Q @ R, A, rtol=0, atol=1e-13 * np.abs(A).max() * m)
    np.testing.assert_allclose(Q.T @ Q, np.eye(n), rtol=0, atol=1e-14 * m)
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.diag(R) >= 0)
    Qn, Rn = np.linalg.qr(A)
    s = np.sign(np.diag(Rn))
    np.testing.assert_allclose(Q, Qn * s, rtol=0, atol=1e-12)


def test_right_solve_spd(orc):
    A = rand_tensor((6, 9), 50)
    S = A @ A.T
    B = rand_tensor((11, 6), 51)
    X = orc.right_solve_spd(S, B)
    np.testing.assert_allclose(X @ S, B, rtol=0, atol=1e-10)
    with pytest.raises(np.linalg.LinAlgError):
        orc.right_solve_spd(-np.eye(3), np.ones((2, 3)))


# -------------------------------------------------- st-HOSVD (Alg. 1/2) ----

def alg1_svd(X, ranks):
    """Alg. 1 (st-HOSVD-SVD) written with LAPACK's SVD: the brute-force pin."""
    Y = np.array(X, dtype=np.float64)
    Us, sig2 = [], []
    for n in range(X.ndim):
        Yn = numpy_unfold(Y, n)
        u, s, vt = np.linalg.svd(Yn, full_matrices=False)
        R = ranks[n]
        Us.append(u[:, :R])
        sig2.append(s ** 2)
        core = (s[:R, None] * vt[:R, :])
        shape = list(Y.shape)
        shape[n] = R
        Y = np.moveaxis(np.reshape(core, [R] + [shape[m] for m in range(X.ndim) if m != n],
                                   order="F"), 0, n)
    return Y, Us, sig2


@pytest.mark.parametrize("shape,ranks", [((5, 4, 3), (2, 3, 2)), ((6, 6, 6), (3, 3, 3)),
                                         ((4, 3, 5, 2), (2, 2, 3, 1)), ((3, 3, 3), (3, 3, 3))])
def test_sthosvd_equals_alg1_brute_force(orc, shape, ranks):
    """P4: Alg. 2 with every mode EIG equals Alg. 1 (SVD of the explicit
    matricization): same eigenvalues = sigma^2, same subspaces, same core up
    to the signs of the factor columns."""
    X = rand_tensor(shape, sum(shape))
    G, U, lam = orc.sthosvd(X, ranks)
    Gs, Us, sig2 = alg1_svd(X, ranks)
    Gal = np.array(G)
    for n in range(len(shape)):
        k = min(len(sig2[n]), shape[n])
        np.testing.assert_allclose(lam[n][:k], sig2[n][:k], rtol=1e-10,
                                   atol=1e-12 * sig2[n][0])
        P = U[n] @ U[n].T
        Ps = Us[n] @ Us[n].T
        np.testing.assert_allclose(P, Ps, rtol=0, atol=1e-9)
        d = np.sign(np.sum(U[n] * Us[n], axis=0))
        Gal = np.moveaxis(np.moveaxis(Gal, n, -1) * d, -1, n)
    np.testing.assert_allclose(Gal, Gs, rtol=0, atol=1e-9 * np.abs(Gs).max())


def test_exact_multilinear_rank_reconstructs(orc):
    """P1: nu = 0 and R_n = true rank: e <= 1e-13 and ||G|| = ||X||."""
    X = wl.lowrank_plus_noise((12, 10, 9), (3, 4, 2), "none", 0.0, 7, "float64")
    G, U, _ = orc.sthosvd(X, (3, 4, 2))
    Xh = orc.reconstruct(G, U)
    e = np.linalg.norm(X - Xh) / np.linalg.norm(X)
    assert e <= 1e-13
    assert abs(np.linalg.norm(G) - np.linalg.norm(X)) <= 1e-13 * np.linalg.norm(X)


@pytest.mark.parametrize("order", [None, (2, 0, 1)])
def test_energy_invariant_and_discarded_eigenvalues(orc, order):
    """P2: ||X||^2 - ||G||^2 = ||X - X^||^2 (absolute residual, orthonormal
    factors).  P3: e^2 ||X||^2 = sum over modes of the discarded eigenvalues
    of each working-tensor Gram."""
    X = wl.lowrank_plus_noise((14, 12, 10), (4, 3, 5), "none", 0.05, 11, "float64")
    ranks = (4, 3, 5)
    G, U, lam = orc.sthosvd(X, ranks, order=order)
    Xh = orc.reconstruct(G, U)
    x2 = np.sum(X * X)
    lhs = x2 - np.sum(G * G)
    rhs = np.sum((X - Xh) ** 2)
    assert abs(lhs - rhs) <= 100 * EPS * x2
    disc = sum(float(np.sum(lam[n][ranks[n]:])) for n in range(3))
    assert abs(disc - rhs) <= 1e-10 * x2
    for n in range(3):
        np.testing.assert_allclose(U[n].T @ U[n], np.eye(ranks[n]), atol=1e-13)


def test_two_way_is_truncated_svd(orc):
    """P5: N = 2 reduces to the truncated SVD (Eckart-Young)."""
    A = rand_tensor((30, 20), 60)
    R = 6
    G, U, lam = orc.sthosvd(A, (R, R))
    s = np.linalg.svd(A, compute_uv=False)
    Ah = orc.reconstruct(G, U)
    np.testing.assert_allclose(np.sum((A - Ah) ** 2), np.sum(s[R:] ** 2), rtol=1e-11)
    np.testing.assert_allclose(np.sort(np.abs(np.diag(G)))[::-1], s[:R], rtol=1e-11)


def test_noise_closed_form(orc):
    """P6: for a low-rank tensor plus relative Gaussian noise nu, the error of
    the rank-R st-HOSVD approaches nu*sqrt(1 - prod R / prod I)/sqrt(1+nu^2)."""
    dims, ranks, nu = (40, 40, 40), (5, 5, 5), 1e-3
    X = wl.lowrank_plus_noise(dims, ranks, "none", nu, 99, "float64")
    G, U, _ = orc.sthosvd(X, ranks)
    e = np.linalg.norm(X - orc.reconstruct(G, U)) / np.linalg.norm(X)
    pred = nu * np.sqrt(1 - np.prod(ranks) / np.prod(dims)) / np.sqrt(1 + nu * nu)
    assert abs(e - pred) <= 0.01 * pred


def test_golden_hand_worked_example(orc):
    """Hand-derived example (tests/golden/diag2x2x2.json)."""
    with open(os.path.join(GOLDEN, "diag2x2x2.json")) as f:
        g = json.load(f)
    X = np.zeros((2, 2, 2), order="F")
    for (i, j, k), v in g["entries"]:
        X[i, j, k] = v
    G, U, lam = orc.sthosvd(X, g["ranks"])
    for n in range(3):
        np.testing.assert_allclose(lam[n], g["gram_eigenvalues"][n], rtol=0, atol=1e-14)
        np.testing.assert_allclose(U[n][:, 0], g["U_first_column"][n], rtol=0, atol=1e-14)
    np.testing.assert_allclose(G.reshape(-1), g["core"], rtol=0, atol=1e-14)
    e = np.linalg.norm(X - orc.reconstruct(G, U)) / np.linalg.norm(X)
    assert abs(e - g["rel_error"]) <= 1e-14


# --------------------------------------------------------- ALS (Alg. 3) ----

def test_als_variants_agree_and_mode_invariant(orc):
    """Plain Alg. 3 and the re-orthonormalized variant span the same
    subspaces: same projector, same new working tensor up to the rotation
    of U; and the per-mode energy identity holds for both."""
    X = wl.lowrank_plus_noise((20, 15, 12), (4, 3, 3), "none", 0.01, 5, "float64")
    Yn = numpy_unfold(X, 0)
    L0 = wl.gaussian_init(20, 4, 1, 0)
    outs = []
    for variant in (0, 1):
        U, Ynew = orc.als_mode(Yn, L0, iters=5, variant=variant)
        np.testing.assert_allclose(U.T @ U, np.eye(4), atol=1e-13)
        Yh = U @ Ynew
        y2 = np.sum(Yn * Yn)
        assert abs((y2 - np.sum(Ynew * Ynew)) - np.sum((Yn - Yh) ** 2)) <= 1e3 * EPS * y2
        outs.append((U, Ynew, Yh))
    np.testing.assert_allclose(outs[0][2], outs[1][2], rtol=0, atol=1e-10 * np.abs(Yn).max())
    np.testing.assert_allclose(outs[0][0] @ outs[0][0].T, outs[1][0] @ outs[1][0].T, atol=1e-10)


def test_als_converges_to_eig_subspace(orc):
    """ALS is a subspace iteration on Yn Yn^T: many sweeps reach the leading
    eigenspace, and the angle decays at least like (lam_{R+1}/lam_R)^k."""
    X = wl.lowrank_plus_noise((24, 18, 10), (3, 3, 3), "none", 0.05, 8, "float64")
    Yn = numpy_unfold(X, 0)
    L0 = wl.gaussian_init(24, 3, 2, 0)
    S = Yn @ Yn.T
    w, V = np.linalg.eigh(S)
    w, V = w[::-1], V[:, ::-1]
    P = V[:, :3] @ V[:, :3].T
    U, _ = orc.als_mode(Yn, L0, iters=40, variant=1)
    assert np.linalg.norm(U @ U.T - P, 2) <= 1e-9
    Q0, _ = np.linalg.qr(L0)
    s0 = np.linalg.norm((np.eye(24) - P) @ Q0, 2)
    c0 = np.sqrt(max(1e-300, 1 - s0 ** 2))
    for k in (1, 2, 3):
        Uk, _ = orc.als_mode(Yn, L0, iters=k, variant=1)
        sk = np.linalg.norm((np.eye(24) - P) @ Uk, 2)
        assert sk <= 1.01 * (s0 / c0) * (w[3] / w[2]) ** k + 1e-12


def test_flexible_all_als_matches_eig_on_exact_rank(orc):
    """Alg. 2 with every mode ALS (and mixed choices) on an exact-rank tensor
    recovers it exactly, like the all-EIG path."""
    X = wl.lowrank_plus_noise((16, 14, 12), (3, 4, 2), "none", 0.0, 3, "float64")
    L0 = [wl.gaussian_init(d, r, 4, n) for n, (d, r) in enumerate(zip(X.shape, (3, 4, 2)))]
    for methods in ((1, 1, 1), (0, 1, 0), (1, 0, 1)):
        for variant in (0, 1):
            G, U, _ = orc.sthosvd(X, (3, 4, 2), methods=methods, L0=L0, als_variant=variant)
            e = np.linalg.norm(X - orc.reconstruct(G, U)) / np.linalg.norm(X)
            assert e <= 1e-11
            assert abs(np.linalg.norm(G) - np.linalg.norm(X)) <= 1e-11 * np.linalg.norm(X)


# ---------------------------------------------------- reconstruction ----

def test_reconstruct_matches_einsum(orc):
    G = rand_tensor((2, 3, 4), 70)
    U = [rand_tensor((5, 2), 71), rand_tensor((6, 3), 72), rand_tensor((7, 4), 73)]
    ref = np.einsum("abc,ia,jb,kc->ijk", G, *U)
    np.testing.assert_allclose(orc.reconstruct(G, U), ref, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ MLP ----

def test_mlp_gradients_against_finite_differences(orc):
    rng = np.random.default_rng(5)
    widths = [10, 8, 6, 2]
    Ws = [rng.standard_normal((widths[i + 1], widths[i])) * 0.5 for i in range(3)]
    bs = [rng.standard_normal(widths[i + 1]) * 0.1 for i in range(3)]
    X = rng.standard_normal((10, 7))
    T = rng.standard_normal((2, 7))
    loss, dW, db = orc.mlp_loss_grad(Ws, bs, X, T)
    Y = orc.mlp_forward(Ws, bs, X)
    assert abs(loss - 0.5 / 7 * np.sum((Y - T) ** 2)) <= 1e-14
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0), (1, 2), (widths[l + 1] - 1, widths[l] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (orc.mlp_loss_grad(Wp, bs, X, T)[0] - orc.mlp_loss_grad(Wm, bs, X, T)[0]) / (2 * h)
            assert abs(fd - dW[l][idx]) <= 1e-7 * max(1.0, abs(fd))
        for o in (0, widths[l + 1] - 1):
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[l][o] += h
            bm[l][o] -= h
            fd = (orc.mlp_loss_grad(Ws, bp, X, T)[0] - orc.mlp_loss_grad(Ws, bm, X, T)[0]) / (2 * h)
            assert abs(fd - db[l][o]) <= 1e-7 * max(1.0, abs(fd))
    # a linear one-layer net is ordinary least squares
    W1 = [rng.standard_normal((2, 10))]
    b1 = [np.zeros(2)]
    _, g1, gb1 = orc.mlp_loss_grad(W1, b1, X, T)
    np.testing.assert_allclose(g1[0], (W1[0] @ X - T) @ X.T / 7, rtol=1e-12, atol=1e-14)


def test_mlp_forward_tanh_pins(orc):
    """The hidden activation pinned by properties of tanh itself, independent
    of the oracle's backward pass: (1) saturation: pre-activations of size
    >= 40 give exactly +-1, so a two-hidden-layer net reduces to
    W3 sign(W2 sign(W1 X + b1) + b2) + b3; (2) small signal: tanh z = z - z^3/3
    + O(z^5), so with inputs of size 1e-3 the net's deviation from the
    linear map W2 W1 X + b2 is -W2 (W1 X)^3 / 3 to relative O(z^2) (a sigmoid,
    ReLU or sine hidden layer fails one of the two)."""
    rng = np.random.default_rng(17)
    # (1) saturation through two hidden layers
    W1 = rng.choice([-1.0, 1.0], size=(6, 4)) * 50.0
    b1 = np.zeros(6)
    W2 = rng.choice([-1.0, 1.0], size=(5, 6)) * 50.0
    b2 = np.full(5, 25.0)                        # z2 = 50 * (odd count of +-1) + 25: |z2| >= 25
    W3 = rng.standard_normal((2, 5))
    b3 = rng.standard_normal(2)
    X = rng.choice([-1.0, 1.0], size=(4, 9)) * rng.uniform(1.0, 2.0, size=(4, 9))
    X[:, 0] = [1.0, 1.0, 1.0, 1.0]
    z1 = W1 @ X
    keep = np.all(np.abs(z1) >= 40.0, axis=0)    # columns whose every pre-activation saturates
    assert keep.sum() >= 1
    X = X[:, keep]
    h1 = np.sign(W1 @ X)
    h2 = np.sign(W2 @ h1 + b2[:, None])
    assert np.all(np.abs(W2 @ h1 + b2[:, None]) >= 25.0)
    Y = orc.mlp_forward([W1, W2, W3], [b1, b2, b3], X)
    np.testing.assert_allclose(Y, W3 @ h2 + b3[:, None], rtol=0, atol=1e-13)
    # (2) the cubic term of one hidden layer
    V1 = rng.standard_normal((7, 3))
    V2 = rng.standard_normal((2, 7))
    c2 = rng.standard_normal(2)
    Xs = rng.standard_normal((3, 11)) * 1e-3
    z = V1 @ Xs
    Ys = orc.mlp_forward([V1, V2], [np.zeros(7), c2], Xs)
    dev = Ys - (V2 @ z + c2[:, None])
    cubic = -V2 @ (z ** 3) / 3.0
    assert np.max(np.abs(dev - cubic)) <= 1e-4 * np.max(np.abs(cubic)), (dev, cubic)
