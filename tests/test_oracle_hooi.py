"""Pins of the oracle's HOOI (higher-order orthogonal iteration) against
what the mathematics fixes: for N = 2 it is the truncated SVD (Eckart-Young
error from numpy's SVD), the core norm never decreases from sweep to sweep
(HOOI maximizes ||G|| over orthonormal factors), a tensor of exact
multilinear rank is a fixed point of the st-HOSVD start, and the error
identity ||X - X^||^2 = ||X||^2 - ||G||^2 holds for orthonormal factors."""
import numpy as np
import pytest

import oracle
import workloads as wl


def err2(X, G, U):
    return float(np.linalg.norm(oracle.reconstruct(G, U) - X) ** 2)


def test_matrix_case_is_the_truncated_svd():
    rng = np.random.default_rng(1)
    X = np.asfortranarray(rng.standard_normal((30, 20)) @ np.diag(0.8 ** np.arange(20)) @ rng.standard_normal((20, 20)))
    R = (4, 4)
    s = np.linalg.svd(X, compute_uv=False)
    best = float(np.sum(s[4:] ** 2))
    G0, U0, _ = oracle.sthosvd(X, R)
    G, U = oracle.hooi(X, U0, sweeps=2)
    assert err2(X, G, U) == pytest.approx(best, rel=1e-10)
    # from a random orthonormal start it converges to the same optimum
    Q = [np.linalg.qr(rng.standard_normal((d, r)))[0] for d, r in zip(X.shape, R)]
    G, U = oracle.hooi(X, Q, sweeps=60)
    assert err2(X, G, U) == pytest.approx(best, rel=1e-8)


def test_core_norm_never_decreases_and_beats_sthosvd():
    rng = np.random.default_rng(2)
    X = np.asfortranarray(rng.standard_normal((12, 10, 8)))
    R = (3, 3, 2)
    G0, U0, _ = oracle.sthosvd(X, R)
    norms = [np.linalg.norm(G0)]
    U = U0
    for _ in range(6):
        G, U = oracle.hooi(X, U, sweeps=1)
        norms.append(np.linalg.norm(G))
    assert all(b >= a - 1e-12 * a for a, b in zip(norms, norms[1:])), norms
    assert norms[-1] > norms[0]   # a generic tensor: st-HOSVD is not optimal
    # orthonormal factors: ||X - X^||^2 = ||X||^2 - ||G||^2
    x2 = float(np.sum(X ** 2))
    assert err2(X, G, U) == pytest.approx(x2 - norms[-1] ** 2, rel=1e-10)
    for u in U:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-13)


def test_exact_multilinear_rank_is_a_fixed_point():
    X = wl.lowrank_plus_noise((14, 12, 10), (3, 4, 2), "none", 0.0, 5, "float64")
    R = (3, 4, 2)
    G0, U0, _ = oracle.sthosvd(X, R)
    G, U = oracle.hooi(X, U0, sweeps=1)
    for a, b in zip(U0, U):
        np.testing.assert_allclose(a @ a.T, b @ b.T, atol=1e-12)
    assert err2(X, G, U) <= 1e-24 * float(np.sum(X ** 2)) + 1e-26
    assert np.linalg.norm(G) == pytest.approx(np.linalg.norm(X), rel=1e-13)


def test_zero_sweeps_is_the_projection_of_the_start():
    rng = np.random.default_rng(3)
    X = np.asfortranarray(rng.standard_normal((6, 5, 4)))
    U0 = [np.linalg.qr(rng.standard_normal((d, r)))[0] for d, r in zip(X.shape, (2, 3, 2))]
    G, U = oracle.hooi(X, U0, sweeps=0)
    want = np.einsum("abc,ai,bj,ck->ijk", X, *U0)
    np.testing.assert_allclose(G, want, atol=1e-13)
