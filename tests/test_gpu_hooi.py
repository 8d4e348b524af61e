"""HOOI on the device (sth_hooi: the decomposition's Gram, eigensolver and
TTM launches) against the oracle's HOOI from the same starting factors."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2010_10131_amd import api
    return api


def run(api, X, U0, sweeps, gp, tp):
    import torch
    dev = torch.device("cuda:0")
    Xd = api.to_device(X)
    U = [api.to_device(np.asfortranarray(u)) for u in U0]
    G, _ = api.hooi(Xd, U, sweeps, gp, tp)
    torch.cuda.synchronize(dev)
    return api.to_numpy(G), [api.to_numpy(u) for u in U]


def t2(X, G, U, Go, Uo):
    Xh = oracle.reconstruct(G, U)
    Xho = oracle.reconstruct(Go, Uo)
    return float(np.linalg.norm(Xh - Xho) / np.linalg.norm(np.asarray(X, dtype=np.float64)))


@pytest.mark.parametrize("dims,ranks,sweeps", [
    ((30, 24, 20), (5, 4, 3), 1),
    ((30, 24, 20), (5, 4, 3), 3),
    ((20, 18, 16, 14), (4, 4, 3, 3), 2),
    ((40, 33), (6, 5), 2),
])
def test_fp64_hooi_matches_oracle(api, dims, ranks, sweeps):
    rng = np.random.default_rng(sum(dims))
    X = np.asfortranarray(wl.lowrank_plus_noise(dims, ranks, "none", 1e-2, 9, "float64")
                          + 1e-3 * rng.standard_normal(dims))
    _, U0, _ = oracle.sthosvd(X, ranks)
    Go, Uo = oracle.hooi(X, U0, sweeps)
    G, U = run(api, X, U0, sweeps, "fp64", "fp64")
    assert t2(X, G, U, Go, Uo) <= 1e-12
    assert abs(np.linalg.norm(G) - np.linalg.norm(Go)) <= 1e-12 * np.linalg.norm(Go)
    for u in U:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)


@pytest.mark.parametrize("dims,ranks,gp,tp", [
    ((96, 64, 50), (24, 16, 8), "bf16x6", "bf16x3"),   # subspace iteration orders
    ((150, 40, 36), (12, 6, 5), "fp64", "fp32"),
])
def test_fp32_hooi_matches_oracle(api, dims, ranks, gp, tp):
    X = wl.lowrank_plus_noise(dims, ranks, "0.9", 1e-4, 13, "float32")
    _, U0, _ = oracle.sthosvd(X, ranks)
    Go, Uo = oracle.hooi(X, U0, 2)
    G, U = run(api, X, U0, 2, gp, tp)
    assert t2(X, G, U, Go, Uo) <= 1e-5
    assert abs(np.linalg.norm(G) - np.linalg.norm(Go)) <= 1e-5 * np.linalg.norm(Go)


def test_zero_sweeps_is_the_core_of_the_start(api):
    X = wl.lowrank_plus_noise((24, 20, 18), (4, 5, 3), "none", 1e-3, 3, "float64")
    _, U0, _ = oracle.sthosvd(X, (4, 5, 3))
    Go, _ = oracle.hooi(X, U0, 0)
    G, U = run(api, X, U0, 0, "fp64", "fp64")
    np.testing.assert_allclose(G, Go, atol=1e-12 * np.abs(Go).max())
    for a, b in zip(U, U0):
        np.testing.assert_array_equal(a, b)
