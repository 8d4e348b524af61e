"""The explicit-matricization st-HOSVD of the Fig. 8 comparison (Sec. V),
as bench.py runs it, against the oracle and against the matricization-free
path on the same input."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2010_10131_amd import api
    import bench
    return torch, api, bench


@pytest.mark.parametrize("dims,ranks", [((60, 40, 30), (8, 6, 5)), ((200, 150, 100), (20, 15, 10)),
                                        ((24, 20, 18, 16), (5, 4, 4, 3))])
def test_explicit_matricization_matches_oracle(env, dims, ranks):
    """Permuted copies + FP32 GEMMs + the library eigensolver give the
    oracle's X^ (FP64, explicit matricization, Jacobi) to FP32 product
    accuracy, and the same X^ as sthosvd_run with FP32 products."""
    torch, api, bench = env
    X = wl.lowrank_plus_noise(dims, ranks, "0.9", 1e-4, 41, "float32")
    Xd = api.to_device(X)
    Ge, Ue = bench.explicit_sthosvd(api, torch, Xd, ranks)
    Go, Uo, _ = oracle.sthosvd(X, ranks)
    Xo = oracle.reconstruct(Go, Uo)
    xn = np.linalg.norm(X.astype(np.float64))
    Xe = oracle.reconstruct(api.to_numpy(Ge).astype(np.float64), [api.to_numpy(u) for u in Ue])
    t_oracle = np.linalg.norm(Xe - Xo) / xn
    assert t_oracle <= 1e-5, t_oracle
    Gf, Uf, _ = api.sthosvd(Xd, ranks, "fp32", "fp32")
    Xf = oracle.reconstruct(api.to_numpy(Gf).astype(np.float64), [api.to_numpy(u) for u in Uf])
    assert np.linalg.norm(Xe - Xf) / xn <= 1e-5
    # the factors themselves agree with the oracle's up to FP32 rounding
    for u, uo in zip(Ue, Uo):
        u = api.to_numpy(u)
        assert np.linalg.norm(u @ u.T - uo @ uo.T, 2) <= 1e-3
