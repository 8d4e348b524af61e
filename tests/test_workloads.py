"""The seeded input generators (host and device recipes) produce what their
recipe states: exact multilinear rank before noise, the stated relative noise,
column-major layout, and the batched workload's shape ranges."""
import numpy as np
import pytest

import workloads as wl


def unfold_sv(X, n):
    M = np.moveaxis(np.asarray(X, dtype=np.float64), n, 0).reshape(X.shape[n], -1)
    return np.linalg.svd(M, compute_uv=False)


@pytest.mark.parametrize("dims,ranks", [((9, 7, 6), (3, 2, 4)), ((5, 6, 4, 3), (2, 3, 2, 2))])
def test_host_generator_rank_noise_layout(dims, ranks):
    X0 = wl.lowrank_plus_noise(dims, ranks, "none", 0.0, 11, "float64")
    X = wl.lowrank_plus_noise(dims, ranks, "none", 1e-2, 11, "float64")
    assert X.flags.f_contiguous
    for n in range(len(dims)):
        s = unfold_sv(X0, n)
        assert s[ranks[n] - 1] > 1e-8 * s[0]
        assert np.all(s[ranks[n]:] <= 1e-12 * s[0])
    assert abs(np.linalg.norm(X - X0) / np.linalg.norm(X0) - 1e-2) < 1e-12


@pytest.mark.parametrize("dims,ranks", [((9, 7, 6), (3, 2, 4)), ((5, 6, 4, 3, 4), (2, 3, 2, 2, 1))])
def test_device_generator_rank_noise_layout(dims, ranks):
    torch = pytest.importorskip("torch")
    X0 = wl.lowrank_plus_noise_device(dims, ranks, "none", 0.0, 5, "cpu")
    X = wl.lowrank_plus_noise_device(dims, ranks, "none", 1e-3, 5, "cpu")
    assert tuple(X.shape) == tuple(dims) and X.dtype == torch.float32
    # column-major strides: first index fastest
    st = [1]
    for d in dims[:-1]:
        st.append(st[-1] * d)
    assert tuple(X.stride()) == tuple(st)
    x0 = X0.numpy()
    for n in range(len(dims)):
        s = unfold_sv(x0, n)
        assert s[ranks[n] - 1] > 1e-3 * s[0]
        assert np.all(s[ranks[n]:] <= 1e-6 * s[0])     # FP32 storage
    rel = np.linalg.norm((X - X0).numpy().astype(np.float64)) / np.linalg.norm(x0.astype(np.float64))
    assert abs(rel - 1e-3) < 1e-6


def test_batch_shapes_ranges_and_parallel_equality():
    sh = wl.batch_shapes(64)
    for d, r in sh:
        assert len(d) == 3 and all(32 <= x <= 256 for x in d)
        for x, y in zip(d, r):
            assert 1 <= y and abs(y / x - 0.175) <= 0.075 + 0.5 / x
    a = wl.batch_tensors(3)[1]
    b = wl.batch_tensors(3, workers=3)[1]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
