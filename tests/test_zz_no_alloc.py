"""ttm_mode_n_noalloc: the TTM entry point that allocates nothing (its
pre-split factor lives in the library's per-device scratch array).

Checked against ttm_mode_n on the same inputs -- the same kernels, so the
same bits -- and against the FP64 oracle's TTM within the contraction bound
of each precision, on two calls in a row (the second on a smaller input, so a
stale part of the shared scratch from the first call would show), and with
the output buffer passed in, so the call itself allocates nothing."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


def tol_for(prec, K):
    acc = U24 * (1 + 2 * K)
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


def randn(shape, seed, dtype):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape).astype(dtype))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_noalloc_matches_ttm_mode_n_twice_second_smaller(api, prec):
    dtype = "float64" if prec == "fp64" else "float32"
    # first call: a wide factor (many chunks and r-tiles of scratch in use);
    # second call: fewer chunks and tiles, on a smaller tensor
    for dims, n, R, seed in [((48, 520, 6), 1, 70, 1), ((33, 37, 5), 1, 9, 2)]:
        Y = randn(dims, seed, dtype)
        U = np.asfortranarray(np.random.default_rng(10 + seed).standard_normal((dims[n], R)))
        Yd, Ud = api.to_device(Y), api.to_device(U)
        oshape = list(dims)
        oshape[n] = R
        Z = api.fortran_empty(oshape, Yd.dtype, Yd.device)
        Z.fill_(float("nan"))
        api.ttm_mode_n_noalloc(Yd, Ud, n, prec, out=Z)
        got = api.to_numpy(Z)
        ref_lib = api.to_numpy(api.ttm_mode_n(Yd, Ud, n, prec))
        assert np.array_equal(got, ref_lib), f"{prec} {dims}: differs from ttm_mode_n"
        ref = oracle.ttm_tensor(Y, U.T, n)
        bound = oracle.ttm_tensor(np.abs(Y), np.abs(U).T, n)
        err = np.abs(got - ref)
        assert (err <= tol_for(prec, dims[n]) * bound + 1e-300).all(), f"{prec} {dims}: outside bound"


def test_noalloc_transposed_factor_and_fp32_data(api):
    Y = randn((6, 5, 7), 3, "float32")
    W = np.asfortranarray(np.random.default_rng(4).standard_normal((40, 5)))   # applied as is
    Yd, Wd = api.to_device(Y), api.to_device(W)
    a = api.to_numpy(api.ttm_mode_n_noalloc(Yd, Wd, 1, "fp32", transpose_u=True))
    b = api.to_numpy(api.ttm_mode_n(Yd, Wd, 1, "fp32", transpose_u=True))
    assert np.array_equal(a, b)


def test_noalloc_rejects_a_factor_above_the_scratch(api):
    from paper_2010_10131_amd import _lib
    L = _lib.load()
    cap = L.ttm_mode_n_noalloc_max_bytes()
    assert cap == 4 << 20
    # a 4096 x 512 factor in FP64 pieces needs 16 MiB of split factor
    assert L.ttm_factor_bytes(4096, 512, 0) > cap
    import torch
    Yd = api.fortran_empty((2, 4096), torch.float64, "cuda")
    Ud = api.fortran_empty((4096, 512), torch.float64, "cuda")
    with pytest.raises(_lib.SthError) as ei:
        api.ttm_mode_n_noalloc(Yd, Ud, 1, "fp64")
    assert ei.value.status == _lib.STH_ERR_NOMEM
