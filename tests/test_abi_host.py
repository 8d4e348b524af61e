"""Host-side checks of the C ABI: the library loads, exports every function
include/sthosvd.h declares, and validates plans before any launch.  No
kernel runs here (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sthosvd.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "defined")))


@pytest.fixture(scope="module")
def lib():
    from paper_2010_10131_amd import _lib
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    from paper_2010_10131_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_version_and_error_string(lib):
    assert lib.sth_version().startswith(b"sthosvd")
    assert isinstance(lib.sth_last_error(), bytes)


def _plan(**kw):
    import torch
    from paper_2010_10131_amd import api
    args = dict(dims=(16, 12, 10), ranks=(4, 3, 2), dtype=torch.float32, gram_prec="fp32",
                ttm_prec="fp32")
    args.update(kw)
    return api.Plan(**args)


def _err(**kw):
    from paper_2010_10131_amd._lib import SthError
    with pytest.raises(SthError) as e:
        _plan(**kw)
    return e.value.status


def test_plan_validation_errors():
    import torch
    from paper_2010_10131_amd import _lib
    INV, NOMEM, UNSUP = _lib.STH_ERR_INVALID, _lib.STH_ERR_NOMEM, _lib.STH_ERR_UNSUPPORTED
    assert _err(ranks=(4, 13, 2)) == INV           # R > I
    assert _err(ranks=(4, 0, 2)) == INV            # R < 1
    assert _err(dims=(16, 0, 10)) == INV           # empty mode
    assert _err(dims=(2,) * 9, ranks=(1,) * 9) == INV   # order > 8
    assert _err(mode_order=(0, 0, 1)) == INV       # not a permutation
    assert _err(dtype=torch.float64) == INV        # FP64 data needs FP64 contractions
    assert _err(gram_prec=7) == INV
    assert _err(solver=9) == INV
    assert _err(per_mode=(0, 5, 0)) == INV
    assert _err(workspace_cap=1024) == NOMEM       # cap below the need
    assert _err(dims=(600, 4, 4), ranks=(8, 2, 2)) == UNSUP  # EIG beyond the eigensolver limit
    assert _err(dims=(600, 300, 4), ranks=(8, 200, 2), per_mode=("als", "als", "eig")) == UNSUP


def test_als_above_the_rank_bound_of_the_unfolding():
    """Mode 1 of (64, 2, 2) with R_1 = 5 > J_1 = 4: ALS's normal equations
    would be singular.  Either learned selector takes EIG there; an explicit
    ALS request is refused before anything runs."""
    from paper_2010_10131_amd import _lib
    for solver in ("auto", "auto_tree"):
        assert _plan(dims=(64, 2, 2), ranks=(5, 2, 2), solver=solver).solvers[0] == 0
    assert _err(dims=(64, 2, 2), ranks=(5, 2, 2), per_mode=("als", "eig", "eig")) == _lib.STH_ERR_UNSUPPORTED
    # R_1 = J_1 is allowed
    assert _plan(dims=(64, 2, 2), ranks=(4, 2, 2), per_mode=("als", "eig", "eig")).solvers == [1, 0, 0]


def test_memory_model_moves_selected_eig_modes_to_als():
    """Under a workspace cap the learned selectors' EIG modes move to ALS,
    the largest EIG footprint (I_n^2 Gram, partial sums, eigensolver) first,
    until the plan fits; an explicit EIG request over the cap is NOMEM."""
    import torch
    from paper_2010_10131_amd import _lib
    dims, ranks = (512, 64, 64), (32, 8, 8)
    for solver in ("auto", "auto_tree"):
        free = _plan(dims=dims, ranks=ranks, solver=solver)
        assert free.solvers == [0, 0, 0]
        als1 = _plan(dims=dims, ranks=ranks, per_mode=("als", "eig", "eig"))
        assert als1.workspace_bytes < free.workspace_bytes
        capped = _plan(dims=dims, ranks=ranks, solver=solver, workspace_cap=als1.workspace_bytes)
        assert capped.solvers == [1, 0, 0]
        assert capped.workspace_bytes <= als1.workspace_bytes
        # a cap nothing fits under stays NOMEM
        assert _err(dims=dims, ranks=ranks, solver=solver, workspace_cap=1 << 20) == _lib.STH_ERR_NOMEM
    assert _err(dims=dims, ranks=ranks, per_mode=("eig", "eig", "eig"),
                workspace_cap=als1.workspace_bytes) == _lib.STH_ERR_NOMEM


def test_plan_shapes_solvers_and_workspace():
    import torch
    p = _plan()
    assert p.solvers == [0, 0, 0]
    base = p.workspace_bytes
    # the ping-pong buffers hold at least the mode-1 and mode-2 outputs
    assert base >= 4 * (4 * 12 * 10 + 4 * 3 * 10)
    q = _plan(per_mode=("als", "eig", "als"))
    assert q.solvers == [1, 0, 1]
    # ALS keeps R_k as a (L, R, M) tensor beside the working tensors (mode 1:
    # 4 x 12 x 10 FP32) and its small matrices (5 I x R + 9 R x R doubles)
    assert q.workspace_bytes >= 4 * (4 * 12 * 10) * 2 + 8 * (5 * 16 * 4 + 9 * 16)
    assert q.workspace_bytes != base
    r = _plan(dims=(16, 12, 10), ranks=(16, 12, 10))  # R = I: a rotation
    assert r.workspace_bytes > 0
    s = _plan(dims=(16, 12, 10), ranks=(4, 3, 2), mode_order=(2, 0, 1))
    assert s.solvers == [0, 0, 0]
    f = _plan(dtype=torch.float64, gram_prec="fp64", ttm_prec="fp64")
    assert f.workspace_bytes > base                 # FP64 working tensors


def test_building_block_workspace_queries(lib):
    from paper_2010_10131_amd._lib import i64arr
    dims = i64arr([64, 32, 16])
    assert lib.gram_mode_n_workspace(3, dims, 1, 0) > 0
    assert lib.gram_mode_n_workspace(3, dims, 1, 8) > 0
    assert lib.gram_mode_n_workspace(3, dims, 3, 0) == 0      # bad mode
    assert lib.ttm_mode_n_workspace(64, 8) >= 2 * 1 * 64 * 16 * 4
    assert lib.eig_leading_workspace(64) >= 2 * 64 * 64 * 8
    ranks = i64arr([4, 4, 4])
    assert lib.tucker_reconstruct_workspace(3, dims, ranks, 1) > 0
    assert lib.tucker_error_workspace(3, dims, ranks, 1) > lib.tucker_reconstruct_workspace(3, dims, ranks, 1)


def test_entry_points_reject_bad_arguments_before_launch(lib):
    from paper_2010_10131_amd import _lib
    dims = _lib.i64arr([8, 8, 8])
    # NULL pointers and misaligned pointers are rejected without touching the device
    st = lib.gram_mode_n(3, dims, 0, 1, 1, None, None, None, 0, None)
    assert st == _lib.STH_ERR_INVALID
    st = lib.gram_mode_n(3, dims, 0, 1, 1, ctypes.c_void_p(0x1004), ctypes.c_void_p(0x2000),
                         ctypes.c_void_p(0x3000), 1 << 20, None)
    assert st == _lib.STH_ERR_LAYOUT
    st = lib.gram_mode_n(3, dims, 5, 1, 1, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                         ctypes.c_void_p(0x3000), 1 << 20, None)
    assert st == _lib.STH_ERR_INVALID
    st = lib.gram_mode_n(3, dims, 0, 1, 1, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                         ctypes.c_void_p(0x3000), 16, None)
    assert st == _lib.STH_ERR_NOMEM
    st = lib.eig_leading(600, 4, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), None, 0,
                         ctypes.c_void_p(0x3000), 1 << 30, None)
    assert st == _lib.STH_ERR_UNSUPPORTED
    st = lib.ttm_mode_n(3, dims, 1, 0, 1, 1, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 0,
                        ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), 1 << 20, None)
    assert st == _lib.STH_ERR_INVALID
    assert b"R" in lib.sth_last_error()
    # prepared factors: sizes and argument checks before any launch
    assert 0 < lib.ttm_factor_bytes(64, 16, 1) <= lib.ttm_mode_n_workspace(64, 16)
    assert lib.ttm_factor_bytes(64, 16, 9) == 0 and lib.ttm_factor_bytes(0, 16, 1) == 0
    nb = lib.ttm_factor_bytes(40, 8, 2)
    st = lib.ttm_factor_prepare(40, 8, 2, ctypes.c_void_p(0x1000), 0, ctypes.c_void_p(0x2000),
                                nb - 16, None)
    assert st == _lib.STH_ERR_NOMEM
    st = lib.ttm_factor_prepare(40, 8, 2, ctypes.c_void_p(0x1001), 0, ctypes.c_void_p(0x2000),
                                nb, None)
    assert st == _lib.STH_ERR_LAYOUT
    st = lib.ttm_mode_n_prepared(3, dims, 1, 8, 1, 2, ctypes.c_void_p(0x1000),
                                 ctypes.c_void_p(0x2000), 16, ctypes.c_void_p(0x3000), None)
    assert st == _lib.STH_ERR_INVALID
    st = lib.ttm_mode_n_prepared(3, dims, 1, 8, 0, 2, ctypes.c_void_p(0x1000),
                                 ctypes.c_void_p(0x2000), 1 << 20, ctypes.c_void_p(0x3000), None)
    assert st == _lib.STH_ERR_INVALID      # FP64 data needs FP64 products
    # the entry point that allocates nothing: a factor whose split exceeds the
    # library scratch is refused before any device call
    assert lib.ttm_mode_n_noalloc_max_bytes() == 4 << 20
    big = _lib.i64arr([2, 4096])
    st = lib.ttm_mode_n_noalloc(2, big, 1, 512, 0, 0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 0,
                                ctypes.c_void_p(0x3000), None)
    assert st == _lib.STH_ERR_NOMEM and b"scratch" in lib.sth_last_error()
    st = lib.ttm_mode_n_noalloc(3, dims, 1, 4, 1, 2, ctypes.c_void_p(0x1008), ctypes.c_void_p(0x2000), 0,
                                ctypes.c_void_p(0x3000), None)
    assert st == _lib.STH_ERR_LAYOUT


def test_batched_plan_validation():
    import workloads as wl
    from paper_2010_10131_amd import api
    from paper_2010_10131_amd._lib import SthError, STH_ERR_UNSUPPORTED, STH_ERR_INVALID
    sh = wl.batch_shapes(16)
    p = api.BatchPlan(sh)
    assert p.count == 16 and p.workspace_bytes > 0
    with pytest.raises(SthError) as e:
        api.BatchPlan([((300, 20, 20), (100, 5, 5))])        # R_n > 64
    assert e.value.status == STH_ERR_UNSUPPORTED
    with pytest.raises(SthError) as e:
        api.BatchPlan([((30, 20, 20), (5, 5, 5)), ((30, 20), (5, 5))])  # mixed orders
    assert e.value.status == STH_ERR_INVALID


def test_batched_tiles_validation():
    import workloads as wl
    from paper_2010_10131_amd import api
    from paper_2010_10131_amd._lib import SthError, STH_ERR_INVALID
    sh = wl.batch_shapes(16)
    base = api.BatchPlan(sh).workspace_bytes
    # the default tiles are what a zero field selects
    assert api.BatchPlan(sh, tiles=(0, 0, 0)).workspace_bytes == base
    assert api.BatchPlan(sh, tiles=(4, 4, 4)).workspace_bytes == base
    for t in [(2, 1, 1), (16, 2, 8), (64, 4, 64)]:
        assert api.BatchPlan(sh, tiles=t).workspace_bytes > 0
    for bad in [(-1, 4, 4), (65, 4, 4), (4, 3, 4), (4, 8, 4), (4, 4, -2), (4, 4, 65)]:
        with pytest.raises(SthError) as e:
            api.BatchPlan(sh, tiles=bad)
        assert e.value.status == STH_ERR_INVALID, bad


def test_batched_plan_accepts_rank_above_the_gram_rank_bound():
    """Mode 3 of (33, 20, 150) with ranks (5, 3, 24): the Gram has rank <= 15
    < 24.  The batched eigen phase runs the direct solver for every order, so
    such a mode is planned like any other (the completing eigenvectors are an
    orthonormal basis of the null space)."""
    from paper_2010_10131_amd import api
    assert api.BatchPlan([((33, 20, 150), (5, 3, 24))]).workspace_bytes > 0
    assert api.BatchPlan([((33, 20, 150), (5, 4, 18))]).workspace_bytes > 0


def test_hooi_rejects_bad_arguments_before_launch(lib):
    from paper_2010_10131_amd import _lib
    vp = ctypes.c_void_p
    dims, ranks = _lib.i64arr([8, 8, 8]), _lib.i64arr([2, 3, 2])
    U = _lib.ptrarr([0x1000, 0x2000, 0x3000])
    need = lib.sth_hooi_workspace(3, dims, ranks, 1, 1)
    assert need > 0
    assert lib.sth_hooi_workspace(3, dims, _lib.i64arr([9, 2, 2]), 1, 1) == 0
    args = (vp(0x4000), U, vp(0x5000))
    assert lib.sth_hooi(3, _lib.i64arr([8, 600, 8]), ranks, 1, 1, 1, *args, 1, vp(0x6000), 1 << 40,
                        None) == _lib.STH_ERR_UNSUPPORTED
    assert lib.sth_hooi(3, dims, ranks, 1, 1, 1, *args, 1, vp(0x6000), need - 1, None) == _lib.STH_ERR_NOMEM
    assert lib.sth_hooi(3, dims, ranks, 1, 1, 1, *args, -1, vp(0x6000), need, None) == _lib.STH_ERR_INVALID
    assert lib.sth_hooi(1, dims, ranks, 1, 1, 1, *args, 1, vp(0x6000), need, None) == _lib.STH_ERR_INVALID
    assert lib.sth_hooi(3, dims, ranks, 0, 1, 1, *args, 1, vp(0x6000), need, None) == _lib.STH_ERR_INVALID
    assert lib.sth_hooi(3, dims, ranks, 1, 1, 1, vp(0x4000), None, vp(0x5000), 1, vp(0x6000), need,
                        None) == _lib.STH_ERR_INVALID


def test_exhaustive_selection_validates_before_launch(lib):
    from paper_2010_10131_amd import _lib
    dims, ranks = _lib.i64arr([64, 32, 16]), _lib.i64arr([8, 4, 4])
    nb = lib.sthosvd_choose_exhaustive_workspace(3, dims, ranks, _lib.STH_F32, 1, 1, 5)
    # at least the three tensor buffers of the largest intermediate (64 x 32 x 16 -> 8 x 32 x 16)
    assert nb >= 3 * 8 * 32 * 16 * 4
    assert lib.sthosvd_choose_exhaustive_workspace(3, dims, _lib.i64arr([65, 4, 4]), _lib.STH_F32, 1, 1, 5) == 0
    assert lib.sthosvd_choose_exhaustive_workspace(3, dims, None, _lib.STH_F32, 1, 1, 5) == 0
    out = (ctypes.c_int32 * 3)()
    assert lib.sthosvd_choose_exhaustive(3, dims, ranks, _lib.STH_F32, 1, 1, 5, None, out, None, None, 0,
                                         None) == _lib.STH_ERR_INVALID
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: the size check fails first
    assert lib.sthosvd_choose_exhaustive(3, dims, ranks, _lib.STH_F32, 1, 1, 5, fake, out, None, fake, nb - 1,
                                         None) == _lib.STH_ERR_NOMEM
