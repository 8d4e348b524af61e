"""Seeded synthetic inputs for st-HOSVD (shared by the tests, the benchmark and
the CPU baseline).

This module only draws random numbers and assembles the low-rank-plus-noise
test tensors; it holds none of the decomposition's arithmetic and imports
neither the oracle nor the HIP library.  All tensors are column-major
(first index fastest), as the library expects.

Recipe (one per workload, numpy PCG64, seed = 20101013 + workload index):
  core    G0 with N(0,1) entries times an optional per-index decay
          (0.9^(i+j+k) or 2^-(sum k), 0-based indices);
  factors Q_n = Q of the QR of an I_n x R_n Gaussian with diag(R) > 0;
  X0      = G0 x_1 Q_1 ... x_N Q_N (the Tucker model);
  noise   X = X0 + E with ||E||_F = nu ||X0||_F exactly
          (E = nu ||X0|| Z / ||Z||, Z ~ N(0,1)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20101013


@dataclass
class Workload:
    name: str
    dims: tuple
    ranks: tuple
    decay: str = "none"          # "none" | "0.9" | "2^-k"
    nu: float = 0.0              # relative noise level
    dtype: str = "float32"       # storage dtype of the tensor
    seed: int = BASE_SEED
    notes: str = ""
    extra: dict = field(default_factory=dict)


# The five workloads (small parity case, headline case, 4-way, batched, 5-way).
C1 = Workload("c1_64cubed_fp64", (64, 64, 64), (8, 8, 8), "none", 1e-3, "float64", BASE_SEED + 0)
C2 = Workload("c2_512cubed_fp32", (512, 512, 512), (64, 64, 64), "0.9", 1e-4, "float32",
              BASE_SEED + 1)
C3 = Workload("c3_160pow4_fp32", (160, 160, 160, 160), (16, 16, 16, 16), "2^-k", 1e-5, "float32",
              BASE_SEED + 2)
C5 = Workload("c5_48pow5_fp32", (48, 48, 48, 48, 48), (8, 8, 8, 8, 8), "none", 1e-4, "float32",
              BASE_SEED + 4)


def orthonormal(rng: np.random.Generator, m: int, r: int) -> np.ndarray:
    """Q of the QR of an m x r Gaussian, signed so that diag(R) > 0."""
    A = rng.standard_normal((m, r))
    Q, R = np.linalg.qr(A)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return np.asfortranarray(Q * s)


def decay_weights(ranks, decay: str) -> np.ndarray:
    if decay == "none":
        return np.ones(tuple(ranks))
    idx = np.indices(tuple(ranks)).sum(axis=0).astype(np.float64)
    if decay == "0.9":
        return 0.9 ** idx
    if decay == "2^-k":
        return 2.0 ** (-idx)
    raise ValueError(decay)


def _mode_product(T: np.ndarray, A: np.ndarray, n: int) -> np.ndarray:
    """T x_n A for the generator only (numpy tensordot)."""
    out = np.tensordot(A, T, axes=([1], [n]))      # new axis first
    return np.moveaxis(out, 0, n)


def lowrank_plus_noise(dims, ranks, decay="none", nu=0.0, seed=BASE_SEED,
                       dtype="float32") -> np.ndarray:
    """Column-major tensor X = G0 x {Q_n} + E, ||E|| = nu ||X0|| (see module doc).

    Built slab by slab along the last mode so that 4-way and 5-way inputs of
    several GB never need a full FP64 copy."""
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(r) for r in ranks)
    N = len(dims)
    rng = np.random.default_rng(seed)
    G0 = rng.standard_normal(ranks) * decay_weights(ranks, decay)
    Q = [orthonormal(rng, dims[n], ranks[n]) for n in range(N)]
    noise_seed = int(rng.integers(0, 2**63 - 1))
    # Partial product over modes 0..N-2, then slab-wise over the last mode.
    T = G0
    for n in range(N - 1):
        T = _mode_product(T, Q[n], n)
    out = np.empty(dims, dtype=dtype, order="F")
    last = dims[-1]
    slab = max(1, int(2**26 // max(1, int(np.prod(dims[:-1])))))
    x0sq = 0.0
    for s0 in range(0, last, slab):
        s1 = min(last, s0 + slab)
        blk = np.tensordot(T, Q[-1][s0:s1, :], axes=([N - 1], [1]))
        x0sq += float(np.sum(blk * blk))
        out[..., s0:s1] = blk
    if nu > 0.0:
        # pass 1: ||Z||^2; pass 2: add the scaled noise (same stream)
        zsq = 0.0
        g = np.random.default_rng(noise_seed)
        for s0 in range(0, last, slab):
            s1 = min(last, s0 + slab)
            z = g.standard_normal(dims[:-1] + (s1 - s0,))
            zsq += float(np.sum(z * z))
        scale = nu * np.sqrt(x0sq) / np.sqrt(zsq)
        g = np.random.default_rng(noise_seed)
        for s0 in range(0, last, slab):
            s1 = min(last, s0 + slab)
            z = g.standard_normal(dims[:-1] + (s1 - s0,))
            blk = np.tensordot(T, Q[-1][s0:s1, :], axes=([N - 1], [1]))
            out[..., s0:s1] = (blk + scale * z).astype(dtype)
    return out


def make(w: Workload) -> np.ndarray:
    return lowrank_plus_noise(w.dims, w.ranks, w.decay, w.nu, w.seed, w.dtype)


def batch_shapes(count=256, seed=BASE_SEED + 3, lo=32, hi=256, rlo=0.10, rhi=0.25):
    """Shapes of the batched workload: 3-way tensors, each mode uniform in
    [lo, hi], rank = max(1, round(u * I_n)), u ~ U[rlo, rhi] per mode."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(count):
        d = tuple(int(x) for x in rng.integers(lo, hi + 1, size=3))
        r = tuple(max(1, int(round(float(rng.uniform(rlo, rhi)) * x))) for x in d)
        shapes.append((d, r))
    return shapes


def batch_tensors(count=256, seed=BASE_SEED + 3, nu=1e-4, dtype="float32", workers=1, **kw):
    """The batched workload: (shapes, tensors); tensor t uses seed + 1000 + t.

    Each tensor has its own seed, so `workers` > 1 (a thread pool; numpy's
    generators and BLAS release the GIL) gives the same tensors faster."""
    shapes = batch_shapes(count, seed, **kw)

    def one(t):
        d, r = shapes[t]
        return lowrank_plus_noise(d, r, "none", nu, seed + 1000 + t, dtype)

    if workers <= 1:
        return shapes, [one(t) for t in range(count)]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=int(workers)) as ex:
        xs = list(ex.map(one, range(count)))
    return shapes, xs


def gaussian_init(I: int, R: int, seed: int, mode: int) -> np.ndarray:
    """ALS initial guess L0 for one mode: I x R standard normal (column-major),
    seeded by (seed, mode); passed identically to both implementations."""
    rng = np.random.default_rng([int(seed), int(mode), 0xA15])
    return np.asfortranarray(rng.standard_normal((I, R)))


def lowrank_plus_noise_device(dims, ranks, decay="none", nu=0.0, seed=BASE_SEED, device="cuda"):
    """The same recipe as lowrank_plus_noise, drawn on the device with torch's
    seeded generator (different numbers, same distribution), for inputs of
    several GB where host generation would dominate.  FP32, column-major."""
    import torch
    dims = [int(d) for d in dims]
    ranks = [int(r) for r in ranks]
    N = len(dims)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    w = torch.from_numpy(decay_weights(ranks, decay)).to(device=device, dtype=torch.float64)
    G0 = torch.randn(ranks, generator=g, device=device, dtype=torch.float64) * w
    Q = []
    for n in range(N):
        A = torch.randn(dims[n], ranks[n], generator=g, device=device, dtype=torch.float64)
        q, r = torch.linalg.qr(A)
        Q.append(q * torch.sign(torch.diagonal(r)))
    # T in C order over reversed modes: element (i_N, ..., i_1)
    T = G0.permute(*range(N - 1, -1, -1)).contiguous()
    for n in range(N):
        ax = N - 1 - n
        T = torch.movedim(torch.tensordot(T, Q[n].t(), dims=([ax], [0])), -1, ax)
    X0 = T.to(torch.float32).contiguous()
    del T
    if nu > 0.0:
        E = torch.randn(X0.shape, generator=g, device=device, dtype=torch.float32)
        scale = nu * torch.linalg.vector_norm(X0.double()) / torch.linalg.vector_norm(E.double())
        X0.add_(E * scale.float())
        del E
    return X0.permute(*range(N - 1, -1, -1))
