// Batched st-HOSVD: many independent tensors decomposed together, one
// launch per phase of a mode step for the whole batch:
//   grouped Gram      every (tensor, row range, output block) workgroup of
//                     one tile class in one grid, XCD-aware ids;
//   grouped reduce    the FP64 partial blocks of every tensor;
//   batched eigen     one workgroup per tensor: cyclic Jacobi (n <= 128) or
//                     subspace iteration + Rayleigh-Ritz (n > 128), all in the
//                     workgroup (small FP64 GEMMs, Cholesky-QR, Jacobi);
//   grouped split     every factor into matrix-core quads;
//   grouped TTM       workgroups assigned to tensors in proportion to rows.
// Shapes, workspace offsets and launch prefix sums are fixed at plan time
// and copied into the workspace at the start of a run; the caller's tensors
// are reached through device arrays of pointers.  The run is enqueue-only
// and graph-capturable.
#include "chol_body.h"
#include "common.h"
#include "eig_body.h"
#include "gram_body.h"
#include "internal.h"
#include "ttm_body.h"

namespace sth {

constexpr int BE_THREADS = 512;  // batched eigen workgroup (matches the Jacobi body)
// Dynamic LDS for Jacobi's A and V in the batched eigen kernel: the kernel's
// static LDS (Jacobi, Cholesky and selection arrays, about 11.3 KiB) must fit
// beside it in the 160 KiB of a workgroup; batch_step_launch checks the sum.
constexpr int BATCH_LDS_AV = 148 * 1024;
constexpr size_t WG_LDS_MAX = 160 * 1024;

__device__ __forceinline__ int find_segment(const int64_t *__restrict__ pref, int len, int64_t x) {
    // largest k with pref[k] <= x (pref[0] = 0, pref[len] = total)
    int lo = 0, hi = len;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ const float *bsrc(const BatchStep &d, char *ws, const void *const *Xp) {
    return d.src_off < 0 ? (const float *)Xp[d.tensor] : (const float *)(ws + d.src_off);
}
__device__ __forceinline__ float *bdst(const BatchStep &d, char *ws, void *const *Cp) {
    return d.dst_off < 0 ? (float *)Cp[d.tensor] : (float *)(ws + d.dst_off);
}

// ------------------------------------------------------------ grouped Gram

template <int PREC, int WT>
__global__ __launch_bounds__(256) void batch_gram_kernel(const BatchStep *__restrict__ descs,
                                                         const int32_t *__restrict__ list,
                                                         const int64_t *__restrict__ pref, int len,
                                                         int64_t total, char *__restrict__ ws,
                                                         const void *const *__restrict__ Xp) {
    const int64_t per_xcd = (total + 7) / 8;
    const int64_t lid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (lid >= total) return;
    const int k = find_segment(pref, len, lid);
    const BatchStep &d = descs[list[k]];
    const float *Y = bsrc(d, ws, Xp);
    double *part = (double *)(ws + d.part_off);
    const int64_t local = lid - pref[k];
    const int64_t P = d.L * d.M;
    if (d.L == 1 && WT >= 2) {
        if ((d.I & 3) == 0 && ((reinterpret_cast<uintptr_t>(Y) & 15) == 0))
            gram_l1_body<PREC, WT, WT, 2, 2, true>(Y, d.I, P, d.kper, d.nkc, d.nblocks, d.gram_wg, local, part);
        else
            gram_l1_body<PREC, WT, WT, 2, 2, false>(Y, d.I, P, d.kper, d.nkc, d.nblocks, d.gram_wg, local, part);
    } else {
        gram_body<float, PREC, WT, true>(Y, Y, d.L, d.I, d.I, P, d.kper, d.nkc, d.nbi, d.nbi,
                                        d.nblocks, d.gram_wg, local, part);
    }
}

template <int TB>
__global__ void batch_reduce_kernel(const BatchStep *__restrict__ descs,
                                    const int32_t *__restrict__ list,
                                    const int64_t *__restrict__ pref, int len,
                                    char *__restrict__ ws) {
    const int64_t gb = blockIdx.y;  // global block index over the class
    const int k = find_segment(pref, len, gb);
    const BatchStep &d = descs[list[k]];
    const int q = (int)(gb - pref[k]);
    int bi = 0;
    while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
    const int bj = q - bi * (bi + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= TB * TB) return;
    const int il = e % TB, jl = e / TB;
    const int64_t i = (int64_t)bi * TB + il, j = (int64_t)bj * TB + jl;
    if (i >= d.I || j >= d.I) return;
    if (bi == bj && il < jl) return;
    const double *part = (const double *)(ws + d.part_off);
    double *S = (double *)(ws + d.S_off);
    double s = 0.0;
    for (int c = 0; c < d.nkc; ++c) s += part[((int64_t)c * d.nblocks + q) * TB * TB + e];
    S[i + d.I * j] = s;
    if (i != j) S[j + d.I * i] = s;
}

// -------------------------------------------------- one-workgroup eigen

// C (m x n, ldc) = op(A) op(B) by one workgroup, 32 x 32 output tiles with
// 32-deep LDS slabs (tile storage in the dynamic LDS).
__device__ void wg_gemm(int ta, int tb, int m, int n, int k, const double *__restrict__ A,
                        int64_t lda, const double *__restrict__ B, int64_t ldb,
                        double *__restrict__ C, int64_t ldc) {
    extern __shared__ __align__(16) double s_dyn[];
    double *sA = s_dyn;             // [kk][33]
    double *sB = s_dyn + 32 * 33;   // [kk][33]
    const int tid = threadIdx.x;
    const int tx = tid % 32, ty = tid / 32;  // 512 threads: ty in 0..15, two columns each
    for (int r0 = 0; r0 < m; r0 += 32)
        for (int c0 = 0; c0 < n; c0 += 32) {
            double acc0 = 0.0, acc1 = 0.0;
            for (int kc = 0; kc < k; kc += 32) {
                __syncthreads();
                for (int e = tid; e < 32 * 32; e += BE_THREADS) {
                    const int a = e % 32, b = e / 32;
                    {
                        int r, kk;
                        if (ta) { kk = a; r = b; } else { r = a; kk = b; }
                        const int gr = r0 + r, gk = kc + kk;
                        double v = 0.0;
                        if (gr < m && gk < k) v = ta ? A[gk + lda * gr] : A[gr + lda * gk];
                        sA[kk * 33 + r] = v;
                    }
                    {
                        int cc, kk;
                        if (tb) { cc = a; kk = b; } else { kk = a; cc = b; }
                        const int gc = c0 + cc, gk = kc + kk;
                        double v = 0.0;
                        if (gc < n && gk < k) v = tb ? B[gc + ldb * gk] : B[gk + ldb * gc];
                        sB[kk * 33 + cc] = v;
                    }
                }
                __syncthreads();
#pragma unroll 8
                for (int kk = 0; kk < 32; ++kk) {
                    const double a = sA[kk * 33 + tx];
                    acc0 += a * sB[kk * 33 + ty];
                    acc1 += a * sB[kk * 33 + ty + 16];
                }
            }
            const int r = r0 + tx;
            if (r < m) {
                if (c0 + ty < n) C[r + ldc * (c0 + ty)] = acc0;
                if (c0 + ty + 16 < n) C[r + ldc * (c0 + ty + 16)] = acc1;
            }
        }
    __syncthreads();
}

// Cholesky-QR pass of the n x p matrix A into Q (one workgroup).
__device__ void wg_cholqr(const double *A, double *Q, int n, int p, double shift_rel, double *G,
                          double *Rinv, int64_t *flag) {
    wg_gemm(1, 0, p, p, n, A, n, A, n, G, p);
    chol_body<BE_THREADS>(G, p, p, shift_rel, nullptr, Rinv, flag);
    __syncthreads();
    wg_gemm(0, 0, n, p, p, A, n, Rinv, p, Q, n);
}

__device__ void wg_orth(double *A, double *Q, double *Z2, int n, int p, int passes, double *G,
                        double *Rinv, int64_t *flag) {
    const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * 1.1102230246251565e-16;
    wg_cholqr(A, Z2, n, p, shift * p, G, Rinv, flag);
    if (passes == 2) {
        wg_cholqr(Z2, Q, n, p, 0.0, G, Rinv, flag);
        return;
    }
    wg_cholqr(Z2, A, n, p, 0.0, G, Rinv, flag);
    wg_cholqr(A, Q, n, p, 0.0, G, Rinv, flag);
}

__global__ __launch_bounds__(BE_THREADS) void batch_eig_kernel(const BatchStep *__restrict__ descs,
                                                               char *__restrict__ ws,
                                                               double *const *__restrict__ Up,
                                                               int order, int mode,
                                                               int64_t *__restrict__ flag,
                                                               double tol, int max_sweeps) {
    const BatchStep &d = descs[blockIdx.x];
    const int n = (int)d.I, R = (int)d.R;
    const double *S = (const double *)(ws + d.S_off);
    double *U = Up[(int64_t)d.tensor * order + mode];
    double *scr = (double *)(ws + d.eig_off);
    if (d.sib == 0) {   // direct Jacobi
        if (jacobi_small_lds(n, true) <= (size_t)BATCH_LDS_AV)
            jacobi_small_body<true>(S, n, R, scr, U, nullptr, tol, max_sweeps, flag);
        else
            jacobi_small_body<false>(S, n, R, scr, U, nullptr, tol, max_sweeps, flag);
        return;
    }
    const int p = d.sib;
    double *Q = scr, *Z = Q + (int64_t)n * p, *Z2 = Z + (int64_t)n * p, *G = Z2 + (int64_t)n * p;
    double *Rinv = G + p * p, *T = Rinv + p * p, *W = T + p * p, *jac = W + p * p;
    for (int e = threadIdx.x; e < n * p; e += BE_THREADS)
        Q[e] = gaussian_value(0x5EED5EEDull, (uint64_t)n * 1000 + p, (uint64_t)e);
    __syncthreads();
    for (int it = 0; it < SI_ITERS_DEV; ++it) {
        wg_gemm(0, 0, n, p, n, S, n, Q, n, Z, n);
        wg_orth(Z, Q, Z2, n, p, it + 1 == SI_ITERS_DEV ? 3 : 2, G, Rinv, flag);
    }
    wg_gemm(0, 0, n, p, n, S, n, Q, n, Z, n);
    wg_gemm(1, 0, p, p, n, Q, n, Z, n, T, p);
    if (jacobi_small_lds(p, true) <= (size_t)BATCH_LDS_AV)
        jacobi_small_body<true>(T, p, R, jac, W, nullptr, tol, max_sweeps, flag);
    else
        jacobi_small_body<false>(T, p, R, jac, W, nullptr, tol, max_sweeps, flag);
    __syncthreads();
    wg_gemm(0, 0, n, R, p, Q, n, W, p, U, n);
    // sign rule on the columns of U
    for (int r = threadIdx.x; r < R; r += BE_THREADS) {
        int arg = 0;
        double best = fabs(U[(int64_t)n * r]);
        for (int i = 1; i < n; ++i) {
            const double v = fabs(U[i + (int64_t)n * r]);
            if (v > best) {
                best = v;
                arg = i;
            }
        }
        if (U[arg + (int64_t)n * r] < 0.0)
            for (int i = 0; i < n; ++i) U[i + (int64_t)n * r] = -U[i + (int64_t)n * r];
    }
}

// --------------------------------------------------- grouped split / TTM

template <int PREC>
__global__ void batch_prep_kernel(const BatchStep *__restrict__ descs, const int64_t *__restrict__ pref,
                                  int len, int64_t total, char *__restrict__ ws,
                                  double *const *__restrict__ Up, int order, int mode) {
    constexpr int NQ = Frag<PREC>::NQ;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const int k = find_segment(pref, len, gid);
    const BatchStep &d = descs[k];
    const double *U = Up[(int64_t)d.tensor * order + mode];
    uint4 *out = (uint4 *)(ws + d.uq_off);
    const int64_t g2 = gid - pref[k];
    const int lane = (int)(g2 % 64);
    const int64_t blk = g2 / 64;
    const int rt = (int)(blk % d.ntiles);
    const int c = (int)(blk / d.ntiles);
    const int g = lane / 16;
    const int64_t r = (int64_t)rt * 16 + lane % 16;
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int64_t kk = (int64_t)c * KC + 8 * g + j;
        x[j] = (kk < d.I && r < d.R) ? U[kk + d.I * r] : 0.0;
    }
    FragQ<PREC> f;
    make_frag(x, f.f);
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[(blk * NQ + q) * 64 + lane] = f.q[q];
}

template <int PREC, int RTB>
__global__ __launch_bounds__(64 * BT_WAVES) void batch_ttm_kernel(
    const BatchStep *__restrict__ descs, const int32_t *__restrict__ list,
    const int64_t *__restrict__ pref, int len, char *__restrict__ ws,
    const void *const *__restrict__ Xp, void *const *__restrict__ Cp) {
    constexpr int NT = (PREC == P_FP64) ? (RTB == 1 ? 2 : 1) : (RTB == 1 ? 4 : 2);
    const int k = find_segment(pref, len, blockIdx.x);
    const BatchStep &d = descs[list[k]];
    const float *Y = bsrc(d, ws, Xp);
    float *Z = bdst(d, ws, Cp);
    const uint4 *uq = (const uint4 *)(ws + d.uq_off);
    const int64_t wg = blockIdx.x - pref[k], nwg = pref[k + 1] - pref[k];
    const int64_t P = d.L * d.M;
    const int64_t nrb = (P + 16 * NT - 1) / (16 * NT);
    if (d.contig)
        ttm_body<float, PREC, NT, RTB, true, true, BT_WAVES>(Y, uq, Z, d.L, d.I, d.R, P, d.nchunks,
                                                             d.ntiles, nrb, wg, nwg, 0);
    else
        ttm_body<float, PREC, NT, RTB, false, true, BT_WAVES>(Y, uq, Z, d.L, d.I, d.R, P, d.nchunks,
                                                              d.ntiles, nrb, wg, nwg, 0);
}

// ---------------------------------------------------------------- host

size_t batch_gram_lds(int prec, int wt) {
    const int tb = 32 * wt, nq = prec_nq(prec);
    const size_t l1 = (size_t)2 * 2 * nq * 4 * tb * 16;
    const size_t gen = (size_t)2 * nq * tb * 4 * 16;
    return std::max(l1, gen);
}

size_t batch_eig_lds(int64_t n, int64_t p) {
    auto jac = [](int64_t m) -> size_t {
        const size_t both = jacobi_small_lds(m, true);
        return both <= (size_t)BATCH_LDS_AV ? both : jacobi_small_lds(m, false);
    };
    if (p == 0) return jac(n);
    return std::max({jac(p), chol_lds_bytes(p), (size_t)2 * 32 * 33 * 8});
}

size_t batch_eig_scratch(int64_t n, int64_t p) {
    if (p == 0) return std::max((size_t)2 * n * n * 8, jacobi_small_vg(n));
    return (size_t)(3 * n * p + 4 * p * p + 2 * p * p) * 8;
}

namespace {
template <int PREC, int WT>
hipError_t launch_bgram(const BatchLaunch &bl, const BatchTables &t, char *ws, const void *const *Xp,
                        size_t lds, hipStream_t s) {
    auto kern = batch_gram_kernel<PREC, WT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int64_t per_xcd = (bl.total + 7) / 8;
    hipLaunchKernelGGL(kern, dim3((unsigned)(per_xcd * 8)), dim3(256), lds, s, t.descs, bl.list, bl.pref,
                       bl.len, bl.total, ws, Xp);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_bgram_p(int wt, const BatchLaunch &bl, const BatchTables &t, char *ws,
                          const void *const *Xp, hipStream_t s) {
    const size_t lds = batch_gram_lds(PREC, wt);
    switch (wt) {
        case 1: return launch_bgram<PREC, 1>(bl, t, ws, Xp, lds, s);
        case 2: return launch_bgram<PREC, 2>(bl, t, ws, Xp, lds, s);
        default: return launch_bgram<PREC, 4>(bl, t, ws, Xp, lds, s);
    }
}

template <int PREC, int RTB>
hipError_t launch_bttm(const BatchLaunch &bl, const BatchTables &t, char *ws, const void *const *Xp,
                       void *const *Cp, size_t lds, hipStream_t s) {
    auto kern = batch_ttm_kernel<PREC, RTB>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)bl.total), dim3(64 * BT_WAVES), lds, s, t.descs, bl.list,
                       bl.pref, bl.len, ws, Xp, Cp);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_bttm_p(int rtb, const BatchLaunch &bl, const BatchTables &t, char *ws,
                         const void *const *Xp, void *const *Cp, size_t lds, hipStream_t s) {
    switch (rtb) {
        case 1: return launch_bttm<PREC, 1>(bl, t, ws, Xp, Cp, lds, s);
        case 2: return launch_bttm<PREC, 2>(bl, t, ws, Xp, Cp, lds, s);
        default: return launch_bttm<PREC, 4>(bl, t, ws, Xp, Cp, lds, s);
    }
}
}  // namespace

hipError_t batch_step_launch(const BatchTables &t, const BatchStepPlan &sp, int gram_prec,
                             int ttm_prec, int order, int mode, char *ws, const void *const *Xp,
                             void *const *Cp, double *const *Up, int64_t *flag, int max_sweeps,
                             hipStream_t s) {
    hipError_t e;
    for (const BatchLaunch &bl : sp.gram) {
        if (bl.len == 0) continue;
        switch (gram_prec) {
            case P_FP64: e = launch_bgram_p<P_FP64>(bl.cls, bl, t, ws, Xp, s); break;
            case P_FP32: e = launch_bgram_p<P_FP32>(bl.cls, bl, t, ws, Xp, s); break;
            case P_BF16X3: e = launch_bgram_p<P_BF16X3>(bl.cls, bl, t, ws, Xp, s); break;
            default: e = launch_bgram_p<P_BF16X6>(bl.cls, bl, t, ws, Xp, s); break;
        }
        if (e != hipSuccess) return e;
    }
    for (const BatchLaunch &bl : sp.reduce) {
        if (bl.len == 0) continue;
        const int tb = 32 * bl.cls;
        dim3 grid((unsigned)((tb * tb + 255) / 256), (unsigned)bl.total);
        if (bl.cls == 1) hipLaunchKernelGGL(batch_reduce_kernel<32>, grid, dim3(256), 0, s, t.descs, bl.list, bl.pref, bl.len, ws);
        else if (bl.cls == 2) hipLaunchKernelGGL(batch_reduce_kernel<64>, grid, dim3(256), 0, s, t.descs, bl.list, bl.pref, bl.len, ws);
        else hipLaunchKernelGGL(batch_reduce_kernel<128>, grid, dim3(256), 0, s, t.descs, bl.list, bl.pref, bl.len, ws);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        const size_t lds = sp.eig_lds;
        hipFuncAttributes fa;
        if ((e = hipFuncGetAttributes(&fa, (const void *)batch_eig_kernel)) != hipSuccess) return e;
        if (lds + fa.sharedSizeBytes > WG_LDS_MAX) return hipErrorInvalidConfiguration;
        if (lds > 64 * 1024) {
            e = hipFuncSetAttribute((const void *)batch_eig_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(batch_eig_kernel, dim3((unsigned)sp.count), dim3(BE_THREADS), lds, s, t.descs, ws, Up,
                           order, mode, flag, 1e-15, max_sweeps);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        const BatchLaunch &bl = sp.prep;
        const unsigned grid = (unsigned)((bl.total + 255) / 256);
        switch (ttm_prec) {
            case P_FP64: hipLaunchKernelGGL(batch_prep_kernel<P_FP64>, dim3(grid), dim3(256), 0, s, t.descs, bl.pref, bl.len, bl.total, ws, Up, order, mode); break;
            case P_FP32: hipLaunchKernelGGL(batch_prep_kernel<P_FP32>, dim3(grid), dim3(256), 0, s, t.descs, bl.pref, bl.len, bl.total, ws, Up, order, mode); break;
            case P_BF16X3: hipLaunchKernelGGL(batch_prep_kernel<P_BF16X3>, dim3(grid), dim3(256), 0, s, t.descs, bl.pref, bl.len, bl.total, ws, Up, order, mode); break;
            default: hipLaunchKernelGGL(batch_prep_kernel<P_BF16X6>, dim3(grid), dim3(256), 0, s, t.descs, bl.pref, bl.len, bl.total, ws, Up, order, mode); break;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (const BatchLaunch &bl : sp.ttm) {
        if (bl.len == 0) continue;
        const size_t lds = (size_t)sp.max_nchunks * bl.cls * prec_nq(ttm_prec) * 64 * 16;
        switch (ttm_prec) {
            case P_FP64: e = launch_bttm_p<P_FP64>(bl.cls, bl, t, ws, Xp, Cp, lds, s); break;
            case P_FP32: e = launch_bttm_p<P_FP32>(bl.cls, bl, t, ws, Xp, Cp, lds, s); break;
            case P_BF16X3: e = launch_bttm_p<P_BF16X3>(bl.cls, bl, t, ws, Xp, Cp, lds, s); break;
            default: e = launch_bttm_p<P_BF16X6>(bl.cls, bl, t, ws, Xp, Cp, lds, s); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sth
