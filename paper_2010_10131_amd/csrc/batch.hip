// Batched st-HOSVD: many independent tensors decomposed together, one
// launch per phase of a mode step for the whole batch:
//   grouped Gram      every (tensor, row range, output block) workgroup of
//                     one tile class in one grid, XCD-aware ids;
//   grouped reduce    the FP64 partial blocks of every tensor;
//   batched eigen     one workgroup per tensor: the direct solver of
//                     teig_body.h (tridiagonalization, bisection, inverse
//                     iteration), the matrix in LDS up to order 128;
//   grouped split     every factor into matrix-core quads;
//   grouped TTM       workgroups assigned to tensors in proportion to rows.
// Shapes, workspace offsets and launch prefix sums are fixed at plan time
// and copied into the workspace at the start of a run; the caller's tensors
// are reached through device arrays of pointers.  The run is enqueue-only
// and graph-capturable.
#include "common.h"
#include "gram_body.h"
#include "internal.h"
#include "teig_body.h"
#include "ttm_body.h"

namespace sth {

constexpr int BE_THREADS = TE_T;  // batched eigen workgroup (the direct solver's)
// the eigen kernel's dynamic and static LDS must fit the 160 KiB of a
// workgroup; batch_step_launch checks the sum
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
__global__ __launch_bounds__(BE_THREADS) void batch_eig_kernel(const BatchStep *__restrict__ descs,
                                                               char *__restrict__ ws,
                                                               double *const *__restrict__ Up,
                                                               int order, int mode,
                                                               int64_t *__restrict__ flag) {
    const BatchStep &d = descs[blockIdx.x];
    const int n = (int)d.I, R = (int)d.R;
    const double *S = (const double *)(ws + d.S_off);
    double *U = Up[(int64_t)d.tensor * order + mode];
    const bool alds = n <= TE_LDS_N, zlds = teig_z_fits(n, R, alds);
    const TeScratch sc = teig_scratch_layout((double *)(ws + d.eig_off), n, R, alds);
    if (alds) {
        if (zlds) teig_body<true, true>(S, n, n, R, U, n, nullptr, true, sc, flag);
        else teig_body<true, false>(S, n, n, R, U, n, nullptr, true, sc, flag);
    } else {
        if (zlds) teig_body<false, true>(S, n, n, R, U, n, nullptr, true, sc, flag);
        else teig_body<false, false>(S, n, n, R, U, n, nullptr, true, sc, flag);
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

size_t batch_eig_lds(int64_t n, int64_t R) {
    const bool alds = n <= TE_LDS_N;
    return teig_lds_bytes(n, R, alds, teig_z_fits(n, R, alds), teig_v_keep(n, R, alds));
}

size_t batch_eig_scratch(int64_t n, int64_t R) { return teig_scratch_doubles(n, R, n <= TE_LDS_N) * 8; }

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
                           order, mode, flag);
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
