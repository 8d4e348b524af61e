// Batched st-HOSVD: many independent tensors decomposed together, one
// launch per phase of a mode step for the whole batch.  Every intermediate
// is stored rotated (the TTM writes its output transposed), so the mode a
// step contracts is always first and every step is the contiguous L = 1
// view; after the last mode the core is in natural order.
//   grouped Gram      per tile class one grid: the skinny class (I <= 160,
//                     whole triangles per workgroup over column ranges) or
//                     every (tensor, row range, output block) workgroup,
//                     XCD-aware ids;
//   grouped reduce    the FP64 partial blocks of every tensor;
//   batched eigen     one workgroup per tensor: up to order 128 the direct
//                     solver of teig_body.h (tridiagonalization, bisection,
//                     inverse iteration); above it a subspace iteration
//                     inside the workgroup (FP64 matrix-core products,
//                     shifted Cholesky-QR, Rayleigh-Ritz with the direct
//                     solver on the p x p problem) accepted by the Ritz
//                     residual test, the direct solver on S otherwise;
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
        const bool v4 = (d.I & 3) == 0 && ((reinterpret_cast<uintptr_t>(Y) & 15) == 0);
        if constexpr (WT == 2) {
            // the 16-byte loader needs only 4-byte aligned rows
            if (d.I >= 4) {
                gram_l1_body<PREC, 2, 2, 2, 2, true, false, true>(Y, d.I, P, d.kper, d.nkc, d.nblocks, d.gram_wg, local, part);
                return;
            }
        }
        if (v4)
            gram_l1_body<PREC, WT, WT, 2, 2, true>(Y, d.I, P, d.kper, d.nkc, d.nblocks, d.gram_wg, local, part);
        else
            gram_l1_body<PREC, WT, WT, 2, 2, false>(Y, d.I, P, d.kper, d.nkc, d.nblocks, d.gram_wg, local, part);
    } else {
        gram_body<float, PREC, WT, true>(Y, Y, d.L, d.I, d.I, P, d.kper, d.nkc, d.nbi, d.nbi,
                                        d.nblocks, d.gram_wg, local, part);
    }
}

// The 128-wide class of a launch whose tensors all have L = 1 (the first mode
// step): eight waves of 64 x 32 tiles, as the single-tensor mode-1 Gram, with
// the 16-byte loads (any I >= 4).
template <int PREC>
__global__ __launch_bounds__(512) void batch_gram_l1w_kernel(const BatchStep *__restrict__ descs,
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
    if (d.I >= 4)
        gram_l1_body<PREC, 4, 2, 2, 4, true, false, true>(Y, d.I, P, d.kper, d.nkc, d.nblocks, d.gram_wg, local, part);
    else
        gram_l1_body<PREC, 4, 2, 2, 4, false>(Y, d.I, P, d.kper, d.nkc, d.nblocks, d.gram_wg, local, part);
}

// The skinny class (first mode step, I <= SK_MAXI): each workgroup of a
// tensor takes the whole lower triangle of its Gram in 32 x 32 super tiles
// over round-robin column blocks (the single-tensor skinny body), so no
// output tile is padded beyond 32 rows and the tensor is read once.
// 32-column chunks per stage: TBp * CH loader tasks, one per thread; CH = 4
// (twice the bytes in flight per stage) where 32 * ceil(I / 32) <= 128 and the
// two stages fit the LDS (fragments of at most two bf16 parts)
constexpr int BSK_CH = 2, BSK_CH4_MAXI = 128;
__host__ __device__ inline int bsk_ch(int prec, int64_t I) {
    return (I <= BSK_CH4_MAXI && (prec == P_FP32 || prec == P_BF16X3)) ? 4 : BSK_CH;
}
template <int PREC>
__global__ __launch_bounds__(SK_T) void batch_gram_skinny_kernel(const BatchStep *__restrict__ descs,
                                                                const int32_t *__restrict__ list,
                                                                const int64_t *__restrict__ pref, int len,
                                                                int64_t total, char *__restrict__ ws,
                                                                const void *const *__restrict__ Xp) {
    const int64_t per_xcd = (total + 7) / 8;
    const int64_t lid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (lid >= total) return;
    const int k = find_segment(pref, len, lid);
    const BatchStep &d = descs[list[k]];
    if (bsk_ch(PREC, d.I) == 4)
        gram_skinny_body<PREC, 4, true, true>(bsrc(d, ws, Xp), (int)d.I, d.L * d.M, d.nkc, (int)(lid - pref[k]),
                                        (double *)(ws + d.part_off));
    else
        gram_skinny_body<PREC, BSK_CH, true, true>(bsrc(d, ws, Xp), (int)d.I, d.L * d.M, d.nkc, (int)(lid - pref[k]),
                                             (double *)(ws + d.part_off));
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
// ---- subspace iteration inside one workgroup (orders above 128) ----------
// Scratch after the direct solver's (doubles): Q, Z, Z2 (n x p each), G, Rinv,
// T, W (p x p each), th (p), res (R + 1), then the p x p direct solve's.
__host__ __device__ inline size_t bsi_doubles(int64_t n, int64_t p, int64_t R) {
    return (size_t)(3 * n * p + 4 * p * p + p + R + 1) + teig_scratch_doubles(p, R, true) + 64;
}

constexpr int BW = BE_THREADS / 64;   // waves
// Products of the iteration (operands contiguous column-major) stage their
// shared operand through the dynamic LDS in slabs of BK contraction rows
// (column stride BLD doubles: the 16 columns x 4 rows of a matrix-core
// fragment then hit every bank twice, the minimum for 64 lanes of 8 bytes);
// the next slab is prefetched into registers while the current one is
// used.  Operands are read through buffer resources whose range check
// returns zero past the matrix, so ragged edges need no selects.
constexpr int BK = 32;
constexpr int BLD = BK + 4;
constexpr int BK_COLS = BE_THREADS / BK;        // slab columns per pass of the workgroup
constexpr int BSI_PF = 128 / BK_COLS;           // passes for 128 columns
static_assert(BK_COLS == 16, "a pass covers one 16-column tile");
constexpr int BSI_OOB = 0x7FFFFFF0;             // byte offset past every operand

// LDS of the staged products for blocks of width p (two operand slabs)
__host__ __device__ inline size_t bsi_stage_bytes(int64_t p) {
    return (size_t)2 * 16 * ((p + 15) / 16) * BLD * sizeof(double);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t bsi_rsrc(const double *p, int64_t count) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)(count * (int64_t)sizeof(double)), 0x00020000);
}
__device__ __forceinline__ double bsi_ld(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}

// rows k0 .. k0 + BK - 1 of the k x q matrix behind rb into registers (zero
// outside it): the r-th value of a thread is column r * BK_COLS + tid / BK
__device__ __forceinline__ void bsi_slab_load(double (&pf)[BSI_PF], __amdgpu_buffer_rsrc_t rb, int k, int q, int k0) {
    const int kk = k0 + threadIdx.x % BK, c0 = threadIdx.x / BK;
    const bool kok = kk < k;
#pragma unroll
    for (int r = 0; r < BSI_PF; ++r)
        if (BK_COLS * r < q) pf[r] = bsi_ld(rb, kok ? 8 * (kk + k * (c0 + BK_COLS * r)) : BSI_OOB);
}
// columns below 16 * ceil(q / 16) into the slab (uniform in r)
__device__ __forceinline__ void bsi_slab_store(const double (&pf)[BSI_PF], double *s, int q) {
    const int kk = threadIdx.x % BK, c0 = threadIdx.x / BK;
#pragma unroll
    for (int r = 0; r < BSI_PF; ++r)
        if (BK_COLS * r < q) s[kk + BLD * (c0 + BK_COLS * r)] = pf[r];
}

// C (m x q) = A (m x k) B (k x q), q <= 128, on the FP64 matrix cores: each
// wave owns a 16-row strip and every column tile of it (up to 8
// accumulators), its A fragments read from memory (16 consecutive rows per
// column: coalesced), B staged slab by slab in the LDS for all waves.
// TRI_B: B upper triangular (k = q; slabs below a tile's rows skipped).
// NS: C = 1.5 A - 0.5 A B.
template <bool TRI_B, bool NS>
__device__ void bsi_nn(int m, int q, int k, const double *__restrict__ A, const double *__restrict__ B,
                       double *__restrict__ C) {
    extern __shared__ __align__(16) double s_st[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tr = lane & 15, tg = lane >> 4;
    const int mt = (m + 15) >> 4, qt = (q + 15) >> 4, nsl = (k + BK - 1) / BK;
    const __amdgpu_buffer_rsrc_t ra = bsi_rsrc(A, (int64_t)m * k), rb = bsi_rsrc(B, (int64_t)k * q);
    for (int rd = 0; rd * BW < mt; ++rd) {
        const int i0 = (rd * BW + wave) << 4;
        const bool act = i0 < m;
        // byte offset of this lane's row at contraction index 0 (past A when
        // the row is out of range); the range check zeroes k >= k
        const int abase = i0 + tr < m ? 8 * (i0 + tr) + 8 * m * tg : BSI_OOB;
        const int astep = 8 * m * 4;
        f64x4 acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
        double pf[BSI_PF], a[BK / 4], an[BK / 4];
        bsi_slab_load(pf, rb, k, q, 0);
#pragma unroll
        for (int u = 0; u < BK / 4; ++u) an[u] = bsi_ld(ra, abase == BSI_OOB ? BSI_OOB : abase + astep * u);
        for (int sl = 0; sl < nsl; ++sl) {
            const int k0 = sl * BK;
            __syncthreads();   // every wave is done with the previous slab
            bsi_slab_store(pf, s_st, q);
#pragma unroll
            for (int u = 0; u < BK / 4; ++u) a[u] = an[u];
            __syncthreads();
            if (sl + 1 < nsl) {
                bsi_slab_load(pf, rb, k, q, k0 + BK);
#pragma unroll
                for (int u = 0; u < BK / 4; ++u)
                    an[u] = bsi_ld(ra, abase == BSI_OOB ? BSI_OOB : abase + astep * ((k0 + BK) / 4 + u));
            }
            if (act) {
                // one uniform branch per tile and slab; TRI_B skips the
                // slabs below the tile's last row of B
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (j < qt && (!TRI_B || k0 < 16 * j + 16)) {
#pragma unroll
                        for (int u = 0; u < BK / 4; ++u) {
                            const double b = s_st[4 * u + tg + BLD * (16 * j + tr)];
                            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b, acc[j], 0, 0, 0);
                        }
                    }
                }
            }
        }
        if (act) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int col = 16 * j + tr;
                if (j < qt && col < q) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = i0 + tg + 4 * v;
                        if (row < m) C[row + (int64_t)m * col] = NS ? 1.5 * A[row + (int64_t)m * col] - 0.5 * acc[j][v] : acc[j][v];
                    }
                }
            }
        }
    }
}

// C (p x q) = A^T B with A (k x p), B (k x q), p, q <= 128: both operands
// staged slab by slab in the LDS, the output tiles dealt to the waves (up to
// 8 each).  SYM: B = A, tiles on and below the diagonal, each written to
// both halves.
template <bool SYM>
__device__ void bsi_tn(int p, int q, int k, const double *__restrict__ A, const double *__restrict__ B,
                       double *__restrict__ C) {
    extern __shared__ __align__(16) double s_st[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tr = lane & 15, tg = lane >> 4;
    const int pt = (p + 15) >> 4, qt = (q + 15) >> 4, nsl = (k + BK - 1) / BK;
    const int ntile = SYM ? pt * (pt + 1) / 2 : pt * qt;
    const __amdgpu_buffer_rsrc_t ra = bsi_rsrc(A, (int64_t)k * p), rb = bsi_rsrc(B, (int64_t)k * q);
    double *s_a = s_st, *s_b = SYM ? s_st : s_st + BLD * 16 * pt;
    int ti[8], tj[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int t = wave + BW * j;
        int bi = 0, bj = 0;
        if (t < ntile) {
            if (SYM) {
                while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
                bj = t - bi * (bi + 1) / 2;
            } else {
                bi = t % pt;
                bj = t / pt;
            }
        }
        ti[j] = bi << 4;
        tj[j] = bj << 4;
    }
    f64x4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
    double pa[BSI_PF], pb[BSI_PF];
    bsi_slab_load(pa, ra, k, p, 0);
    if (!SYM) bsi_slab_load(pb, rb, k, q, 0);
    for (int sl = 0; sl < nsl; ++sl) {
        __syncthreads();
        bsi_slab_store(pa, s_a, p);
        if (!SYM) bsi_slab_store(pb, s_b, q);
        __syncthreads();
        if (sl + 1 < nsl) {
            bsi_slab_load(pa, ra, k, p, (sl + 1) * BK);
            if (!SYM) bsi_slab_load(pb, rb, k, q, (sl + 1) * BK);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (wave + BW * j < ntile) {
#pragma unroll
                for (int u = 0; u < BK / 4; ++u) {
                    const double a = s_a[4 * u + tg + BLD * (ti[j] + tr)];
                    const double b = s_b[4 * u + tg + BLD * (tj[j] + tr)];
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int col = tj[j] + tr;
        if (wave + BW * j < ntile && col < q) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = ti[j] + tg + 4 * v;
                if (row < p) {
                    C[row + p * col] = acc[j][v];
                    if (SYM && ti[j] != tj[j]) C[col + p * row] = acc[j][v];
                }
            }
        }
    }
}

struct BsiWs {
    double *Q, *Z, *Z2, *G, *Rinv, *T, *W, *th, *res;
    TeScratch te;
};

__device__ inline BsiWs bsi_layout(double *base, int n, int p, int R) {
    BsiWs w;
    double *d = (double *)(((uintptr_t)base + 255) & ~(uintptr_t)255);
    w.Q = d; d += (int64_t)n * p;
    w.Z = d; d += (int64_t)n * p;
    w.Z2 = d; d += (int64_t)n * p;
    w.G = d; d += p * p;
    w.Rinv = d; d += p * p;
    w.T = d; d += p * p;
    w.W = d; d += p * p;
    w.th = d; d += p;
    w.res = d; d += R + 1;
    w.te = teig_scratch_layout(d, p, R, true);
    return w;
}

// One Cholesky-QR pass of the n x p matrix A into Q (shift_rel > 0: the
// shifted pass of the shifted Cholesky-QR3 scheme).
__device__ void bsi_cholqr(const double *A, double *Q, int n, int p, double shift_rel, BsiWs &w, int64_t *flag) {
    bsi_tn<true>(p, p, n, A, A, w.G);
    __syncthreads();
    chol_body<BE_THREADS>(w.G, p, p, shift_rel, nullptr, w.Rinv, flag);
    __syncthreads();
    bsi_nn<true, false>(n, p, p, A, w.Rinv, Q);
    __syncthreads();
}

// R leading eigenpairs of S (n > 128) into U by the subspace iteration of the
// single-tensor path (2 products when S carries single-precision rounding,
// 3 for FP64 data; intermediate bases: shifted + plain Cholesky-QR; the last:
// + a Newton-Schulz step, or + a third plain pass for FP64 data) and
// Rayleigh-Ritz with the direct solver on T = Q^T S Q.  Returns true when
// every Ritz residual passes ||S u - theta u|| <= tol |theta_1|.
__device__ bool bsi_solve(const double *S, int n, int R, int p, double s_unit, double *U, BsiWs &w,
                          int64_t *flag, uint64_t stream) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool loose = s_unit >= 0x1p-24;
    const int iters = loose ? 2 : 3;
    // start block: independent uniform values in [-1, 1) (any block with a
    // component along every wanted eigenvector converges)
    const uint64_t key = splitmix64(0x5EED5EEDull ^ (stream << 20));
    for (int64_t e = tid; e < (int64_t)n * p; e += BE_THREADS)
        w.Q[e] = (double)(int64_t)splitmix64(key + (uint64_t)e) * 0x1p-63;
    __syncthreads();
    const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * 1.1102230246251565e-16 * p;
    for (int it = 0; it < iters; ++it) {
        bsi_nn<false, false>(n, p, n, S, w.Q, w.Z);
        __syncthreads();
        bsi_cholqr(w.Z, w.Z2, n, p, shift, w, flag);
        if (it + 1 < iters) {
            bsi_cholqr(w.Z2, w.Q, n, p, 0.0, w, flag);
        } else if (loose) {
            bsi_cholqr(w.Z2, w.Z, n, p, 0.0, w, flag);
            bsi_tn<true>(p, p, n, w.Z, w.Z, w.G);
            __syncthreads();
            bsi_nn<false, true>(n, p, p, w.Z, w.G, w.Q);
            __syncthreads();
        } else {
            bsi_cholqr(w.Z2, w.Z, n, p, 0.0, w, flag);
            bsi_cholqr(w.Z, w.Q, n, p, 0.0, w, flag);
        }
    }
    // Rayleigh-Ritz
    bsi_nn<false, false>(n, p, n, S, w.Q, w.Z);
    __syncthreads();
    bsi_tn<false>(p, p, n, w.Q, w.Z, w.T);
    __syncthreads();
    if (teig_z_fits(p, R, true)) teig_body<true, true>(w.T, p, p, R, w.W, p, w.th, false, w.te, flag);
    else teig_body<true, false>(w.T, p, p, R, w.W, p, w.th, false, w.te, flag);
    __syncthreads();
    // U = Q W and V = Z W on the matrix cores (V in Z2), then per vector
    // (one wave each) the Ritz residual ||V(:, r) - theta_r U(:, r)|| and the
    // sign rule
    bsi_nn<false, false>(n, R, p, w.Q, w.W, U);
    bsi_nn<false, false>(n, R, p, w.Z, w.W, w.Z2);
    __syncthreads();
    for (int r = wave; r < R; r += BW) {
        const double t = w.th[r];
        double ss = 0.0, best = -1.0, bval = 0.0;
        int arg = 0;
        for (int i = lane; i < n; i += 64) {
            const double u = U[i + (int64_t)n * r];
            const double d = w.Z2[i + (int64_t)n * r] - t * u;
            ss += d * d;
            if (fabs(u) > best) {
                best = fabs(u);
                arg = i;
                bval = u;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            ss += __shfl_xor(ss, o);
            const double b2 = __shfl_xor(best, o), v2 = __shfl_xor(bval, o);
            const int a2 = __shfl_xor(arg, o);
            if (b2 > best || (b2 == best && a2 < arg)) {
                best = b2;
                arg = a2;
                bval = v2;
            }
        }
        if (bval < 0.0)
            for (int i = lane; i < n; i += 64) U[i + (int64_t)n * r] = -U[i + (int64_t)n * r];
        if (lane == 0) w.res[r] = sqrt(ss);
    }
    __syncthreads();
    const double tol = fmax(16.0 * sqrt((double)n) * 2.220446049250313e-16, s_unit) * fabs(w.th[0]);
    int bad = 0;
    for (int r = lane; r < R; r += 64)
        if (!(w.res[r] <= tol)) bad = 1;
    const bool ok = __ballot(bad) == 0;   // every wave reads the same values
    __syncthreads();
    return ok;
}

__global__ __launch_bounds__(BE_THREADS) void batch_eig_kernel(const BatchStep *__restrict__ descs,
                                                               char *__restrict__ ws,
                                                               double *const *__restrict__ Up,
                                                               int order, int mode, double s_unit,
                                                               int64_t *__restrict__ flag) {
    const BatchStep &d = descs[blockIdx.x];
    const int n = (int)d.I, R = (int)d.R;
    const double *S = (const double *)(ws + d.S_off);
    double *U = Up[(int64_t)d.tensor * order + mode];
    const bool alds = n <= TE_LDS_N, zlds = teig_z_fits(n, R, alds);
    double *const base = (double *)(ws + d.eig_off);
    const TeScratch sc = teig_scratch_layout(base, n, R, alds);
    if (d.sib > 0) {
        // the subspace iteration; its scratch follows the direct solver's
        BsiWs w = bsi_layout(base + teig_scratch_doubles(n, R, alds), n, d.sib, R);
        if (bsi_solve(S, n, R, d.sib, s_unit, U, w, flag ? flag + 2 : nullptr,
                      (uint64_t)n * 1000 + d.sib))
            return;
        if (threadIdx.x == 0 && flag) atomicAdd((unsigned long long *)(flag + 1), 1ull);   // direct solves taken
    }
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
    // every step is the L = 1 view of the rotated layout; the output goes out
    // transposed, which makes the next mode the first
    ttm_body<float, PREC, NT, RTB, true, true, BT_WAVES, 1, true>(Y, uq, Z, 1, d.I, d.R, P, d.nchunks,
                                                                 d.ntiles, nrb, wg, nwg, 0);
}

// ---------------------------------------------------------------- host

bool batch_gram_skinny(int prec, int64_t L, int64_t I, int64_t P, int64_t target, int *ns, int *nkc) {
    if (L != 1 || I > SK_MAXI) return false;
    *ns = sk_ns(I);
    const int ch = bsk_ch(prec, I);
    const int64_t nblk = (P + 32 * ch - 1) / (32 * ch);
    // about `target` workgroups, each at least eight stages (the partial
    // triangles a workgroup writes stay well below what it reads)
    *nkc = (int)std::max<int64_t>(1, std::min<int64_t>(target, nblk / 8));
    return true;
}

size_t batch_gram_lds(int prec, int wt) {
    if (wt == BATCH_SKINNY)   // the larger of the two stage shapes
        return std::max((size_t)2 * BSK_CH * prec_nq(prec) * 4 * 32 * sk_ns(SK_MAXI) * 16,
                        (size_t)2 * bsk_ch(prec, BSK_CH4_MAXI) * prec_nq(prec) * 4 * BSK_CH4_MAXI * 16);
    const int tb = 32 * wt, nq = prec_nq(prec);
    const size_t l1 = (size_t)2 * 2 * nq * 4 * tb * 16;
    const size_t gen = (size_t)2 * nq * tb * 4 * 16;
    return std::max(l1, gen);
}

int64_t batch_si_block(int64_t n, int64_t R, int64_t rank_bound) {
    const int64_t p = si_block_host(n, R);
    return (n > TE_LDS_N && p <= SI_BLOCK_MAX && p < n && R <= rank_bound) ? p : 0;
}

size_t batch_eig_lds(int64_t n, int64_t R, int64_t p) {
    const bool alds = n <= TE_LDS_N;
    size_t b = teig_lds_bytes(n, R, alds, teig_z_fits(n, R, alds), teig_v_keep(n, R, alds));
    if (p > 0) {
        b = std::max(b, teig_lds_bytes(p, R, true, teig_z_fits(p, R, true), teig_v_keep(p, R, true)));
        b = std::max(b, chol_lds_bytes(p));
        b = std::max(b, bsi_stage_bytes(p));
    }
    return b;
}

size_t batch_eig_scratch(int64_t n, int64_t R, int64_t p) {
    size_t d = teig_scratch_doubles(n, R, n <= TE_LDS_N);
    if (p > 0) d += bsi_doubles(n, p, R);
    return d * 8;
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
    if (wt == BATCH_SKINNY) {
        auto kern = batch_gram_skinny_kernel<PREC>;
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        const int64_t per_xcd = (bl.total + 7) / 8;
        hipLaunchKernelGGL(kern, dim3((unsigned)(per_xcd * 8)), dim3(SK_T), lds, s, t.descs, bl.list, bl.pref,
                           bl.len, bl.total, ws, Xp);
        return hipGetLastError();
    }
    if (wt == 4 && bl.l1) {
        auto kern = batch_gram_l1w_kernel<PREC>;
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        const int64_t per_xcd = (bl.total + 7) / 8;
        hipLaunchKernelGGL(kern, dim3((unsigned)(per_xcd * 8)), dim3(512), lds, s, t.descs, bl.list, bl.pref,
                           bl.len, bl.total, ws, Xp);
        return hipGetLastError();
    }
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
        const int tb = bl.cls == BATCH_SKINNY ? 32 : 32 * bl.cls;   // skinny partials: 32 x 32 super tiles
        dim3 grid((unsigned)((tb * tb + 255) / 256), (unsigned)bl.total);
        if (tb == 32) hipLaunchKernelGGL(batch_reduce_kernel<32>, grid, dim3(256), 0, s, t.descs, bl.list, bl.pref, bl.len, ws);
        else if (tb == 64) hipLaunchKernelGGL(batch_reduce_kernel<64>, grid, dim3(256), 0, s, t.descs, bl.list, bl.pref, bl.len, ws);
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
                           order, mode, gram_unit(gram_prec), flag);
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
