// Matricization-free mode-n Gram and TTT on the gfx950 matrix cores.
//
//   S(i, j) = sum_{a, b} A(a, i, b) * B(a, j, b)
//
// with A viewed as (L, IA, M) and B as (L, IB, M) along mode n.  B = A gives
// the Gram matrix Y_(n) Y_(n)^T of the EIG branch (Alg. 2); a different B
// gives the TTT of Eq. 3 (read as a contraction over every mode but n) used
// by the ALS branch.  The contraction runs over the P = L*M rows (a, b) in
// place, as the paper's "series of GEMMs accumulated into one result"
// (Sec. V), without forming X_(n).
//
// Design (MI355X):
//   * output blocks of TB x TB (TB = 32 * WT), 4 waves per workgroup in a
//     2 x 2 arrangement, each wave WT x WT tiles of 16 x 16;
//   * split-K over P: each workgroup owns one output block and one range of
//     rows; blocks of the same row range are mapped to the same XCD so the
//     re-reads of a row range across blocks hit that XCD's L2, not HBM;
//   * per 32-row chunk the workgroup loads its A (and B) slab with coalesced
//     reads (lanes along i when L = 1, along a otherwise), converts every
//     element once to the requested precision and stores it in LDS already
//     in matrix-core fragment layout; the next chunk's loads are in flight
//     while the current chunk is multiplied;
//   * FP32 (or bf16-split) products accumulate in FP32 for FLUSH chunks and
//     are then added into FP64 registers; workgroups write FP64 partial
//     blocks and a second kernel reduces them in a fixed order
//     (deterministic), mirroring the lower triangle for the Gram.
#include "common.h"
#include "gram_body.h"
#include "internal.h"

namespace sth {

template <typename T, int PREC, int WT, bool SYM>
__global__ __launch_bounds__(256) void gram_kernel(const T *__restrict__ A, const T *__restrict__ B,
                                                   int64_t L, int64_t IA, int64_t IB, int64_t P,
                                                   int64_t kper, int nkc, int nbi, int nbj,
                                                   int nblocks, int64_t total_wg,
                                                   double *__restrict__ partials) {
    gram_body<T, PREC, WT, SYM>(A, B, L, IA, IB, P, kper, nkc, nbi, nbj, nblocks, total_wg,
                                xcd_logical_id(total_wg), partials);
}

// TB = 32 * WT.  With WT = 4 the block runs eight waves of 64 x 32 each
// (2 x 4 grid): a wave's FP32 accumulators and their FP64 partial sums then
// stay in its own registers (four waves of 64 x 64 need more than a wave's
// 256 registers and shuttle them through the accumulation registers every
// chunk); measured on the 512-wide Gram: FP32 products 1.36x, bf16x3 1.5x
// faster than four waves.
template <int PREC, int WT>
constexpr bool gram_l1_eight_waves() { return WT == 4; }

template <int PREC, int WT, bool VEC4, bool FULLI>
__global__ __launch_bounds__((gram_l1_eight_waves<PREC, WT>() ? 512 : 256)) void gram_l1_kernel(
    const float *__restrict__ Y, int64_t I, int64_t P, int64_t kper, int nkc, int nblocks,
    int64_t total_wg, double *__restrict__ partials) {
    if constexpr (gram_l1_eight_waves<PREC, WT>())
        gram_l1_body<PREC, 4, 2, 2, 4, VEC4, FULLI>(Y, I, P, kper, nkc, nblocks, total_wg,
                                                    xcd_logical_id(total_wg), partials);
    else
        gram_l1_body<PREC, WT, WT, 2, 2, VEC4, FULLI>(Y, I, P, kper, nkc, nblocks, total_wg,
                                                      xcd_logical_id(total_wg), partials);
}

template <int PREC, int CH, bool V4>
__global__ __launch_bounds__(SK_T) void gram_skinny_kernel(const float *__restrict__ Y, int I, int64_t P,
                                                          int nkc, double *__restrict__ partials) {
    gram_skinny_body<PREC, CH, V4>(Y, I, P, nkc, blockIdx.x, partials);
}

// Sums the partial blocks over the row ranges and writes the IA x IB result
// (mirroring the lower triangle when SYM).  64 elements per workgroup, each
// summed by four waves over interleaved ranges of partials (8 loads in
// flight per thread), the four sums combined in a fixed order.
template <int TB, bool SYM>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double *__restrict__ partials, int nkc, int nbi,
                                                          int nblocks, int64_t IA, int64_t IB,
                                                          double *__restrict__ S) {
    const int q = blockIdx.y;
    int bi, bj;
    if (SYM) {
        bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
        bj = q - bi * (bi + 1) / 2;
    } else {
        bi = q % nbi;
        bj = q / nbi;
    }
    __shared__ double s_part[4][64];
    const int el = threadIdx.x & 63, ks = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + el;
    const bool ev = e < TB * TB;
    const int ec = ev ? e : 0;
    const int64_t stride = (int64_t)nblocks * TB * TB;
    const double *src = partials + (int64_t)q * TB * TB + ec;
    double acc = 0.0;
    int k = ks;
    for (; k + 28 < nkc; k += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(k + 4 * u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; k < nkc; k += 4) acc += src[(int64_t)k * stride];
    s_part[ks][el] = acc;
    __syncthreads();
    if (ks != 0 || !ev) return;
    const double sum = (s_part[0][el] + s_part[1][el]) + (s_part[2][el] + s_part[3][el]);
    const int il = e % TB, jl = e / TB;
    const int64_t i = (int64_t)bi * TB + il, j = (int64_t)bj * TB + jl;
    if (i >= IA || j >= IB) return;
    if (SYM && bi == bj && il < jl) return;  // upper part of a diagonal block: mirrored below
    S[i + IA * j] = sum;
    if (SYM && i != j) S[j + IA * i] = sum;
}

// ---------------------------------------------------------------- host ----

namespace {

struct GramShape {
    int wt, tb, nbi, nbj, nblocks, nkc;
    int64_t kper;
};

GramShape gram_shape_t(int64_t IA, int64_t IB, int64_t P, bool sym, int64_t target, int wt_max);

GramShape gram_shape(int64_t IA, int64_t IB, int64_t P, bool sym) {
    return gram_shape_t(IA, IB, P, sym, 2 * (int64_t)device_cu_count(), 4);
}

GramShape gram_shape_t(int64_t IA, int64_t IB, int64_t P, bool sym, int64_t target, int wt_max) {
    GramShape g;
    int64_t imax = std::max(IA, IB);
    g.wt = std::min(wt_max, imax > 64 ? 4 : (imax > 32 ? 2 : 1));
    g.tb = 32 * g.wt;
    g.nbi = (int)((IA + g.tb - 1) / g.tb);
    g.nbj = (int)((IB + g.tb - 1) / g.tb);
    g.nblocks = sym ? g.nbi * (g.nbi + 1) / 2 : g.nbi * g.nbj;
    // aim at `target` workgroups (about 2 per CU for one tensor), rows per
    // workgroup >= 512, and partial traffic well below the input traffic
    int64_t nkc = std::max<int64_t>(1, target / g.nblocks);
    int64_t maxk = std::max<int64_t>(1, P / 512);
    nkc = std::min(nkc, maxk);
    int64_t kper = (P + nkc - 1) / nkc;
    kper = (kper + KC - 1) / KC * KC;
    if (kper < KC) kper = KC;
    g.kper = kper;
    g.nkc = (int)std::max<int64_t>(1, (P + kper - 1) / kper);
    return g;
}

// Skinny path geometry: CH chunks of 32 columns per stage, as many as keep
// the loader at <= SK_TASKS tasks per thread and two stages within the LDS
// budget; one workgroup per CU (the LDS of a stage), each at least 4 stages.
struct SkShape {
    int ch, nkc;
};

SkShape sk_shape(int prec, int64_t I, int64_t P, bool v4) {
    SkShape k;
    const int NQ = prec == P_FP64 ? 4 : (prec == P_BF16X6 ? 3 : 2);
    const int64_t TBp = 32 * (int64_t)sk_ns(I);
    const int64_t tasks_max = (int64_t)(v4 ? 1 : SK_TASKS) * SK_T, rows_per_task = v4 ? 4 : 1;
    k.ch = prec == P_BF16X6 ? 4 : 8;   // bf16x6 at 8 chunks would spill registers
    while (k.ch > 1 && (TBp / rows_per_task * 4 * k.ch > tasks_max || 2 * k.ch * NQ * 4 * TBp * 16 > 150 * 1024)) k.ch >>= 1;
    const int64_t cols = 32 * (int64_t)k.ch;
    k.nkc = (int)std::min<int64_t>(device_cu_count(), std::max<int64_t>(1, P / (4 * cols)));
    return k;
}

size_t sk_lds(int prec, int64_t I, int ch) {
    const int NQ = prec == P_FP64 ? 4 : (prec == P_BF16X6 ? 3 : 2);
    return (size_t)2 * ch * NQ * 4 * 32 * sk_ns(I) * 16;
}

template <int PREC, int CH>
hipError_t launch_skinny_ch(const float *A, int64_t I, int64_t P, const SkShape &k, double *partials, hipStream_t s) {
    const bool v4 = I % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
    auto kern = v4 ? gram_skinny_kernel<PREC, CH, true> : gram_skinny_kernel<PREC, CH, false>;
    const size_t lds = sk_lds(PREC, I, CH);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)k.nkc), dim3(SK_T), lds, s, A, (int)I, P, k.nkc, partials);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_skinny(const float *A, int64_t I, int64_t P, double *partials, double *S, hipStream_t s) {
    const bool v4 = I % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
    const SkShape k = sk_shape(PREC, I, P, v4);
    hipError_t e;
    switch (k.ch) {
        case 8:
            if constexpr (PREC != P_BF16X6) {
                e = launch_skinny_ch<PREC, 8>(A, I, P, k, partials, s);
                break;
            }
            [[fallthrough]];
        case 4: e = launch_skinny_ch<PREC, 4>(A, I, P, k, partials, s); break;
        case 2: e = launch_skinny_ch<PREC, 2>(A, I, P, k, partials, s); break;
        default: e = launch_skinny_ch<PREC, 1>(A, I, P, k, partials, s); break;
    }
    if (e != hipSuccess) return e;
    const int NS = sk_ns(I);
    hipLaunchKernelGGL((gram_reduce_kernel<32, true>), dim3((32 * 32 + 63) / 64, NS * (NS + 1) / 2), dim3(256), 0,
                       s, partials, k.nkc, NS, NS * (NS + 1) / 2, I, I, S);
    return hipGetLastError();
}

template <int PREC, int WT>
hipError_t launch_gram_l1(const float *A, int64_t IA, int64_t M, const GramShape &g,
                          double *partials, hipStream_t s) {
    constexpr int TB = 32 * WT;
    const int64_t total = (int64_t)g.nkc * g.nblocks;
    const int64_t per_xcd = (total + 7) / 8;
    const size_t lds = (size_t)2 * 2 * Frag<PREC>::NQ * 4 * TB * 16;
    const bool vec = (IA % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    // I a multiple of the block edge: the branch-free loads
    // (blocks of 64 and 128: whole fragment octets per thread)
    auto kern = !vec ? gram_l1_kernel<PREC, WT, false, false>
                     : (IA % TB == 0 ? gram_l1_kernel<PREC, WT, true, (WT >= 2)>
                                     : gram_l1_kernel<PREC, WT, true, false>);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)(per_xcd * 8)), dim3(gram_l1_eight_waves<PREC, WT>() ? 512 : 256), lds, s, A, IA, M, g.kper,
                       g.nkc, g.nblocks, total, partials);
    return hipGetLastError();
}

template <typename T, int PREC, int WT, bool SYM>
hipError_t launch_gram_t(const T *A, const T *B, int64_t L, int64_t IA, int64_t IB, int64_t M,
                         const GramShape &g, double *partials, double *S, hipStream_t s) {
    constexpr int TB = 32 * WT;
    const int64_t P = L * M;
    const int64_t total = (int64_t)g.nkc * g.nblocks;
    const int64_t per_xcd = (total + 7) / 8;
    if constexpr (SYM && sizeof(T) == 4) {
        if (L == 1 && IA <= SK_MAXI) return launch_skinny<PREC>(A, IA, M, partials, S, s);
        if (L == 1 && WT >= 2) {
            hipError_t e = launch_gram_l1<PREC, WT>(A, IA, M, g, partials, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((gram_reduce_kernel<TB, SYM>), dim3((TB * TB + 63) / 64, g.nblocks),
                               dim3(256), 0, s, partials, g.nkc, g.nbi, g.nblocks, IA, IB, S);
            return hipGetLastError();
        }
    }
    const size_t lds = (size_t)2 * Frag<PREC>::NQ * TB * 4 * 16;
    auto kern = gram_kernel<T, PREC, WT, SYM>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)(per_xcd * 8)), dim3(256), lds, s, A, B, L, IA, IB, P,
                       g.kper, g.nkc, g.nbi, g.nbj, g.nblocks, total, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gram_reduce_kernel<TB, SYM>), dim3((TB * TB + 63) / 64, g.nblocks),
                       dim3(256), 0, s, partials, g.nkc, g.nbi, g.nblocks, IA, IB, S);
    return hipGetLastError();
}

template <typename T, int PREC, bool SYM>
hipError_t launch_gram_w(const T *A, const T *B, int64_t L, int64_t IA, int64_t IB, int64_t M,
                         const GramShape &g, double *partials, double *S, hipStream_t s) {
    switch (g.wt) {
        case 1: return launch_gram_t<T, PREC, 1, SYM>(A, B, L, IA, IB, M, g, partials, S, s);
        case 2: return launch_gram_t<T, PREC, 2, SYM>(A, B, L, IA, IB, M, g, partials, S, s);
        default: return launch_gram_t<T, PREC, 4, SYM>(A, B, L, IA, IB, M, g, partials, S, s);
    }
}

template <bool SYM>
hipError_t launch_gram_d(int dtype, int prec, const void *A, const void *B, int64_t L, int64_t IA,
                         int64_t IB, int64_t M, const GramShape &g, double *partials, double *S,
                         hipStream_t s) {
    if (dtype == DT_F64)
        return launch_gram_w<double, P_FP64, SYM>((const double *)A, (const double *)B, L, IA, IB, M, g, partials, S, s);
    const float *a = (const float *)A, *b = (const float *)B;
    switch (prec) {
        case P_FP64: return launch_gram_w<float, P_FP64, SYM>(a, b, L, IA, IB, M, g, partials, S, s);
        case P_FP32: return launch_gram_w<float, P_FP32, SYM>(a, b, L, IA, IB, M, g, partials, S, s);
        case P_BF16X3: return launch_gram_w<float, P_BF16X3, SYM>(a, b, L, IA, IB, M, g, partials, S, s);
        default: return launch_gram_w<float, P_BF16X6, SYM>(a, b, L, IA, IB, M, g, partials, S, s);
    }
}

}  // namespace

void gram_geometry(int64_t IA, int64_t IB, int64_t P, bool sym, int64_t target, int wt_max, int *wt,
                   int *nbi, int *nbj, int *nblocks, int *nkc, int64_t *kper) {
    GramShape g = gram_shape_t(IA, IB, P, sym, target, wt_max);
    *wt = g.wt;
    *nbi = g.nbi;
    *nbj = g.nbj;
    *nblocks = g.nblocks;
    *nkc = g.nkc;
    *kper = g.kper;
}

size_t gram_ws_bytes(int64_t IA, int64_t IB, int64_t P, bool sym) {
    GramShape g = gram_shape(IA, IB, P, sym);
    size_t b = (size_t)g.nkc * g.nblocks * g.tb * g.tb * sizeof(double);
    if (sym && IA <= SK_MAXI) {
        // the skinny path (L = 1; any precision)
        const int NS = sk_ns(IA);
        for (int prec = P_FP64; prec <= P_BF16X6; ++prec)
            for (int v4 = 0; v4 < 2; ++v4)
                b = std::max(b, (size_t)sk_shape(prec, IA, P, v4 != 0).nkc * (NS * (NS + 1) / 2) * 1024 * sizeof(double));
    }
    return b;
}

hipError_t gram_launch(int dtype, int prec, const void *A, const void *B, int64_t L, int64_t IA,
                       int64_t IB, int64_t M, bool sym, double *partials, double *S,
                       hipStream_t s) {
    const int64_t P = L * M;
    if (P == 0) {
        return fill_f64(S, IA * IB, 0.0, s);  // a kernel, so that the call stays graph-capturable
    }
    GramShape g = gram_shape(IA, IB, P, sym);
    if (sym) return launch_gram_d<true>(dtype, prec, A, A, L, IA, IA, M, g, partials, S, s);
    return launch_gram_d<false>(dtype, prec, A, B, L, IA, IB, M, g, partials, S, s);
}

}  // namespace sth
