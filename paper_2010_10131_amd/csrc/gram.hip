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
#include "internal.h"

namespace sth {

constexpr int GRAM_FLUSH = 4;  // chunks of 32 rows accumulated in FP32 before an FP64 flush

// Loads the 8 consecutive rows p0..p0+7 of column i of a (L, I, M) tensor.
template <typename T>
__device__ __forceinline__ void gram_load_octet(const T *__restrict__ X, int64_t L, int64_t I,
                                                int64_t i, int64_t p0, int64_t pend, T (&x)[8]) {
    if (i >= I) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = (T)0;
        return;
    }
    if (L == 1) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int64_t p = p0 + j;
            x[j] = (p < pend) ? X[i + I * p] : (T)0;
        }
        return;
    }
    int64_t b = p0 / L;
    int64_t a = p0 - b * L;
    if (a + 8 <= L && p0 + 8 <= pend) {
        const T *src = X + a + L * i + L * I * b;
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = src[j];
        return;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int64_t p = p0 + j;
        x[j] = (p < pend) ? X[a + L * i + L * I * b] : (T)0;
        if (++a == L) {
            a = 0;
            ++b;
        }
    }
}

// Unit u of a TB x 32 slab (TB columns i, 4 octets of rows).  Lanes run along
// i when L = 1 (contiguous in memory), along the octets otherwise.
__device__ __forceinline__ void gram_unit(int u, int TB, bool lfast, int &il, int &oct) {
    if (lfast) {
        il = u % TB;
        oct = u / TB;
    } else {
        oct = u & 3;
        il = u >> 2;
    }
}

template <typename T, int PREC, int WT, bool SYM>
__global__ __launch_bounds__(256) void gram_kernel(const T *__restrict__ A, const T *__restrict__ B,
                                                   int64_t L, int64_t IA, int64_t IB, int64_t P,
                                                   int64_t kper, int nkc, int nbi, int nbj,
                                                   int nblocks, int64_t total_wg,
                                                   double *__restrict__ partials) {
    constexpr int TB = 32 * WT;                 // block edge
    constexpr int NQ = Frag<PREC>::NQ;
    constexpr int UNITS = TB * 4;               // octets per slab
    constexpr int UPT = (UNITS + 255) / 256;    // octets per thread per slab
    typedef typename Acc<PREC>::type AccT;
    constexpr bool F64ACC = (PREC == P_FP64);

    // LDS: slab A then slab B, each [q][il][oct] quads
    extern __shared__ uint4 s_g[];
    uint4 *sA = s_g;
    uint4 *sB = s_g + NQ * TB * 4;

    // XCD-aware mapping: consecutive logical ids (same row range, all blocks)
    // land on the same XCD.
    const int64_t per_xcd = (total_wg + 7) / 8;
    const int64_t lid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (lid >= total_wg) return;
    const int kc = (int)(lid / nblocks);
    const int q = (int)(lid - (int64_t)kc * nblocks);
    int bi, bj;
    if (SYM) {
        // lower-triangle enumeration: q -> (bi >= bj)
        bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
        bj = q - bi * (bi + 1) / 2;
    } else {
        bi = q % nbi;
        bj = q / nbi;
    }
    const bool diag = SYM && (bi == bj);
    const int64_t i0 = (int64_t)bi * TB, j0 = (int64_t)bj * TB;
    const int64_t pbeg = (int64_t)kc * kper;
    const int64_t pend = min(P, pbeg + kper);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const bool active = !(diag && wi < wj);
    const bool lfast = (L == 1);

    AccT acc[WT][WT];
    f64x4 acc64[WT][WT];
#pragma unroll
    for (int x = 0; x < WT; ++x)
#pragma unroll
        for (int y = 0; y < WT; ++y) {
            acc[x][y] = AccT{0, 0, 0, 0};
            acc64[x][y] = f64x4{0, 0, 0, 0};
        }

    T ra[UPT][8], rb[UPT][8];
    auto load_slab = [&](int64_t pc) {
#pragma unroll
        for (int s = 0; s < UPT; ++s) {
            int u = threadIdx.x + 256 * s;
            int il, oct;
            gram_unit(u, TB, lfast, il, oct);
            if (u < UNITS) {
                gram_load_octet<T>(A, L, IA, i0 + il, pc + 8 * oct, pend, ra[s]);
                if (!diag) gram_load_octet<T>(B, L, IB, j0 + il, pc + 8 * oct, pend, rb[s]);
            }
        }
    };
    auto store_slab = [&]() {
#pragma unroll
        for (int s = 0; s < UPT; ++s) {
            int u = threadIdx.x + 256 * s;
            int il, oct;
            gram_unit(u, TB, lfast, il, oct);
            if (u < UNITS) {
                FragQ<PREC> f;
                make_frag(ra[s], f.f);
#pragma unroll
                for (int qq = 0; qq < NQ; ++qq) sA[(qq * TB + il) * 4 + oct] = f.q[qq];
                if (!diag) {
                    make_frag(rb[s], f.f);
#pragma unroll
                    for (int qq = 0; qq < NQ; ++qq) sB[(qq * TB + il) * 4 + oct] = f.q[qq];
                }
            }
        }
    };

    const int nch = (int)((pend - pbeg + KC - 1) / KC);
    if (nch > 0) load_slab(pbeg);
    const uint4 *sBr = diag ? sA : sB;
    for (int c = 0; c < nch; ++c) {
        __syncthreads();  // previous chunk's reads are done
        store_slab();
        __syncthreads();
        if (c + 1 < nch) load_slab(pbeg + (int64_t)(c + 1) * KC);
        if (active) {
            Frag<PREC> fa[WT], fb[WT];
#pragma unroll
            for (int x = 0; x < WT; ++x) {
                FragQ<PREC> t;
                const int il = wi * (16 * WT) + 16 * x + (lane & 15);
#pragma unroll
                for (int qq = 0; qq < NQ; ++qq) t.q[qq] = sA[(qq * TB + il) * 4 + (lane >> 4)];
                fa[x] = t.f;
            }
#pragma unroll
            for (int y = 0; y < WT; ++y) {
                FragQ<PREC> t;
                const int jl = wj * (16 * WT) + 16 * y + (lane & 15);
#pragma unroll
                for (int qq = 0; qq < NQ; ++qq) t.q[qq] = sBr[(qq * TB + jl) * 4 + (lane >> 4)];
                fb[y] = t.f;
            }
#pragma unroll
            for (int x = 0; x < WT; ++x)
#pragma unroll
                for (int y = 0; y < WT; ++y) mma_frag(fa[x], fb[y], acc[x][y]);
            if (!F64ACC && ((c + 1) % GRAM_FLUSH == 0 || c + 1 == nch)) {
#pragma unroll
                for (int x = 0; x < WT; ++x)
#pragma unroll
                    for (int y = 0; y < WT; ++y) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc64[x][y][v] += (double)acc[x][y][v];
                        acc[x][y] = AccT{0, 0, 0, 0};
                    }
            }
        }
    }
    if (!active) return;
    // partial block (TB x TB, column-major) for (kc, q)
    double *dst = partials + ((int64_t)kc * nblocks + q) * (int64_t)TB * TB;
#pragma unroll
    for (int x = 0; x < WT; ++x)
#pragma unroll
        for (int y = 0; y < WT; ++y) {
            const int jl = wj * (16 * WT) + 16 * y + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int il = wi * (16 * WT) + 16 * x + drow<PREC>(lane >> 4, v);
                double val = F64ACC ? (double)acc[x][y][v] : acc64[x][y][v];
                dst[il + TB * jl] = val;
            }
        }
}

// Sums the partial blocks over the row ranges in a fixed order and writes
// the IA x IB result (mirroring the lower triangle when SYM).
template <int TB, bool SYM>
__global__ void gram_reduce_kernel(const double *__restrict__ partials, int nkc, int nbi,
                                   int nblocks, int64_t IA, int64_t IB, double *__restrict__ S) {
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
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= TB * TB) return;
    const int il = e % TB, jl = e / TB;
    const int64_t i = (int64_t)bi * TB + il, j = (int64_t)bj * TB + jl;
    if (i >= IA || j >= IB) return;
    if (SYM && bi == bj && il < jl) return;  // upper part of a diagonal block: mirrored below
    double s = 0.0;
    for (int k = 0; k < nkc; ++k) s += partials[((int64_t)k * nblocks + q) * TB * TB + e];
    S[i + IA * j] = s;
    if (SYM && i != j) S[j + IA * i] = s;
}

// ---------------------------------------------------------------- host ----

namespace {

struct GramShape {
    int wt, tb, nbi, nbj, nblocks, nkc;
    int64_t kper;
};

GramShape gram_shape(int64_t IA, int64_t IB, int64_t P, bool sym) {
    GramShape g;
    int64_t imax = std::max(IA, IB);
    g.wt = imax > 64 ? 4 : (imax > 32 ? 2 : 1);
    g.tb = 32 * g.wt;
    g.nbi = (int)((IA + g.tb - 1) / g.tb);
    g.nbj = (int)((IB + g.tb - 1) / g.tb);
    g.nblocks = sym ? g.nbi * (g.nbi + 1) / 2 : g.nbi * g.nbj;
    // aim at ~2 workgroups per CU overall, rows per workgroup >= 512, and
    // partial traffic well below the input traffic
    const int64_t target = 2 * (int64_t)device_cu_count();
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

template <typename T, int PREC, int WT, bool SYM>
hipError_t launch_gram_t(const T *A, const T *B, int64_t L, int64_t IA, int64_t IB, int64_t M,
                         const GramShape &g, double *partials, double *S, hipStream_t s) {
    constexpr int TB = 32 * WT;
    const int64_t P = L * M;
    const int64_t total = (int64_t)g.nkc * g.nblocks;
    const int64_t per_xcd = (total + 7) / 8;
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
    hipLaunchKernelGGL((gram_reduce_kernel<TB, SYM>), dim3((TB * TB + 255) / 256, g.nblocks),
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

size_t gram_ws_bytes(int64_t IA, int64_t IB, int64_t P, bool sym) {
    GramShape g = gram_shape(IA, IB, P, sym);
    return (size_t)g.nkc * g.nblocks * g.tb * g.tb * sizeof(double);
}

hipError_t gram_launch(int dtype, int prec, const void *A, const void *B, int64_t L, int64_t IA,
                       int64_t IB, int64_t M, bool sym, double *partials, double *S,
                       hipStream_t s) {
    const int64_t P = L * M;
    if (P == 0) {
        return hipMemsetAsync(S, 0, sizeof(double) * IA * IB, s);
    }
    GramShape g = gram_shape(IA, IB, P, sym);
    if (sym) return launch_gram_d<true>(dtype, prec, A, A, L, IA, IA, M, g, partials, S, s);
    return launch_gram_d<false>(dtype, prec, A, B, L, IA, IB, M, g, partials, S, s);
}

}  // namespace sth
