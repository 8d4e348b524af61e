// Device bodies of the Gram / TTT kernels (one workgroup each), shared by the
// single-tensor kernels and the batched ones.
#pragma once
#include "common.h"

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

// XCD-aware mapping of a launch of total_wg workgroups: consecutive logical
// ids (same row range, all blocks) land on the same XCD.
__device__ __forceinline__ int64_t xcd_logical_id(int64_t total_wg) {
    const int64_t per_xcd = (total_wg + 7) / 8;
    return (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
}

// One workgroup of the Gram/TTT: logical id lid = row range * nblocks + block.
template <typename T, int PREC, int WT, bool SYM>
__device__ __forceinline__ void gram_body(const T *__restrict__ A, const T *__restrict__ B,
                                          int64_t L, int64_t IA, int64_t IB, int64_t P,
                                          int64_t kper, int nkc, int nbi, int nbj, int nblocks,
                                          int64_t total_wg, int64_t lid,
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

// ---------------------------------------------------------------------------
// First-mode (L = 1) variant for FP32 data.  Each row p of the contraction
// is a contiguous run of I floats, so a slab of TB columns x 32 rows is read
// with 16-byte loads along i (lanes 0..TB/4-1 cover one row).  A thread
// holds 4 columns x LPT rows; the rows it holds are mapped to LPT
// consecutive fragment slots of one lane group:
//   row pc + ph + PH*s  ->  group g = ph % 4, slot j = LPT*(ph / 4) + s,
// the same bijection for A and B, which is all the matrix cores need.
// LDS holds two slabs per operand (double buffering, one barrier per chunk)
// and the loads run two chunks ahead of the matrix cores.
template <int PREC>
__device__ __forceinline__ void l1_store(uint8_t *slab, int TB, int g, int row, int slot0,
                                         const float *v, int nv) {
    // slab: base of one operand buffer, quads [qq][g][row]
    if constexpr (PREC == P_BF16X3 || PREC == P_BF16X6) {
        constexpr int NP = (PREC == P_BF16X3) ? 2 : 3;
        __bf16 part[NP][4];
        for (int k = 0; k < nv; ++k) {
            float x = v[k];
            __bf16 h = to_bf16(x);
            float r1 = x - from_bf16(h);
            __bf16 m = to_bf16(r1);
            part[0][k] = h;
            part[1][k] = m;
            if constexpr (NP == 3) part[2][k] = to_bf16(r1 - from_bf16(m));
        }
#pragma unroll
        for (int qq = 0; qq < NP; ++qq) {
            uint8_t *q = slab + ((size_t)((qq * 4 + g) * TB + row)) * 16 + 2 * slot0;
            if (nv == 4) {
                uint2 w;
                __builtin_memcpy(&w, part[qq], 8);
                *reinterpret_cast<uint2 *>(q) = w;
            } else {
                uint32_t w;
                __builtin_memcpy(&w, part[qq], 4);
                *reinterpret_cast<uint32_t *>(q) = w;
            }
        }
    } else if constexpr (PREC == P_FP32) {
        // slot j -> quad j / 4, element j % 4
        const int qq = slot0 / 4, e = slot0 % 4;
        float *q = reinterpret_cast<float *>(slab + ((size_t)((qq * 4 + g) * TB + row)) * 16) + e;
        for (int k = 0; k < nv; ++k) q[k] = v[k];
    } else {
        // FP64: slot j -> quad j / 2, element j % 2
        for (int k = 0; k < nv; ++k) {
            const int j = slot0 + k;
            double *q = reinterpret_cast<double *>(slab + ((size_t)(((j / 2) * 4 + g) * TB + row)) * 16) + (j % 2);
            *q = (double)v[k];
        }
    }
}

// Waves form a WI x WJ grid over the TB x TB output block, each owning
// WTI x WTJ tiles of 16 x 16 (TB = 16 WTI WI = 16 WTJ WJ).
// FULLI: I is a multiple of TB and rows are 16-byte aligned, so every load is
// one float4 with no branch (rows past the range are clamped and zeroed by a
// select) and the prefetches are issued unconditionally (chunk index clamped;
// a diagonal block loads its one operand twice, from cache).  Branch-free
// loads let the compiler wait for exactly the chunk being stored instead of
// draining every load in flight before the next ones are issued.
// V4LD (batched mode-1 launches, any I >= 4, rows 4-byte aligned): thread
// (parity, operand, row quad iq, group g) owns rows 4 iq .. 4 iq + 3 of one
// operand and the 8 columns g of every chunk of its parity (threads [0, 2 TB)
// the even chunks, the rest the odd ones): eight 16-byte loads per chunk give
// four rows' fragments (quads past I zeroed, a quad across row I read value
// by value); the same
// 32 values per thread as two chunks of two operands in flight.  Its LDS
// stores are 64 bytes apart across lanes; where the matrix cores bound the
// Gram (bf16x6 at I = 512) the FULLI loads are faster, so the single-tensor
// path keeps those.
template <int PREC, int WTI, int WTJ, int WI, int WJ, bool VEC4, bool FULLI = false, bool V4LD = false>
__device__ __forceinline__ void gram_l1_body(const float *__restrict__ Y, int64_t I, int64_t P,
                                             int64_t kper, int nkc, int nblocks, int64_t total_wg,
                                             int64_t lid, double *__restrict__ partials) {
    constexpr int TB = 16 * WTI * WI;
    static_assert(TB == 16 * WTJ * WJ, "square output block");
    constexpr int NTH = 64 * WI * WJ;
    constexpr int NQ = Frag<PREC>::NQ;
    constexpr int IQ = TB / 4;          // 16-byte column quads per row
    constexpr int PH = NTH / IQ;        // rows covered by one pass of the workgroup
    constexpr int LPT = KC / PH;        // rows (loads) per thread per chunk
    constexpr int SLAB = NQ * 4 * TB * 16;  // bytes of one operand buffer
    typedef typename Acc<PREC>::type AccT;
    constexpr bool F64ACC = (PREC == P_FP64);
    extern __shared__ uint4 s_g[];
    uint8_t *lds = reinterpret_cast<uint8_t *>(s_g);  // [buf][operand][SLAB]

    if (lid >= total_wg) return;
    const int kc = (int)(lid / nblocks);
    const int q = (int)(lid - (int64_t)kc * nblocks);
    int bi = 0;
    while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
    const int bj = q - bi * (bi + 1) / 2;
    const bool diag = (bi == bj);
    const int64_t i0 = (int64_t)bi * TB, j0 = (int64_t)bj * TB;
    const int64_t pbeg = (int64_t)kc * kper;
    const int64_t pend = min(P, pbeg + kper);
    const int nch = (int)((pend - pbeg + KC - 1) / KC);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave / WJ, wj = wave % WJ;
    // a wave whose tiles lie wholly above the diagonal of a diagonal block idles
    const bool active = !(diag && (wi + 1) * 16 * WTI <= wj * 16 * WTJ);
    const int iq = tid % IQ, ph = tid / IQ;
    const int g_st = ph % 4, slot0 = LPT * (ph / 4);

    // FULLI: thread (il, kq) owns column il of the block and the KPT
    // consecutive rows kq * KPT .. of each chunk (lanes along the column, so
    // every load instruction reads 256 contiguous bytes); it splits them into
    // whole fragment quads and writes 16 bytes per quad, consecutive lanes to
    // consecutive rows of the slab (no LDS bank conflicts).
    constexpr int KG = NTH / TB;      // row groups per chunk
    constexpr int KPT = KC / KG;      // rows per thread per chunk (4 * LPT floats)
    static_assert(!FULLI || (KPT == 4 * LPT && KPT % 8 == 0), "thread tiling of the full path");
    const int il = tid % TB, kq = tid / TB;
    auto load = [&](int64_t pc, int64_t c0, float4 (&r)[LPT]) {
        if constexpr (FULLI) {
            float *rf = &r[0].x;
            const float *src = Y + c0 + il;
#pragma unroll
            for (int s = 0; s < KPT; ++s) {
                const int64_t p = pc + kq * KPT + s;
                const int64_t pcl = p < pend ? p : pend - 1;
                const float v = src[I * pcl];
                rf[s] = p < pend ? v : 0.f;
            }
            return;
        }
        const int64_t col = c0 + 4 * iq;
#pragma unroll
        for (int s = 0; s < LPT; ++s) {
            const int64_t p = pc + ph + PH * s;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (p < pend) {
                const float *src = Y + I * p + col;
                if (VEC4 && col + 4 <= I) {
                    v = *reinterpret_cast<const float4 *>(src);
                } else {
                    if (col + 0 < I) v.x = src[0];
                    if (col + 1 < I) v.y = src[1];
                    if (col + 2 < I) v.z = src[2];
                    if (col + 3 < I) v.w = src[3];
                }
            }
            r[s] = v;
        }
    };
    auto store = [&](int buf, int op, const float4 (&r)[LPT]) {
        uint8_t *slab = lds + (size_t)(buf * 2 + op) * SLAB;
        if constexpr (FULLI) {
            const float *rf = &r[0].x;
            uint4 *sq = reinterpret_cast<uint4 *>(slab);
#pragma unroll
            for (int o = 0; o < KPT / 8; ++o) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = rf[8 * o + e];
                FragQ<PREC> t;
                make_frag(v, t.f);
                const int g = kq * (KPT / 8) + o;
#pragma unroll
                for (int qq = 0; qq < NQ; ++qq) sq[(qq * 4 + g) * TB + il] = t.q[qq];
            }
            return;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float v[LPT];
#pragma unroll
            for (int s = 0; s < LPT; ++s) v[s] = (&r[s].x)[c];
            l1_store<PREC>(slab, TB, g_st, 4 * iq + c, slot0, v, LPT);
        }
    };

    AccT acc[WTI][WTJ];
    f64x4 acc64[WTI][WTJ];
#pragma unroll
    for (int x = 0; x < WTI; ++x)
#pragma unroll
        for (int y = 0; y < WTJ; ++y) {
            acc[x][y] = AccT{0, 0, 0, 0};
            acc64[x][y] = f64x4{0, 0, 0, 0};
        }

    auto compute = [&](int buf, int c) {
        if (!active) return;
        const uint4 *sA = reinterpret_cast<const uint4 *>(lds + (size_t)(buf * 2 + 0) * SLAB);
        const uint4 *sB = reinterpret_cast<const uint4 *>(lds + (size_t)(buf * 2 + (diag ? 0 : 1)) * SLAB);
        const int g = lane >> 4;
        Frag<PREC> fa[WTI], fb[WTJ];
#pragma unroll
        for (int x = 0; x < WTI; ++x) {
            FragQ<PREC> t;
            const int row = wi * (16 * WTI) + 16 * x + (lane & 15);
#pragma unroll
            for (int qq = 0; qq < NQ; ++qq) t.q[qq] = sA[(qq * 4 + g) * TB + row];
            fa[x] = t.f;
        }
#pragma unroll
        for (int y = 0; y < WTJ; ++y) {
            FragQ<PREC> t;
            const int row = wj * (16 * WTJ) + 16 * y + (lane & 15);
#pragma unroll
            for (int qq = 0; qq < NQ; ++qq) t.q[qq] = sB[(qq * 4 + g) * TB + row];
            fb[y] = t.f;
        }
#pragma unroll
        for (int x = 0; x < WTI; ++x)
#pragma unroll
            for (int y = 0; y < WTJ; ++y) mma_frag(fa[x], fb[y], acc[x][y]);
        if (!F64ACC && ((c + 1) % GRAM_FLUSH == 0 || c + 1 == nch)) {
#pragma unroll
            for (int x = 0; x < WTI; ++x)
#pragma unroll
                for (int y = 0; y < WTJ; ++y) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[x][y][v] += (double)acc[x][y][v];
                    acc[x][y] = AccT{0, 0, 0, 0};
                }
        }
    };

    if constexpr (V4LD) {
        static_assert(NTH == 4 * TB, "one task per thread");
        constexpr int TQ4 = TB / 4;
        const int par4 = tid / (2 * TB), op4 = (tid / TB) & 1, iq4 = (tid % TB) % TQ4, g4 = (tid % TB) / TQ4;
        // a quad wholly inside the column is one 16-byte load (4-byte
        // aligned when I % 4 != 0); the quad that runs past row I - 1 reads
        // its rows below I one value at a time, so no load leaves the column
        const int64_t rq = (op4 ? j0 : i0) + 4 * iq4;
        const bool rok4 = rq < I, full4 = rq + 4 <= I;
        const float *src4 = Y + (rok4 ? rq : 0);
        float rv[4][8];
        auto load4 = [&](int cn) {
            const int64_t pc = pbeg + (int64_t)(cn < nch ? cn : nch - 1) * KC;
            if (full4) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t pp = pc + 8 * g4 + j;
                    const int64_t pcl = pp < pend ? pp : pend - 1;
                    const f32x4u v = *reinterpret_cast<const f32x4u *>(src4 + I * pcl);
                    const bool in = pp < pend;
                    rv[0][j] = in ? v.x : 0.f;
                    rv[1][j] = in ? v.y : 0.f;
                    rv[2][j] = in ? v.z : 0.f;
                    rv[3][j] = in ? v.w : 0.f;
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t pp = pc + 8 * g4 + j;
                    const int64_t pcl = pp < pend ? pp : pend - 1;
                    const bool in = rok4 && pp < pend;
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const bool ok = in && rq + rr < I;
                        rv[rr][j] = ok ? src4[I * pcl + (ok ? rr : 0)] : 0.f;
                    }
                }
            }
        };
        auto store4 = [&](int buf) {
            uint4 *sq = reinterpret_cast<uint4 *>(lds + (size_t)(buf * 2 + op4) * SLAB);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                FragQ<PREC> t;
                make_frag(rv[rr], t.f);
#pragma unroll
                for (int qq = 0; qq < NQ; ++qq) sq[(qq * 4 + g4) * TB + 4 * iq4 + rr] = t.q[qq];
            }
        };
        if (nch > 0) {
            load4(par4);
            if (par4 == 0) store4(0);
        }
        __syncthreads();
        // chunk c in buffer 0 and chunk c + 1 in flight on the odd threads;
        // every load and LDS store is issued unconditionally (clamped chunks
        // past the end are stored and never multiplied)
        for (int c = 0; c < nch; c += 2) {
            if (par4 == 0) load4(c + 2);
            compute(0, c);
            if (par4 == 1) store4(1);
            __syncthreads();
            if (par4 == 1) load4(c + 3);
            if (c + 1 < nch) compute(1, c + 1);
            if (par4 == 0) store4(0);
            __syncthreads();
        }
    } else {
    float4 ra0[LPT], rb0[LPT], ra1[LPT], rb1[LPT];
    auto prefetch = [&](int cn, float4 (&ra)[LPT], float4 (&rb)[LPT]) {
        if (FULLI) {
            const int64_t pc = pbeg + (int64_t)(cn < nch ? cn : nch - 1) * KC;
            load(pc, i0, ra);
            load(pc, j0, rb);
        } else if (cn < nch) {
            load(pbeg + (int64_t)cn * KC, i0, ra);
            if (!diag) load(pbeg + (int64_t)cn * KC, j0, rb);
        }
    };
    if (FULLI && nch > 0) {
        prefetch(0, ra0, rb0);
        prefetch(1, ra1, rb1);
        store(0, 0, ra0);
        store(0, 1, rb0);
    } else if (nch > 0) {
        load(pbeg, i0, ra0);
        if (!diag) load(pbeg, j0, rb0);
        if (nch > 1) {
            load(pbeg + KC, i0, ra1);
            if (!diag) load(pbeg + KC, j0, rb1);
        }
        store(0, 0, ra0);
        if (!diag) store(0, 1, rb0);
    }
    __syncthreads();
    if constexpr (FULLI) {
        // the same two-stage pipeline with every load and LDS store issued
        // unconditionally (clamped chunks past the end are stored and never
        // multiplied); only the matrix-core work of a missing odd chunk is skipped
        for (int c = 0; c < nch; c += 2) {
            prefetch(c + 2, ra0, rb0);
            compute(0, c);
            store(1, 0, ra1);
            store(1, 1, rb1);
            __syncthreads();
            prefetch(c + 3, ra1, rb1);
            if (c + 1 < nch) compute(1, c + 1);
            store(0, 0, ra0);
            store(0, 1, rb0);
            __syncthreads();
        }
    } else
    for (int c = 0; c < nch; c += 2) {
        // chunk c in buffer 0; chunk c+1 in flight in ra1/rb1
        prefetch(c + 2, ra0, rb0);
        compute(0, c);
        if (c + 1 < nch) {
            store(1, 0, ra1);
            if (!diag) store(1, 1, rb1);
        }
        __syncthreads();
        if (c + 1 >= nch) break;
        // chunk c+1 in buffer 1; chunk c+2 in flight in ra0/rb0
        prefetch(c + 3, ra1, rb1);
        compute(1, c + 1);
        if (c + 2 < nch) {
            store(0, 0, ra0);
            if (!diag) store(0, 1, rb0);
        }
        __syncthreads();
    }
    }
    if (!active) return;
    double *dst = partials + ((int64_t)kc * nblocks + q) * (int64_t)TB * TB;
#pragma unroll
    for (int x = 0; x < WTI; ++x)
#pragma unroll
        for (int y = 0; y < WTJ; ++y) {
            const int jl = wj * (16 * WTJ) + 16 * y + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int il = wi * (16 * WTI) + 16 * x + drow<PREC>(lane >> 4, v);
                dst[il + TB * jl] = F64ACC ? (double)acc[x][y][v] : acc64[x][y][v];
            }
        }
}

// ---- skinny Gram: L = 1 and I <= 160 (a short first mode, J_1 = M huge) --
// Y (I x P, column-major) is read once, in blocks of 32 CH columns (each one
// contiguous run of 128 I CH bytes) dealt round-robin to the workgroups:
// workgroup k takes blocks k, k + nkc, ..., so that at any moment the chip
// streams one contiguous region (independent far-apart streams per
// workgroup camp on a few HBM channels).
// The whole lower triangle of its partial Gram is held in registers as 32 x 32
// super tiles (2 x 2 tiles of 16 x 16), at most SK_MS per wave.  Per stage CH
// chunks of 32 columns go through LDS as matrix-core fragments: thread task
// (row i, group g, chunk c) loads the 8 values Y(i, p0 + 32 c + 8 g + j),
// consecutive lanes on consecutive rows (256-byte loads), splits them into
// the precision's fragment and stores it; the next stage's loads are in flight
// while the current one is multiplied.  FP32 accumulators are flushed into
// FP64 every GRAM_FLUSH chunks; partial super tiles go to the workspace and
// gram_reduce_kernel<32, true> sums them in a fixed order.
constexpr int SK_MAXI = 160;
constexpr int SK_W = 8, SK_T = 64 * SK_W;
constexpr int SK_MS = 2;      // super tiles per wave: 15 lower 32 x 32 tiles at I = 160
constexpr int SK_TASKS = 4;   // loader tasks per thread and stage

__host__ __device__ inline int sk_ns(int64_t I) { return (int)(((I + 15) / 16 + 1) / 2); }

// ANYI (with V4): I need not be a multiple of 4 (the batched class); the
// quad across row I - 1 is then read value by value.
template <int PREC, int CH, bool V4, bool ANYI = false>
__device__ __forceinline__ void gram_skinny_body(const float *__restrict__ Y, int I, int64_t P, int nkc, int kc,
                                                 double *__restrict__ partials) {
    constexpr int NQ = Frag<PREC>::NQ;
    typedef typename Acc<PREC>::type AccT;
    constexpr bool F64ACC = (PREC == P_FP64);
    extern __shared__ uint4 s_sk[];
    const int NS = sk_ns(I), NSS = NS * (NS + 1) / 2, TBp = 32 * NS;
    const int64_t nblk = (P + 32 * CH - 1) / (32 * CH);
    const int nst = kc < nblk ? (int)((nblk - 1 - kc) / nkc + 1) : 0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4;
    const int stage_q = CH * NQ * 4 * TBp;   // uint4 per stage buffer

    int sbi[SK_MS], sbj[SK_MS];
#pragma unroll
    for (int m = 0; m < SK_MS; ++m) {
        const int q = wave + SK_W * m;
        int bi = -1, bj = 0;
        if (q < NSS) {
            bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
            bj = q - bi * (bi + 1) / 2;
        }
        sbi[m] = bi;
        sbj[m] = bj;
    }
    AccT acc[SK_MS][2][2];
    f64x4 acc64[SK_MS][2][2];
#pragma unroll
    for (int m = 0; m < SK_MS; ++m)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                acc[m][x][y] = AccT{0, 0, 0, 0};
                acc64[m][x][y] = f64x4{0, 0, 0, 0};
            }

    // V4 (I % 4 == 0, or any I with ANYI): task (row quad iq, group g, chunk c)
    // loads the 4 x 8 block Y(4 iq .. 4 iq + 3, p0 + 32 c + 8 g + j) with eight
    // 16-byte loads (consecutive lanes on consecutive row quads) and builds
    // the four rows' fragments.  Otherwise task (row i, group g, chunk c)
    // loads the 8 values of one row with 4-byte loads.
    constexpr int RPT = V4 ? 4 : 1;                 // rows per task
    constexpr int NTK = V4 ? 1 : SK_TASKS;          // tasks per thread
    const int TQ = TBp / RPT;                       // row groups
    const int ntask = TQ * 4 * CH;
    float raw[NTK][RPT][8];
    auto load = [&](int st) {
        const int64_t p0 = ((int64_t)st * nkc + kc) * 32 * CH;
#pragma unroll
        for (int u = 0; u < NTK; ++u) {
            const int t = tid + SK_T * u;
            const int iq = t % TQ, rest = t / TQ, gg = rest & 3, c = rest >> 2;
            const bool ok = t < ntask && RPT * iq < I;
            if (ANYI && RPT * iq + RPT > I) {
                // the quad across row I - 1: its rows below I one at a time
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t pp = p0 + 32 * c + 8 * gg + j;
                    const bool in = ok && pp < P;
                    const int64_t a = (int64_t)(ok ? RPT * iq : 0) + (int64_t)I * (in ? pp : p0);
#pragma unroll
                    for (int rr = 0; rr < RPT; ++rr) {
                        const bool rin = in && RPT * iq + rr < I;
                        raw[u][rr][j] = rin ? Y[a + (rin ? rr : 0)] : 0.f;
                    }
                }
                continue;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t pp = p0 + 32 * c + 8 * gg + j;
                const bool in = ok && pp < P;
                const int64_t pc = in ? pp : p0;
                const int64_t a = (int64_t)(ok ? RPT * iq : 0) + (int64_t)I * pc;
                if constexpr (V4) {
                    // 4-byte alignment suffices (ANYI: rows of any length)
                    const f32x4u v = *reinterpret_cast<const f32x4u *>(Y + a);
                    raw[u][0][j] = in ? v.x : 0.f;
                    raw[u][1][j] = in ? v.y : 0.f;
                    raw[u][2][j] = in ? v.z : 0.f;
                    raw[u][3][j] = in ? v.w : 0.f;
                } else {
                    const float v = Y[a];
                    raw[u][0][j] = in ? v : 0.f;
                }
            }
        }
    };
    auto store = [&](int buf) {
        uint4 *sb = s_sk + (size_t)buf * stage_q;
#pragma unroll
        for (int u = 0; u < NTK; ++u) {
            const int t = tid + SK_T * u;
            if (t < ntask) {
                const int iq = t % TQ, rest = t / TQ, gg = rest & 3, c = rest >> 2;
#pragma unroll
                for (int rr = 0; rr < RPT; ++rr) {
                    FragQ<PREC> f;
                    make_frag(raw[u][rr], f.f);
#pragma unroll
                    for (int qq = 0; qq < NQ; ++qq) sb[((c * NQ + qq) * 4 + gg) * TBp + RPT * iq + rr] = f.q[qq];
                }
            }
        }
    };
    auto frag = [&](const uint4 *sb, int c, int row, Frag<PREC> &f) {
        FragQ<PREC> t;
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) t.q[qq] = sb[((c * NQ + qq) * 4 + g) * TBp + row];
        f = t.f;
    };

    int chunk = 0;
    if (nst > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        if (st + 1 < nst) load(st + 1);
        const uint4 *sb = s_sk + (size_t)(st & 1) * stage_q;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
#pragma unroll
            for (int m = 0; m < SK_MS; ++m) {
                if (sbi[m] < 0) continue;   // uniform within the wave
                Frag<PREC> fa[2], fb[2];
#pragma unroll
                for (int x = 0; x < 2; ++x) frag(sb, c, 32 * sbi[m] + 16 * x + (lane & 15), fa[x]);
                if (sbi[m] != sbj[m]) {
#pragma unroll
                    for (int y = 0; y < 2; ++y) frag(sb, c, 32 * sbj[m] + 16 * y + (lane & 15), fb[y]);
                } else {
                    fb[0] = fa[0];
                    fb[1] = fa[1];
                }
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) mma_frag(fa[x], fb[y], acc[m][x][y]);
            }
            ++chunk;
            if (!F64ACC && chunk % GRAM_FLUSH == 0) {
#pragma unroll
                for (int m = 0; m < SK_MS; ++m)
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int y = 0; y < 2; ++y) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc64[m][x][y][v] += (double)acc[m][x][y][v];
                            acc[m][x][y] = AccT{0, 0, 0, 0};
                        }
            }
        }
        if (st + 1 < nst) store((st + 1) & 1);
        __syncthreads();
    }
    // partial super tiles: element (il, jl) of super tile q at [(kc NSS + q) 1024 + il + 32 jl]
#pragma unroll
    for (int m = 0; m < SK_MS; ++m) {
        if (sbi[m] < 0) continue;
        const int q = wave + SK_W * m;
        double *dst = partials + ((int64_t)kc * NSS + q) * 1024;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double val = F64ACC ? (double)acc[m][x][y][v] : acc64[m][x][y][v] + (double)acc[m][x][y][v];
                    dst[(16 * x + drow<PREC>(g, v)) + 32 * (16 * y + (lane & 15))] = val;
                }
    }
}

}  // namespace sth
