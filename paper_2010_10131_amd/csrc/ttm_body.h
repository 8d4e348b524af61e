// Device body of the TTM kernel (one workgroup), shared by the single-tensor
// kernel and the batched one.
#pragma once
#include "common.h"

namespace sth {

template <typename T, bool CONTIG>
__device__ __forceinline__ void ttm_load_chunk(const T *__restrict__ Y, int64_t base, int64_t L,
                                               int64_t K, int64_t kb, T (&x)[8]) {
    // kb = first of this lane's 8 consecutive k
    if (CONTIG && kb + 8 <= K) {
        const T *src = Y + base + kb;
        if constexpr (sizeof(T) == 4) {
            // 4-byte alignment suffices (rows of any length K)
            const f32x4u u = *reinterpret_cast<const f32x4u *>(src);
            const f32x4u w = *reinterpret_cast<const f32x4u *>(src + 4);
            x[0] = u.x; x[1] = u.y; x[2] = u.z; x[3] = u.w;
            x[4] = w.x; x[5] = w.y; x[6] = w.z; x[7] = w.w;
        } else {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                double2 u = *reinterpret_cast<const double2 *>(src + 2 * h);
                x[2 * h] = u.x;
                x[2 * h + 1] = u.y;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int64_t k = kb + j;
            x[j] = (k < K) ? Y[base + L * k] : (T)0;
        }
    }
}

// Body of the TTM for one workgroup: wg of nwg workgroups sharing the row
// blocks of this tensor, r-block rb.  Also used by the batched kernels.
// PF = chunks of Y in flight per wave (1 or 2).
// ZT (with CONTIG): the output is stored transposed, Z(r, p) at p + P r, which
// puts the next mode first in the batched path's rotated layout.
// ERR: nothing is stored; each output value z (rounded to T, as a store
// would) is compared with Xe at the address it would have been stored to, and
// the workgroup's sums of (Xe - z)^2 and Xe^2 (FP64) go to epart[2 wg_id],
// epart[2 wg_id + 1] (wg_id = blockIdx.y * gridDim.x + blockIdx.x).
template <typename T, int PREC, int NT, int RTB, bool CONTIG, bool ULDS, int WAVES, int PF = 1, bool ZT = false,
          bool ERR = false>
__device__ __forceinline__ void ttm_body(const T *__restrict__ Y, const uint4 *__restrict__ Uq,
                                         T *__restrict__ Z, int64_t L, int64_t K, int64_t Rout,
                                         int64_t P, int nchunks, int ntiles, int64_t nrowblocks,
                                         int64_t wg, int64_t nwg, int rb, const T *__restrict__ Xe = nullptr,
                                         double *__restrict__ epart = nullptr) {
    if (CONTIG) L = 1;  // the contiguous variant is the L = 1 view; a constant for the compiler
    constexpr int NQ = Frag<PREC>::NQ;
    typedef typename Acc<PREC>::type AccT;
    extern __shared__ uint4 s_u[];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int rt0 = rb * RTB;
    const int rtn = min(RTB, ntiles - rt0);

    if (ULDS) {
        // stage this r-block's factor quads: [c][rt in block][q][lane]
        const int per_chunk = RTB * NQ * 64;
        const int total = nchunks * per_chunk;
        for (int e = threadIdx.x; e < total; e += 64 * WAVES) {
            int c = e / per_chunk;
            int rem = e - c * per_chunk;  // (rtl * NQ + q) * 64 + lane
            int rtl = rem / (NQ * 64);
            uint4 v = make_uint4(0, 0, 0, 0);
            if (rtl < rtn) v = Uq[((int64_t)c * ntiles + rt0) * NQ * 64 + rem];
            s_u[e] = v;
        }
        __syncthreads();
    }

    double esq_d = 0.0, esq_x = 0.0;   // ERR: this lane's sums
    const int64_t wstride = nwg * WAVES;
    for (int64_t wb = wg * WAVES + wave; wb < nrowblocks; wb += wstride) {
        const int64_t p0 = wb * (16 * NT);
        int64_t base[NT];
        int64_t zoff[NT];
        bool pvalid[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            int64_t p = p0 + 16 * nt + (lane & 15);
            pvalid[nt] = p < P;
            int64_t pc = pvalid[nt] ? p : (P - 1);
            int64_t a, b;
            if (CONTIG) {
                a = 0;
                b = pc;
            } else {
                b = pc / L;
                a = pc - b * L;
            }
            base[nt] = a + L * K * b;
            zoff[nt] = a + L * Rout * b;
        }
        AccT acc[NT][RTB];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int rt = 0; rt < RTB; ++rt) acc[nt][rt] = AccT{0, 0, 0, 0};

        auto chunk_mma = [&](int c, const Frag<PREC>(&yb)[NT]) {
#pragma unroll
            for (int rt = 0; rt < RTB; ++rt) {
                FragQ<PREC> ua;
                if (ULDS) {
                    const uint4 *src = s_u + ((c * RTB + rt) * NQ) * 64 + lane;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) ua.q[q] = src[q * 64];
                } else {
                    const int rtg = min(rt0 + rt, ntiles - 1);
                    const uint4 *src = Uq + (((int64_t)c * ntiles + rtg) * NQ) * 64 + lane;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) ua.q[q] = src[q * 64];
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) mma_frag(ua.f, yb[nt], acc[nt][rt]);
            }
        };

        if constexpr (PF == 1) {
            // one chunk buffer: chunk c + 1 loads while chunk c is multiplied
            T nxt[NT][8];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) ttm_load_chunk<T, CONTIG>(Y, base[nt], L, K, 8 * g, nxt[nt]);
            for (int c = 0; c < nchunks; ++c) {
                Frag<PREC> yb[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) make_frag(nxt[nt], yb[nt]);
                if (c + 1 < nchunks) {
                    const int64_t kb = (int64_t)(c + 1) * KC + 8 * g;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) ttm_load_chunk<T, CONTIG>(Y, base[nt], L, K, kb, nxt[nt]);
                }
                chunk_mma(c, yb);
            }
        } else {
        // two chunk buffers: chunk c is consumed from one while chunks c + 1
        // (already in flight) and c + 2 (issued right after c is split) load
        T xa[NT][8], xb[NT][8];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) ttm_load_chunk<T, CONTIG>(Y, base[nt], L, K, 8 * g, xa[nt]);
        if (nchunks > 1) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) ttm_load_chunk<T, CONTIG>(Y, base[nt], L, K, KC + 8 * g, xb[nt]);
        }
        for (int c = 0; c < nchunks; c += 2) {
            {
                Frag<PREC> yb[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) make_frag(xa[nt], yb[nt]);
                if (c + 2 < nchunks) {
                    const int64_t kb = (int64_t)(c + 2) * KC + 8 * g;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) ttm_load_chunk<T, CONTIG>(Y, base[nt], L, K, kb, xa[nt]);
                }
                chunk_mma(c, yb);
            }
            if (c + 1 < nchunks) {
                Frag<PREC> yb[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) make_frag(xb[nt], yb[nt]);
                if (c + 3 < nchunks) {
                    const int64_t kb = (int64_t)(c + 3) * KC + 8 * g;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) ttm_load_chunk<T, CONTIG>(Y, base[nt], L, K, kb, xb[nt]);
                }
                chunk_mma(c + 1, yb);
            }
        }
        }

        // D[r][p]: lane holds r = 16*rt + drow(g, v), p = 16*nt + lane%16
        static_assert(!ZT || CONTIG, "the transposed output is the L = 1 view's");
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (!pvalid[nt]) continue;
            if constexpr (ERR) {
#pragma unroll
                for (int rt = 0; rt < RTB; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t r = (int64_t)(rt0 + rt) * 16 + drow<PREC>(g, v);
                        if (r < Rout) {
                            const double x = (double)Xe[zoff[nt] + L * r];
                            const double d = x - (double)(T)acc[nt][rt][v];
                            esq_d += d * d;
                            esq_x += x * x;
                        }
                    }
                continue;
            }
            if constexpr (ZT) {
                const int64_t p = p0 + 16 * nt + (lane & 15);
#pragma unroll
                for (int rt = 0; rt < RTB; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t r = (int64_t)(rt0 + rt) * 16 + drow<PREC>(g, v);
                        if (r < Rout) Z[p + P * r] = (T)acc[nt][rt][v];
                    }
                continue;
            }
#pragma unroll
            for (int rt = 0; rt < RTB; ++rt) {
                const int64_t rbase = (int64_t)(rt0 + rt) * 16;
                const int64_t r0 = rbase + 4 * g;
                if (PREC != P_FP64 && CONTIG && sizeof(T) == 4 && (Rout & 3) == 0 && r0 + 4 <= Rout) {
                    float4 v = make_float4((float)acc[nt][rt][0], (float)acc[nt][rt][1],
                                           (float)acc[nt][rt][2], (float)acc[nt][rt][3]);
                    *reinterpret_cast<float4 *>(Z + zoff[nt] + r0) = v;
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int64_t r = rbase + drow<PREC>(g, v);
                        if (r < Rout) Z[zoff[nt] + L * r] = (T)acc[nt][rt][v];
                    }
                }
            }
        }
    }
    if constexpr (ERR) {
        // fixed-order workgroup sums: lanes by xor shuffles, then waves in order
        __shared__ double s_err[2][WAVES];
        for (int o = 32; o > 0; o >>= 1) {
            esq_d += __shfl_xor(esq_d, o);
            esq_x += __shfl_xor(esq_x, o);
        }
        if (lane == 0) {
            s_err[0][wave] = esq_d;
            s_err[1][wave] = esq_x;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < WAVES; ++w) {
                a += s_err[0][w];
                b += s_err[1][w];
            }
            const int64_t id = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
            epart[2 * id] = a;
            epart[2 * id + 1] = b;
        }
    }
}


}  // namespace sth

namespace sth {

// ---------------------------------------------------------------------------
// K-split TTM for the contiguous view (L = 1: row p of Y is K consecutive
// values).  The eight waves of a workgroup share every block of 16 * NT rows:
// wave w takes the CPW chunks [w * CPW, (w + 1) * CPW) of the K range, holds
// the matching factor fragments in registers for the whole run, and
// multiplies its slice of the block's rows; the eight partial 16*NT x 64
// results meet in LDS (double-buffered, one barrier per block) and are summed
// into Z in a fixed order.  So a workgroup streams whole blocks of
// consecutive rows (16 * NT * K * 4 bytes) and keeps the next block's loads
// in flight while the current one is reduced.
constexpr int KS_WAVES = 8;
constexpr int KS_RS = 68;  // LDS row stride of the partials (64 columns + 4: no bank conflicts)

__host__ __device__ inline size_t ttm_ks_lds(int nt) { return (size_t)2 * KS_WAVES * 16 * nt * KS_RS * 4; }

// PERM: lane group g holds k = 4g .. 4g+3 and 16 + 4g .. 16 + 4g + 3 of each
// 32-wide chunk (the factor quads are prepared with the same order), so the
// four groups of a row read its 64 bytes in one contiguous run per load.
// FULL: K = KS_WAVES * CPW * 32 exactly, so every wave's chunks are whole and
// the loads need no branch; the prefetches are then issued unconditionally
// (the block index clamped to the last block), which lets the compiler wait
// for exactly the block being multiplied instead of for every load in
// flight.
template <int PREC, int NT, int CPW, bool PERM = false, bool FULL = false>
__device__ __forceinline__ void ttm_ks_body(const float *__restrict__ Y, const uint4 *__restrict__ Uq,
                                            float *__restrict__ Z, int64_t K, int64_t Rout, int64_t P,
                                            int nchunks, int ntiles, int64_t nblocks, int64_t wg,
                                            int64_t nwg, int rb) {
    constexpr int NQ = Frag<PREC>::NQ;
    constexpr int RTB = 4;
    constexpr int ROWS = 16 * NT;
    extern __shared__ __align__(16) float s_part[];  // [2][KS_WAVES][ROWS][KS_RS], read as float4
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int rt0 = rb * RTB;
    const int c0 = wave * CPW;

    // this wave's factor fragments: chunks c0 .. c0 + CPW - 1, r-tiles of block rb
    FragQ<PREC> uf[CPW][RTB];
#pragma unroll
    for (int j = 0; j < CPW; ++j)
#pragma unroll
        for (int rt = 0; rt < RTB; ++rt) {
            const int c = c0 + j, rtg = rt0 + rt;
            const bool ok = c < nchunks && rtg < ntiles;
            const uint4 *src = Uq + (((int64_t)(ok ? c : 0) * ntiles + (ok ? rtg : 0)) * NQ) * 64 + lane;
#pragma unroll
            for (int q = 0; q < NQ; ++q) uf[j][rt].q[q] = ok ? src[q * 64] : make_uint4(0, 0, 0, 0);
        }

    auto load_block = [&](int64_t blk, float (&x)[CPW][NT][8]) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t p = blk * ROWS + 16 * nt + (lane & 15);
            const int64_t pc = p < P ? p : P - 1;
            if constexpr (FULL) {
#pragma unroll
                for (int j = 0; j < CPW; ++j) {
                    const float *src = Y + K * pc + (int64_t)(c0 + j) * KC + 8 * g;
                    const float4 u = *reinterpret_cast<const float4 *>(src);
                    const float4 w = *reinterpret_cast<const float4 *>(src + 4);
                    x[j][nt][0] = u.x; x[j][nt][1] = u.y; x[j][nt][2] = u.z; x[j][nt][3] = u.w;
                    x[j][nt][4] = w.x; x[j][nt][5] = w.y; x[j][nt][6] = w.z; x[j][nt][7] = w.w;
                }
                continue;
            }
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int64_t kb = (int64_t)(c0 + j) * KC + 8 * g;
                if (c0 + j < nchunks) {
                    if (PERM) {
                        const int64_t kc = (int64_t)(c0 + j) * KC;
                        const float *src = Y + K * pc + kc + 4 * g;
                        if (kc + KC <= K) {
                            const float4 u = *reinterpret_cast<const float4 *>(src);
                            const float4 w = *reinterpret_cast<const float4 *>(src + 16);
                            x[j][nt][0] = u.x; x[j][nt][1] = u.y; x[j][nt][2] = u.z; x[j][nt][3] = u.w;
                            x[j][nt][4] = w.x; x[j][nt][5] = w.y; x[j][nt][6] = w.z; x[j][nt][7] = w.w;
                        } else {
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                const int64_t k = kc + 4 * g + (e < 4 ? e : 12 + e);
                                x[j][nt][e] = k < K ? Y[K * pc + k] : 0.f;
                            }
                        }
                    } else {
                        ttm_load_chunk<float, true>(Y, K * pc, 1, K, kb, x[j][nt]);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) x[j][nt][e] = 0.f;
                }
            }
        }
    };
    auto compute_store = [&](const float (&x)[CPW][NT][8], int buf) {
        f32x4 acc[NT][RTB];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int rt = 0; rt < RTB; ++rt) acc[nt][rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            Frag<PREC> yb[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) make_frag(x[j][nt], yb[nt]);
#pragma unroll
            for (int rt = 0; rt < RTB; ++rt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) mma_frag(uf[j][rt].f, yb[nt], acc[nt][rt]);
        }
        // partial D[r][p]: lane holds r = 16 rt + 4 g + v, p = 16 nt + lane % 16
        float *dst = s_part + ((size_t)(buf * KS_WAVES + wave) * ROWS) * KS_RS;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int rt = 0; rt < RTB; ++rt)
                *reinterpret_cast<float4 *>(dst + (16 * nt + (lane & 15)) * KS_RS + 16 * rt + 4 * g) =
                    make_float4(acc[nt][rt][0], acc[nt][rt][1], acc[nt][rt][2], acc[nt][rt][3]);
    };
    auto reduce_store = [&](int64_t blk, int buf) {
        // ROWS x 64 outputs, four consecutive r per thread, waves summed in order
        for (int o = threadIdx.x; o < ROWS * 16; o += 64 * KS_WAVES) {
            const int pl = o >> 4, r4 = (o & 15) * 4;
            const float *src = s_part + ((size_t)(buf * KS_WAVES) * ROWS + pl) * KS_RS + r4;
            float4 s = *reinterpret_cast<const float4 *>(src);
#pragma unroll
            for (int w = 1; w < KS_WAVES; ++w) {
                const float4 t = *reinterpret_cast<const float4 *>(src + (size_t)w * ROWS * KS_RS);
                s.x += t.x;
                s.y += t.y;
                s.z += t.z;
                s.w += t.w;
            }
            const int64_t p = blk * ROWS + pl;
            const int64_t r = (int64_t)rt0 * 16 + r4;
            if (p < P && r < Rout) {
                float *z = Z + r + Rout * p;
                if ((Rout & 3) == 0) {
                    *reinterpret_cast<float4 *>(z) = s;
                } else {
                    z[0] = s.x;
                    if (r + 1 < Rout) z[1] = s.y;
                    if (r + 2 < Rout) z[2] = s.z;
                    if (r + 3 < Rout) z[3] = s.w;
                }
            }
        }
    };

    // three register buffers: while block b is multiplied, blocks b + nwg and
    // b + 2 nwg are in flight
    float xa[CPW][NT][8], xb[CPW][NT][8], xc[CPW][NT][8];
    int64_t blk = wg;
    const int64_t last = nblocks - 1;
    if (FULL) {
        load_block(blk < last ? blk : last, xa);
        load_block(blk + nwg < last ? blk + nwg : last, xb);
    } else {
        if (blk < nblocks) load_block(blk, xa);
        if (blk + nwg < nblocks) load_block(blk + nwg, xb);
    }
    int buf = 0;
    auto step = [&](float (&cur)[CPW][NT][8], float (&nx2)[CPW][NT][8]) {
        if (FULL) {
            load_block(blk + 2 * nwg < last ? blk + 2 * nwg : last, nx2);
            // keep these loads ahead of the block's products: issued here they
            // are in flight for the whole multiply
            __builtin_amdgcn_sched_barrier(0);
        } else if (blk + 2 * nwg < nblocks) {
            load_block(blk + 2 * nwg, nx2);
        }
        compute_store(cur, buf);
        __syncthreads();
        reduce_store(blk, buf);
        buf ^= 1;
        blk += nwg;
    };
    while (blk < nblocks) {
        step(xa, xc);
        if (blk >= nblocks) break;
        step(xb, xa);
        if (blk >= nblocks) break;
        step(xc, xb);
    }
}

}  // namespace sth
