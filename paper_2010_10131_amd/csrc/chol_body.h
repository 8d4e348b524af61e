// Small FP64 Cholesky factorization + in-place triangular inverse for one
// workgroup (used by the Cholesky-QR of the ALS branch and of the subspace
// iteration eigensolver, and by the batched eigensolver).
#pragma once
#include "common.h"

namespace sth {

// One workgroup of NTH threads (a multiple of 64, at least 256), n <= 128,
// everything in LDS (dynamic LDS of chol_lds_bytes(n)).
//
// G (n x n, symmetric, ldg) + shift_rel * trace(G) / n * I = L L^T.  The
// matrix is padded with an identity block to np = 16 * ceil(n / 16), so that
// every block is a full 16 x 16 tile (the padded factor is diag(L, I)).
// Blocked right-looking Cholesky with 16-column panels:
//   * the diagonal block is factored by one wave in registers (row l of the
//     block in lane l, right-looking within the block, columns broadcast with
//     lane reads, 1 / sqrt from the reciprocal square root), and the same
//     wave inverts it (lane c solves for column c of D^{-1} = L(K, K)^{-1});
//     D^{-1} is kept, transposed, in the unused upper half of the block;
//   * the panel below it is P = A(B, K) D^{-T}, one 16 x 16 x 16 product per
//     row tile on the FP64 matrix cores;
//   * the trailing matrix gets the rank-16 update A(bi, bj) -= P(bi) P(bj)^T
//     on the matrix cores (16 x 16 tiles of the lower triangle).
// L is then inverted in place block column by block column from the last
// one:  L^{-1}(B, K) = -(sum_{J in (K, B]} L^{-1}(B, J) L(J, K)) D_K^{-1},
// both products on the matrix cores, D_K^{-1} the kept inverse.
// Writes R = L^T (upper, may be NULL) and Rinv = L^{-T} (upper), n x n.  A
// non-positive pivot sets flag[0] = 2 and is replaced by a tiny positive one
// so that the run continues.
//
// L lives in LDS with an odd leading dimension (np + 1), so that walking a
// row and walking a column are both free of bank conflicts.
constexpr int CB = 16;

__host__ __device__ inline int chol_np(int64_t n) { return (int)((n + CB - 1) / CB * CB); }
__host__ __device__ inline int chol_ld(int64_t n) { return chol_np(n) + 1; }

// Dynamic LDS of chol_body: L (np x ld), the product buffer (np x CB) and the
// reciprocals of the diagonal of L (np).
__host__ __device__ inline size_t chol_lds_bytes(int64_t n) {
    return (size_t)(chol_np(n) * chol_ld(n) + chol_np(n) * CB + chol_np(n)) * 8;
}

// value of v in lane `src` (src uniform across the wave)
__device__ __forceinline__ double lane_value(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

template <int NTH>
__device__ __forceinline__ void chol_body(const double *__restrict__ G, int n, int64_t ldg,
                                          double shift_rel, double *__restrict__ Rout,
                                          double *__restrict__ Rinv, int64_t *__restrict__ flag) {
    constexpr int NW = NTH / 64;
    constexpr int LC = 8;   // columns per wave and load step (16 loads in flight per thread)
    extern __shared__ __align__(16) double s_l[];  // L, column-major, leading dimension ld
    const int np = chol_np(n), ld = np + 1, nb = np / CB;
    double *s_tmp = s_l + np * ld;   // np x CB
    double *s_rd = s_tmp + np * CB;  // 1 / L(i, i)
    __shared__ double s_dinv[CB * CB];
    __shared__ double s_tr;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int tr = lane & 15, tg = lane >> 4;   // matrix-core tile coordinates

    // lower triangle of G padded with the identity
    for (int j0 = LC * wave; j0 < np; j0 += LC * NW) {
        double v[LC][2];
#pragma unroll
        for (int u = 0; u < LC; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = j0 + u, i = lane + 64 * h;
                double x = 0.0;
                if (j < n && i < n) x = (i >= j) ? G[i + ldg * j] : 0.0;
                else if (i == j) x = 1.0;
                v[u][h] = x;
            }
#pragma unroll
        for (int u = 0; u < LC; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = j0 + u, i = lane + 64 * h;
                if (j < np && i < np) s_l[i + ld * j] = v[u][h];
            }
    }
    __syncthreads();
    if (wave == 0) {
        double t = 0.0;
        for (int i = lane; i < n; i += 64) t += s_l[i + ld * i];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) s_tr = t;
    }
    __syncthreads();
    if (shift_rel != 0.0) {
        const double sh = shift_rel * s_tr / n;
        for (int i = tid; i < n; i += NTH) s_l[i + ld * i] += sh;
        __syncthreads();
    }
    const double tiny = 1e-300 + 1e-30 * fabs(s_tr);
    bool bad = false;
    for (int kb = 0; kb < nb; ++kb) {
        const int k0 = kb * CB, t0 = k0 + CB;
        // 1. diagonal block: wave 0, row l of the block in lane l
        if (wave == 0) {
            double row[CB];
            double myrd = 0.0;
#pragma unroll
            for (int c = 0; c < CB; ++c) row[c] = (lane < CB) ? s_l[k0 + lane + ld * (k0 + c)] : 0.0;
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                double d = lane_value(row[j], j);
                if (!(d > 0.0)) {
                    bad = true;
                    d = tiny;
                }
                const double rd = rsqrt(d);
                if (lane == j) {
                    row[j] = d * rd;
                    myrd = rd;
                } else if (lane > j) {
                    row[j] *= rd;
                }
                // rank-1 update of the block's remaining columns
#pragma unroll
                for (int c = j + 1; c < CB; ++c) row[c] -= row[j] * lane_value(row[j], c);
            }
            // column `lane` of D^{-1}: x_r = (delta_{r,lane} - sum_{d<r} L(r, d) x_d) / L(r, r)
            double x[CB];
#pragma unroll
            for (int r = 0; r < CB; ++r) {
                double sacc = (r == lane) ? 1.0 : 0.0;
#pragma unroll
                for (int d = 0; d < r; ++d) sacc -= lane_value(row[d], r) * x[d];
                x[r] = sacc * lane_value(myrd, r);
            }
            // row `lane` of the block: L(lane, c) for c <= lane, D^{-1}(c, lane) above
            if (lane < CB) {
#pragma unroll
                for (int c = 0; c < CB; ++c) s_l[k0 + lane + ld * (k0 + c)] = (c <= lane) ? row[c] : x[c];
                s_rd[k0 + lane] = myrd;
            }
        }
        __syncthreads();
        if (t0 >= np) break;
        // 2. panel P(bi) = A(bi, K) D^{-T}, one row tile per wave at a time;
        //    D^{-T}(k, c) = D^{-1}(c, k): the upper half for c > k, 1 / L(k, k) for c = k
        for (int bi = kb + 1 + wave; bi < nb; bi += NW) {
            const int ri = CB * bi;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + tg;
                const double a = s_l[ri + tr + ld * (k0 + k)];
                const double dup = s_l[k0 + k + ld * (k0 + tr)];
                const double b = tr > k ? dup : (tr == k ? s_rd[k0 + k] : 0.0);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) s_l[ri + tg + 4 * v + ld * (k0 + tr)] = acc[v];
        }
        __syncthreads();
        // 3. trailing update A(bi, bj) -= P(bi) P(bj)^T on the matrix cores,
        //    lower-triangle tiles bi >= bj > kb, one tile per wave at a time
        const int nt = nb - kb - 1;
        for (int q = wave; q < nt * (nt + 1) / 2; q += NW) {
            int bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
            const int bj = q - bi * (bi + 1) / 2;
            const int ri = t0 + CB * bi, cj = t0 + CB * bj;
            f64x4 acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = s_l[ri + tg + 4 * v + ld * (cj + tr)];
            // A operand: P(ri.., k) = s_l[ri + i + ld * (k0 + k)];  B operand:
            // P^T(k, cj..) = s_l[cj + j + ld * (k0 + k)], i.e. b(k, j) with ldb swapped
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const double a = -s_l[ri + tr + ld * (k0 + 4 * kk + tg)];
                const double b = s_l[cj + tr + ld * (k0 + 4 * kk + tg)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) s_l[ri + tg + 4 * v + ld * (cj + tr)] = acc[v];
        }
        __syncthreads();
    }
    if (bad && flag) flag[0] = 2;
    if (Rout)
        for (int j = wave; j < n; j += NW)       // R(i, j) = L(j, i)
            for (int i = lane; i < n; i += 64) Rout[i + (int64_t)n * j] = (i <= j) ? s_l[j + ld * i] : 0.0;
    __syncthreads();
    // in-place inverse, block columns from the last one
    for (int kb = nb - 1; kb >= 0; --kb) {
        const int k0 = kb * CB, t0 = k0 + CB;
        // D^{-1} of the diagonal block (lower) from its kept transpose
        for (int e = tid; e < CB * CB; e += NTH) {
            const int r = e % CB, c = e / CB;
            s_dinv[e] = r > c ? s_l[k0 + c + ld * (k0 + r)] : (r == c ? s_rd[k0 + r] : 0.0);
        }
        // T(bi) = sum_{bj = kb+1..bi} Linv(bi, bj) L(bj, kb): one row tile per wave
        for (int bi = kb + 1 + wave; bi < nb; bi += NW) {
            const int ri = CB * bi;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int bj = kb + 1; bj <= bi; ++bj) {
                const int cj = CB * bj;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double a = s_l[ri + tr + ld * (cj + 4 * kk + tg)];   // Linv(ri + r, cj + k)
                    const double b = s_l[cj + 4 * kk + tg + ld * (k0 + tr)];   // L(cj + k, k0 + c)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) s_tmp[(ri - t0) + tg + 4 * v + np * tr] = acc[v];
        }
        __syncthreads();
        // Linv(bi, kb) = -T(bi) Dinv;  Linv(kb, kb) = Dinv
        for (int bi = kb + 1 + wave; bi < nb; bi += NW) {
            const int ri = CB * bi;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const double a = -s_tmp[(ri - t0) + tr + np * (4 * kk + tg)];
                const double b = s_dinv[(4 * kk + tg) + CB * tr];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) s_l[ri + tg + 4 * v + ld * (k0 + tr)] = acc[v];
        }
        for (int e = tid; e < CB * CB; e += NTH) {
            const int r = e % CB, c = e / CB;
            s_l[k0 + r + ld * (k0 + c)] = s_dinv[e];
        }
        __syncthreads();
    }
    for (int j = wave; j < n; j += NW)           // Rinv(i, j) = Linv(j, i)
        for (int i = lane; i < n; i += 64) Rinv[i + (int64_t)n * j] = (i <= j) ? s_l[j + ld * i] : 0.0;
}

}  // namespace sth
