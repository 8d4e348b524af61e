// Small FP64 Cholesky factorization + in-place triangular inverse for one
// workgroup (used by the Cholesky-QR of the ALS branch and of the subspace
// iteration eigensolver, and by the batched eigensolver).
#pragma once
#include "common.h"

namespace sth {

// One workgroup of NTH threads, n <= 128, everything in LDS (dynamic LDS of
// chol_lds_bytes(n)).
// G (n x n, symmetric, ldg) + shift_rel * trace(G) / n * I = L L^T, blocked
// right-looking Cholesky with 16-column panels: the diagonal block is
// factored by one wave in registers (row i of the block in lane i, columns
// broadcast with cross-lane shuffles), the panel below by a row-parallel
// forward substitution and the trailing matrix by an element-parallel
// rank-16 update.  L is then inverted in place block column by block column
// from the last one:  L^{-1}(B, K) = -(sum_{J in (K, B]} L^{-1}(B, J) L(J, K))
// L(K, K)^{-1}.  Writes R = L^T (upper, may be NULL) and Rinv = L^{-T}
// (upper).  A non-positive pivot sets flag[0] = 2 and is replaced by a tiny
// positive one so that the run continues.
constexpr int CB = 16;

// Dynamic LDS of chol_body: L (n x n), the panel buffer (n x CB) and the
// reciprocals of the diagonal of L (n).
__host__ __device__ inline size_t chol_lds_bytes(int64_t n) { return (size_t)(n * n + n * CB + n) * 8; }

template <int CHOL_THREADS>
__device__ __forceinline__ void chol_body(const double *__restrict__ G, int n, int64_t ldg,
                                          double shift_rel, double *__restrict__ Rout,
                                          double *__restrict__ Rinv, int64_t *__restrict__ flag) {
    extern __shared__ double s_l[];  // L, column-major, leading dimension n; then T (n x CB)
    double *s_tmp = s_l + n * n;
    double *s_rd = s_tmp + n * CB;    // 1 / L(i, i)
    __shared__ double s_dinv[CB * CB];
    __shared__ double s_tr;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < n * n; e += CHOL_THREADS) {
        int i = e % n, j = e / n;
        s_l[e] = (i >= j) ? G[i + ldg * j] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
        // trace, reduced across one wave from the copy in LDS
        double t = 0.0;
        for (int i = lane; i < n; i += 64) t += s_l[i + n * i];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) s_tr = t;
    }
    __syncthreads();
    if (shift_rel != 0.0) {
        const double sh = shift_rel * s_tr / n;
        for (int i = tid; i < n; i += CHOL_THREADS) s_l[i + n * i] += sh;
        __syncthreads();
    }
    const double tiny = 1e-300 + 1e-30 * fabs(s_tr);
    bool bad = false;
    for (int k0 = 0; k0 < n; k0 += CB) {
        const int kn = min(CB, n - k0);
        // 1. diagonal block, wave 0, row i in lane i
        if (wave == 0) {
            double row[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) row[c] = (lane < kn && c < kn) ? s_l[k0 + lane + n * (k0 + c)] : 0.0;
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                if (j < kn) {
                    // d = a(j,j) - sum_{c<j} L(j,c)^2, computed in lane j, then broadcast
                    double sacc = row[j];
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c < j) sacc -= row[c] * __shfl(row[c], j);
                    double d = __shfl(sacc, j);
                    if (!(d > 0.0)) {
                        bad = true;
                        d = tiny;
                    }
                    d = sqrt(d);
                    const double rd = 1.0 / d;
                    if (lane == j) {
                        row[j] = d;
                        s_rd[k0 + j] = rd;
                    } else if (lane > j) {
                        row[j] = sacc * rd;
                    }
                }
            }
            if (lane < kn)
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c < kn) s_l[k0 + lane + n * (k0 + c)] = (c <= lane) ? row[c] : 0.0;
        }
        __syncthreads();
        // 2. panel rows i >= k0 + kn: forward substitution against the block
        for (int i = k0 + kn + tid; i < n; i += CHOL_THREADS) {
            double x[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                if (c < kn) {
                    double sacc = s_l[i + n * (k0 + c)];
#pragma unroll
                    for (int d = 0; d < CB; ++d)
                        if (d < c) sacc -= x[d] * s_l[k0 + c + n * (k0 + d)];
                    x[c] = sacc * s_rd[k0 + c];
                }
            }
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < kn) s_l[i + n * (k0 + c)] = x[c];
        }
        __syncthreads();
        // 3. trailing update of the lower part
        const int t0 = k0 + kn, w = n - t0;
        for (int e = tid; e < w * w; e += CHOL_THREADS) {
            const int i = t0 + e % w, j = t0 + e / w;
            if (i < j) continue;
            double sacc = 0.0;
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < kn) sacc += s_l[i + n * (k0 + c)] * s_l[j + n * (k0 + c)];
            s_l[i + n * j] -= sacc;
        }
        __syncthreads();
    }
    if (bad && flag) flag[0] = 2;
    if (Rout)
        for (int e = tid; e < n * n; e += CHOL_THREADS) {
            int i = e % n, j = e / n;  // R(i, j) = L(j, i)
            Rout[e] = (i <= j) ? s_l[j + n * i] : 0.0;
        }
    __syncthreads();
    // in-place inverse, block columns from the last one
    const int nb = (n + CB - 1) / CB;
    for (int kb = nb - 1; kb >= 0; --kb) {
        const int k0 = kb * CB, kn = min(CB, n - k0), t0 = k0 + kn;
        // D^{-1} of the diagonal block (lower), one thread per column
        if (tid < kn) {
            const int c = tid;
            double x[CB];
#pragma unroll
            for (int r = 0; r < CB; ++r) {
                if (r < kn) {
                    double sacc = (r == c) ? 1.0 : 0.0;
#pragma unroll
                    for (int d = 0; d < CB; ++d)
                        if (d < r) sacc -= s_l[k0 + r + n * (k0 + d)] * x[d];
                    x[r] = (r < c) ? 0.0 : sacc * s_rd[k0 + r];
                }
            }
#pragma unroll
            for (int r = 0; r < CB; ++r)
                if (r < kn) s_dinv[r + CB * c] = x[r];
        }
        // T(i, c) = sum_{j in [t0, i]} Linv(i, j) L(j, k0 + c) for rows i >= t0
        for (int e = tid; e < (n - t0) * kn; e += CHOL_THREADS) {
            const int i = t0 + e % (n - t0), c = e / (n - t0);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int j = t0;
            for (; j + 3 <= i; j += 4) {
                s0 += s_l[i + n * j] * s_l[j + n * (k0 + c)];
                s1 += s_l[i + n * (j + 1)] * s_l[j + 1 + n * (k0 + c)];
                s2 += s_l[i + n * (j + 2)] * s_l[j + 2 + n * (k0 + c)];
                s3 += s_l[i + n * (j + 3)] * s_l[j + 3 + n * (k0 + c)];
            }
            for (; j <= i; ++j) s0 += s_l[i + n * j] * s_l[j + n * (k0 + c)];
            s_tmp[(i - t0) + (n - t0) * c] = (s0 + s1) + (s2 + s3);
        }
        __syncthreads();
        // Linv(i, k0 + c) = -sum_d T(i, d) Dinv(d, c);  diagonal block = Dinv
        for (int e = tid; e < (n - t0) * kn; e += CHOL_THREADS) {
            const int i = t0 + e % (n - t0), c = e / (n - t0);
            double sacc = 0.0;
#pragma unroll
            for (int d = 0; d < CB; ++d)
                if (d >= c && d < kn) sacc += s_tmp[(i - t0) + (n - t0) * d] * s_dinv[d + CB * c];
            s_l[i + n * (k0 + c)] = -sacc;
        }
        for (int e = tid; e < kn * kn; e += CHOL_THREADS) {
            const int r = e % kn, c = e / kn;
            s_l[k0 + r + n * (k0 + c)] = (r >= c) ? s_dinv[r + CB * c] : 0.0;
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += CHOL_THREADS) {
        int i = e % n, j = e / n;  // Rinv(i, j) = Linv(j, i)
        Rinv[e] = (i <= j) ? s_l[j + n * i] : 0.0;
    }
}


}  // namespace sth
