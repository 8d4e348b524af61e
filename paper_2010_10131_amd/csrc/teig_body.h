// Device body of the direct FP64 symmetric eigensolver used for the R
// leading eigenpairs (Alg. 2, EIG branch: the leading eigenvectors of the
// mode-n Gram), run by one 512-thread workgroup:
//
//   1. Householder tridiagonalization A = Q T Q^T.  Step k builds the
//      reflector H_k = I - tau_k v_k v_k^T (v_k(k+1) = 1) from column k and
//      applies it to the trailing block as A <- A - v w^T - w v^T with
//      p = tau A v, w = p - (tau/2)(p^T v) v.  The rank-2 update of step k
//      is folded into the pass that forms p for step k + 1 (one read and one
//      write of the trailing block per step); column k + 1 gets its pending
//      update first so that v_{k+1} is known before that pass.
//   2. Eigenvalues of T by bisection on Sturm counts, the R largest only.
//      The count of eigenvalues below sigma is the number of sign changes in
//      the leading principal minors p_i of T - sigma I, taken with the
//      three-term recurrence p_i = (d_i - sigma) p_{i-1} - e_{i-1}^2 p_{i-2}
//      (no division; every 8 steps the pair is rescaled by a power of two,
//      which keeps every sign).  e^2 is floored at
//      (2^-60 ||T||)^2, so a vanishing minor is never followed by another
//      and counts as positive (the LDL^T count with a negative-zero pivot).
//      Each eigenvalue is searched by a group of
//      lanes, each lane counting at 4 points at once (independent chains),
//      which splits the bracket into (4 x group size + 1) parts per round.
//   3. Eigenvectors of T by inverse iteration: two solves of
//      (T - lambda I) x = b by Gaussian elimination with partial pivoting,
//      from a pseudo-random start vector of each eigenvector's own.
//   4. Orthogonalization: eigenvalues closer than 1e-9 ||T|| form clusters,
//      whose vectors (combinations inside the cluster's eigenspace) are made
//      orthonormal by classical Gram-Schmidt applied twice; then one
//      Newton-Schulz step Z <- Z (3 I - Z^T Z) / 2 on the whole block, on the
//      FP64 matrix cores, removes the O(eps ||T|| / gap) overlaps that
//      inverse iteration leaves between distinct eigenvalues.
//   5. Back-transformation Z <- H_0 H_1 ... H_{n-3} Z.
//   6. Optional sign rule (the entry of largest magnitude of each column is
//      made positive, first index on ties), eigenvalues in descending order.
//
// The matrix is scaled by a power of two so that its largest entry lies in
// [1, 2) (exact; eigenvalues are scaled back).  Accuracy is that of a
// backward-stable method: residuals and departure from orthogonality of
// order eps ||S||, eigenvectors to eps ||S|| / gap.  Non-finite input sets
// flag[0] = 3 and the run still ends with every index in range.
#pragma once
#include "common.h"

namespace sth {

constexpr int TE_T = 512;            // threads per workgroup
constexpr int TE_W = TE_T / 64;      // waves
constexpr int TE_LDS_N = 128;        // the matrix is kept in LDS up to this order
constexpr int TE_LDS_BUDGET = 154 * 1024;   // dynamic LDS bytes a teig workgroup may take

// Global scratch of one solve (doubles):
//   Vr  n * n    reflector k in column k, rows k+1..n-1 (only when A is in
//                LDS; otherwise the reflectors stay in the working copy Ag)
//   F   3 n R    inverse-iteration factors, [(3 i + c) R + r]
//   G   R * R    Gram of the eigenvector block (Newton-Schulz)
//   Zg  n * R    eigenvector block, row-major (only when it is not in LDS);
//                also the staging buffer of the Newton-Schulz product
//   Ag  n * n    working copy of A (only when A is not in LDS)
struct TeScratch {
    double *Vr, *F, *G, *Zg, *Ag;
};

__host__ __device__ inline int64_t te_part_doubles(int64_t n) { return 16 * n > 1024 ? 16 * n : 1024; }
// dynamic LDS of teig_body: the main region (A while tridiagonalizing, then
// the eigenvector block), the partial sums and the vectors.
__host__ __device__ inline size_t teig_lds_bytes(int64_t n, int64_t R, bool alds, bool zlds, bool vkeep = false) {
    int64_t main = 0;
    if (alds) main = n * n;
    if (zlds && n * R > main) main = n * R;
    if (alds && vkeep) main = n * n + n * R;   // reflectors stay in A's lower part, Z beside them
    return (size_t)(main + te_part_doubles(n) + 8 * n + R) * 8 + (size_t)R * 4 + 16;
}
__host__ __device__ inline bool teig_z_fits(int64_t n, int64_t R, bool alds) {
    return teig_lds_bytes(n, R, alds, true) <= (size_t)TE_LDS_BUDGET;
}
// the reflectors can stay in LDS through the back-transformation
__host__ __device__ inline bool teig_v_keep(int64_t n, int64_t R, bool alds) {
    return alds && teig_lds_bytes(n, R, true, true, true) <= (size_t)TE_LDS_BUDGET;
}
__host__ __device__ inline size_t teig_scratch_doubles(int64_t n, int64_t R, bool alds) {
    return (size_t)((alds ? n * n : 0) + 3 * n * R + R * R + n * R + (alds ? 0 : n * n)) + 64;
}
__host__ __device__ inline TeScratch teig_scratch_layout(double *base, int64_t n, int64_t R, bool alds) {
    TeScratch t;
    double *d = (double *)(((uintptr_t)base + 255) & ~(uintptr_t)255);
    t.Vr = alds ? d : nullptr;
    d += alds ? n * n : 0;
    t.F = d;
    d += 3 * n * R;
    t.G = d;
    d += R * R;
    t.Zg = d;
    d += n * R;
    t.Ag = alds ? nullptr : d;
    if (!alds) t.Vr = t.Ag;
    return t;
}

// DPP move of both halves of a double (lanes the pattern leaves out read 0)
template <int CTRL, int ROWS>
__device__ __forceinline__ double te_dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, true);
    return __hiloint2double(hi, lo);
}
// Sum over the 64 lanes of a wave, returned in every lane: row_shr 1, 2, 4, 8
// leave each 16-lane row's sum in its last lane, row_bcast 15 and 31 carry
// them into lane 63, read back with readlane (register moves only, no LDS).
__device__ __forceinline__ double te_wave_sum(double v) {
    v += te_dpp<0x111, 0xf>(v);   // row_shr:1
    v += te_dpp<0x112, 0xf>(v);   // row_shr:2
    v += te_dpp<0x114, 0xf>(v);   // row_shr:4
    v += te_dpp<0x118, 0xf>(v);   // row_shr:8
    v += te_dpp<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += te_dpp<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double te_wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double te_wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

// value of v in lane src (src uniform across the wave)
__device__ __forceinline__ double te_lane(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// 1 / x: the hardware reciprocal refined by one Newton step
__device__ __forceinline__ double te_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Numbers of eigenvalues of the tridiagonal (d, e2 = e^2) below sig[c],
// TE_NC independent counts interleaved: the sign changes of the leading
// principal minors p_i of T - sigma I.  A zero minor counts as positive (the
// LDL^T count with a negative-zero pivot): adding +0 turns -0 into +0, and
// the caller floors e^2 at a tiny positive value so that a zero minor is
// never followed by another.  Every 8 steps the pair (p_{i-1}, p_i) of each
// count is multiplied by the power of two that brings the exponent of the
// larger one to zero (exact, signs kept): the entries of T are at most
// 2 n <= 2^10 after scaling, so the larger one grows by less than 2^22 per step
// and shrinks by less than the e^2 floor (2^-120 ||T||^2) per two steps,
// which keeps every value normal between normalizations.
constexpr int TE_NC = 4;
__device__ __forceinline__ double te_pow2_inv(double m) {
    // 2^-e with e the unbiased exponent of the normal number m > 0
    const int e = (__double2hiint(m) >> 20) & 0x7ff;
    return __hiloint2double((2046 - e) << 20, 0);
}
__device__ __forceinline__ void te_sturm(const double *__restrict__ d, const double *__restrict__ e2, int n,
                                         const double (&sig)[TE_NC], int (&cnt)[TE_NC]) {
    double p0[TE_NC], p1[TE_NC];
#pragma unroll
    for (int c = 0; c < TE_NC; ++c) {
        p0[c] = 1.0;
        p1[c] = (d[0] - sig[c]) + 0.0;
        cnt[c] = (int)((unsigned)__double2hiint(p1[c]) >> 31);
    }
    int i = 1;
    for (; i + 8 <= n; i += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double di = d[i + u], ei = e2[i + u - 1];
#pragma unroll
            for (int c = 0; c < TE_NC; ++c) {
                const double p2 = fma(di - sig[c], p1[c], -ei * p0[c]) + 0.0;
                cnt[c] += (int)((unsigned)(__double2hiint(p2) ^ __double2hiint(p1[c])) >> 31);
                p0[c] = p1[c];
                p1[c] = p2;
            }
        }
#pragma unroll
        for (int c = 0; c < TE_NC; ++c) {
            const double sc = te_pow2_inv(fmax(fabs(p0[c]), fabs(p1[c])));
            p0[c] *= sc;
            p1[c] *= sc;
        }
    }
    for (; i < n; ++i) {
        const double di = d[i], ei = e2[i - 1];
#pragma unroll
        for (int c = 0; c < TE_NC; ++c) {
            const double p2 = fma(di - sig[c], p1[c], -ei * p0[c]) + 0.0;
            cnt[c] += (int)((unsigned)(__double2hiint(p2) ^ __double2hiint(p1[c])) >> 31);
            p0[c] = p1[c];
            p1[c] = p2;
        }
    }
}

// Start vector entry of eigenvector r: uniform in [-1, 1).
__device__ __forceinline__ double te_start(int r, int i) {
    const uint64_t h = splitmix64(0x7E16ull ^ ((uint64_t)(uint32_t)r << 32) ^ (uint64_t)(uint32_t)i);
    return (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// R leading eigenpairs of the symmetric n x n matrix S (column-major,
// leading dimension lds; (S + S^T) / 2 is used).  U (n x R, leading
// dimension ldu) receives the eigenvectors, lam (R, may be NULL) the
// eigenvalues in descending order.  ALDS: A in LDS (n <= TE_LDS_N); ZLDS:
// the eigenvector block in LDS (teig_z_fits).
template <bool ALDS, bool ZLDS>
__device__ void teig_body(const double *__restrict__ S, int64_t lds, int n, int R, double *__restrict__ U,
                          int64_t ldu, double *__restrict__ lam, bool sign_rule, TeScratch sc,
                          int64_t *__restrict__ flag) {
    extern __shared__ __align__(16) double te_dyn[];
    __shared__ double s_red[TE_W], s_red2[TE_W];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nn = (int64_t)n * n;
    const bool vkeep = teig_v_keep(n, R, ALDS);   // uniform
    int64_t main_sz = ALDS ? nn : 0;
    if (ZLDS && (int64_t)n * R > main_sz) main_sz = (int64_t)n * R;
    if (vkeep) main_sz = nn + (int64_t)n * R;
    double *const A = ALDS ? te_dyn : sc.Ag;            // column-major, leading dimension n
    double *const part = te_dyn + main_sz;              // te_part_doubles(n)
    double *const s_v = part + te_part_doubles(n);      // 2 n (double-buffered reflector)
    double2 *const s_vw = (double2 *)(s_v + 2 * n);     // n pairs (v, w) of the last step
    double *const s_p = s_v + 4 * n;                    // n (p of the last step; later e^2)
    double *const s_d = s_p + n;                        // n
    double *const s_e = s_d + n;                        // n
    double *const s_tau = s_e + n;                      // n
    double *const s_lam = s_tau + n;                    // R
    int *const s_cs = (int *)(s_lam + R);               // R cluster starts
    double *const Z = ZLDS ? (vkeep ? te_dyn + nn : te_dyn) : sc.Zg;   // row-major n x R (after step 1)
    // reflectors: column k of A holds v_k below the diagonal (LDS or the
    // scratch copy of A); without vkeep an LDS A is copied to sc.Vr after
    // step 1, because Z then takes its place
    const double *const Vr = (ALDS && !vkeep) ? sc.Vr : A;

    // ---- scale by a power of two, load (S + S^T) / 2 --------------------
    double mx = 0.0;
    int bad = 0;
    for (int64_t e = tid; e < nn; e += TE_T) {
        const double v = S[(e % n) + lds * (e / n)];
        if (!(fabs(v) <= 1.7976931348623157e308)) bad = 1;
        else mx = fmax(mx, fabs(v));
    }
    if (tid == 0) s_bad = 0;
    mx = te_wave_max(mx);
    if (lane == 0) s_red[wave] = mx;
    __syncthreads();
    if (bad) s_bad = 1;
    mx = 0.0;
    for (int w = 0; w < TE_W; ++w) mx = fmax(mx, s_red[w]);
    __syncthreads();
    const bool nonfinite = s_bad != 0;
    if (nonfinite && tid == 0 && flag) flag[0] = 3;
    if (mx == 0.0 && !nonfinite) {   // the zero matrix: e_1 .. e_R
        for (int64_t e = tid; e < (int64_t)n * R; e += TE_T) {
            const int i = (int)(e % n), r = (int)(e / n);
            U[i + ldu * r] = (i == r) ? 1.0 : 0.0;
        }
        if (lam)
            for (int r = tid; r < R; r += TE_T) lam[r] = 0.0;
        return;
    }
    const int sexp = (mx > 0.0 && !nonfinite) ? ilogb(mx) : 0;
    const double sc_in = ldexp(1.0, -sexp), sc_out = ldexp(1.0, sexp);
    if (!ALDS) {
        for (int64_t e = tid; e < nn; e += TE_T) {
            const int i = (int)(e % n), j = (int)(e / n);
            A[e] = 0.5 * (S[i + lds * j] + S[j + lds * i]) * sc_in;
        }
        __syncthreads();
    }

    // ---- 1. tridiagonalization -------------------------------------------
    if constexpr (ALDS) {
        // A in registers: thread (wave w, lane l) holds rows l and l + 64 of
        // the columns w + 8 q, q < 16.  Step k: the wave owning column k turns
        // the partial sums of step k - 1 into p and K, publishes (v, w) of step
        // k - 1, applies that step's update to column k and builds H_k
        // (v_k goes to column k of the LDS matrix area); after a barrier every
        // wave applies step k - 1's update to its columns j > k and
        // accumulates A v_k, the column operands taken from LDS once per wave
        // and broadcast with readlane.  Only vectors cross LDS.
        constexpr int NQ = TE_LDS_N / TE_W;   // 16
        double ar[2][NQ];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // all 32 pairs of loads issued before any use (indices clamped)
            double x[NQ], y[NQ];
            const int i = lane + 64 * h, ic = i < n ? i : n - 1;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int j = wave + TE_W * q, jc = j < n ? j : n - 1;
                x[q] = S[ic + lds * jc];
                y[q] = S[jc + lds * ic];
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int j = wave + TE_W * q;
                ar[h][q] = (i < n && j < n) ? 0.5 * (x[q] + y[q]) * sc_in : 0.0;
            }
        }
        for (int i = tid; i < 2 * n; i += TE_T) s_v[i] = 0.0;
        for (int i = tid; i < n; i += TE_T) s_vw[i] = make_double2(0.0, 0.0);
        // s_p (unused by this path) carries the next owner's column: column
        // k + 1 as updated through step k - 1, staged by the wave holding it
        if (wave == 0)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (lane + 64 * h < n) s_p[lane + 64 * h] = ar[h][0];
        __syncthreads();
        double Kprev = 0.0;
        for (int k = 0; k + 2 < n; ++k) {
            double *const vc = s_v + (k & 1) * n;
            const double *const vp = s_v + ((k & 1) ^ 1) * n;
            if (wave == k % TE_W) {
                const int qk = k / TE_W;
                double pr[2] = {0.0, 0.0}, vpr[2] = {0.0, 0.0}, wr[2] = {0.0, 0.0};
                if (k > 0) {
                    const double taup = s_tau[k - 1];
                    double t = 0.0;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int i = lane + 64 * h;
                        if (i >= k && i < n) {
                            double sp = 0.0;
#pragma unroll
                            for (int w = 0; w < TE_W; ++w) sp += part[w * n + i];
                            pr[h] = taup * sp;
                            vpr[h] = vp[i];
                            t += pr[h] * vpr[h];
                        }
                    }
                    Kprev = 0.5 * taup * te_wave_sum(t);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int i = lane + 64 * h;
                        wr[h] = pr[h] - Kprev * vpr[h];
                        if (i >= k && i < n) s_vw[i] = make_double2(vpr[h], wr[h]);
                    }
                }
                const int hk = k >> 6, lk = k & 63;
                const double vpk = te_lane(hk ? vpr[1] : vpr[0], lk);
                const double wpk = te_lane(hk ? wr[1] : wr[0], lk);
                double col[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = lane + 64 * h;
                    col[h] = (i < n ? s_p[i] : 0.0) - (vpr[h] * wpk + wr[h] * vpk);
                }
                double sig = 0.0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = lane + 64 * h;
                    if (i >= k + 2 && i < n) sig += col[h] * col[h];
                }
                sig = te_wave_sum(sig);
                const double akk = te_lane(hk ? col[1] : col[0], lk);
                const int h1 = (k + 1) >> 6, l1 = (k + 1) & 63;
                const double x0 = te_lane(h1 ? col[1] : col[0], l1);
                double beta = x0, tau = 0.0, scl = 0.0;
                if (sig > 0.0) {
                    // reciprocals refined by a Newton step in place of the
                    // divisions (H stays orthogonal to working accuracy)
                    const double nrm = sqrt(x0 * x0 + sig);
                    beta = x0 >= 0.0 ? -nrm : nrm;
                    tau = (beta - x0) * te_rcp(beta);
                    scl = te_rcp(x0 - beta);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = lane + 64 * h;
                    if (i >= k + 1 && i < n) {
                        const double v = (i == k + 1) ? 1.0 : (tau == 0.0 ? 0.0 : col[h] * scl);
                        vc[i] = v;
                        A[i + (int64_t)n * k] = v;
                    }
                }
                if (lane == 0) {
                    s_d[k] = akk;
                    s_e[k] = beta;
                    s_tau[k] = tau;
                }
            }
            __syncthreads();
            // column operands of this wave's columns (lane q < 16 loads column
            // wave + 8 q), row operands of this thread's rows
            double2 cvw = make_double2(0.0, 0.0);
            double cvc = 0.0;
            if (lane < NQ) {
                const int j = wave + TE_W * lane;
                if (j < n) {
                    cvw = s_vw[j];
                    cvc = vc[j];
                }
            }
            double2 rvw[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = lane + 64 * h;
                rvw[h] = i < n ? s_vw[i] : make_double2(0.0, 0.0);
            }
            double acc[2] = {0.0, 0.0};
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int j = wave + TE_W * q;
                if (j >= k + 1 && j < n) {   // uniform within the wave
                    const double vpj = te_lane(cvw.x, q), wj = te_lane(cvw.y, q), vcj = te_lane(cvc, q);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        double a = ar[h][q];
                        if (k > 0) {
                            a -= rvw[h].x * wj + rvw[h].y * vpj;
                            ar[h][q] = a;
                        }
                        acc[h] += a * vcj;
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = lane + 64 * h;
                if (i < n) part[wave * n + i] = acc[h];
            }
            if (wave == (k + 1) % TE_W && k + 1 < n) {
                const int q1 = (k + 1) / TE_W;   // uniform: a branch chain, no lane selects
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (q == q1) {
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            if (lane + 64 * h < n) s_p[lane + 64 * h] = ar[h][q];
                    }
            }
            __syncthreads();
        }
        // the last 2 x 2 block (or the whole matrix when n <= 2): raw entries
        // from their owners, p and K of step n - 3 from the partial sums
        double *const s_fin = s_red2;   // 6 doubles
        if (n >= 2) {
            const int c0 = n - 2, c1 = n - 1;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = lane + 64 * h;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    if (q == c0 / TE_W) a0 = ar[h][q];
                    if (q == c1 / TE_W) a1 = ar[h][q];
                }
                if (wave == c0 % TE_W && i == n - 2) s_fin[0] = a0;
                if (wave == c0 % TE_W && i == n - 1) s_fin[1] = a0;
                if (wave == c1 % TE_W && i == n - 1) s_fin[2] = a1;
            }
        } else if (tid == 0) {
            s_fin[0] = ar[0][0];
        }
        if (n >= 3 && wave == 0) {
            const double taup = s_tau[n - 3];
            const double *vq = s_v + ((n - 3) & 1) * n;
            double t = 0.0, pl = 0.0;
            const int i = n - 2 + lane;
            if (lane < 2) {
                double sp = 0.0;
#pragma unroll
                for (int w = 0; w < TE_W; ++w) sp += part[w * n + i];
                pl = taup * sp;
                t = pl * vq[i];
            }
            const double K = 0.5 * taup * te_wave_sum(t);
            if (lane < 2) s_fin[3 + lane] = pl;
            if (lane == 0) s_fin[5] = K;
        }
        __syncthreads();
        if (tid == 0) {
            if (n >= 3) {
                const double *v = s_v + ((n - 3) & 1) * n;
                const double v1 = v[n - 2], v2 = v[n - 1], K = s_fin[5];
                const double w1 = s_fin[3] - K * v1, w2 = s_fin[4] - K * v2;
                s_d[n - 2] = s_fin[0] - 2.0 * v1 * w1;
                s_e[n - 2] = s_fin[1] - (v2 * w1 + w2 * v1);
                s_d[n - 1] = s_fin[2] - 2.0 * v2 * w2;
            } else if (n == 2) {
                s_d[0] = s_fin[0];
                s_e[0] = s_fin[1];
                s_d[1] = s_fin[2];
            } else {
                s_d[0] = s_fin[0];
            }
        }
        __syncthreads();
    } else {
        // Per step k two barriers: wave 0 first turns the partial sums of step
        // k - 1 into p = tau A v and K = (tau / 2) p^T v, forms (v, w) of step
        // k - 1, updates column k and builds H_k; then every wave applies step
        // k - 1's update to the trailing block and accumulates A v_k.
        constexpr int TU = 4;   // columns per thread whose loads are issued together
        double Kprev = 0.0;
        for (int k = 0; k + 2 < n; ++k) {
            double *const vc = s_v + (k & 1) * n;
            const double *const vp = s_v + ((k & 1) ^ 1) * n;
            if (wave == 0) {
                if (k > 0) {
                    const double taup = s_tau[k - 1];
                    double t = 0.0;
                    for (int i = k + lane; i < n; i += 64) {
                        double sp = 0.0;
#pragma unroll
                        for (int w = 0; w < TE_W; ++w) sp += part[w * n + i];
                        const double p = taup * sp;
                        s_p[i] = p;
                        t += p * vp[i];
                    }
                    Kprev = 0.5 * taup * te_wave_sum(t);
                }
                // (v, w) of step k - 1 for rows >= k, column k with that step's
                // pending update, then H_k
                double sig = 0.0, a0 = 0.0;
                double wpk = 0.0, vpk = 0.0;
                if (k > 0) {
                    vpk = vp[k];
                    wpk = s_p[k] - Kprev * vpk;
                }
                for (int i = k + lane; i < n; i += 64) {
                    double a = A[i + (int64_t)n * k];
                    if (k > 0) {
                        const double vpi = vp[i], wpi = s_p[i] - Kprev * vpi;
                        s_vw[i] = make_double2(vpi, wpi);
                        a -= vpi * wpk + wpi * vpk;
                    }
                    if (i >= k + 2) sig += a * a;
                    if (i == k + lane && lane < 2) a0 = a;
                    part[i] = a;
                }
                sig = te_wave_sum(sig);
                const double akk = te_lane(a0, 0), x0 = te_lane(a0, 1);
                double beta = x0, tau = 0.0, scl = 0.0;
                if (sig > 0.0) {
                    const double nrm = sqrt(x0 * x0 + sig);
                    beta = x0 >= 0.0 ? -nrm : nrm;
                    tau = (beta - x0) / beta;
                    scl = 1.0 / (x0 - beta);
                }
                for (int i = k + 1 + lane; i < n; i += 64) {
                    const double v = (i == k + 1) ? 1.0 : (tau == 0.0 ? 0.0 : part[i] * scl);
                    vc[i] = v;
                    A[i + (int64_t)n * k] = v;   // column k is not read again by the reduction
                }
                if (lane == 0) {
                    s_d[k] = akk;
                    s_e[k] = beta;
                    s_tau[k] = tau;
                }
            }
            __syncthreads();
            // trailing block: pending update of step k - 1, and partial sums of A v_k
            for (int i0 = k + 1; i0 < n; i0 += 64) {
                const int i = i0 + lane;
                if (i < n) {
                    double acc = 0.0;
                    double2 pwi = make_double2(0.0, 0.0);
                    if (k > 0) pwi = s_vw[i];
                    for (int jb = k + 1 + wave; jb < n; jb += TE_W * TU) {
                        double a[TU], vcj[TU];
                        double2 pw[TU];
#pragma unroll
                        for (int u = 0; u < TU; ++u) {
                            const int j = jb + TE_W * u;
                            const int jc = j < n ? j : n - 1;
                            a[u] = A[i + (int64_t)n * jc];
                            vcj[u] = j < n ? vc[jc] : 0.0;
                            pw[u] = (k > 0) ? s_vw[jc] : make_double2(0.0, 0.0);
                        }
#pragma unroll
                        for (int u = 0; u < TU; ++u) {
                            const int j = jb + TE_W * u;
                            if (k > 0) {
                                a[u] -= pwi.x * pw[u].y + pwi.y * pw[u].x;
                                if (j < n) A[i + (int64_t)n * j] = a[u];
                            }
                            acc += a[u] * vcj[u];
                        }
                    }
                    part[wave * n + i] = acc;
                }
            }
            __syncthreads();
        }
        if (n >= 3 && wave == 0) {
            // p and K of the last step (n - 3)
            const double taup = s_tau[n - 3];
            const double *vp = s_v + ((n - 3) & 1) * n;
            double t = 0.0;
            for (int i = n - 2 + lane; i < n; i += 64) {
                double sp = 0.0;
#pragma unroll
                for (int w = 0; w < TE_W; ++w) sp += part[w * n + i];
                const double p = taup * sp;
                s_p[i] = p;
                t += p * vp[i];
            }
            Kprev = 0.5 * taup * te_wave_sum(t);
        }
        if (tid == 0) {
            if (n >= 3) {
                // the last 2 x 2 block with the update of step n - 3
                const double *v = s_v + ((n - 3) & 1) * n;
                const double v1 = v[n - 2], v2 = v[n - 1];
                const double w1 = s_p[n - 2] - Kprev * v1, w2 = s_p[n - 1] - Kprev * v2;
                s_d[n - 2] = A[(n - 2) + (int64_t)n * (n - 2)] - 2.0 * v1 * w1;
                s_e[n - 2] = A[(n - 1) + (int64_t)n * (n - 2)] - (v2 * w1 + w2 * v1);
                s_d[n - 1] = A[(n - 1) + (int64_t)n * (n - 1)] - 2.0 * v2 * w2;
            } else if (n == 2) {
                s_d[0] = A[0];
                s_e[0] = A[1];
                s_d[1] = A[3];
            } else {
                s_d[0] = A[0];
            }
        }
        __syncthreads();
    }

    if (ALDS && !vkeep)
        for (int64_t e = tid; e < nn; e += TE_T) sc.Vr[e] = A[e];

    // ---- 2. bisection for the R largest eigenvalues ----------------------
    double glo = 1e300, ghi = -1e300;
    for (int i = tid; i < n; i += TE_T) {
        const double r = (i > 0 ? fabs(s_e[i - 1]) : 0.0) + (i + 1 < n ? fabs(s_e[i]) : 0.0);
        glo = fmin(glo, s_d[i] - r);
        ghi = fmax(ghi, s_d[i] + r);
    }
    glo = te_wave_min(glo);
    ghi = te_wave_max(ghi);
    if (lane == 0) {
        s_red[wave] = glo;
        s_red2[wave] = ghi;
    }
    __syncthreads();
    glo = s_red[0];
    ghi = s_red2[0];
    for (int w = 1; w < TE_W; ++w) {
        glo = fmin(glo, s_red[w]);
        ghi = fmax(ghi, s_red2[w]);
    }
    const double tnorm = fmax(fmax(fabs(glo), fabs(ghi)), 1e-300);
    glo -= 4.0 * 2.220446049250313e-16 * tnorm;
    ghi += 4.0 * 2.220446049250313e-16 * tnorm;
    {
        // e^2, floored at (2^-60 ||T||)^2: a change of the off-diagonal below
        // 1e-18 ||T||, far under the eps ||T|| accuracy of the eigenvalues
        const double e2min = 0x1p-120 * tnorm * tnorm;
        for (int i = tid; i + 1 < n; i += TE_T) s_p[i] = fmax(s_e[i] * s_e[i], e2min);
    }
    __syncthreads();
    {
        // a group of tpe lanes searches one eigenvalue, TE_NC points per lane:
        // each round splits the bracket into tpe * TE_NC + 1 parts.  Groups
        // cover at most 256 lanes (one wave per SIMD) at a time: more lanes
        // would only add FP64 work per round (the counts, not their latency,
        // bound the search)
        int tpe = 64;
        while (tpe > 1 && tpe * R > 256) tpe >>= 1;   // at most four waves: the counts are FP64-throughput bound
        const int ngroups = TE_T / tpe, g = tid / tpe, t = tid % tpe;
        const double npts1 = (double)(tpe * TE_NC + 1);
        const int rounds_r = (R + ngroups - 1) / ngroups;
        for (int rr = 0; rr < rounds_r; ++rr) {
            const int r = g + rr * ngroups;
            if (r < R) {   // uniform within the group
                const int kk = n - 1 - r;   // the kk-th smallest, 0-based
                double lo = glo, hi = ghi;
                for (int round = 0; round < 64; ++round) {
                    if (!(hi - lo > 2.220446049250313e-16 * (tnorm + fabs(lo) + fabs(hi)))) break;
                    double sig[TE_NC];
                    int cnt[TE_NC];
#pragma unroll
                    for (int c = 0; c < TE_NC; ++c) sig[c] = lo + (hi - lo) * (double)(t * TE_NC + c + 1) / npts1;
                    te_sturm(s_d, s_p, n, sig, cnt);
                    double nlo = -HUGE_VAL, nhi = HUGE_VAL;
#pragma unroll
                    for (int c = 0; c < TE_NC; ++c) {
                        if (cnt[c] <= kk) nlo = fmax(nlo, sig[c]);
                        else nhi = fmin(nhi, sig[c]);
                    }
                    for (int o = 1; o < tpe; o <<= 1) {
                        nlo = fmax(nlo, __shfl_xor(nlo, o));
                        nhi = fmin(nhi, __shfl_xor(nhi, o));
                    }
                    lo = fmax(lo, nlo);
                    hi = fmin(hi, nhi);
                }
                if (t == 0) s_lam[r] = 0.5 * (lo + hi);
            }
        }
    }
    __syncthreads();

    // ---- 3. inverse iteration, one thread per eigenvector ----------------
    {
        const double tiny = 2.220446049250313e-16 * tnorm;
        double *__restrict__ F = sc.F;
        double *__restrict__ Zr = Z;
        for (int r = tid; r < R; r += TE_T) {
            const double lm = s_lam[r];
            double nrm2 = 0.0;
            for (int i = 0; i < n; ++i) {
                const double b = te_start(r, i);
                Zr[(int64_t)i * R + r] = b;
                nrm2 += b * b;
            }
            for (int pass = 0; pass < 2; ++pass) {
                const double inv = te_rcp(sqrt(nrm2));
                // forward elimination with partial pivoting: U rows (1 / u0, u1, u2) to F, y to Z
                double cd = s_d[0] - lm, cu = n > 1 ? s_e[0] : 0.0, cb = Zr[r] * inv;
#pragma unroll 4
                for (int i = 0; i + 1 < n; ++i) {
                    const double sub = s_e[i], nd = s_d[i + 1] - lm, nu = i + 2 < n ? s_e[i + 1] : 0.0;
                    const double nb = Zr[(int64_t)(i + 1) * R + r] * inv;
                    double ru0, u1, u2, y;
                    if (fabs(cd) >= fabs(sub)) {
                        if (cd == 0.0) cd = tiny;
                        ru0 = te_rcp(cd);
                        const double ml = sub * ru0;
                        u1 = cu;
                        u2 = 0.0;
                        y = cb;
                        cd = nd - ml * cu;
                        cu = nu;
                        cb = nb - ml * cb;
                    } else {
                        ru0 = te_rcp(sub);
                        const double ml = cd * ru0;
                        u1 = nd;
                        u2 = nu;
                        y = nb;
                        cd = cu - ml * nd;
                        cu = -ml * nu;
                        cb = cb - ml * nb;
                    }
                    F[(int64_t)(3 * i) * R + r] = ru0;
                    F[(int64_t)(3 * i + 1) * R + r] = u1;
                    F[(int64_t)(3 * i + 2) * R + r] = u2;
                    Zr[(int64_t)i * R + r] = y;
                }
                if (cd == 0.0) cd = tiny;
                // back substitution, the factors of 4 rows loaded ahead
                double x1 = cb * te_rcp(cd), x2 = 0.0;
                Zr[(int64_t)(n - 1) * R + r] = x1;
                nrm2 = x1 * x1;
                for (int i0 = n - 2; i0 >= 0; i0 -= 4) {
                    double f0[4], f1[4], f2[4], y[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 - u >= 0 ? i0 - u : 0;
                        f0[u] = F[(int64_t)(3 * i) * R + r];
                        f1[u] = F[(int64_t)(3 * i + 1) * R + r];
                        f2[u] = F[(int64_t)(3 * i + 2) * R + r];
                        y[u] = Zr[(int64_t)i * R + r];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (i0 - u < 0) break;
                        const double x = (y[u] - f1[u] * x1 - f2[u] * x2) * f0[u];
                        Zr[(int64_t)(i0 - u) * R + r] = x;
                        nrm2 += x * x;
                        x2 = x1;
                        x1 = x;
                    }
                }
            }
            const double inv = te_rcp(sqrt(nrm2));
            for (int i = 0; i < n; ++i) Zr[(int64_t)i * R + r] *= inv;
        }
    }
    __syncthreads();

    // ---- 4a. clusters: classical Gram-Schmidt twice inside each ----------
    if (tid == 0) {
        int cs = 0;
        s_cs[0] = 0;
        for (int r = 1; r < R; ++r) {
            if (!(s_lam[r - 1] - s_lam[r] <= 1e-9 * tnorm)) cs = r;
            s_cs[r] = cs;
        }
    }
    __syncthreads();
    for (int j = 1; j < R; ++j) {
        const int c0 = s_cs[j];
        if (c0 == j) continue;
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = c0 + wave; i < j; i += TE_W) {
                double s = 0.0;
                for (int q = lane; q < n; q += 64) s += Z[(int64_t)q * R + i] * Z[(int64_t)q * R + j];
                s = te_wave_sum(s);
                if (lane == 0) part[i] = s;
            }
            __syncthreads();
            for (int q = tid; q < n; q += TE_T) {
                double acc = Z[(int64_t)q * R + j];
                for (int i = c0; i < j; ++i) acc -= part[i] * Z[(int64_t)q * R + i];
                Z[(int64_t)q * R + j] = acc;
            }
            __syncthreads();
        }
        double s = 0.0;
        for (int q = tid; q < n; q += TE_T) s += Z[(int64_t)q * R + j] * Z[(int64_t)q * R + j];
        s = te_wave_sum(s);
        if (lane == 0) s_red[wave] = s;
        __syncthreads();
        s = 0.0;
        for (int w = 0; w < TE_W; ++w) s += s_red[w];
        const double inv = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
        for (int q = tid; q < n; q += TE_T) Z[(int64_t)q * R + j] *= inv;
        __syncthreads();
    }

    // ---- 4b. one Newton-Schulz step on the FP64 matrix cores -------------
    {
        const int tr = lane & 15, tg = lane >> 4;
        const int nt = (R + 15) / 16, ntr = (n + 15) / 16;
        // G = Z^T Z (tiles bi <= bj, mirrored)
        for (int q = wave; q < nt * (nt + 1) / 2; q += TE_W) {
            int bi = 0;
            while ((bi + 1) * nt - bi * (bi + 1) / 2 <= q) ++bi;
            const int bj = bi + q - (bi * nt - bi * (bi - 1) / 2);
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
            const int ra = 16 * bi + tr, cb = 16 * bj + tr;
            for (int k0 = 0; k0 < n; k0 += 4) {
                const int k = k0 + tg;
                const double a = (ra < R && k < n) ? Z[(int64_t)k * R + ra] : 0.0;
                const double b = (cb < R && k < n) ? Z[(int64_t)k * R + cb] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * bi + tg + 4 * v;
                if (row < R && cb < R) {
                    sc.G[row + (int64_t)R * cb] = acc[v];
                    sc.G[cb + (int64_t)R * row] = acc[v];
                }
            }
        }
        __syncthreads();
        // Znew = 1.5 Z - 0.5 Z G into the staging buffer (row tile per task)
        double *const Zs = ZLDS ? sc.Zg : sc.F;
        for (int q = wave; q < ntr * nt; q += TE_W) {
            const int bi = q / nt, bj = q % nt;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
            const int ra = 16 * bi + tr, cb = 16 * bj + tr;
            for (int k0 = 0; k0 < R; k0 += 4) {
                const int k = k0 + tg;
                const double a = (ra < n && k < R) ? Z[(int64_t)ra * R + k] : 0.0;
                const double b = (k < R && cb < R) ? sc.G[k + (int64_t)R * cb] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * bi + tg + 4 * v;
                if (row < n && cb < R) Zs[(int64_t)row * R + cb] = 1.5 * Z[(int64_t)row * R + cb] - 0.5 * acc[v];
            }
        }
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)n * R; e += TE_T) Z[e] = Zs[e];
        __syncthreads();
    }

    // ---- 5. back-transformation ------------------------------------------
    if constexpr (ALDS) {
        // Z in registers: lane r (of each 64-column chunk) of wave w holds
        // rows w + 8 q, q < 16, of column r.  Per applied reflector: lanes
        // q < 16 load v(w + 8 q) (LDS, or the scratch with the load issued a
        // step ahead), readlane broadcasts them, the partial dot products are
        // summed over the waves in LDS (double-buffered, one barrier per step).
        constexpr int NQ = TE_LDS_N / TE_W;
        auto next_k = [&](int k) {
            while (k >= 0 && s_tau[k] == 0.0) --k;
            return k;
        };
        auto vload = [&](int k) -> double {
            const int i = wave + TE_W * lane;
            return (k >= 0 && lane < NQ && i > k && i < n) ? Vr[i + (int64_t)n * k] : 0.0;
        };
        for (int rc = 0; rc < R; rc += 64) {
            const int r = rc + lane;
            const bool rv = r < R;
            double zr[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = wave + TE_W * q;
                zr[q] = (rv && i < n) ? Z[(int64_t)i * R + r] : 0.0;
            }
            int kc = next_k(n - 3);
            double vl = vload(kc);
            int par = 0;
            while (kc >= 0) {
                const int kn = next_k(kc - 1);
                double sacc = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) sacc += te_lane(vl, q) * zr[q];
                double *pb = part + par * (TE_W * 64);
                pb[wave * 64 + lane] = sacc;
                __syncthreads();
                const double vnext = vload(kn);   // in flight during the update
                double c = 0.0;
#pragma unroll
                for (int w = 0; w < TE_W; ++w) c += pb[w * 64 + lane];
                c *= s_tau[kc];
#pragma unroll
                for (int q = 0; q < NQ; ++q) zr[q] -= c * te_lane(vl, q);
                vl = vnext;
                kc = kn;
                par ^= 1;
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = wave + TE_W * q;
                if (rv && i < n) Z[(int64_t)i * R + r] = zr[q];
            }
            __syncthreads();
        }
    } else {
        // Each wave owns the rows i = wave (mod 8) of Z, so the only exchange is
        // the partial dot products (double-buffered).  With the reflectors in
        // LDS (vkeep) they are read in place.  Otherwise the reflectors of the
        // applied steps k_0 > k_1 > ... (tau != 0) are staged from the scratch
        // into three LDS buffers two steps ahead: step t issues the loads of
        // v_{k_{t+2}} right after its barrier and stores them after its update
        // (so their latency overlaps the update and the next step's dot products;
        // a barrier waits for every load in flight), the barrier of step t + 1
        // orders the stores before their use, and the buffer they overwrite was
        // last read in step t - 1, which every wave finished before the barrier
        // of step t.
        {
            double *const s_vb = s_v;   // 3 n doubles (the vectors of step 1 are dead)
            auto next_k = [&](int k) {
                while (k >= 0 && s_tau[k] == 0.0) --k;
                return k;
            };
            const int nper = (n + TE_T - 1) / TE_T;   // staged entries per thread (n <= 4 * TE_T)
            for (int rc = 0; rc < R; rc += 64) {
                const int r = rc + lane;
                const bool rv = r < R;
                int kc = next_k(n - 3);
                int kn = kc >= 0 ? next_k(kc - 1) : -1;
                int kf = kn >= 0 ? next_k(kn - 1) : -1;   // staged two steps ahead
                if (!vkeep) {
                    if (kc >= 0)
                        for (int i = kc + 1 + tid; i < n; i += TE_T) s_vb[i] = Vr[i + (int64_t)n * kc];
                    if (kn >= 0)
                        for (int i = kn + 1 + tid; i < n; i += TE_T) s_vb[n + i] = Vr[i + (int64_t)n * kn];
                    __syncthreads();
                }
                int buf = 0, par = 0;
                while (kc >= 0) {
                    const double *v = vkeep ? Vr + (int64_t)n * kc : s_vb + buf * n;
                    const double tau = s_tau[kc];
                    const int i0 = kc + 1 + (((wave - kc - 1) % TE_W) + TE_W) % TE_W;
                    // rows i0, i0 + 8, ... in batches of 4 whose loads are issued
                    // together (indices clamped; the extra terms are multiplied by 0)
                    double sacc = 0.0;
                    if (rv)
                        for (int i = i0; i < n; i += 4 * TE_W) {
                            double vv[4], zz[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int ii = i + u * TE_W, ic = ii < n ? ii : n - 1;
                                vv[u] = ii < n ? v[ic] : 0.0;
                                zz[u] = Z[(int64_t)ic * R + r];
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) sacc += vv[u] * zz[u];
                        }
                    double *pb = part + par * (TE_W * 64);
                    pb[wave * 64 + lane] = sacc;
                    __syncthreads();
                    double pre[4];
                    if (!vkeep && kf >= 0) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int i = tid + q * TE_T;
                            pre[q] = (q < nper && i > kf && i < n) ? Vr[i + (int64_t)n * kf] : 0.0;
                        }
                    }
                    double c = 0.0;
#pragma unroll
                    for (int w = 0; w < TE_W; ++w) c += pb[w * 64 + lane];
                    c *= tau;
                    if (rv)
                        for (int i = i0; i < n; i += 4 * TE_W) {
                            double vv[4], zz[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int ii = i + u * TE_W, ic = ii < n ? ii : n - 1;
                                vv[u] = v[ic];
                                zz[u] = Z[(int64_t)ic * R + r];
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (i + u * TE_W < n) Z[(int64_t)(i + u * TE_W) * R + r] = zz[u] - c * vv[u];
                        }
                    if (!vkeep && kf >= 0) {
                        double *vf = s_vb + ((buf + 2) % 3) * n;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int i = tid + q * TE_T;
                            if (q < nper && i > kf && i < n) vf[i] = pre[q];
                        }
                    }
                    kc = kn;
                    kn = kf;
                    kf = kf >= 0 ? next_k(kf - 1) : -1;
                    buf = (buf + 1) % 3;
                    par ^= 1;
                }
                __syncthreads();
            }
        }
    }

    // ---- 6. sign rule and output -----------------------------------------
    double *const s_sgn = part;
    for (int r = tid; r < R; r += TE_T) {
        double best = -1.0;
        int arg = 0;   // in range even when every entry is NaN
        for (int i = 0; i < n; ++i) {
            const double v = fabs(Z[(int64_t)i * R + r]);
            if (v > best) {
                best = v;
                arg = i;
            }
        }
        s_sgn[r] = (sign_rule && Z[(int64_t)arg * R + r] < 0.0) ? -1.0 : 1.0;
        if (lam) lam[r] = s_lam[r] * sc_out;
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)n * R; e += TE_T) {
        const int i = (int)(e % n), r = (int)(e / n);
        U[i + ldu * r] = s_sgn[r] * Z[(int64_t)i * R + r];
    }
}

}  // namespace sth
