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
//      (no division; the pair is rescaled by a power of two when it leaves
//      [2^-200, 2^200], which keeps every sign).  A minor that vanishes is
//      replaced by -pivmin times its predecessor (the pivot -pivmin of the
//      LDL^T form of the count).  Each eigenvalue is searched by a group of
//      lanes that splits its interval into (group size + 1) parts per round.
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
__host__ __device__ inline size_t teig_lds_bytes(int64_t n, int64_t R, bool alds, bool zlds) {
    int64_t main = 0;
    if (alds) main = n * n;
    if (zlds && n * R > main) main = n * R;
    return (size_t)(main + te_part_doubles(n) + 6 * n + R) * 8 + (size_t)R * 4 + 16;
}
__host__ __device__ inline bool teig_z_fits(int64_t n, int64_t R, bool alds) {
    return teig_lds_bytes(n, R, alds, true) <= (size_t)TE_LDS_BUDGET;
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

__device__ __forceinline__ double te_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
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

// Number of eigenvalues of the tridiagonal (d, e2 = e^2) below sig.
__device__ __forceinline__ int te_sturm(const double *__restrict__ d, const double *__restrict__ e2, int n,
                                        double sig, double pivmin) {
    double p0 = 1.0, p1 = d[0] - sig;
    if (fabs(p1) < pivmin) p1 = -pivmin;
    int cnt = p1 < 0.0;
    for (int i = 1; i < n; ++i) {
        double p2 = (d[i] - sig) * p1 - e2[i - 1] * p0;
        if (fabs(p2) < pivmin * fabs(p1)) p2 = -pivmin * p1;
        cnt += (p2 < 0.0) != (p1 < 0.0);
        const double m = fmax(fabs(p1), fabs(p2));
        if (m > 0x1p200 || m < 0x1p-200) {
            const int ex = ilogb(m);
            p1 = ldexp(p1, -ex);
            p2 = ldexp(p2, -ex);
        }
        p0 = p1;
        p1 = p2;
    }
    return cnt;
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
    int64_t main_sz = ALDS ? nn : 0;
    if (ZLDS && (int64_t)n * R > main_sz) main_sz = (int64_t)n * R;
    double *const A = ALDS ? te_dyn : sc.Ag;            // column-major, leading dimension n
    double *const part = te_dyn + main_sz;              // te_part_doubles(n)
    double *const s_v = part + te_part_doubles(n);      // 2 n (double-buffered reflector)
    double *const s_p = s_v + 2 * n;                    // n (p of the last step; later e^2)
    double *const s_d = s_p + n;                        // n
    double *const s_e = s_d + n;                        // n
    double *const s_tau = s_e + n;                      // n
    double *const s_lam = s_tau + n;                    // R
    int *const s_cs = (int *)(s_lam + R);               // R cluster starts
    double *const Z = ZLDS ? te_dyn : sc.Zg;            // row-major n x R (after step 1)
    double *const Vr = ALDS ? sc.Vr : sc.Ag;            // reflectors

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
    for (int64_t e = tid; e < nn; e += TE_T) {
        const int i = (int)(e % n), j = (int)(e / n);
        A[e] = 0.5 * (S[i + lds * j] + S[j + lds * i]) * sc_in;
    }
    __syncthreads();

    // ---- 1. tridiagonalization -------------------------------------------
    double Kprev = 0.0;
    for (int k = 0; k + 2 < n; ++k) {
        double *const vc = s_v + (k & 1) * n;
        const double *const vp = s_v + ((k & 1) ^ 1) * n;
        if (wave == 0) {
            // column k with the pending update of step k - 1, then H_k
            const double vpk = k > 0 ? vp[k] : 0.0;
            const double wpk = k > 0 ? s_p[k] - Kprev * vpk : 0.0;
            double sig = 0.0, x0 = 0.0, akk = 0.0;
            for (int i = k + lane; i < n; i += 64) {
                double a = A[i + (int64_t)n * k];
                if (k > 0) {
                    const double vpi = vp[i], wpi = s_p[i] - Kprev * vpi;
                    a -= vpi * wpk + wpi * vpk;
                }
                if (i == k) akk = a;
                else if (i == k + 1) x0 = a;
                else sig += a * a;
                part[i] = a;
            }
            sig = te_wave_sum(sig);
            x0 = te_wave_sum(x0);
            akk = te_wave_sum(akk);
            double beta = x0, tau = 0.0, scl = 0.0;
            if (sig > 0.0) {
                const double nrm = sqrt(x0 * x0 + sig);
                beta = x0 >= 0.0 ? -nrm : nrm;
                tau = (beta - x0) / beta;
                scl = 1.0 / (x0 - beta);
            }
            for (int i = k + lane; i < n; i += 64) {
                if (i == k) continue;
                const double v = (i == k + 1) ? 1.0 : part[i] * scl;
                vc[i] = v;
                Vr[i + (int64_t)n * k] = v;
            }
            if (lane == 0) {
                s_d[k] = akk;
                s_e[k] = beta;
                s_tau[k] = tau;
            }
        }
        __syncthreads();
        const double tau = s_tau[k];
        // trailing block: pending update of step k - 1, and partial sums of A v
        for (int i0 = k + 1; i0 < n; i0 += 64) {
            const int i = i0 + lane;
            if (i < n) {
                double acc = 0.0, vpi = 0.0, wpi = 0.0;
                if (k > 0) {
                    vpi = vp[i];
                    wpi = s_p[i] - Kprev * vpi;
                }
                for (int j = k + 1 + wave; j < n; j += TE_W) {
                    double a = A[i + (int64_t)n * j];
                    if (k > 0) {
                        const double vpj = vp[j], wpj = s_p[j] - Kprev * vpj;
                        a -= vpi * wpj + wpi * vpj;
                        A[i + (int64_t)n * j] = a;
                    }
                    acc += a * vc[j];
                }
                part[wave * n + i] = acc;
            }
        }
        __syncthreads();
        double t = 0.0;
        for (int i = k + 1 + tid; i < n; i += TE_T) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < TE_W; ++w) s += part[w * n + i];
            const double p = tau * s;
            s_p[i] = p;
            t += p * vc[i];
        }
        t = te_wave_sum(t);
        if (lane == 0) s_red[wave] = t;
        __syncthreads();
        double pv = 0.0;
#pragma unroll
        for (int w = 0; w < TE_W; ++w) pv += s_red[w];
        Kprev = 0.5 * tau * pv;
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
    for (int i = tid; i + 1 < n; i += TE_T) s_p[i] = s_e[i] * s_e[i];
    __syncthreads();
    glo = s_red[0];
    ghi = s_red2[0];
    for (int w = 1; w < TE_W; ++w) {
        glo = fmin(glo, s_red[w]);
        ghi = fmax(ghi, s_red2[w]);
    }
    const double tnorm = fmax(fmax(fabs(glo), fabs(ghi)), 1e-300);
    const double pivmin = 1e-80;
    glo -= 4.0 * 2.220446049250313e-16 * tnorm;
    ghi += 4.0 * 2.220446049250313e-16 * tnorm;
    {
        int tpe = 64;
        while (tpe > 1 && tpe * R > TE_T) tpe >>= 1;
        const int ngroups = TE_T / tpe, g = tid / tpe, t = tid % tpe;
        const int rounds_r = (R + ngroups - 1) / ngroups;
        for (int rr = 0; rr < rounds_r; ++rr) {
            const int r = g + rr * ngroups;
            if (r < R) {   // uniform within the group
                const int kk = n - 1 - r;   // the kk-th smallest, 0-based
                double lo = glo, hi = ghi;
                for (int round = 0; round < 96; ++round) {
                    if (!(hi - lo > 2.220446049250313e-16 * (tnorm + fabs(lo) + fabs(hi)))) break;
                    const double sig = lo + (hi - lo) * (double)(t + 1) / (double)(tpe + 1);
                    const int c = te_sturm(s_d, s_p, n, sig, pivmin);
                    double nlo = c <= kk ? sig : -HUGE_VAL;
                    double nhi = c > kk ? sig : HUGE_VAL;
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
    const double tiny = 2.220446049250313e-16 * tnorm;
    for (int r = tid; r < R; r += TE_T) {
        const double lm = s_lam[r];
        double nrm2 = 0.0;
        for (int i = 0; i < n; ++i) {
            const double b = te_start(r, i);
            Z[(int64_t)i * R + r] = b;
            nrm2 += b * b;
        }
        for (int s = 0; s < 2; ++s) {
            const double inv = 1.0 / sqrt(nrm2);
            double cd = s_d[0] - lm, cu = n > 1 ? s_e[0] : 0.0, cb = Z[r] * inv;
            for (int i = 0; i + 1 < n; ++i) {
                const double sub = s_e[i], nd = s_d[i + 1] - lm, nu = i + 2 < n ? s_e[i + 1] : 0.0;
                const double nb = Z[(int64_t)(i + 1) * R + r] * inv;
                double u0, u1, u2, y;
                if (fabs(cd) >= fabs(sub)) {
                    if (cd == 0.0) cd = tiny;
                    const double ml = sub / cd;
                    u0 = cd;
                    u1 = cu;
                    u2 = 0.0;
                    y = cb;
                    cd = nd - ml * cu;
                    cu = nu;
                    cb = nb - ml * cb;
                } else {
                    const double ml = cd / sub;
                    u0 = sub;
                    u1 = nd;
                    u2 = nu;
                    y = nb;
                    cd = cu - ml * nd;
                    cu = -ml * nu;
                    cb = cb - ml * nb;
                }
                sc.F[(int64_t)(3 * i) * R + r] = 1.0 / u0;
                sc.F[(int64_t)(3 * i + 1) * R + r] = u1;
                sc.F[(int64_t)(3 * i + 2) * R + r] = u2;
                Z[(int64_t)i * R + r] = y;
            }
            if (cd == 0.0) cd = tiny;
            double x1 = cb / cd, x2 = 0.0;
            Z[(int64_t)(n - 1) * R + r] = x1;
            nrm2 = x1 * x1;
#pragma unroll 4
            for (int i = n - 2; i >= 0; --i) {
                const double x = (Z[(int64_t)i * R + r] - sc.F[(int64_t)(3 * i + 1) * R + r] * x1 -
                                  sc.F[(int64_t)(3 * i + 2) * R + r] * x2) *
                                 sc.F[(int64_t)(3 * i) * R + r];
                Z[(int64_t)i * R + r] = x;
                nrm2 += x * x;
                x2 = x1;
                x1 = x;
            }
        }
        const double inv = 1.0 / sqrt(nrm2);
        for (int i = 0; i < n; ++i) Z[(int64_t)i * R + r] *= inv;
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
    // Each wave owns the rows i = wave (mod 8) of Z, so the only exchange is
    // the partial dot products, double-buffered by the parity of the applied
    // reflectors (skipped identity reflectors do not flip it).
    for (int rc = 0; rc < R; rc += 64) {
        const int r = rc + lane;
        const bool rv = r < R;
        int par = 0;
        for (int k = n - 3; k >= 0; --k) {
            const double tau = s_tau[k];
            if (tau == 0.0) continue;   // uniform
            const int i0 = k + 1 + (((wave - k - 1) % TE_W) + TE_W) % TE_W;
            const double *v = Vr + (int64_t)n * k;
            double s = 0.0;
            if (rv)
                for (int i = i0; i < n; i += TE_W) s += v[i] * Z[(int64_t)i * R + r];
            double *pb = part + par * (TE_W * 64);
            par ^= 1;
            pb[wave * 64 + lane] = s;
            __syncthreads();
            double c = 0.0;
#pragma unroll
            for (int w = 0; w < TE_W; ++w) c += pb[w * 64 + lane];
            c *= tau;
            if (rv)
                for (int i = i0; i < n; i += TE_W) Z[(int64_t)i * R + r] -= c * v[i];
        }
        __syncthreads();
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
