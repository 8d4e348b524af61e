// FP64 symmetric eigensolver for the EIG branch of Alg. 2: the R_n leading
// eigenvectors of the mode-n Gram matrix.
//
// Routes (eig_launch):
//   * eig_leading up to order 128: two-sided cyclic Jacobi with a parallel
//     (round-robin) ordering in one 512-thread workgroup, A and V in LDS when
//     they fit (jacobi_*_kernel; relative accuracy, sweep cap reported).
//   * decompositions up to order 128, and every order where the subspace
//     iteration does not apply: the direct solver of teig_body.h
//     (tridiagonalization, bisection, inverse iteration) in one workgroup.
//   * above order 128 with a block p = R + 16 (rounded to 8) <= 128: subspace
//     iteration Q <- orth(S Q) from a seeded Gaussian block (2 products when
//     S carries single-precision rounding, 3 for FP64 data; orth = shifted
//     Cholesky-QR, see orth()), Rayleigh-Ritz with the direct solver on
//     T = Q^T S Q, then a residual test: the R Ritz pairs are accepted when
//     every ||S u - theta u|| <= max(16 sqrt(n) eps, u_S) |theta_1|, i.e. when
//     they are exact eigenpairs of a perturbation of S no larger than that of
//     a backward-stable direct solver or than the rounding S already carries
//     (u_S: the unit roundoff of the products that formed S, eps for FP64
//     products, 2^-24 for FP32 and bf16x6, 2^-17 for bf16x3).  A failed test
//     runs a second round (2 more products and Rayleigh-Ritz from the same
//     basis); when that fails too, the direct solver runs on S itself.  Every
//     launch after the first round is gated on the device by the residuals
//     (it returns at once when they passed), so the whole solve is one
//     fixed, capturable sequence, and the result is the leading eigenpairs
//     on every spectrum, with or without a gap after R.
//
// Selection: eigenvalues in descending order, the R leading eigenvectors
// signed so that their entry of largest magnitude is positive (first index
// on ties).
#include "common.h"
#include "eig_body.h"
#include "internal.h"
#include "teig_body.h"

namespace sth {

template <bool ALDS, bool VLDS>
__global__ __launch_bounds__(EIG_THREADS) void jacobi_kernel(const double *__restrict__ S, int n,
                                                             int R, double *__restrict__ Ag,
                                                             double *__restrict__ Vg,
                                                             double *__restrict__ U,
                                                             double *__restrict__ lam, double tol,
                                                             int max_sweeps,
                                                             int64_t *__restrict__ flag) {
    jacobi_body<ALDS, VLDS>(S, n, R, Ag, Vg, U, lam, tol, max_sweeps, flag);
}

template <bool VLDS>
__global__ __launch_bounds__(EIG_THREADS) void jacobi_small_kernel(const double *__restrict__ S, int n,
                                                                   int R, double *__restrict__ Vg,
                                                                   double *__restrict__ U,
                                                                   double *__restrict__ lam, double tol,
                                                                   int max_sweeps,
                                                                   int64_t *__restrict__ flag) {
    jacobi_small_body<VLDS>(S, n, R, Vg, U, lam, tol, max_sweeps, flag);
}

// Sign rule on the columns of an n x R matrix: the entry of largest
// magnitude of each column is made positive (first index on ties).
__global__ void sign_fix_kernel(double *__restrict__ U, int n, int R) {
    const int r = blockIdx.x;
    __shared__ double s_v[256];
    __shared__ int s_i[256];
    double best = -1.0;
    int arg = 0;   // in range even when every entry is NaN (no comparison succeeds)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double v = fabs(U[i + (int64_t)n * r]);
        if (v > best) {
            best = v;
            arg = i;
        }
    }
    s_v[threadIdx.x] = best;
    s_i[threadIdx.x] = arg;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            double v2 = s_v[threadIdx.x + o];
            int i2 = s_i[threadIdx.x + o];
            if (v2 > s_v[threadIdx.x] || (v2 == s_v[threadIdx.x] && i2 < s_i[threadIdx.x])) {
                s_v[threadIdx.x] = v2;
                s_i[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const bool neg = U[s_i[0] + (int64_t)n * r] < 0.0;
    __syncthreads();
    if (neg)
        for (int i = threadIdx.x; i < n; i += blockDim.x) U[i + (int64_t)n * r] = -U[i + (int64_t)n * r];
}

template <bool ALDS, bool ZLDS>
__global__ __launch_bounds__(TE_T) void teig_kernel(const double *__restrict__ S, int64_t lds, int n, int R,
                                                   double *__restrict__ U, int64_t ldu,
                                                   double *__restrict__ lam, int sign_rule, TeScratch sc,
                                                   int64_t *__restrict__ flag, const double *__restrict__ chk,
                                                   double chk_tol, int64_t *__restrict__ count) {
    // gated on a residual test (chk): runs only when some chk[r] exceeds
    // chk_tol * chk[R] or is not finite; count records that it ran
    if (!gate_open(chk, R, chk_tol)) return;
    if (chk && count && threadIdx.x == 0) *count += 1;
    teig_body<ALDS, ZLDS>(S, lds, n, R, U, ldu, lam, sign_rule != 0, sc, flag);
}

// ---- subspace-iteration products: one 16 x 16 tile of C per workgroup on
// the FP64 matrix cores, the four waves splitting the contraction (steps of
// 4, four steps' loads issued together), their partial tiles summed in LDS
// in a fixed order.  Out-of-range rows and columns read clamped addresses
// and use zeros.  All take a gate (see gate_open).
constexpr int SI_T = 256;

// C (m x q) = A (m x k) B (k x q).  TRI_B: B upper triangular (k = q), so a
// tile of columns j0.. needs k < j0 + 16 only.  NS: C = 1.5 A - 0.5 A B, one
// Newton-Schulz step toward orthonormal columns (B = A^T A, k = q).
template <bool TRI_B, bool NS>
__global__ __launch_bounds__(SI_T) void si_nn_kernel(int m, int q, int k, const double *__restrict__ A, int64_t lda,
                                                    const double *__restrict__ B, int64_t ldb,
                                                    double *__restrict__ C, int64_t ldc,
                                                    const double *__restrict__ gate, int gate_R,
                                                    double gate_tol) {
    if (!gate_open(gate, gate_R, gate_tol)) return;
    __shared__ f64x4 s_acc[3][64];
    const int mt = (m + 15) >> 4;
    const int bi = blockIdx.x % mt, bj = blockIdx.x / mt;
    const int i0 = bi << 4, j0 = bj << 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tr = lane & 15, tg = lane >> 4;
    const int kmax = TRI_B ? min(k, j0 + 16) : k;
    const int ia = min(i0 + tr, m - 1), jb = min(j0 + tr, q - 1);
    const bool rok = i0 + tr < m, cok = j0 + tr < q;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = 4 * wave; 4 * s0 < kmax; s0 += 16) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = 4 * (s0 + u) + tg;
            const bool ok = kk < kmax;
            const int kc = ok ? kk : 0;
            a[u] = A[ia + lda * kc];
            b[u] = B[kc + ldb * jb];
            if (!(ok && rok)) a[u] = 0.0;
            if (!(ok && cok)) b[u] = 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
    if (wave > 0) s_acc[wave - 1][lane] = acc;
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < 3; ++w) acc += s_acc[w][lane];
        const int col = j0 + tr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = i0 + tg + 4 * v;
            if (row < m && col < q) {
                double c = acc[v];
                if (NS) c = 1.5 * A[row + lda * col] - 0.5 * c;
                C[row + ldc * col] = c;
            }
        }
    }
}

// C (p x q) = A^T B with A (k x p), B (k x q).  SYM: B = A, only the tiles
// on and below the diagonal are formed and each is written to both halves.
template <bool SYM>
__global__ __launch_bounds__(SI_T) void si_tn_kernel(int p, int q, int k, const double *__restrict__ A, int64_t lda,
                                                    const double *__restrict__ B, int64_t ldb,
                                                    double *__restrict__ C, int64_t ldc,
                                                    const double *__restrict__ gate, int gate_R,
                                                    double gate_tol) {
    if (!gate_open(gate, gate_R, gate_tol)) return;
    __shared__ f64x4 s_acc[3][64];
    int bi, bj;
    if (SYM) {
        const int t = blockIdx.x;
        bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
        bj = t - bi * (bi + 1) / 2;
    } else {
        const int pt = (p + 15) >> 4;
        bi = blockIdx.x % pt;
        bj = blockIdx.x / pt;
    }
    const int i0 = bi << 4, j0 = bj << 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tr = lane & 15, tg = lane >> 4;
    const int ia = min(i0 + tr, p - 1), jb = min(j0 + tr, q - 1);
    const bool rok = i0 + tr < p, cok = j0 + tr < q;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = 4 * wave; 4 * s0 < k; s0 += 16) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = 4 * (s0 + u) + tg;
            const bool ok = kk < k;
            const int kc = ok ? kk : 0;
            a[u] = A[kc + lda * ia];
            b[u] = B[kc + ldb * jb];
            if (!(ok && rok)) a[u] = 0.0;
            if (!(ok && cok)) b[u] = 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
    if (wave > 0) s_acc[wave - 1][lane] = acc;
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < 3; ++w) acc += s_acc[w][lane];
        const int col = j0 + tr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = i0 + tg + 4 * v;
            if (row < p && col < q) {
                C[row + ldc * col] = acc[v];
                if (SYM && bi != bj) C[col + ldc * row] = acc[v];
            }
        }
    }
}

// Rayleigh-Ritz finish, one workgroup per Ritz vector r:
//   U(:, r) = Q W(:, r), then the sign rule on it;
//   res[r] = ||Z W(:, r) - theta_r U(:, r)|| with Z = S Q (the Ritz residual);
//   lam[r] = theta_r; res[R] = |theta_1| (workgroup 0); res2 (may be null)
//   gets the same values.  Gated (see gate_open); gate must not be res.
__global__ __launch_bounds__(256) void rr_finish_kernel(const double *__restrict__ Q, const double *__restrict__ Zs,
                                                        int n, int p, const double *__restrict__ W,
                                                        const double *__restrict__ th, int R,
                                                        double *__restrict__ U, double *__restrict__ lam,
                                                        double *__restrict__ res, double *__restrict__ res2,
                                                        const double *__restrict__ gate, double gate_tol) {
    if (!gate_open(gate, R, gate_tol)) return;
    const int r = blockIdx.x, tid = threadIdx.x;
    __shared__ double s_w[SI_BLOCK_MAX];
    __shared__ double s_ss[4], s_bv[4], s_vv[4];
    __shared__ int s_bi[4];
    __shared__ double s_sign;
    for (int k = tid; k < p; k += 256) s_w[k] = W[k + (int64_t)p * r];
    __syncthreads();
    const double t = th[r];
    double ss = 0.0, best = -1.0, bval = 0.0;
    int arg = 0;
    for (int i = tid; i < n; i += 256) {
        double u = 0.0, z = 0.0;
        for (int k = 0; k < p; ++k) {
            u += Q[i + (int64_t)n * k] * s_w[k];
            z += Zs[i + (int64_t)n * k] * s_w[k];
        }
        const double d = z - t * u;
        ss += d * d;
        U[i + (int64_t)n * r] = u;
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
    if ((tid & 63) == 0) {
        s_ss[tid >> 6] = ss;
        s_bv[tid >> 6] = best;
        s_bi[tid >> 6] = arg;
        s_vv[tid >> 6] = bval;
    }
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0, b = s_bv[0], v = s_vv[0];
        int a = s_bi[0];
        for (int w = 0; w < 4; ++w) tot += s_ss[w];
        for (int w = 1; w < 4; ++w)
            if (s_bv[w] > b || (s_bv[w] == b && s_bi[w] < a)) {
                b = s_bv[w];
                a = s_bi[w];
                v = s_vv[w];
            }
        s_sign = v < 0.0 ? -1.0 : 1.0;
        res[r] = sqrt(tot);
        if (res2) res2[r] = res[r];
        if (lam) lam[r] = t;
        if (r == 0) {
            res[R] = fabs(t);
            if (res2) res2[R] = fabs(t);
        }
    }
    __syncthreads();
    if (s_sign < 0.0)
        for (int i = tid; i < n; i += 256) U[i + (int64_t)n * r] = -U[i + (int64_t)n * r];
}

namespace {

int64_t si_block(int64_t n, int64_t R) { return si_block_host(n, R); }

// The subspace iteration applies above order 128 when its block fits and
// leaves a guard (p < n) and R is within the Gram's rank bound.
bool use_si(int64_t n, int64_t R, int64_t rank_bound) {
    const int64_t p = si_block(n, R);
    return n > EIG_DIRECT_MAX && p <= SI_BLOCK_MAX && p < n && R <= rank_bound;
}

// residual test of the Ritz pairs: ||S u - theta u|| <= max(SI_RES_C sqrt(n) eps, u_S) |theta_1|
constexpr double SI_RES_C = 16.0;
// iterations of the first round: 2 when S carries single-precision rounding
// (u_S >= 2^-24: the test is that loose), 3 for FP64 data; the gated second
// round adds SI_ITERS_MORE
constexpr int SI_ITERS_LOOSE = 2, SI_ITERS_FP64 = 3, SI_ITERS_MORE = 2;

struct SiWs {
    double *Q, *Z, *Z2, *G, *Rinv, *T, *W, *th, *res, *res2;
    double *te;   // teig scratch of the p x p Rayleigh-Ritz problem
    double *fb;   // teig scratch of the direct solve of S (fallback)
};

size_t jacobi_ws(int64_t n) { return (size_t)(256 + 2 * n * n * sizeof(double)); }

SiWs si_layout(char *ws, int64_t n, int64_t p, int64_t R) {
    SiWs w;
    double *d = (double *)(ws + 256);
    w.Q = d; d += n * p;
    w.Z = d; d += n * p;
    w.Z2 = d; d += n * p;
    w.G = d; d += p * p;
    w.Rinv = d; d += p * p;
    w.T = d; d += p * p;
    w.W = d; d += p * p;
    w.th = d; d += p;
    w.res = d; d += p + 1;
    w.res2 = d; d += p + 1;
    w.te = d; d += teig_scratch_doubles(p, R, true);
    w.fb = d;
    return w;
}

size_t si_bytes(int64_t n, int64_t p, int64_t R) {
    return 256 + (size_t)(3 * n * p + 4 * p * p + 3 * p + 2) * 8 + teig_scratch_doubles(p, R, true) * 8 +
           teig_scratch_doubles(n, R, n <= TE_LDS_N) * 8 + 256;
}

size_t teig_bytes(int64_t n, int64_t R) { return 256 + teig_scratch_doubles(n, R, n <= TE_LDS_N) * 8; }

hipError_t si_nn(bool tri, bool ns, int m, int q, int k, const double *A, int64_t lda, const double *B, int64_t ldb,
                 double *C, int64_t ldc, const double *gate, int gR, double gtol, hipStream_t s) {
    const dim3 grid((unsigned)(((m + 15) / 16) * ((q + 15) / 16)));
    if (ns)
        hipLaunchKernelGGL((si_nn_kernel<false, true>), grid, dim3(SI_T), 0, s, m, q, k, A, lda, B, ldb, C, ldc,
                           gate, gR, gtol);
    else if (tri)
        hipLaunchKernelGGL((si_nn_kernel<true, false>), grid, dim3(SI_T), 0, s, m, q, k, A, lda, B, ldb, C, ldc,
                           gate, gR, gtol);
    else
        hipLaunchKernelGGL((si_nn_kernel<false, false>), grid, dim3(SI_T), 0, s, m, q, k, A, lda, B, ldb, C, ldc,
                           gate, gR, gtol);
    return hipGetLastError();
}

hipError_t si_tn(bool sym, int p, int q, int k, const double *A, int64_t lda, const double *B, int64_t ldb,
                 double *C, int64_t ldc, const double *gate, int gR, double gtol, hipStream_t s) {
    const int pt = (p + 15) / 16, qt = (q + 15) / 16;
    if (sym)
        hipLaunchKernelGGL((si_tn_kernel<true>), dim3((unsigned)(pt * (pt + 1) / 2)), dim3(SI_T), 0, s, p, q, k, A,
                           lda, B, ldb, C, ldc, gate, gR, gtol);
    else
        hipLaunchKernelGGL((si_tn_kernel<false>), dim3((unsigned)(pt * qt)), dim3(SI_T), 0, s, p, q, k, A, lda, B,
                           ldb, C, ldc, gate, gR, gtol);
    return hipGetLastError();
}

struct Gate {
    const double *res;
    int R;
    double tol;
};

// Cholesky-QR of the n x p matrix A into Q: G = A^T A (+ shift), G = R^T R,
// Q = A R^{-1}; shift_rel > 0 gives the shifted first pass of the shifted
// Cholesky-QR3 scheme (stable for condition numbers up to ~1/eps).
hipError_t cholqr_pass(const double *A, double *Q, int n, int p, double shift_rel, SiWs &w, int64_t *flag,
                       const Gate &g, hipStream_t s) {
    hipError_t e;
    if ((e = si_tn(true, p, p, n, A, n, A, n, w.G, p, g.res, g.R, g.tol, s))) return e;
    if ((e = chol_launch(w.G, p, p, shift_rel, nullptr, w.Rinv, flag, s, g.res, g.R, g.tol))) return e;
    return si_nn(true, false, n, p, p, A, n, w.Rinv, p, Q, n, g.res, g.R, g.tol, s);
}

enum OrthKind { ORTH_MID, ORTH_QR3, ORTH_NS };

// Orthonormalization of the iterate A (overwritten) into Q:
//   ORTH_MID: the shifted pass and one plain pass; the intermediate bases
//     only need to be well conditioned (the shifted pass alone leaves them
//     too ill-conditioned for the next product's orthonormalization);
//   ORTH_QR3: shifted Cholesky-QR3, orthonormal to working accuracy for
//     condition numbers up to ~1/eps;
//   ORTH_NS: the shifted pass, one plain pass and one Newton-Schulz step
//     (the two passes leave ||Q^T Q - I|| far below 1, the step squares it),
//     for Grams that carry single-precision rounding.
hipError_t orth(double *A, double *Q, int n, int p, OrthKind kind, SiWs &w, int64_t *flag, const Gate &g,
                hipStream_t s) {
    hipError_t e;
    const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * 1.1102230246251565e-16;
    if ((e = cholqr_pass(A, w.Z2, n, p, shift * p, w, flag, g, s))) return e;   // trace/p * p = trace
    if (kind == ORTH_MID) return cholqr_pass(w.Z2, Q, n, p, 0.0, w, flag, g, s);
    if ((e = cholqr_pass(w.Z2, A, n, p, 0.0, w, flag, g, s))) return e;
    if (kind == ORTH_QR3) return cholqr_pass(A, Q, n, p, 0.0, w, flag, g, s);
    if ((e = si_tn(true, p, p, n, A, n, A, n, w.G, p, g.res, g.R, g.tol, s))) return e;
    return si_nn(false, true, n, p, p, A, n, w.G, p, Q, n, g.res, g.R, g.tol, s);
}

hipError_t jacobi_launch(int64_t n, int64_t R, const double *S, double *U, double *lam, double tol,
                         int max_sweeps, void *ws, int64_t *flag, hipStream_t s) {
    double *Ag = (double *)((char *)ws + 256);
    double *Vg = Ag + n * n;
    const size_t mat = (size_t)n * n * sizeof(double);
    const size_t budget = EIG_LDS_AV;
    if (n <= 2 * JS_MAXM) {
        // A in LDS; V too when both fit (V in the workspace otherwise)
        const bool vl = jacobi_small_lds(n, true) <= budget;
        const size_t lds = jacobi_small_lds(n, vl);
        if (vl) {
            if (hipError_t ea = hipFuncSetAttribute((const void *)jacobi_small_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) return ea;
            hipLaunchKernelGGL(jacobi_small_kernel<true>, dim3(1), dim3(EIG_THREADS), lds, s, S, (int)n, (int)R, Ag, U, lam, tol, max_sweeps, flag);
        } else {
            if (hipError_t ea = hipFuncSetAttribute((const void *)jacobi_small_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) return ea;
            hipLaunchKernelGGL(jacobi_small_kernel<false>, dim3(1), dim3(EIG_THREADS), lds, s, S, (int)n, (int)R, Ag, U, lam, tol, max_sweeps, flag);
        }
    } else if (2 * mat <= budget) {
        auto k = jacobi_kernel<true, true>;
        if (hipError_t ea = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * mat))) return ea;
        hipLaunchKernelGGL(k, dim3(1), dim3(EIG_THREADS), 2 * mat, s, S, (int)n, (int)R, Ag, Vg, U, lam, tol, max_sweeps, flag);
    } else if (mat <= budget) {
        auto k = jacobi_kernel<true, false>;
        if (hipError_t ea = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mat)) return ea;
        hipLaunchKernelGGL(k, dim3(1), dim3(EIG_THREADS), mat, s, S, (int)n, (int)R, Ag, Vg, U, lam, tol, max_sweeps, flag);
    } else {
        hipLaunchKernelGGL((jacobi_kernel<false, false>), dim3(1), dim3(EIG_THREADS), 0, s, S, (int)n, (int)R, Ag, Vg, U, lam, tol, max_sweeps, flag);
    }
    return hipGetLastError();
}

template <bool ALDS, bool ZLDS>
hipError_t teig_go(const double *S, int64_t lds, int64_t n, int64_t R, double *U, int64_t ldu, double *lam,
                   bool sign_rule, TeScratch sc, int64_t *flag, const double *chk, double chk_tol, int64_t *count,
                   size_t lds_b, hipStream_t s) {
    auto k = teig_kernel<ALDS, ZLDS>;
    if (hipError_t ea = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_b))
        return ea;
    hipLaunchKernelGGL(k, dim3(1), dim3(TE_T), lds_b, s, S, lds, (int)n, (int)R, U, ldu, lam, sign_rule ? 1 : 0, sc,
                       flag, chk, chk_tol, count);
    return hipGetLastError();
}

}  // namespace

// Direct solver (teig_body.h) on the n x n matrix S: the matrix in LDS up to
// order TE_LDS_N, in the scratch above; scratch holds teig_bytes(n, R).
hipError_t teig_launch(const double *S, int64_t lds, int64_t n, int64_t R, double *U, int64_t ldu, double *lam,
                       bool sign_rule, void *scratch, int64_t *flag, const double *chk, double chk_tol,
                       int64_t *count, hipStream_t s) {
    const bool alds = n <= TE_LDS_N;
    const bool zlds = teig_z_fits(n, R, alds);
    const TeScratch sc = teig_scratch_layout((double *)scratch, n, R, alds);
    const size_t lb = teig_lds_bytes(n, R, alds, zlds, teig_v_keep(n, R, alds));
    if (alds) {
        return zlds ? teig_go<true, true>(S, lds, n, R, U, ldu, lam, sign_rule, sc, flag, chk, chk_tol, count, lb, s)
                    : teig_go<true, false>(S, lds, n, R, U, ldu, lam, sign_rule, sc, flag, chk, chk_tol, count, lb, s);
    }
    return zlds ? teig_go<false, true>(S, lds, n, R, U, ldu, lam, sign_rule, sc, flag, chk, chk_tol, count, lb, s)
                : teig_go<false, false>(S, lds, n, R, U, ldu, lam, sign_rule, sc, flag, chk, chk_tol, count, lb, s);
}

size_t eig_ws_bytes(int64_t n) {
    // every R <= n: the direct solver, the subspace iteration, or Jacobi
    size_t b = std::max(jacobi_ws(n), teig_bytes(n, n));
    for (int64_t R = 1; R <= n; ++R)
        if (use_si(n, R, n)) b = std::max(b, si_bytes(n, si_block(n, R), R));
    return b;
}

// R leading eigenpairs of the symmetric n x n matrix S (routes: see the top
// of this file).  jacobi_small: eig_leading's route for n <= 128 (Jacobi);
// otherwise the direct solver there.  rank_bound: rank(S) <= rank_bound (the
// subspace block is capped at it, and more vectors than that need the direct
// solver).  s_unit: unit roundoff of the products that formed S (0 when S is
// exact data).
hipError_t eig_launch(int64_t n, int64_t R, const double *S, double *U, double *lam, double tol,
                      int max_sweeps, void *ws, int64_t *flag, hipStream_t s, int64_t rank_bound,
                      bool jacobi_small, double s_unit) {
    if (n <= EIG_DIRECT_MAX) {
        if (jacobi_small) return jacobi_launch(n, R, S, U, lam, tol, max_sweeps, ws, flag, s);
        return teig_launch(S, n, n, R, U, n, lam, true, (char *)ws + 256, flag, nullptr, 0.0, nullptr, s);
    }
    if (!use_si(n, R, rank_bound))
        return teig_launch(S, n, n, R, U, n, lam, true, (char *)ws + 256, flag, nullptr, 0.0, nullptr, s);
    const int64_t p = std::min(si_block(n, R), rank_bound);
    SiWs w = si_layout((char *)ws, n, p, R);
    const int ni = (int)n, pi = (int)p, Ri = (int)R;
    hipError_t e;
    // start block: seeded Gaussian, used as it is (its span is all that
    // matters to the iteration, and an n x p Gaussian is well conditioned)
    if ((e = gaussian_f64(w.Q, n * p, 0x5EED5EEDull, (uint64_t)n * 1000 + p, s))) return e;
    // a Cholesky breakdown inside the iteration (S of rank below p) is not an
    // error of the result: it spoils the Ritz pairs, the residual test then
    // sends the solve on; it is recorded in flag[2] only.  flag[3] counts the
    // second rounds, flag[1] the direct solves of S.
    int64_t *si_flag = flag ? flag + 2 : nullptr;
    const bool loose = s_unit >= 0x1p-24;
    const double tol_res = std::max(SI_RES_C * std::sqrt((double)n) * 2.220446049250313e-16, s_unit);
    // round 0 runs always; round 1 continues from round 0's basis only when
    // a Ritz residual of round 0 fails the test (every launch gated on it)
    for (int round = 0; round < 2; ++round) {
        const Gate g = {round ? w.res : nullptr, Ri, tol_res};
        const int iters = round ? SI_ITERS_MORE : (loose ? SI_ITERS_LOOSE : SI_ITERS_FP64);
        for (int it = 0; it < iters; ++it) {
            if ((e = si_nn(false, false, ni, pi, ni, S, n, w.Q, n, w.Z, n, g.res, g.R, g.tol, s))) return e;
            const OrthKind kind = it + 1 < iters ? ORTH_MID : (loose ? ORTH_NS : ORTH_QR3);
            if ((e = orth(w.Z, w.Q, ni, pi, kind, w, si_flag, g, s))) return e;
        }
        // Rayleigh-Ritz: T = Q^T S Q, its R leading pairs (W, theta), U = Q W
        if ((e = si_nn(false, false, ni, pi, ni, S, n, w.Q, n, w.Z, n, g.res, g.R, g.tol, s))) return e;
        if ((e = si_tn(false, pi, pi, ni, w.Q, n, w.Z, n, w.T, p, g.res, g.R, g.tol, s))) return e;
        if ((e = teig_launch(w.T, p, p, R, w.W, p, w.th, false, w.te, si_flag, g.res, g.tol,
                             round && flag ? flag + 3 : nullptr, s)))
            return e;
        hipLaunchKernelGGL(rr_finish_kernel, dim3((unsigned)R), dim3(256), 0, s, w.Q, w.Z, ni, pi, w.W, w.th, Ri, U,
                           lam, round ? w.res2 : w.res, round ? nullptr : w.res2, g.res, g.tol);
        if ((e = hipGetLastError())) return e;
    }
    // the direct solver on S when the last round's Ritz pairs fail the test
    return teig_launch(S, n, n, R, U, n, lam, true, w.fb, flag, w.res2, tol_res, flag ? flag + 1 : nullptr, s);
}

}  // namespace sth
