// FP64 symmetric eigensolver for the EIG branch of Alg. 2: the R_n leading
// eigenvectors of the mode-n Gram matrix.
//
// Two-sided cyclic Jacobi with a parallel (round-robin tournament) ordering,
// run by one 512-thread workgroup.  In every round the n/2 disjoint
// rotations are computed first; then A <- J^T A J is applied block-wise
// (each thread transforms whole 2x2 blocks (pair I, pair J), which are
// independent within a round) and V <- V J.  After each sweep the
// off-diagonal mass is measured and the iteration stops when
// off(A) <= tol * ||A||_F.  A and V live in LDS when they fit and in the
// workspace otherwise.
//
// Selection: eigenvalues sorted in descending order (ties by index), the R
// leading eigenvectors signed so that their entry of largest magnitude is
// positive (first index on ties).
#include "common.h"
#include "eig_body.h"
#include "internal.h"

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

namespace {

constexpr int SI_ITERS = SI_ITERS_DEV;
int64_t si_block(int64_t n, int64_t R) { return si_block_host(n, R); }

// si_min: the order above which the subspace iteration may be used
bool use_si(int64_t n, int64_t R, int64_t si_min) {
    const int64_t p = si_block(n, R);
    return n > si_min && p <= SI_BLOCK_MAX && p < n && (n > EIG_LDS_DIRECT_MAX || 2 * p <= n);
}

struct SiWs {
    double *Q, *Z, *Z2, *G, *Rf, *Rinv, *T, *W, *gws;
    char *jac;
};

size_t jacobi_ws(int64_t n) { return (size_t)(256 + 2 * n * n * sizeof(double)); }

SiWs si_layout(char *ws, int64_t n, int64_t p) {
    SiWs w;
    double *d = (double *)(ws + 256);
    w.Q = d; d += n * p;
    w.Z = d; d += n * p;
    w.Z2 = d; d += n * p;
    w.G = d; d += p * p;
    w.Rf = d; d += p * p;
    w.Rinv = d; d += p * p;
    w.T = d; d += p * p;
    w.W = d; d += p * p;
    w.gws = d; d += std::max<size_t>(gemm_ws_bytes((int)p, (int)p, (int)n), gemm_ws_bytes((int)n, (int)p, (int)n)) / 8 + 1;
    w.jac = (char *)(((uintptr_t)d + 255) & ~(uintptr_t)255);   // 16-byte accesses in the Jacobi
    return w;
}

size_t si_bytes(int64_t n, int64_t p) {
    return 256 + (size_t)(3 * n * p + 5 * p * p) * 8 +
           std::max<size_t>(gemm_ws_bytes((int)p, (int)p, (int)n), gemm_ws_bytes((int)n, (int)p, (int)n)) + 8 +
           jacobi_ws(p) + 256;
}

// Cholesky-QR of the n x p matrix A into Q; shift_rel > 0 gives the shifted
// first pass of the shifted Cholesky-QR3 scheme (stable for condition numbers
// up to ~1/eps).
hipError_t cholqr_pass(const double *A, double *Q, int n, int p, double shift_rel, SiWs &w,
                       int64_t *flag, hipStream_t s) {
    hipError_t e;
    if ((e = gemm_f64(1, 0, p, p, n, 1.0, A, n, A, n, 0.0, w.G, p, w.gws, s))) return e;
    if ((e = chol_launch(w.G, p, p, shift_rel, nullptr, w.Rinv, flag, s))) return e;
    return gemm_f64(0, 0, n, p, p, 1.0, A, n, w.Rinv, p, 0.0, Q, n, w.gws, s);
}

// passes = 3: shifted Cholesky-QR3 (orthonormal to working accuracy for
// condition numbers up to ~1/eps); passes = 2: the shifted pass and one plain
// pass, enough for the intermediate bases of the subspace iteration, which
// only need to be well conditioned (the shifted pass alone leaves them too
// ill-conditioned for the next product's orthonormalization).
hipError_t orth(double *A, double *Q, int n, int p, int passes, SiWs &w, int64_t *flag, hipStream_t s) {
    hipError_t e;
    const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * 1.1102230246251565e-16;
    if ((e = cholqr_pass(A, w.Z2, n, p, shift * p, w, flag, s))) return e;   // trace/p * p = trace
    if (passes == 2) return cholqr_pass(w.Z2, Q, n, p, 0.0, w, flag, s);
    if ((e = cholqr_pass(w.Z2, A, n, p, 0.0, w, flag, s))) return e;
    return cholqr_pass(A, Q, n, p, 0.0, w, flag, s);
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

}  // namespace

size_t eig_ws_bytes(int64_t n) {
    size_t b = jacobi_ws(n);
    // subspace iteration for any R that selects it
    for (int64_t R = 1; R <= n; ++R)
        if (use_si(n, R, EIG_SI_MIN)) b = std::max(b, si_bytes(n, si_block(n, R)));
    return b;
}

// R leading eigenpairs of the symmetric n x n matrix S.
//   n <= si_min (128 for eig_leading, 96 for the decompositions, which need
//   the leading subspace only): cyclic Jacobi on S itself (one workgroup,
//   LDS; V in the workspace above order 96).
//   n > si_min with a block p = R + 16 (rounded up to 8) <= 96, p < n: subspace iteration
//     Q <- orth(S Q) from a seeded Gaussian block (SI_ITERS = 3 times; orth is
//     shifted Cholesky-QR, three passes for the last basis, two before), then
//     Rayleigh-Ritz: Jacobi on T = Q^T S Q and U = Q W(:, :R), with the sign
//     rule applied to U.
//   otherwise (large R, or R above the rank bound of S): Jacobi on S with A
//   and V in the workspace.
hipError_t eig_launch(int64_t n, int64_t R, const double *S, double *U, double *lam, double tol,
                      int max_sweeps, void *ws, int64_t *flag, hipStream_t s, int64_t rank_bound,
                      int64_t si_min) {
    // rank(S) <= rank_bound: a block wider than that would be rank deficient
    // (Cholesky-QR breaks down), so the block shrinks to the bound, and a
    // request of more than rank_bound vectors goes to the direct solver
    if (!use_si(n, R, si_min) || R > rank_bound) return jacobi_launch(n, R, S, U, lam, tol, max_sweeps, ws, flag, s);
    const int64_t p = std::min(si_block(n, R), rank_bound);
    SiWs w = si_layout((char *)ws, n, p);
    const int ni = (int)n, pi = (int)p;
    hipError_t e;
    // start block: seeded Gaussian, used as it is (its span is all that
    // matters to the iteration, and an n x p Gaussian is well conditioned)
    if ((e = gaussian_f64(w.Q, n * p, 0x5EED5EEDull, (uint64_t)n * 1000 + p, s))) return e;
    for (int it = 0; it < SI_ITERS; ++it) {
        if ((e = gemm_f64(0, 0, ni, pi, ni, 1.0, S, n, w.Q, n, 0.0, w.Z, n, w.gws, s))) return e;
        if ((e = orth(w.Z, w.Q, ni, pi, it + 1 == SI_ITERS ? 3 : 2, w, flag, s))) return e;
    }
    // Rayleigh-Ritz
    if ((e = gemm_f64(0, 0, ni, pi, ni, 1.0, S, n, w.Q, n, 0.0, w.Z, n, w.gws, s))) return e;
    if ((e = gemm_f64(1, 0, pi, pi, ni, 1.0, w.Q, n, w.Z, n, 0.0, w.T, p, w.gws, s))) return e;
    if ((e = jacobi_launch(p, R, w.T, w.W, lam, tol, max_sweeps, w.jac, flag, s))) return e;
    if ((e = gemm_f64(0, 0, ni, (int)R, pi, 1.0, w.Q, n, w.W, p, 0.0, U, n, w.gws, s))) return e;
    hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)R), dim3(256), 0, s, U, ni, (int)R);
    return hipGetLastError();
}

}  // namespace sth
