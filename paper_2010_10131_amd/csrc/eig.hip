// FP64 symmetric eigensolver for the EIG branch of Alg. 2: the R_n leading
// eigenvectors of the mode-n Gram matrix.
//
// Two-sided cyclic Jacobi with a parallel (round-robin tournament) ordering,
// run by one 1024-thread workgroup.  In every round the n/2 disjoint
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
#include "internal.h"

namespace sth {

constexpr int EIG_THREADS = 256;

__device__ __forceinline__ int rr_player(int x, int r, int ne) {
    // round-robin position x (0..ne-1) in round r (0..ne-2): player 0 fixed
    if (x == 0) return 0;
    int y = x - 1 + r;
    if (y >= ne - 1) y -= ne - 1;
    return y + 1;
}

template <bool ALDS, bool VLDS>
__global__ __launch_bounds__(EIG_THREADS) void jacobi_kernel(const double *__restrict__ S, int n,
                                                             int R, double *__restrict__ Ag,
                                                             double *__restrict__ Vg,
                                                             double *__restrict__ U,
                                                             double *__restrict__ lam, double tol,
                                                             int max_sweeps,
                                                             int64_t *__restrict__ flag) {
    extern __shared__ double s_e[];
    __shared__ double s_c[256], s_s[256];
    __shared__ int s_p[256], s_q[256];
    __shared__ double s_red[2][EIG_THREADS / 64];
    __shared__ int s_sel[512];
    __shared__ double s_sign[512];
    __shared__ int s_stop;

    double *A = ALDS ? s_e : Ag;
    double *V = VLDS ? (ALDS ? s_e + n * n : s_e) : Vg;
    const int tid = threadIdx.x;
    const int nn = n * n;
    for (int e = tid; e < nn; e += EIG_THREADS) {
        const int i = e % n, j = e / n;
        A[e] = 0.5 * (S[e] + S[j + n * i]);
        V[e] = (i == j) ? 1.0 : 0.0;
    }
    const int ne = n + (n & 1);
    const int m = ne / 2;
    __syncthreads();

    int sweep = 0;
    bool converged = false;
    double prev_off2 = -1.0;
    for (;;) {
        // convergence test: off(A)^2 <= tol^2 ||A||_F^2
        double off = 0.0, fro = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = tid; i < n; i += EIG_THREADS) {
                const double v = A[i + n * j];
                fro += v * v;
                if (i != j) off += v * v;
            }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            fro += __shfl_xor(fro, o);
        }
        if ((tid & 63) == 0) {
            s_red[0][tid >> 6] = off;
            s_red[1][tid >> 6] = fro;
        }
        __syncthreads();
        if (tid == 0) {
            double o2 = 0.0, f2 = 0.0;
            for (int w = 0; w < EIG_THREADS / 64; ++w) {
                o2 += s_red[0][w];
                f2 += s_red[1][w];
            }
            int stop = 0;
            if (o2 <= tol * tol * f2 || o2 == 0.0) stop = 1;
            // roundoff floor: off(A) already at the FP64 noise level of an
            // n x n rotation sequence and no longer shrinking
            else if (o2 <= (double)n * n * 1.2e-32 * f2 && prev_off2 >= 0.0 && o2 >= 0.25 * prev_off2) stop = 1;
            else if (sweep >= max_sweeps) stop = 2;
            s_stop = stop;
            s_red[0][0] = o2;  // broadcast for the stagnation test
        }
        __syncthreads();
        if (s_stop) {
            converged = (s_stop == 1);
            break;
        }
        prev_off2 = s_red[0][0];
        for (int r = 0; r < ne - 1; ++r) {
            // rotations of this round
            for (int k = tid; k < m; k += EIG_THREADS) {
                int p = rr_player(k, r, ne), q = rr_player(ne - 1 - k, r, ne);
                if (p > q) {
                    int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    double apq = A[p + n * q];
                    if (apq != 0.0) {
                        double app = A[p + n * p], aqq = A[q + n * q];
                        double theta = (aqq - app) / (2.0 * apq);
                        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                s_p[k] = p;
                s_q[k] = q;
                s_c[k] = c;
                s_s[k] = s;
            }
            __syncthreads();
            // A <- J^T A J, block (I, J) of pairs; V <- V J
            const int nb = m * m;
            int I = tid % m, J = tid / m;
            const int dI = EIG_THREADS % m, dJ = EIG_THREADS / m;
            for (int e = tid; e < nb; e += EIG_THREADS) {
                const int pi = s_p[I], qi = s_q[I], pj = s_p[J], qj = s_q[J];
                const double ci = s_c[I], si = s_s[I], cj = s_c[J], sj = s_s[J];
                const bool vi = qi < n, vj = qj < n;  // pair contains the dummy player?
                // rows {pi, qi} (qi may be the dummy), cols {pj, qj}
                double a00 = A[pi + n * pj];
                double a01 = vj ? A[pi + n * qj] : 0.0;
                double a10 = vi ? A[qi + n * pj] : 0.0;
                double a11 = (vi && vj) ? A[qi + n * qj] : 0.0;
                // left: rows' = [c -s; s c]^T-rotation as in the oracle: row p' = c p - s q, row q' = s p + c q
                double b00 = ci * a00 - si * a10, b01 = ci * a01 - si * a11;
                double b10 = si * a00 + ci * a10, b11 = si * a01 + ci * a11;
                // right: col p' = c p - s q, col q' = s p + c q
                double d00 = cj * b00 - sj * b01, d01 = sj * b00 + cj * b01;
                double d10 = cj * b10 - sj * b11, d11 = sj * b10 + cj * b11;
                A[pi + n * pj] = d00;
                if (vj) A[pi + n * qj] = d01;
                if (vi) A[qi + n * pj] = d10;
                if (vi && vj) A[qi + n * qj] = d11;
                I += dI;
                J += dJ;
                if (I >= m) {
                    I -= m;
                    ++J;
                }
            }
            const int nv = n * m;
            int row = tid % n, Jv = tid / n;
            const int dr = EIG_THREADS % n, dJv = EIG_THREADS / n;
            for (int e = tid; e < nv; e += EIG_THREADS) {
                const int pj = s_p[Jv], qj = s_q[Jv];
                if (qj < n) {
                    const double cj = s_c[Jv], sj = s_s[Jv];
                    double vp = V[row + n * pj], vq = V[row + n * qj];
                    V[row + n * pj] = cj * vp - sj * vq;
                    V[row + n * qj] = sj * vp + cj * vq;
                }
                row += dr;
                Jv += dJv;
                if (row >= n) {
                    row -= n;
                    ++Jv;
                }
            }
            __syncthreads();
        }
        ++sweep;
    }
    if (!converged && tid == 0 && flag) flag[0] = 1;

    // descending order of the diagonal, ties by index
    for (int i = tid; i < n; i += EIG_THREADS) {
        const double li = A[i + n * i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j + n * j];
            rank += (lj > li) || (lj == li && j < i);
        }
        if (rank < R) s_sel[rank] = i;
    }
    __syncthreads();
    for (int r = tid; r < R; r += EIG_THREADS) {
        const int col = s_sel[r];
        int arg = 0;
        double best = fabs(V[n * col]);
        for (int i = 1; i < n; ++i) {
            double v = fabs(V[i + n * col]);
            if (v > best) {
                best = v;
                arg = i;
            }
        }
        s_sign[r] = V[arg + n * col] < 0 ? -1.0 : 1.0;
        if (lam) lam[r] = A[col + n * col];
    }
    __syncthreads();
    const int nr = n * R;
    for (int e = tid; e < nr; e += EIG_THREADS) {
        const int i = e % n, r = e / n;
        U[e] = s_sign[r] * V[i + n * s_sel[r]];
    }
}

// Sign rule on the columns of an n x R matrix: the entry of largest
// magnitude of each column is made positive (first index on ties).
__global__ void sign_fix_kernel(double *__restrict__ U, int n, int R) {
    const int r = blockIdx.x;
    __shared__ double s_v[256];
    __shared__ int s_i[256];
    double best = -1.0;
    int arg = n;
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

constexpr int64_t EIG_DIRECT_MAX = 128;  // Jacobi on the whole matrix up to this order
constexpr int64_t SI_BLOCK_MAX = 96;     // Rayleigh-Ritz block kept in LDS (A and V)
constexpr int SI_ITERS = 6;              // subspace iterations before Rayleigh-Ritz

int64_t si_block(int64_t n, int64_t R) {
    int64_t p = std::max<int64_t>(R + 16, (3 * R + 1) / 2);
    p = (p + 7) / 8 * 8;
    return std::min(p, n);
}

bool use_si(int64_t n, int64_t R) { return n > EIG_DIRECT_MAX && si_block(n, R) <= SI_BLOCK_MAX; }

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
    w.jac = (char *)d;
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

hipError_t orth3(double *A, double *Q, int n, int p, SiWs &w, int64_t *flag, hipStream_t s) {
    hipError_t e;
    const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * 1.1102230246251565e-16;
    if ((e = cholqr_pass(A, w.Z2, n, p, shift * p, w, flag, s))) return e;   // trace/p * p = trace
    if ((e = cholqr_pass(w.Z2, A, n, p, 0.0, w, flag, s))) return e;
    return cholqr_pass(A, Q, n, p, 0.0, w, flag, s);
}

hipError_t jacobi_launch(int64_t n, int64_t R, const double *S, double *U, double *lam, double tol,
                         int max_sweeps, void *ws, int64_t *flag, hipStream_t s) {
    double *Ag = (double *)((char *)ws + 256);
    double *Vg = Ag + n * n;
    const size_t mat = (size_t)n * n * sizeof(double);
    const size_t budget = 150 * 1024;
    if (2 * mat <= budget) {
        auto k = jacobi_kernel<true, true>;
        hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * mat));
        hipLaunchKernelGGL(k, dim3(1), dim3(EIG_THREADS), 2 * mat, s, S, (int)n, (int)R, Ag, Vg, U, lam, tol, max_sweeps, flag);
    } else if (mat <= budget) {
        auto k = jacobi_kernel<true, false>;
        hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mat);
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
        if (use_si(n, R)) b = std::max(b, si_bytes(n, si_block(n, R)));
    return b;
}

// R leading eigenpairs of the symmetric n x n matrix S.
//   n <= 128: cyclic Jacobi on S itself (one workgroup, LDS).
//   n > 128 with a block p = max(R + 16, 1.5 R) <= 96: subspace iteration
//     Q <- orth(S Q) from a seeded Gaussian block (SI_ITERS times; orth is
//     shifted Cholesky-QR3), then Rayleigh-Ritz: Jacobi on T = Q^T S Q and
//     U = Q W(:, :R), with the sign rule applied to U.
//   otherwise: Jacobi on S with A and V in the workspace (slow; large R only).
hipError_t eig_launch(int64_t n, int64_t R, const double *S, double *U, double *lam, double tol,
                      int max_sweeps, void *ws, int64_t *flag, hipStream_t s) {
    if (!use_si(n, R)) return jacobi_launch(n, R, S, U, lam, tol, max_sweeps, ws, flag, s);
    const int64_t p = si_block(n, R);
    SiWs w = si_layout((char *)ws, n, p);
    const int ni = (int)n, pi = (int)p;
    hipError_t e;
    if ((e = gaussian_f64(w.Z, n * p, 0x5EED5EEDull, (uint64_t)n * 1000 + p, s))) return e;
    if ((e = orth3(w.Z, w.Q, ni, pi, w, flag, s))) return e;
    for (int it = 0; it < SI_ITERS; ++it) {
        if ((e = gemm_f64(0, 0, ni, pi, ni, 1.0, S, n, w.Q, n, 0.0, w.Z, n, w.gws, s))) return e;
        if ((e = orth3(w.Z, w.Q, ni, pi, w, flag, s))) return e;
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
