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

constexpr int EIG_THREADS = 1024;

__device__ __forceinline__ int rr_player(int x, int r, int ne) {
    // round-robin position x (0..ne-1) in round r: player 0 fixed
    return x == 0 ? 0 : ((x - 1 + r) % (ne - 1)) + 1;
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
        A[e] = S[e];
        V[e] = ((e % n) == (e / n)) ? 1.0 : 0.0;
    }
    const int ne = n + (n & 1);
    const int m = ne / 2;
    __syncthreads();

    int sweep = 0;
    bool converged = false;
    for (;;) {
        // convergence test: off(A)^2 <= tol^2 ||A||_F^2
        double off = 0.0, fro = 0.0;
        for (int e = tid; e < nn; e += EIG_THREADS) {
            double v = A[e];
            fro += v * v;
            if ((e % n) != (e / n)) off += v * v;
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
            else if (sweep >= max_sweeps) stop = 2;
            s_stop = stop;
        }
        __syncthreads();
        if (s_stop) {
            converged = (s_stop == 1);
            break;
        }
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
            for (int e = tid; e < nb; e += EIG_THREADS) {
                const int I = e % m, J = e / m;
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
            }
            const int nv = n * m;
            for (int e = tid; e < nv; e += EIG_THREADS) {
                const int row = e % n, J = e / n;
                const int pj = s_p[J], qj = s_q[J];
                if (qj >= n) continue;
                const double cj = s_c[J], sj = s_s[J];
                double vp = V[row + n * pj], vq = V[row + n * qj];
                V[row + n * pj] = cj * vp - sj * vq;
                V[row + n * qj] = sj * vp + cj * vq;
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

size_t eig_ws_bytes(int64_t n) { return (size_t)(8 + 2 * n * n * sizeof(double) + 256); }

hipError_t eig_launch(int64_t n, int64_t R, const double *S, double *U, double *lam, double tol,
                      int max_sweeps, void *ws, hipStream_t s) {
    int64_t *flag = (int64_t *)ws;
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

}  // namespace sth
