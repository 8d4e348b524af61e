/*
 * Plain FP64 CPU oracle for sequentially truncated HOSVD (st-HOSVD).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * Every routine is the plain definition of the operation it names, written
 * with explicit matricization and triple loops, in double precision:
 *   - mode-n matricization / tensorization      (Sec. II-A, Fig. 3)
 *   - Frobenius norm                            (Sec. II-A, Eq. 1)
 *   - TTM, y = x  x_n  U                        (Sec. II-A, Eq. 2)
 *   - TTT / Gram  Z = X_(n) Y_(n)^T             (Sec. II-A, Eq. 3; Gram = TTT(X, X))
 *   - cyclic Jacobi symmetric eigensolver       (leading eigenvectors, Alg. 2 EIG branch)
 *   - Householder QR, Cholesky solves           (Alg. 2 ALS branch, Alg. 3)
 *   - st-HOSVD with per-mode EIG / ALS choice   (Alg. 2, Alg. 3)
 *   - Tucker reconstruction                     (Sec. II-B)
 *   - a small dense MLP forward/backward        (solver-selector cost model)
 *
 * Layout: every tensor is column-major, the first index fastest
 * (Sec. II-A, Sec. V).  Matrices are column-major, A[i + rows*j].
 *
 * Readings of the paper that this file adopts (the paper is silent or
 * ambiguous there):
 *   - column order of X_(n): lower modes vary fastest (Kolda order); Gram
 *     and TTM do not depend on it;
 *   - "leading" eigenvectors: eigenvalues sorted in descending order; each
 *     eigenvector is signed so that its entry of largest magnitude is
 *     positive (first such index on ties);
 *   - Eq. 2 takes U as R_n x I_n, factors are I_n x R_n: the core update
 *     applies the transpose of the I_n x R_n factor;
 *   - ALS (Alg. 3): a fixed number of sweeps; the returned pair is the last
 *     computed (L_k, R_{k-1}), so the core update is R^ R_{k-1}^T.  The
 *     "ortho" variant re-orthonormalizes L_k by QR before each sweep, which
 *     spans the same subspaces in exact arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

/* ------------------------------------------------------------------ */
/* threads                                                             */
/* ------------------------------------------------------------------ */

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* shapes and matricization (Sec. II-A)                                */
/* ------------------------------------------------------------------ */

i64 orc_numel(int N, const i64 *dims) {
    i64 p = 1;
    for (int k = 0; k < N; ++k) p *= dims[k];
    return p;
}

/* Mode-n unfolding: Yn is I_n x J_n, column index in Kolda order
 * j = sum_{m != n} i_m * prod_{k < m, k != n} I_k. */
void orc_unfold(int N, const i64 *dims, int n, const double *X, double *Yn) {
    i64 total = orc_numel(N, dims);
    i64 In = dims[n];
#pragma omp parallel for schedule(static)
    for (i64 lin = 0; lin < total; ++lin) {
        i64 rem = lin, col = 0, stride = 1, in = 0;
        for (int m = 0; m < N; ++m) {
            i64 im = rem % dims[m];
            rem /= dims[m];
            if (m == n) {
                in = im;
            } else {
                col += im * stride;
                stride *= dims[m];
            }
        }
        Yn[in + In * col] = X[lin];
    }
}

/* Inverse of orc_unfold (tensorization). */
void orc_fold(int N, const i64 *dims, int n, const double *Yn, double *X) {
    i64 total = orc_numel(N, dims);
    i64 In = dims[n];
#pragma omp parallel for schedule(static)
    for (i64 lin = 0; lin < total; ++lin) {
        i64 rem = lin, col = 0, stride = 1, in = 0;
        for (int m = 0; m < N; ++m) {
            i64 im = rem % dims[m];
            rem /= dims[m];
            if (m == n) {
                in = im;
            } else {
                col += im * stride;
                stride *= dims[m];
            }
        }
        X[lin] = Yn[in + In * col];
    }
}

/* Eq. 1: sum of squares (the square of the Frobenius norm). */
double orc_sumsq(i64 n, const double *x) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (i64 i = 0; i < n; ++i) s += x[i] * x[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* dense products                                                      */
/* ------------------------------------------------------------------ */

/* C (m x n) = A^T B with A (k x m), B (k x n), all column-major. */
void orc_matmul_tn(i64 m, i64 n, i64 k, const double *A, const double *B, double *C) {
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 j = 0; j < n; ++j)
        for (i64 i = 0; i < m; ++i) {
            double s = 0.0;
            for (i64 p = 0; p < k; ++p) s += A[p + k * i] * B[p + k * j];
            C[i + m * j] = s;
        }
}

/* C (m x n) = A B with A (m x k), B (k x n). */
void orc_matmul_nn(i64 m, i64 n, i64 k, const double *A, const double *B, double *C) {
    /* each C(i, j) is summed over p in increasing order; the loops are
     * interchanged only so that columns of A and C are walked contiguously */
#pragma omp parallel for schedule(static)
    for (i64 j = 0; j < n; ++j) {
        double *c = C + m * j;
        for (i64 i = 0; i < m; ++i) c[i] = 0.0;
        for (i64 p = 0; p < k; ++p) {
            const double b = B[p + k * j];
            const double *a = A + m * p;
            for (i64 i = 0; i < m; ++i) c[i] += a[i] * b;
        }
    }
}

/* C (m x n) = A B^T with A (m x k), B (n x k). */
void orc_matmul_nt(i64 m, i64 n, i64 k, const double *A, const double *B, double *C) {
    /* each C(i, j) is summed over p in increasing order (loop interchange as
     * in orc_matmul_nn) */
#pragma omp parallel for schedule(static)
    for (i64 j = 0; j < n; ++j) {
        double *c = C + m * j;
        for (i64 i = 0; i < m; ++i) c[i] = 0.0;
        for (i64 p = 0; p < k; ++p) {
            const double b = B[j + n * p];
            const double *a = A + m * p;
            for (i64 i = 0; i < m; ++i) c[i] += a[i] * b;
        }
    }
}

/* Gram S = Yn Yn^T of an I x J matrix (Alg. 2 EIG branch; Gram = TTT(Y, Y)). */
void orc_gram(i64 I, i64 J, const double *Yn, double *S) {
    orc_matmul_nt(I, I, J, Yn, Yn, S);
}

/* TTT (Eq. 3) in matricized form: Z (I x R) = X_(n) Y_(n)^T, with X_(n) I x J
 * and Y_(n) R x J. */
void orc_ttt(i64 I, i64 R, i64 J, const double *Xn, const double *Yn, double *Z) {
    orc_matmul_nt(I, R, J, Xn, Yn, Z);
}

/* Eq. 2 in matricized form with the transpose of an I x R factor:
 * out (R x J) = U^T Yn. */
void orc_ttm_t(i64 I, i64 R, i64 J, const double *U, const double *Yn, double *out) {
    orc_matmul_tn(R, J, I, U, Yn, out);
}

/* Tensor-level TTM, y = x  x_n  A with A given as (rows x I_n):
 * out has dims[n] replaced by rows.  Explicit unfold -> GEMM -> fold. */
int orc_ttm_tensor(int N, const i64 *dims, int n, i64 rows, const double *A,
                   const double *X, double *out) {
    i64 In = dims[n];
    i64 total = orc_numel(N, dims);
    i64 J = total / In;
    double *Xn = (double *)malloc(sizeof(double) * (size_t)total);
    double *On = (double *)malloc(sizeof(double) * (size_t)(rows * J));
    if (!Xn || !On) {
        free(Xn);
        free(On);
        return -1;
    }
    orc_unfold(N, dims, n, X, Xn);
    orc_matmul_nn(rows, J, In, A, Xn, On);
    i64 odims[16];
    for (int m = 0; m < N; ++m) odims[m] = dims[m];
    odims[n] = rows;
    orc_fold(N, odims, n, On, out);
    free(Xn);
    free(On);
    return 0;
}

/* ------------------------------------------------------------------ */
/* cyclic Jacobi eigensolver (symmetric, FP64)                         */
/* ------------------------------------------------------------------ */

/* Sorts (lam, V) by descending eigenvalue and applies the sign rule:
 * the entry of largest magnitude of each column is positive (first index
 * on ties). */
static void sort_and_sign(i64 n, double *lam, double *V) {
    /* selection sort, n is small */
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    for (i64 a = 0; a < n; ++a) {
        i64 best = a;
        for (i64 b = a + 1; b < n; ++b)
            if (lam[b] > lam[best]) best = b;
        if (best != a) {
            double t = lam[a];
            lam[a] = lam[best];
            lam[best] = t;
            memcpy(tmp, V + n * a, sizeof(double) * (size_t)n);
            memcpy(V + n * a, V + n * best, sizeof(double) * (size_t)n);
            memcpy(V + n * best, tmp, sizeof(double) * (size_t)n);
        }
    }
    free(tmp);
    for (i64 c = 0; c < n; ++c) {
        double *v = V + n * c;
        i64 arg = 0;
        for (i64 i = 1; i < n; ++i)
            if (fabs(v[i]) > fabs(v[arg])) arg = i;
        if (v[arg] < 0)
            for (i64 i = 0; i < n; ++i) v[i] = -v[i];
    }
}

/* Two-sided cyclic Jacobi (row-cyclic order) on a symmetric n x n matrix.
 * The input S is not modified.  On return lam holds the eigenvalues in
 * descending order and V (n x n) the matching orthonormal eigenvectors.
 * Stops when off(A) <= tol * ||A||_F or after max_sweeps sweeps.
 * Returns the number of sweeps taken, or -1 if the cap was hit. */
int orc_jacobi_eig(i64 n, const double *S, double *lam, double *V, double tol,
                   int max_sweeps) {
    double *A = (double *)malloc(sizeof(double) * (size_t)(n * n));
    memcpy(A, S, sizeof(double) * (size_t)(n * n));
    for (i64 j = 0; j < n; ++j)
        for (i64 i = 0; i < n; ++i) V[i + n * j] = (i == j) ? 1.0 : 0.0;
    double fro2 = 0.0;
    for (i64 k = 0; k < n * n; ++k) fro2 += A[k] * A[k];
    int sweep = 0, converged = 0;
    for (; sweep <= max_sweeps; ++sweep) {
        double off2 = 0.0;
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i)
                if (i != j) off2 += A[i + n * j] * A[i + n * j];
        if (off2 <= tol * tol * fro2 || off2 == 0.0) {
            converged = 1;
            break;
        }
        if (sweep == max_sweeps) break;
        for (i64 p = 0; p < n - 1; ++p) {
            for (i64 q = p + 1; q < n; ++q) {
                double apq = A[p + n * q];
                if (apq == 0.0) continue;
                double app = A[p + n * p], aqq = A[q + n * q];
                /* rotation that zeroes A(p,q): symmetric 2x2 Schur form */
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* A <- J^T A J with J = [[c, s], [-s, c]] in rows/cols (p, q) */
                for (i64 k = 0; k < n; ++k) { /* columns p, q */
                    double akp = A[k + n * p], akq = A[k + n * q];
                    A[k + n * p] = c * akp - s * akq;
                    A[k + n * q] = s * akp + c * akq;
                }
                for (i64 k = 0; k < n; ++k) { /* rows p, q */
                    double apk = A[p + n * k], aqk = A[q + n * k];
                    A[p + n * k] = c * apk - s * aqk;
                    A[q + n * k] = s * apk + c * aqk;
                }
                for (i64 k = 0; k < n; ++k) { /* V <- V J */
                    double vkp = V[k + n * p], vkq = V[k + n * q];
                    V[k + n * p] = c * vkp - s * vkq;
                    V[k + n * q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (i64 i = 0; i < n; ++i) lam[i] = A[i + n * i];
    free(A);
    sort_and_sign(n, lam, V);
    return converged ? sweep : -1;
}

/* ------------------------------------------------------------------ */
/* small dense LA for the ALS branch                                   */
/* ------------------------------------------------------------------ */

/* Householder QR of an m x n matrix A (m >= n): A = Q R with Q m x n having
 * orthonormal columns and R n x n upper triangular with a non-negative
 * diagonal.  Returns 0 on success. */
int orc_qr_householder(i64 m, i64 n, const double *A, double *Q, double *R) {
    if (m < n) return -1;
    double *W = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *vs = (double *)malloc(sizeof(double) * (size_t)(m * n)); /* reflectors */
    double *beta = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(W, A, sizeof(double) * (size_t)(m * n));
    for (i64 k = 0; k < n; ++k) {
        double *v = vs + m * k;
        double nrm2 = 0.0;
        for (i64 i = k; i < m; ++i) nrm2 += W[i + m * k] * W[i + m * k];
        double nrm = sqrt(nrm2);
        double x0 = W[k + m * k];
        double alpha = (x0 >= 0) ? -nrm : nrm;
        for (i64 i = 0; i < m; ++i) v[i] = 0.0;
        for (i64 i = k; i < m; ++i) v[i] = W[i + m * k];
        v[k] -= alpha;
        double vnorm2 = 0.0;
        for (i64 i = k; i < m; ++i) vnorm2 += v[i] * v[i];
        beta[k] = (vnorm2 > 0) ? 2.0 / vnorm2 : 0.0;
        /* W <- (I - beta v v^T) W */
        for (i64 j = k; j < n; ++j) {
            double d = 0.0;
            for (i64 i = k; i < m; ++i) d += v[i] * W[i + m * j];
            d *= beta[k];
            for (i64 i = k; i < m; ++i) W[i + m * j] -= d * v[i];
        }
    }
    /* R = upper triangle of W */
    for (i64 j = 0; j < n; ++j)
        for (i64 i = 0; i < n; ++i) R[i + n * j] = (i <= j) ? W[i + m * j] : 0.0;
    /* Q = H_0 H_1 ... H_{n-1} applied to the first n columns of the identity */
    for (i64 j = 0; j < n; ++j)
        for (i64 i = 0; i < m; ++i) Q[i + m * j] = (i == j) ? 1.0 : 0.0;
    for (i64 k = n - 1; k >= 0; --k) {
        double *v = vs + m * k;
        for (i64 j = 0; j < n; ++j) {
            double d = 0.0;
            for (i64 i = k; i < m; ++i) d += v[i] * Q[i + m * j];
            d *= beta[k];
            for (i64 i = k; i < m; ++i) Q[i + m * j] -= d * v[i];
        }
    }
    /* make diag(R) non-negative */
    for (i64 k = 0; k < n; ++k) {
        if (R[k + n * k] < 0) {
            for (i64 j = 0; j < n; ++j) R[k + n * j] = -R[k + n * j];
            for (i64 i = 0; i < m; ++i) Q[i + m * k] = -Q[i + m * k];
        }
    }
    free(W);
    free(vs);
    free(beta);
    return 0;
}

/* Cholesky factorization of an SPD n x n matrix: A = C C^T, C lower.
 * Returns 0 on success, -1 if A is not numerically SPD. */
int orc_cholesky(i64 n, const double *A, double *C) {
    memset(C, 0, sizeof(double) * (size_t)(n * n));
    for (i64 j = 0; j < n; ++j) {
        double d = A[j + n * j];
        for (i64 k = 0; k < j; ++k) d -= C[j + n * k] * C[j + n * k];
        if (!(d > 0.0)) return -1;
        double cjj = sqrt(d);
        C[j + n * j] = cjj;
        for (i64 i = j + 1; i < n; ++i) {
            double s = A[i + n * j];
            for (i64 k = 0; k < j; ++k) s -= C[i + n * k] * C[j + n * k];
            C[i + n * j] = s / cjj;
        }
    }
    return 0;
}

/* Solves X A = B for X (m x n) with A SPD n x n, B m x n (i.e. X = B A^{-1}).
 * Uses A = C C^T: X C C^T = B, solved row by row. */
int orc_right_solve_spd(i64 m, i64 n, const double *A, const double *B, double *X) {
    double *C = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (orc_cholesky(n, A, C) != 0) {
        free(C);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (i64 r = 0; r < m; ++r) {
        /* row r of X: x C C^T = b  ->  y C^T = b ... solve y^T: C y^T = b^T (forward)
         * then x C = y  ->  C^T x^T = y^T (backward). */
        double y[1024];
        double *yy = (n <= 1024) ? y : (double *)malloc(sizeof(double) * (size_t)n);
        for (i64 i = 0; i < n; ++i) {
            double s = B[r + m * i];
            for (i64 k = 0; k < i; ++k) s -= C[i + n * k] * yy[k];
            yy[i] = s / C[i + n * i];
        }
        for (i64 i = n - 1; i >= 0; --i) {
            double s = yy[i];
            for (i64 k = i + 1; k < n; ++k) s -= C[k + n * i] * X[r + m * k];
            X[r + m * i] = s / C[i + n * i];
        }
        if (yy != y) free(yy);
    }
    free(C);
    return 0;
}

/* ------------------------------------------------------------------ */
/* ALS factor solver (Alg. 3) and the ALS branch of Alg. 2             */
/* ------------------------------------------------------------------ */

/* One mode of the ALS branch on the matricized working tensor Yn (I x J).
 * L0 (I x R) is the initial guess.  variant 0: Alg. 3 as printed (explicit
 * normal equations); variant 1: L_k re-orthonormalized by QR before each
 * sweep.  Outputs U (I x R, orthonormal) and the new matricized working
 * tensor Ynew (R x J) = R^ R_{k-1}^T.  Returns 0 on success. */
int orc_als_mode(i64 I, i64 J, i64 R, const double *Yn, const double *L0, int iters,
                 int variant, double *U, double *Ynew) {
    double *L = (double *)malloc(sizeof(double) * (size_t)(I * R));
    double *Rk = (double *)malloc(sizeof(double) * (size_t)(J * R)); /* J x R */
    double *T = (double *)malloc(sizeof(double) * (size_t)(J * R));
    double *G = (double *)malloc(sizeof(double) * (size_t)(R * R));
    double *P = (double *)malloc(sizeof(double) * (size_t)(I * R));
    double *Qt = (double *)malloc(sizeof(double) * (size_t)(I * R));
    double *Rt = (double *)malloc(sizeof(double) * (size_t)(R * R));
    int rc = 0;
    memcpy(L, L0, sizeof(double) * (size_t)(I * R));
    for (int k = 0; k < iters && rc == 0; ++k) {
        if (variant == 1) {
            if (orc_qr_householder(I, R, L, Qt, Rt) != 0) { rc = -1; break; }
            memcpy(L, Qt, sizeof(double) * (size_t)(I * R));
        }
        /* R_k = (Yn^T L_k)(L_k^T L_k)^{-1} */
        orc_matmul_tn(J, R, I, Yn, L, T);         /* T = Yn^T L (J x R) */
        orc_matmul_tn(R, R, I, L, L, G);          /* G = L^T L */
        if (orc_right_solve_spd(J, R, G, T, Rk) != 0) { rc = -2; break; }
        /* L_{k+1} = (Yn R_k)(R_k^T R_k)^{-1} */
        orc_matmul_nn(I, R, J, Yn, Rk, P);        /* P = Yn R_k (I x R) */
        orc_matmul_tn(R, R, J, Rk, Rk, G);        /* G = R_k^T R_k */
        if (orc_right_solve_spd(I, R, G, P, L) != 0) { rc = -3; break; }
    }
    if (rc == 0 && iters <= 0) rc = -4;
    if (rc == 0) {
        /* Q^ R^ = L;  U = Q^;  Ynew = R^ R_{k-1}^T  (R x J) */
        if (orc_qr_householder(I, R, L, U, Rt) != 0) rc = -1;
        else orc_matmul_nt(R, J, R, Rt, Rk, Ynew);
    }
    free(L);
    free(Rk);
    free(T);
    free(G);
    free(P);
    free(Qt);
    free(Rt);
    return rc;
}

/* ------------------------------------------------------------------ */
/* st-HOSVD driver (Alg. 2)                                            */
/* ------------------------------------------------------------------ */

/* X: input tensor (dims), read only.  ranks[n] = R_n.  order: the mode
 * order (NULL -> 0..N-1).  methods[n]: 0 = EIG, 1 = ALS for mode n
 * (NULL -> all EIG).  L0[n]: I_n x R_n initial guess for an ALS mode.
 * Outputs: G (prod R_n), U[n] (I_n x R_n), lam[n] (I_n eigenvalues of the
 * mode-n Gram for an EIG mode, descending; may be NULL).  Returns 0 or a
 * negative code. */
int orc_sthosvd(int N, const i64 *dims, const i64 *ranks, const int *order,
                const int *methods, const double *const *L0, int als_iters,
                int als_variant, const double *X, double *G, double *const *U,
                double *const *lam, double jacobi_tol, int jacobi_max_sweeps) {
    if (N < 1 || N > 16) return -10;
    i64 cur[16];
    for (int m = 0; m < N; ++m) cur[m] = dims[m];
    i64 total = orc_numel(N, dims);
    double *Y = (double *)malloc(sizeof(double) * (size_t)total);
    double *Yn = (double *)malloc(sizeof(double) * (size_t)total);
    double *On = (double *)malloc(sizeof(double) * (size_t)total);
    if (!Y || !Yn || !On) { free(Y); free(Yn); free(On); return -11; }
    memcpy(Y, X, sizeof(double) * (size_t)total);
    int rc = 0;
    for (int step = 0; step < N && rc == 0; ++step) {
        int n = order ? order[step] : step;
        i64 In = cur[n], Rn = ranks[n];
        i64 J = orc_numel(N, cur) / In;
        orc_unfold(N, cur, n, Y, Yn);
        int meth = methods ? methods[n] : 0;
        if (meth == 0) {
            double *S = (double *)malloc(sizeof(double) * (size_t)(In * In));
            double *lv = (double *)malloc(sizeof(double) * (size_t)In);
            double *V = (double *)malloc(sizeof(double) * (size_t)(In * In));
            orc_gram(In, J, Yn, S);
            int sw = orc_jacobi_eig(In, S, lv, V, jacobi_tol, jacobi_max_sweeps);
            if (sw < 0) rc = -12;
            memcpy(U[n], V, sizeof(double) * (size_t)(In * Rn));
            if (lam && lam[n]) memcpy(lam[n], lv, sizeof(double) * (size_t)In);
            orc_ttm_t(In, Rn, J, U[n], Yn, On);
            free(S);
            free(lv);
            free(V);
        } else {
            /* ALS starts from the caller's initial guesses (Alg. 3 input) */
            if (!L0 || !L0[n]) {
                rc = -30;
                break;
            }
            int r = orc_als_mode(In, J, Rn, Yn, L0[n], als_iters, als_variant, U[n], On);
            if (r != 0) rc = -20 + r;
        }
        cur[n] = Rn;
        orc_fold(N, cur, n, On, Y);
    }
    if (rc == 0) memcpy(G, Y, sizeof(double) * (size_t)orc_numel(N, cur));
    free(Y);
    free(Yn);
    free(On);
    return rc;
}

/* Tucker reconstruction X^ = G x_1 U1 x_2 U2 ... x_N UN (Sec. II-B). */
int orc_reconstruct(int N, const i64 *dims, const i64 *ranks, const double *G,
                    const double *const *U, double *Xhat) {
    i64 cur[16];
    for (int m = 0; m < N; ++m) cur[m] = ranks[m];
    i64 maxn = orc_numel(N, dims);
    double *A = (double *)malloc(sizeof(double) * (size_t)maxn);
    double *B = (double *)malloc(sizeof(double) * (size_t)maxn);
    if (!A || !B) { free(A); free(B); return -1; }
    memcpy(A, G, sizeof(double) * (size_t)orc_numel(N, ranks));
    for (int n = 0; n < N; ++n) {
        if (orc_ttm_tensor(N, cur, n, dims[n], U[n], A, B) != 0) { free(A); free(B); return -1; }
        cur[n] = dims[n];
        double *t = A; A = B; B = t;
    }
    memcpy(Xhat, A, sizeof(double) * (size_t)maxn);
    free(A);
    free(B);
    return 0;
}

/* ------------------------------------------------------------------ */
/* MLP cost model: layers of dense y = act(W x + b), FP64               */
/* ------------------------------------------------------------------ */

/* Forward pass of a fully connected network on a batch.
 * widths[0..nl]: layer widths (widths[0] = inputs, widths[nl] = outputs).
 * W[l]: widths[l+1] x widths[l] column-major; b[l]: widths[l+1].
 * Hidden layers use tanh, the output layer is linear.
 * X: widths[0] x B (column per sample).  acts: workspace receiving every
 * layer's output, concatenated (sum widths[1..nl] * B doubles).
 * Y: widths[nl] x B. */
void orc_mlp_forward(int nl, const int *widths, const double *const *W,
                     const double *const *b, i64 B, const double *X, double *acts,
                     double *Y) {
    const double *in = X;
    double *out = acts;
    for (int l = 0; l < nl; ++l) {
        int ni = widths[l], no = widths[l + 1];
        for (i64 s = 0; s < B; ++s)
            for (int o = 0; o < no; ++o) {
                double z = b[l][o];
                for (int i = 0; i < ni; ++i) z += W[l][o + no * i] * in[i + ni * s];
                out[o + no * s] = (l + 1 < nl) ? tanh(z) : z;
            }
        in = out;
        out += (i64)no * B;
    }
    memcpy(Y, in, sizeof(double) * (size_t)(widths[nl] * B));
}

/* Mean squared error loss 0.5/B * sum (Y - T)^2 and its gradients with
 * respect to every W[l], b[l] (backpropagation through the forward pass
 * above).  Returns the loss. */
double orc_mlp_loss_grad(int nl, const int *widths, const double *const *W,
                         const double *const *b, i64 B, const double *X,
                         const double *T, double *const *dW, double *const *db) {
    i64 tot = 0;
    for (int l = 1; l <= nl; ++l) tot += (i64)widths[l] * B;
    int maxw = 0;
    for (int l = 0; l <= nl; ++l) if (widths[l] > maxw) maxw = widths[l];
    double *acts = (double *)malloc(sizeof(double) * (size_t)tot);
    double *Y = (double *)malloc(sizeof(double) * (size_t)(widths[nl] * B));
    double *d = (double *)malloc(sizeof(double) * (size_t)(maxw * B));
    double *dn = (double *)malloc(sizeof(double) * (size_t)(maxw * B));
    orc_mlp_forward(nl, widths, W, b, B, X, acts, Y);
    double loss = 0.0;
    int no = widths[nl];
    for (i64 k = 0; k < (i64)no * B; ++k) {
        double e = Y[k] - T[k];
        loss += e * e;
        d[k] = e / (double)B;
    }
    loss *= 0.5 / (double)B;
    /* offsets of each layer's activations */
    i64 off[64];
    off[0] = 0;
    for (int l = 1; l <= nl; ++l) off[l] = off[l - 1] + (i64)widths[l] * B;
    for (int l = nl - 1; l >= 0; --l) {
        int ni = widths[l], nout = widths[l + 1];
        const double *in = (l == 0) ? X : acts + off[l - 1];
        /* d holds dLoss/dz for layer l (pre-activation) */
        for (int o = 0; o < nout; ++o) {
            double s = 0.0;
            for (i64 q = 0; q < B; ++q) s += d[o + nout * q];
            db[l][o] = s;
            for (int i = 0; i < ni; ++i) {
                double t = 0.0;
                for (i64 q = 0; q < B; ++q) t += d[o + nout * q] * in[i + ni * q];
                dW[l][o + nout * i] = t;
            }
        }
        if (l > 0) {
            for (i64 q = 0; q < B; ++q)
                for (int i = 0; i < ni; ++i) {
                    double s = 0.0;
                    for (int o = 0; o < nout; ++o) s += W[l][o + nout * i] * d[o + nout * q];
                    double a = in[i + ni * q]; /* tanh output */
                    dn[i + ni * q] = s * (1.0 - a * a);
                }
            double *t = d; d = dn; dn = t;
        }
    }
    free(acts);
    free(Y);
    free(d);
    free(dn);
    return loss;
}
