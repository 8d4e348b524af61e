// Small dense FP64 linear algebra for the ALS branch (Alg. 3 and the QR of
// Alg. 2) and the FP64 norm reductions (Eq. 1).
//
//   gemm_f64      C = alpha op(A) op(B) + beta C, 32x32 tiles, optional
//                 split-K with a fixed-order reduction (deterministic)
//   chol_kernel   one workgroup: G (+ shift) = R^T R (Cholesky, R upper),
//                 writes R and R^{-1}; used for the normal equations of
//                 Alg. 3 and for Cholesky-QR
//   sumsq / diff  FP64 sums of squares with per-block partials reduced in a
//                 fixed order
#include "chol_body.h"
#include "common.h"
#include "internal.h"

namespace sth {

constexpr int GT = 32;   // gemm tile (rows and columns of C)
constexpr int GK = 128;  // k-extent staged in LDS per step

// C_part[z] (m x n, ldc) = op(A) op(B) over k-slice z.  The skinny products
// of the eigensolver and the ALS branch are latency-bound, so every step
// loads a whole GT x GK panel of each operand with all loads in flight at
// once (coalesced along the contiguous index of each operand), then runs
// GK rank-1 updates from LDS: one global round trip per 128 values of k.
__global__ __launch_bounds__(256) void gemm_f64_kernel(int ta, int tb, int m, int n, int k,
                                                       double alpha, const double *__restrict__ A,
                                                       int64_t lda, const double *__restrict__ B,
                                                       int64_t ldb, double beta, double *__restrict__ C,
                                                       int64_t ldc, int kslice, double *__restrict__ part) {
    extern __shared__ __align__(16) double s_gemm[];
    double *sA = s_gemm;                  // sA[kk * (GT + 1) + r] = op(A)(row0 + r, kc + kk)
    double *sB = s_gemm + GK * (GT + 1);  // sB[kk * (GT + 1) + c] = op(B)(kc + kk, col0 + c)
    constexpr int PER = GT * GK / 256;    // elements of each panel per thread
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int row0 = blockIdx.x * GT, col0 = blockIdx.y * GT;
    const int kz = blockIdx.z;
    const int kbeg = kz * kslice, kend = min(k, kbeg + kslice);
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (int kc = kbeg; kc < kend; kc += GK) {
        double ra[PER], rb[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            // A panel: contiguous along r (op = A) or along kk (op = A^T)
            int r, kk;
            if (ta) { kk = e % GK; r = e / GK; } else { r = e % GT; kk = e / GT; }
            int gr = row0 + r, gk = kc + kk;
            ra[u] = (gr < m && gk < kend) ? (ta ? A[gk + lda * gr] : A[gr + lda * gk]) : 0.0;
            // B panel: contiguous along kk (op = B) or along c (op = B^T)
            int cc, kb;
            if (tb) { cc = e % GT; kb = e / GT; } else { kb = e % GK; cc = e / GK; }
            int gc = col0 + cc, gk2 = kc + kb;
            rb[u] = (gc < n && gk2 < kend) ? (tb ? B[gc + ldb * gk2] : B[gk2 + ldb * gc]) : 0.0;
        }
        __syncthreads();  // the previous step's reads of the panels are done
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            int r, kk;
            if (ta) { kk = e % GK; r = e / GK; } else { r = e % GT; kk = e / GT; }
            sA[kk * (GT + 1) + r] = ra[u];
            int cc, kb;
            if (tb) { cc = e % GT; kb = e / GT; } else { kb = e % GK; cc = e / GK; }
            sB[kb * (GT + 1) + cc] = rb[u];
        }
        __syncthreads();
        const int kn = min(GK, kend - kc);
#pragma unroll 8
        for (int kk = 0; kk < kn; ++kk) {
            const double a0 = sA[kk * (GT + 1) + tx], a1 = sA[kk * (GT + 1) + tx + 16];
            const double b0 = sB[kk * (GT + 1) + ty], b1 = sB[kk * (GT + 1) + ty + 16];
            acc[0][0] += a0 * b0;
            acc[1][0] += a1 * b0;
            acc[0][1] += a0 * b1;
            acc[1][1] += a1 * b1;
        }
    }
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
            int r = row0 + tx + 16 * x, c = col0 + ty + 16 * y;
            if (r < m && c < n) {
                if (part) {
                    part[(int64_t)kz * m * n + r + (int64_t)m * c] = acc[x][y];
                } else {
                    double old = (beta != 0.0) ? C[r + ldc * c] : 0.0;
                    C[r + ldc * c] = alpha * acc[x][y] + beta * old;
                }
            }
        }
}

constexpr size_t GEMM_LDS = (size_t)2 * GK * (GT + 1) * sizeof(double);

__global__ void gemm_reduce_kernel(int m, int n, int nz, const double *__restrict__ part,
                                   double alpha, double beta, double *__restrict__ C, int64_t ldc) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    int r = (int)(e % m), c = (int)(e / m);
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * m * n + e];
    double old = (beta != 0.0) ? C[r + ldc * c] : 0.0;
    C[r + ldc * c] = alpha * s + beta * old;
}

size_t gemm_ws_bytes(int m, int n, int k) {
    int nz = gemm_splits(m, n, k);
    return nz > 1 ? (size_t)nz * m * n * sizeof(double) : 0;
}

// k-slices: one LDS step (GK values of k) per workgroup where the tile count
// leaves the chip idle, at most 32 slices.
int gemm_splits(int m, int n, int k) {
    const int tiles = ((m + GT - 1) / GT) * ((n + GT - 1) / GT);
    if (tiles >= 256) return 1;
    int nz = (k + GK - 1) / GK;
    nz = std::min(nz, 32);
    while (nz > 1 && tiles * nz > 1024) nz = (nz + 1) / 2;
    return std::max(nz, 1);
}

hipError_t gemm_f64(int ta, int tb, int m, int n, int k, double alpha, const double *A,
                    int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                    void *ws, hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    int nz = gemm_splits(m, n, k);
    int kslice = (k + nz - 1) / nz;
    kslice = (kslice + GT - 1) / GT * GT;
    if (kslice == 0) kslice = GT;
    nz = std::max(1, (k + kslice - 1) / kslice);
    dim3 grid((m + GT - 1) / GT, (n + GT - 1) / GT, nz);
    double *part = nz > 1 ? (double *)ws : nullptr;
    hipError_t ea = hipFuncSetAttribute((const void *)gemm_f64_kernel,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)GEMM_LDS);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), GEMM_LDS, s, ta, tb, m, n, k, alpha, A, lda, B,
                       ldb, beta, C, ldc, kslice, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nz == 1) return e;
    int64_t tot = (int64_t)m * n;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m,
                       n, nz, part, alpha, beta, C, ldc);
    return hipGetLastError();
}

constexpr int CHOL_THREADS = 512;

__global__ __launch_bounds__(CHOL_THREADS) void chol_kernel(const double *__restrict__ G, int n,
                                                            int64_t ldg, double shift_rel,
                                                            double *__restrict__ Rout,
                                                            double *__restrict__ Rinv,
                                                            int64_t *__restrict__ flag,
                                                            const double *__restrict__ gate, int gate_R,
                                                            double gate_tol) {
    if (!gate_open(gate, gate_R, gate_tol)) return;
    chol_body<CHOL_THREADS>(G, n, ldg, shift_rel, Rout, Rinv, flag);
}

hipError_t chol_launch(const double *G, int n, int64_t ldg, double shift_rel, double *R,
                       double *Rinv, int64_t *flag, hipStream_t s, const double *gate, int gate_R,
                       double gate_tol) {
    const size_t lds = chol_lds_bytes(n);
    if (lds > 64 * 1024)
        if (hipError_t ea = hipFuncSetAttribute((const void *)chol_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) return ea;
    hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(CHOL_THREADS), lds, s, G, n, ldg, shift_rel, R, Rinv, flag,
                       gate, gate_R, gate_tol);
    return hipGetLastError();
}

// ------------------------------------------------------------- norms ----

template <typename T>
__global__ __launch_bounds__(256) void sumsq_kernel(const T *__restrict__ x, const T *__restrict__ y,
                                                    int64_t count, double *__restrict__ part) {
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
        double v = (double)x[e];
        if (y) v -= (double)y[e];
        s += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double sw[4];
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((sw[0] + sw[1]) + sw[2]) + sw[3];
}

__global__ void sum_parts_kernel(const double *__restrict__ part, int n, double *__restrict__ out,
                                 int64_t *__restrict__ flag) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s;
    if (flag && !(fabs(s) <= 1.7e308)) flag[0] = 3;  // NaN or Inf
}

hipError_t sumsq_launch(int dtype, const void *x, const void *y, int64_t count, double *out,
                        double *part, int64_t *flag, hipStream_t s) {
    int nb = (int)std::min<int64_t>(SUMSQ_BLOCKS, std::max<int64_t>(1, (count + 255) / 256));
    if (dtype == DT_F64)
        hipLaunchKernelGGL(sumsq_kernel<double>, dim3(nb), dim3(256), 0, s, (const double *)x,
                           (const double *)y, count, part);
    else
        hipLaunchKernelGGL(sumsq_kernel<float>, dim3(nb), dim3(256), 0, s, (const float *)x,
                           (const float *)y, count, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, s, part, nb, out, flag);
    return hipGetLastError();
}

// --------------------------------------------------------------- misc ----

__global__ void fill_f64_kernel(double *p, int64_t n, double v) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

hipError_t fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void copy_f64_kernel(const double *src, double *dst, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[e];
}

hipError_t copy_f64(const double *src, double *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

__global__ void zero_bytes_kernel(uint32_t *p, int64_t nwords) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nwords) p[e] = 0u;
}

hipError_t zero_words(void *p, int64_t nwords, hipStream_t s) {
    if (nwords <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_bytes_kernel, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, s,
                       (uint32_t *)p, nwords);
    return hipGetLastError();
}

// Gaussian initial guess (ALS L_0, subspace-iteration start block).
__global__ void gaussian_kernel(double *p, int64_t n, uint64_t seed, uint64_t stream) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    p[e] = gaussian_value(seed, stream, (uint64_t)e);
}

hipError_t gaussian_f64(double *p, int64_t n, uint64_t seed, uint64_t stream, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, seed, stream);
    return hipGetLastError();
}

}  // namespace sth
