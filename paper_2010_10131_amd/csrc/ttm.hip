// Matricization-free mode-n TTM on the gfx950 matrix cores.
//
// Computes, for a column-major tensor viewed as (L, K, M) along mode n
// (L = product of the dims before n, M = product after), the mode-n product
// with the transpose of a K x Rout factor V (Eq. 2; the core update of
// Alg. 2 and the expansion step of the Tucker reconstruction):
//
//     Z(a, r, b) = sum_k V(k, r) * Y(a, k, b)          (Z is (L, Rout, M))
//
// The loops are split at mode n into "inside" (a), "along" (k) and
// "outside" (b) as in Sec. V / Fig. 4; the (a, b) pairs are the rows of one
// GEMM with K-long rows that are strided by L in memory.  Nothing is
// transposed or copied.
//
// Design (MI355X): the kernel is HBM-bound for bf16x3 and for small Rout, so
// each Y element is read from HBM exactly once, straight into the lane that
// feeds it to the matrix cores (no LDS round trip for Y):
//   * a wave owns NT row tiles of 16 rows and RTB r-tiles of 16 columns;
//   * per 32-wide chunk of k a lane loads the 8 consecutive k of its row
//     (two 16-byte loads when L = 1, 8 strided loads otherwise), splits them
//     once into the requested precision and multiplies them against every
//     r-tile of the factor;
//   * the factor is pre-split by ttm_prep_u into matrix-core-ready 16-byte
//     quads and staged once per workgroup in LDS (read from L2 when it does
//     not fit), so the only HBM traffic is one read of Y and one write of Z;
//   * the next chunk's loads are issued before the current chunk's
//     matrix-core work (register double buffering).
#include "common.h"
#include "internal.h"
#include "ttm_body.h"

#include <mutex>

namespace sth {

// V (K x Rout) -> quads [c][rt][q][lane] (16 bytes each), zero padded.
// transpose = 0: V = U with U (K x Rout) column-major.
// transpose = 1: V = U^T with U (Rout x K) column-major.
template <int PREC>
__global__ void ttm_prep_u_kernel(const double *__restrict__ U, int64_t K, int64_t Rout,
                                  int transpose, uint4 *__restrict__ out, int nchunks,
                                  int ntiles) {
    constexpr int NQ = Frag<PREC>::NQ;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nchunks * ntiles * 64;
    if (gid >= total) return;
    int lane = (int)(gid % 64);
    int64_t blk = gid / 64;  // c * ntiles + rt
    int rt = (int)(blk % ntiles);
    int c = (int)(blk / ntiles);
    int g = lane / 16;
    int64_t r = (int64_t)rt * 16 + lane % 16;
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int64_t k = (int64_t)c * KC + 8 * g + j;
        double v = 0.0;
        if (k < K && r < Rout) v = transpose ? U[r + Rout * k] : U[k + K * r];
        x[j] = v;
    }
    FragQ<PREC> f;
    make_frag(x, f.f);
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[(blk * NQ + q) * 64 + lane] = f.q[q];
}

template <typename T, int PREC, int NT, int RTB, bool CONTIG, bool ULDS, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void ttm_kernel(
    const T *__restrict__ Y, const uint4 *__restrict__ Uq, T *__restrict__ Z, int64_t L, int64_t K,
    int64_t Rout, int64_t P, int nchunks, int ntiles, int64_t nrowblocks) {
    ttm_body<T, PREC, NT, RTB, CONTIG, ULDS, WAVES>(Y, Uq, Z, L, K, Rout, P, nchunks, ntiles,
                                                    nrowblocks, blockIdx.x, gridDim.x, blockIdx.y);
}

// The TTM fused with the error sums of a reconstruction (nothing stored):
// per-workgroup sums of (X - Z)^2 and X^2 into epart.
template <typename T, int PREC, int NT, int RTB, bool CONTIG, bool ULDS, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void ttm_err_kernel(
    const T *__restrict__ Y, const uint4 *__restrict__ Uq, const T *__restrict__ X, int64_t L, int64_t K,
    int64_t Rout, int64_t P, int nchunks, int ntiles, int64_t nrowblocks, double *__restrict__ epart) {
    ttm_body<T, PREC, NT, RTB, CONTIG, ULDS, WAVES, 1, false, true>(Y, Uq, nullptr, L, K, Rout, P, nchunks, ntiles,
                                                                   nrowblocks, blockIdx.x, gridDim.x, blockIdx.y,
                                                                   X, epart);
}

// out[0], out[1] = the sums of the n (d, x) pairs: 256 threads each sum a
// strided subset in order, then a fixed tree
__global__ __launch_bounds__(256) void sum_pairs_kernel(const double *__restrict__ part, int64_t n,
                                                        double *__restrict__ out) {
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sb[threadIdx.x] += sb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sa[0];
        out[1] = sb[0];
    }
}

template <int PREC, int NT, int CPW, bool FULL>
__global__ __launch_bounds__(64 * KS_WAVES) void ttm_ks_kernel(
    const float *__restrict__ Y, const uint4 *__restrict__ Uq, float *__restrict__ Z, int64_t K,
    int64_t Rout, int64_t P, int nchunks, int ntiles, int64_t nblocks) {
    ttm_ks_body<PREC, NT, CPW, false, FULL>(Y, Uq, Z, K, Rout, P, nchunks, ntiles, nblocks, blockIdx.x,
                                            gridDim.x, blockIdx.y);
}

// Scratch for callers that cannot allocate (ttm_mode_n_noalloc): the
// pre-split factor of one call lives here instead of in a caller workspace.
// Each device that runs the library holds its own copy until the process
// ends.  Host code must never pass `scratch` itself to a kernel (on the host
// it names a stand-in, not a device address); it uses the address that
// ttm_scratch_ptr() looked up for the current device.
constexpr size_t TTM_SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[TTM_SCRATCH_BYTES];

// ---------------------------------------------------------------- host ----

size_t ttm_prep_bytes(int64_t K, int64_t Rout, int prec) {
    int64_t nchunks = (K + KC - 1) / KC;
    int64_t ntiles = (Rout + 15) / 16;
    return (size_t)(nchunks * ntiles * 64 * 16 * prec_nq(prec));
}

size_t ttm_scratch_bytes() { return TTM_SCRATCH_BYTES; }

// Device address of `scratch` on the current device, looked up once per
// device with that device current and kept for later calls.
hipError_t ttm_scratch_ptr(void **out) {
    static std::mutex mu;
    static void *addr[64] = {nullptr};
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t ttm_prep_u(const double *U, int64_t K, int64_t Rout, int transpose, int prec,
                      void *out, hipStream_t s) {
    int nchunks = (int)((K + KC - 1) / KC);
    int ntiles = (int)((Rout + 15) / 16);
    int64_t total = (int64_t)nchunks * ntiles * 64;
    dim3 grid((unsigned)((total + 255) / 256));
    uint4 *o = (uint4 *)out;
    switch (prec) {
        case P_FP64: hipLaunchKernelGGL(ttm_prep_u_kernel<P_FP64>, grid, dim3(256), 0, s, U, K, Rout, transpose, o, nchunks, ntiles); break;
        case P_FP32: hipLaunchKernelGGL(ttm_prep_u_kernel<P_FP32>, grid, dim3(256), 0, s, U, K, Rout, transpose, o, nchunks, ntiles); break;
        case P_BF16X3: hipLaunchKernelGGL(ttm_prep_u_kernel<P_BF16X3>, grid, dim3(256), 0, s, U, K, Rout, transpose, o, nchunks, ntiles); break;
        default: hipLaunchKernelGGL(ttm_prep_u_kernel<P_BF16X6>, grid, dim3(256), 0, s, U, K, Rout, transpose, o, nchunks, ntiles); break;
    }
    return hipGetLastError();
}

namespace {

constexpr int TTM_WAVES = 8;
constexpr size_t TTM_LDS_MAX = 144 * 1024;

template <typename T, int PREC, int NT, int RTB, bool CONTIG, bool ULDS>
hipError_t launch_ttm_t(const T *Y, const uint4 *Uq, T *Z, int64_t L, int64_t K, int64_t Rout,
                        int64_t M, hipStream_t s) {
    const int64_t P = L * M;
    const int nchunks = (int)((K + KC - 1) / KC);
    const int ntiles = (int)((Rout + 15) / 16);
    const int nrb = (ntiles + RTB - 1) / RTB;
    const int64_t nrowblocks = (P + 16 * NT - 1) / (16 * NT);
    const size_t lds = ULDS ? (size_t)nchunks * RTB * Frag<PREC>::NQ * 64 * 16 : 0;
    int64_t wgs = (nrowblocks + TTM_WAVES - 1) / TTM_WAVES;
    const int per_cu = ULDS ? (int)std::max<size_t>(1, std::min<size_t>(2, (160 * 1024) / std::max<size_t>(lds, 1))) : 2;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    if (ULDS && wgs > cap) wgs = cap;  // persistent: amortize the factor staging
    if (wgs < 1) wgs = 1;
    auto kern = ttm_kernel<T, PREC, NT, RTB, CONTIG, ULDS, TTM_WAVES>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)wgs, (unsigned)nrb), dim3(64 * TTM_WAVES), lds, s, Y, Uq,
                       Z, L, K, Rout, P, nchunks, ntiles, nrowblocks);
    return hipGetLastError();
}

template <int PREC, int CPW>
hipError_t launch_ttm_ks(const float *Y, const uint4 *Uq, float *Z, int64_t K, int64_t Rout, int64_t M,
                         hipStream_t s) {
    constexpr int NT = 2;
    const int nchunks = (int)((K + KC - 1) / KC);
    const int ntiles = (int)((Rout + 15) / 16);
    const int nrb = (ntiles + 3) / 4;
    const int64_t nblocks = (M + 16 * NT - 1) / (16 * NT);
    const size_t lds = ttm_ks_lds(NT);
    const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>(nblocks, (int64_t)device_cu_count()));
    // whole chunks for every wave: the branch-free kernel
    auto kern = (K == (int64_t)KS_WAVES * CPW * KC) ? ttm_ks_kernel<PREC, NT, CPW, true>
                                                    : ttm_ks_kernel<PREC, NT, CPW, false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)wgs, (unsigned)nrb), dim3(64 * KS_WAVES), lds, s, Y, Uq, Z, K,
                       Rout, M, nchunks, ntiles, nblocks);
    return hipGetLastError();
}

template <typename T, int PREC, int RTB>
hipError_t launch_ttm_r(const T *Y, const uint4 *Uq, T *Z, int64_t L, int64_t K, int64_t Rout,
                        int64_t M, hipStream_t s) {
    const int nchunks = (int)((K + KC - 1) / KC);
    const size_t lds = (size_t)nchunks * RTB * Frag<PREC>::NQ * 64 * 16;
    const bool contig = (L == 1) && (K % (16 / sizeof(T)) == 0) &&
                        ((reinterpret_cast<uintptr_t>(Y) & 15) == 0);
    // contiguous rows of 256 < K <= 512 values in FP32 storage: the K-split
    // kernel (all eight waves busy, whole row blocks streamed)
    if constexpr (sizeof(T) == 4 && (PREC == P_FP32 || PREC == P_BF16X3) && RTB == 4) {
        const int nchunks = (int)((K + KC - 1) / KC);
        if (contig && nchunks > 8 && nchunks <= 16)
            return launch_ttm_ks<PREC, 2>(reinterpret_cast<const float *>(Y), Uq, reinterpret_cast<float *>(Z),
                                          K, Rout, M, s);
    }
    // row tiles per wave: keeps a lane under 256 VGPRs (8 waves per workgroup)
    constexpr int NT = (PREC == P_FP64) ? (RTB == 1 ? 2 : 1) : (RTB == 1 ? 4 : 2);
    if (lds <= TTM_LDS_MAX) {
        if (contig) return launch_ttm_t<T, PREC, NT, RTB, true, true>(Y, Uq, Z, L, K, Rout, M, s);
        return launch_ttm_t<T, PREC, NT, RTB, false, true>(Y, Uq, Z, L, K, Rout, M, s);
    }
    if (contig) return launch_ttm_t<T, PREC, NT, RTB, true, false>(Y, Uq, Z, L, K, Rout, M, s);
    return launch_ttm_t<T, PREC, NT, RTB, false, false>(Y, Uq, Z, L, K, Rout, M, s);
}

template <typename T, int PREC>
hipError_t launch_ttm_p(const T *Y, const uint4 *Uq, T *Z, int64_t L, int64_t K, int64_t Rout,
                        int64_t M, hipStream_t s) {
    const int64_t ntiles = (Rout + 15) / 16;
    if (ntiles <= 1) return launch_ttm_r<T, PREC, 1>(Y, Uq, Z, L, K, Rout, M, s);
    if (ntiles <= 2) return launch_ttm_r<T, PREC, 2>(Y, Uq, Z, L, K, Rout, M, s);
    return launch_ttm_r<T, PREC, 4>(Y, Uq, Z, L, K, Rout, M, s);
}

// ---- the TTM fused with the reconstruction error ----
constexpr int64_t TTM_ERR_WGS = 1024;   // workgroups per r-block at most (partial sums stay small)

int ttm_err_rtb(int64_t Rout) {
    const int64_t ntiles = (Rout + 15) / 16;
    return ntiles <= 1 ? 1 : (ntiles <= 2 ? 2 : 4);
}

template <typename T, int PREC, int RTB>
hipError_t launch_ttm_err_r(const T *Y, const uint4 *Uq, const T *X, int64_t L, int64_t K, int64_t Rout,
                            int64_t M, double *part, double *out, hipStream_t s) {
    constexpr int NT = (PREC == P_FP64) ? (RTB == 1 ? 2 : 1) : (RTB == 1 ? 4 : 2);
    const int64_t P = L * M;
    const int nchunks = (int)((K + KC - 1) / KC);
    const int ntiles = (int)((Rout + 15) / 16);
    const int nrb = (ntiles + RTB - 1) / RTB;
    const int64_t nrowblocks = (P + 16 * NT - 1) / (16 * NT);
    const size_t lds = (size_t)nchunks * RTB * Frag<PREC>::NQ * 64 * 16;
    const bool ulds = lds <= TTM_LDS_MAX;
    int64_t wgs = std::min<int64_t>(TTM_ERR_WGS, (nrowblocks + TTM_WAVES - 1) / TTM_WAVES);
    if (ulds) {
        const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(2, (160 * 1024) / std::max<size_t>(lds, 1)));
        wgs = std::min<int64_t>(wgs, (int64_t)device_cu_count() * per_cu);
    }
    if (wgs < 1) wgs = 1;
    const bool contig = L == 1;
    hipError_t e;
    auto go = [&](auto kern, size_t lb) -> hipError_t {
        if (lb > 64 * 1024) {
            hipError_t r = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb);
            if (r != hipSuccess) return r;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)wgs, (unsigned)nrb), dim3(64 * TTM_WAVES), lb, s, Y, Uq, X, L, K,
                           Rout, P, nchunks, ntiles, nrowblocks, part);
        return hipGetLastError();
    };
    if (ulds) e = contig ? go(ttm_err_kernel<T, PREC, NT, RTB, true, true, TTM_WAVES>, lds)
                         : go(ttm_err_kernel<T, PREC, NT, RTB, false, true, TTM_WAVES>, lds);
    else e = contig ? go(ttm_err_kernel<T, PREC, NT, RTB, true, false, TTM_WAVES>, 0)
                    : go(ttm_err_kernel<T, PREC, NT, RTB, false, false, TTM_WAVES>, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(256), 0, s, part, wgs * nrb, out);
    return hipGetLastError();
}

template <typename T, int PREC>
hipError_t launch_ttm_err_p(const T *Y, const uint4 *Uq, const T *X, int64_t L, int64_t K, int64_t Rout,
                            int64_t M, double *part, double *out, hipStream_t s) {
    switch (ttm_err_rtb(Rout)) {
        case 1: return launch_ttm_err_r<T, PREC, 1>(Y, Uq, X, L, K, Rout, M, part, out, s);
        case 2: return launch_ttm_err_r<T, PREC, 2>(Y, Uq, X, L, K, Rout, M, part, out, s);
        default: return launch_ttm_err_r<T, PREC, 4>(Y, Uq, X, L, K, Rout, M, part, out, s);
    }
}

}  // namespace

size_t ttm_err_part_doubles(int64_t Rout) {
    const int64_t ntiles = (Rout + 15) / 16, rtb = ttm_err_rtb(Rout);
    return (size_t)(2 * TTM_ERR_WGS * ((ntiles + rtb - 1) / rtb));
}

hipError_t ttm_err_launch(int dtype, int prec, const void *Y, const void *Uq, const void *X, int64_t L, int64_t K,
                          int64_t Rout, int64_t M, double *part, double *out, hipStream_t s) {
    const uint4 *uq = (const uint4 *)Uq;
    if (dtype == DT_F64)
        return launch_ttm_err_p<double, P_FP64>((const double *)Y, uq, (const double *)X, L, K, Rout, M, part, out, s);
    const float *y = (const float *)Y, *x = (const float *)X;
    switch (prec) {
        case P_FP64: return launch_ttm_err_p<float, P_FP64>(y, uq, x, L, K, Rout, M, part, out, s);
        case P_FP32: return launch_ttm_err_p<float, P_FP32>(y, uq, x, L, K, Rout, M, part, out, s);
        case P_BF16X3: return launch_ttm_err_p<float, P_BF16X3>(y, uq, x, L, K, Rout, M, part, out, s);
        default: return launch_ttm_err_p<float, P_BF16X6>(y, uq, x, L, K, Rout, M, part, out, s);
    }
}

hipError_t ttm_launch(int dtype, int prec, const void *Y, const void *Uq, void *Z, int64_t L,
                      int64_t K, int64_t Rout, int64_t M, hipStream_t s) {
    if (L * M == 0 || Rout == 0) return hipSuccess;
    const uint4 *uq = (const uint4 *)Uq;
    if (dtype == DT_F64) {
        return launch_ttm_p<double, P_FP64>((const double *)Y, uq, (double *)Z, L, K, Rout, M, s);
    }
    const float *y = (const float *)Y;
    float *z = (float *)Z;
    switch (prec) {
        case P_FP64: return launch_ttm_p<float, P_FP64>(y, uq, z, L, K, Rout, M, s);
        case P_FP32: return launch_ttm_p<float, P_FP32>(y, uq, z, L, K, Rout, M, s);
        case P_BF16X3: return launch_ttm_p<float, P_BF16X3>(y, uq, z, L, K, Rout, M, s);
        default: return launch_ttm_p<float, P_BF16X6>(y, uq, z, L, K, Rout, M, s);
    }
}

}  // namespace sth
