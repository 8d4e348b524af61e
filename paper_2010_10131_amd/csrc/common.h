// Device-side building blocks shared by the gfx950 kernels: matrix-core
// (MFMA) wrappers, bf16 splitting and the 8-element operand fragments every
// contraction kernel feeds to the matrix cores.
//
// Matrix-core conventions used throughout (16x16 output tiles, 64 lanes,
// lane t, group g = t / 16):
//   A operand: lane t supplies row (t % 16) of A for the k-slice owned by g;
//   B operand: lane t supplies column (t % 16) of B for the same k-slice;
//   D:         lane t holds D[4g + v][t % 16], v = 0..3, for the FP32 and
//              bf16 instructions, but D[g + 4v][t % 16] for the FP64 one
//              (measured on gfx950; see drow()).
// Each lane owns 8 consecutive contraction indices k = 8g .. 8g+7 of a
// 32-wide chunk.  The 16x16x32 bf16 instruction consumes all 8 at once; the
// 16x16x4 FP32 / FP64 instructions consume one per instruction (8 of them
// per chunk, instruction j taking k = 8g + j), so the same fragment layout
// serves every precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sth {

typedef float f32x4 __attribute__((ext_vector_type(4)));
// four floats at a 4-byte aligned address (one 16-byte load on this target)
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16X3 = 2, P_BF16X6 = 3 };

constexpr int KC = 32;  // contraction chunk (elements) per fragment group

__device__ __forceinline__ f32x4 mma(const bf16x8 &a, const bf16x8 &b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even float -> bf16 and back (exact widening).
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf16(__bf16 h) { return (float)h; }

// Operand fragment: the 8 values one lane contributes for one 32-wide chunk,
// already in the representation the matrix cores consume.
template <int PREC> struct Frag;
template <> struct Frag<P_FP64> {
    double v[8];
    static constexpr int NQ = 4;  // 16-byte quads
};
template <> struct Frag<P_FP32> {
    float v[8];
    static constexpr int NQ = 2;
};
template <> struct Frag<P_BF16X3> {
    bf16x8 hi, mid;
    static constexpr int NQ = 2;
};
template <> struct Frag<P_BF16X6> {
    bf16x8 hi, mid, lo;
    static constexpr int NQ = 3;
};

// Row of the 16x16 output tile held by lane group g in accumulator slot v.
template <int PREC> __device__ __forceinline__ int drow(int g, int v) { return 4 * g + v; }
template <> __device__ __forceinline__ int drow<P_FP64>(int g, int v) { return g + 4 * v; }

template <int PREC> struct Acc { typedef f32x4 type; };
template <> struct Acc<P_FP64> { typedef f64x4 type; };

// Builds a fragment from 8 raw values (float or double).
template <typename T>
__device__ __forceinline__ void make_frag(const T (&x)[8], Frag<P_FP64> &f) {
#pragma unroll
    for (int j = 0; j < 8; ++j) f.v[j] = (double)x[j];
}
template <typename T>
__device__ __forceinline__ void make_frag(const T (&x)[8], Frag<P_FP32> &f) {
#pragma unroll
    for (int j = 0; j < 8; ++j) f.v[j] = (float)x[j];
}
template <typename T>
__device__ __forceinline__ void make_frag(const T (&x)[8], Frag<P_BF16X3> &f) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float v = (float)x[j];
        __bf16 h = to_bf16(v);
        f.hi[j] = h;
        f.mid[j] = to_bf16(v - from_bf16(h));
    }
}
template <typename T>
__device__ __forceinline__ void make_frag(const T (&x)[8], Frag<P_BF16X6> &f) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float v = (float)x[j];
        __bf16 h = to_bf16(v);
        float r1 = v - from_bf16(h);
        __bf16 m = to_bf16(r1);
        f.hi[j] = h;
        f.mid[j] = m;
        f.lo[j] = to_bf16(r1 - from_bf16(m));
    }
}

// acc += A_frag (rows) x B_frag (cols) over one 32-wide chunk.
__device__ __forceinline__ void mma_frag(const Frag<P_FP64> &a, const Frag<P_FP64> &b, f64x4 &c) {
#pragma unroll
    for (int j = 0; j < 8; ++j) c = mma(a.v[j], b.v[j], c);
}
__device__ __forceinline__ void mma_frag(const Frag<P_FP32> &a, const Frag<P_FP32> &b, f32x4 &c) {
#pragma unroll
    for (int j = 0; j < 8; ++j) c = mma(a.v[j], b.v[j], c);
}
__device__ __forceinline__ void mma_frag(const Frag<P_BF16X3> &a, const Frag<P_BF16X3> &b,
                                         f32x4 &c) {
    c = mma(a.mid, b.hi, c);
    c = mma(a.hi, b.mid, c);
    c = mma(a.hi, b.hi, c);
}
__device__ __forceinline__ void mma_frag(const Frag<P_BF16X6> &a, const Frag<P_BF16X6> &b,
                                         f32x4 &c) {
    c = mma(a.lo, b.hi, c);
    c = mma(a.hi, b.lo, c);
    c = mma(a.mid, b.mid, c);
    c = mma(a.mid, b.hi, c);
    c = mma(a.hi, b.mid, c);
    c = mma(a.hi, b.hi, c);
}

// Fragments as raw 16-byte quads, for copies between global memory and LDS.
template <int PREC> union FragQ {
    Frag<PREC> f;
    uint4 q[Frag<PREC>::NQ];
};

// Counter-based standard normal sample: SplitMix64 (Steele, Lea & Flood,
// OOPSLA 2014) on (seed, stream, element), two uniforms -> Box-Muller.
// Gate of the launches that repeat a solve step only when a residual test
// failed: true when res is null (ungated) or when some res[r], r < R, is
// above tol * res[R] or not finite.  Every wave reads the same R + 1 values,
// so the answer is uniform across the workgroup (no barrier needed).
__device__ __forceinline__ bool gate_open(const double *res, int R, double tol) {
    if (!res) return true;
    const double thr = tol * res[R];
    int bad = 0;
    for (int r = (int)(threadIdx.x & 63); r < R; r += 64)
        if (!(res[r] <= thr)) bad = 1;
    return __ballot(bad) != 0;
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double gaussian_value(uint64_t seed, uint64_t stream, uint64_t e) {
    const uint64_t base = splitmix64(seed ^ splitmix64(stream + 0x5851F42D4C957F2Dull));
    const uint64_t a = splitmix64(base + 2 * e);
    const uint64_t b = splitmix64(base + 2 * e + 1);
    const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);           // [0, 1)
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace sth
