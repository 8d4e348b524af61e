// Device body of the FP64 cyclic Jacobi eigensolver (one workgroup) and the
// eigensolver constants, shared by the single-matrix and batched kernels.
#pragma once
#include "common.h"

namespace sth {

constexpr int64_t EIG_DIRECT_MAX = 128;  // Jacobi on the whole matrix up to this order
// Largest order whose A and V both fit in LDS for the Jacobi (V goes to the
// workspace above it).  The decompositions, which need the leading subspace
// only, take the subspace iteration from the next order on when its block fits.
constexpr int64_t EIG_LDS_DIRECT_MAX = 96;
// FP32-data decompositions take the subspace iteration from order 49 when
// its block is at most half the order (leading subspace to working accuracy
// on a gapped spectrum at a fraction of the full Jacobi's sweeps).
constexpr int64_t EIG_SI_MIN = 48;
constexpr int64_t SI_BLOCK_MAX = 128;    // Rayleigh-Ritz block (Cholesky-QR and small Jacobi reach 128)
constexpr int EIG_LDS_AV = 150 * 1024;   // LDS bytes available for Jacobi's A and V

// Block size of the subspace iteration: R + 16 guard vectors, rounded up to
// 8; near the cap the guard shrinks, down to 4 vectors.
__host__ __device__ inline int64_t si_block_dev(int64_t n, int64_t R) {
    int64_t p = R + 16;
    p = (p + 7) / 8 * 8;
    if (p > SI_BLOCK_MAX && R + 4 <= SI_BLOCK_MAX) p = SI_BLOCK_MAX;
    return p < n ? p : n;
}
inline int64_t si_block_host(int64_t n, int64_t R) { return si_block_dev(n, R); }

constexpr int EIG_THREADS = 512;
constexpr int EIG_BATCH = 4;  // items per thread whose loads are issued before any store

__device__ __forceinline__ int rr_player(int x, int r, int ne) {
    // round-robin position x (0..ne-1) in round r (0..ne-2): player 0 fixed
    if (x == 0) return 0;
    int y = x - 1 + r;
    if (y >= ne - 1) y -= ne - 1;
    return y + 1;
}

// Rotation (c, s) that annihilates a_pq against the diagonal pair (a_pp,
// a_qq).  A rotation is skipped (identity, returns false) when a_pq is at
// the roundoff level: |a_pq| <= rel sqrt(|a_pp|) sqrt(|a_qq|) (its own
// diagonal pair, rel = n eps) or |a_pq| <= abs (abs = 4 eps ||A||_F, the
// error one rotation leaves in the entry it annihilates).  Rotating such an
// entry would only stir roundoff; a sweep in which every rotation is skipped
// ends the iteration (threshold Jacobi).
//
// With d = a_qq - a_pp the tangent of the smaller rotation angle is
//   t = 2 a_pq sgn(d) / (|d| + sqrt(d^2 + 4 a_pq^2))     (sgn(0) = +1),
// the classical t = sgn(theta) / (|theta| + sqrt(1 + theta^2)) with
// theta = d / (2 a_pq) multiplied through by |2 a_pq|; c = 1 / sqrt(1 + t^2)
// and s = t c.  One square root, one division and one reciprocal square root;
// when d^2 + 4 a_pq^2 leaves the FP64 range the theta form is used instead.
__device__ __forceinline__ bool jacobi_rotation(double app, double aqq, double apq, double rel,
                                                double abs_floor, double &c, double &s) {
    c = 1.0;
    s = 0.0;
    const double a = fabs(apq);
    if (a <= abs_floor || a <= rel * sqrt(fabs(app)) * sqrt(fabs(aqq))) return false;
    const double d = aqq - app;
    const double h = sqrt(d * d + 4.0 * apq * apq);
    double t;
    if (h <= 1.0e300) {
        t = (d >= 0.0 ? 2.0 * apq : -2.0 * apq) / (fabs(d) + h);
        c = rsqrt(1.0 + t * t);
    } else {
        const double theta = d / (2.0 * apq);
        t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
        c = 1.0 / sqrt(1.0 + t * t);
    }
    s = t * c;
    return true;
}

// ------------------------------------------------------------------------
// Small matrices (n <= 128, at most JS_MAXM pairs per round).  The same
// parallel round-robin sweep as jacobi_body, with A padded to an even order
// ne (a zero row and column: the odd player's partner, whose rotation is the
// identity, so no bound tests in the update) and a fixed work split computed
// once.  V does not feed the rotations, so its update lags one round behind:
// while wave 0 computes the rotations of round r from A, waves 1.. apply the
// rotations of round r - 1 to V (two sets of rotation parameters in LDS);
// then every thread applies round r to A.
//
// The round is bound by LDS latency, so every update first reads all the
// rotation parameters it needs (packed (p, q) and (c, s) pairs, indices
// clamped to a valid pair so that the reads need no branch), then all its
// matrix entries (predicated), then writes.  V is ne x ne with an even
// leading dimension and each thread of its update owns a pair of adjacent
// rows, so its entries move 16 bytes at a time.  A round whose rotations are
// all the identity (the last sweep of the threshold rule) updates nothing.
constexpr int JS_MAXM = 64;
constexpr int JS_VTHREADS = EIG_THREADS - 64;   // waves 1.. update V
constexpr int JS_CV = 4;                        // V pairs per batch of reads

// Dynamic LDS of jacobi_small_body: A (upper triangle of an ne x ne array
// with the odd leading dimension ne + 1) and, when v_lds, V (ne x ne).
__host__ __device__ inline size_t jacobi_small_lds(int64_t n, bool v_lds) {
    const int64_t ne = n + (n & 1);
    return (size_t)(ne * (ne + 1) + (v_lds ? ne * ne : 0)) * 8;
}
// Global V (when not in LDS): ne x ne doubles, 16-byte aligned.
__host__ __device__ inline size_t jacobi_small_vg(int64_t n) {
    const int64_t ne = n + (n & 1);
    return (size_t)(ne * ne) * 8;
}

// Position of the symmetric entry (r, c) in the stored upper triangle.
__device__ __forceinline__ int sym_at(int r, int c, int la) {
    return min(r, c) + la * max(r, c);
}

// A <- J^T A J for the rotations of `set`, on the upper triangle only: the
// m (m + 1) / 2 blocks of pair rows I <= pair columns J are dealt to the
// threads in row order, block b to thread b mod EIG_THREADS (the thread's
// blocks bI[k], bJ[k], k < nb, decoded once; unused slots hold pair 0).  A
// block's four entries are read from and written to their stored positions;
// in a diagonal block (I = J) the (1, 0) entry is the stored (0, 1) entry
// again, so its result goes to the unused lower slot.  The odd leading
// dimension keeps both access directions (consecutive rows or consecutive
// columns across a wave) free of bank conflicts.
constexpr int JS_SB = 5;   // blocks per thread: 64 * 65 / 2 = 2080 over 512 threads
template <int SB>
__device__ __forceinline__ void jacobi_small_update_sym(double *__restrict__ A, int la,
                                                        const int2 *__restrict__ pq,
                                                        const double2 *__restrict__ cs,
                                                        const int *bI, const int *bJ, int nb) {
    int r00[SB], r01[SB], r10[SB], r11[SB], w10[SB];
    double ci[SB], si[SB], cj[SB], sj[SB], a[SB][4];
#pragma unroll
    for (int k = 0; k < SB; ++k) {
        const int2 tI = pq[bI[k]], tJ = pq[bJ[k]];
        const double2 uI = cs[bI[k]], uJ = cs[bJ[k]];
        ci[k] = uI.x;
        si[k] = uI.y;
        cj[k] = uJ.x;
        sj[k] = uJ.y;
        r00[k] = sym_at(tI.x, tJ.x, la);
        r01[k] = sym_at(tI.x, tJ.y, la);
        r10[k] = sym_at(tI.y, tJ.x, la);
        r11[k] = sym_at(tI.y, tJ.y, la);
        w10[k] = bI[k] == bJ[k] ? tI.y + la * tI.x : r10[k];
    }
#pragma unroll
    for (int k = 0; k < SB; ++k) {
        if (k < nb) {
            a[k][0] = A[r00[k]];
            a[k][1] = A[r01[k]];
            a[k][2] = A[r10[k]];
            a[k][3] = A[r11[k]];
        } else {
            a[k][0] = a[k][1] = a[k][2] = a[k][3] = 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < SB; ++k)
        if (k < nb) {
            const double b00 = ci[k] * a[k][0] - si[k] * a[k][2], b01 = ci[k] * a[k][1] - si[k] * a[k][3];
            const double b10 = si[k] * a[k][0] + ci[k] * a[k][2], b11 = si[k] * a[k][1] + ci[k] * a[k][3];
            A[r00[k]] = cj[k] * b00 - sj[k] * b01;
            A[r01[k]] = sj[k] * b00 + cj[k] * b01;
            A[w10[k]] = cj[k] * b10 - sj[k] * b11;
            A[r11[k]] = sj[k] * b10 + cj[k] * b11;
        }
}

// V <- V J for the rotations of `set`: the thread owns rows (2 rp, 2 rp + 1)
// of the pairs jw0, jw0 + jw, ... (nkw of them).  V2 views V (ne x ne,
// leading dimension ne) as ne / 2 x ne pairs of doubles.
__device__ __forceinline__ void jacobi_small_update_v(double2 *__restrict__ V2, int nh, int m,
                                                      const int2 *__restrict__ pq,
                                                      const double2 *__restrict__ cs, int rp,
                                                      int jw0, int jw, int nkw) {
#pragma unroll 1
    for (int k0 = 0; k0 < nkw; k0 += JS_CV) {
        int pj[JS_CV], qj[JS_CV];
        double cj[JS_CV], sj[JS_CV];
        double2 vp[JS_CV], vq[JS_CV];
#pragma unroll
        for (int k = 0; k < JS_CV; ++k) {
            const int J = min(jw0 + (k0 + k) * jw, m - 1);
            const int2 t = pq[J];
            const double2 u = cs[J];
            pj[k] = rp + nh * t.x;
            qj[k] = rp + nh * t.y;
            cj[k] = u.x;
            sj[k] = u.y;
        }
#pragma unroll
        for (int k = 0; k < JS_CV; ++k) {
            if (k0 + k < nkw) {
                vp[k] = V2[pj[k]];
                vq[k] = V2[qj[k]];
            } else {
                vp[k] = vq[k] = make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int k = 0; k < JS_CV; ++k)
            if (k0 + k < nkw) {
                V2[pj[k]] = make_double2(cj[k] * vp[k].x - sj[k] * vq[k].x, cj[k] * vp[k].y - sj[k] * vq[k].y);
                V2[qj[k]] = make_double2(sj[k] * vp[k].x + cj[k] * vq[k].x, sj[k] * vp[k].y + cj[k] * vq[k].y);
            }
    }
}

template <bool VLDS>
__device__ __forceinline__ void jacobi_small_body(const double *__restrict__ S, int n, int R,
                                                  double *__restrict__ Vg, double *__restrict__ U,
                                                  double *__restrict__ lam, double tol,
                                                  int max_sweeps, int64_t *__restrict__ flag) {
    extern __shared__ __align__(16) double s_e[];   // 16-byte aligned: V is read 16 bytes at a time
    __shared__ int2 s_pq[2][JS_MAXM];
    __shared__ double2 s_cs[2][JS_MAXM];
    __shared__ int s_any[2];
    __shared__ double s_red[2][EIG_THREADS / 64];
    __shared__ int s_sel[2 * JS_MAXM];
    __shared__ double s_sign[2 * JS_MAXM];
    __shared__ int s_stop, s_rot;
    __shared__ double s_floor;

    const int ne = n + (n & 1), m = ne / 2;
    const double thresh = (double)n * 2.220446049250313e-16;
    const int la = ne + 1;                   // odd leading dimension of A
    double *A = s_e;                         // upper triangle of ne x ne, leading dimension la
    double *V = VLDS ? s_e + ne * la : Vg;   // ne x ne, leading dimension ne
    const int tid = threadIdx.x;
    for (int e0 = tid; e0 < ne * ne; e0 += 4 * EIG_THREADS) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {   // 8 global loads in flight per thread
            const int e = e0 + u * EIG_THREADS;
            const int i = e % ne, j = e / ne;
            v[u] = (e < ne * ne && i < n && j < n) ? 0.5 * (S[i + n * j] + S[j + n * i]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * EIG_THREADS;
            if (e < ne * ne) A[e % ne + la * (e / ne)] = v[u];
        }
    }
    for (int e = tid; e < ne * ne; e += EIG_THREADS) {
        const int i = e % ne, j = e / ne;
        V[e] = (i == j && i < n) ? 1.0 : 0.0;
    }
    // A: the thread's pair blocks (I, J), I <= J: b = tid + k EIG_THREADS in row order
    const int nblk = m * (m + 1) / 2;
    const int cap = (nblk + EIG_THREADS - 1) / EIG_THREADS;   // the most blocks of any thread
    int bI[JS_SB], bJ[JS_SB], nb = 0;
#pragma unroll
    for (int k = 0; k < JS_SB; ++k) {
        int b = tid + k * EIG_THREADS, I = 0;
        if (b < nblk) {
            while (b >= m - I) {
                b -= m - I;
                ++I;
            }
            nb = k + 1;
        } else {
            b = 0;
        }
        bI[k] = I;
        bJ[k] = I + b;
    }
    // V (waves 1..): thread owns row pair rp for the pairs jw0, jw0 + jw, ...
    const int tv = tid - 64;
    const int jw = JS_VTHREADS / m, rp = tv >= 0 ? tv % m : 0, jw0 = tv >= 0 ? tv / m : jw;
    const int nkw = (tv >= 0 && jw0 < jw) ? (m - jw0 + jw - 1) / jw : 0;
    double2 *V2 = reinterpret_cast<double2 *>(V);
    auto update_a = [&](int set) {
        if (cap <= 1) jacobi_small_update_sym<1>(A, la, s_pq[set], s_cs[set], bI, bJ, nb);
        else if (cap <= 2) jacobi_small_update_sym<2>(A, la, s_pq[set], s_cs[set], bI, bJ, nb);
        else if (cap <= 3) jacobi_small_update_sym<3>(A, la, s_pq[set], s_cs[set], bI, bJ, nb);
        else jacobi_small_update_sym<JS_SB>(A, la, s_pq[set], s_cs[set], bI, bJ, nb);
    };
    __syncthreads();

    int sweep = 0;
    bool converged = false;
    double prev_off2 = -1.0;
    for (;;) {
        double off = 0.0, fro = 0.0;   // over the stored triangle, off-diagonal entries twice
        for (int j = 0; j < n; ++j)
            for (int i = tid; i <= j; i += EIG_THREADS) {
                const double v = A[i + la * j];
                fro += (i == j ? 1.0 : 2.0) * v * v;
                if (i != j) off += 2.0 * v * v;
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
            else if (sweep > 0 && s_rot == 0) stop = 1;   // the last sweep rotated nothing
            else if (o2 <= (double)n * n * 1.2e-32 * f2 && prev_off2 >= 0.0 && o2 >= 0.25 * prev_off2) stop = 1;
            else if (sweep >= max_sweeps) stop = 2;
            s_stop = stop;
            s_rot = 0;
            s_floor = 4.0 * 2.220446049250313e-16 * sqrt(f2);
            s_red[0][0] = o2;
        }
        __syncthreads();
        if (s_stop) {
            converged = (s_stop == 1);
            break;
        }
        prev_off2 = s_red[0][0];
        for (int r = 0; r < ne - 1; ++r) {
            const int set = r & 1;
            if (tid < 64) {
                bool rot = false;
                if (tid < m) {
                    int p = rr_player(tid, r, ne), q = rr_player(ne - 1 - tid, r, ne);
                    if (p > q) {
                        const int t = p;
                        p = q;
                        q = t;
                    }
                    double c, sn;
                    rot = jacobi_rotation(A[p + la * p], A[q + la * q], A[p + la * q], thresh, s_floor, c, sn);
                    s_pq[set][tid] = make_int2(p, q);
                    s_cs[set][tid] = make_double2(c, sn);
                }
                const bool any = __ballot(rot) != 0;
                if (tid == 0) {
                    s_any[set] = any ? 1 : 0;
                    if (any) s_rot = 1;
                }
            } else if (r > 0 && s_any[set ^ 1]) {
                jacobi_small_update_v(V2, m, m, s_pq[set ^ 1], s_cs[set ^ 1], rp, jw0, jw, nkw);   // round r - 1
            }
            __syncthreads();
            if (s_any[set]) update_a(set);
            __syncthreads();
        }
        // the last round's V update
        if (tid >= 64 && s_any[(ne - 2) & 1])
            jacobi_small_update_v(V2, m, m, s_pq[(ne - 2) & 1], s_cs[(ne - 2) & 1], rp, jw0, jw, nkw);
        __syncthreads();
        ++sweep;
    }
    if (!converged && tid == 0 && flag) flag[0] = 1;

    // descending order of the diagonal, ties by index.  A NaN on the diagonal
    // (non-finite input) sorts last and raises flag 3, so that the ranks stay
    // a permutation of 0..n-1 and every selected column is in range.
    for (int i = tid; i < n; i += EIG_THREADS) {
        const double di = A[i + la * i];
        const double li = (di == di) ? di : -HUGE_VAL;
        if (di != di && flag) flag[0] = 3;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = A[j + la * j];
            const double lj = (dj == dj) ? dj : -HUGE_VAL;
            rank += (lj > li) || (lj == li && j < i);
        }
        if (rank < R) s_sel[rank] = i;
    }
    __syncthreads();
    for (int r = tid; r < R; r += EIG_THREADS) {
        const int col = s_sel[r];
        int arg = 0;
        double best = fabs(V[ne * col]);
        for (int i = 1; i < n; ++i) {
            const double v = fabs(V[i + ne * col]);
            if (v > best) {
                best = v;
                arg = i;
            }
        }
        s_sign[r] = V[arg + ne * col] < 0 ? -1.0 : 1.0;
        if (lam) lam[r] = A[col + la * col];
    }
    __syncthreads();
    for (int e = tid; e < n * R; e += EIG_THREADS) {
        const int i = e % n, r = e / n;
        U[e] = s_sign[r] * V[i + ne * s_sel[r]];
    }
}

template <bool ALDS, bool VLDS>
__device__ __forceinline__ void jacobi_body(const double *__restrict__ S, int n, int R,
                                            double *__restrict__ Ag, double *__restrict__ Vg,
                                            double *__restrict__ U, double *__restrict__ lam,
                                            double tol, int max_sweeps,
                                            int64_t *__restrict__ flag) {
    extern __shared__ __align__(16) double s_e[];   // 16-byte aligned: V is read 16 bytes at a time
    __shared__ double s_c[256], s_s[256];
    __shared__ int s_p[256], s_q[256];
    __shared__ double s_red[2][EIG_THREADS / 64];
    __shared__ int s_sel[512];
    __shared__ double s_sign[512];
    __shared__ int s_stop, s_rot;
    __shared__ double s_floor;
    const double thresh = (double)n * 2.220446049250313e-16;

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
            else if (sweep > 0 && s_rot == 0) stop = 1;   // the last sweep rotated nothing
            // roundoff floor: off(A) already at the FP64 noise level of an
            // n x n rotation sequence and no longer shrinking
            else if (o2 <= (double)n * n * 1.2e-32 * f2 && prev_off2 >= 0.0 && o2 >= 0.25 * prev_off2) stop = 1;
            else if (sweep >= max_sweeps) stop = 2;
            s_stop = stop;
            s_rot = 0;
            s_floor = 4.0 * 2.220446049250313e-16 * sqrt(f2);
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
                if (q < n && jacobi_rotation(A[p + n * p], A[q + n * q], A[p + n * q], thresh, s_floor, c, s))
                    s_rot = 1;
                s_p[k] = p;
                s_q[k] = q;
                s_c[k] = c;
                s_s[k] = s;
            }
            __syncthreads();
            // A <- J^T A J, block (I, J) of pairs; V <- V J.  Each thread takes
            // EIG_BATCH items at a time and issues all their loads before any
            // store (the items of a round are disjoint).
            const int nb = m * m;
            for (int e0 = tid; e0 < nb; e0 += EIG_BATCH * EIG_THREADS) {
                int pi[EIG_BATCH], qi[EIG_BATCH], pj[EIG_BATCH], qj[EIG_BATCH];
                double a[EIG_BATCH][4];
#pragma unroll
                for (int u = 0; u < EIG_BATCH; ++u) {
                    const int e = e0 + u * EIG_THREADS;
                    const int I = e % m, J = e / m;
                    pi[u] = -1;
                    if (e < nb) {
                        pi[u] = s_p[I];
                        qi[u] = s_q[I];
                        pj[u] = s_p[J];
                        qj[u] = s_q[J];
                        const bool vi = qi[u] < n, vj = qj[u] < n;
                        a[u][0] = A[pi[u] + n * pj[u]];
                        a[u][1] = vj ? A[pi[u] + n * qj[u]] : 0.0;
                        a[u][2] = vi ? A[qi[u] + n * pj[u]] : 0.0;
                        a[u][3] = (vi && vj) ? A[qi[u] + n * qj[u]] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < EIG_BATCH; ++u) {
                    if (pi[u] < 0) continue;
                    const int e = e0 + u * EIG_THREADS;
                    const int I = e % m, J = e / m;
                    const double ci = s_c[I], si = s_s[I], cj = s_c[J], sj = s_s[J];
                    const bool vi = qi[u] < n, vj = qj[u] < n;
                    // rows: p' = c p - s q, q' = s p + c q; then the same on columns
                    const double b00 = ci * a[u][0] - si * a[u][2], b01 = ci * a[u][1] - si * a[u][3];
                    const double b10 = si * a[u][0] + ci * a[u][2], b11 = si * a[u][1] + ci * a[u][3];
                    A[pi[u] + n * pj[u]] = cj * b00 - sj * b01;
                    if (vj) A[pi[u] + n * qj[u]] = sj * b00 + cj * b01;
                    if (vi) A[qi[u] + n * pj[u]] = cj * b10 - sj * b11;
                    if (vi && vj) A[qi[u] + n * qj[u]] = sj * b10 + cj * b11;
                }
            }
            const int nv = n * m;
            for (int e0 = tid; e0 < nv; e0 += EIG_BATCH * EIG_THREADS) {
                int row[EIG_BATCH], pj[EIG_BATCH], qj[EIG_BATCH];
                double vp[EIG_BATCH], vq[EIG_BATCH];
#pragma unroll
                for (int u = 0; u < EIG_BATCH; ++u) {
                    const int e = e0 + u * EIG_THREADS;
                    row[u] = -1;
                    if (e < nv) {
                        const int J = e / n;
                        if (s_q[J] < n) {
                            row[u] = e - J * n;
                            pj[u] = s_p[J];
                            qj[u] = s_q[J];
                            vp[u] = V[row[u] + n * pj[u]];
                            vq[u] = V[row[u] + n * qj[u]];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < EIG_BATCH; ++u) {
                    if (row[u] < 0) continue;
                    const int J = (e0 + u * EIG_THREADS) / n;
                    const double cj = s_c[J], sj = s_s[J];
                    V[row[u] + n * pj[u]] = cj * vp[u] - sj * vq[u];
                    V[row[u] + n * qj[u]] = sj * vp[u] + cj * vq[u];
                }
            }
            __syncthreads();
        }
        ++sweep;
    }
    if (!converged && tid == 0 && flag) flag[0] = 1;

    // descending order of the diagonal, ties by index (NaN last, flag 3;
    // the ranks stay a permutation, so every selected column is in range)
    for (int i = tid; i < n; i += EIG_THREADS) {
        const double di = A[i + n * i];
        const double li = (di == di) ? di : -HUGE_VAL;
        if (di != di && flag) flag[0] = 3;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = A[j + n * j];
            const double lj = (dj == dj) ? dj : -HUGE_VAL;
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

}  // namespace sth
