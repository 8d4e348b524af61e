// Host side of the C ABI: validation, plans, workspace layout and the
// mode-wise driver of Alg. 2 (EIG branch: Gram -> FP64 eigensolver -> TTM;
// ALS branch: Alg. 3 sweeps -> QR -> TTM).  Every numeric step runs in the
// library's HIP kernels; this file only computes shapes and enqueues work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sthosvd.h"
#include "internal.h"
#include "selector.h"

using namespace sth;

// ------------------------------------------------------------ errors ----

static thread_local std::string g_err = "no error";

static sth_status fail(sth_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

static sth_status hip_fail(hipError_t e, const char *what) {
    return fail(STH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(expr, what)                       \
    do {                                         \
        hipError_t _e = (expr);                  \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

extern "C" const char *sth_last_error(void) { return g_err.c_str(); }
extern "C" const char *sth_version(void) { return "sthosvd-gfx950 0.1"; }

namespace sth {
int device_cu_count() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (cache[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
            cu = 256;
        cache[dev] = cu;
    }
    return cache[dev];
}
}  // namespace sth

// ------------------------------------------------------- validation ----

static const int MAX_ORDER = 8;
static const int64_t MAX_EIG_N = SEL_MAX_EIG_N;   // I_n x I_n Gram and eigensolver
static const int64_t MAX_ALS_R = SEL_MAX_ALS_R;   // R x R Cholesky in LDS

static size_t esize(int dtype) { return dtype == STH_F64 ? 8 : 4; }
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static sth_status check_shape(int32_t order, const int64_t *dims) {
    if (order < 1 || order > MAX_ORDER) return fail(STH_ERR_INVALID, "order %d outside 1..%d", order, MAX_ORDER);
    if (!dims) return fail(STH_ERR_INVALID, "dims is NULL");
    double numel = 1.0;
    for (int k = 0; k < order; ++k) {
        if (dims[k] < 1) return fail(STH_ERR_INVALID, "dims[%d] = %lld < 1", k, (long long)dims[k]);
        numel *= (double)dims[k];
    }
    if (numel > 9.0e15) return fail(STH_ERR_INVALID, "tensor too large");
    return STH_OK;
}

static sth_status check_dtype_prec(int32_t dtype, int32_t prec, const char *what) {
    if (dtype != STH_F64 && dtype != STH_F32) return fail(STH_ERR_INVALID, "dtype %d", dtype);
    if (prec < STH_PREC_FP64 || prec > STH_PREC_BF16X6) return fail(STH_ERR_INVALID, "%s %d", what, prec);
    if (dtype == STH_F64 && prec != STH_PREC_FP64)
        return fail(STH_ERR_INVALID, "FP64 data needs %s = STH_PREC_FP64", what);
    return STH_OK;
}

static sth_status check_ptr(const void *p, const char *what, bool allow_null = false) {
    if (!p) return allow_null ? STH_OK : fail(STH_ERR_INVALID, "%s is NULL", what);
    if (reinterpret_cast<uintptr_t>(p) & 15) return fail(STH_ERR_LAYOUT, "%s is not 16-byte aligned", what);
    return STH_OK;
}

// (L, I, M) of mode n
static void lim(int order, const int64_t *dims, int n, int64_t &L, int64_t &I, int64_t &M) {
    L = 1;
    M = 1;
    for (int k = 0; k < n; ++k) L *= dims[k];
    I = dims[n];
    for (int k = n + 1; k < order; ++k) M *= dims[k];
}

// -------------------------------------------------------------- plan ----

struct Step {
    int n;
    int64_t L, I, M, R;
    int solver;
    bool chosen;   // solver picked by the selector (the memory model may move it to ALS)
    int src, dst;  // 0 = X, 1 = buffer A, 2 = buffer B, 3 = core
};

struct Arena {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    }
};

struct sth_plan_s {
    int N;
    std::vector<int64_t> dims, ranks;
    std::vector<int> order;
    int dtype, gram_prec, ttm_prec, als_iters, max_sweeps;
    std::vector<Step> steps;
    std::vector<int> solver_of_mode;
    // workspace offsets
    size_t o_flag, o_bufA, o_bufB, o_bufZ, o_part, o_S, o_eig, o_uq, o_small, o_gemm, o_sum, total;
    size_t small_bytes;
};

static int ttm_prec_of(const sth_plan_s &p) { return p.dtype == STH_F64 ? STH_PREC_FP64 : p.ttm_prec; }
static int gram_prec_of(const sth_plan_s &p) { return p.dtype == STH_F64 ? STH_PREC_FP64 : p.gram_prec; }

// ALS small-matrix scratch (doubles): Q, P, Lk, T1 (I x R each); C, Rc, Rcinv,
// G2, R1, R1inv, R2, R2inv, Rhat (R x R each); L0 (I x R).
static size_t als_small_doubles(int64_t I, int64_t R) { return (size_t)(5 * I * R + 9 * R * R); }

static sth_status make_plan(const sth_desc *d, int max_steps, sth_plan **plan_out, size_t *ws_out);

// Workspace bytes a step needs for the EIG branch beyond the ping-pong
// buffers: the Gram partial sums, the I_n x I_n Gram and the eigensolver.
static size_t eig_step_bytes(const sth_plan_s &p, const Step &st) {
    (void)p;
    return gram_ws_bytes(st.I, st.I, st.L * st.M, true) + (size_t)(st.I * st.I) * sizeof(double) + eig_ws_bytes(st.I);
}

// Workspace offsets of a plan from its steps and their solvers.
static void plan_layout(sth_plan_s &pl) {
    size_t maxA = 0, maxB = 0, maxZ = 0, maxPart = 0, maxS = 0, maxEig = 0, maxUq = 0, maxSmall = 0, maxGemm = 0;
    const int tp = ttm_prec_of(pl);
    for (const Step &stp : pl.steps) {
        const size_t out_elems = (size_t)(stp.L * stp.R * stp.M);
        if (stp.dst == 1) maxA = std::max(maxA, out_elems);
        if (stp.dst == 2) maxB = std::max(maxB, out_elems);
        const int64_t P = stp.L * stp.M;
        if (stp.solver == STH_SOLVER_EIG) {
            maxPart = std::max(maxPart, gram_ws_bytes(stp.I, stp.I, P, true));
            maxS = std::max(maxS, (size_t)(stp.I * stp.I) * sizeof(double));
            maxEig = std::max(maxEig, eig_ws_bytes(stp.I));
            maxUq = std::max(maxUq, ttm_prep_bytes(stp.I, stp.R, tp));
        } else {
            maxZ = std::max(maxZ, out_elems);
            maxPart = std::max(maxPart, gram_ws_bytes(stp.I, stp.R, P, false));
            maxUq = std::max(maxUq, std::max(ttm_prep_bytes(stp.I, stp.R, tp), ttm_prep_bytes(stp.R, stp.R, tp)));
            maxSmall = std::max(maxSmall, als_small_doubles(stp.I, stp.R) * sizeof(double));
            const int I = (int)stp.I, R = (int)stp.R;
            maxGemm = std::max({maxGemm, gemm_ws_bytes(R, R, I), gemm_ws_bytes(I, R, R), gemm_ws_bytes(R, R, R)});
        }
    }
    Arena a;
    pl.o_flag = a.take(256);
    pl.o_bufA = a.take(maxA * esize(pl.dtype));
    pl.o_bufB = a.take(maxB * esize(pl.dtype));
    pl.o_bufZ = a.take(maxZ * esize(pl.dtype));
    pl.o_part = a.take(maxPart);
    pl.o_S = a.take(maxS);
    pl.o_eig = a.take(maxEig);
    pl.o_uq = a.take(maxUq);
    pl.o_small = a.take(maxSmall);
    pl.o_gemm = a.take(maxGemm);
    pl.o_sum = a.take(SUMSQ_BLOCKS * sizeof(double));
    pl.total = a.off;
}

extern "C" sth_status sthosvd_plan(const sth_desc *d, sth_plan **plan_out, size_t *ws_out) {
    return make_plan(d, MAX_ORDER, plan_out, ws_out);
}

static sth_status make_plan(const sth_desc *d, int max_steps, sth_plan **plan_out, size_t *ws_out) {
    if (!d || !plan_out || !ws_out) return fail(STH_ERR_INVALID, "NULL argument");
    *plan_out = nullptr;
    sth_status st = check_shape(d->order, d->dims);
    if (st) return st;
    if (!d->ranks) return fail(STH_ERR_INVALID, "ranks is NULL");
    const int N = d->order;
    for (int k = 0; k < N; ++k)
        if (d->ranks[k] < 1 || d->ranks[k] > d->dims[k])
            return fail(STH_ERR_INVALID, "ranks[%d] = %lld outside 1..%lld", k, (long long)d->ranks[k], (long long)d->dims[k]);
    if ((st = check_dtype_prec(d->dtype, d->gram_prec, "gram_prec"))) return st;
    if ((st = check_dtype_prec(d->dtype, d->ttm_prec, "ttm_prec"))) return st;
    std::vector<int> order(N);
    if (d->mode_order) {
        std::vector<int> seen(N, 0);
        for (int k = 0; k < N; ++k) {
            int m = d->mode_order[k];
            if (m < 0 || m >= N || seen[m]) return fail(STH_ERR_INVALID, "mode_order is not a permutation");
            seen[m] = 1;
            order[k] = m;
        }
    } else {
        for (int k = 0; k < N; ++k) order[k] = k;
    }
    if (d->solver < STH_SOLVER_EIG || d->solver > STH_SOLVER_AUTO_TREE) return fail(STH_ERR_INVALID, "solver %d", d->solver);
    if (d->als_iters < 0) return fail(STH_ERR_INVALID, "als_iters < 0");
    if (d->eig_max_sweeps < 0) return fail(STH_ERR_INVALID, "eig_max_sweeps < 0");

    sth_plan_s *p = new sth_plan_s();
    p->N = N;
    p->dims.assign(d->dims, d->dims + N);
    p->ranks.assign(d->ranks, d->ranks + N);
    p->order = order;
    p->dtype = d->dtype;
    p->gram_prec = d->gram_prec;
    p->ttm_prec = d->ttm_prec;
    p->als_iters = d->als_iters ? d->als_iters : 5;
    p->max_sweeps = d->eig_max_sweeps ? d->eig_max_sweeps : 60;
    p->solver_of_mode.assign(N, STH_SOLVER_EIG);

    // shapes on the current working tensor, solver choice (Alg. 2 line 3)
    std::vector<int64_t> cur = p->dims;
    const int nsteps = std::min(N, max_steps);
    for (int s = 0; s < nsteps; ++s) {
        Step stp;
        stp.n = order[s];
        lim(N, cur.data(), stp.n, stp.L, stp.I, stp.M);
        stp.R = p->ranks[stp.n];
        int solver = d->solver;
        if (d->per_mode) {
            solver = d->per_mode[stp.n];
            if (solver != STH_SOLVER_EIG && solver != STH_SOLVER_ALS && solver != STH_SOLVER_AUTO &&
                solver != STH_SOLVER_AUTO_TREE) {
                delete p;
                return fail(STH_ERR_INVALID, "per_mode[%d] = %d", stp.n, solver);
            }
        }
        const bool chosen = solver == STH_SOLVER_AUTO || solver == STH_SOLVER_AUTO_TREE;
        if (solver == STH_SOLVER_AUTO) {
            solver = selector_choose(stp.I, stp.R, stp.L * stp.M, N, d->mlp_weights);
        } else if (solver == STH_SOLVER_AUTO_TREE) {
            solver = selector_tree_choose(stp.I, stp.R, stp.L * stp.M);
        }
        if (solver == STH_SOLVER_EIG && stp.I > MAX_EIG_N) {
            delete p;
            return fail(STH_ERR_UNSUPPORTED, "EIG mode %d: I_n = %lld exceeds the eigensolver limit %lld (use ALS)", stp.n, (long long)stp.I, (long long)MAX_EIG_N);
        }
        if (solver == STH_SOLVER_ALS && stp.R > MAX_ALS_R) {
            delete p;
            return fail(STH_ERR_UNSUPPORTED, "ALS mode %d: R_n = %lld exceeds %lld", stp.n, (long long)stp.R, (long long)MAX_ALS_R);
        }
        if (solver == STH_SOLVER_ALS && stp.R > stp.L * stp.M) {
            delete p;
            return fail(STH_ERR_UNSUPPORTED, "ALS mode %d: R_n = %lld exceeds the rank bound %lld of the unfolding (its normal equations are singular; use EIG)", stp.n, (long long)stp.R, (long long)(stp.L * stp.M));
        }
        stp.solver = solver;
        stp.chosen = chosen;
        stp.src = (s == 0) ? 0 : ((s - 1) % 2 == 0 ? 1 : 2);
        stp.dst = (s == nsteps - 1) ? 3 : (s % 2 == 0 ? 1 : 2);
        cur[stp.n] = stp.R;
        p->steps.push_back(stp);
    }
    plan_layout(*p);
    // memory model: over the cap, the modes the selector sent to EIG move to
    // ALS (where ALS applies), the one with the largest EIG footprint (the
    // I_n^2 Gram, its partial sums and the eigensolver scratch) first
    while (d->workspace_cap > 0 && p->total > (size_t)d->workspace_cap) {
        Step *best = nullptr;
        size_t best_bytes = 0;
        for (Step &st : p->steps) {
            if (!st.chosen || st.solver != STH_SOLVER_EIG) continue;
            if (st.R > MAX_ALS_R || st.R > st.L * st.M) continue;
            const size_t b = eig_step_bytes(*p, st);
            if (!best || b > best_bytes) {
                best = &st;
                best_bytes = b;
            }
        }
        if (!best) break;
        best->solver = STH_SOLVER_ALS;
        plan_layout(*p);
    }
    for (const Step &st : p->steps) p->solver_of_mode[st.n] = st.solver;
    if (d->workspace_cap > 0 && p->total > (size_t)d->workspace_cap) {
        size_t need = p->total;
        delete p;
        return fail(STH_ERR_NOMEM, "workspace %zu bytes exceeds the cap %lld", need, (long long)d->workspace_cap);
    }
    *plan_out = p;
    *ws_out = p->total;
    return STH_OK;
}

extern "C" sth_status sthosvd_plan_solvers(const sth_plan *plan, int32_t *out) {
    if (!plan || !out) return fail(STH_ERR_INVALID, "NULL argument");
    for (int k = 0; k < plan->N; ++k) out[k] = plan->solver_of_mode[k];
    return STH_OK;
}

extern "C" void sthosvd_plan_destroy(sth_plan *plan) { delete plan; }

// ---------------------------------------------------------------- ALS ----

namespace {

struct AlsBufs {
    double *Q, *P, *Lk, *T1, *L0, *C, *Rc, *Rcinv, *G2, *R1, *R1inv, *R2, *R2inv, *Rhat;
};

AlsBufs als_bufs(double *base, int64_t I, int64_t R) {
    AlsBufs b;
    double *p = base;
    auto take = [&](int64_t n) { double *r = p; p += n; return r; };
    b.Q = take(I * R);
    b.P = take(I * R);
    b.Lk = take(I * R);
    b.T1 = take(I * R);
    b.L0 = take(I * R);
    b.C = take(R * R);
    b.Rc = take(R * R);
    b.Rcinv = take(R * R);
    b.G2 = take(R * R);
    b.R1 = take(R * R);
    b.R1inv = take(R * R);
    b.R2 = take(R * R);
    b.R2inv = take(R * R);
    b.Rhat = take(R * R);
    return b;
}

// Shifted Cholesky-QR3 of the I x R matrix A: Q = A R^{-1} with R = R3 R2 R1
// upper triangular with a positive diagonal.  The first pass factors
// A^T A + s I (s = 11 (I R + R (R + 1)) u ||A||_F^2, u = 2^-53), which exists
// for any condition number up to ~1/u and leaves A R1^{-1} well conditioned;
// two plain passes then make the columns orthonormal to working accuracy.
// The bases of the ALS sweeps need this: on steeply decaying spectra (the
// 2^-k core of the 4-way workload) L_k has a condition number near 1e9,
// beyond what plain Cholesky-QR twice tolerates.  Uses b.T1, b.P, b.G2 and
// the R x R buffers; Q may alias nothing in A.
hipError_t cholqr3(const double *A, int I, int R, double *Q, double *Rfac, AlsBufs &b, void *gws,
                   int64_t *flag, hipStream_t s) {
    hipError_t e;
    const double shift = 11.0 * ((double)I * R + (double)R * (R + 1)) * 1.1102230246251565e-16 * R;
    if ((e = gemm_f64(1, 0, R, R, I, 1.0, A, I, A, I, 0.0, b.G2, R, gws, s))) return e;
    if ((e = chol_launch(b.G2, R, R, shift, b.R1, b.R1inv, flag, s))) return e;
    if ((e = gemm_f64(0, 0, I, R, R, 1.0, A, I, b.R1inv, R, 0.0, b.T1, I, gws, s))) return e;
    if ((e = gemm_f64(1, 0, R, R, I, 1.0, b.T1, I, b.T1, I, 0.0, b.G2, R, gws, s))) return e;
    if ((e = chol_launch(b.G2, R, R, 0.0, b.R2, b.R2inv, flag, s))) return e;
    if ((e = gemm_f64(0, 0, I, R, R, 1.0, b.T1, I, b.R2inv, R, 0.0, b.P, I, gws, s))) return e;
    if ((e = gemm_f64(1, 0, R, R, I, 1.0, b.P, I, b.P, I, 0.0, b.G2, R, gws, s))) return e;
    if ((e = chol_launch(b.G2, R, R, 0.0, b.Rc, b.Rcinv, flag, s))) return e;
    if ((e = gemm_f64(0, 0, I, R, R, 1.0, b.P, I, b.Rcinv, R, 0.0, Q, I, gws, s))) return e;
    if (Rfac) {
        if ((e = gemm_f64(0, 0, R, R, R, 1.0, b.R2, R, b.R1, R, 0.0, b.C, R, gws, s))) return e;
        if ((e = gemm_f64(0, 0, R, R, R, 1.0, b.Rc, R, b.C, R, 0.0, Rfac, R, gws, s))) return e;
    }
    return hipSuccess;
}

}  // namespace

// One mode of Alg. 2 on the working tensor src (L, I, M) -> dst (L, R, M).
static sth_status exec_step(const sth_plan_s &pl, const Step &stp, const void *src, void *dst,
                            double *Un, double *lam, const double *L0in, uint64_t seed, char *w,
                            hipStream_t s) {
    const sth_plan_s *p = &pl;
    int64_t *flag = (int64_t *)(w + p->o_flag);
    void *bufZ = w + p->o_bufZ;
    double *part = (double *)(w + p->o_part);
    double *S = (double *)(w + p->o_S);
    void *eigws = w + p->o_eig;
    void *uq = w + p->o_uq;
    void *gws = w + p->o_gemm;
    const int gp = gram_prec_of(*p), tp = ttm_prec_of(*p);
    const int n = stp.n;
    if (stp.solver == STH_SOLVER_EIG) {
        // Alg. 2 lines 6-8
        HIPCHK(gram_launch(p->dtype, gp, src, src, stp.L, stp.I, stp.I, stp.M, true, part, S, s), "gram");
        HIPCHK(eig_launch(stp.I, stp.R, S, Un, lam, 1e-15, p->max_sweeps, eigws, flag, s, stp.L * stp.M, false,
                          gram_unit(gp)),
               "eig");
        HIPCHK(ttm_prep_u(Un, stp.I, stp.R, 0, tp, uq, s), "ttm prep");
        HIPCHK(ttm_launch(p->dtype, tp, src, uq, dst, stp.L, stp.I, stp.R, stp.M, s), "ttm");
        return STH_OK;
    }
    // Alg. 2 lines 10-13 with Alg. 3 (L_k re-orthonormalized before each sweep)
    const int I = (int)stp.I, R = (int)stp.R;
    AlsBufs b = als_bufs((double *)(w + p->o_small), I, R);
    const double *L0 = L0in;
    if (!L0) {
        HIPCHK(gaussian_f64(b.L0, (int64_t)I * R, seed, (uint64_t)n, s), "als init");
        L0 = b.L0;
    }
    HIPCHK(cholqr3(L0, I, R, b.Q, nullptr, b, gws, flag, s), "als qr0");
    for (int k = 0; k < p->als_iters; ++k) {
        // Z = Y x_n Q^T  (R_k as a tensor)
        HIPCHK(ttm_prep_u(b.Q, I, R, 0, tp, uq, s), "als prep");
        HIPCHK(ttm_launch(p->dtype, tp, src, uq, bufZ, stp.L, I, R, stp.M, s), "als ttm");
        // P = Y_(n) Z_(n)^T  (TTT)
        HIPCHK(gram_launch(p->dtype, gp, src, bufZ, stp.L, I, R, stp.M, false, part, b.P, s), "als ttt");
        // C = R_k^T R_k = Q^T P ;  L_{k+1} = P C^{-1}
        HIPCHK(gemm_f64(1, 0, R, R, I, 1.0, b.Q, I, b.P, I, 0.0, b.C, R, gws, s), "als C");
        HIPCHK(chol_launch(b.C, R, R, 0.0, b.Rc, b.Rcinv, flag, s), "als chol");
        HIPCHK(gemm_f64(0, 0, I, R, R, 1.0, b.P, I, b.Rcinv, R, 0.0, b.T1, I, gws, s), "als L1");
        HIPCHK(gemm_f64(0, 1, I, R, R, 1.0, b.T1, I, b.Rcinv, R, 0.0, b.Lk, I, gws, s), "als L2");
        const bool last = (k + 1 == p->als_iters);
        // next basis, or the final Q^ R^ = L
        HIPCHK(cholqr3(b.Lk, I, R, last ? Un : b.Q, last ? b.Rhat : nullptr, b, gws, flag, s), "als qr");
    }
    // core update: Y' = R x_n R^  (Z'(a, r, b) = sum_s R^(r, s) Z(a, s, b))
    HIPCHK(ttm_prep_u(b.Rhat, R, R, 1, tp, uq, s), "als core prep");
    HIPCHK(ttm_launch(p->dtype, tp, bufZ, uq, dst, stp.L, R, R, stp.M, s), "als core ttm");
    return STH_OK;
}

// ---------------------------------------------------------------- run ----

extern "C" sth_status sthosvd_run(const sth_plan *p, const void *X, void *core, double *const *U,
                                  double *const *eigvals, const double *const *als_init,
                                  uint64_t seed, void *ws, size_t ws_bytes, sth_stream_t stream) {
    if (!p) return fail(STH_ERR_INVALID, "plan is NULL");
    sth_status st;
    if ((st = check_ptr(X, "X"))) return st;
    if ((st = check_ptr(core, "core"))) return st;
    if ((st = check_ptr(ws, "workspace"))) return st;
    if (!U) return fail(STH_ERR_INVALID, "U is NULL");
    for (int k = 0; k < p->N; ++k) {
        if ((st = check_ptr(U[k], "U[n]"))) return st;
        if (eigvals && eigvals[k] && (st = check_ptr(eigvals[k], "eigvals[n]"))) return st;
        if (als_init && als_init[k] && (st = check_ptr(als_init[k], "als_init[n]"))) return st;
    }
    if (ws_bytes < p->total) return fail(STH_ERR_NOMEM, "workspace %zu < required %zu bytes", ws_bytes, p->total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int64_t *flag = (int64_t *)(w + p->o_flag);
    char *bufA = w + p->o_bufA, *bufB = w + p->o_bufB;
    HIPCHK(zero_words(flag, 8, s), "flag clear");

    for (const Step &stp : p->steps) {
        const void *src = stp.src == 0 ? X : (stp.src == 1 ? (const void *)bufA : (const void *)bufB);
        void *dst = stp.dst == 3 ? core : (stp.dst == 1 ? (void *)bufA : (void *)bufB);
        const int n = stp.n;
        sth_status st2 = exec_step(*p, stp, src, dst, U[n], eigvals ? eigvals[n] : nullptr,
                                   als_init ? als_init[n] : nullptr, seed, w, s);
        if (st2) return st2;
    }
    return STH_OK;
}

extern "C" sth_status sthosvd_check(const sth_plan *p, void *ws, sth_stream_t stream) {
    if (!p || !ws) return fail(STH_ERR_INVALID, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int64_t flag = 0;
    int64_t *dflag = (int64_t *)((char *)ws + p->o_flag);
    HIPCHK(hipStreamSynchronize(s), "sync");
    HIPCHK(hipMemcpy(&flag, dflag, sizeof(flag), hipMemcpyDeviceToHost), "flag read");
    int64_t zero = 0;
    HIPCHK(hipMemcpy(dflag, &zero, sizeof(zero), hipMemcpyHostToDevice), "flag clear");
    if (flag == 1) return fail(STH_ERR_NUMERIC, "eigensolver hit its sweep cap");
    if (flag == 2) return fail(STH_ERR_NUMERIC, "Cholesky met a non-positive pivot (rank-deficient ALS basis)");
    if (flag == 3) return fail(STH_ERR_NUMERIC, "NaN or Inf met");
    if (flag) return fail(STH_ERR_NUMERIC, "numeric flag %lld", (long long)flag);
    return STH_OK;
}

// ------------------------------------------------------ building blocks ----

extern "C" size_t gram_mode_n_workspace(int32_t order, const int64_t *dims, int32_t n, int32_t other_rows) {
    if (check_shape(order, dims) || n < 0 || n >= order) return 0;
    int64_t L, I, M;
    lim(order, dims, n, L, I, M);
    if (other_rows > 0) return align_up(gram_ws_bytes(I, other_rows, L * M, false));
    return align_up(gram_ws_bytes(I, I, L * M, true));
}

extern "C" sth_status gram_mode_n(int32_t order, const int64_t *dims, int32_t n, int32_t dtype,
                                  int32_t prec, const void *Y, double *S, void *ws, size_t ws_bytes,
                                  sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (n < 0 || n >= order) return fail(STH_ERR_INVALID, "mode %d outside 0..%d", n, order - 1);
    if ((st = check_dtype_prec(dtype, prec, "prec"))) return st;
    if ((st = check_ptr(Y, "Y")) || (st = check_ptr(S, "S")) || (st = check_ptr(ws, "ws"))) return st;
    int64_t L, I, M;
    lim(order, dims, n, L, I, M);
    size_t need = gram_ws_bytes(I, I, L * M, true);
    if (ws_bytes < need) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    HIPCHK(gram_launch(dtype, prec, Y, Y, L, I, I, M, true, (double *)ws, S, (hipStream_t)stream), "gram");
    return STH_OK;
}

extern "C" sth_status ttt_mode_n(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                                 int32_t dtype, int32_t prec, const void *Y, const void *Z, double *P,
                                 void *ws, size_t ws_bytes, sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (n < 0 || n >= order) return fail(STH_ERR_INVALID, "mode %d outside 0..%d", n, order - 1);
    if (R < 1) return fail(STH_ERR_INVALID, "R < 1");
    if ((st = check_dtype_prec(dtype, prec, "prec"))) return st;
    if ((st = check_ptr(Y, "Y")) || (st = check_ptr(Z, "Z")) || (st = check_ptr(P, "P")) || (st = check_ptr(ws, "ws"))) return st;
    int64_t L, I, M;
    lim(order, dims, n, L, I, M);
    size_t need = gram_ws_bytes(I, R, L * M, false);
    if (ws_bytes < need) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    HIPCHK(gram_launch(dtype, prec, Y, Z, L, I, R, M, false, (double *)ws, P, (hipStream_t)stream), "ttt");
    return STH_OK;
}

extern "C" size_t ttm_mode_n_workspace(int64_t I, int64_t R) {
    if (I < 1 || R < 1) return 0;
    return align_up(ttm_prep_bytes(I, R, STH_PREC_FP64));  // the largest precision
}

extern "C" sth_status ttm_mode_n(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                                 int32_t dtype, int32_t prec, const void *Y, const double *U,
                                 int32_t transpose_u, void *Z, void *ws, size_t ws_bytes,
                                 sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (n < 0 || n >= order) return fail(STH_ERR_INVALID, "mode %d outside 0..%d", n, order - 1);
    if (R < 1) return fail(STH_ERR_INVALID, "R < 1");
    if ((st = check_dtype_prec(dtype, prec, "prec"))) return st;
    if ((st = check_ptr(Y, "Y")) || (st = check_ptr(U, "U")) || (st = check_ptr(Z, "Z")) || (st = check_ptr(ws, "ws"))) return st;
    int64_t L, I, M;
    lim(order, dims, n, L, I, M);
    size_t need = ttm_prep_bytes(I, R, prec);
    if (ws_bytes < need) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(ttm_prep_u(U, I, R, transpose_u ? 1 : 0, prec, ws, s), "ttm prep");
    HIPCHK(ttm_launch(dtype, prec, Y, ws, Z, L, I, R, M, s), "ttm");
    return STH_OK;
}

extern "C" size_t ttm_mode_n_noalloc_max_bytes(void) { return ttm_scratch_bytes(); }

extern "C" sth_status ttm_mode_n_noalloc(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                                         int32_t dtype, int32_t prec, const void *Y, const double *U,
                                         int32_t transpose_u, void *Z, sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (n < 0 || n >= order) return fail(STH_ERR_INVALID, "mode %d outside 0..%d", n, order - 1);
    if (R < 1) return fail(STH_ERR_INVALID, "R < 1");
    if ((st = check_dtype_prec(dtype, prec, "prec"))) return st;
    if ((st = check_ptr(Y, "Y")) || (st = check_ptr(U, "U")) || (st = check_ptr(Z, "Z"))) return st;
    int64_t L, I, M;
    lim(order, dims, n, L, I, M);
    const size_t need = ttm_prep_bytes(I, R, prec);
    if (need > ttm_scratch_bytes())
        return fail(STH_ERR_NOMEM, "the pre-split %lld x %lld factor needs %zu bytes, above the library scratch of %zu bytes (use ttm_mode_n)",
                    (long long)I, (long long)R, need, ttm_scratch_bytes());
    void *scr = nullptr;
    HIPCHK(ttm_scratch_ptr(&scr), "scratch address");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(ttm_prep_u(U, I, R, transpose_u ? 1 : 0, prec, scr, s), "ttm prep");
    HIPCHK(ttm_launch(dtype, prec, Y, scr, Z, L, I, R, M, s), "ttm");
    return STH_OK;
}

extern "C" size_t ttm_factor_bytes(int64_t I, int64_t R, int32_t prec) {
    if (I < 1 || R < 1 || prec < STH_PREC_FP64 || prec > STH_PREC_BF16X6) return 0;
    return ttm_prep_bytes(I, R, prec);
}

extern "C" sth_status ttm_factor_prepare(int64_t I, int64_t R, int32_t prec, const double *U,
                                         int32_t transpose_u, void *out, size_t out_bytes,
                                         sth_stream_t stream) {
    if (I < 1 || R < 1) return fail(STH_ERR_INVALID, "factor %lld x %lld", (long long)I, (long long)R);
    sth_status st;
    if ((st = check_dtype_prec(STH_F32, prec, "prec"))) return st;
    if ((st = check_ptr(U, "U")) || (st = check_ptr(out, "out"))) return st;
    size_t need = ttm_prep_bytes(I, R, prec);
    if (out_bytes < need) return fail(STH_ERR_NOMEM, "prepared factor %zu < %zu bytes", out_bytes, need);
    HIPCHK(ttm_prep_u(U, I, R, transpose_u ? 1 : 0, prec, out, (hipStream_t)stream), "ttm prep");
    return STH_OK;
}

extern "C" sth_status ttm_mode_n_prepared(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                                          int32_t dtype, int32_t prec, const void *Y,
                                          const void *Uprep, size_t uprep_bytes, void *Z,
                                          sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (n < 0 || n >= order) return fail(STH_ERR_INVALID, "mode %d outside 0..%d", n, order - 1);
    if (R < 1) return fail(STH_ERR_INVALID, "R < 1");
    if ((st = check_dtype_prec(dtype, prec, "prec"))) return st;
    if ((st = check_ptr(Y, "Y")) || (st = check_ptr(Uprep, "Uprep")) || (st = check_ptr(Z, "Z"))) return st;
    int64_t L, I, M;
    lim(order, dims, n, L, I, M);
    size_t need = ttm_prep_bytes(I, R, prec);
    if (uprep_bytes < need) return fail(STH_ERR_INVALID, "prepared factor %zu < %zu bytes", uprep_bytes, need);
    HIPCHK(ttm_launch(dtype, prec, Y, Uprep, Z, L, I, R, M, (hipStream_t)stream), "ttm");
    return STH_OK;
}

extern "C" size_t eig_leading_workspace(int64_t n) { return n >= 1 ? align_up(eig_ws_bytes(n)) : 0; }

static sth_status eig_leading_impl(int64_t n, int64_t R, const double *S, double *U, double *lam,
                                   int32_t max_sweeps, double s_unit, void *ws, size_t ws_bytes,
                                   sth_stream_t stream) {
    if (n < 1 || n > MAX_EIG_N) return fail(n < 1 ? STH_ERR_INVALID : STH_ERR_UNSUPPORTED, "n = %lld outside 1..%lld", (long long)n, (long long)MAX_EIG_N);
    if (R < 1 || R > n) return fail(STH_ERR_INVALID, "R = %lld outside 1..n", (long long)R);
    if (!(s_unit >= 0.0 && s_unit < 1.0)) return fail(STH_ERR_INVALID, "s_unit outside [0, 1)");
    sth_status st;
    if ((st = check_ptr(S, "S")) || (st = check_ptr(U, "U")) || (st = check_ptr(lam, "lam", true)) || (st = check_ptr(ws, "ws"))) return st;
    if (ws_bytes < eig_ws_bytes(n)) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, eig_ws_bytes(n));
    HIPCHK(zero_words(ws, 8, (hipStream_t)stream), "flag clear");
    HIPCHK(eig_launch(n, R, S, U, lam, 1e-15, max_sweeps > 0 ? max_sweeps : 60, ws, (int64_t *)ws,
                      (hipStream_t)stream, n, true, s_unit), "eig");
    return STH_OK;
}

extern "C" sth_status eig_leading(int64_t n, int64_t R, const double *S, double *U, double *lam,
                                  int32_t max_sweeps, void *ws, size_t ws_bytes, sth_stream_t stream) {
    return eig_leading_impl(n, R, S, U, lam, max_sweeps, 0.0, ws, ws_bytes, stream);
}

extern "C" sth_status eig_leading_ex(int64_t n, int64_t R, const double *S, double *U, double *lam,
                                     int32_t max_sweeps, double s_unit, void *ws, size_t ws_bytes,
                                     sth_stream_t stream) {
    return eig_leading_impl(n, R, S, U, lam, max_sweeps, s_unit, ws, ws_bytes, stream);
}

// --------------------------------------------------------------- HOOI ----
// Higher-order orthogonal iteration, the Tucker algorithm Sec. II-B names
// beside st-HOSVD and seeds from it: per sweep and mode n, Y = X x_m U_m^T
// for every m != n (increasing m), U_n = the R_n leading eigenvectors of the
// mode-n Gram of Y; finally G = X x_1 U_1^T ... x_N U_N^T.  The same Gram,
// eigensolver and TTM launches as the decomposition, on caller buffers.

namespace {
struct HooiWs {
    size_t flag, bufA, bufB, part, S, eig, uq, total;
};

HooiWs hooi_layout(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype, int tp) {
    size_t maxY = 0, maxPart = 0, maxS = 0, maxEig = 0, maxUq = 0;
    for (int n = 0; n <= order; ++n) {   // n = order: the core chain
        std::vector<int64_t> cur(dims, dims + order);
        for (int m = 0; m < order; ++m) {
            if (m == n) continue;
            cur[m] = ranks[m];
            size_t e = 1;
            for (int k = 0; k < order; ++k) e *= (size_t)cur[k];
            maxY = std::max(maxY, e);
            maxUq = std::max(maxUq, ttm_prep_bytes(dims[m], ranks[m], tp));
        }
        if (n < order) {
            int64_t L, I, M;
            lim(order, cur.data(), n, L, I, M);
            maxPart = std::max(maxPart, gram_ws_bytes(I, I, L * M, true));
            maxS = std::max(maxS, (size_t)(I * I) * sizeof(double));
            maxEig = std::max(maxEig, eig_ws_bytes(I));
        }
    }
    HooiWs w;
    Arena a;
    w.flag = a.take(256);
    w.bufA = a.take(maxY * esize(dtype));
    w.bufB = a.take(maxY * esize(dtype));
    w.part = a.take(maxPart);
    w.S = a.take(maxS);
    w.eig = a.take(maxEig);
    w.uq = a.take(maxUq);
    w.total = a.off;
    return w;
}

sth_status flag_check(int64_t *dflag, hipStream_t s) {
    int64_t flag = 0;
    HIPCHK(hipStreamSynchronize(s), "sync");
    HIPCHK(hipMemcpy(&flag, dflag, sizeof(flag), hipMemcpyDeviceToHost), "flag read");
    int64_t zero = 0;
    HIPCHK(hipMemcpy(dflag, &zero, sizeof(zero), hipMemcpyHostToDevice), "flag clear");
    if (flag == 1) return fail(STH_ERR_NUMERIC, "eigensolver hit its sweep cap");
    if (flag == 2) return fail(STH_ERR_NUMERIC, "Cholesky met a non-positive pivot");
    if (flag == 3) return fail(STH_ERR_NUMERIC, "NaN or Inf met");
    if (flag) return fail(STH_ERR_NUMERIC, "numeric flag %lld", (long long)flag);
    return STH_OK;
}
}  // namespace

extern "C" size_t sth_hooi_workspace(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype,
                                     int32_t ttm_prec) {
    if (check_shape(order, dims) || !ranks) return 0;
    for (int k = 0; k < order; ++k)
        if (ranks[k] < 1 || ranks[k] > dims[k]) return 0;
    return hooi_layout(order, dims, ranks, dtype, ttm_prec).total;
}

extern "C" sth_status sth_hooi(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype,
                               int32_t gram_prec, int32_t ttm_prec, const void *X, double *const *U,
                               void *core, int32_t sweeps, void *ws, size_t ws_bytes, sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (order < 2) return fail(STH_ERR_INVALID, "HOOI needs order >= 2");
    if (!ranks || !U) return fail(STH_ERR_INVALID, "NULL argument");
    for (int k = 0; k < order; ++k) {
        if (ranks[k] < 1 || ranks[k] > dims[k]) return fail(STH_ERR_INVALID, "ranks[%d] out of range", k);
        if (dims[k] > MAX_EIG_N)
            return fail(STH_ERR_UNSUPPORTED, "I_%d = %lld exceeds the eigensolver limit %lld", k, (long long)dims[k], (long long)MAX_EIG_N);
        if ((st = check_ptr(U[k], "U[n]"))) return st;
    }
    if (sweeps < 0) return fail(STH_ERR_INVALID, "sweeps = %d < 0", sweeps);
    if ((st = check_dtype_prec(dtype, gram_prec, "gram_prec"))) return st;
    if ((st = check_dtype_prec(dtype, ttm_prec, "ttm_prec"))) return st;
    if ((st = check_ptr(X, "X")) || (st = check_ptr(core, "core")) || (st = check_ptr(ws, "ws"))) return st;
    const HooiWs L = hooi_layout(order, dims, ranks, dtype, ttm_prec);
    if (ws_bytes < L.total) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int64_t *flag = (int64_t *)(w + L.flag);
    void *uq = w + L.uq;
    HIPCHK(zero_words(flag, 8, s), "flag clear");
    // X x_m U_m^T for every m != skip, increasing m; the last product goes to
    // last_dst (or a buffer); returns the result and its dims in cur
    auto chain = [&](int skip, void *last_dst, std::vector<int64_t> &cur, const void *&res) -> sth_status {
        cur.assign(dims, dims + order);
        const void *src = X;
        int k = 0, nprod = order - (skip < order ? 1 : 0);
        for (int m = 0; m < order; ++m) {
            if (m == skip) continue;
            int64_t Lm, Im, Mm;
            lim(order, cur.data(), m, Lm, Im, Mm);
            void *dst = (k == nprod - 1 && last_dst) ? last_dst : (void *)(w + (k % 2 == 0 ? L.bufA : L.bufB));
            HIPCHK(ttm_prep_u(U[m], dims[m], ranks[m], 0, ttm_prec, uq, s), "hooi prep");
            HIPCHK(ttm_launch(dtype, ttm_prec, src, uq, dst, Lm, Im, ranks[m], Mm, s), "hooi ttm");
            cur[m] = ranks[m];
            src = dst;
            ++k;
        }
        res = src;
        return STH_OK;
    };
    std::vector<int64_t> cur;
    const void *Y = nullptr;
    for (int sw = 0; sw < sweeps; ++sw)
        for (int n = 0; n < order; ++n) {
            if ((st = chain(n, nullptr, cur, Y))) return st;
            int64_t Ln, In, Mn;
            lim(order, cur.data(), n, Ln, In, Mn);
            double *S = (double *)(w + L.S);
            HIPCHK(gram_launch(dtype, gram_prec, Y, Y, Ln, In, In, Mn, true, (double *)(w + L.part), S, s), "hooi gram");
            HIPCHK(eig_launch(In, ranks[n], S, U[n], nullptr, 1e-15, 60, w + L.eig, flag, s, Ln * Mn, false,
                              gram_unit(gram_prec)),
                   "hooi eig");
        }
    return chain(order, core, cur, Y);
}

extern "C" sth_status sth_hooi_check(void *ws, sth_stream_t stream) {
    if (!ws) return fail(STH_ERR_INVALID, "NULL argument");
    return flag_check((int64_t *)ws, (hipStream_t)stream);
}

// -------------------------------------------------------- reconstruct ----

static void recon_sizes(int32_t order, const int64_t *dims, const int64_t *ranks, size_t &maxA, size_t &maxB) {
    std::vector<int64_t> cur(ranks, ranks + order);
    maxA = maxB = 0;
    for (int n = 0; n < order - 1; ++n) {
        cur[n] = dims[n];
        size_t e = 1;
        for (int k = 0; k < order; ++k) e *= (size_t)cur[k];
        if (n % 2 == 0) maxA = std::max(maxA, e);
        else maxB = std::max(maxB, e);
    }
}

extern "C" size_t tucker_reconstruct_workspace(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype) {
    if (check_shape(order, dims) || !ranks) return 0;
    size_t a, b, uq = 0;
    recon_sizes(order, dims, ranks, a, b);
    for (int n = 0; n < order; ++n) uq = std::max(uq, ttm_prep_bytes(ranks[n], dims[n], STH_PREC_FP64));
    return align_up(a * esize(dtype)) + align_up(b * esize(dtype)) + align_up(uq);
}

extern "C" sth_status tucker_reconstruct(int32_t order, const int64_t *dims, const int64_t *ranks,
                                         int32_t dtype, int32_t prec, const void *G,
                                         const double *const *U, void *Xhat, void *ws, size_t ws_bytes,
                                         sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (!ranks || !U) return fail(STH_ERR_INVALID, "NULL argument");
    for (int k = 0; k < order; ++k) {
        if (ranks[k] < 1 || ranks[k] > dims[k]) return fail(STH_ERR_INVALID, "ranks[%d] out of range", k);
        if ((st = check_ptr(U[k], "U[n]"))) return st;
    }
    if ((st = check_dtype_prec(dtype, prec, "prec"))) return st;
    if ((st = check_ptr(G, "G")) || (st = check_ptr(Xhat, "Xhat")) || (st = check_ptr(ws, "ws"))) return st;
    size_t need = tucker_reconstruct_workspace(order, dims, ranks, dtype);
    if (ws_bytes < need) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    size_t a, b;
    recon_sizes(order, dims, ranks, a, b);
    char *bufA = (char *)ws, *bufB = bufA + align_up(a * esize(dtype));
    void *uq = bufB + align_up(b * esize(dtype));
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> cur(ranks, ranks + order);
    const void *src = G;
    for (int n = 0; n < order; ++n) {
        int64_t L, I, M;
        lim(order, cur.data(), n, L, I, M);
        void *dst = (n == order - 1) ? Xhat : (n % 2 == 0 ? (void *)bufA : (void *)bufB);
        // expand mode n: Z(a, i, b) = sum_r U(i, r) Y(a, r, b)
        HIPCHK(ttm_prep_u(U[n], ranks[n], dims[n], 1, prec, uq, s), "recon prep");
        HIPCHK(ttm_launch(dtype, prec, src, uq, dst, L, ranks[n], dims[n], M, s), "recon ttm");
        cur[n] = dims[n];
        src = dst;
    }
    return STH_OK;
}

extern "C" size_t tucker_error_workspace(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype) {
    if (check_shape(order, dims) || !ranks) return 0;
    // the reconstruction's intermediates and factor split, then the fused
    // last expansion's partial sums (X^ itself is never stored)
    return tucker_reconstruct_workspace(order, dims, ranks, dtype) +
           align_up(ttm_err_part_doubles(dims[order - 1]) * sizeof(double));
}

extern "C" sth_status tucker_error(int32_t order, const int64_t *dims, const int64_t *ranks,
                                   int32_t dtype, int32_t prec, const void *X, const void *G,
                                   const double *const *U, double *out, void *ws, size_t ws_bytes,
                                   sth_stream_t stream) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (!ranks) return fail(STH_ERR_INVALID, "ranks is NULL");
    if ((st = check_ptr(X, "X")) || (st = check_ptr(out, "out"))) return st;
    size_t need = tucker_error_workspace(order, dims, ranks, dtype);
    if (ws_bytes < need) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    if (!U) return fail(STH_ERR_INVALID, "NULL argument");
    for (int k = 0; k < order; ++k) {
        if (ranks[k] < 1 || ranks[k] > dims[k]) return fail(STH_ERR_INVALID, "ranks[%d] out of range", k);
        if ((st = check_ptr(U[k], "U[n]"))) return st;
    }
    if ((st = check_dtype_prec(dtype, prec, "prec")) || (st = check_ptr(G, "G")) || (st = check_ptr(ws, "ws")))
        return st;
    // the expansions of modes 1 .. N-1 as tucker_reconstruct runs them, the
    // last one fused with the sums: X^ is never written
    const size_t rw = tucker_reconstruct_workspace(order, dims, ranks, dtype);
    double *part = (double *)((char *)ws + rw);
    size_t a, b;
    recon_sizes(order, dims, ranks, a, b);
    char *bufA = (char *)ws, *bufB = bufA + align_up(a * esize(dtype));
    void *uq = bufB + align_up(b * esize(dtype));
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> cur(ranks, ranks + order);
    const void *src = G;
    for (int n = 0; n < order; ++n) {
        int64_t L, I, M;
        lim(order, cur.data(), n, L, I, M);
        HIPCHK(ttm_prep_u(U[n], ranks[n], dims[n], 1, prec, uq, s), "error prep");
        if (n == order - 1) {
            HIPCHK(ttm_err_launch(dtype, prec, src, uq, X, L, ranks[n], dims[n], M, part, out, s), "error ttm");
            break;
        }
        void *dst = n % 2 == 0 ? (void *)bufA : (void *)bufB;
        HIPCHK(ttm_launch(dtype, prec, src, uq, dst, L, ranks[n], dims[n], M, s), "error expand");
        cur[n] = dims[n];
        src = dst;
    }
    return STH_OK;
}

extern "C" sth_status sth_sumsq(int32_t dtype, const void *x, int64_t count, double *out, void *ws,
                                size_t ws_bytes, sth_stream_t stream) {
    if (dtype != STH_F64 && dtype != STH_F32) return fail(STH_ERR_INVALID, "dtype %d", dtype);
    if (count < 0) return fail(STH_ERR_INVALID, "count < 0");
    sth_status st;
    if ((st = check_ptr(x, "x")) || (st = check_ptr(out, "out")) || (st = check_ptr(ws, "ws"))) return st;
    if (ws_bytes < SUMSQ_BLOCKS * sizeof(double)) return fail(STH_ERR_NOMEM, "workspace too small");
    HIPCHK(sumsq_launch(dtype, x, nullptr, count, out, (double *)ws, nullptr, (hipStream_t)stream), "sumsq");
    return STH_OK;
}

// ------------------------------------------------------------ one mode ----

static sth_status mode_step_plan(int32_t order, const int64_t *dims, int32_t n, int64_t R, int32_t dtype,
                                 int32_t gram_prec, int32_t ttm_prec, int32_t solver, int32_t als_iters,
                                 sth_plan **pl, size_t *bytes) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (n < 0 || n >= order) return fail(STH_ERR_INVALID, "mode %d outside 0..%d", n, order - 1);
    if (solver != STH_SOLVER_EIG && solver != STH_SOLVER_ALS) return fail(STH_ERR_INVALID, "solver %d", solver);
    std::vector<int64_t> ranks(dims, dims + order);
    ranks[n] = R;
    std::vector<int32_t> mo;
    mo.push_back(n);
    for (int k = 0; k < order; ++k)
        if (k != n) mo.push_back(k);
    sth_desc d;
    memset(&d, 0, sizeof(d));
    d.order = order;
    d.dims = dims;
    d.ranks = ranks.data();
    d.mode_order = mo.data();
    d.dtype = dtype;
    d.gram_prec = gram_prec;
    d.ttm_prec = ttm_prec;
    d.solver = solver;
    d.als_iters = als_iters;
    return make_plan(&d, 1, pl, bytes);
}

extern "C" size_t sthosvd_mode_step_workspace(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                                              int32_t dtype, int32_t gram_prec, int32_t ttm_prec,
                                              int32_t solver, int32_t als_iters) {
    sth_plan *pl = nullptr;
    size_t b = 0;
    if (mode_step_plan(order, dims, n, R, dtype, gram_prec, ttm_prec, solver, als_iters, &pl, &b)) return 0;
    delete pl;
    return b;
}

extern "C" sth_status sthosvd_mode_step(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                                        int32_t dtype, int32_t gram_prec, int32_t ttm_prec,
                                        int32_t solver, int32_t als_iters, const void *Y, void *Z,
                                        double *U, double *eigvals, const double *als_init,
                                        uint64_t seed, void *ws, size_t ws_bytes, sth_stream_t stream) {
    sth_plan *pl = nullptr;
    size_t need = 0;
    sth_status st = mode_step_plan(order, dims, n, R, dtype, gram_prec, ttm_prec, solver, als_iters, &pl, &need);
    if (st) return st;
    std::unique_ptr<sth_plan> hold(pl);
    if ((st = check_ptr(Y, "Y")) || (st = check_ptr(Z, "Z")) || (st = check_ptr(U, "U")) ||
        (st = check_ptr(ws, "ws")) || (st = check_ptr(eigvals, "eigvals", true)) ||
        (st = check_ptr(als_init, "als_init", true)))
        return st;
    if (ws_bytes < need) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    HIPCHK(zero_words(w + pl->o_flag, 8, s), "flag clear");
    return exec_step(*pl, pl->steps[0], Y, Z, U, eigvals, als_init, seed, w, s);
}

// ------------------------------------------------- exhaustive selection ----

namespace {
struct ExhLayout {
    size_t step, zbuf, u, ev, total;
};
// [step workspace][three tensor buffers: the working tensor and the two
// steps' outputs][U][eigvals]
sth_status exh_layout(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype,
                      int32_t gram_prec, int32_t ttm_prec, int32_t als_iters, ExhLayout *L) {
    sth_status st;
    if ((st = check_shape(order, dims))) return st;
    if (!ranks) return fail(STH_ERR_INVALID, "ranks is NULL");
    const size_t esz = dtype == STH_F64 ? 8 : 4;
    std::vector<int64_t> cur(dims, dims + order);
    size_t step = 0, zmax = 0, umax = 0, rmax = 0;
    for (int n = 0; n < order; ++n) {
        if (ranks[n] < 1 || ranks[n] > cur[n]) return fail(STH_ERR_INVALID, "ranks[%d] out of range", n);
        const size_t be = sthosvd_mode_step_workspace(order, cur.data(), n, ranks[n], dtype, gram_prec, ttm_prec,
                                                      STH_SOLVER_EIG, als_iters);
        if (be == 0) {
            const std::string why = sth_last_error();
            return fail(STH_ERR_UNSUPPORTED, "mode %d: no EIG step (%s)", n, why.c_str());
        }
        const size_t ba = sthosvd_mode_step_workspace(order, cur.data(), n, ranks[n], dtype, gram_prec, ttm_prec,
                                                      STH_SOLVER_ALS, als_iters);
        step = std::max(step, std::max(be, ba));
        umax = std::max(umax, (size_t)(cur[n] * ranks[n]) * 8);
        rmax = std::max(rmax, (size_t)ranks[n] * 8);
        cur[n] = ranks[n];
        size_t z = esz;
        for (int k = 0; k < order; ++k) z *= (size_t)cur[k];
        zmax = std::max(zmax, z);
    }
    L->step = align_up(step);
    L->zbuf = align_up(zmax);
    L->u = align_up(umax);
    L->ev = align_up(rmax);
    L->total = L->step + 3 * L->zbuf + L->u + L->ev;
    return STH_OK;
}
}  // namespace

extern "C" size_t sthosvd_choose_exhaustive_workspace(int32_t order, const int64_t *dims, const int64_t *ranks,
                                                      int32_t dtype, int32_t gram_prec, int32_t ttm_prec,
                                                      int32_t als_iters) {
    ExhLayout L;
    if (exh_layout(order, dims, ranks, dtype, gram_prec, ttm_prec, als_iters, &L)) return 0;
    return L.total;
}

extern "C" sth_status sthosvd_choose_exhaustive(int32_t order, const int64_t *dims, const int64_t *ranks,
                                                int32_t dtype, int32_t gram_prec, int32_t ttm_prec,
                                                int32_t als_iters, const void *X, int32_t *solvers_out,
                                                float *ms_out, void *ws, size_t ws_bytes,
                                                sth_stream_t stream) {
    ExhLayout L;
    sth_status st = exh_layout(order, dims, ranks, dtype, gram_prec, ttm_prec, als_iters, &L);
    if (st) return st;
    if ((st = check_ptr(X, "X")) || (st = check_ptr(ws, "ws"))) return st;
    if (!solvers_out) return fail(STH_ERR_INVALID, "solvers_out is NULL");
    if (ws_bytes < L.total) return fail(STH_ERR_NOMEM, "workspace %zu < %zu", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    char *const zb[3] = {w + L.step, w + L.step + L.zbuf, w + L.step + 2 * L.zbuf};
    double *const U = (double *)(w + L.step + 3 * L.zbuf);
    double *const ev = (double *)(w + L.step + 3 * L.zbuf + L.u);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(STH_ERR_HIP, "event");
    }
    std::vector<int64_t> cur(dims, dims + order);
    const void *Y = X;
    int yi = -1;   // buffer holding the working tensor (-1: X)
    st = STH_OK;
    for (int n = 0; n < order && st == STH_OK; ++n) {
        float ms[2] = {-1.f, -1.f};
        int ob[2], m = 0;   // the two steps' outputs: the buffers other than the input
        for (int b = 0; b < 3 && m < 2; ++b)
            if (b != yi) ob[m++] = b;
        for (int sv = 0; sv < 2; ++sv) {
            const int32_t solver = sv == 0 ? STH_SOLVER_EIG : STH_SOLVER_ALS;
            // one untimed run (first-touch and code loading), then one timed
            sth_status r = sthosvd_mode_step(order, cur.data(), n, ranks[n], dtype, gram_prec, ttm_prec, solver,
                                             als_iters, Y, zb[ob[sv]], U, sv == 0 ? ev : nullptr, nullptr, 0, w,
                                             L.step, stream);
            if (r == STH_OK) {
                hipEventRecord(e0, s);
                r = sthosvd_mode_step(order, cur.data(), n, ranks[n], dtype, gram_prec, ttm_prec, solver, als_iters,
                                      Y, zb[ob[sv]], U, sv == 0 ? ev : nullptr, nullptr, 0, w, L.step, stream);
                hipEventRecord(e1, s);
            }
            if (r != STH_OK) {
                if (sv == 0) {   // the EIG step must run
                    st = r;
                    break;
                }
                continue;        // ALS cannot run this mode
            }
            if (hipEventSynchronize(e1) != hipSuccess) {
                st = fail(STH_ERR_HIP, "event sync");
                break;
            }
            // a step that raised the numerical flag (e.g. a broken-down ALS
            // basis) does not count
            sth_plan *pl = nullptr;
            size_t need = 0;
            int64_t flag = 0;
            if (mode_step_plan(order, cur.data(), n, ranks[n], dtype, gram_prec, ttm_prec, solver, als_iters, &pl,
                               &need) == STH_OK) {
                const size_t off = pl->o_flag;
                delete pl;
                if (hipMemcpy(&flag, w + off, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) {
                    st = fail(STH_ERR_HIP, "flag read");
                    break;
                }
            }
            float t = 0.f;
            hipEventElapsedTime(&t, e0, e1);
            if (flag == 0) ms[sv] = t;
            else if (sv == 0) {
                st = fail(STH_ERR_NUMERIC, "mode %d: the EIG step raised numeric flag %lld", n, (long long)flag);
                break;
            }
        }
        if (st != STH_OK) break;
        const int pick = (ms[1] >= 0.f && ms[1] < ms[0]) ? 1 : 0;
        solvers_out[n] = pick == 0 ? STH_SOLVER_EIG : STH_SOLVER_ALS;
        if (ms_out) {
            ms_out[2 * n] = ms[0];
            ms_out[2 * n + 1] = ms[1];
        }
        yi = ob[pick];
        Y = zb[yi];
        cur[n] = ranks[n];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// ----------------------------------------------------- learned selector ----

extern "C" int32_t sth_selector_num_params(void) { return SEL_NPARAM; }
extern "C" int32_t sth_selector_num_trainable(void) { return mlp_num_trainable(); }

extern "C" sth_status sth_selector_features(int64_t I, int64_t R, int64_t J, float *out10) {
    if (I < 1 || R < 1 || J < 1 || !out10) return fail(STH_ERR_INVALID, "bad selector features input");
    selector_features(I, R, J, out10);
    return STH_OK;
}

extern "C" sth_status sth_selector_choose(const float *weights, int64_t I, int64_t R, int64_t J,
                                          int32_t *solver_out) {
    if (I < 1 || R < 1 || R > I || J < 1 || !solver_out) return fail(STH_ERR_INVALID, "bad selector input");
    *solver_out = selector_choose(I, R, J, 0, weights);
    return STH_OK;
}

extern "C" sth_status sth_selector_tree_choose(int64_t I, int64_t R, int64_t J, int32_t *solver_out) {
    if (I < 1 || R < 1 || R > I || J < 1 || !solver_out) return fail(STH_ERR_INVALID, "bad selector input");
    *solver_out = selector_tree_choose(I, R, J);
    return STH_OK;
}

extern "C" sth_status sth_selector_predict(const float *weights, int64_t I, int64_t R, int64_t J,
                                           float *out2) {
    if (I < 1 || R < 1 || J < 1 || !out2) return fail(STH_ERR_INVALID, "bad selector input");
    float f[SEL_IN];
    selector_features(I, R, J, f);
    selector_predict(weights, f, out2);
    return STH_OK;
}

extern "C" size_t sth_mlp_workspace(int64_t B) { return B > 0 ? align_up(mlp_ws_bytes(B)) : 0; }

extern "C" sth_status sth_mlp_forward(const float *params, int64_t B, const float *X, float *Y, void *ws,
                                      size_t ws_bytes, sth_stream_t stream) {
    sth_status st;
    if (B < 1) return fail(STH_ERR_INVALID, "B < 1");
    if ((st = check_ptr(params, "params")) || (st = check_ptr(X, "X")) || (st = check_ptr(Y, "Y")) ||
        (st = check_ptr(ws, "ws")))
        return st;
    if (ws_bytes < mlp_ws_bytes(B)) return fail(STH_ERR_NOMEM, "workspace too small");
    HIPCHK(mlp_forward_launch(params, B, X, Y, ws, (hipStream_t)stream), "mlp forward");
    return STH_OK;
}

extern "C" sth_status sth_mlp_loss_grad(const float *params, int64_t B, const float *X, const float *T,
                                        float *grad, float *loss, void *ws, size_t ws_bytes,
                                        sth_stream_t stream) {
    sth_status st;
    if (B < 1) return fail(STH_ERR_INVALID, "B < 1");
    if ((st = check_ptr(params, "params")) || (st = check_ptr(X, "X")) || (st = check_ptr(T, "T")) ||
        (st = check_ptr(grad, "grad")) || (st = check_ptr(loss, "loss", true)) || (st = check_ptr(ws, "ws")))
        return st;
    if (ws_bytes < mlp_ws_bytes(B)) return fail(STH_ERR_NOMEM, "workspace too small");
    HIPCHK(mlp_loss_grad_launch(params, B, X, T, grad, loss, ws, (hipStream_t)stream), "mlp grad");
    return STH_OK;
}

extern "C" sth_status sth_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count,
                                   float lr, float beta1, float beta2, float eps, int32_t step,
                                   sth_stream_t stream) {
    sth_status st;
    if (count < 1 || step < 1) return fail(STH_ERR_INVALID, "count < 1 or step < 1");
    if ((st = check_ptr(params, "params")) || (st = check_ptr(grad, "grad")) || (st = check_ptr(m, "m")) ||
        (st = check_ptr(v, "v")))
        return st;
    HIPCHK(adam_launch(params, grad, m, v, count, lr, beta1, beta2, eps, step, (hipStream_t)stream), "adam");
    return STH_OK;
}

// ------------------------------------------------------------- batched ----

struct BatchLaunchT {
    size_t list_off, pref_off;
    int len;
    int64_t total;
    int cls;
    int l1 = 0;   // every tensor of the list has L = 1
};
struct BatchStepT {
    size_t descs_off;
    std::vector<BatchLaunchT> gram, reduce, ttm;
    BatchLaunchT prep;
    size_t eig_lds;
    int max_nchunks;
};
struct sth_batch_plan_s {
    int count = 0, N = 0, dtype = 0, gram_prec = 0, ttm_prec = 0, max_sweeps = 60;
    std::vector<BatchStepT> steps;
    std::vector<char> blob;                // every table, host copy
    mutable void *pinned = nullptr;        // pinned copy, filled at plan time (first run without a device)
    mutable std::mutex mu;
    size_t table_bytes = 0, tables_off = 0, flag_off = 0, total = 0;
    ~sth_batch_plan_s() {
        if (pinned) (void)hipHostFree(pinned);
    }
};

extern "C" sth_status sthosvd_plan_batched(const sth_desc *descs, int32_t count, sth_batch_plan **out,
                                           size_t *ws_out) {
    return sthosvd_plan_batched_tiles(descs, count, nullptr, out, ws_out);
}

extern "C" sth_status sthosvd_plan_batched_tiles(const sth_desc *descs, int32_t count,
                                                 const sth_batch_tiles *tiles, sth_batch_plan **out,
                                                 size_t *ws_out) {
    if (!descs || !out || !ws_out || count < 1) return fail(STH_ERR_INVALID, "bad batched arguments");
    *out = nullptr;
    sth_batch_tiles tile = {4, 4, 4, 0};
    if (tiles) {
        if (tiles->reserved != 0) return fail(STH_ERR_INVALID, "tiles.reserved must be 0");
        if (tiles->gram_wg_per_cu < 0 || tiles->gram_wg_per_cu > 64)
            return fail(STH_ERR_INVALID, "tiles.gram_wg_per_cu = %d out of 0..64", tiles->gram_wg_per_cu);
        if (tiles->gram_wt_max != 0 && tiles->gram_wt_max != 1 && tiles->gram_wt_max != 2 &&
            tiles->gram_wt_max != 4)
            return fail(STH_ERR_INVALID, "tiles.gram_wt_max = %d is not 0, 1, 2 or 4", tiles->gram_wt_max);
        if (tiles->ttm_rows_per_wave < 0 || tiles->ttm_rows_per_wave > 64)
            return fail(STH_ERR_INVALID, "tiles.ttm_rows_per_wave = %d out of 0..64", tiles->ttm_rows_per_wave);
        if (tiles->gram_wg_per_cu) tile.gram_wg_per_cu = tiles->gram_wg_per_cu;
        if (tiles->gram_wt_max) tile.gram_wt_max = tiles->gram_wt_max;
        if (tiles->ttm_rows_per_wave) tile.ttm_rows_per_wave = tiles->ttm_rows_per_wave;
    }
    const sth_desc &d0 = descs[0];
    sth_status st;
    for (int t = 0; t < count; ++t) {
        const sth_desc &d = descs[t];
        if ((st = check_shape(d.order, d.dims))) return st;
        if (!d.ranks) return fail(STH_ERR_INVALID, "ranks[%d] is NULL", t);
        if (d.order != d0.order || d.dtype != d0.dtype || d.gram_prec != d0.gram_prec ||
            d.ttm_prec != d0.ttm_prec)
            return fail(STH_ERR_INVALID, "batched tensors must share order, dtype and precisions");
        if (d.mode_order || d.per_mode || d.solver != STH_SOLVER_EIG)
            return fail(STH_ERR_UNSUPPORTED, "the batched path runs the EIG branch in mode order 1..N");
        for (int k = 0; k < d.order; ++k)
            if (d.ranks[k] < 1 || d.ranks[k] > d.dims[k])
                return fail(STH_ERR_INVALID, "tensor %d: ranks[%d] out of range", t, k);
    }
    if (d0.dtype != STH_F32) return fail(STH_ERR_UNSUPPORTED, "the batched path takes FP32 tensors");
    if ((st = check_dtype_prec(d0.dtype, d0.gram_prec, "gram_prec"))) return st;
    if ((st = check_dtype_prec(d0.dtype, d0.ttm_prec, "ttm_prec"))) return st;
    const int N = d0.order;
    std::unique_ptr<sth_batch_plan_s> p(new sth_batch_plan_s());
    p->count = count;
    p->N = N;
    p->dtype = d0.dtype;
    p->gram_prec = d0.gram_prec;
    p->ttm_prec = d0.ttm_prec;
    p->max_sweeps = d0.eig_max_sweeps ? d0.eig_max_sweeps : 60;
    const int64_t target = std::max<int64_t>(1, (int64_t)tile.gram_wg_per_cu * device_cu_count() / count);

    // per tensor regions and per step descriptors
    Arena a;
    p->flag_off = a.take(256);
    std::vector<std::vector<BatchStep>> sd(N, std::vector<BatchStep>(count));
    for (int t = 0; t < count; ++t) {
        const sth_desc &d = descs[t];
        std::vector<int64_t> cur(d.dims, d.dims + N);
        size_t maxA = 0, maxB = 0, maxPart = 0, maxS = 0, maxUq = 0, maxEig = 0;
        for (int s = 0; s < N; ++s) {
            BatchStep &b = sd[s][t];
            memset(&b, 0, sizeof(b));
            // rotated layout: every intermediate is stored with the mode it
            // feeds first (the TTM writes its output transposed), so each step
            // is the L = 1 view: I = I_s, M = the product of the other modes;
            // after the last step the rotation has come full circle and the
            // core is in natural order
            b.L = 1;
            b.I = cur[s];
            b.M = 1;
            for (int k = 0; k < N; ++k)
                if (k != s) b.M *= cur[k];
            b.R = d.ranks[s];
            b.tensor = t;
            const int64_t P = b.L * b.M;
            const size_t out = (size_t)(b.L * b.R * b.M);
            if (s < N - 1) (s % 2 == 0 ? maxA : maxB) = std::max(s % 2 == 0 ? maxA : maxB, out);
            int wt, nbi, nbj, nblocks, nkc, ns;
            int64_t kper;
            if (batch_gram_skinny(d0.gram_prec, b.L, b.I, P, target, &ns, &nkc)) {
                // whole lower triangles in 32 x 32 super tiles, one workgroup each
                b.wt = BATCH_SKINNY;
                b.nbi = ns;
                b.nblocks = ns * (ns + 1) / 2;
                b.nkc = nkc;
                b.kper = 0;
                b.gram_wg = nkc;
                maxPart = std::max(maxPart, (size_t)nkc * b.nblocks * 32 * 32 * 8);
            } else {
                gram_geometry(b.I, b.I, P, true, target, tile.gram_wt_max, &wt, &nbi, &nbj, &nblocks, &nkc, &kper);
                b.wt = wt;
                b.nbi = nbi;
                b.nblocks = nblocks;
                b.nkc = nkc;
                b.kper = kper;
                b.gram_wg = (int64_t)nkc * nblocks;
                maxPart = std::max(maxPart, (size_t)nkc * nblocks * (32 * wt) * (32 * wt) * 8);
            }
            maxS = std::max(maxS, (size_t)(b.I * b.I) * 8);
            maxUq = std::max(maxUq, ttm_prep_bytes(b.I, b.R, d0.ttm_prec));
            if (b.I > MAX_EIG_N)
                return fail(STH_ERR_UNSUPPORTED, "tensor %d mode %d: I_n = %lld exceeds the eigensolver limit %lld", t, s, (long long)b.I, (long long)MAX_EIG_N);
            if (b.R > 64) return fail(STH_ERR_UNSUPPORTED, "tensor %d mode %d: R_n > 64 in the batched path", t, s);
            b.sib = (int32_t)batch_si_block(b.I, b.R, b.L * b.M);
            maxEig = std::max(maxEig, batch_eig_scratch(b.I, b.R, b.sib));
            b.nchunks = (int)((b.I + 31) / 32);
            b.ntiles = (int)((b.R + 15) / 16);
            b.rtb = b.ntiles <= 1 ? 1 : (b.ntiles <= 2 ? 2 : 4);
            b.contig = 1;
            cur[s] = b.R;
        }
        const size_t oA = a.take(maxA * 4), oB = a.take(maxB * 4), oPart = a.take(maxPart), oS = a.take(maxS),
                     oUq = a.take(maxUq), oEig = a.take(maxEig);
        for (int s = 0; s < N; ++s) {
            BatchStep &b = sd[s][t];
            b.src_off = (s == 0) ? -1 : (int64_t)((s - 1) % 2 == 0 ? oA : oB);
            b.dst_off = (s == N - 1) ? -1 : (int64_t)(s % 2 == 0 ? oA : oB);
            b.part_off = (int64_t)oPart;
            b.S_off = (int64_t)oS;
            b.uq_off = (int64_t)oUq;
            b.eig_off = (int64_t)oEig;
        }
    }
    // tables: per step descriptors, then launch lists and prefix sums
    std::vector<char> blob;
    auto put = [&](const void *src, size_t bytes) {
        size_t off = (blob.size() + 15) & ~(size_t)15;
        blob.resize(off + bytes);
        memcpy(blob.data() + off, src, bytes);
        return off;
    };
    for (int s = 0; s < N; ++s) {
        BatchStepT T;
        T.descs_off = put(sd[s].data(), sizeof(BatchStep) * count);
        T.eig_lds = 0;
        T.max_nchunks = 0;
        for (int t = 0; t < count; ++t) {
            T.eig_lds = std::max(T.eig_lds, batch_eig_lds(sd[s][t].I, sd[s][t].R, sd[s][t].sib));
            T.max_nchunks = std::max(T.max_nchunks, sd[s][t].nchunks);
        }
        auto make = [&](const std::vector<int32_t> &list, const std::vector<int64_t> &units, int cls) {
            BatchLaunchT L;
            std::vector<int64_t> pref(list.size() + 1, 0);
            for (size_t k = 0; k < list.size(); ++k) pref[k + 1] = pref[k] + units[k];
            L.list_off = put(list.data(), sizeof(int32_t) * std::max<size_t>(1, list.size()));
            L.pref_off = put(pref.data(), sizeof(int64_t) * pref.size());
            L.len = (int)list.size();
            L.total = pref.back();
            L.cls = cls;
            return L;
        };
        for (int cls : {BATCH_SKINNY, 1, 2, 4}) {
            std::vector<int32_t> gl;
            std::vector<int64_t> gw, gb;
            for (int t = 0; t < count; ++t)
                if (sd[s][t].wt == cls) {
                    gl.push_back(t);
                    gw.push_back(sd[s][t].gram_wg);
                    gb.push_back(sd[s][t].nblocks);
                }
            if (!gl.empty()) {
                BatchLaunchT G = make(gl, gw, cls);
                G.l1 = 1;
                for (int32_t t : gl) G.l1 &= sd[s][t].L == 1 ? 1 : 0;
                T.gram.push_back(G);
                T.reduce.push_back(make(gl, gb, cls));
            }
            std::vector<int32_t> tl;
            std::vector<int64_t> tw;
            for (int t = 0; t < count; ++t)
                if (sd[s][t].rtb == cls) {
                    const BatchStep &b = sd[s][t];
                    const int nt = (cls == 1) ? 4 : 2;
                    const int64_t rows = (b.L * b.M + 16 * nt - 1) / (16 * nt);
                    tl.push_back(t);
                    const int64_t per_wg = (int64_t)BT_WAVES * tile.ttm_rows_per_wave;
                    tw.push_back(std::max<int64_t>(1, (rows + per_wg - 1) / per_wg));
                }
            if (!tl.empty()) T.ttm.push_back(make(tl, tw, cls));
        }
        std::vector<int32_t> all(count);
        std::vector<int64_t> pw(count);
        for (int t = 0; t < count; ++t) {
            all[t] = t;
            pw[t] = (int64_t)sd[s][t].nchunks * sd[s][t].ntiles * 64;
        }
        T.prep = make(all, pw, 0);
        p->steps.push_back(T);
    }
    p->table_bytes = blob.size();
    p->tables_off = a.take(p->table_bytes);
    p->total = a.off;
    p->blob = std::move(blob);
    // the pinned copy the runs enqueue from: allocated here, so that a run
    // (possibly under graph capture) allocates nothing.  Planning stays
    // host-only work: without a usable device the copy is made by the first
    // run instead.
    {
        void *h = nullptr;
        if (hipHostMalloc(&h, p->table_bytes > 0 ? p->table_bytes : 16, hipHostMallocDefault) == hipSuccess) {
            memcpy(h, p->blob.data(), p->table_bytes);
            p->pinned = h;
        } else {
            (void)hipGetLastError();
        }
    }
    *ws_out = p->total;
    *out = p.release();
    return STH_OK;
}

extern "C" void sthosvd_plan_batched_destroy(sth_batch_plan *plan) { delete plan; }

extern "C" sth_status sthosvd_run_batched(const sth_batch_plan *p, const void *const *X_dev,
                                          void *const *core_dev, double *const *U_dev, void *ws,
                                          size_t ws_bytes, sth_stream_t stream) {
    if (!p) return fail(STH_ERR_INVALID, "plan is NULL");
    sth_status st;
    if ((st = check_ptr(X_dev, "X pointer array")) || (st = check_ptr(core_dev, "core pointer array")) ||
        (st = check_ptr(U_dev, "U pointer array")) || (st = check_ptr(ws, "workspace")))
        return st;
    if (ws_bytes < p->total) return fail(STH_ERR_NOMEM, "workspace %zu < required %zu bytes", ws_bytes, p->total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    char *tab = w + p->tables_off;
    int64_t *flag = (int64_t *)(w + p->flag_off);
    {
        std::lock_guard<std::mutex> lk(p->mu);
        if (!p->pinned) {
            void *h = nullptr;
            HIPCHK(hipHostMalloc(&h, p->table_bytes > 0 ? p->table_bytes : 16, hipHostMallocDefault), "pinned tables");
            memcpy(h, p->blob.data(), p->table_bytes);
            p->pinned = h;
        }
    }
    HIPCHK(hipMemcpyAsync(tab, p->pinned, p->table_bytes, hipMemcpyHostToDevice, s), "tables");
    HIPCHK(zero_words(flag, 8, s), "flag clear");
    auto res = [&](const BatchLaunchT &L) {
        BatchLaunch b;
        b.list = (const int32_t *)(tab + L.list_off);
        b.pref = (const int64_t *)(tab + L.pref_off);
        b.len = L.len;
        b.total = L.total;
        b.cls = L.cls;
        b.l1 = L.l1;
        return b;
    };
    for (int s2 = 0; s2 < p->N; ++s2) {
        const BatchStepT &T = p->steps[s2];
        BatchStepPlan sp;
        sp.count = p->count;
        sp.eig_lds = T.eig_lds;
        sp.max_nchunks = T.max_nchunks;
        for (auto &L : T.gram) sp.gram.push_back(res(L));
        for (auto &L : T.reduce) sp.reduce.push_back(res(L));
        for (auto &L : T.ttm) sp.ttm.push_back(res(L));
        sp.prep = res(T.prep);
        BatchTables bt;
        bt.descs = (const BatchStep *)(tab + T.descs_off);
        HIPCHK(batch_step_launch(bt, sp, p->gram_prec, p->ttm_prec, p->N, s2, w, X_dev, core_dev, U_dev,
                                 flag, p->max_sweeps, s),
               "batched step");
    }
    return STH_OK;
}

extern "C" sth_status sthosvd_check_batched(const sth_batch_plan *p, void *ws, sth_stream_t stream) {
    if (!p || !ws) return fail(STH_ERR_INVALID, "NULL argument");
    int64_t flag = 0;
    int64_t *dflag = (int64_t *)((char *)ws + p->flag_off);
    HIPCHK(hipStreamSynchronize((hipStream_t)stream), "sync");
    HIPCHK(hipMemcpy(&flag, dflag, sizeof(flag), hipMemcpyDeviceToHost), "flag read");
    const int64_t zero = 0;
    HIPCHK(hipMemcpy(dflag, &zero, sizeof(zero), hipMemcpyHostToDevice), "flag clear");
    if (flag == 2) return fail(STH_ERR_NUMERIC, "Cholesky met a non-positive pivot");
    if (flag == 3) return fail(STH_ERR_NUMERIC, "NaN or Inf met");
    if (flag) return fail(STH_ERR_NUMERIC, "numeric flag %lld", (long long)flag);
    return STH_OK;
}
