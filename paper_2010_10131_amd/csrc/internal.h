// Internal interfaces between the host driver and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace sth {

enum { DT_F64 = 0, DT_F32 = 1 };
constexpr int SUMSQ_BLOCKS = 1024;

inline int prec_nq(int prec) { return prec == 0 ? 4 : (prec == 3 ? 3 : 2); }

int device_cu_count();

// TTM (ttm.hip)
size_t ttm_prep_bytes(int64_t K, int64_t Rout, int prec);
hipError_t ttm_prep_u(const double *U, int64_t K, int64_t Rout, int transpose, int prec, void *out,
                      hipStream_t s);
// The TTM of a reconstruction's last expansion fused with its error sums:
// out[0] = sum (X - Z)^2, out[1] = sum X^2 (FP64, device) with Z never stored;
// part: device, ttm_err_part_doubles(Rout) doubles.
size_t ttm_err_part_doubles(int64_t Rout);
hipError_t ttm_err_launch(int dtype, int prec, const void *Y, const void *Uq, const void *X, int64_t L, int64_t K,
                          int64_t Rout, int64_t M, double *part, double *out, hipStream_t s);
hipError_t ttm_launch(int dtype, int prec, const void *Y, const void *Uq, void *Z, int64_t L,
                      int64_t K, int64_t Rout, int64_t M, hipStream_t s);
// the library-held scratch of ttm_mode_n_noalloc (its size, and its address on
// the current device)
size_t ttm_scratch_bytes();
hipError_t ttm_scratch_ptr(void **out);

// Gram / TTT (gram.hip)
size_t gram_ws_bytes(int64_t IA, int64_t IB, int64_t P, bool sym);
hipError_t gram_launch(int dtype, int prec, const void *A, const void *B, int64_t L, int64_t IA,
                       int64_t IB, int64_t M, bool sym, double *partials, double *S,
                       hipStream_t s);

// Eigensolver (eig.hip)
size_t eig_ws_bytes(int64_t n);
// jacobi_small: Jacobi up to order 128 (eig_leading), else the direct solver
// there (decompositions); rank_bound: rank(S) <= rank_bound; s_unit: unit
// roundoff of the products that formed S (gram_unit(prec); 0 for exact data)
hipError_t eig_launch(int64_t n, int64_t R, const double *S, double *U, double *lam, double tol,
                      int max_sweeps, void *ws, int64_t *flag, hipStream_t s, int64_t rank_bound,
                      bool jacobi_small, double s_unit);
inline double gram_unit(int prec) {
    return prec == 0 ? 1.1102230246251565e-16 : (prec == 2 ? 7.62939453125e-06 : 5.9604644775390625e-08);
}
// the direct solver alone (scratch: teig_scratch_doubles(n, R, n <= 128) doubles)
// chk (may be null): run only when gate_open(chk, R, chk_tol); count (may be
// null): incremented when it runs
hipError_t teig_launch(const double *S, int64_t lds, int64_t n, int64_t R, double *U, int64_t ldu, double *lam,
                       bool sign_rule, void *scratch, int64_t *flag, const double *chk, double chk_tol,
                       int64_t *count, hipStream_t s);

// Small FP64 LA and reductions (la.hip)
int gemm_splits(int m, int n, int k);
size_t gemm_ws_bytes(int m, int n, int k);
hipError_t gemm_f64(int ta, int tb, int m, int n, int k, double alpha, const double *A,
                    int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                    void *ws, hipStream_t s);
// gate (may be null): run only when gate_open(gate, gate_R, gate_tol)
hipError_t chol_launch(const double *G, int n, int64_t ldg, double shift_rel, double *R,
                       double *Rinv, int64_t *flag, hipStream_t s, const double *gate = nullptr,
                       int gate_R = 0, double gate_tol = 0.0);
hipError_t sumsq_launch(int dtype, const void *x, const void *y, int64_t count, double *out,
                        double *part, int64_t *flag, hipStream_t s);
hipError_t fill_f64(double *p, int64_t n, double v, hipStream_t s);
hipError_t copy_f64(const double *src, double *dst, int64_t n, hipStream_t s);
hipError_t zero_words(void *p, int64_t nwords, hipStream_t s);
hipError_t gaussian_f64(double *p, int64_t n, uint64_t seed, uint64_t stream, hipStream_t s);

// Gram geometry with a target number of workgroups and a cap on the tile
// width in units of 32 (gram.hip)
void gram_geometry(int64_t IA, int64_t IB, int64_t P, bool sym, int64_t target, int wt_max, int *wt,
                   int *nbi, int *nbj, int *nblocks, int *nkc, int64_t *kper);

// Batched path (batch.hip).  One descriptor per tensor per mode step.
constexpr int BT_WAVES = 8;
struct BatchStep {
    int64_t L, I, M, R;
    int64_t src_off, dst_off;  // byte offsets into the workspace; -1 = caller's X / core
    int64_t part_off, S_off, uq_off, eig_off;
    int64_t kper, gram_wg;
    int32_t nkc, nbi, nblocks, wt;
    int32_t nchunks, ntiles, rtb, contig;   // contig: 1 (every batched step is the L = 1 view)
    int32_t tensor, sib;   // sib: subspace block of the eigensolve (0: the direct solver)
};
struct BatchLaunch {
    const int32_t *list;  // device: indices into the step's descriptors
    const int64_t *pref;  // device: prefix sums of the work units (len + 1)
    int len;
    int64_t total;
    int cls;  // tile class (Gram: WT, or BATCH_SKINNY; TTM: r-tiles per workgroup)
    int l1;   // Gram: every tensor of the list has L = 1
};
struct BatchTables {
    const BatchStep *descs;  // device
};
struct BatchStepPlan {
    int count;
    size_t eig_lds;
    int max_nchunks;
    std::vector<BatchLaunch> gram, reduce, ttm;
    BatchLaunch prep;
};
// Gram class of the skinny path (L = 1, I <= 160): whole triangles per workgroup
constexpr int BATCH_SKINNY = 8;
// true when the step's Gram takes the skinny class: ns = super tiles per side,
// nkc = its workgroups
bool batch_gram_skinny(int prec, int64_t L, int64_t I, int64_t P, int64_t target, int *ns, int *nkc);
size_t batch_gram_lds(int prec, int wt);
// subspace block of a batched eigensolve (0: the direct solver)
int64_t batch_si_block(int64_t n, int64_t R, int64_t rank_bound);
size_t batch_eig_lds(int64_t n, int64_t R, int64_t p);      // dynamic LDS of the batched eigen workgroup
size_t batch_eig_scratch(int64_t n, int64_t R, int64_t p);  // its global scratch (bytes)
hipError_t batch_step_launch(const BatchTables &t, const BatchStepPlan &sp, int gram_prec,
                             int ttm_prec, int order, int mode, char *ws, const void *const *Xp,
                             void *const *Cp, double *const *Up, int64_t *flag, int max_sweeps,
                             hipStream_t s);

// Learned selector MLP (mlp.hip)
size_t mlp_ws_bytes(int64_t B);
hipError_t mlp_forward_launch(const float *w, int64_t B, const float *X, float *Y, void *ws, hipStream_t s);
hipError_t mlp_loss_grad_launch(const float *w, int64_t B, const float *X, const float *T, float *grad,
                                float *loss, void *ws, hipStream_t s);
hipError_t adam_launch(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
int mlp_num_trainable();

}  // namespace sth
