// Learned per-mode solver selector (the Sec. IV analogue): a small MLP cost
// model evaluated on the host at plan time.
#pragma once
#include <stdint.h>

namespace sth {

constexpr int SEL_IN = 10;      // Table I features
constexpr int SEL_HID = 32;
constexpr int SEL_OUT = 2;      // predicted log time of EIG and of ALS
// parameter count: W1 (32x10), b1, W2 (32x32), b2, W3 (2x32), b3, plus the
// feature normalization (mean, inverse std: 2 x 10) and the output scale
constexpr int SEL_NPARAM = SEL_HID * SEL_IN + SEL_HID + SEL_HID * SEL_HID + SEL_HID +
                           SEL_OUT * SEL_HID + SEL_OUT + 2 * SEL_IN;

// Table I features of one mode, log-scaled: I, R, J, I^2, R^2, I R, R^2/I,
// R^2/J, I/J, R/J.
void selector_features(int64_t I, int64_t R, int64_t J, float *out10);

// Predicted (log t_EIG, log t_ALS) for one mode with the given weights
// (NULL = the built-in weights).
void selector_predict(const float *weights, const float *feat10, float *out2);

// Limits of the two solvers (a mode the chosen solver cannot run goes to
// the other one).
constexpr int64_t SEL_MAX_EIG_N = 512;   // eigensolver: I_n x I_n Gram
constexpr int64_t SEL_MAX_ALS_R = 128;   // ALS: R_n x R_n Cholesky in LDS
// EIG above order 128 with R_n > 124 leaves no room for the subspace block's
// guard vectors and runs the direct solver on the whole Gram from the
// workspace, several times slower than ALS there: ALS is taken whenever its
// limits allow.
constexpr int64_t SEL_EIG_SI_MAX_R = 124;
constexpr int64_t SEL_EIG_DIRECT_MAX = 128;

// The solver limits applied to a choice (0 = EIG, 1 = ALS) for a mode with
// (I_n, R_n, J_n): ALS needs R_n <= SEL_MAX_ALS_R and R_n <= J_n (the rank
// bound of the unfolding), EIG needs I_n <= SEL_MAX_EIG_N; a mode that the
// chosen solver cannot run goes to the other one when it can, and the
// whole-Gram rule above.
int apply_limits(int choice, int64_t I, int64_t R, int64_t J);

// 0 = EIG, 1 = ALS: argmin of the predicted times (EIG on ties), then
// apply_limits.
int selector_choose(int64_t I, int64_t R, int64_t J, int order, const float *weights);

// 0 = EIG, 1 = ALS: the compiled-in decision tree's class, then apply_limits.
int selector_tree_choose(int64_t I, int64_t R, int64_t J);

}  // namespace sth
