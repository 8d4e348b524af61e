// Host inference of the learned solver selector (runs in sthosvd_plan,
// "before each mode" of Alg. 2, from shape features only).
#include "selector.h"

#include <cmath>

#include "../../include/sthosvd.h"

namespace sth {

#include "selector_weights.inc"  // kSelectorWeights[SEL_NPARAM], kSelectorTrained
#include "selector_tree.inc"     // kTreeNodes, kTreeFeature, kTreeThreshold, kTreeLeft, kTreeRight, kTreeClass

void selector_features(int64_t I, int64_t R, int64_t J, float *f) {
    const double i = (double)I, r = (double)R, j = (double)J;
    const double v[SEL_IN] = {i, r, j, i * i, r * r, i * r, r * r / i, r * r / j, i / j, r / j};
    for (int k = 0; k < SEL_IN; ++k) f[k] = (float)std::log(v[k]);
}

void selector_predict(const float *w, const float *x, float *y) {
    if (!w) w = kSelectorWeights;
    const float *W1 = w, *b1 = W1 + SEL_HID * SEL_IN;
    const float *W2 = b1 + SEL_HID, *b2 = W2 + SEL_HID * SEL_HID;
    const float *W3 = b2 + SEL_HID, *b3 = W3 + SEL_OUT * SEL_HID;
    const float *mu = b3 + SEL_OUT, *isd = mu + SEL_IN;
    float xn[SEL_IN], h1[SEL_HID], h2[SEL_HID];
    for (int k = 0; k < SEL_IN; ++k) xn[k] = (x[k] - mu[k]) * isd[k];
    for (int o = 0; o < SEL_HID; ++o) {
        float z = b1[o];
        for (int k = 0; k < SEL_IN; ++k) z += W1[o + SEL_HID * k] * xn[k];
        h1[o] = std::tanh(z);
    }
    for (int o = 0; o < SEL_HID; ++o) {
        float z = b2[o];
        for (int k = 0; k < SEL_HID; ++k) z += W2[o + SEL_HID * k] * h1[k];
        h2[o] = std::tanh(z);
    }
    for (int o = 0; o < SEL_OUT; ++o) {
        float z = b3[o];
        for (int k = 0; k < SEL_HID; ++k) z += W3[o + SEL_OUT * k] * h2[k];
        y[o] = z;
    }
}

int apply_limits(int choice, int64_t I, int64_t R, int64_t J) {
    // ALS needs R_n <= J_n (R_k = Y^T L_k has rank <= J_n: above it the
    // normal equations are singular) and the R_n x R_n Cholesky in LDS
    const bool als_ok = R <= SEL_MAX_ALS_R && R <= J;
    if (choice == STH_SOLVER_ALS && !als_ok) choice = STH_SOLVER_EIG;
    if (choice == STH_SOLVER_EIG && I > SEL_EIG_DIRECT_MAX && R > SEL_EIG_SI_MAX_R && als_ok)
        choice = STH_SOLVER_ALS;
    if (choice == STH_SOLVER_EIG && I > SEL_MAX_EIG_N && als_ok) choice = STH_SOLVER_ALS;
    return choice;
}

int selector_choose(int64_t I, int64_t R, int64_t J, int order, const float *weights) {
    (void)order;
    float f[SEL_IN], y[SEL_OUT];
    selector_features(I, R, J, f);
    selector_predict(weights, f, y);
    return apply_limits((y[1] < y[0]) ? STH_SOLVER_ALS : STH_SOLVER_EIG, I, R, J);
}

int selector_tree_choose(int64_t I, int64_t R, int64_t J) {
    float f[SEL_IN];
    selector_features(I, R, J, f);
    int k = 0;
    for (int depth = 0; kTreeFeature[k] >= 0 && depth < kTreeNodes; ++depth)
        k = (f[kTreeFeature[k]] <= kTreeThreshold[k]) ? kTreeLeft[k] : kTreeRight[k];
    return apply_limits(kTreeClass[k] ? STH_SOLVER_ALS : STH_SOLVER_EIG, I, R, J);
}

}  // namespace sth
