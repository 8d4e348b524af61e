// Learned cost model of the solver selector (the Sec. IV decision tree's
// role, with an MLP): 10 Table I features -> 32 -> 32 -> 2 (tanh hidden
// layers, linear output = predicted log t_EIG and log t_ALS of one mode).
// Training runs on the device with these kernels:
//   forward    one thread per sample: normalized features, both hidden
//              layers and the output, kept for the backward pass;
//   backward   one thread per sample: output and hidden deltas of the loss
//              L = 0.5/B * sum (Y - T)^2;
//   gradient   one thread per parameter: the sum over samples of
//              delta x activation, in sample order (deterministic);
//   Adam       one thread per parameter.
// Parameter packing (float): W1 (32x10, column-major), b1 (32), W2 (32x32),
// b2 (32), W3 (2x32), b3 (2), then the feature normalization mu (10) and
// inverse std (10), which are not trained.
#include "common.h"
#include "internal.h"
#include "selector.h"

namespace sth {

namespace {
constexpr int NI = SEL_IN, NH = SEL_HID, NO = SEL_OUT;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NO * NH, OMU = OB3 + NO, OISD = OMU + NI;
constexpr int NTRAIN = OMU;  // trainable parameters
}  // namespace

__global__ void mlp_forward_kernel(const float *__restrict__ w, int64_t B, const float *__restrict__ X,
                                   float *__restrict__ XN, float *__restrict__ H1,
                                   float *__restrict__ H2, float *__restrict__ Y) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float xn[NI], h1[NH], h2[NH];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        xn[k] = (X[k + NI * s] - w[OMU + k]) * w[OISD + k];
        XN[k + NI * s] = xn[k];
    }
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float z = w[OB1 + o];
#pragma unroll
        for (int k = 0; k < NI; ++k) z += w[OW1 + o + NH * k] * xn[k];
        h1[o] = tanhf(z);
        H1[o + NH * s] = h1[o];
    }
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float z = w[OB2 + o];
#pragma unroll
        for (int k = 0; k < NH; ++k) z += w[OW2 + o + NH * k] * h1[k];
        h2[o] = tanhf(z);
        H2[o + NH * s] = h2[o];
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        float z = w[OB3 + o];
#pragma unroll
        for (int k = 0; k < NH; ++k) z += w[OW3 + o + NO * k] * h2[k];
        Y[o + NO * s] = z;
    }
}

__global__ void mlp_backward_kernel(const float *__restrict__ w, int64_t B, const float *__restrict__ H1,
                                    const float *__restrict__ H2, const float *__restrict__ Y,
                                    const float *__restrict__ T, float *__restrict__ D1,
                                    float *__restrict__ D2, float *__restrict__ D3) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float d3[NO], d2[NH];
    const float invB = 1.0f / (float)B;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        d3[o] = (Y[o + NO * s] - T[o + NO * s]) * invB;
        D3[o + NO * s] = d3[o];
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        float a = 0.0f;
#pragma unroll
        for (int o = 0; o < NO; ++o) a += w[OW3 + o + NO * k] * d3[o];
        const float h = H2[k + NH * s];
        d2[k] = a * (1.0f - h * h);
        D2[k + NH * s] = d2[k];
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        float a = 0.0f;
#pragma unroll
        for (int o = 0; o < NH; ++o) a += w[OW2 + o + NH * k] * d2[o];
        const float h = H1[k + NH * s];
        D1[k + NH * s] = a * (1.0f - h * h);
    }
}

// grad[p] = sum_s delta(s) * activation(s) for the parameter p (sample order).
__global__ void mlp_grad_kernel(int64_t B, const float *__restrict__ XN, const float *__restrict__ H1,
                                const float *__restrict__ H2, const float *__restrict__ D1,
                                const float *__restrict__ D2, const float *__restrict__ D3,
                                float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= SEL_NPARAM) return;
    const float *d = nullptr, *a = nullptr;
    int dn = 0, an = 0, o = 0, k = 0;
    if (p < OB1) { dn = NH; an = NI; d = D1; a = XN; o = (p - OW1) % NH; k = (p - OW1) / NH; }
    else if (p < OW2) { dn = NH; d = D1; o = p - OB1; }
    else if (p < OB2) { dn = NH; an = NH; d = D2; a = H1; o = (p - OW2) % NH; k = (p - OW2) / NH; }
    else if (p < OW3) { dn = NH; d = D2; o = p - OB2; }
    else if (p < OB3) { dn = NO; an = NH; d = D3; a = H2; o = (p - OW3) % NO; k = (p - OW3) / NO; }
    else if (p < OMU) { dn = NO; d = D3; o = p - OB3; }
    else { grad[p] = 0.0f; return; }  // normalization constants are not trained
    float acc = 0.0f;
    if (a) {
        for (int64_t s = 0; s < B; ++s) acc += d[o + dn * s] * a[k + an * s];
    } else {
        for (int64_t s = 0; s < B; ++s) acc += d[o + dn * s];
    }
    grad[p] = acc;
}

__global__ void mlp_loss_kernel(int64_t B, const float *__restrict__ Y, const float *__restrict__ T,
                                float *__restrict__ loss) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < B * NO; e += 256) {
        const double r = (double)Y[e] - (double)T[e];
        acc += r * r;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(0.5 * red[0] / (double)B);
}

__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

size_t mlp_ws_bytes(int64_t B) {
    return (size_t)B * (NI + 2 * NH + NO + 2 * NH + NO) * sizeof(float) + 256;
}

namespace {
struct MlpWs {
    float *XN, *H1, *H2, *Y, *D1, *D2, *D3;
};
MlpWs mlp_layout(void *ws, int64_t B) {
    MlpWs m;
    float *p = (float *)ws;
    m.XN = p; p += NI * B;
    m.H1 = p; p += NH * B;
    m.H2 = p; p += NH * B;
    m.Y = p; p += NO * B;
    m.D1 = p; p += NH * B;
    m.D2 = p; p += NH * B;
    m.D3 = p;
    return m;
}
}  // namespace

hipError_t mlp_forward_launch(const float *w, int64_t B, const float *X, float *Y, void *ws, hipStream_t s) {
    MlpWs m = mlp_layout(ws, B);
    const unsigned g = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(g), dim3(256), 0, s, w, B, X, m.XN, m.H1, m.H2, Y ? Y : m.Y);
    return hipGetLastError();
}

hipError_t mlp_loss_grad_launch(const float *w, int64_t B, const float *X, const float *T, float *grad,
                                float *loss, void *ws, hipStream_t s) {
    MlpWs m = mlp_layout(ws, B);
    const unsigned g = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(g), dim3(256), 0, s, w, B, X, m.XN, m.H1, m.H2, m.Y);
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(g), dim3(256), 0, s, w, B, m.H1, m.H2, m.Y, T, m.D1, m.D2, m.D3);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((SEL_NPARAM + 255) / 256), dim3(256), 0, s, B, m.XN, m.H1, m.H2,
                       m.D1, m.D2, m.D3, grad);
    if (loss) hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, s, B, m.Y, T, loss);
    return hipGetLastError();
}

hipError_t adam_launch(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.0f / (1.0f - powf(b1, (float)step));
    const float c2 = 1.0f / (1.0f - powf(b2, (float)step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, g, m, v, n, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

int mlp_num_trainable() { return NTRAIN; }

}  // namespace sth
