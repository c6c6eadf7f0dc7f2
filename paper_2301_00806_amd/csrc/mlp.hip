// Cost-model MLP kernels: 16 -> 64 -> 64 -> 2, fp32, ReLU hidden layers.
//
// The model predicts, per instance, [log of sweep time per kernel vector,
// log10 of the survivor density] from the 16 features the packer computes.
// It only orders and sizes work for the persistent scheduler; counts never
// depend on it.
//
// Parameters (WPM_MLP_PARAMS floats): W1[64][16] b1[64] W2[64][64] b2[64]
// W3[2][64] b3[2].  Normalisation (WPM_MLP_NORM floats, not trained):
// mean_x[16] std_x[16] mean_y[2] std_y[2]; inputs are standardised and outputs
// de-standardised inside the kernels.  Loss: mean over samples and outputs of
// the squared error on standardised targets.
//
// Kernels:
//   mlp_forward     one thread per sample, parameters broadcast from LDS
//   mlp_deltas      per-sample forward pass that stores activations and the
//                   back-propagated deltas, plus the per-sample loss
//   mlp_param_grad  one thread per parameter: a fixed-order sum over samples
//                   (deterministic, no atomics)
//   mlp_loss_sum    one workgroup reduces the per-sample losses
//   mlp_adam        one thread per parameter
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace wpm {

namespace {
constexpr int IN = 16, H = 64, OUT = 2;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * IN;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + OUT * H;
constexpr int NPARAM = OFF_B3 + OUT;
constexpr int NNORM = 2 * IN + 2 * OUT;
static_assert(NPARAM == WPM_MLP_PARAMS, "parameter layout");
static_assert(NNORM == WPM_MLP_NORM, "normalisation layout");

// work buffer layout per sample (floats): xn[16] a1[64] a2[64] dz1[64] dz2[64] dy[2] loss[1]
constexpr int WS = IN + 4 * H + OUT + 1;

__device__ __forceinline__ void load_params(float *sp, const float *p, const float *norm) {
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) sp[i] = p[i];
    for (int i = threadIdx.x; i < NNORM; i += blockDim.x) sp[NPARAM + i] = norm[i];
    __syncthreads();
}

__device__ __forceinline__ void forward_one(const float *sp, const float *x, float *xn, float *z1,
                                            float *z2, float *y) {
    const float *mx = sp + NPARAM, *sx = mx + IN;
#pragma unroll
    for (int j = 0; j < IN; ++j) xn[j] = (x[j] - mx[j]) / sx[j];
#pragma unroll 8
    for (int i = 0; i < H; ++i) {
        float s = sp[OFF_B1 + i];
#pragma unroll
        for (int j = 0; j < IN; ++j) s = fmaf(sp[OFF_W1 + i * IN + j], xn[j], s);
        z1[i] = s;
    }
#pragma unroll 4
    for (int i = 0; i < H; ++i) {
        float s = sp[OFF_B2 + i];
#pragma unroll
        for (int j = 0; j < H; ++j) s = fmaf(sp[OFF_W2 + i * H + j], fmaxf(z1[j], 0.0f), s);
        z2[i] = s;
    }
#pragma unroll
    for (int o = 0; o < OUT; ++o) {
        float s = sp[OFF_B3 + o];
#pragma unroll
        for (int j = 0; j < H; ++j) s = fmaf(sp[OFF_W3 + o * H + j], fmaxf(z2[j], 0.0f), s);
        y[o] = s;
    }
}

__global__ __launch_bounds__(256) void mlp_forward(const float *__restrict__ params,
                                                   const float *__restrict__ norm,
                                                   const float *__restrict__ X, int B,
                                                   float *__restrict__ Y) {
    __shared__ float sp[NPARAM + NNORM];
    load_params(sp, params, norm);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float x[IN], xn[IN], z1[H], z2[H], y[OUT];
#pragma unroll
    for (int j = 0; j < IN; ++j) x[j] = X[(int64_t)b * IN + j];
    forward_one(sp, x, xn, z1, z2, y);
    const float *my = sp + NPARAM + 2 * IN, *sy = my + OUT;
#pragma unroll
    for (int o = 0; o < OUT; ++o) Y[(int64_t)b * OUT + o] = y[o] * sy[o] + my[o];
}

__global__ __launch_bounds__(256) void mlp_deltas(const float *__restrict__ params,
                                                  const float *__restrict__ norm,
                                                  const float *__restrict__ X,
                                                  const float *__restrict__ T, int B,
                                                  float *__restrict__ work) {
    __shared__ float sp[NPARAM + NNORM];
    load_params(sp, params, norm);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float x[IN], xn[IN], z1[H], z2[H], y[OUT];
#pragma unroll
    for (int j = 0; j < IN; ++j) x[j] = X[(int64_t)b * IN + j];
    forward_one(sp, x, xn, z1, z2, y);
    const float *my = sp + NPARAM + 2 * IN, *sy = my + OUT;
    float dy[OUT], loss = 0.0f;
    const float scale = 2.0f / ((float)B * (float)OUT);
#pragma unroll
    for (int o = 0; o < OUT; ++o) {
        const float tn = (T[(int64_t)b * OUT + o] - my[o]) / sy[o];
        const float e = y[o] - tn;
        loss += e * e;
        dy[o] = scale * e;
    }
    float dz2[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int o = 0; o < OUT; ++o) s = fmaf(sp[OFF_W3 + o * H + j], dy[o], s);
        dz2[j] = z2[j] > 0.0f ? s : 0.0f;
    }
    float *w = work + (int64_t)b * WS;
#pragma unroll 4
    for (int j = 0; j < H; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < H; ++i) s = fmaf(sp[OFF_W2 + i * H + j], dz2[i], s);
        w[IN + 2 * H + j] = z1[j] > 0.0f ? s : 0.0f;  // dz1
    }
#pragma unroll
    for (int j = 0; j < IN; ++j) w[j] = xn[j];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        w[IN + j] = fmaxf(z1[j], 0.0f);          // a1
        w[IN + H + j] = fmaxf(z2[j], 0.0f);      // a2
        w[IN + 3 * H + j] = dz2[j];
    }
#pragma unroll
    for (int o = 0; o < OUT; ++o) w[IN + 4 * H + o] = dy[o];
    w[IN + 4 * H + OUT] = loss;
}

__global__ __launch_bounds__(256) void mlp_param_grad(const float *__restrict__ work, int B,
                                                      float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    // grad = sum_b delta[b][row] * act[b][col]  (act = 1 for biases)
    int drow, acol;  // offsets into a work record; acol < 0 means bias
    if (p < OFF_B1) {
        drow = IN + 2 * H + (p - OFF_W1) / IN;
        acol = (p - OFF_W1) % IN;
    } else if (p < OFF_W2) {
        drow = IN + 2 * H + (p - OFF_B1);
        acol = -1;
    } else if (p < OFF_B2) {
        drow = IN + 3 * H + (p - OFF_W2) / H;
        acol = IN + (p - OFF_W2) % H;
    } else if (p < OFF_W3) {
        drow = IN + 3 * H + (p - OFF_B2);
        acol = -1;
    } else if (p < OFF_B3) {
        drow = IN + 4 * H + (p - OFF_W3) / H;
        acol = IN + H + (p - OFF_W3) % H;
    } else {
        drow = IN + 4 * H + (p - OFF_B3);
        acol = -1;
    }
    float s = 0.0f;
    for (int b = 0; b < B; ++b) {
        const float *w = work + (int64_t)b * WS;
        s = fmaf(w[drow], acol >= 0 ? w[acol] : 1.0f, s);
    }
    grad[p] = s;
}

__global__ __launch_bounds__(256) void mlp_loss_sum(const float *__restrict__ work, int B,
                                                    float *__restrict__ loss) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += blockDim.x) s += work[(int64_t)b * WS + IN + 4 * H + OUT];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / ((float)B * (float)OUT);
}

__global__ __launch_bounds__(256) void mlp_adam(float *__restrict__ params,
                                                const float *__restrict__ grad,
                                                float *__restrict__ m, float *__restrict__ v,
                                                float lr, float b1, float b2, float eps,
                                                float bc1, float bc2, float wd) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float g = grad[p] + wd * params[p];
    const float mp = b1 * m[p] + (1.0f - b1) * g;
    const float vp = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mp;
    v[p] = vp;
    params[p] -= lr * (mp / bc1) / (sqrtf(vp / bc2) + eps);
}

int hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return WPM_OK;
    set_hip_error(what, (int)e, hipGetErrorString(e));
    return WPM_EHIP;
}

}  // namespace

int64_t mlp_work_floats(int B) { return (int64_t)B * WS; }

int mlp_forward_launch(const float *params, const float *norm, const float *X, int B, float *Y,
                       void *stream) {
    if (!params || !norm || (B > 0 && (!X || !Y)) || B < 0) return WPM_EINVAL;
    if (B == 0) return WPM_OK;
    hipLaunchKernelGGL(mlp_forward, dim3((B + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       params, norm, X, B, Y);
    return hip_status(hipGetLastError(), "mlp_forward");
}

int mlp_grad_launch(const float *params, const float *norm, const float *X, const float *T, int B,
                    float *grad, float *work, float *loss, void *stream) {
    if (!params || !norm || !X || !T || !grad || !work || B <= 0) return WPM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(mlp_deltas, dim3((B + 255) / 256), dim3(256), 0, st, params, norm, X, T, B,
                       work);
    int rc = hip_status(hipGetLastError(), "mlp_deltas");
    if (rc) return rc;
    hipLaunchKernelGGL(mlp_param_grad, dim3((NPARAM + 255) / 256), dim3(256), 0, st, work, B, grad);
    rc = hip_status(hipGetLastError(), "mlp_param_grad");
    if (rc) return rc;
    if (loss) {
        hipLaunchKernelGGL(mlp_loss_sum, dim3(1), dim3(256), 0, st, work, B, loss);
        rc = hip_status(hipGetLastError(), "mlp_loss_sum");
    }
    return rc;
}

int mlp_adam_launch(float *params, const float *grad, float *m, float *v, int step, float lr,
                    float beta1, float beta2, float eps, float weight_decay, void *stream) {
    if (!params || !grad || !m || !v || step < 1) return WPM_EINVAL;
    const float bc1 = 1.0f - powf(beta1, (float)step);
    const float bc2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       params, grad, m, v, lr, beta1, beta2, eps, bc1, bc2, weight_decay);
    return hip_status(hipGetLastError(), "mlp_adam");
}

}  // namespace wpm
