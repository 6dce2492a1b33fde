// FP32 MLP cost model (8 -> 64 -> 64 -> 1, ReLU) for choosing HE-convolution
// parameters: its training (forward, backward, Adam) and inference kernels.
//
// Parameters live in one fp32 array theta (HYENA_MLP_PARAMS = 4801 words):
//   W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1]
// The network maps a standardised feature vector of a layer configuration
// (ring degree, RNS limbs, channel partition, Walsh group, layer shape) to the
// logarithm of its measured time. The loss is the mean squared error.
//
// Gradients are deterministic: a block of 256 threads owns 64 samples, keeps
// their activations and back-propagated errors in LDS and sums each parameter's
// contributions over its samples in a fixed order; a second kernel adds the
// per-block partial gradients in block order. No floating-point atomics.
#include "internal.h"

namespace {

constexpr int IN = 8, H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == 4801, "parameter layout");
constexpr int SPB = 64;  // samples per block in the backward kernel

// Forward of one sample held by the calling thread; theta in LDS.
__device__ __forceinline__ float mlp_sample(const float *th, const float *x, float *h1, float *h2) {
#pragma unroll 4
    for (int j = 0; j < H; j++) {
        float a = th[OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < IN; i++) a = fmaf(th[OFF_W1 + j * IN + i], x[i], a);
        h1[j] = fmaxf(a, 0.f);
    }
    float y = th[OFF_B3];
    for (int j = 0; j < H; j++) {
        float a = th[OFF_B2 + j];
#pragma unroll 8
        for (int i = 0; i < H; i++) a = fmaf(th[OFF_W2 + j * H + i], h1[i], a);
        h2[j] = fmaxf(a, 0.f);
        y = fmaf(th[OFF_W3 + j], h2[j], y);
    }
    return y;
}

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float *__restrict__ theta,
                                                          const float *__restrict__ X, uint32_t B,
                                                          float *__restrict__ Y) {
    __shared__ float th[NPARAM];
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) th[i] = theta[i];
    __syncthreads();
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float x[IN], h1[H], h2[H];
#pragma unroll
    for (int i = 0; i < IN; i++) x[i] = X[(size_t)s * IN + i];
    Y[s] = mlp_sample(th, x, h1, h2);
}

// Partial gradients of one block of SPB samples: part[blockIdx.x][NPARAM + 1]
// (the last word is the block's sum of squared errors).
__global__ void __launch_bounds__(256) mlp_backward_kernel(const float *__restrict__ theta,
                                                           const float *__restrict__ X,
                                                           const float *__restrict__ T, uint32_t B,
                                                           float *__restrict__ part) {
    __shared__ float th[NPARAM];
    __shared__ float sx[SPB][IN], sh1[SPB][H + 1], sdh1[SPB][H + 1], sh2[SPB][H + 1], sdh2[SPB][H + 1];
    __shared__ float sdy[SPB], sse[SPB];
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) th[i] = theta[i];
    __syncthreads();
    const uint32_t t = threadIdx.x;
    if (t < SPB) {
        const uint32_t s = blockIdx.x * SPB + t;
        float x[IN], h1[H], h2[H];
        if (s < B) {
#pragma unroll
            for (int i = 0; i < IN; i++) x[i] = X[(size_t)s * IN + i];
        } else {
#pragma unroll
            for (int i = 0; i < IN; i++) x[i] = 0.f;
        }
        const float y = mlp_sample(th, x, h1, h2);
        // L = (1/B) sum (y - t)^2  ->  dL/dy = 2 (y - t) / B; padded samples contribute 0
        const float err = s < B ? y - T[s] : 0.f;
        const float dy = 2.f * err / (float)B;
        sdy[t] = dy;
        sse[t] = err * err;
#pragma unroll
        for (int i = 0; i < IN; i++) sx[t][i] = x[i];
        float dh2[H];
        for (int j = 0; j < H; j++) {
            sh1[t][j] = h1[j];
            sh2[t][j] = h2[j];
            dh2[j] = h2[j] > 0.f ? dy * th[OFF_W3 + j] : 0.f;
            sdh2[t][j] = dh2[j];
        }
        for (int i = 0; i < H; i++) {
            float a = 0.f;
#pragma unroll 8
            for (int j = 0; j < H; j++) a = fmaf(dh2[j], th[OFF_W2 + j * H + i], a);
            sdh1[t][i] = h1[i] > 0.f ? a : 0.f;
        }
    }
    __syncthreads();
    float *out = part + (size_t)blockIdx.x * (NPARAM + 1);
    for (int p = t; p < NPARAM + 1; p += blockDim.x) {
        float g = 0.f;
        if (p < OFF_B1) {  // W1[j][i] = sum_s dh1[s][j] x[s][i]
            const int j = p / IN, i = p % IN;
            for (int s = 0; s < SPB; s++) g = fmaf(sdh1[s][j], sx[s][i], g);
        } else if (p < OFF_W2) {
            const int j = p - OFF_B1;
            for (int s = 0; s < SPB; s++) g += sdh1[s][j];
        } else if (p < OFF_B2) {  // W2[j][i] = sum_s dh2[s][j] h1[s][i]
            const int j = (p - OFF_W2) / H, i = (p - OFF_W2) % H;
            for (int s = 0; s < SPB; s++) g = fmaf(sdh2[s][j], sh1[s][i], g);
        } else if (p < OFF_W3) {
            const int j = p - OFF_B2;
            for (int s = 0; s < SPB; s++) g += sdh2[s][j];
        } else if (p < OFF_B3) {  // W3[i] = sum_s dy[s] h2[s][i]
            const int i = p - OFF_W3;
            for (int s = 0; s < SPB; s++) g = fmaf(sdy[s], sh2[s][i], g);
        } else if (p == OFF_B3) {
            for (int s = 0; s < SPB; s++) g += sdy[s];
        } else {
            for (int s = 0; s < SPB; s++) g += sse[s];
        }
        out[p] = g;
    }
}

// grad[p] = sum over blocks of part[b][p], in block order; loss = sse / B.
__global__ void mlp_reduce_kernel(const float *__restrict__ part, uint32_t nblocks, uint32_t B,
                                  float *__restrict__ grad, float *__restrict__ loss) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > (uint32_t)NPARAM) return;
    float g = 0.f;
    for (uint32_t b = 0; b < nblocks; b++) g += part[(size_t)b * (NPARAM + 1) + p];
    if (p < (uint32_t)NPARAM) grad[p] = g;
    else if (loss) *loss = g / (float)B;
}

__global__ void mlp_adam_kernel(float *__restrict__ theta, const float *__restrict__ grad, float *__restrict__ m,
                                float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint32_t)NPARAM) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace

extern "C" uint32_t hyena_mlp_params(void) { return NPARAM; }

extern "C" size_t hyena_mlp_workspace_floats(uint32_t B) {
    return (size_t)((B + SPB - 1) / SPB) * (NPARAM + 1);
}

extern "C" int hyena_mlp_forward(const float *d_theta, const float *d_x, uint32_t B, float *d_y,
                                 hyena_stream_t stream) {
    if (!d_theta || (B && (!d_x || !d_y))) return set_error(HYENA_EINVAL, "hyena_mlp_forward: NULL argument");
    if (B == 0) return HYENA_OK;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_theta, d_x,
                       B, d_y);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HYENA_OK : set_error(HYENA_EHIP, std::string("hyena_mlp_forward: ") + hipGetErrorString(e));
}

extern "C" int hyena_mlp_loss_grad(const float *d_theta, const float *d_x, const float *d_t, uint32_t B,
                                   float *d_grad, float *d_loss, float *d_work, hyena_stream_t stream) {
    if (!d_theta || !d_x || !d_t || !d_grad || !d_work || B == 0)
        return set_error(HYENA_EINVAL, "hyena_mlp_loss_grad: bad argument");
    const hipStream_t s = (hipStream_t)stream;
    const uint32_t nb = (B + SPB - 1) / SPB;
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(nb), dim3(256), 0, s, d_theta, d_x, d_t, B, d_work);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, s, (const float *)d_work,
                       nb, B, d_grad, d_loss);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HYENA_OK : set_error(HYENA_EHIP, std::string("hyena_mlp_loss_grad: ") + hipGetErrorString(e));
}

extern "C" int hyena_mlp_adam(float *d_theta, const float *d_grad, float *d_m, float *d_v, uint32_t step, float lr,
                              float beta1, float beta2, float eps, hyena_stream_t stream) {
    if (!d_theta || !d_grad || !d_m || !d_v || step == 0) return set_error(HYENA_EINVAL, "hyena_mlp_adam: bad argument");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_theta, d_grad,
                       d_m, d_v, lr, beta1, beta2, eps, c1, c2);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HYENA_OK : set_error(HYENA_EHIP, std::string("hyena_mlp_adam: ") + hipGetErrorString(e));
}
