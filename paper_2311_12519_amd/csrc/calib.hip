// Integer instruction rates of the chip, measured: the ALU roof that the
// multiply-accumulate's and the NTT's roofline fractions are quoted against.
// Every lane runs eight independent dependency chains of one operation; the
// chains' results are combined and stored so that nothing is optimised away.
#include <string>

#include "internal.h"

namespace {

constexpr int kChains = 8;

template <int OP>
__global__ void __launch_bounds__(256) rate_kernel(uint32_t iters, uint32_t seed, uint32_t *out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[kChains];
    uint64_t w[kChains];
#pragma unroll
    for (int c = 0; c < kChains; c++) {
        a[c] = t * 2654435761u + seed + c;
        w[c] = a[c];
    }
    const uint32_t m = seed | 1u;
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
#pragma unroll
            for (int c = 0; c < kChains; c++) {
                // the empty asm makes each result opaque, so that the compiler
                // cannot merge consecutive operations of a chain (a m m into
                // a m^2, a + m + m into a + 2m)
                if constexpr (OP == 0) {
                    // v_mad_u64_u32: 32 x 32 -> 64-bit product plus a 64-bit addend
                    w[c] = (uint64_t)(uint32_t)w[c] * m + w[c];
                    asm volatile("" : "+v"(w[c]));
                } else if constexpr (OP == 1) {
                    a[c] = a[c] * m;            // v_mul_lo_u32
                    asm volatile("" : "+v"(a[c]));
                } else if constexpr (OP == 2) {
                    a[c] = __umulhi(a[c], m);   // v_mul_hi_u32
                    asm volatile("" : "+v"(a[c]));
                } else {
                    a[c] = a[c] + m;            // v_add_u32
                    asm volatile("" : "+v"(a[c]));
                }
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; c++) r ^= a[c] ^ (uint32_t)w[c] ^ (uint32_t)(w[c] >> 32);
    out[t] = r;
}

}  // namespace

extern "C" int hyena_valu_rate(int op, uint32_t blocks, uint32_t iters, uint32_t *d_out, float *ms,
                               double *lane_ops) {
    if (!d_out || !ms || !lane_ops || op < 0 || op > 3 || !blocks || !iters)
        return set_error(HYENA_EINVAL, "hyena_valu_rate: bad argument");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto launch = [&] {
        switch (op) {
            case 0: hipLaunchKernelGGL(rate_kernel<0>, dim3(blocks), dim3(256), 0, 0, iters, 12345u, d_out); break;
            case 1: hipLaunchKernelGGL(rate_kernel<1>, dim3(blocks), dim3(256), 0, 0, iters, 12345u, d_out); break;
            case 2: hipLaunchKernelGGL(rate_kernel<2>, dim3(blocks), dim3(256), 0, 0, iters, 12345u, d_out); break;
            default: hipLaunchKernelGGL(rate_kernel<3>, dim3(blocks), dim3(256), 0, 0, iters, 12345u, d_out); break;
        }
    };
    launch();   // warm-up (clocks up)
    launch();
    HIP_TRY(hipEventRecord(e0, 0));
    launch();
    HIP_TRY(hipEventRecord(e1, 0));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_valu_rate: ") + hipGetErrorString(e));
    *lane_ops = (double)blocks * 256.0 * iters * 4.0 * kChains;
    return HYENA_OK;
}
