// Issue-rate measurement of the vector ALU on the device (a profiling tool,
// not part of the library): every thread runs 8 independent chains of one
// instruction kind, many waves per SIMD, and the rate is lane-operations per
// second from HIP events around the launch.  It backs the VALU peak that the
// tracer's roofline uses: a plain FP32 FMA stream against the 256 CUs x 4
// SIMDs x 2.4 GHz of the device, and the rate of the hardware transcendentals.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

template <int OP>
__global__ __launch_bounds__(256) void chains(float *out, int iters) {
    float x[8];
    for (int j = 0; j < 8; ++j) x[j] = 0.5f + 0.01f * (float)(threadIdx.x + j);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (OP == 0) x[j] = x[j] * 0.999f + 0.0001f;                         // v_fma_f32
            if (OP == 1) x[j] = x[j] + 0.25f;                                     // v_add_f32
            if (OP == 2) x[j] = __builtin_amdgcn_exp2f(x[j]) * 0.25f;             // v_exp_f32 (+ v_mul_f32)
            if (OP == 3) x[j] = __builtin_amdgcn_sqrtf(x[j]) + 0.25f;             // v_sqrt_f32 (+ v_add_f32)
            if (OP == 4)                                                          // v_mul_hi_u32
                x[j] = __builtin_bit_cast(float, __umulhi(__builtin_bit_cast(unsigned, x[j]), 0xD2511F53u) | 1u);
        }
    }
    float s = 0.0f;
    for (int j = 0; j < 8; ++j) s += x[j];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int OP>
float run(float *out, int blocks, int iters) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0f;
    float ms = -1.0f;
    for (int rep = 0; rep < 2; ++rep) {   // the first launch warms up
        if (hipEventRecord(a) != hipSuccess) return -1.0f;
        hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(256), 0, 0, out, iters);
        if (hipEventRecord(b) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return -1.0f;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

}  // namespace

int main() {
    const int blocks = 8192, iters = 4096;
    float *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return 1;
    const char *names[] = {"fma_f32", "add_f32", "exp_f32+mul_f32", "sqrt_f32+add_f32", "mul_hi_u32+or_b32"};
    float ms[5] = {run<0>(out, blocks, iters), run<1>(out, blocks, iters), run<2>(out, blocks, iters),
                   run<3>(out, blocks, iters), run<4>(out, blocks, iters)};
    const double lane_ops = (double)blocks * 256 * iters * 8;
    for (int k = 0; k < 5; ++k) {
        if (ms[k] < 0.0f) return 2;
        std::printf("{\"op\": \"%s\", \"ms\": %.4f, \"lane_ops_per_s\": %.4e}\n", names[k], ms[k],
                    lane_ops / (ms[k] * 1e-3));
    }
    (void)hipFree(out);
    return 0;
}
