// Measurement helper, not part of the method: the sustained FP32 multiply-add
// rate of the vector ALUs, against which the fused kernels' roofline
// fraction is also stated.  Built into its own library (libwb_peak.so) and
// used only by the benchmark.
//
// Each lane runs `iters` trips of 16 independent fused multiply-adds
// x <- x * b + c (one v_fma_f32 each, 2 FLOP; packed FP32 is disabled in
// this build, as in the library), so the 16 chains cover the FMA latency;
// b and c are run-time values, so nothing folds.  Each lane stores the sum
// of its chains, which keeps them live.  A launch does
// blocks * 256 * iters * 32 FLOP.
#include <hip/hip_runtime.h>
#include <cstdint>

namespace {

constexpr int CHAINS = 16;

__global__ void __launch_bounds__(256) k_fma_peak(float *__restrict__ out, int iters, float b, float c) {
    float x[CHAINS];
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) x[i] = (float)threadIdx.x * 1e-7f + (float)i;
    for (int t = 0; t < iters; ++t) {
#pragma unroll
        for (int i = 0; i < CHAINS; ++i) x[i] = __builtin_fmaf(x[i], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) s += x[i];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

// Launches `blocks` workgroups of 256 lanes on `stream`; out holds
// blocks * 256 floats (device memory, caller-owned).  Returns the HIP
// status of the launch (0 on success); invalid sizes return
// hipErrorInvalidValue without launching.
extern "C" int wb_peak_fma(int64_t blocks, int32_t iters, float b, float c, float *out, hipStream_t stream) {
    if (blocks <= 0 || blocks > (1 << 20) || iters <= 0 || !out) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fma_peak, dim3((unsigned)blocks), dim3(256), 0, stream, out, iters, b, c);
    return (int)hipGetLastError();
}

// FLOP of one wb_peak_fma launch.
extern "C" double wb_peak_fma_flop(int64_t blocks, int32_t iters) {
    return (double)blocks * 256.0 * (double)iters * (double)CHAINS * 2.0;
}
