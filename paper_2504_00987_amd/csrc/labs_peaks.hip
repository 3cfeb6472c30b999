// Measured throughput of the units the walk kernels are bound by, for the
// roofline the benchmark reports beside the published figures:
//
//   dot4_peak_kernel   v_dot4_i32_i8 (four int8 products summed into an
//                      int32 per lane per instruction): the contraction of
//                      the neighbour scoring
//   add_peak_kernel    plain 32-bit integer adds (one per lane per instruction)
//   lds_peak_kernel    conflict-free 16-byte LDS reads
//
// Each kernel runs independent dependency chains per lane on a grid of
// several workgroups per compute unit; the host times one launch with HIP
// events after a warm-up launch.
#include <hip/hip_runtime.h>

#include "../../include/liblabs.h"
#include "labs_handle.h"

namespace liblabs {

namespace {

constexpr int kPeakThreads = 256;
constexpr int kChains = 8;

// Wavefront 0 of workgroup 0 also times its loop in shader clocks and in
// ticks of the 100 MHz constant counter: the clock under this full load.
__global__ __launch_bounds__(kPeakThreads) void dot4_peak_kernel(int32_t *out, int iters,
                                                                 int seed, long long *clk) {
    const int t = blockIdx.x * kPeakThreads + threadIdx.x;
    const long long r0 = (long long)__builtin_amdgcn_s_memrealtime();
    const long long c0 = (long long)__builtin_readcyclecounter();
    int a[kChains], acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = t * 0x01010101 + 7 * c + seed;
        acc[c] = c;
    }
    int b = seed ^ 0x5a5a5a5a;  // wave-uniform: one scalar add per iteration
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_sdot4(a[c], b, acc[c], false);
        b += 0x01030507;
    }
    int s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s ^= acc[c];
    const long long c1 = (long long)__builtin_readcyclecounter();
    const long long r1 = (long long)__builtin_amdgcn_s_memrealtime();
    out[t] = s;
    if (t == 0) {
        clk[0] = c1 - c0;
        clk[1] = r1 - r0;
    }
}

__global__ __launch_bounds__(kPeakThreads) void add_peak_kernel(int32_t *out, int iters,
                                                                int seed) {
    const int t = blockIdx.x * kPeakThreads + threadIdx.x;
    int acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = t + c + seed;
    for (int i = 0; i < iters; ++i) {
        // one two-operand add per chain and iteration (nothing to fuse)
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] += acc[(c + 1) % kChains];
    }
    int s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s ^= acc[c];
    out[t] = s;
}

constexpr int kLdsRecords = 1024;  // 16 KB of 16-byte records per workgroup
constexpr int kLdsUnroll = 4;

// `step` is odd and only known at run time, so the compiler can neither
// hoist the reads nor fold their repetition; a wavefront reads 64
// consecutive records (1 KB, no bank conflict) per instruction.
__global__ __launch_bounds__(kPeakThreads) void lds_peak_kernel(int32_t *out, int iters,
                                                                int seed, int step) {
    __shared__ uint4 buf[kLdsRecords];
    for (int i = threadIdx.x; i < kLdsRecords; i += kPeakThreads)
        buf[i] = make_uint4(i, i ^ seed, i + seed, ~i);
    __syncthreads();
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    int base = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kLdsUnroll; ++k) {
            const uint4 v = buf[(base + 64 * (wave + 4 * k)) & (kLdsRecords - 1)];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        base += 64 * step;
    }
    out[blockIdx.x * kPeakThreads + threadIdx.x] = (int)(acc.x ^ acc.y ^ acc.z ^ acc.w);
}

}  // namespace

}  // namespace liblabs

using namespace liblabs;

extern "C" int labs_device_peaks(labs_handle *h, double *dot4_products_per_s, double *int32_ops_per_s,
                                 double *lds_bytes_per_s, double *clock_hz) {
    if (!h) return LABS_E_INVAL;
    h->last_error.clear();
    if (!dot4_products_per_s || !int32_ops_per_s || !lds_bytes_per_s || !clock_hz)
        return fail(h, LABS_E_INVAL, "null output");
    DeviceGuard g(h->device);
    hipStream_t s = h->stream;
    const int groups_alu = 16 * h->num_cus;  // four wavefronts per SIMD
    const int groups_lds = 8 * h->num_cus;   // 128 KB of LDS per compute unit
    const size_t threads = (size_t)groups_alu * kPeakThreads;
    int32_t *out = nullptr;
    hipError_t e = hipMalloc(&out, threads * sizeof(int32_t) + 64);
    long long *clk = (long long *)(out + threads);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, LABS_E_NOMEM, "peak buffers");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    constexpr int kIters = 4096;
    constexpr int kLdsIters = 2048;
    float ms[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // warm-up, then timed
            if (rep == 1) e = hipEventRecord(e0, s);
            if (e != hipSuccess) break;
            if (k == 0)
                hipLaunchKernelGGL(dot4_peak_kernel, dim3(groups_alu), dim3(kPeakThreads), 0, s,
                                   out, kIters, 12345, clk);
            else if (k == 1)
                hipLaunchKernelGGL(add_peak_kernel, dim3(groups_alu), dim3(kPeakThreads), 0, s,
                                   out, kIters, 12345);
            else
                hipLaunchKernelGGL(lds_peak_kernel, dim3(groups_lds), dim3(kPeakThreads), 0, s,
                                   out, kLdsIters, 12345, 2 * (int)(h->num_cus & 7) + 5);
            e = hipGetLastError();
            if (e == hipSuccess && rep == 1) e = hipEventRecord(e1, s);
        }
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[k], e0, e1);
    }
    long long ticks[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(ticks, clk, sizeof(ticks), hipMemcpyDeviceToHost);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(out);
    if (e != hipSuccess) return hip_fail(h, e, "peak kernels");
    *dot4_products_per_s = (double)threads * kIters * kChains * 4 / (ms[0] * 1e-3);
    *int32_ops_per_s = (double)threads * kIters * kChains / (ms[1] * 1e-3);
    *lds_bytes_per_s = (double)groups_lds * kPeakThreads * kLdsIters * kLdsUnroll * 16 /
                       (ms[2] * 1e-3);
    *clock_hz = ticks[1] > 0 ? (double)ticks[0] / ((double)ticks[1] * 1e-8) : 0.0;
    return LABS_OK;
}
