// gb_peaks.hip -- measured throughput ceilings of the units the kernels use:
// integer VALU issue (a two-operand and a three-operand instruction), LDS
// reads and LDS atomics without bank conflicts, and a streaming HBM copy.
// The roofline fractions reported beside the nominal peaks divide by these.
#include <cstring>

#include "gb_runtime.h"

namespace {

constexpr int PK_THREADS = 256;
constexpr int PK_CHAINS = 16;      // independent dependency chains per lane

// Each lane runs PK_CHAINS independent chains of one instruction, iters times.
#define GB_PEAK_VALU(NAME, ASM)                                                         \
    __global__ __launch_bounds__(PK_THREADS) void NAME(uint32_t *out, int iters)         \
    {                                                                                    \
        const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;                        \
        const uint32_t a = t * 2654435761u | 1u, b = (t ^ 0x5bd1e995u) | 3u;             \
        uint32_t c[PK_CHAINS];                                                           \
        for (int j = 0; j < PK_CHAINS; ++j) c[j] = t + (uint32_t)j;                      \
        for (int i = 0; i < iters; ++i) {                                                \
            _Pragma("unroll") for (int j = 0; j < PK_CHAINS; ++j)                        \
                asm volatile(ASM : "+v"(c[j]) : "v"(a), "v"(b));                         \
        }                                                                                \
        uint32_t r = 0;                                                                  \
        for (int j = 0; j < PK_CHAINS; ++j) r ^= c[j];                                   \
        out[t] = r;                                                                      \
    }

GB_PEAK_VALU(k_peak_vop2, "v_xor_b32 %0, %1, %0")
GB_PEAK_VALU(k_peak_vop3, "v_alignbit_b32 %0, %0, %1, %2")

// Every lane reads its own 16 bytes (consecutive lanes, consecutive words):
// two 16-byte reads per round.
__global__ __launch_bounds__(PK_THREADS) void k_peak_lds_read(uint32_t *out, int iters)
{
    __shared__ __align__(16) uint32_t s[4096];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < 4096; i += PK_THREADS) s[i] = i * 2654435761u;
    __syncthreads();
    const uint32_t addr = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)s + 16u * t;
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
        uint4 v0, v1;
        asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:4096\n\ts_waitcnt lgkmcnt(0)"
                     : "=v"(v0), "=v"(v1) : "v"(addr));
        acc += v0.x ^ v1.w;
    }
    out[blockIdx.x * blockDim.x + t] = acc;
}

// Every lane ANDs a mask into its own word: four atomics per round.
__global__ __launch_bounds__(PK_THREADS) void k_peak_lds_and(uint32_t *out, int iters)
{
    __shared__ uint32_t s[4096];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < 4096; i += PK_THREADS) s[i] = ~0u;
    __syncthreads();
    const uint32_t addr = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)s + 4u * t;
    const uint32_t m = ~(1u << (t & 31u));
    for (int i = 0; i < iters; ++i)
        asm volatile("ds_and_b32 %0, %1\n\tds_and_b32 %0, %1 offset:1024\n\t"
                     "ds_and_b32 %0, %1 offset:2048\n\tds_and_b32 %0, %1 offset:3072"
                     : : "v"(addr), "v"(m) : "memory");
    __syncthreads();
    out[blockIdx.x * blockDim.x + t] = s[t];
}

__global__ __launch_bounds__(PK_THREADS) void k_peak_copy(const uint4 *src, uint4 *dst, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * PK_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * PK_THREADS + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

using namespace gbrt;

gb_status gb_measure_peaks(gb_ctx *c, gb_peaks *out, void *stream)
{
    if (!c || !out) return fail(c, GB_EINVAL, "null argument");
    std::memset(out, 0, sizeof *out);
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t grid = (uint32_t)c->num_cu * 16u;
    const size_t lanes = (size_t)grid * PK_THREADS;
    const uint64_t copy_bytes = 256ull << 20;       // per buffer
    if (2 * copy_bytes + lanes * 4 > c->prm.mem_budget) return fail(c, GB_ENOMEM, "mem_budget too small");
    uint32_t *sink = nullptr;
    uint4 *src = nullptr, *dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    gb_status stt = GB_OK;
    auto hip = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && stt == GB_OK) stt = fail(c, GB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return e == hipSuccess;
    };
    // best of three timed launches of one kernel
    auto best_ms = [&](auto launch) {
        float best = 0.f;
        for (int rep = 0; rep < 4 && stt == GB_OK; ++rep) {
            hip(hipEventRecord(e0, st), "hipEventRecord");
            launch();
            hip(hipGetLastError(), "launch");
            hip(hipEventRecord(e1, st), "hipEventRecord");
            hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (rep > 0 && (best == 0.f || ms < best)) best = ms;   // the first run warms up
        }
        return (double)best;
    };
    if (hip(hipMalloc(&sink, lanes * 4), "hipMalloc") && hip(hipMalloc(&src, copy_bytes), "hipMalloc") &&
        hip(hipMalloc(&dst, copy_bytes), "hipMalloc") && hip(hipEventCreate(&e0), "hipEventCreate") &&
        hip(hipEventCreate(&e1), "hipEventCreate")) {
        const int iters = 2048;
        const double wave_instr = (double)lanes / 64.0 * iters * PK_CHAINS;
        double ms = best_ms([&] { hipLaunchKernelGGL(k_peak_vop2, dim3(grid), dim3(PK_THREADS), 0, st, sink, iters); });
        if (ms > 0) out->valu_vop2_ops = wave_instr * 64.0 / (ms * 1e-3);
        ms = best_ms([&] { hipLaunchKernelGGL(k_peak_vop3, dim3(grid), dim3(PK_THREADS), 0, st, sink, iters); });
        if (ms > 0) out->valu_vop3_ops = wave_instr * 64.0 / (ms * 1e-3);
        ms = best_ms([&] { hipLaunchKernelGGL(k_peak_lds_read, dim3(grid), dim3(PK_THREADS), 0, st, sink, iters); });
        if (ms > 0) out->lds_read_bytes = (double)lanes * iters * 32.0 / (ms * 1e-3);
        ms = best_ms([&] { hipLaunchKernelGGL(k_peak_lds_and, dim3(grid), dim3(PK_THREADS), 0, st, sink, iters); });
        if (ms > 0) out->lds_atomic_ops = (double)lanes * iters * 4.0 / (ms * 1e-3);
        hip(hipMemsetAsync(src, 1, copy_bytes, st), "hipMemsetAsync");
        const uint64_t n16 = copy_bytes / 16;
        ms = best_ms([&] { hipLaunchKernelGGL(k_peak_copy, dim3(grid * 4), dim3(PK_THREADS), 0, st, src, dst, n16); });
        if (ms > 0) out->hbm_copy_bytes = 2.0 * (double)copy_bytes / (ms * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    return stt;
}
