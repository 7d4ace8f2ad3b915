// gb_noalloc.hip -- gb_verify_many_noalloc: the single-n batch of
// gb_verify_many with no device allocation in the call.  Its scratch (the
// exhaustive phase's work list of GbExh entries, the list's length and a
// flags word) is the file-scope device array `scratch` below, of a fixed
// size: every context on a device shares that device's copy, which keeps the
// last call's contents until the process ends.  Calls that overlap on one
// device race on it.
#include <algorithm>
#include <mutex>
#include <string>

#include "gb_runtime.h"

namespace {

constexpr uint64_t kNoAllocMaxN = 1ull << 16;                 // n per call
constexpr size_t kListBytes = kNoAllocMaxN * sizeof(GbExh);   // 2 MiB
constexpr size_t kScratchBytes = kListBytes + 256;            // + list length, flags

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Host-side record of each device's copy of `scratch`: the name above is
// only a host stand-in, so kernels and copies get the address found here.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];
bool g_done[kMaxDevices];

constexpr unsigned long long kBadN = 1ull, kUnresolved = 2ull;

// List entry i is query n[i] from table index 0; an n that is odd, below 4
// or above 2^63 is replaced by 4 (so the search stays bounded) and flagged.
__global__ void k_make_queries_checked(GbExh *list, const unsigned long long *n, uint64_t k,
                                       unsigned long long *count, unsigned long long *flags)
{
    const unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    if (i < k) {
        unsigned long long v = n[i];
        if (v < 4ull || (v & 1ull) || v > 9223372036854775808ull) {
            atomicOr(flags, kBadN);
            v = 4ull;
        }
        GbExh x;
        x.n = v;
        x.out_index = ~0ull;
        x.slot = 0;
        x.start_k = 0;
        x.p = 0;
        list[i] = x;
    }
    if (i == 0) *count = k;
}

__global__ void k_finish_queries_checked(const GbExh *list, uint64_t k, unsigned long long *p_out,
                                         unsigned long long *flags)
{
    const unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    if (i < k) {
        const unsigned long long p = list[i].p;
        p_out[i] = p;
        if (p == 0ull) atomicOr(flags, kUnresolved);
    }
}

}  // namespace

namespace gbrt {

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) {
        void *p = nullptr;
        g_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[device] = g_err[device] == hipSuccess ? p : nullptr;
        g_done[device] = true;
    }
    return g_err[device];
}

}  // namespace gbrt

using namespace gbrt;

extern "C" gb_status gb_verify_many_noalloc(gb_ctx *c, const uint64_t *n, uint64_t *p, size_t k, void *stream)
{
    if (!c) return GB_EINVAL;
    if (k == 0) return GB_OK;
    if (!n || !p) return fail(c, GB_EINVAL, "null argument");
    if (k > kNoAllocMaxN)
        return fail(c, GB_EINVAL, "the no-allocation form takes at most " + std::to_string(kNoAllocMaxN) +
                                      " n per call (" + std::to_string(k) + " given)");
    const int dev = c->prm.device;
    if (hipSetDevice(dev) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (dev >= 0 && dev < kMaxDevices) base = g_ptr[dev];
    }
    if (!base) return fail(c, GB_EDEVICE, "the scratch array's device address is not known on this device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    GbExh *list = static_cast<GbExh *>(base);
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(static_cast<unsigned char *>(base) + kListBytes);
    // ctr[0]: list length, ctr[1]: flags; both from zero (a fill kernel)
    GB_HIP(c, gb_launch_init(nullptr, 0, nullptr, 0, ctr, 2, st));
    const uint32_t grid = (uint32_t)((k + 255) / 256);
    hipLaunchKernelGGL(k_make_queries_checked, dim3(grid), dim3(256), 0, st, list,
                       reinterpret_cast<const unsigned long long *>(n), (uint64_t)k, ctr, ctr + 1);
    GB_HIP(c, hipGetLastError());
    GbMrArgs m{};
    m.list = list;
    m.list_count = ctr;
    m.list_cap = kNoAllocMaxN;
    m.primes = c->d_primes;
    m.ntab = c->ntab;
    m.budget = c->prm.exhaustive_budget_p;
    GB_HIP(c, gb_launch_mr(m, (uint32_t)std::min<uint64_t>((uint64_t)c->num_cu * 8u, (k + 3) / 4), st));
    hipLaunchKernelGGL(k_finish_queries_checked, dim3(grid), dim3(256), 0, st, list, (uint64_t)k,
                       reinterpret_cast<unsigned long long *>(p), ctr + 1);
    GB_HIP(c, hipGetLastError());
    unsigned long long flags = 0;
    GB_HIP(c, hipMemcpyAsync(&flags, ctr + 1, sizeof flags, hipMemcpyDeviceToHost, st));
    GB_HIP(c, hipStreamSynchronize(st));
    if (flags & kBadN) return fail(c, GB_EINVAL, "n must be even with 4 <= n <= 2^63");
    if (flags & kUnresolved) return fail(c, GB_EUNRESOLVED, "n without a partition within the budget");
    return GB_OK;
}
