// gb_device.h -- device helpers shared by the tile kernels (gb_kernels.hip,
// gb_class.hip).  Not a public header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gb_internal.h"

namespace {

typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4u32 lds_v4;

// LDS byte address bw + bits 31..16 of the packed prime word x.
__device__ __forceinline__ const lds_u32 *probe_addr(uint32_t x, uint32_t bw)
{
    uint32_t d;
    asm("v_mad_u32_u16 %0, 1, %1, %2 op_sel:[0,1,0,0]" : "=v"(d) : "v"(x), "v"(bw));
    return reinterpret_cast<const lds_u32 *>(static_cast<uintptr_t>(d));
}

// p * (bits 15..0 of x) + acc, p < 2^16, in one v_mad_u32_u16.
__device__ __forceinline__ uint32_t mad_lo16(uint32_t p, uint32_t x, uint32_t acc)
{
    uint32_t d;
    asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(d) : "v"(p), "v"(x), "v"(acc));
    return d;
}

template <int PB>
__device__ __forceinline__ void store_p(void *out, unsigned long long idx, uint32_t p)
{
    if constexpr (PB == 16) static_cast<uint16_t *>(out)[idx] = (uint16_t)p;
    if constexpr (PB == 32) static_cast<uint32_t *>(out)[idx] = p;
}

// The histogram row a workgroup's LDS hit counts belong to, and the n
// counted into them since they were last flushed (the same in every thread).
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
struct HistCarry {
    uint32_t row = kNoRow;
    unsigned long long n = 0;
    bool stored = false;   // the counts went to the workgroup's own row once
};

// The slot summaries a workgroup carries from tile to tile (thread 0, in
// LDS): one set of slot atomics and one argmax record per run of tiles of
// one slot instead of per tile.
constexpr unsigned long long kNoSlot = ~0ull;
enum { CY_COUNT, CY_SUM, CY_EXH, CY_ARGN, CY_SLOT, CY_MAXP };

__device__ inline void flush_slot(const GbTileArgs &a, unsigned long long *C)
{
    if (C[CY_SLOT] == kNoSlot) return;
    GbSlot *S = a.slots + C[CY_SLOT];
    atomicAdd(&S->count, C[CY_COUNT]);
    if (C[CY_SUM]) atomicAdd(&S->checksum, C[CY_SUM]);
    if (C[CY_EXH]) atomicAdd(&S->n_exhaustive, C[CY_EXH]);
    if (C[CY_MAXP]) {
        atomicMax(&S->max_p, C[CY_MAXP]);
        const unsigned long long e = atomicAdd(a.rec_count, 1ull);
        if (e < a.rec_cap) {
            GbTileRec r;
            r.argmax_n = C[CY_ARGN];
            r.max_p = (uint32_t)C[CY_MAXP];
            r.slot = (uint32_t)C[CY_SLOT];
            a.recs[e] = r;
        }
    }
    C[CY_SLOT] = kNoSlot;
}

}  // namespace
