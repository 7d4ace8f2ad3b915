// gb_internal.h -- device-side data layout shared by the kernels and the
// host runtime of the Goldbach verifier (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GB_HIST_BINS_I 6543u

// One window of consecutive even n.  A range call uses one window per
// segment; the batched forms put many windows in one table.
// The planner moves first_n down to a multiple of 384 and masks the `lead`
// n it adds in front, so a block of 64 n of one class mod 6 always lies in
// one stretch of 384 integers.
struct GbWindow {
    uint64_t first_n;    // even; a multiple of 384 for the search
    uint64_t count;      // even n in the window, the lead included
    uint64_t tile_base;  // global index of the window's first tile
    uint64_t out_off;    // per-n output index of the first n after the lead
    uint32_t slot;       // summary slot of the window
    uint32_t np_sieve;   // odd primes p of the table with p*p <= window top
    uint32_t lead;       // masked n in front of the window (0..191)
    uint32_t pad;
};

// Per-slot summary accumulators, combined with 64-bit atomics (sums, max,
// min), so the result does not depend on the order tiles finish in.
struct GbSlot {
    unsigned long long count, max_p, argmax_n, checksum, n_exhaustive,
        n_failed, first_failed_n, pad;
};

// Record for the argmax pass: the largest p_min of a run of tiles of one
// slot that one workgroup took in turn, and the smallest n of the run that
// has it.
struct GbTileRec {
    unsigned long long argmax_n;
    uint32_t max_p;
    uint32_t slot;
};

// One n sent to the exhaustive phase (or one single-n query).
struct GbExh {
    unsigned long long n;
    unsigned long long out_index;  // index into the per-n output, or ~0
    uint32_t slot;
    uint32_t start_k;              // first odd-prime index to try
    unsigned long long p;          // result: p_min, or 0 for a failure
};

struct GbTileArgs {
    const GbWindow *win;
    uint32_t nwin;
    uint32_t tile_n;        // T, even n per tile (multiple of 64)
    uint64_t ntiles;        // tiles in the whole table (persistent mode)
    uint64_t tile0;         // first tile of this launch (non-persistent)
    uint32_t halo_bits;     // HB: bits below the tile's first n (multiple of 64)
    const uint32_t *primes; // odd primes 3, 5, 7, ... ascending
    const unsigned long long *magic;  // floor((2^64-1)/p) per prime
    uint32_t k_first;       // first prime index above the wheel
    uint32_t k_wg_end;      // primes [k_first, k_wg_end): whole-workgroup marking
    uint32_t k_wave_end;    // primes [k_wg_end, k_wave_end): one wave per prime
    const uint32_t *wheel;  // wheel pattern bits, period wheel_len, padded by 64
    uint32_t wheel_len;     // product of the odd wheel primes
    uint32_t wheel_max;     // largest wheel prime
    void *pmin;             // per-n output (nullable)
    GbSlot *slots;
    unsigned long long *hist;  // rows of GB_HIST_BINS_I
    uint32_t hist_per_slot;    // 1: row = slot, 0: row 0
    GbTileRec *recs;           // argmax records, appended by workgroups
    unsigned long long *rec_count;  // records appended so far
    unsigned long long rec_cap;     // capacity of recs (at least the tile count)
    GbExh *list;
    unsigned long long *list_count;
    unsigned long long list_cap;
    unsigned long long *queue; // persistent work counter
    uint32_t *sieve_out;       // sieve-only mode: bitset dump
    // the search split by residue mod 6 (gb_class.hip): tile_n = 192 sb_per_tile
    const uint32_t *cls;       // class headers, sieve tables and probe records (GB_CLS_*)
    uint32_t cls_words;
    uint32_t np_cls;           // odd primes on the class lists (the first np_cls of the table)
    uint32_t hk;               // plane bits below a tile's first stretch (a multiple of 64)
    uint32_t sb_per_tile;      // stretches of 384 integers per full tile
    const uint32_t *wheel6;    // two plane patterns of period wheel6_len, wheel6_stride words each
    uint32_t wheel6_len;
    uint32_t wheel6_stride;
    uint32_t k6_first;         // first prime index above the wheel
    uint32_t k6_wave_end;      // [k6_first, k6_wave_end): one wave per prime
    uint32_t k6_single;        // from here on p >= plane bits of a full tile: one strike per plane at most
    uint64_t sieve_stride;     // plane dump: words per plane in sieve_out
    uint32_t pmax_fast;        // P_max: n with a larger p_min count as exhaustive
    const uint4 *prime6;       // per odd prime of the table below 2^27: GB_PRIME6 entry
    uint32_t n_prime6;         // entries of prime6 (the first n_prime6 odd primes)
    // persistent k_cls: each workgroup's first histogram flush is stored (no
    // atomics) as row blockIdx.x of wg_hist, wg_hist_stride words each: the
    // histogram row it belongs to, then the hit count of every probe record
    // in class order (GB_CLS_*); k_hist_reduce adds the rows up.  Null: every
    // flush is a set of 64-bit atomics into hist.
    uint32_t *wg_hist;
    uint32_t wg_hist_stride;
    // persistent k_cls: tiles [0, static_tiles) go to workgroup t mod
    // gridDim.x in turn (static_tiles a multiple of gridDim.x), the rest to
    // whichever workgroup asks the queue first
    unsigned long long static_tiles;
};

// GbTileArgs::prime6 entry of the odd prime p: x = p, y = the least k >= 0
// with p | 6 k + 1, (w:z) = the bits of the double nearest 1/p.  The least
// k >= 0 with p | 6 k + 5 is then p - 1 - y.

// Layout of GbTileArgs::cls (32-bit words).  Class h = a/2 (a = 0, 2, 4):
// words 3h, 3h+1, 3h+2 = byte offset of its first probe record group from
// the records, number of its groups with real entries, byte offset of the
// end of the last of them (two more groups of copies follow).  Records from
// GB_CLS_HDR: groups of four entries, 12 words each (four packed probe
// words, four g = 2^16 - (p+1)/2, four hit counts).  A packed probe word
// holds the funnel shift in bits 4..0, the probe's row within the group's
// window in bit 5, its plane in bit 6 and, in bits 31..16, the byte offset
// of the group's window (rows R .. R+3 of both planes) from the block's
// first plane row.
#define GB_CLS_HDR 12u

struct GbMrArgs {
    GbExh *list;
    const unsigned long long *list_count;
    unsigned long long list_cap;
    const uint32_t *primes;
    uint64_t ntab;
    unsigned long long budget;   // 0 = n/2
    void *pmin;                  // per-n output of the range call (nullable)
    uint32_t pmin_bits;
    GbSlot *slots;               // nullable (queries)
    unsigned long long *hist;
    uint32_t hist_per_slot;
    uint32_t count_exh;          // count n_exhaustive here: an n whose p is 0 or above pmax_fast
    uint64_t pmax_fast;
};

// Kernel launchers (gb_kernels.hip).
// The odd-number sieve dump (non-persistent, one workgroup per tile).
hipError_t gb_launch_tiles(const GbTileArgs &a, uint32_t grid, uint32_t threads, size_t lds_bytes, hipStream_t st);
hipError_t gb_prepare_tiles(uint32_t threads, size_t lds_bytes);
size_t gb_tile_lds_bytes(uint32_t tile_n, uint32_t halo_bits, uint32_t n_off);
hipError_t gb_launch_mr(const GbMrArgs &a, uint32_t grid, hipStream_t st);
// The kernel of the search split by residue mod 6 (gb_class.hip).
size_t gb_cls_lds_bytes(uint32_t sb_per_tile, uint32_t hk, uint32_t cls_words);
hipError_t gb_cls_prepare(uint32_t threads, size_t lds_bytes);
hipError_t gb_cls_occupancy(uint32_t threads, size_t lds_bytes, int *blocks_per_cu);
hipError_t gb_launch_cls(const GbTileArgs &a, uint32_t grid, uint32_t threads, size_t lds_bytes, int pmin_bits,
                         bool persistent, bool sieve_only, hipStream_t st);
// Sum of the rows of GbTileArgs::wg_hist into the histogram rows they name
// (rows whose first word is 0xFFFFFFFF are skipped); rec_bin[r] is the
// histogram bin of probe record r.
hipError_t gb_launch_hist_reduce(const uint32_t *wg_hist, uint32_t nwg, uint32_t stride, uint32_t nrec,
                                 const uint32_t *rec_bin, unsigned long long *hist, hipStream_t st);
hipError_t gb_launch_argmax(GbSlot *slots, const GbTileRec *recs, const unsigned long long *rec_count,
                            unsigned long long rec_cap, const GbExh *list,
                            const unsigned long long *list_count, unsigned long long list_cap,
                            hipStream_t st);
hipError_t gb_launch_init(GbSlot *slots, uint64_t nslots, unsigned long long *hist,
                          uint64_t hist_words, unsigned long long *counters,
                          uint32_t ncounters, hipStream_t st);
hipError_t gb_launch_finish_queries(const GbExh *list, uint64_t k,
                                    unsigned long long *p_out, hipStream_t st);
hipError_t gb_launch_make_queries(GbExh *list, const unsigned long long *n, uint64_t k,
                                  unsigned long long *list_count, hipStream_t st);
