/*
 * goldbach.h -- C ABI of the MI355X segmented Goldbach verifier.
 *
 * The library computes, for every even n in a range (or a set of windows, or
 * a single n), the minimal Goldbach prime
 *
 *     p_min(n) = min { p prime : n - p prime },        n even, n >= 4,
 *
 * which is the first hit of the scan "primes p from 2 upward, stop when
 * q = n - p is prime" that the GoldbachGPU paper verifies (section "Methods",
 * CPU baseline; section "Segmented Double-Sieve Verifier").  The work is the
 * paper's segmented double sieve with the loop inverted (subsection "Correct
 * segmentation"): a bit-packed odd-only sieve of each tile's window is built
 * on the GPU, every candidate prime p up to P_max is probed against it for 64
 * even n at a time, and any n left unresolved goes to an exhaustive phase
 * that scans the primes above P_max in ascending order with a deterministic
 * Miller-Rabin test of q (the paper's Phase 2, done on the GPU here).
 *
 * Conventions shared by every call:
 *  - Ranges are inclusive: a range call covers every even n with
 *    max(lo, 4) <= n <= hi.  lo > hi (after rounding lo up and hi down to
 *    even) is an empty range and returns GB_OK with count 0.
 *  - n never exceeds GB_MAX_N = 2^63; range calls also need hi <= the
 *    context's max_hi.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call below is synchronous: it enqueues its work on `stream`,
 *    waits for it, and returns with all outputs written.
 *  - Device pointers must belong to the context's device.  Host pointers
 *    are ordinary (pageable) memory.
 *  - A context is not thread-safe; use one per host thread.  No call aborts
 *    or throws; on a status other than GB_OK the outputs are unspecified and
 *    gb_last_error() describes the failure.
 */
#ifndef GOLDBACH_H
#define GOLDBACH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gb_status {
    GB_OK = 0,
    GB_EINVAL = 1,      /* bad argument: n odd or < 4, n > 2^63, bad params */
    GB_ERANGE = 2,      /* hi above the context's max_hi */
    GB_ENOMEM = 3,      /* allocation failed, or the unresolved list overflowed */
    GB_EDEVICE = 4,     /* a HIP runtime error; text in gb_last_error() */
    GB_EUNRESOLVED = 5  /* some n had no partition with p <= min(n/2, budget):
                           the summaries are complete, n_failed > 0 and
                           first_failed_n names the smallest such n */
} gb_status;

/* Histogram bins: one per prime below 2^16 (2 -> bin 0, 3 -> bin 1, ...,
 * 65521 -> bin 6541) plus bin 6542 for p_min >= 2^16. */
#define GB_HIST_BINS 6543
#define GB_MAX_N 9223372036854775808ull /* 2^63 */

typedef struct gb_ctx gb_ctx;

/* Context parameters.  A zero field takes the documented default. */
typedef struct gb_params {
    int32_t  device;        /* HIP device ordinal */
    uint32_t pmax;          /* fast-path bound P_max on p, 0..65535 (0 -> 8192).
                               Odd primes p <= P_max are probed against the
                               tile sieve; larger p belong to the exhaustive
                               phase.  Any value gives the same p_min. */
    uint32_t seg_log2;      /* plain form: S = 2^seg_log2 even n per segment
                               (one launch per segment), 16..30 (0 -> 24) */
    uint32_t tile_log2;     /* T = 2^tile_log2 even n per tile (one workgroup
                               sieves and searches one tile in LDS), 12..20
                               (0 -> 19) */
    uint32_t wg_threads;    /* threads per tile workgroup: 256, 512 or 1024
                               (0 -> 512) */
    uint32_t wheel_max;     /* largest prime of the pre-sieved wheel pattern:
                               7, 11, 13, 17 or 19 (0 -> 19) */
    uint32_t search_mode;   /* search variant; 1 (0 -> 1) is the only one:
                               each lane does the bookkeeping of its own hits.
                               Other values give GB_EINVAL. */
    uint32_t reserved;      /* must be 0 */
    uint64_t max_hi;        /* largest n any range call may reach; sizes the
                               resident sieving-prime table to sqrt(max_hi)
                               (0 -> 2^50; at most 2^63) */
    uint64_t exhaustive_budget_p; /* the exhaustive phase stops past this p
                               (0 -> n/2, i.e. a complete search) */
    uint64_t max_unresolved;/* capacity of the device list of n that the fast
                               path leaves to the exhaustive phase
                               (0 -> 2^20 entries, 32 bytes each) */
    uint64_t mem_budget;    /* serving: bytes of request buffers admitted at
                               once (0 -> 4 GiB) */
} gb_params;

/* Result of a range call.  The caller fills the first group (all optional)
 * and the library fills the second. */
typedef struct gb_result {
    void     *pmin;           /* per-n p_min, entry i for n = lo' + 2i, or NULL */
    uint32_t  pmin_bits;      /* 16 (p_min >= 2^16 and failures stored as 0)
                                 or 32 (failures stored as 0) */
    uint32_t  pmin_on_device; /* 1: pmin is device memory; 0: host memory */
    uint64_t *hist;           /* host, GB_HIST_BINS entries, or NULL */
    uint64_t *seg_hist;       /* host, seg_hist_rows * GB_HIST_BINS entries:
                                 one histogram per segment of S even n, or NULL */
    uint64_t  seg_hist_rows;
    /* filled by the library */
    uint64_t count;           /* even n examined */
    uint64_t max_p;           /* largest p_min */
    uint64_t argmax_n;        /* smallest n attaining max_p */
    uint64_t checksum;        /* sum of w(n) * p_min(n) modulo 2^64 over the
                                 n with a partition, where
                                 w(n) = 2^33 floor(n/128) + (2c+1) 2^i and
                                 (n/2) mod 64 = 32c + i, 0 <= i < 32.  The
                                 paper defines no checksum; sums over
                                 disjoint sets of n add up. */
    uint64_t n_exhaustive;    /* n that no odd prime p <= P_max resolved */
    uint64_t n_failed;        /* n without a partition within the budget */
    uint64_t first_failed_n;  /* smallest such n, or 0 */
    uint64_t n_segments;      /* segments (plain) or windows (batched) used */
    double   device_ms;       /* device time of the call, from HIP events */
    double   tile_ms;         /* device time of the sieve-and-search tile
                                 launches alone (HIP events on the same
                                 stream, around those launches) */
    uint64_t tile_launches;   /* tile kernel launches in the call */
} gb_result;

/* One window of the batched form: the even n start, start+2, ...,
 * start + 2*(len-1).  start is even and >= 4. */
typedef struct gb_window {
    uint64_t start;
    uint64_t len;
} gb_window;

/* Per-window summary of the batched form (fields as in gb_result). */
typedef struct gb_summary {
    uint64_t count, max_p, argmax_n, checksum, n_exhaustive, n_failed,
             first_failed_n;
} gb_summary;

/* Create a context on prm->device: builds the resident table of odd primes
 * up to sqrt(max_hi) (plus per-prime reciprocals), the wheel pattern and the
 * fast-path prime list, and keeps them in device memory until gb_destroy.
 * prm may be NULL (all defaults).  On failure *ctx is NULL. */
gb_status gb_create(gb_ctx **ctx, const gb_params *prm);
void      gb_destroy(gb_ctx *ctx);

/* The parameters in effect (defaults resolved). */
gb_status gb_get_params(const gb_ctx *ctx, gb_params *out);

/* The tile geometry the parameters resolve to (host values; no device
 * work): even n per tile of the minimal-p search (n split by residue mod 6:
 * the largest multiple of 192 whose two planes and probe lists fit the LDS,
 * from twice 2^tile_log2 down; the paper's tile is one segment, subsection
 * "Correct segmentation"), the LDS bytes of its workgroup, the odd primes on
 * its probe lists (P_max's, or fewer when LDS is short), and even n per tile
 * of the batched bulk form (the same tiles).  Any pointer may be NULL.
 * GB_EINVAL for a NULL ctx. */
gb_status gb_tile_geometry(const gb_ctx *ctx, uint64_t *cls_tile_n, uint64_t *cls_lds_bytes,
                           uint64_t *cls_list_primes, uint64_t *bulk_tile_n);

/* Plain form: p_min for every even n in [max(lo,4), hi], one kernel launch
 * per segment of S even n; consecutive segments go round-robin to `stream`
 * and up to seven library streams forked from it (no more than the process
 * has hardware queues, GPU_MAX_HW_QUEUES, 4 when unset) and joined back into
 * `stream`; then the exhaustive phase and the summary reduction.  (Problem statement: section "Methods"; the
 * segment loop: subsection "Correct segmentation".)  Returns GB_EUNRESOLVED
 * when some n has no partition within the budget. */
gb_status gb_verify_range(gb_ctx *ctx, uint64_t lo, uint64_t hi,
                          gb_result *res, void *stream);

/* Batched form of the same computation: all segments' tiles go to one
 * persistent launch that pulls tiles from a device work queue, captured with
 * the exhaustive phase and the reduction in one HIP graph, replayed on later
 * calls of the same shape.  Same results as gb_verify_range, bit for bit.
 * The paper has no such form: it runs its segments one after another, each
 * sieved on the host and copied over (subsection "Correct segmentation"),
 * and names that host loop as its bottleneck (section "Limitations"); this
 * call is the same computation with the segment loop moved onto the device. */
gb_status gb_verify_range_batched(gb_ctx *ctx, uint64_t lo, uint64_t hi,
                                  gb_result *res, void *stream);

/* Bulk verification of the same range (paper section "Discussion",
 * "Algorithmic gap with the state of the art": the verified set kept as a
 * bitset into which each prime's shifted segment window is OR-ed, instead of
 * a per-n lookup).  Every even n in [max(lo,4), hi] is shown to have a
 * partition p + q with p <= P_max from the tile sieve, or goes to the
 * exhaustive phase as in gb_verify_range.  No minimal p per n is recorded:
 * res->pmin, res->hist and res->seg_hist must be NULL (GB_EINVAL otherwise)
 * and res->checksum is 0.  res->count, max_p, argmax_n, n_exhaustive,
 * n_failed and first_failed_n equal those of gb_verify_range (the largest
 * p_min of a 64-n block is the prime that resolves its last n).  Batched
 * (persistent, graph-replayed) form only; same status codes. */
gb_status gb_verify_range_bulk(gb_ctx *ctx, uint64_t lo, uint64_t hi,
                               gb_result *res, void *stream);

/* Batched windows: k windows of uneven length in one persistent graph
 * launch.  pmin (nullable) is device memory of sum(len) uint16 entries,
 * window j's n at offset sum_{i<j} len_i.  sums (nullable, host, k entries)
 * receives each window's summary; hist (nullable, host, GB_HIST_BINS) the
 * histogram over all windows.  Windows may overlap.  The paper defines no
 * windows call (its verifier covers one range [4, N]); each window is the
 * range computation of gb_verify_range on [start, start + 2(len-1)], and
 * many of them share one launch.  The outputs are separate arguments rather
 * than one gb_result per window so that the k summaries come back in one
 * array and the per-n output of all windows in one device buffer. */
gb_status gb_verify_windows(gb_ctx *ctx, const gb_window *w, size_t k,
                            uint16_t *pmin, gb_summary *sums, uint64_t *hist,
                            void *stream);

/* Single n (section "GPU Single-Number Checker", but returning the minimal
 * p): one wavefront scans odd primes from 3 upward, 64 candidates at a time,
 * testing q = n - p with deterministic Miller-Rabin (bases 2..37), and takes
 * the lowest passing lane.  n must be even, 4 <= n <= 2^63.  *p receives
 * p_min(n), or 0 with GB_EUNRESOLVED if none exists within the budget.  The
 * result is the bare p (q = n - p): for one n the range summaries would
 * only repeat it. */
gb_status gb_verify_one(gb_ctx *ctx, uint64_t n, uint64_t *p, void *stream);

/* Even n beyond 64 bits (section "Arbitrary Precision Checker": small
 * primes p in ascending order, q = n - p tested with Miller-Rabin), for
 * 2^64 <= n < 2^(32 nlimbs), nlimbs <= 32 (n below 2^1024).  n holds k
 * numbers of nlimbs little-endian 32-bit limbs each (host memory); p (host,
 * k entries) receives for each the smallest odd prime p from the resident
 * table whose q passes the strong probable-prime test to each of the 25
 * prime bases 2..97.  Every smaller p's q failed one of those bases and is
 * certainly composite; the returned q is a probable prime (the first 12
 * bases alone are deterministic below 3.3e24).  A base-2 search over the
 * p not ruled out by a small base, then a confirmation over the other 24
 * bases, in passes planned on the device; the call synchronises the stream
 * after every six passes and at its end.  Status: GB_EINVAL for an
 * odd n, an n below 2^64, nlimbs outside 3..32 or more than 2^24 n;
 * GB_EUNRESOLVED (entry 0) if no prime of the table works; GB_EDEVICE on a
 * HIP error or when the passes do not settle. */
gb_status gb_verify_big(gb_ctx *ctx, const uint32_t *n, uint32_t nlimbs, size_t k,
                        uint64_t *p, void *stream);

/* Many single n in one launch (one wavefront per n; the checker of section
 * "GPU Single-Number Checker" applied to a batch, minimal p as in
 * gb_verify_one).  n and p are arrays of
 * k uint64 entries, both in device memory when on_device is 1, else both in
 * host memory.  Entries with no partition within the budget get 0 and the
 * call returns GB_EUNRESOLVED; odd or out-of-range n give GB_EINVAL. */
gb_status gb_verify_many(gb_ctx *ctx, const uint64_t *n, uint64_t *p, size_t k,
                         int on_device, void *stream);

/* gb_verify_many without any allocation in the call, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  n and p are device arrays of k
 * entries (inputs and outputs stay the caller's); the exhaustive phase's
 * work list and counters live in a fixed device array inside the library,
 * 2 MiB per device, so k is at most 65536 (GB_EINVAL above).  Every call on
 * one device shares that array: calls that overlap on a device race.  The
 * call synchronises `stream`.  Same results as gb_verify_many; GB_EINVAL when
 * an n is odd, below 4 or above 2^63 (p unspecified), GB_EUNRESOLVED when an
 * n has no partition within the budget (its p is 0). */
gb_status gb_verify_many_noalloc(gb_ctx *ctx, const uint64_t *n, uint64_t *p, size_t k, void *stream);

/* The sieve alone (the segment bitset of subsection "Correct segmentation",
 * there built on the host; a GPU-built sieve is a direction of section
 * "Future work"): bit i of the output (LSB-first uint32 words) is 1 iff the
 * odd number w0 + 2i is prime, for 0 <= i < nbits, built by the LDS tile
 * sieve of the bulk form (wheel pattern, then strided marking of the odd
 * multiples of each sieving prime from max(p^2, w0)).  w0 is odd, w0 >= 1,
 * w0 + 2*nbits <= max_hi; nbits is a multiple of 64; bits is device memory of
 * nbits/32 words. */
gb_status gb_sieve_window(gb_ctx *ctx, uint64_t w0, uint64_t nbits,
                          uint32_t *bits, void *stream);

/* The sieve of the minimal-p range calls alone (the same segment bitset,
 * in the layout those calls search): the numbers 6k + 1 and 6k + 5 in two
 * planes.  Bit k of plane i (LSB-first uint32 words, plane i at word offset
 * i*nk/32 of planes) is 1 iff 6(k0 + k) + c_i is prime, c = (1, 5), for
 * 0 <= k < nk.  k0 and nk are multiples of 64, nk > 0, 6(k0 + nk) <= max_hi;
 * planes is device memory of nk/16 words.  Status: GB_EINVAL for bad
 * arguments, GB_ERANGE above max_hi, GB_EDEVICE on a HIP error. */
gb_status gb_sieve_planes(gb_ctx *ctx, uint64_t k0, uint64_t nk, uint32_t *planes, void *stream);

/* Goldbach partition counts (paper section "Future work": large-scale
 * counts c(n) of the partitions n = p + q into primes p <= q).  c(4) = 1;
 * for even n >= 6, c(n) is the number of odd primes p <= n/2 with n - p
 * prime.  For every even n in [max(lo,4), hi]:
 *   counts (nullable) is device memory of one uint64 per n, n_first + 2i at
 *     index i (n_first the first even n >= max(lo,4)), overwritten;
 *   res receives the summaries below.
 * The call sieves the odd numbers up to hi into a device bitset (the tile
 * sieve of gb_sieve_window), then each workgroup counts for 512 consecutive n
 * the pairs (p, n - p) word by word: the flags of 32 consecutive p ANDed with
 * the bit-reversed flags of the matching q, and a popcount.  Limits:
 * hi <= max_hi, at most 2^25 even n per call, and the bitset (hi/16 bytes)
 * plus the internal counts (when counts is NULL) within prm.mem_budget.
 * Status: GB_EINVAL for a NULL res or too many n, GB_ERANGE above max_hi,
 * GB_ENOMEM over the budget, GB_EDEVICE on a HIP error.  lo > hi, or no even
 * n >= 4 in the range, gives an empty result with GB_OK. */
typedef struct gb_pc_result {
    uint64_t count;        /* even n examined */
    uint64_t sum;          /* sum of c(n), modulo 2^64 */
    uint64_t min_c;        /* smallest c(n) (0 when count is 0) */
    uint64_t argmin_n;     /* the smallest n attaining it */
    uint64_t max_c;        /* largest c(n) */
    uint64_t argmax_n;     /* the smallest n attaining it */
    double device_ms;      /* sieve, counting and summary, device time */
    double kernel_ms;      /* the counting kernel alone */
} gb_pc_result;

gb_status gb_partition_counts(gb_ctx *ctx, uint64_t lo, uint64_t hi,
                              uint64_t *counts, gb_pc_result *res, void *stream);

/* Measured throughput ceilings of the units the kernels use, for roofline
 * fractions beside the nominal peaks.  Not part of the paper's method: a
 * measurement aid for this device (every figure is for the whole device,
 * the best of three timed launches after a warm-up launch):
 *   valu_vop2_ops   int32 lane-ops/s of a two-operand instruction (v_xor_b32)
 *   valu_vop3_ops   int32 lane-ops/s of a three-operand one (v_alignbit_b32)
 *   lds_read_bytes  LDS bytes/s of 16-byte reads without bank conflicts
 *   lds_atomic_ops  lane-ops/s of ds_and_b32 without bank conflicts
 *   hbm_copy_bytes  HBM bytes/s (read plus write) of a 256 MiB device copy
 * Allocates 512 MiB of device memory for the call (GB_ENOMEM if that exceeds
 * prm.mem_budget); GB_EDEVICE on a HIP error. */
typedef struct gb_peaks {
    double valu_vop2_ops;
    double valu_vop3_ops;
    double lds_read_bytes;
    double lds_atomic_ops;
    double hbm_copy_bytes;
} gb_peaks;

gb_status gb_measure_peaks(gb_ctx *ctx, gb_peaks *out, void *stream);

/* The (n, p) pairs the last range or window call sent to the exhaustive
 * phase (section "Phase 2: exhaustive CPU fallback", run on the GPU here;
 * p = 0 for a failure), at most cap of them, into host arrays; *count
 * receives the total number.  These are the n whose uint16 entry can be 0
 * (p_min >= 2^16 or no partition) together with their true p, and the n the
 * fast path left, so the list is the exhaustive phase's work list rather
 * than only the overflow of the uint16 output. */
gb_status gb_exhaustive_list(gb_ctx *ctx, uint64_t *n, uint64_t *p, size_t cap,
                             size_t *count);

/* Autotuner: time the batched form over a sample of windows for every
 * combination of the candidate tile sizes, workgroup sizes, P_max and wheel
 * values, then the plain form for segment sizes S = 2^20 .. 2^26, check that
 * every combination gives bit-identical results, keep the fastest in the
 * context and, when cache_path is not NULL, write it there as one JSON
 * object.  best (nullable) receives the chosen parameters.  The paper fixes
 * SEG_SIZE and PSMALL and reports that data-centre GPUs need them tuned to
 * the hardware (sections "Multi-GPU Scaling and Efficiency", "Limitations"
 * and "Future work"); this call is that tuning.  P_max plays PSMALL's part. */
gb_status gb_autotune(gb_ctx *ctx, const gb_window *sample, size_t k,
                      const char *cache_path, gb_params *best);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of single-n and range requests.  The paper
 * has no serving mode; these calls put the range computation of
 * gb_verify_windows and the single-n checker of gb_verify_many behind a
 * request queue.
 *
 * A server owns a context and `streams` device streams, each with its own
 * scratch.  A scheduler thread takes submitted requests in arrival order,
 * admits them while the bytes of device memory they need fit in
 * prm->mem_budget, packs up to `max_batch` of them into one launch on an
 * idle stream (single n: one wavefront each, as gb_verify_many; ranges: one
 * persistent tile launch over all their windows, as gb_verify_windows), and
 * keeps admitting new requests onto other streams while earlier launches
 * run, so their work overlaps on the device.  Every result is the same as the
 * request run alone.  The prime table and wheel stay resident for the
 * server's lifetime.  Submit and poll may be called from any thread.
 * ---------------------------------------------------------------------- */
typedef struct gb_server gb_server;

#define GB_REQ_ONE 0u    /* one even n */
#define GB_REQ_RANGE 1u  /* the even n n, n+2, ..., n + 2(len-1) */

#define GB_REQ_PMIN_DEVICE 1u  /* flags: pmin is device memory of the
                                  server's device, written by the kernels */

typedef struct gb_request {
    uint32_t  kind;      /* GB_REQ_ONE or GB_REQ_RANGE */
    uint32_t  flags;     /* 0, or GB_REQ_PMIN_DEVICE for a range with pmin */
    uint64_t  n;         /* the n (GB_REQ_ONE) or the first n (GB_REQ_RANGE) */
    uint64_t  len;       /* GB_REQ_RANGE: number of even n (>= 1) */
    uint16_t *pmin;      /* GB_REQ_RANGE: buffer of len entries for the per-n
                            p_min (0 for p_min >= 2^16), written before the
                            completion is reported; host memory, or device
                            memory with GB_REQ_PMIN_DEVICE; or NULL */
    uint64_t  tag;       /* caller's value, returned with the completion */
} gb_request;

typedef struct gb_completion {
    uint64_t   id;              /* the id gb_server_submit returned */
    uint64_t   tag;
    int32_t    status;          /* gb_status of this request */
    uint32_t   kind;
    uint64_t   p;               /* GB_REQ_ONE: p_min(n) */
    gb_summary summary;         /* GB_REQ_RANGE: the range's summary */
    uint64_t   submit_ns;       /* steady-clock times of submit, launch and */
    uint64_t   launch_ns;       /* observed completion */
    uint64_t   done_ns;
    uint32_t   batch_requests;  /* requests in the launch that served it */
    uint32_t   stream;          /* index of the stream that ran it */
} gb_completion;

typedef struct gb_server_stats {
    uint64_t submitted, completed, rejected, queued, inflight;
    uint64_t bytes_inflight, peak_bytes_inflight;
    uint64_t launches, peak_concurrent_launches;
} gb_server_stats;

/* Start a server on prm->device (prm may be NULL) with `streams` device
 * streams (1..8, 0 -> 2) and at most `max_batch` requests per launch
 * (0 -> 4096).  Unlike gb_create, a tile_log2 or wg_threads left 0 takes
 * 16 and 1024: small tiles spread one range over many workgroups, which
 * cuts request latency (tiles of 2^19 n suit whole-range throughput). */
gb_status gb_server_start(gb_server **srv, const gb_params *prm, uint32_t streams,
                          uint32_t max_batch);
/* Queue one request; *id receives its id.  GB_EINVAL for a malformed
 * request, GB_ERANGE above max_hi, GB_ENOMEM if it alone needs more than
 * mem_budget.  Never blocks on the device. */
gb_status gb_server_submit(gb_server *srv, const gb_request *req, uint64_t *id);
/* Take up to cap finished requests into out[]; *count receives how many.
 * Waits up to wait_ms milliseconds for the first one (0: do not wait). */
gb_status gb_server_poll(gb_server *srv, gb_completion *out, size_t cap, size_t *count,
                         int32_t wait_ms);
gb_status gb_server_stats_get(gb_server *srv, gb_server_stats *stats);
/* Replay a request trace (a load generator inside the library, so that the
 * offered load does not depend on the caller's language): request i is
 * submitted arrival_ns[i] nanoseconds after the call starts (arrival_ns
 * ascending), and the call returns when all k have completed, with out[i]
 * the completion of req[i].  Its submit_ns is the scheduled arrival time, so
 * done_ns - submit_ns includes any delay in submitting (an open-loop
 * measurement).  The paper has no serving mode; this drives the continuous
 * batching above with a Poisson or any other arrival process.  No other
 * thread may poll the server during the call.  GB_EINVAL for a malformed
 * request (nothing submitted after it), GB_EDEVICE when the requests have
 * not all completed within timeout_ms. */
gb_status gb_server_replay(gb_server *srv, const gb_request *req, const uint64_t *arrival_ns,
                           size_t k, gb_completion *out, uint32_t timeout_ms);
/* Finish every queued and running request, then free the server. */
gb_status gb_server_stop(gb_server *srv);
const char *gb_server_last_error(const gb_server *srv);

const char *gb_status_str(gb_status st);
const char *gb_last_error(const gb_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GOLDBACH_H */
