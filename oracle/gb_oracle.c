/*
 * gb_oracle.c -- plain, slow, CPU reference for minimal Goldbach partitions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source with the HIP path.
 *
 * What it computes (GoldbachGPU paper, section "Methods", subsection "CPU
 * Baseline"): for every even n in a range, scan primes p upward from 2 and
 * stop at the first p for which q = n - p is prime.  The first hit is the
 * minimal Goldbach prime p_min(n), which is unique by definition and never
 * exceeds n/2.  Primality of q comes from a segmented Sieve of Eratosthenes
 * over the odd numbers of the segment (a byte per odd number, on purpose not
 * the bit layout of the GPU path); a q below the sieved window (only possible
 * once p exceeds 2^16) is tested directly.  Outside any window, primality is
 * the deterministic Miller-Rabin test with the twelve prime bases 2..37 that
 * the paper's single-number checker uses (section "GPU Single-Number
 * Checker"), with 128-bit products and plain square-and-multiply.
 *
 * Summaries (the paper prints none; their definitions are fixed here):
 *   count          number of even n examined
 *   max_p/argmax_n largest p_min and the smallest n attaining it
 *   checksum       sum over n of w(n) * p_min(n), modulo 2^64, with the
 *                  weight w(n) = 2^33 * b(n) + (2c+1) * 2^i, where
 *                  b(n) = 3 floor(n/384) + (n mod 6)/2 numbers the sets of
 *                  64 even n of one residue class mod 6 and one stretch of
 *                  384, j = floor(n/6) mod 64 is the place of n in its set,
 *                  c = floor(j/32), i = j mod 32 (orc_checksum_weight).
 *                  w(n) has exactly i <= 31 factors of 2 and the
 *                  difference of two p below 2^16 at most 15, so any single
 *                  wrong p_min changes it; so does any exchange of p
 *                  between two n whose b differ by less than 2^16 (n closer
 *                  than 8 million): their weights differ by at most 33 + 15
 *                  factors of 2.
 *   hist[i]        number of n whose p_min is the i-th prime (2 -> 0,
 *                  3 -> 1, ...) for p_min < 2^16; bin 6542 counts larger p
 *   n_exhaustive   number of n that no prime p <= P_max resolves (the n a
 *                  fast path bounded by P_max leaves to an exhaustive phase)
 *   n_failed       number of n with no partition at all (a counterexample)
 *   first_failed_n smallest such n, or 0
 *
 * The file also counts Goldbach partitions c(n) (orc_partition_counts).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_P_EXT 65536u        /* window halo below the segment, and bin bound */
#define ORC_HIST_BINS 6543u     /* pi(2^16) = 6542 prime bins + 1 overflow bin */
#define ORC_TRIAL_MAX 1000000000000ull  /* trial division up to 10^12 */

typedef struct {
    uint64_t count, max_p, argmax_n, checksum, n_exhaustive, n_failed,
             first_failed_n;
} orc_summary;

/* ------------------------------------------------------------------ */
/* integer helpers                                                     */
/* ------------------------------------------------------------------ */

uint64_t orc_isqrt(uint64_t x)
{
    /* floor(sqrt(x)) by bisection on the exact square, no floating point */
    uint64_t lo = 0, hi = 4294967295ull;
    if (hi > x) hi = x;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        if ((unsigned __int128)mid * mid <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Plain trial division by every odd d with d*d <= q. */
int orc_trial_is_prime(uint64_t q)
{
    if (q < 2) return 0;
    if (q % 2 == 0) return q == 2;
    for (uint64_t d = 3; (unsigned __int128)d * d <= q; d += 2)
        if (q % d == 0) return 0;
    return 1;
}

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)a * b) % m);
}

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

/* Strong probable-prime test of odd q > 2 to one base a (Miller 1976,
 * Rabin 1980): write q-1 = d*2^s with d odd; q passes when a^d = 1 or
 * a^(d*2^r) = q-1 for some 0 <= r < s.  Returns 1 on pass. */
int orc_mr_base(uint64_t q, uint64_t a)
{
    if (q < 3 || q % 2 == 0) return q == 2;
    a %= q;
    if (a == 0) return 1;            /* the base carries no information */
    uint64_t d = q - 1;
    int s = 0;
    while (d % 2 == 0) { d /= 2; s++; }
    uint64_t x = powmod(a, d, q);
    if (x == 1 || x == q - 1) return 1;
    for (int r = 1; r < s; r++) {
        x = mulmod(x, x, q);
        if (x == q - 1) return 1;
    }
    return 0;
}

static const uint64_t ORC_MR_BASES[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};

/* Deterministic for every q < 2^64 with the first twelve primes as bases. */
int orc_mr(uint64_t q)
{
    if (q < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (q == ORC_MR_BASES[i]) return 1;
        if (q % ORC_MR_BASES[i] == 0) return 0;
    }
    for (int i = 0; i < 12; i++)
        if (!orc_mr_base(q, ORC_MR_BASES[i])) return 0;
    return 1;
}

/* Primality for a q that lies outside the sieved window. */
int orc_is_prime(uint64_t q)
{
    if (q <= ORC_TRIAL_MAX) return orc_trial_is_prime(q);
    return orc_mr(q);
}

/* ------------------------------------------------------------------ */
/* sieves                                                              */
/* ------------------------------------------------------------------ */

/* All odd primes <= limit, from a plain byte-per-integer sieve. */
static uint32_t *odd_primes_upto(uint64_t limit, uint64_t *count)
{
    uint8_t *comp = calloc(limit + 1, 1);
    uint64_t n = 0;
    if (!comp) { *count = 0; return NULL; }
    for (uint64_t i = 3; i * i <= limit; i += 2)
        if (!comp[i])
            for (uint64_t j = i * i; j <= limit; j += 2 * i) comp[j] = 1;
    for (uint64_t i = 3; i <= limit; i += 2) n += !comp[i];
    uint32_t *out = malloc((n ? n : 1) * sizeof(uint32_t));
    uint64_t k = 0;
    if (out)
        for (uint64_t i = 3; i <= limit; i += 2)
            if (!comp[i]) out[k++] = (uint32_t)i;
    free(comp);
    *count = out ? n : 0;
    return out;
}

/* Byte per odd number in [wlo, whi] (both odd): 1 = prime.  The odd multiples
 * of each base prime p are struck from max(p*p, first odd multiple >= wlo). */
static void sieve_window(uint8_t *win, uint64_t wlo, uint64_t whi,
                         const uint32_t *base, uint64_t nbase)
{
    uint64_t nw = (whi - wlo) / 2 + 1;
    memset(win, 1, nw);
    if (wlo == 1) win[0] = 0;
    for (uint64_t i = 0; i < nbase; i++) {
        uint64_t p = base[i];
        if (p * p > whi) break;
        uint64_t m = p * p;
        if (m < wlo) {
            m = ((wlo + p - 1) / p) * p;
            if (m % 2 == 0) m += p;
        }
        for (; m <= whi; m += 2 * p) win[(m - wlo) / 2] = 0;
    }
}

/* pi(x): number of primes <= x, counting the odd numbers of a segmented byte
 * sieve plus the prime 2. */
uint64_t orc_prime_count(uint64_t x)
{
    if (x < 2) return 0;
    if (x < 3) return 1;
    uint64_t nbase;
    uint32_t *base = odd_primes_upto(orc_isqrt(x) + 1, &nbase);
    const uint64_t SEG = 1u << 22;             /* odd numbers per segment */
    uint8_t *win = malloc(SEG);
    uint64_t total = 1;                        /* the prime 2 */
    uint64_t top = (x % 2) ? x : x - 1;
    for (uint64_t lo = 1; lo <= top; lo += 2 * SEG) {
        uint64_t hi = lo + 2 * (SEG - 1);
        if (hi > top) hi = top;
        sieve_window(win, lo, hi, base, nbase);
        for (uint64_t i = 0; i <= (hi - lo) / 2; i++) total += win[i];
    }
    free(win);
    free(base);
    return total;
}

/* ------------------------------------------------------------------ */
/* minimal Goldbach prime                                              */
/* ------------------------------------------------------------------ */

/* Index of prime p among all primes (2 -> 0, 3 -> 1, ...) when p < 2^16,
 * else the overflow bin.  `small` lists the odd primes below 2^16. */
static uint32_t hist_bin(uint64_t p, const uint32_t *small, uint64_t nsmall)
{
    if (p == 2) return 0;
    if (p >= 65536) return ORC_HIST_BINS - 1;
    uint64_t lo = 0, hi = nsmall;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (small[mid] < p) lo = mid + 1; else hi = mid;
    }
    return (uint32_t)(lo + 1);
}

/* The checksum weight of n, written out from its definition above. */
uint64_t orc_checksum_weight(uint64_t n)
{
    uint64_t b = 3 * (n / 384) + (n % 6) / 2;
    uint64_t j = (n / 6) % 64;
    uint64_t c = j / 32, i = j % 32;
    return (b << 33) + ((2 * c + 1) << i);
}

static void record(orc_summary *s, uint64_t *hist, const uint32_t *small,
                   uint64_t nsmall, uint64_t n, uint64_t p, uint32_t pmax)
{
    s->count++;
    if (p == 0) {
        s->n_failed++;
        s->n_exhaustive++;
        if (s->first_failed_n == 0 || n < s->first_failed_n) s->first_failed_n = n;
        return;
    }
    if (hist) hist[hist_bin(p, small, nsmall)]++;
    s->checksum += orc_checksum_weight(n) * p;
    if (p > s->max_p) { s->max_p = p; s->argmax_n = n; }
    if (p > pmax) s->n_exhaustive++;
}

/* Combine two summaries of disjoint n sets. */
static void merge(orc_summary *a, const orc_summary *b)
{
    a->count += b->count;
    a->checksum += b->checksum;
    a->n_exhaustive += b->n_exhaustive;
    a->n_failed += b->n_failed;
    if (b->first_failed_n && (a->first_failed_n == 0 || b->first_failed_n < a->first_failed_n))
        a->first_failed_n = b->first_failed_n;
    if (b->max_p > a->max_p || (b->max_p == a->max_p && b->max_p && b->argmax_n < a->argmax_n)) {
        a->max_p = b->max_p;
        a->argmax_n = b->argmax_n;
    }
}

static void store_p(void *out, int bits, uint64_t idx, uint64_t p)
{
    if (!out) return;
    if (bits == 32) ((uint32_t *)out)[idx] = (uint32_t)p;
    else ((uint16_t *)out)[idx] = (uint16_t)(p < 65536 ? p : 0);
}

/* p_min for every even n in [lo, hi] (lo, hi even, 4 <= lo <= hi), one
 * segment of n at a time.  `out[k]` receives p_min(lo + 2k). */
static void range_core(uint64_t lo, uint64_t hi, uint32_t pmax,
                       const uint32_t *base, uint64_t nbase,
                       const uint32_t *small, uint64_t nsmall,
                       void *out, int bits, uint64_t *hist, orc_summary *s)
{
    const uint64_t SEGN = 1u << 21;            /* even n per segment */
    uint8_t *win = malloc(SEGN + ORC_P_EXT);
    uint64_t top_base = nbase ? base[nbase - 1] : 2;
    for (uint64_t a = lo; a <= hi; a += 2 * SEGN) {
        uint64_t b = a + 2 * (SEGN - 1);
        if (b > hi || b < a) b = hi;
        /* odd q in [wlo, b-3]: every q = n - p with p <= 2^16 */
        uint64_t wlo = (a > ORC_P_EXT + 3) ? a - ORC_P_EXT + 1 : 3;
        uint64_t whi = b - 3;
        if (whi < wlo) whi = wlo;              /* only n = 4, 6 */
        sieve_window(win, wlo, whi, base, nbase);
        for (uint64_t n = a; n <= b; n += 2) {
            uint64_t found = 0;
            if (n == 4) {
                found = 2;
            } else {
                uint64_t p = 0;
                for (uint64_t i = 0; i < nbase; i++) {
                    p = base[i];
                    if (p > n / 2) break;
                    uint64_t q = n - p;
                    int isp = (q >= wlo) ? win[(q - wlo) / 2] : orc_is_prime(q);
                    if (isp) { found = p; break; }
                }
                /* past the base-prime list: odd p tested directly */
                if (!found && p <= n / 2)
                    for (uint64_t c = top_base + 2; c <= n / 2; c += 2)
                        if (orc_is_prime(c) && orc_is_prime(n - c)) { found = c; break; }
            }
            store_p(out, bits, (n - lo) / 2, found);
            record(s, hist, small, nsmall, n, found, pmax);
        }
    }
    free(win);
}

static void normalise(uint64_t *lo, uint64_t *hi)
{
    if (*lo < 4) *lo = 4;
    if (*lo % 2) (*lo)++;
    if (*hi % 2) (*hi)--;
}

/* Single-threaded: p_min for every even n with max(lo,4) <= n <= hi.
 * out (nullable) has one entry per even n, width `bits` (16 or 32; a 16-bit
 * entry holds 0 for p_min >= 2^16 or no partition).  hist (nullable) has
 * ORC_HIST_BINS entries and is accumulated into.  Returns 0, or -1 on
 * allocation failure. */
int orc_verify_range(uint64_t lo, uint64_t hi, uint32_t pmax, void *out,
                     int bits, uint64_t *hist, orc_summary *s)
{
    memset(s, 0, sizeof *s);
    normalise(&lo, &hi);
    if (lo > hi) return 0;
    uint64_t nbase, nsmall;
    uint64_t lim = orc_isqrt(hi) + 1;
    if (lim < ORC_P_EXT) lim = ORC_P_EXT;
    uint32_t *base = odd_primes_upto(lim, &nbase);
    uint32_t *small = odd_primes_upto(ORC_P_EXT, &nsmall);
    if (!base || !small) { free(base); free(small); return -1; }
    range_core(lo, hi, pmax, base, nbase, small, nsmall, out, bits, hist, s);
    free(base);
    free(small);
    return 0;
}

/* ---- the same computation spread over threads, for timing only ---- */

typedef struct {
    uint64_t lo, hi, chunk_n, nchunks;
    uint32_t pmax;
    const uint32_t *base, *small;
    uint64_t nbase, nsmall;
    void *out;
    int bits;
    uint64_t next;               /* shared chunk counter */
    pthread_mutex_t mu;
    uint64_t *hist;              /* shared result, merged under mu */
    orc_summary sum;
} mt_job;

static void *mt_worker(void *arg)
{
    mt_job *j = arg;
    uint64_t *h = j->hist ? calloc(ORC_HIST_BINS, sizeof(uint64_t)) : NULL;
    orc_summary mine;
    memset(&mine, 0, sizeof mine);
    for (;;) {
        uint64_t c = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (c >= j->nchunks) break;
        uint64_t a = j->lo + 2 * c * j->chunk_n;
        uint64_t b = a + 2 * (j->chunk_n - 1);
        if (b > j->hi || b < a) b = j->hi;
        orc_summary part;
        memset(&part, 0, sizeof part);
        void *o = NULL;
        if (j->out)
            o = (char *)j->out + (size_t)((a - j->lo) / 2) * (j->bits / 8);
        range_core(a, b, j->pmax, j->base, j->nbase, j->small, j->nsmall,
                   o, j->bits, h, &part);
        merge(&mine, &part);
    }
    pthread_mutex_lock(&j->mu);
    merge(&j->sum, &mine);
    if (h)
        for (uint32_t i = 0; i < ORC_HIST_BINS; i++) j->hist[i] += h[i];
    pthread_mutex_unlock(&j->mu);
    free(h);
    return NULL;
}

int orc_verify_range_mt(uint64_t lo, uint64_t hi, uint32_t pmax, void *out,
                        int bits, uint64_t *hist, orc_summary *s, int nthreads)
{
    memset(s, 0, sizeof *s);
    normalise(&lo, &hi);
    if (lo > hi) return 0;
    if (nthreads < 1) nthreads = 1;
    mt_job j;
    memset(&j, 0, sizeof j);
    uint64_t lim = orc_isqrt(hi) + 1;
    if (lim < ORC_P_EXT) lim = ORC_P_EXT;
    j.base = odd_primes_upto(lim, &j.nbase);
    j.small = odd_primes_upto(ORC_P_EXT, &j.nsmall);
    if (!j.base || !j.small) { free((void *)j.base); free((void *)j.small); return -1; }
    uint64_t total = (hi - lo) / 2 + 1;
    j.chunk_n = 1u << 21;
    if (total / ((uint64_t)nthreads * 4) < j.chunk_n)
        j.chunk_n = total / ((uint64_t)nthreads * 4) + 1;
    j.nchunks = (total + j.chunk_n - 1) / j.chunk_n;
    j.lo = lo; j.hi = hi; j.pmax = pmax; j.out = out; j.bits = bits; j.hist = hist;
    pthread_mutex_init(&j.mu, NULL);
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, mt_worker, &j);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&j.mu);
    *s = j.sum;
    free((void *)j.base);
    free((void *)j.small);
    return 0;
}

/* ---- many windows of consecutive even n (the batched and serving
 * workloads): the base primes once, then each window is the plain scan of
 * range_core, windows spread over threads.  Window i is the even n
 * start[i], start[i] + 2, ..., start[i] + 2 (len[i] - 1), start[i] even and
 * >= 4; its per-n p_min (uint16, 0 for p >= 2^16 or none) goes to out
 * (nullable) at offset len[0] + ... + len[i-1], its summary to sums[i].
 * Returns 0, -1 on allocation failure, -2 for a malformed window. */

typedef struct {
    const uint64_t *start, *len, *off;
    uint64_t k, next;
    uint32_t pmax;
    const uint32_t *base, *small;
    uint64_t nbase, nsmall;
    uint16_t *out;
    orc_summary *sums;
} win_job;

static void *win_worker(void *arg)
{
    win_job *j = arg;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (i >= j->k) break;
        memset(&j->sums[i], 0, sizeof j->sums[i]);
        range_core(j->start[i], j->start[i] + 2 * (j->len[i] - 1), j->pmax, j->base, j->nbase,
                   j->small, j->nsmall, j->out ? j->out + j->off[i] : NULL, 16, NULL, &j->sums[i]);
    }
    return NULL;
}

int orc_verify_windows(const uint64_t *start, const uint64_t *len, uint64_t k, uint32_t pmax,
                       uint16_t *out, orc_summary *sums, int nthreads)
{
    if (k == 0) return 0;
    uint64_t top = 0;
    uint64_t *off = malloc(k * sizeof(uint64_t));
    if (!off) return -1;
    for (uint64_t i = 0, o = 0; i < k; i++) {
        if (start[i] < 4 || start[i] % 2 || len[i] == 0) { free(off); return -2; }
        uint64_t last = start[i] + 2 * (len[i] - 1);
        if (last > top) top = last;
        off[i] = o;
        o += len[i];
    }
    if (nthreads < 1) nthreads = 1;
    win_job j;
    memset(&j, 0, sizeof j);
    uint64_t lim = orc_isqrt(top) + 1;
    if (lim < ORC_P_EXT) lim = ORC_P_EXT;
    j.base = odd_primes_upto(lim, &j.nbase);
    j.small = odd_primes_upto(ORC_P_EXT, &j.nsmall);
    if (!j.base || !j.small) { free((void *)j.base); free((void *)j.small); free(off); return -1; }
    j.start = start; j.len = len; j.off = off; j.k = k; j.pmax = pmax; j.out = out; j.sums = sums;
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, win_worker, &j);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    free((void *)j.base);
    free((void *)j.small);
    free(off);
    return 0;
}

/* p_min of one even n (4 <= n < 2^64) by scanning odd primes p upward and
 * testing q = n - p with the deterministic Miller-Rabin test.  Candidate p
 * come from the odd primes below 2^16 and, past them, from odd numbers that
 * pass the same test.  Returns 0 when no p <= min(n/2, limit) works
 * (limit 0 = no limit), or when n is odd or below 4. */
uint64_t orc_verify_one(uint64_t n, uint64_t limit)
{
    if (n < 4 || n % 2) return 0;
    if (n == 4) return 2;
    uint64_t bound = n / 2;
    if (limit && limit < bound) bound = limit;
    uint64_t nsmall;
    uint32_t *small = odd_primes_upto(ORC_P_EXT, &nsmall);
    uint64_t found = 0, p = 3;
    for (uint64_t i = 0; small && i < nsmall; i++) {
        p = small[i];
        if (p > bound) break;
        if (orc_mr(n - p)) { found = p; break; }
    }
    if (!found && small && p <= bound)
        for (uint64_t c = small[nsmall - 1] + 2; c <= bound; c += 2)
            if (orc_mr(c) && orc_mr(n - c)) { found = c; break; }
    free(small);
    return found;
}

/* Batch form of orc_verify_one over an array of n (threads over entries). */
typedef struct {
    const uint64_t *n;
    uint64_t *p;
    uint64_t count, limit, next;
} one_job;

static void *one_worker(void *arg)
{
    one_job *j = arg;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (i >= j->count) break;
        j->p[i] = orc_verify_one(j->n[i], j->limit);
    }
    return NULL;
}

void orc_verify_many(const uint64_t *n, uint64_t *p, uint64_t count,
                     uint64_t limit, int nthreads)
{
    one_job j = {n, p, count, limit, 0};
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, one_worker, &j);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
}

uint32_t orc_hist_bins(void) { return ORC_HIST_BINS; }

/* Primality byte (1 = prime) of each odd number w0, w0+2, ..., w0+2(count-1)
 * from the same plain byte sieve, for comparing with a sieved bitset.
 * w0 odd, w0 >= 1.  Returns 0, or -1 on allocation failure. */
int orc_odd_primality(uint64_t w0, uint64_t count, uint8_t *out)
{
    if (count == 0) return 0;
    uint64_t whi = w0 + 2 * (count - 1);
    uint64_t nbase;
    uint32_t *base = odd_primes_upto(orc_isqrt(whi) + 1, &nbase);
    if (!base) return -1;
    sieve_window(out, w0, whi, base, nbase);
    free(base);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Goldbach partition counts                                           */
/* ------------------------------------------------------------------ */

/* c(n) = number of ways to write the even n >= 4 as p + q with primes
 * p <= q (the counts the paper's "Future work" subsection lists as the next
 * large-scale computation; the "Discussion" links their growth to the small
 * p_min it observes).  4 = 2 + 2 is the one partition with an even prime;
 * for n >= 6 both primes are odd, so c(n) counts the odd primes p <= n/2
 * with n - p prime.  Plain definition: a byte per odd number up to the
 * largest n, and for every n a scan over the odd primes p <= n/2.
 *
 * Summaries of a set of n:
 *   count              number of even n examined
 *   sum                sum of c(n), modulo 2^64
 *   min_c / argmin_n   smallest c(n) and the smallest n attaining it
 *   max_c / argmax_n   largest c(n) and the smallest n attaining it
 */
typedef struct {
    uint64_t count, sum, min_c, argmin_n, max_c, argmax_n;
} orc_pc_summary;

typedef struct {
    const uint64_t *n;      /* the even n, any order */
    uint64_t *c;
    uint64_t count, next;
    const uint8_t *oddp;    /* oddp[k] = 1 iff 2k+1 is prime, k <= (top-1)/2 */
} pc_job;

static uint64_t partition_count(uint64_t n, const uint8_t *oddp)
{
    if (n == 4) return 1;
    uint64_t c = 0;
    for (uint64_t p = 3; p <= n / 2; p += 2)
        if (oddp[(p - 1) / 2] && oddp[(n - p - 1) / 2]) c++;
    return c;
}

static void *pc_worker(void *arg)
{
    pc_job *j = arg;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (i >= j->count) break;
        j->c[i] = partition_count(j->n[i], j->oddp);
    }
    return NULL;
}

/* c(n) for each even n >= 4 of n[0..count) into c[]; summaries into *s
 * (nullable).  Returns 0, -1 on allocation failure, -2 on an odd or small n. */
int orc_partition_counts(const uint64_t *n, uint64_t *c, uint64_t count,
                         orc_pc_summary *s, int nthreads)
{
    uint64_t top = 3;
    for (uint64_t i = 0; i < count; i++) {
        if (n[i] < 4 || (n[i] & 1)) return -2;
        if (n[i] > top) top = n[i];
    }
    if (!(top & 1)) top -= 1;
    uint64_t nbase;
    uint32_t *base = odd_primes_upto(orc_isqrt(top) + 1, &nbase);
    uint8_t *oddp = malloc((top - 1) / 2 + 1);
    if (!base || !oddp) { free(base); free(oddp); return -1; }
    sieve_window(oddp, 1, top, base, nbase);
    free(base);
    pc_job j = {n, c, count, 0, oddp};
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, pc_worker, &j);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    free(oddp);
    if (s) {
        memset(s, 0, sizeof *s);
        s->min_c = ~0ull;
        for (uint64_t i = 0; i < count; i++) {
            s->count++;
            s->sum += c[i];
            if (s->argmin_n == 0 || c[i] < s->min_c || (c[i] == s->min_c && n[i] < s->argmin_n)) {
                s->min_c = c[i];
                s->argmin_n = n[i];
            }
            if (s->argmax_n == 0 || c[i] > s->max_c || (c[i] == s->max_c && n[i] < s->argmax_n)) {
                s->max_c = c[i];
                s->argmax_n = n[i];
            }
        }
        if (count == 0) s->min_c = 0;
    }
    return 0;
}
