/*
 * Seeded synthetic workloads for the SneakySnake filter.
 *
 * This module only produces inputs: DNA read/reference pairs over {A,C,G,T}
 * as ASCII bytes, their lengths and thresholds.  It contains none of the
 * filter's arithmetic and is shared, as an input source only, by the GPU
 * library's tests/benchmarks and by the CPU oracle's tests.
 *
 * Randomness: every pair (and every serving request) owns an independent
 * SplitMix64 stream (Steele, Lea & Flood, OOPSLA 2014): the stream state is
 * initialised from the finaliser of (seed, stream id) and advanced by the
 * golden-ratio increment, so any pair can be regenerated alone and the
 * output does not depend on the number of threads.
 *
 * Edit model for a "k-edit" reference: k events are drawn, each with a type,
 * a position on the read (substitutions and deletions: one of the m bases;
 * insertions: one of the m+1 gaps) and, for indels, a length.  Events are
 * applied in one left-to-right pass in position order; events that fall in a
 * span already deleted are dropped.  A substitution writes one of the three
 * other bases; insertions write uniform bases.  The edited string is then cut
 * or padded (uniform bases) at its 3' end to exactly m.  The read is the
 * query Q, the edited string is the reference R.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

static const uint8_t BASES[4] = {'A', 'C', 'G', 'T'};

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s; } rng_t;

static inline rng_t rng_stream(uint64_t seed, uint64_t stream)
{
    rng_t r;
    r.s = mix64(mix64(seed ^ 0x5EED5EED5EED5EEDULL) + (stream + 1) * 0x9E3779B97F4A7C15ULL);
    return r;
}

static inline uint64_t rng_next(rng_t* r)
{
    r->s += 0x9E3779B97F4A7C15ULL;
    return mix64(r->s);
}

/* uniform integer in [0, n) by the multiply-shift reduction */
static inline uint64_t rng_below(rng_t* r, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)rng_next(r) * n) >> 64);
}

static inline double rng_unit(rng_t* r) { return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* ASCII of the four bases held by one byte of a random word, lowest bit pair first. */
static uint32_t QUAD[256];
static pthread_once_t quad_once = PTHREAD_ONCE_INIT;

static void quad_init(void)
{
    for (int v = 0; v < 256; v++) {
        uint8_t c[4];
        for (int t = 0; t < 4; t++) c[t] = BASES[(v >> (2 * t)) & 3];
        memcpy(&QUAD[v], c, 4);
    }
}

/* n uniform bases: each random word gives 32 of them, two bits each, lowest pair first. */
static void rand_bases(rng_t* r, uint8_t* dst, int64_t n)
{
    pthread_once(&quad_once, quad_init);
    int64_t i = 0;
    while (n - i >= 32) {
        uint64_t x = rng_next(r);
        for (int j = 0; j < 8; j++, x >>= 8) memcpy(dst + i + 4 * j, &QUAD[x & 255], 4);
        i += 32;
    }
    if (i < n) {
        uint64_t x = rng_next(r);
        for (; i < n; i++) { dst[i] = BASES[x & 3]; x >>= 2; }
    }
}

/* Poisson(lambda) by Knuth's product-of-uniforms method (small lambda). */
static int rng_poisson(rng_t* r, double lambda)
{
    double L = exp(-lambda), p = 1.0;
    int k = 0;
    do { k++; p *= rng_unit(r); } while (p > L);
    return k - 1;
}

/* Geometric(1/2) on {1,2,...}: one plus the number of failures. */
static int rng_geom_half(rng_t* r)
{
    int len = 1;
    for (;;) {
        uint64_t x = rng_next(r);
        for (int b = 0; b < 64; b++) { if (x & 1) return len; len++; x >>= 1; }
    }
}

typedef struct { int32_t pos; int32_t type; int32_t len; int32_t ord; } edit_ev;
enum { EV_SUB = 0, EV_INS = 1, EV_DEL = 2 };

static int ev_cmp(const void* a, const void* b)
{
    const edit_ev* x = (const edit_ev*)a; const edit_ev* y = (const edit_ev*)b;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return x->ord < y->ord ? -1 : (x->ord > y->ord);
}

/* Events in (position, draw order) order.  Every caller numbers its events by
 * draw order (ord = index), so this is a stable sort by position: insertion
 * sort for a few events, a counting sort over the positions 0..maxpos else. */
static void sort_events(edit_ev* ev, int k, int maxpos)
{
    if (k <= 1) return;
    if (k <= 24) {
        for (int a = 1; a < k; a++) {
            edit_ev v = ev[a];
            int b = a - 1;
            while (b >= 0 && ev_cmp(&ev[b], &v) > 0) { ev[b + 1] = ev[b]; b--; }
            ev[b + 1] = v;
        }
        return;
    }
    int* cnt = (int*)calloc((size_t)maxpos + 2, sizeof(int));
    edit_ev* tmp = (edit_ev*)malloc(sizeof(edit_ev) * (size_t)k);
    if (!cnt || !tmp) {
        free(cnt); free(tmp);
        qsort(ev, (size_t)k, sizeof(edit_ev), ev_cmp);
        return;
    }
    for (int a = 0; a < k; a++) cnt[ev[a].pos + 1]++;
    for (int p = 0; p <= maxpos; p++) cnt[p + 1] += cnt[p];
    for (int a = 0; a < k; a++) tmp[cnt[ev[a].pos]++] = ev[a];
    memcpy(ev, tmp, sizeof(edit_ev) * (size_t)k);
    free(cnt); free(tmp);
}

/* Apply sorted events to read[0..m) producing exactly m bases in out. */
static void apply_events(rng_t* r, const uint8_t* read, int m, edit_ev* ev, int k, uint8_t* out)
{
    sort_events(ev, k, m);
    int o = 0, i = 0, e = 0;
    while (o < m && (i < m || e < k)) {
        if (e < k && ev[e].pos <= i) {
            edit_ev* v = &ev[e++];
            if (v->pos < i) continue;                 /* fell inside a deleted span */
            if (v->type == EV_INS) {
                for (int t = 0; t < v->len && o < m; t++) out[o++] = BASES[rng_below(r, 4)];
            } else if (v->type == EV_DEL) {
                i += v->len;
            } else if (i < m) {                        /* substitution: one of the 3 others */
                int code = 0;
                while (BASES[code] != read[i]) code++;
                out[o++] = BASES[(code + 1 + (int)rng_below(r, 3)) & 3];
                i++;
            }
            continue;
        }
        if (i >= m) break;
        /* copy the read up to the next event (or until the output is full) */
        int run = (e < k ? ev[e].pos : m) - i;
        if (run > m - i) run = m - i;
        if (run > m - o) run = m - o;
        memcpy(out + o, read + i, (size_t)run);
        o += run;
        i += run;
    }
    if (o < m) rand_bases(r, out + o, m - o);
}

/* The same pass without the cut or pad: the edited string keeps its natural
 * length (at most m plus the inserted bases), which is returned. */
static int apply_events_free(rng_t* r, const uint8_t* read, int m, edit_ev* ev, int k, uint8_t* out)
{
    sort_events(ev, k, m);
    int o = 0, i = 0, e = 0;
    while (i < m || e < k) {
        if (e < k && ev[e].pos <= i) {
            edit_ev* v = &ev[e++];
            if (v->pos < i) continue;                 /* fell inside a deleted span */
            if (v->type == EV_INS) {
                for (int t = 0; t < v->len; t++) out[o++] = BASES[rng_below(r, 4)];
            } else if (v->type == EV_DEL) {
                i += v->len;
            } else if (i < m) {
                int code = 0;
                while (BASES[code] != read[i]) code++;
                out[o++] = BASES[(code + 1 + (int)rng_below(r, 3)) & 3];
                i++;
            }
            continue;
        }
        if (i >= m) break;
        int run = (e < k ? ev[e].pos : m) - i;
        if (run > m - i) run = m - i;
        memcpy(out + o, read + i, (size_t)run);
        o += run;
        i += run;
    }
    return o;
}

/* ---------------------------------------------------------------------------
 * Pairs of unequal length: read (query) p has m bases; its reference is the
 * read with k ~ U{0..kmax} events (substitution, insertion or deletion with
 * probability 1/3 each, length one, positions uniform) kept at its natural
 * length, or, for unrel_pct percent of the pairs, an unrelated uniform string
 * of a length uniform in [max(0, m - kmax), m + kmax].  Reads are stored back
 * to back (read p at p*m); ssgen_uneq_plan gives the reference lengths (and
 * returns their sum), ssgen_uneq_fill writes the bases, references at ref_off.
 * ------------------------------------------------------------------------- */
static int uneq_pair(uint64_t seed, int64_t p, int32_t m, int32_t kmax, int32_t unrel_pct, uint8_t* Q, uint8_t* R)
{
    rng_t r = rng_stream(seed, (uint64_t)p);
    rand_bases(&r, Q, m);
    if ((int32_t)rng_below(&r, 100) < unrel_pct) {
        int lo = m - kmax < 0 ? 0 : m - kmax;
        int len = lo + (int)rng_below(&r, (uint64_t)(m + kmax - lo + 1));
        rand_bases(&r, R, len);
        return len;
    }
    int k = (int)rng_below(&r, (uint64_t)kmax + 1);
    edit_ev ev[64];
    if (k > 64) k = 64;
    for (int e = 0; e < k; e++) {
        ev[e].ord = e; ev[e].len = 1;
        ev[e].type = (int)rng_below(&r, 3);
        ev[e].pos = (int)rng_below(&r, (uint64_t)(ev[e].type == EV_INS ? m + 1 : (m > 0 ? m : 1)));
    }
    return apply_events_free(&r, Q, m, ev, k, R);
}

int64_t ssgen_uneq_plan(uint64_t seed, int64_t n, int32_t m, int32_t kmax, int32_t unrel_pct, int32_t* ref_len)
{
    if (n < 0 || m < 0 || kmax < 0 || kmax > 64) return -1;
    uint8_t* Q = (uint8_t*)malloc((size_t)m + 1);
    uint8_t* R = (uint8_t*)malloc((size_t)(m + kmax) + 1);
    int64_t total = 0;
    for (int64_t p = 0; p < n; p++) {
        ref_len[p] = uneq_pair(seed, p, m, kmax, unrel_pct, Q, R);
        total += ref_len[p];
    }
    free(Q);
    free(R);
    return total;
}

int ssgen_uneq_fill(uint64_t seed, int64_t n, int32_t m, int32_t kmax, int32_t unrel_pct, const int64_t* ref_off,
                    uint8_t* reads, uint8_t* refs)
{
    if (n < 0 || m < 0 || kmax < 0 || kmax > 64) return -1;
    for (int64_t p = 0; p < n; p++) uneq_pair(seed, p, m, kmax, unrel_pct, reads + p * (int64_t)m, refs + ref_off[p]);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Configurations (all sizes are defaults; n can be overridden).
 *  0: n pairs, m=100, k~U{0..10}, types 1/3 each, length-1 indels.
 *  1: m=100; 40% k~U{0..3}, 40% k~U{4..15}, 20% unrelated (exact counts, shuffled).
 *  2: m=250; k=min(Poisson(8),40); 20% unrelated (exact count, shuffled).
 *  3: mixed: short pairs m~U{100,150,250} with config 1's mix, k bounds scaled
 *     by m/100; plus long pairs (m=10000) at an edit rate ~U[500,1500] basis
 *     points, round(rate*m/1e4) events, half substitutions, half indels
 *     (insertion/deletion equally likely) of Geometric(1/2) length; per-pair
 *     E = ceil(bpE*m/1e4) with bpE ~ U{100,200,500,1000} (integer arithmetic).
 * Categories: 0 low-edit, 1 high-edit, 2 unrelated, 3 long.
 * ------------------------------------------------------------------------- */
enum { CAT_LOW = 0, CAT_HIGH = 1, CAT_UNREL = 2, CAT_LONG = 3 };

int64_t ssgen_default_pairs(int config)
{
    switch (config) {
    case 0: return 10000;
    case 1: return 30000000;
    case 2: return 10000000;
    case 3: return 5020000;
    default: return -1;
    }
}

static int ceil_bp(int bp, int m) { return (int)(((int64_t)bp * m + 9999) / 10000); }

static void shuffle_u8(uint8_t* a, int64_t n, uint64_t seed)
{
    rng_t r = rng_stream(seed, 0xFFFFFFFFFFFFULL);
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)rng_below(&r, (uint64_t)(i + 1));
        uint8_t t = a[i]; a[i] = a[j]; a[j] = t;
    }
}

/* Per-pair plan: category, length and (config 3) threshold.  E_out gets -1
 * for configs whose threshold is swept by the caller.  Returns 0 or -1. */
int ssgen_plan(int config, uint64_t seed, int64_t n, int64_t n_long, uint8_t* cat, int32_t* len, int32_t* E_out)
{
    if (n < 0 || config < 0 || config > 3) return -1;
    int64_t a = 0, b = 0;
    if (config == 0) { for (int64_t i = 0; i < n; i++) cat[i] = CAT_LOW; }
    else if (config == 1 || config == 3) {
        int64_t ns = config == 3 ? n - n_long : n;
        if (ns < 0) return -1;
        a = ns * 2 / 5; b = ns * 4 / 5;
        for (int64_t i = 0; i < n; i++)
            cat[i] = i < a ? CAT_LOW : (i < b ? CAT_HIGH : (i < ns ? CAT_UNREL : CAT_LONG));
        shuffle_u8(cat, n, seed);
    } else {
        a = n * 4 / 5;
        for (int64_t i = 0; i < n; i++) cat[i] = i < a ? CAT_LOW : CAT_UNREL;
        shuffle_u8(cat, n, seed);
    }
    static const int SHORT_M[3] = {100, 150, 250};
    static const int BP_E[4] = {100, 200, 500, 1000};
    for (int64_t i = 0; i < n; i++) {
        rng_t r = rng_stream(seed, (uint64_t)i);
        int m, E = -1;
        if (config == 0 || config == 1) m = 100;
        else if (config == 2) m = 250;
        else {
            m = cat[i] == CAT_LONG ? 10000 : SHORT_M[rng_below(&r, 3)];
            E = ceil_bp(BP_E[rng_below(&r, 4)], m);
        }
        len[i] = m;
        if (E_out) E_out[i] = E;
    }
    return 0;
}

/* Fill one pair; rng r continues the pair's stream after the plan draws. */
static void fill_pair(int config, rng_t* r, uint8_t category, int m, uint8_t* Q, uint8_t* R, edit_ev* ev, int evcap)
{
    rand_bases(r, Q, m);
    if (category == CAT_UNREL) { rand_bases(r, R, m); return; }
    int k = 0;
    int indel_geom = 0;
    if (config == 0) k = (int)rng_below(r, 11);
    else if (config == 1) k = category == CAT_LOW ? (int)rng_below(r, 4) : 4 + (int)rng_below(r, 12);
    else if (config == 2) { k = rng_poisson(r, 8.0); if (k > 40) k = 40; }
    else if (category == CAT_LONG) {
        int bp = 500 + (int)rng_below(r, 1001);
        k = (int)(((int64_t)bp * m + 5000) / 10000);
        indel_geom = 1;
    } else {
        int lo_hi = (3 * m + 50) / 100, hi_lo = (4 * m + 50) / 100, hi_hi = (15 * m + 50) / 100;
        k = category == CAT_LOW ? (int)rng_below(r, (uint64_t)lo_hi + 1)
                                : hi_lo + (int)rng_below(r, (uint64_t)(hi_hi - hi_lo + 1));
    }
    if (k > evcap) k = evcap;
    for (int e = 0; e < k; e++) {
        edit_ev* v = &ev[e];
        v->ord = e; v->len = 1;
        if (indel_geom) {
            if (rng_below(r, 2) == 0) v->type = EV_SUB;
            else { v->type = rng_below(r, 2) == 0 ? EV_INS : EV_DEL; v->len = rng_geom_half(r); }
        } else v->type = (int)rng_below(r, 3);
        v->pos = (int)rng_below(r, (uint64_t)(v->type == EV_INS ? m + 1 : m));
    }
    apply_events(r, Q, m, ev, k, R);
}

typedef struct {
    int config; uint64_t seed; int64_t lo, hi;
    const uint8_t* cat; const int64_t* off; const int32_t* len;
    uint8_t* reads; uint8_t* refs;
} fill_job;

static void* fill_worker(void* arg)
{
    fill_job* J = (fill_job*)arg;
    int evcap = 4096;
    edit_ev* ev = (edit_ev*)malloc(sizeof(edit_ev) * (size_t)evcap);
    for (int64_t i = J->lo; i < J->hi; i++) {
        rng_t r = rng_stream(J->seed, (uint64_t)i);
        if (J->config == 3) { (void)rng_next(&r); (void)rng_next(&r); }   /* plan draws */
        fill_pair(J->config, &r, J->cat[i], J->len[i], J->reads + J->off[i], J->refs + J->off[i], ev, evcap);
    }
    free(ev);
    return NULL;
}

int ssgen_fill(int config, uint64_t seed, int64_t n, const uint8_t* cat, const int64_t* off,
               const int32_t* len, uint8_t* reads, uint8_t* refs, int threads)
{
    if (config < 0 || config > 3 || n < 0) return -1;
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    if (n < 4096) threads = 1;
    fill_job jobs[64];
    pthread_t tid[64];
    for (int t = 0; t < threads; t++) {
        fill_job* J = &jobs[t];
        J->config = config; J->seed = seed; J->lo = n * t / threads; J->hi = n * (t + 1) / threads;
        J->cat = cat; J->off = off; J->len = len; J->reads = reads; J->refs = refs;
    }
    if (threads == 1) fill_worker(&jobs[0]);
    else {
        for (int t = 0; t < threads; t++) pthread_create(&tid[t], NULL, fill_worker, &jobs[t]);
        for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Serving workload: Poisson arrivals; each request owns stream (seed, id).
 * Request: pairs = floor(exp(U(0, ln 4097))) clipped to [1, max_pairs];
 * per-pair length floor(exp(U(ln 100, ln 10001))) clipped to [min_len, max_len];
 * one E rate in basis points ~U{100..1000} per request, E = ceil(bp*m/1e4);
 * pairs follow the long-pair edit model above.
 * ------------------------------------------------------------------------- */
int64_t ssgen_arrivals(uint64_t seed, double rate, double duration, double* t_out, int64_t cap)
{
    rng_t r = rng_stream(seed, 0xA771A1ULL);
    double t = 0.0;
    int64_t n = 0;
    for (;;) {
        double u = rng_unit(&r);
        t += -log(1.0 - u) / rate;
        if (t >= duration) break;
        if (t_out && n < cap) t_out[n] = t;
        n++;
    }
    return n;
}

int32_t ssgen_request_pairs(uint64_t seed, int64_t req, int32_t max_pairs)
{
    rng_t r = rng_stream(seed ^ 0x5E4B1C0ULL, (uint64_t)req);
    int32_t n = (int32_t)floor(exp(rng_unit(&r) * log(4097.0)));
    if (n < 1) n = 1;
    if (n > max_pairs) n = max_pairs;
    return n;
}

/* lengths and E for the request's n pairs; returns the request's total bases */
int64_t ssgen_request_plan(uint64_t seed, int64_t req, int32_t n, int32_t min_len, int32_t max_len,
                           int32_t* len, int32_t* E)
{
    rng_t r = rng_stream(seed ^ 0x5E4B1C0ULL, (uint64_t)req);
    (void)rng_next(&r);                                   /* pair-count draw */
    int bp = 100 + (int)rng_below(&r, 901);
    int64_t tot = 0;
    for (int32_t i = 0; i < n; i++) {
        int m = (int)floor(exp(log(100.0) + rng_unit(&r) * (log(10001.0) - log(100.0))));
        if (m < min_len) m = min_len;
        if (m > max_len) m = max_len;
        len[i] = m;
        E[i] = ceil_bp(bp, m);
        tot += m;
    }
    return tot;
}

int ssgen_request_fill(uint64_t seed, int64_t req, int32_t n, const int64_t* off, const int32_t* len,
                       uint8_t* reads, uint8_t* refs)
{
    int evcap = 4096;
    edit_ev* ev = (edit_ev*)malloc(sizeof(edit_ev) * (size_t)evcap);
    for (int32_t i = 0; i < n; i++) {
        rng_t r = rng_stream(seed ^ ((uint64_t)req * 0x100000001B3ULL), (uint64_t)i);
        fill_pair(3, &r, CAT_LONG, len[i], reads + off[i], refs + off[i], ev, evcap);
    }
    free(ev);
    return 0;
}

/* n long pairs of length m (pair i at byte i*m): per pair an edit rate
 * ~U[bp_lo, bp_hi] basis points, round(rate*m/1e4) events, half substitutions,
 * half indels of Geometric(1/2) length (the long-pair model of configuration 3
 * at any length and rate range).  Pair i draws from stream i of the seed. */
int ssgen_long_fill(uint64_t seed, int64_t n, int32_t m, int32_t bp_lo, int32_t bp_hi, uint8_t* reads,
                    uint8_t* refs)
{
    if (n < 0 || m < 0 || bp_lo < 0 || bp_hi < bp_lo) return -1;
    int evcap = m + 1;
    edit_ev* ev = (edit_ev*)malloc(sizeof(edit_ev) * (size_t)evcap);
    if (!ev) return -1;
    for (int64_t i = 0; i < n; i++) {
        rng_t r = rng_stream(seed ^ 0x10C4B9ULL, (uint64_t)i);
        uint8_t* Q = reads + i * (int64_t)m;
        uint8_t* R = refs + i * (int64_t)m;
        rand_bases(&r, Q, m);
        const int bp = bp_lo + (int)rng_below(&r, (uint64_t)(bp_hi - bp_lo + 1));
        int k = (int)(((int64_t)bp * m + 5000) / 10000);
        if (k > evcap) k = evcap;
        for (int e = 0; e < k; e++) {
            edit_ev* v = &ev[e];
            v->ord = e; v->len = 1;
            if (rng_below(&r, 2) == 0) v->type = EV_SUB;
            else { v->type = rng_below(&r, 2) == 0 ? EV_INS : EV_DEL; v->len = rng_geom_half(&r); }
            v->pos = (int)rng_below(&r, (uint64_t)(v->type == EV_INS ? m + 1 : m));
        }
        apply_events(&r, Q, m, ev, k, R);
    }
    free(ev);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Native load driver for serving benchmarks.
 *
 * Generates the requests of a Poisson schedule on worker threads (each request
 * from its own stream) and submits them at their scheduled times
 * (CLOCK_MONOTONIC) through a caller supplied submit function with the
 * signature of the filter server's submit entry point.  Output buffers are allocated here and kept until
 * ssgen_drive_free.  This keeps the client's cost per request to a few
 * memcpys, so the measured latency is the server's.
 * ------------------------------------------------------------------------- */
#include <stdatomic.h>
#include <time.h>

typedef int (*ssgen_submit_fn)(void* server, const uint8_t* reads, const uint8_t* refs, const int32_t* lengths,
                               const int32_t* E, int64_t n, uint8_t* accept_out, int32_t* edits_out,
                               uint64_t* ticket);

/* staged submission: a block of the server's staging, freed back to it, and the submit that hands
 * a block over (signatures of ss_server_stage_alloc, ss_server_stage_free, ss_server_submit_staged) */
typedef void* (*ssgen_stage_alloc_fn)(void* server, size_t bytes);
typedef int (*ssgen_stage_free_fn)(void* server, void* block);
typedef int (*ssgen_submit_staged_fn)(void* server, void* block, size_t refs_offset, const int32_t* lengths,
                                      const int32_t* E, int64_t n, uint8_t* accept_out, int32_t* edits_out,
                                      uint64_t* ticket);

typedef struct {
    int32_t n;
    int64_t total;
    uint8_t* reads; uint8_t* refs;
    int32_t* lengths; int32_t* E;
    void* block;                 /* staged: reads and refs live in this block of the server's staging */
    size_t roff;                 /* where refs start in it */
} pool_req;

typedef struct {
    uint64_t seed; int64_t n_req; int32_t max_pairs, min_len, max_len;
    pool_req* pool; int64_t n_pool; _Atomic int64_t next_pool;
    /* on the fly: a ring of `lead` requests generated ahead of the clock; slot k holds position
     * ring_pos[k] once generated (-1: free) */
    pool_req* ring; _Atomic int64_t* ring_pos; int64_t lead;
    _Atomic int64_t next_gen;
    _Atomic int stop_gen;
    const double* arrivals; int64_t t0_ns;
    ssgen_submit_fn submit; void* server;
    ssgen_stage_alloc_fn stage_alloc; ssgen_stage_free_fn stage_free; ssgen_submit_staged_fn submit_staged;
    uint64_t* tickets; int64_t* due_ns; int64_t* call_ns; int32_t* pairs; int64_t* bases;
    uint8_t** accept_out; int32_t** edits_out;
    _Atomic int64_t next;
    _Atomic int failed;          /* first failing status, 0 if none */
    _Atomic int64_t submitted;
} drive_ctx;

static int64_t mono_ns(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

static void sleep_until(int64_t due)
{
    for (;;) {
        const int64_t now = mono_ns();
        if (now >= due) return;
        const int64_t left = due - now;
        if (left > 200000) {
            struct timespec ts = {(time_t)((left - 100000) / 1000000000LL), (long)((left - 100000) % 1000000000LL)};
            nanosleep(&ts, NULL);
        }
    }
}

static void make_request(drive_ctx* D, int64_t id, pool_req* q)
{
    const int32_t n = ssgen_request_pairs(D->seed, id, D->max_pairs);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    q->n = n;
    q->lengths = (int32_t*)malloc(sizeof(int32_t) * nn);
    q->E = (int32_t*)malloc(sizeof(int32_t) * nn);
    int64_t* offsets = (int64_t*)malloc(sizeof(int64_t) * nn);
    q->total = ssgen_request_plan(D->seed, id, n, D->min_len, D->max_len, q->lengths, q->E);
    int64_t o = 0;
    for (int32_t k = 0; k < n; k++) { offsets[k] = o; o += q->lengths[k]; }
    q->block = NULL;
    if (D->stage_alloc && D->n_pool == 0) {
        /* generated straight into the server's staging (no copy at submission) */
        q->roff = (size_t)((q->total + 15) / 16 * 16);
        q->block = D->stage_alloc(D->server, q->roff + (size_t)(q->total > 0 ? q->total : 1));
    }
    if (q->block) {
        q->reads = (uint8_t*)q->block;
        q->refs = (uint8_t*)q->block + q->roff;
    } else {
        q->reads = (uint8_t*)malloc((size_t)(q->total > 0 ? q->total : 1));
        q->refs = (uint8_t*)malloc((size_t)(q->total > 0 ? q->total : 1));
    }
    ssgen_request_fill(D->seed, id, n, offsets, q->lengths, q->reads, q->refs);
    free(offsets);
}

static void* pool_worker(void* arg)
{
    drive_ctx* D = (drive_ctx*)arg;
    for (;;) {
        const int64_t k = atomic_fetch_add(&D->next_pool, 1);
        if (k >= D->n_pool) break;
        make_request(D, k, &D->pool[k]);
    }
    return NULL;
}

static void nap_us(long us)
{
    struct timespec ts = {0, us * 1000L};
    nanosleep(&ts, NULL);
}

/* On the fly: generator threads make the requests in schedule order into the
 * ring, each waiting for its slot to be freed by the submission of the
 * request `lead` positions earlier. */
static void* gen_worker(void* arg)
{
    drive_ctx* D = (drive_ctx*)arg;
    for (;;) {
        const int64_t i = atomic_fetch_add(&D->next_gen, 1);
        if (i >= D->n_req) break;
        const int64_t k = i % D->lead;
        while (atomic_load(&D->ring_pos[k]) != -1) {
            if (atomic_load(&D->stop_gen)) return NULL;
            nap_us(50);
        }
        make_request(D, i, &D->ring[k]);
        atomic_store(&D->ring_pos[k], i);
    }
    return NULL;
}

/* Each submitter takes the next schedule position i, sleeps until it is due
 * and submits request (i mod pool size) itself, so the submit-time copies run
 * on all submitters.  Without a pool it first waits for request i in the ring
 * and frees the slot after submitting. */
static void* drive_worker(void* arg)
{
    drive_ctx* D = (drive_ctx*)arg;
    for (;;) {
        const int64_t i = atomic_fetch_add(&D->next, 1);
        if (i >= D->n_req || atomic_load(&D->failed)) break;
        const pool_req* q;
        if (D->n_pool > 0) q = &D->pool[i % D->n_pool];
        else {
            while (atomic_load(&D->ring_pos[i % D->lead]) != i) nap_us(20);
            q = &D->ring[i % D->lead];
        }
        const size_t nn = (size_t)(q->n > 0 ? q->n : 1);
        const int64_t due = D->t0_ns + (int64_t)(D->arrivals[i] * 1e9);
        D->accept_out[i] = (uint8_t*)malloc(nn);
        D->edits_out[i] = (int32_t*)malloc(sizeof(int32_t) * nn);
        D->due_ns[i] = due;
        D->pairs[i] = q->n;
        D->bases[i] = q->total;
        sleep_until(due);
        D->call_ns[i] = mono_ns();
        const int rc = q->block ? D->submit_staged(D->server, q->block, q->roff, q->lengths, q->E, q->n,
                                                   D->accept_out[i], D->edits_out[i], &D->tickets[i])
                                : D->submit(D->server, q->reads, q->refs, q->lengths, q->E, q->n, D->accept_out[i],
                                            D->edits_out[i], &D->tickets[i]);
        if (D->n_pool <= 0) {
            pool_req* own = &D->ring[i % D->lead];
            if (own->block) {
                if (rc != 0) D->stage_free(D->server, own->block);   /* refused: still ours */
                own->block = NULL;                                    /* else the server's now */
            } else {
                free(own->reads); free(own->refs);
            }
            free(own->lengths); free(own->E);
            atomic_store(&D->ring_pos[i % D->lead], -1);
        }
        if (rc != 0) {
            int zero = 0;
            atomic_compare_exchange_strong(&D->failed, &zero, rc);
            break;
        }
        atomic_fetch_add(&D->submitted, 1);
    }
    return NULL;
}

/* Runs the whole schedule; returns the number of requests submitted, or
 * -1 + (status of a failed submission).  Per request (n_req entries, indexed
 * by schedule position): ticket, due time and time of the submit call
 * (CLOCK_MONOTONIC ns), pairs, bases,
 * and output buffers owned here until ssgen_drive_free.  pool > 0: requests
 * 0..pool-1 are generated (on `threads` threads) before the schedule starts,
 * and position i replays request i mod pool, submitted by `threads`
 * submitters.  pool = 0: every position's request is generated from its own
 * seed on the fly by `threads` generator threads, running up to
 * min(n_req, 2048) positions ahead of the submissions (the first ones before
 * the clock starts), and submitted by 8 submitters.  With stage_alloc,
 * stage_free and submit_staged given (pool = 0 only), each request is
 * generated into a block of the server's staging and handed over without a
 * copy (a request falls back to submit when the staging is full), 512 ahead.
 * t0_ns: schedule time zero (0 = 100 ms after the pool or the head start is
 * ready). */
int64_t ssgen_drive(uint64_t seed, const double* arrivals, int64_t n_req, int32_t max_pairs, int32_t min_len,
                    int32_t max_len, ssgen_submit_fn submit, void* server, int threads, int64_t pool,
                    int64_t t0_ns, uint64_t* tickets, int64_t* due_ns, int64_t* call_ns, int32_t* pairs,
                    int64_t* bases,
                    uint8_t** accept_out, int32_t** edits_out, ssgen_stage_alloc_fn stage_alloc,
                    ssgen_stage_free_fn stage_free, ssgen_submit_staged_fn submit_staged)
{
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    drive_ctx D;
    D.seed = seed; D.n_req = n_req; D.max_pairs = max_pairs; D.min_len = min_len; D.max_len = max_len;
    D.arrivals = arrivals; D.submit = submit; D.server = server;
    /* staged only with all three functions, and only on the fly (a replayed pool is submitted many times) */
    const int staged = stage_alloc && stage_free && submit_staged && pool <= 0;
    D.stage_alloc = staged ? stage_alloc : NULL;
    D.stage_free = staged ? stage_free : NULL;
    D.submit_staged = staged ? submit_staged : NULL;
    D.tickets = tickets; D.due_ns = due_ns; D.call_ns = call_ns; D.pairs = pairs; D.bases = bases;
    D.accept_out = accept_out; D.edits_out = edits_out;
    for (int64_t i = 0; i < n_req; i++) { accept_out[i] = NULL; edits_out[i] = NULL; }
    D.n_pool = pool > 0 ? pool : 0;
    D.pool = (pool_req*)calloc((size_t)(D.n_pool > 0 ? D.n_pool : 1), sizeof(pool_req));
    atomic_store(&D.next_pool, 0);
    /* staged: the ring holds server staging, so it runs 512 ahead instead of 2,048 */
    const int64_t lead_max = staged ? 512 : 2048;
    D.lead = D.n_pool > 0 ? 1 : (n_req < lead_max ? (n_req > 0 ? n_req : 1) : lead_max);
    D.ring = (pool_req*)calloc((size_t)D.lead, sizeof(pool_req));
    D.ring_pos = (_Atomic int64_t*)malloc(sizeof(_Atomic int64_t) * (size_t)D.lead);
    for (int64_t k = 0; k < D.lead; k++) atomic_store(&D.ring_pos[k], -1);
    atomic_store(&D.next_gen, 0);
    atomic_store(&D.stop_gen, 0);
    pthread_t gt[64];
    int n_gen = 0;
    if (D.n_pool > 0) {
        pthread_t pt[64];
        for (int t = 0; t < threads; t++) pthread_create(&pt[t], NULL, pool_worker, &D);
        for (int t = 0; t < threads; t++) pthread_join(pt[t], NULL);
    } else {
        n_gen = threads;
        for (int t = 0; t < n_gen; t++) pthread_create(&gt[t], NULL, gen_worker, &D);
        /* head start: the ring full (or every request) before the clock starts */
        const int64_t head = D.lead < n_req ? D.lead : n_req;
        for (int64_t k = 0; k < head; k++)
            while (atomic_load(&D.ring_pos[k]) != k) nap_us(200);
    }
    D.t0_ns = t0_ns ? t0_ns : mono_ns() + 100000000LL;
    atomic_store(&D.next, 0);
    atomic_store(&D.failed, 0);
    atomic_store(&D.submitted, 0);
    const int n_sub = D.n_pool > 0 ? threads : 8;
    pthread_t tid[64];
    for (int t = 0; t < n_sub; t++) pthread_create(&tid[t], NULL, drive_worker, &D);
    for (int t = 0; t < n_sub; t++) pthread_join(tid[t], NULL);
    atomic_store(&D.stop_gen, 1);
    for (int t = 0; t < n_gen; t++) pthread_join(gt[t], NULL);
    for (int64_t k = 0; k < D.lead; k++) {
        /* requests generated but never submitted (a submission failed) */
        if (D.n_pool == 0 && atomic_load(&D.ring_pos[k]) != -1) {
            if (D.ring[k].block) D.stage_free(D.server, D.ring[k].block);
            else { free(D.ring[k].reads); free(D.ring[k].refs); }
            free(D.ring[k].lengths); free(D.ring[k].E);
        }
    }
    free(D.ring);
    free((void*)D.ring_pos);
    for (int64_t k = 0; k < D.n_pool; k++) {
        free(D.pool[k].reads); free(D.pool[k].refs); free(D.pool[k].lengths); free(D.pool[k].E);
    }
    free(D.pool);
    const int f = atomic_load(&D.failed);
    return f ? (int64_t)(-1 + f) : atomic_load(&D.submitted);
}

void ssgen_drive_free(int64_t n_req, uint8_t** accept_out, int32_t** edits_out)
{
    for (int64_t i = 0; i < n_req; i++) {
        free(accept_out[i]);
        free(edits_out[i]);
    }
}
