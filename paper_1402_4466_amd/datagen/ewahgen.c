/*
 * Seeded synthetic bitmap generators.
 *
 * This module only produces inputs.  It contains no threshold logic and is
 * shared by the CPU oracle tests and the GPU path, so that both sides see the
 * same bytes.  Each bitmap is produced directly as an EWAH word stream
 * (64-bit words, marker word = fill bit | L << 1 | K << 33, see the EWAH
 * description of Section 3.1), optionally with non-canonical but well-formed
 * perturbations (split runs, empty markers, fill-valued literals) so that
 * decoders can be exercised on streams a canonical encoder never writes.
 *
 * Random numbers: counter-based SplitMix64 (Steele, Lea, Flood 2014): draw i
 * of stream key k is mix64(k + (i + 1) * 0x9E3779B97F4A7C15).
 *
 * Bitmap models (workload shapes of Section 7.2 and Table real-data-char):
 *   model 0: every bit iid Bernoulli(p), set bits placed by geometric gaps;
 *   model 1: two-state Markov chain over bits, 1-runs geometric with mean m1,
 *            0-runs geometric with mean m0, first state drawn from the
 *            stationary distribution P(1) = m1 / (m0 + m1).
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t key, ctr; } rng_t;

static inline uint64_t rng_next(rng_t* r) { r->ctr += 1; return mix64(r->key + r->ctr * GOLDEN); }
/* uniform in (0, 1] */
static inline double rng_unit(rng_t* r) { return ((double)((rng_next(r) >> 11) + 1)) * (1.0 / 9007199254740992.0); }

uint64_t ewahgen_key(uint64_t seed, uint64_t stream_id) {
    return mix64(seed ^ mix64(stream_id + 0x5851F42D4C957F2DULL));
}

/* ---------------------------------------------------------------- writer */

#define MAXL 0xFFFFFFFFULL      /* 32-bit fill counter */
#define MAXK 0x7FFFFFFFULL      /* 31-bit literal counter */

typedef struct {
    uint64_t* out; uint64_t cap; uint64_t n;   /* output stream */
    int64_t mk;                                /* index of open marker, -1 if none */
    uint64_t f, L, K;                          /* fields of open marker */
    int overflow;
    int noncanon; rng_t prng;                  /* perturbation stream */
} writer_t;

static void w_put(writer_t* w, uint64_t v) {
    if (w->n < w->cap) w->out[w->n] = v; else w->overflow = 1;
    w->n++;
}
static void w_flush_marker(writer_t* w) {
    if (w->mk >= 0 && (uint64_t)w->mk < w->cap) w->out[w->mk] = w->f | (w->L << 1) | (w->K << 33);
}
static void w_new_marker(writer_t* w, uint64_t f) {
    w_flush_marker(w);
    w->mk = (int64_t)w->n; w->f = f; w->L = 0; w->K = 0;
    w_put(w, 0);
}
/* Maybe emit an empty marker (L = 0, K = 0) or split here: non-canonical streams. */
static void w_perturb(writer_t* w) {
    if (!w->noncanon) return;
    uint64_t x = rng_next(&w->prng);
    if ((x & 63) == 0) { w_new_marker(w, (x >> 6) & 1); }
}
/* append `count` fill words of value f (0 or 1) */
static void w_fill(writer_t* w, uint64_t f, uint64_t count) {
    while (count) {
        w_perturb(w);
        if (!(w->mk >= 0 && w->K == 0 && w->f == f && w->L < MAXL)) w_new_marker(w, f);
        uint64_t room = MAXL - w->L;
        uint64_t take = count < room ? count : room;
        if (w->noncanon && take > 1 && (rng_next(&w->prng) & 7) == 0) take = 1 + rng_next(&w->prng) % take;
        w->L += take; count -= take;
        if (w->noncanon && count && (rng_next(&w->prng) & 3) == 0) w_new_marker(w, f); /* split run */
    }
}
static void w_literal(writer_t* w, uint64_t v) {
    w_perturb(w);
    if (w->mk < 0 || w->K == MAXK) w_new_marker(w, 0);
    w->K += 1;
    w_put(w, v);
}
/* append one uncompressed word (already masked if it is the last partial one) */
static void w_word(writer_t* w, uint64_t v, int is_last_partial) {
    int fill0 = (v == 0), fill1 = (v == ~0ULL) && !is_last_partial;
    if (w->noncanon && (fill0 || fill1) && (rng_next(&w->prng) % 11) == 0) { w_literal(w, v); return; }
    if (fill0) w_fill(w, 0, 1);
    else if (fill1) w_fill(w, 1, 1);
    else w_literal(w, v);
}
static uint64_t w_finish(writer_t* w) {
    w_flush_marker(w);
    return w->overflow ? (uint64_t)(-1) : w->n;
}

/* ------------------------------------------------------------- bit sink */
/* Accumulates set-bit runs [a, b) in increasing order and writes words. */
typedef struct {
    writer_t* w; uint64_t n_bits, U;
    uint64_t cur_idx; uint64_t cur;   /* word being built */
} sink_t;

static void s_emit_upto(sink_t* s, uint64_t idx) {  /* flush words < idx */
    if (s->cur_idx >= idx) return;
    uint64_t v = s->cur;
    int partial = (s->n_bits & 63) != 0 && s->cur_idx == s->U - 1;
    if (partial) v &= (1ULL << (s->n_bits & 63)) - 1;
    w_word(s->w, v, partial);
    s->cur = 0; s->cur_idx++;
    if (s->cur_idx < idx) {          /* zero words in between are zero fills */
        w_fill(s->w, 0, idx - s->cur_idx);
        s->cur_idx = idx;
    }
}
static void s_set_run(sink_t* s, uint64_t a, uint64_t b) {  /* set bits [a, b), b <= n_bits */
    while (a < b) {
        uint64_t wi = a >> 6;
        s_emit_upto(s, wi);
        uint64_t lo = a & 63;
        uint64_t hi_abs = (wi + 1) << 6;
        if (lo == 0 && b >= hi_abs && (b - a) >= 128) {
            /* whole words of ones: emit them as a run */
            uint64_t nw = (b - a) >> 6;
            if (wi + nw > s->U - 1 && (s->n_bits & 63)) nw = s->U - 1 - wi;   /* keep last partial word separate */
            if (nw >= 2) {
                w_fill(s->w, 1, nw);
                s->cur_idx = wi + nw; s->cur = 0;
                a += nw << 6;
                continue;
            }
        }
        uint64_t end = b < hi_abs ? b : hi_abs;
        uint64_t hi = end - (wi << 6);
        uint64_t m = (hi == 64 ? ~0ULL : ((1ULL << hi) - 1)) & ~((1ULL << lo) - 1);
        s->cur |= m;
        a = end;
    }
}
static uint64_t s_finish(sink_t* s) {
    if (s->U) s_emit_upto(s, s->U);
    return w_finish(s->w);
}

/* -------------------------------------------------------------- models */

/* geometric number of failures before a success with success prob p (p in (0,1)) */
static inline uint64_t geom_fail(rng_t* r, double lq) { /* lq = log(1-p) */
    double u = rng_unit(r);
    double g = floor(log(u) / lq);
    if (g > 1.8e19) g = 1.8e19;
    return (uint64_t)g;
}

/*
 * Generate one bitmap as an EWAH stream.
 *   model 0: iid Bernoulli(a)           (b ignored)
 *   model 1: Markov, mean 1-run a bits, mean 0-run b bits
 *   flags bit 0: non-canonical perturbations
 * Returns the number of words, or (uint64_t)-1 if cap was too small
 * (cap = ceil(n_bits/64) + 1 always suffices for canonical output; use
 * 2 * ceil(n_bits/64) + 64 with flags bit 0).
 */
uint64_t ewahgen_bitmap(int model, double a, double b, uint64_t n_bits, uint64_t key, int flags,
                        uint64_t* out, uint64_t cap) {
    writer_t w; memset(&w, 0, sizeof w);
    w.out = out; w.cap = cap; w.mk = -1;
    w.noncanon = flags & 1; w.prng.key = mix64(key ^ 0xD1B54A32D192ED03ULL); w.prng.ctr = 0;
    sink_t s; s.w = &w; s.n_bits = n_bits; s.U = (n_bits + 63) >> 6; s.cur_idx = 0; s.cur = 0;
    rng_t r; r.key = key; r.ctr = 0;
    if (n_bits == 0) return w_finish(&w);
    if (model == 0) {
        double p = a;
        if (p >= 1.0) { s_set_run(&s, 0, n_bits); }
        else if (p > 0.0) {
            double lq = log1p(-p);
            uint64_t pos = geom_fail(&r, lq);
            while (pos < n_bits) {
                s_set_run(&s, pos, pos + 1);
                uint64_t g = geom_fail(&r, lq);
                if (g >= n_bits) break;
                pos += 1 + g;
            }
        }
    } else {
        double m1 = a, m0 = b;
        double l1 = log1p(-1.0 / m1), l0 = log1p(-1.0 / m0);
        int state = rng_unit(&r) <= m1 / (m0 + m1);
        uint64_t pos = 0;
        while (pos < n_bits) {
            uint64_t len = 1 + geom_fail(&r, state ? l1 : l0);
            uint64_t end = (len > n_bits - pos) ? n_bits : pos + len;
            if (state) s_set_run(&s, pos, end);
            pos = end; state ^= 1;
        }
    }
    return s_finish(&s);
}

/* Generate `count` bitmaps in parallel into out + i * cap_each; n_out[i] gets the word count. */
void ewahgen_batch(int count, const int* model, const double* a, const double* b, uint64_t n_bits,
                   const uint64_t* keys, int flags, uint64_t* out, uint64_t cap_each, uint64_t* n_out) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < count; ++i)
        n_out[i] = ewahgen_bitmap(model[i], a[i], b[i], n_bits, keys[i], flags, out + (uint64_t)i * cap_each, cap_each);
}

/*
 * Query generator for the batched workloads: query q draws N uniform in
 * [nmin, nmax], N distinct pool indices (partial Fisher-Yates), T uniform in
 * [1, N].  idx must hold n_queries * nmax entries; query q's indices are at
 * idx + q * nmax.
 */
void ewahgen_queries(uint64_t seed, int n_queries, int n_pool, int nmin, int nmax,
                     uint32_t* n_out, uint32_t* t_out, uint32_t* idx) {
    #pragma omp parallel
    {
        uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n_pool);
        #pragma omp for schedule(static)
        for (int q = 0; q < n_queries; ++q) {
            rng_t r; r.key = ewahgen_key(seed, 0x100000000ULL + (uint64_t)q); r.ctr = 0;
            uint32_t n = (uint32_t)(nmin + rng_next(&r) % (uint64_t)(nmax - nmin + 1));
            if (n > (uint32_t)n_pool) n = (uint32_t)n_pool;
            for (int i = 0; i < n_pool; ++i) perm[i] = (uint32_t)i;
            for (uint32_t i = 0; i < n; ++i) {
                uint32_t j = i + (uint32_t)(rng_next(&r) % (uint64_t)(n_pool - i));
                uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
                idx[(uint64_t)q * nmax + i] = perm[i];
            }
            n_out[q] = n;
            t_out[q] = (uint32_t)(1 + rng_next(&r) % n);
        }
        free(perm);
    }
}

/* iid uniform doubles in (0,1] for stream key (used for log-uniform densities) */
void ewahgen_uniform(uint64_t key, int count, double* out) {
    rng_t r; r.key = key; r.ctr = 0;
    for (int i = 0; i < count; ++i) out[i] = rng_unit(&r);
}

/*
 * Bitmaps of a bitmap index from row lists: bitmap i holds the rows
 * rows[row_off[i] .. row_off[i+1]) (strictly increasing, each < n_bits) and is
 * written canonically into out + out_off[i], at most out_off[i+1] - out_off[i]
 * words.  n_out[i] gets its word count, or (uint64_t)-1 if that room was too
 * small (2 * rows + 2 words, or ceil(n_bits/64) + 1, always suffice).
 */
void ewahgen_rows_batch(int count, const uint64_t* row_off, const uint32_t* rows, uint64_t n_bits,
                        const uint64_t* out_off, uint64_t* out, uint64_t* n_out) {
    #pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < count; ++i) {
        writer_t w; memset(&w, 0, sizeof w);
        w.out = out + out_off[i]; w.cap = out_off[i + 1] - out_off[i]; w.mk = -1;
        sink_t s; s.w = &w; s.n_bits = n_bits; s.U = (n_bits + 63) >> 6; s.cur_idx = 0; s.cur = 0;
        uint64_t j = row_off[i], e = row_off[i + 1];
        int bad = 0;
        while (j < e) {                     /* consecutive rows become one run */
            uint64_t a = rows[j], b = a + 1;
            if (a >= n_bits || (j > row_off[i] && a <= rows[j - 1])) { bad = 1; break; }
            ++j;
            while (j < e && rows[j] == b && b < n_bits) { ++b; ++j; }
            s_set_run(&s, a, b);
        }
        n_out[i] = bad ? (uint64_t)(-1) : (n_bits ? s_finish(&s) : w_finish(&w));
    }
}
