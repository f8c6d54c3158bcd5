/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference for the T-of-N threshold query over
 * EWAH-compressed bitmaps (Kaser & Lemire, "Compressed bitmap indexes: beyond
 * unions and intersections").  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the GPU library
 * never links, calls or includes anything from here, and this file shares no
 * code with it.
 *
 * What is computed, and where the paper defines it:
 *   - threshold function: output row i is 1 iff at least T of the N input
 *     bitmaps have row i set (Section 2, Formulation; Fig. basicexample);
 *   - uncompressed layout: row i is bit (i mod 64) of word floor(i / 64), the
 *     least-significant bit holding the smallest row (Section 3.1,
 *     "Uncompressed Bitmaps", with W = 64);
 *   - counting method: ScanCount (Section 5.1) -- one counter per row, the
 *     bitmaps scanned one at a time, every set bit incrementing its row's
 *     counter, then a final pass comparing each counter with T;
 *   - EWAH stream (Section 3.1, "Compressed Bitmaps"; the paper defers the
 *     exact layout to the EWAH format paper and states that 64-bit EWAH uses
 *     32-bit run counters).  Reading adopted here: a marker word holds the fill
 *     bit in bit 0, the number L of fill words in bits 1..32 and the number K
 *     of literal (dirty) words that follow it in bits 33..63; a stream is
 *     marker, K literals, marker, ...
 *
 * Decoder: lenient.  Any well-formed stream is accepted (literal words equal
 * to 0 or ~0, split runs, empty markers).  It requires that the runs cover
 * exactly U = ceil(r / 64) words and that no literal run is cut off by the end
 * of the stream.  Padding bits beyond row r - 1 are masked to zero.
 *
 * Encoder: canonical.  (C1) every word equal to 0 or ~0 after masking is a
 * fill, never a literal; (C2) a marker starts at word 0 and at every fill word
 * whose predecessor is a literal or a fill of the other value, and also when L
 * would exceed 2^32 - 1 or, with L = 0, when K would exceed 2^31 - 1;
 * (C3) literals attach to the preceding marker; (C4) the stream covers exactly
 * U words, trailing zero fills included, and r = 0 gives the empty stream.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 malformed stream,
 * -3 out of memory, -4 output capacity too small.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EFORMAT (-2)
#define ORC_ENOMEM (-3)
#define ORC_ENOSPC (-4)

static uint64_t words_for_bits(uint64_t n_bits) { return (n_bits + 63) / 64; }

static uint64_t last_word_mask(uint64_t n_bits) {
    uint64_t rem = n_bits % 64;
    return rem == 0 ? ~(uint64_t)0 : (((uint64_t)1 << rem) - 1);
}

/* Decode one EWAH stream into U = ceil(n_bits / 64) uncompressed words. */
int orc_decode(const uint64_t* words, uint64_t n_words, uint64_t n_bits, uint64_t* dense) {
    uint64_t U = words_for_bits(n_bits);
    uint64_t pos = 0;   /* next uncompressed word */
    uint64_t p = 0;     /* next compressed word */
    if (n_words > 0 && words == NULL) return ORC_EINVAL;
    if (U > 0 && dense == NULL) return ORC_EINVAL;
    while (p < n_words) {
        uint64_t marker = words[p];
        p += 1;
        uint64_t fill_bit = marker & 1;
        uint64_t L = (marker >> 1) & 0xFFFFFFFFULL;
        uint64_t K = marker >> 33;
        if (L > U - pos) return ORC_EFORMAT;
        for (uint64_t i = 0; i < L; ++i) dense[pos + i] = fill_bit ? ~(uint64_t)0 : 0;
        pos += L;
        if (K > n_words - p) return ORC_EFORMAT;   /* stream ends inside a literal run */
        if (K > U - pos) return ORC_EFORMAT;
        for (uint64_t i = 0; i < K; ++i) dense[pos + i] = words[p + i];
        pos += K;
        p += K;
    }
    if (pos != U) return ORC_EFORMAT;
    if (U > 0) dense[U - 1] &= last_word_mask(n_bits);
    return ORC_OK;
}

/* Canonical EWAH encoding of U uncompressed words. */
int orc_encode(const uint64_t* dense, uint64_t n_bits, uint64_t* out, uint64_t cap, uint64_t* n_out) {
    const uint64_t MAXL = 0xFFFFFFFFULL, MAXK = 0x7FFFFFFFULL;
    uint64_t U = words_for_bits(n_bits);
    uint64_t n = 0;
    int have_marker = 0;
    uint64_t mk = 0, f = 0, L = 0, K = 0;
    int overflow = 0;
    for (uint64_t i = 0; i < U; ++i) {
        uint64_t v = dense[i];
        if (i == U - 1) v &= last_word_mask(n_bits);
        int cls = (v == 0) ? 0 : (v == ~(uint64_t)0 ? 1 : 2);
        if (cls != 2) {
            if (have_marker && K == 0 && f == (uint64_t)cls && L < MAXL) {
                L += 1;
            } else {
                if (have_marker) { if (mk < cap) out[mk] = f | (L << 1) | (K << 33); }
                have_marker = 1; mk = n; f = (uint64_t)cls; L = 1; K = 0;
                n += 1;
            }
        } else {
            if (!have_marker || K == MAXK) {
                if (have_marker) { if (mk < cap) out[mk] = f | (L << 1) | (K << 33); }
                have_marker = 1; mk = n; f = 0; L = 0; K = 0;
                n += 1;
            }
            K += 1;
            if (n < cap) out[n] = v; else overflow = 1;
            n += 1;
        }
    }
    if (have_marker) { if (mk < cap) out[mk] = f | (L << 1) | (K << 33); else overflow = 1; }
    *n_out = n;
    return overflow || n > cap ? ORC_ENOSPC : ORC_OK;
}

/*
 * T-of-N threshold by ScanCount.  streams[k] / n_words[k] describe input k,
 * all over n_bits rows.  Writes the canonical EWAH encoding of the result to
 * out (capacity cap words) and its length to *n_out.  If hist is not NULL it
 * receives the count histogram hist[c] = number of rows covered by exactly c
 * inputs, c = 0..N.
 */
int orc_threshold(const uint64_t* const* streams, const uint64_t* n_words, uint32_t N, uint64_t n_bits,
                  uint32_t T, uint64_t* out, uint64_t cap, uint64_t* n_out, uint64_t* hist) {
    uint64_t U = words_for_bits(n_bits);
    uint32_t* counter = (uint32_t*)calloc(n_bits ? n_bits : 1, sizeof(uint32_t));
    uint64_t* dense = (uint64_t*)malloc((U ? U : 1) * sizeof(uint64_t));
    if (!counter || !dense) { free(counter); free(dense); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (uint32_t k = 0; k < N; ++k) {
        rc = orc_decode(streams[k], n_words[k], n_bits, dense);
        if (rc != ORC_OK) goto done;
        for (uint64_t i = 0; i < U; ++i) {
            uint64_t v = dense[i];
            if (v == 0) continue;
            for (uint64_t b = 0; b < 64; ++b)
                if ((v >> b) & 1) counter[i * 64 + b] += 1;
        }
    }
    if (hist) {
        for (uint32_t c = 0; c <= N; ++c) hist[c] = 0;
        for (uint64_t row = 0; row < n_bits; ++row) hist[counter[row]] += 1;
    }
    for (uint64_t i = 0; i < U; ++i) dense[i] = 0;
    for (uint64_t row = 0; row < n_bits; ++row)
        if (counter[row] >= T) dense[row / 64] |= (uint64_t)1 << (row % 64);
    rc = orc_encode(dense, n_bits, out, cap, n_out);
done:
    free(counter);
    free(dense);
    return rc;
}

/*
 * Symmetric function of the inputs (Section 2: threshold functions are the
 * symmetric Boolean functions given by "count >= T"; Section 3.2: a symmetric
 * function depends only on the number of ones among its inputs; Section 5.1:
 * ScanCount handles any user function from [0, N] to the Booleans).  Same
 * counting as orc_threshold; output row i is f[counter[i]], where f holds N + 1
 * entries (0 or non-zero).  Padding rows stay 0.
 */
int orc_symmetric(const uint64_t* const* streams, const uint64_t* n_words, uint32_t N, uint64_t n_bits,
                  const uint8_t* f, uint64_t* out, uint64_t cap, uint64_t* n_out) {
    if (!f) return ORC_EINVAL;
    uint64_t U = words_for_bits(n_bits);
    uint32_t* counter = (uint32_t*)calloc(n_bits ? n_bits : 1, sizeof(uint32_t));
    uint64_t* dense = (uint64_t*)malloc((U ? U : 1) * sizeof(uint64_t));
    if (!counter || !dense) { free(counter); free(dense); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (uint32_t k = 0; k < N; ++k) {
        rc = orc_decode(streams[k], n_words[k], n_bits, dense);
        if (rc != ORC_OK) goto done;
        for (uint64_t i = 0; i < U; ++i) {
            uint64_t v = dense[i];
            if (v == 0) continue;
            for (uint64_t b = 0; b < 64; ++b)
                if ((v >> b) & 1) counter[i * 64 + b] += 1;
        }
    }
    for (uint64_t i = 0; i < U; ++i) dense[i] = 0;
    for (uint64_t row = 0; row < n_bits; ++row)
        if (f[counter[row]]) dense[row / 64] |= (uint64_t)1 << (row % 64);
    rc = orc_encode(dense, n_bits, out, cap, n_out);
done:
    free(counter);
    free(dense);
    return rc;
}
