/* Drives the C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host only):
 * random uncompressed words are encoded and decoded back, random thresholds are taken
 * over encoded streams (checked row by row against counts of the uncompressed words),
 * and random word sequences are fed to the decoder as streams, which must either
 * decode or be rejected with a status, never read or write out of bounds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_decode(const uint64_t* words, uint64_t n_words, uint64_t n_bits, uint64_t* dense);
int orc_encode(const uint64_t* dense, uint64_t n_bits, uint64_t* out, uint64_t cap, uint64_t* n_out);
int orc_threshold(const uint64_t* const* streams, const uint64_t* n_words, uint32_t N, uint64_t n_bits, uint32_t T,
                  uint64_t* out, uint64_t cap, uint64_t* n_out, uint64_t* hist);

static uint64_t st = 0x1402446614024466ull;
static uint64_t rnd(void) {   /* SplitMix64 */
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t word_of_class(void) {
    switch (rnd() % 4) {
        case 0: return 0;
        case 1: return ~(uint64_t)0;
        default: return rnd() & rnd();
    }
}

int main(void) {
    for (int it = 0; it < 400; ++it) {
        const uint64_t n_bits = 1 + rnd() % 3000, U = (n_bits + 63) / 64;
        const uint32_t N = 1 + (uint32_t)(rnd() % 6);
        uint64_t* dense = malloc(N * U * 8);
        uint64_t** enc = malloc(N * sizeof(uint64_t*));
        uint64_t* nw = malloc(N * 8);
        for (uint32_t k = 0; k < N; ++k) {
            for (uint64_t w = 0; w < U; ++w) dense[k * U + w] = word_of_class();
            if (n_bits % 64) dense[k * U + U - 1] &= ((uint64_t)1 << (n_bits % 64)) - 1;
            enc[k] = malloc((U + 1) * 8);
            if (orc_encode(dense + k * U, n_bits, enc[k], U + 1, &nw[k]) != 0) { printf("FAIL encode\n"); return 1; }
            uint64_t* back = malloc(U * 8);
            if (orc_decode(enc[k], nw[k], n_bits, back) != 0 || memcmp(back, dense + k * U, U * 8) != 0) {
                printf("FAIL roundtrip\n");
                return 1;
            }
            free(back);
        }
        const uint32_t T = (uint32_t)(rnd() % (N + 2));
        uint64_t* out = malloc((U + 1) * 8);
        uint64_t* hist = malloc((N + 1) * 8);
        uint64_t n_out = 0;
        if (orc_threshold((const uint64_t* const*)enc, nw, N, n_bits, T, out, U + 1, &n_out, hist) != 0) {
            printf("FAIL threshold\n");
            return 1;
        }
        uint64_t* res = malloc(U * 8);
        if (orc_decode(out, n_out, n_bits, res) != 0) { printf("FAIL decode of result\n"); return 1; }
        for (uint64_t i = 0; i < n_bits; ++i) {
            uint32_t c = 0;
            for (uint32_t k = 0; k < N; ++k) c += (uint32_t)((dense[k * U + i / 64] >> (i % 64)) & 1);
            if ((uint32_t)((res[i / 64] >> (i % 64)) & 1) != (c >= T)) { printf("FAIL row %llu\n", (unsigned long long)i); return 1; }
        }
        /* random words as a stream: decode or a status, within bounds */
        const uint64_t len = rnd() % 40;
        uint64_t* junk = malloc((len ? len : 1) * 8);
        for (uint64_t j = 0; j < len; ++j) {
            const uint64_t L = rnd() % (U + 2), K = rnd() % 4;
            junk[j] = (rnd() % 3 == 0) ? rnd() : ((rnd() & 1) | (L << 1) | (K << 33));
        }
        uint64_t* dd = malloc(U * 8);
        (void)orc_decode(junk, len, n_bits, dd);
        free(dd);
        free(junk);
        free(res);
        free(out);
        free(hist);
        for (uint32_t k = 0; k < N; ++k) free(enc[k]);
        free(enc);
        free(nw);
        free(dense);
    }
    printf("ok\n");
    return 0;
}
