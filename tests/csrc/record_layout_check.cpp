// Host check of the fine presence record layout (the same __host__ __device__ helpers the
// registration and the kernels use): for every tile count a bitmap can have (1 .. 2^22, every
// count up to 70,000 and a spread of larger ones up to the largest), the per-word bits, the
// quarter bits and the two halves of the 8-row bits of every tile lie in four disjoint arrays in
// that order, each tile's quarter and 8-row parts start on a 128-byte line, and every offset
// fits the 32-bit word index the kernels compute (checked against 64-bit arithmetic).
#include <cstdint>
#include <cstdio>

#include "thr_device.h"

using namespace ewt;

static bool check(uint32_t tiles, long& checks) {
    const uint64_t T = tiles;
    const uint64_t q = pq_quarters(tiles), o0 = pq_octets(tiles, 0u), o1 = pq_octets(tiles, 1u), end = pq_words(tiles);
    // 64-bit reference of the same layout
    const uint64_t q64 = (T * PQ_W_TILE + 31u) / 32u * 32u;
    if (q != q64 || o0 != q64 + T * PQ_Q_TILE || o1 != o0 + T * PQ_O_TILE || end != o1 + T * PQ_O_TILE) {
        std::printf("offsets differ from 64-bit arithmetic at tiles=%u\n", tiles);
        return false;
    }
    if (end >= (1ull << 32)) { std::printf("record words overflow 32 bits at tiles=%u\n", tiles); return false; }
    // the per-word bits of the last tile end before the quarters; parts on 128-byte lines
    if (T * PQ_W_TILE > q || q % 32u || o0 % 32u || o1 % 32u || PQ_Q_TILE % 32u || PQ_O_TILE % 32u) {
        std::printf("layout or alignment broken at tiles=%u\n", tiles);
        return false;
    }
    // the last tile's parts (the first tile's start each array)
    const uint64_t t = T - 1u;
    if (t * PQ_W_TILE + PQ_W_TILE > q || q + t * PQ_Q_TILE + PQ_Q_TILE > o0 || o0 + t * PQ_O_TILE + PQ_O_TILE > o1 ||
        o1 + t * PQ_O_TILE + PQ_O_TILE > end) {
        std::printf("parts overlap at tiles=%u\n", tiles);
        return false;
    }
    ++checks;
    return true;
}

int main() {
    static_assert(PQ_W_TILE * 32u == (uint32_t)TW && PQ_Q_TILE * 32u == (uint32_t)NQ_TILE &&
                  2u * PQ_O_TILE * 32u == (uint32_t)NO_TILE, "one bit per word, quarter and 8-row group");
    long checks = 0;
    const uint32_t max_tiles = 1u << 22;   // U < 2^31 words of 512-word tiles
    for (uint32_t tiles = 1; tiles <= 70000u; ++tiles)
        if (!check(tiles, checks)) return 1;
    for (uint64_t tiles = 70001; tiles <= max_tiles; tiles = tiles * 17 / 16 + 1)
        if (!check((uint32_t)tiles, checks)) return 1;
    for (uint32_t tiles = max_tiles - 64u; tiles <= max_tiles; ++tiles)
        if (!check(tiles, checks)) return 1;
    std::printf("ok %ld tile counts\n", checks);
    return 0;
}
