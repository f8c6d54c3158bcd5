// Host check of the bounds pre-pass item order (pre_item_order, the __host__ __device__ helper the
// kernel calls): for batches of nq queries of `tiles` tiles each, split into NXCD shares the way the
// pre-pass launch splits its workgroups (w wavefronts per workgroup, workgroup b on XCD b mod NXCD,
// contiguous shares of nwg / NXCD workgroups, the first nwg mod NXCD shares one more), every share
// is mapped onto itself one to one, and a share of whole queries is taken in blocks of PRE_TB tiles:
// block k of every query of the share before block k + 1, tiles in order inside a block.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "thr_device.h"

using namespace ewt;

static long whole_shares = 0;

static bool check(uint32_t nq, uint32_t tiles, uint32_t w, long& checks) {
    const uint32_t total = nq * tiles;
    const uint32_t nwg = (total + w - 1) / w, per = nwg / NXCD, ext = nwg % NXCD;
    std::vector<uint8_t> seen(total, 0);
    for (uint32_t x = 0; x < (uint32_t)NXCD; ++x) {
        const uint32_t wg0 = x * per + (x < ext ? x : ext);
        const uint32_t a = wg0 * w;
        const uint32_t e = std::min((wg0 + per + (x < ext ? 1u : 0u)) * w, total);
        if (a >= e) continue;
        const bool whole = tiles > 1u && a % tiles == 0u && e % tiles == 0u;
        const uint32_t nqx = whole ? (e - a) / tiles : 0u;
        if (whole && nqx > 1u && tiles > PRE_TB) ++whole_shares;   // shares the blocks reorder
        const uint32_t TB = tiles < PRE_TB ? tiles : PRE_TB;
        uint32_t prev_block = 0;
        for (uint32_t it = a; it < e; ++it) {
            const uint32_t m = pre_item_order(it, a, e, tiles);
            ++checks;
            if (m < a || m >= e || seen[m]) {
                std::printf("not one to one: nq=%u tiles=%u w=%u share %u item %u -> %u\n", nq, tiles, w, x, it, m);
                return false;
            }
            seen[m] = 1;
            if (!whole) {
                if (m != it) { std::printf("moved an item of a partial share: nq=%u tiles=%u\n", nq, tiles); return false; }
                continue;
            }
            const uint32_t t = (m - a) % tiles, blk = t / TB;
            if (blk < prev_block) { std::printf("blocks out of order: nq=%u tiles=%u w=%u\n", nq, tiles, w); return false; }
            prev_block = blk;
            // inside a block: the items of one query are consecutive and in tile order
            if (it > a) {
                const uint32_t mp = pre_item_order(it - 1u, a, e, tiles);
                const uint32_t tp = (mp - a) % tiles;
                const bool same_query = (mp - a) / tiles == (m - a) / tiles;
                if (tp / TB == blk && same_query && t != tp + 1u) {
                    std::printf("tiles out of order in a block: nq=%u tiles=%u\n", nq, tiles);
                    return false;
                }
            }
        }
        if (whole && nqx * tiles != e - a) return false;
    }
    for (uint32_t i = 0; i < total; ++i)
        if (!seen[i]) { std::printf("item %u never taken: nq=%u tiles=%u w=%u\n", i, nq, tiles, w); return false; }
    return true;
}

int main() {
    long checks = 0;
    const uint32_t ws[] = {1u, 2u, 4u, 8u, 16u};
    for (uint32_t w : ws)
        for (uint32_t nq = 1; nq <= 72; ++nq)
            for (uint32_t tiles = 1; tiles <= 70; ++tiles)
                if (!check(nq, tiles, w, checks)) return 1;
    const uint32_t big[][2] = {{4096u, 128u}, {4000u, 128u}, {512u, 129u}, {1666u, 31u}, {1024u, 37u}, {8u, 4096u},
                               {16u, 2049u}, {9994u, 7u}, {256u, 100u}};
    for (auto& s : big)
        for (uint32_t w : ws)
            if (!check(s[0], s[1], w, checks)) return 1;
    if (whole_shares == 0) { std::printf("no share of whole queries was reordered\n"); return 1; }
    std::printf("ok %ld items, %ld reordered shares\n", checks, whole_shares);
    return 0;
}
