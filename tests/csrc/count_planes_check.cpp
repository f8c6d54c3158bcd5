// Exhaustive check of the kernels' bit-sliced count helpers on the host (the same
// functions the tile routine calls, built __host__ __device__): for every number of
// inputs N' = 1..1024 (P = bits needed to write N' planes), every count 0..N' and every
// threshold x from -1 to 2^P + 1,
//   * sliced_ge gives exactly the rows whose count is >= x (integer comparison);
//   * sliced_row reads every row's count back;
//   * sliced_max gives the largest count over candidate masks (all rows, one row,
//     random subsets, none).
// The counts are packed 64 to a word in bit-sliced form by plain integer code here.
#include <cstdint>
#include <cstdio>

#include "thr_device.h"

using ewt::planes_for;
using ewt::sliced_ge;
using ewt::sliced_max;
using ewt::sliced_row;

static uint64_t rng_state = 0x1402446614024466ull;
static uint64_t next_u64() {   // SplitMix64
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main() {
    long checks = 0;
    for (int n = 1; n <= 1024; ++n) {
        const int P = planes_for((uint32_t)n);
        if ((1 << P) <= n || (P > 1 && (1 << (P - 1)) > n)) {
            std::printf("FAIL planes_for(%d) = %d\n", n, P);
            return 1;
        }
        for (int c0 = 0; c0 <= n; c0 += 64) {
            // row r holds count c0 + r (rows past n repeat n)
            uint32_t cnt[64];
            uint64_t planes[12] = {};
            for (int r = 0; r < 64; ++r) {
                cnt[r] = (uint32_t)(c0 + r <= n ? c0 + r : n);
                for (int p = 0; p < P; ++p)
                    if ((cnt[r] >> p) & 1u) planes[p] |= 1ull << r;
            }
            for (int r = 0; r < 64; ++r) {
                if (sliced_row(planes, 1, P, (uint32_t)r) != cnt[r]) {
                    std::printf("FAIL sliced_row n=%d row count %u\n", n, cnt[r]);
                    return 1;
                }
            }
            for (int x = -1; x <= (1 << P) + 1; ++x) {
                uint64_t want = 0;
                for (int r = 0; r < 64; ++r)
                    if ((int)cnt[r] >= x) want |= 1ull << r;
                if (sliced_ge(planes, 1, P, x) != want) {
                    std::printf("FAIL sliced_ge n=%d counts from %d x=%d\n", n, c0, x);
                    return 1;
                }
                ++checks;
            }
            uint64_t masks[5] = {~0ull, 1ull << (next_u64() & 63), next_u64(), next_u64() & next_u64(), 0ull};
            for (uint64_t m : masks) {
                uint32_t want = 0;
                for (int r = 0; r < 64; ++r)
                    if (((m >> r) & 1ull) && cnt[r] > want) want = cnt[r];
                if (sliced_max(planes, 1, P, m) != want) {
                    std::printf("FAIL sliced_max n=%d counts from %d\n", n, c0);
                    return 1;
                }
                ++checks;
            }
        }
    }
    // strided planes, as the tile routine reads them from LDS (plane p at p * stride)
    uint64_t lds[12 * 8] = {};
    for (int p = 0; p < 12; ++p) lds[p * 8 + 3] = next_u64();
    uint64_t packed[12];
    for (int p = 0; p < 12; ++p) packed[p] = lds[p * 8 + 3];
    for (int x = 0; x < 4097; x += 7)
        if (sliced_ge(lds + 3, 8, 12, x) != sliced_ge(packed, 1, 12, x)) {
            std::printf("FAIL strided sliced_ge x=%d\n", x);
            return 1;
        }
    std::printf("ok %ld checks\n", checks);
    return 0;
}
