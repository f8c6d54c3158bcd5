// Device-side data structures and the per-tile routine of the T-of-N threshold
// query over EWAH bitmaps (64-bit words), written for gfx950 (wave64, 160 KB LDS).
//
// One workgroup computes the output of one tile of TW consecutive uncompressed
// word positions (TW * 64 rows) over all N inputs:
//   1. segment location: per input, the per-tile locator built at registration
//      holds the marker whose run covers the tile start together with that
//      marker word, so the covering marker and the one covering the next tile
//      start bound the input's compressed words that touch the tile without
//      reading the stream (EWAH markers carry both the fill length and the
//      dirty-word count, so dirty runs are skipped without reading them --
//      Section 3.1);
//   2. classify / prune: inputs whose one-fill covers the whole tile and inputs
//      that can hold a one in the tile are counted; the three cases of RBMrg on
//      EWAH (Section 6.4) at tile granularity: >= T full one-fills -> all ones,
//      fewer than T non-empty inputs -> all zeros, else count.  The second case
//      is also applied per group of words: the number of inputs holding a
//      dirty word or a one-fill in the group bounds every row count there, so
//      groups whose bound is below T are all zeros and nothing is added there
//      (registration stores which words and which 4-word groups each input
//      touches; queries of up to 256 inputs take single words);
//   3. decode: short segments are walked by one lane (eight words per read);
//      long ones are cut into 64-word windows aligned to the compressed
//      stream, listed in LDS and shared out among the wavefronts, each window
//      decoded by one wavefront: the skip index gives the window's marker mask
//      (built at registration by following the marker chain next = p + 1 + K)
//      and the position of its first word, and a wavefront prefix scan of the
//      words' spans (L for a marker, 1 for a dirty word) gives every word's
//      uncompressed position;
//   4. count: dirty words are added into a bit-sliced per-row counter in LDS
//      (planes A_1..A_P, least significant first, as in the bit-sliced index of
//      Section 5.3.1) with an atomic ripple-carry add (ScanCount with bit-sliced
//      counters, Section 5.1); inputs whose dirty run covers the whole tile go
//      through a dense carry-save-adder (Harley-Seal) tree in registers, one
//      lane per word position; one-fills are counted per position through a
//      difference array;
//   5. compare: per word position, the bit-sliced count is compared with
//      T' = T - (number of one-fills at that position) (greater-than-or-equal,
//      cf. the comparison step of BSTM, Section 5.3.1);
//   6. encode: canonical EWAH by scan-and-compact.  Each tile writes its words
//      at local output indices to a staging area and publishes its run
//      structure as an associative aggregate; no tile waits for another.  A
//      placement pass then scans the aggregates of each query (exclusive prefix
//      per tile), moves every tile's words to their final index and writes the
//      markers of runs that span tiles (closed by the tile that holds the next
//      marker).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ewt {

#ifndef EWT_TILE_WORDS
#define EWT_TILE_WORDS 512        // compile-time tile width (host and device must agree)
#endif
constexpr int TW = EWT_TILE_WORDS;    // tile width in uncompressed 64-bit words (= locator granularity)
constexpr int BLOCK = EWT_TILE_WORDS; // threads per workgroup (one per word position of a tile)
constexpr int NWAVES = BLOCK / 64;
// Presence records (upper bounds on row counts): which groups of rows of a tile an
// input can hold a one in.  Two kinds are kept: fine records (quarters of a word, 16 rows,
// then 8-row groups for the words the quarters leave in play), used by queries of up to
// 256 inputs, and groups of 4 words, used by wider queries.  Either way the tile routine
// prunes whole words (NG_FINE groups of one word).
constexpr int GW_COARSE = 4;
constexpr int NG_FINE = TW;                   // groups per tile, single words
constexpr int NG_COARSE = TW / GW_COARSE;     // groups per tile, 4-word groups
constexpr int PV_COARSE = NG_COARSE / 128;   // 16-byte 4-word-group records per tile and bitmap
constexpr int PMW_MAX = NG_FINE / 32;         // 32-bit words of the largest group mask
constexpr int NQ_TILE = 4 * TW;               // quarter-word groups per tile
constexpr int NO_TILE = 8 * TW;               // 8-row groups per tile
// Fine presence records of a bitmap of `tiles` tiles: four arrays side by side, each holding the
// tiles in order, so that neighbouring tiles' parts lie next to each other:
//   per-word bits, PQ_W_TILE words per tile from word 0 (bit w: word w of the tile holds a one);
//   quarter bits, PQ_Q_TILE words per tile from pq_quarters(tiles) (bit 4w + j: rows
//   [16j, 16j + 16) of word w hold a one);
//   8-row bits of half h = 0, 1, PQ_O_TILE words per tile from pq_octets(tiles, h) (word l,
//   bit 8i + j: rows [8j, 8j + 8) of word 8l + 4h + i hold a one).
constexpr uint32_t PQ_W_TILE = TW / 32;
constexpr uint32_t PQ_Q_TILE = NQ_TILE / 32;
constexpr uint32_t PQ_O_TILE = NO_TILE / 64;
__host__ __device__ inline uint32_t pq_quarters(uint32_t tiles) { return (tiles * PQ_W_TILE + 31u) & ~31u; }
__host__ __device__ inline uint32_t pq_octets(uint32_t tiles, uint32_t h) {
    return pq_quarters(tiles) + tiles * PQ_Q_TILE + h * tiles * PQ_O_TILE;
}
__host__ __device__ inline uint32_t pq_words(uint32_t tiles) { return pq_octets(tiles, 2u); }
static_assert(PQ_Q_TILE % 32 == 0 && PQ_O_TILE % 32 == 0, "quarter and 8-row parts on 128-byte lines");
static_assert(TW % 512 == 0 && NG_FINE <= BLOCK, "presence groups per tile");
constexpr int CHUNK = 64;         // compressed words per skip-index entry (one wavefront)
constexpr int MAXP = 12;          // bit planes: inputs per query < 2^12 (LDS budget)
constexpr uint32_t MAXN = (1u << MAXP) - 1;

// Registered bitmap as seen by the kernels (56 bytes).
struct BitmapDev {
    const uint64_t* words;   // EWAH stream, zero-padded to a multiple of CHUNK words plus CHUNK more
                             // (reads up to CHUNK words past the end stay inside the allocation)
    const uint4* loc;        // tiles + 1 entries: {marker index, its run start, marker word lo, hi}
                             // for the marker whose run covers the tile start
    const uint4* desc;       // per CHUNK words c: {bit j set iff word 64c + j is a marker (lo, hi),
                             // uncompressed position where word 64c's coverage starts, 0}
    uint32_t n_words;
    uint32_t U;              // uncompressed words
    const uint4* pres;       // per tile PV_COARSE records: bit g set iff words [4g, 4g + 4) of the
                             // tile hold a dirty word or a one-fill (the input can contribute there)
    const uint32_t* presq;   // fine presence records, pq_words(tiles) words (layout at pq_quarters):
                             // a word, quarter or 8-row group holds a one where a one-fill covers it
                             // or a dirty word has a nonzero bit there
    const uint16_t* qcnt;    // per tile: how many quarter-word groups of the tile hold a one (the
                             // tiles of a bitmap side by side, so neighbouring tiles share lines)
};

// Associative run-structure aggregate of a range of output words (see encode step).
struct Agg {
    uint32_t n;        // emitted compressed words, first word counted as a head if it is a fill
    uint32_t lh_pos;   // position of the last head (marker) in the range
    uint32_t lh_out;   // its output index relative to the range's first output word
    uint32_t bits;     // cf | cl << 2 | has_head << 4 | last head fill bit << 5
};

// Published aggregates of one (query, tile), 64 bytes.  Each 64-bit word
// carries the 16-bit tag of the launch that wrote it in its low bits, so a
// reader validates every word on its own (no fences: relaxed agent-scope
// atomics) and words left over from earlier launches are never mistaken for
// current ones.  Tags cycle through 1..65535; the host clears the states when
// they wrap.
struct TileState {
    uint64_t local[3];    // aggregate of this tile alone
    uint64_t incl[3];     // single queries: aggregate of tiles 0..t (look-back); batches: of tiles
                          // 0..t-1, written by the placement scan
    uint64_t head[2];     // first two heads of the tile: position | local output index << 32;
                          // bits 16..17 of head[1]: number of heads, at most 2
    uint64_t blk[3];      // single queries, tiles t = 64 k + 63 only: aggregate of the block of
                          // tiles 64 k .. 64 k + 63 (look-back across blocks)
    uint64_t pad;
};

// Output predicate of a query, a function f of the row count (a symmetric Boolean
// function of the N input bits, Section 2 and Section 3.2).
enum : uint32_t {
    PRED_THRESHOLD = 0,   // count >= T
    PRED_INTERVALS = 1,   // count in one of the n_iv intervals [iv[2j], iv[2j + 1]]
    PRED_ODD = 2,         // count odd (XOR of the inputs)
    PRED_EVEN = 3,        // count even
    PRED_MAXCOUNT = 4,    // no output: the largest row count goes to *acc (atomic maximum)
    PRED_HIST = 5,        // no output: acc[c] += rows of count c, for c = 1..N (count histogram)
    PRED_TABLE = 6,       // any f: bit c of tab is f(c), c = 0..N
};
constexpr int MAX_IV = 8;

// Predicate of a query other than a plain threshold (device memory).
struct PredDev {          // 96 bytes
    uint32_t kind;        // PRED_*
    uint32_t n_iv;        // PRED_INTERVALS: sorted, disjoint intervals of counts giving 1
    uint32_t tz;          // every count below tz gives v0
    uint32_t v0;
    uint32_t iv[2 * MAX_IV];
    unsigned long long* acc;   // PRED_MAXCOUNT: running maximum; else, if not null, receives
                               // the number of output rows (added)
    const uint32_t* tab;  // PRED_TABLE: (N + 32) / 32 words, bit c = f(c)
};
constexpr uint32_t TAB_WORDS = (MAXN + 32) / 32;   // words of the largest table (counts 0..MAXN)

struct QueryDev {         // 88 bytes
    const uint32_t* ids;  // N bitmap slots
    uint64_t* out;        // canonical EWAH output (device)
    uint64_t* out_n;      // output length (device)
    TileState* state;     // tiles entries
    uint64_t* stage;      // tiles * STAGE_WORDS words: each tile's output before placement
    uint64_t cap;         // output capacity in words
    uint32_t N, T, U, tiles;
    uint32_t tail_bits;   // n_bits % 64
    uint32_t variant;     // VAR_* flags
    const PredDev* pd;    // null: count >= T
    const BitmapDev* bms; // batches: the N inputs' descriptors in query order (null: table[ids[k]])
};
static_assert(sizeof(QueryDev) % 8 == 0, "query records are copied as 64-bit words");

// Variant flags (kernel strategy knobs; results never depend on them).
enum : uint32_t {
    VAR_DENSE = 1u << 0,        // whole-tile dirty runs through the register CSA tree
    VAR_WALK_SHIFT = 8,         // bits 8..15: max compressed words for a one-lane walk
    VAR_LITWALK_SHIFT = 16,     // bits 16..23: max literal-block words for a one-lane loop
    VAR_LOOPED = 1u << 24,      // unary (saturating) per-row counter, for T <= planes_for(N)
    VAR_GATE_SHIFT = 25,        // bits 25..26: when the per-group bounds are counted (GATE_*)
    VAR_EXPLICIT = 1u << 31,    // set in every explicit code so that 0 can mean "default"
};
// Gate of the per-group bounds of a tile that is not settled by its run counts:
// counted when T exceeds 1.1 times the mean bound (default), always, never, or when T
// exceeds 1.5 times the mean bound.  Bounds only drop groups that cannot reach T, so
// every gate gives the same result.
enum : uint32_t { GATE_1_1 = 0, GATE_ALWAYS = 1, GATE_NEVER = 2, GATE_1_5 = 3 };

__host__ __device__ inline uint32_t var_make(bool dense, uint32_t walk, uint32_t litwalk, bool looped = false,
                                             uint32_t gate = GATE_1_1) {
    return VAR_EXPLICIT | (dense ? VAR_DENSE : 0u) | ((walk & 255u) << VAR_WALK_SHIFT) |
           ((litwalk & 255u) << VAR_LITWALK_SHIFT) | (looped ? VAR_LOOPED : 0u) | ((gate & 3u) << VAR_GATE_SHIFT);
}

__host__ __device__ inline int planes_for(uint32_t n) {
    int p = 1;
    while (p < MAXP && (n >> p) != 0) ++p;
    return p;
}

// Bit-sliced counts: word p * stride of `planes` holds bit p of the counts of the 64
// rows of a word (least significant plane first), as in the bit-sliced index of
// Section 5.3.1.  The rows whose count is at least x (the final comparison of BSTM,
// there against T - 1): from the top plane down, a row is greater once it has a 1
// where x has a 0 while all higher bits were equal, and equal while every bit matches.
__host__ __device__ __forceinline__ uint64_t sliced_ge(const uint64_t* planes, int stride, int P, int x) {
    if (x <= 0) return ~0ull;
    if (x >= (1 << P)) return 0ull;
    uint64_t gt = 0, eq = ~0ull;
    for (int p = P - 1; p >= 0; --p) {
        const uint64_t a = planes[p * stride];
        const uint64_t tb = ((x >> p) & 1) ? ~0ull : 0ull;
        gt |= eq & a & ~tb;
        eq &= ~(a ^ tb);
    }
    return gt | eq;
}

// Largest count among the rows of cand (0 if cand is empty): from the top plane down,
// keep the candidates holding a 1 whenever any does.
__host__ __device__ __forceinline__ uint32_t sliced_max(const uint64_t* planes, int stride, int P, uint64_t cand) {
    uint32_t m = 0;
    for (int p = P - 1; p >= 0; --p) {
        const uint64_t tb = cand & planes[p * stride];
        if (tb) { cand = tb; m |= 1u << p; }
    }
    return m;
}

// Count of row r (0..63) read back from the planes.
__host__ __device__ __forceinline__ uint32_t sliced_row(const uint64_t* planes, int stride, int P, uint32_t r) {
    uint32_t c = 0;
    for (int p = 0; p < P; ++p) c |= (uint32_t)((planes[p * stride] >> r) & 1ull) << p;
    return c;
}

// The unary counter keeps one level per count 1..T in the planes' storage, so it
// applies when T fits there; otherwise the binary counter runs (same result).
__host__ __device__ inline bool use_looped(uint32_t variant, uint32_t N, uint32_t T) {
    return (variant & VAR_LOOPED) && T >= 1u && (int)T <= planes_for(N);
}

constexpr int WCAP = 2 * BLOCK;   // cooperative windows listed in LDS per round
constexpr int MISC_WORDS = 128;   // LDS counters and scratch of the tile routine

// Batched launches: work state of WORK_WORDS words.  work[1] = epoch; the item
// counter of XCD x at work[WORK_CTR + WORK_STRIDE * x] (one 64-byte line each); with the
// bounds pre-pass, the lengths of the front part (items of queries of at least 128 inputs) and
// the back part (the others) of XCD x's list of items left to the tile routine at
// work[WORK_LIST + WORK_STRIDE * x] and the word after it.  Item i belongs to XCD i * NXCD / total.
constexpr int NXCD = 8;           // XCDs of the MI355X
constexpr int WORK_CTR = 16, WORK_STRIDE = 16;
constexpr int WORK_LIST = WORK_CTR + WORK_STRIDE * NXCD;
constexpr int WORK_WORDS = WORK_LIST + WORK_STRIDE * NXCD;
constexpr int STAGE_WORDS = TW + 8;   // staged output words per tile (at most TW + 1 are used)

// Bounds pre-pass of a batched launch: per item (query, tile) one result word and a word mask
// of PRE_MASK_WORDS words (bit w: every row count of word w of the tile is below T).
enum : uint32_t {
    PRE_NONE = 0,      // not evaluated (queries of more than PCAP_FINE inputs, trivial T): the tile
                       // routine takes its own count bounds
    PRE_SETTLED = 1,   // every row count of the tile is below T: its aggregate is published
    PRE_OPEN = 2,      // evaluated, no word pruned (or the gate kept the records unread)
    PRE_MASK = 3,      // evaluated, the words of the mask are pruned
};
constexpr int PRE_MASK_WORDS = TW / 32;
constexpr uint32_t CLAIM_ITEMS = 4;   // items a workgroup of the batched launch claims at once

// Order in which the bounds pre-pass takes the items of one XCD's share [a, e) of a batch whose
// queries all have `tiles` tiles: a share of whole queries goes in blocks of PRE_TB tiles, block 0
// of every query of the share, then block 1, and so on (the last block may be shorter); any other
// share in item order.  Maps the share onto itself one to one; it is in [a, e).
constexpr uint32_t PRE_TB = 16u;   // measured best between 1 and 128
__host__ __device__ inline uint32_t pre_item_order(uint32_t it, uint32_t a, uint32_t e, uint32_t tiles) {
    if (tiles <= 1u || a % tiles != 0u || e % tiles != 0u) return it;
    const uint32_t nqx = (e - a) / tiles, l = it - a;   // queries of the share, rank in it
    const uint32_t TB = tiles < PRE_TB ? tiles : PRE_TB;
    const uint32_t B = l / (nqx * TB), r = l - B * nqx * TB;   // block, rank inside it
    const uint32_t tb = tiles - B * TB < TB ? tiles - B * TB : TB;
    return a + (r / tb) * tiles + B * TB + r % tb;
}

// LDS bytes needed by the tile routine for a query with N inputs.
__host__ __device__ inline size_t tile_smem_bytes(uint32_t N) {
    size_t P = (size_t)planes_for(N);
    size_t b = P * TW * 8;                 // count planes
    b += (TW + 8) * 4;                     // one-fill difference array (+ pad)
    b += (size_t)WCAP * 16;                // window list
    b += BLOCK * 8;                        // dense row pointers
    b += MISC_WORDS * 4;                   // misc counters / scan scratch / group mask
    return b;
}

// Slots of a threshold query of at most IDS_INLINE inputs travel in the kernel
// arguments (no upload before the launch); the kernel reads them where q.ids is null.
constexpr uint32_t IDS_INLINE = 256;
struct InlineIds {
    uint32_t v[IDS_INLINE];
};

// Host-side launchers (defined with the kernels).  ids: the slots when q.ids is null
// (threshold queries of at most IDS_INLINE inputs only).  launch_batch: every query of a batch
// has the same number of tiles (total / nq; the pre-pass orders its items by it).
hipError_t launch_query(const QueryDev& q, const BitmapDev* table, uint32_t* ticket, uint32_t epoch, uint32_t* err,
                        hipStream_t s, uint32_t pred_kind = PRED_THRESHOLD,   // kind of *q.pd
                        const InlineIds* ids = nullptr);
hipError_t launch_batch(const QueryDev* qs, const uint32_t* qtile, const uint32_t* tq, uint32_t nq, uint32_t total,
                        const BitmapDev* table, uint32_t* work, const uint32_t* epoch_ptr, uint32_t* err, uint32_t grid,
                        size_t smem, hipStream_t s,
                        uint32_t* item_t = nullptr,  // 2 * total words: per-item busy ticks of the tile routine, then
                                                     // of the pre-pass wavefront (null: not timed)
                        int win_batch = 6,    // windows per wavefront batch: 4..7
                        uint32_t* pre = nullptr,     // total words: bounds pre-pass results (null: none)
                        uint32_t* pmask = nullptr,   // total * PRE_MASK_WORDS words: its word masks
                        uint32_t* list = nullptr);   // total words: the items it leaves, listed per XCD
hipError_t launch_bump(uint32_t* work, hipStream_t s);   // epoch at work[1], counters cleared
hipError_t launch_zero_len(uint64_t* out_n, hipStream_t s);
hipError_t set_smem_limits(size_t max_bytes);
int batch_blocks_per_cu(size_t smem);   // resident workgroups of the batched kernel per CU
int pre_waves_per_cu();                  // resident wavefronts of the bounds pre-pass per CU
hipError_t launch_features(const QueryDev* qs, uint32_t nq, const float4* stats, float r, float* feat, hipStream_t s);
hipError_t launch_select(const float* pred, uint32_t nq, uint32_t n_arms, const uint32_t* codes, QueryDev* qs,
                         hipStream_t s);

}  // namespace ewt
