// Tile routine and kernels of the T-of-N threshold query (see thr_device.h for
// the step-by-step description and the paper passages each step follows).
#include "thr_device.h"

namespace ewt {

// Pointers read from the device-side bitmap table or query records are
// generic (flat) pointers; flat accesses may alias LDS, which makes the
// compiler wait for every load before the next LDS operation.  All global
// accesses go through the global address space explicitly.
#if defined(__HIP_DEVICE_COMPILE__)
#define EWT_GLOBAL __attribute__((address_space(1)))
#else
#define EWT_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ EWT_GLOBAL T* gp(T* p) {
    return (EWT_GLOBAL T*)p;
}

// ------------------------------------------------------------ wave helpers

// Inclusive prefix sum across the 64 lanes with DPP row shifts and row
// broadcasts (no LDS traffic): shifts by 1, 2, 4, 8 inside each row of 16
// lanes, then lane 15 of each row is added to the next row and lane 31 to the
// upper two rows.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) { return wave_incl_scan_dpp(v); }

// Sum over aligned groups of G consecutive lanes (G = 4, 8, 16, 32 or 64), left in
// the group's last lane: windowed shifts inside each row of 16 lanes (a window of G
// lanes after log2 G shifts), then row broadcasts join the rows of a group.
template <int G>
__device__ __forceinline__ uint32_t group_sum_dpp(uint32_t v) {
    static_assert(G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group of lanes");
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    if (G >= 8) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    if (G >= 16) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    if (G >= 32) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    if (G >= 64) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

// Exclusive scan over the workgroup; tmp needs NWAVES + 1 words.  All threads must call.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t& total) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t incl = wave_incl_scan(v);
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        uint32_t x = lane < NWAVES ? tmp[lane] : 0u;
        uint32_t xi = wave_incl_scan(x);
        if (lane < NWAVES) tmp[lane] = xi - x;
        if (lane == NWAVES - 1) tmp[NWAVES] = xi;
    }
    __syncthreads();
    uint32_t r = tmp[wave] + incl - v;
    total = tmp[NWAVES];
    __syncthreads();
    return r;
}

// Atomic ripple-carry add of one dirty word into the bit-sliced per-row counter:
// plane p holds bit p of every row's count.  Each atomic XOR returns the plane's
// previous value, whose AND with the incoming bits is the carry into plane p + 1;
// concurrent adds to one position serialise per plane, so the counts stay exact.
//
// Unary counter (LOOPED, the per-word form of the Looped recurrence, Section 6.2):
// level j holds the rows whose count has reached j + 1, for j < T.  An atomic OR
// into level j returns its previous value; the rows already there pass on to level
// j + 1 (a count that reaches T stays there).  The final levels do not depend on the
// order of the adds, so concurrent adds need no other ordering.
template <bool LOOPED>
__device__ __forceinline__ uint64_t plane_add(uint64_t* planes, uint32_t p, uint32_t pos, uint64_t v) {
    if constexpr (LOOPED) return atomicOr((unsigned long long*)&planes[p * TW + pos], (unsigned long long)v);
    else return atomicXor((unsigned long long*)&planes[p * TW + pos], (unsigned long long)v);
}

template <bool LOOPED>
__device__ __forceinline__ void ripple_add(uint64_t* planes, uint32_t pos, uint64_t v, int P) {
    for (int p = 0; p < P && v; ++p) {
        uint64_t old = plane_add<LOOPED>(planes, (uint32_t)p, pos, v);
        v &= old;
    }
}

// Carry-save adder: l = a ^ b ^ c (sum), h = majority(a, b, c) (carry).
#define EWT_CSA(h, l, a, b, c)                    \
    do {                                          \
        uint64_t u_ = (a) ^ (b);                  \
        uint64_t c_ = (c);                        \
        h = ((a) & (b)) | (u_ & c_);              \
        l = u_ ^ c_;                              \
    } while (0)

// ------------------------------------------------------ run-structure aggregate

__device__ __forceinline__ Agg agg_combine(const Agg& A, const Agg& B, uint32_t bstart) {
    uint32_t bcf = B.bits & 3u, acl = (A.bits >> 2) & 3u;
    uint32_t merge = (bcf != 2u && acl == bcf) ? 1u : 0u;
    Agg R;
    R.n = A.n + B.n - merge;
    bool bh = (B.bits >> 4) & 1u;
    if (bh && !(merge && B.lh_pos == bstart)) {
        R.lh_pos = B.lh_pos;
        R.lh_out = A.n + B.lh_out - merge;
        R.bits = (A.bits & 3u) | (B.bits & 0xCu) | (1u << 4) | (B.bits & (1u << 5));
    } else {
        R.lh_pos = A.lh_pos;
        R.lh_out = A.lh_out;
        R.bits = (A.bits & 3u) | (B.bits & 0xCu) | (A.bits & (3u << 4));
    }
    return R;
}

// Tagged publication: word 0 = tag | n << 16 | bits << 48, word 1 = tag |
// lh_pos << 16, word 2 = tag | lh_out << 16.
__device__ __forceinline__ void agg_publish(EWT_GLOBAL uint64_t* dst, const Agg& a, uint32_t tag) {
    const uint64_t t = tag & 0xFFFFu;
    __hip_atomic_store(&dst[0], t | ((uint64_t)a.n << 16) | ((uint64_t)(a.bits & 63u) << 48), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&dst[1], t | ((uint64_t)a.lh_pos << 16), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&dst[2], t | ((uint64_t)a.lh_out << 16), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Reads a published aggregate; false if any of its words is not from this launch.
__device__ __forceinline__ bool agg_fetch(EWT_GLOBAL uint64_t* src, uint32_t tag, Agg& a) {
    const uint64_t w0 = __hip_atomic_load(&src[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t w1 = __hip_atomic_load(&src[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t w2 = __hip_atomic_load(&src[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t = tag & 0xFFFFu;
    a.n = (uint32_t)(w0 >> 16);
    a.bits = (uint32_t)(w0 >> 48) & 63u;
    a.lh_pos = (uint32_t)(w1 >> 16);
    a.lh_out = (uint32_t)(w2 >> 16);
    return (w0 & 0xFFFFu) == t && (w1 & 0xFFFFu) == t && (w2 & 0xFFFFu) == t;
}

// ------------------------------------------------------------ segment location

struct Seg {
    uint32_t fa, fb;      // one-fill of the covering marker, clipped to the tile (absolute), empty if fa >= fb
    uint32_t a_lit, cnt;  // its dirty words inside the tile: compressed start, count
    uint32_t la;          // position of the first of them
    uint32_t bs, be;      // later markers touching the tile: compressed range, bs is a marker
    uint32_t y0;          // run start of the marker at bs
    bool onefull, zero;
};

// Segment of one input inside tile t from the locator entries of tiles t and
// t + 1 alone (they carry the covering marker words).
__device__ __forceinline__ Seg locate(const BitmapDev& B, uint32_t t, uint32_t tS, uint32_t tE, uint32_t tiles) {
    Seg s;
    const bool has_next = t + 1 < tiles;
    // both entries loaded without a branch (entry `tiles` is the end record, always present)
    const uint4 l0 = gp(B.loc)[t];
    const uint4 l1 = gp(B.loc)[t + 1];
    const uint32_t pm = l0.x, um = l0.y;
    const uint32_t f = l0.z & 1u, L = (l0.z >> 1) | (l0.w << 31), K = l0.w >> 1;
    const uint32_t fa = max(um, tS), fb = min(um + L, tE);
    s.fa = fa; s.fb = (f && fa < fb) ? fb : fa;
    const uint32_t la = max(um + L, tS), lb = min(um + L + K, tE);
    s.cnt = la < lb ? lb - la : 0u;
    s.la = la;
    s.a_lit = pm + 1u + (la - (um + L));
    s.bs = pm + 1u + K;
    s.y0 = um + L + K;
    // selects rather than branches, so that neither load is sunk into a branch and issued
    // after an earlier wait
    const uint32_t L2 = (l1.z >> 1) | (l1.w << 31), K2 = l1.w >> 1;
    const uint32_t lit_start = l1.y + L2;
    const uint32_t inlit = tE > lit_start ? min(K2, tE - lit_start) : 0u;
    const uint32_t be_next = l1.x != pm ? l1.x + 1u + inlit : s.bs;
    const uint32_t be_last = s.bs < B.n_words ? B.n_words : s.bs;
    s.be = has_next ? be_next : be_last;
    s.onefull = f && fa == tS && fb == tE;
    s.zero = (s.fa >= s.fb) && s.cnt == 0 && s.be <= s.bs;
    return s;
}

// Groups of a tile whose count bound is below T: bit g of the ng-bit mask in LDS
// (words at w; group g covers the words [g << sh, (g + 1) << sh) of the tile), read
// only where some group is pruned.
struct PMask {
    const uint32_t* w;
    uint32_t sh, ng;
    bool on;
    __device__ bool any() const { return on; }
};
__device__ __forceinline__ bool pruned_at(const PMask& pm, uint32_t rel);

// One lane decodes the compressed words [bs, be) (bs is a marker whose run
// starts at y0) and adds whatever falls inside [tS, tE).  Words are read eight
// at a time; streams are padded so reads up to CHUNK words past the end stay
// inside the allocation.
template <bool LOOPED>
__device__ __forceinline__ void walk_lane(const EWT_GLOBAL uint64_t* words, uint32_t bs, uint32_t be, uint32_t y0,
                                          uint32_t tS, uint32_t tE, uint64_t* planes, int32_t* diff, int P,
                                          const PMask& pm) {
    const bool prune = pm.any();
    uint32_t nm = bs;    // index of the next marker
    uint32_t u = y0;     // run start of the next marker
    uint32_t lb = 0;     // the dirty word at index j sits at position lb + j (mod 2^32)
    for (uint32_t g0 = bs; g0 < be; g0 += 8u) {
        uint64_t w[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = words[g0 + (uint32_t)i];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t j = g0 + (uint32_t)i;
            if (j < be) {
                if (j == nm) {
                    const uint64_t h = w[i];
                    const uint32_t L = (uint32_t)((h >> 1) & 0xFFFFFFFFu), K = (uint32_t)(h >> 33);
                    if (h & 1ull) {
                        const uint32_t fa = max(u, tS), fb = min(u + L, tE);
                        if (fa < fb) { atomicAdd(&diff[fa - tS], 1); atomicAdd(&diff[fb - tS], -1); }
                    }
                    lb = u + L - (j + 1u);
                    nm = j + 1u + K;
                    u += L + K;
                } else {
                    const uint32_t pos = lb + j;
                    if (pos >= tS && pos < tE && !(prune && pruned_at(pm, pos - tS))) ripple_add<LOOPED>(planes, pos - tS, w[i], P);
                }
            }
        }
    }
}

// One lane adds cnt consecutive dirty words starting at compressed index a,
// the first at tile-relative position p0.
template <bool LOOPED>
__device__ __forceinline__ void lit_lane(const EWT_GLOBAL uint64_t* words, uint32_t a, uint32_t cnt, uint32_t p0,
                                         uint64_t* planes, int P, const PMask& pm) {
    const bool prune = pm.any();
    for (uint32_t g0 = 0; g0 < cnt; g0 += 8u) {
        uint64_t w[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = words[a + g0 + (uint32_t)i];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (g0 + (uint32_t)i < cnt && !(prune && pruned_at(pm, p0 + g0 + (uint32_t)i)))
                ripple_add<LOOPED>(planes, p0 + g0 + (uint32_t)i, w[i], P);
    }
}

// Per-lane select by a wave-uniform lane mask held in scalar registers:
// bit `lane` of mask set -> b, else a (one v_cndmask with the mask as its
// condition operand).  The mask is passed through readfirstlane, which costs
// nothing where it already sits in scalar registers and keeps the operand a
// scalar pair where the compiler cannot prove it uniform.
__device__ __forceinline__ uint32_t lane_sel(uint64_t mask, uint32_t a, uint32_t b) {
    uint32_t r;
    mask = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(mask >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)mask);
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(mask));
    return r;
}
__device__ __forceinline__ uint64_t lane_sel64(uint64_t mask, uint64_t a, uint64_t b) {
    return ((uint64_t)lane_sel(mask, (uint32_t)(a >> 32), (uint32_t)(b >> 32)) << 32) |
           lane_sel(mask, (uint32_t)a, (uint32_t)b);
}
// Lanes [lo, hi) of a wavefront as a mask (0 <= lo < hi <= 64).
__device__ __forceinline__ uint64_t lane_range(uint32_t lo, uint32_t hi) {
    const uint64_t below_hi = hi >= 64u ? ~0ull : ((1ull << hi) - 1ull);
    return below_hi & (~0ull << lo);
}

// Reduces, in unit order, the aggregates held by the lanes of a wavefront: lane l holds
// unit base - l (a tile or a block of 64 tiles, unit u starting at word u * unit_words);
// `empty` lanes hold nothing and lie past the non-empty ones.  The result is broadcast.
__device__ __forceinline__ Agg wave_reduce_back(Agg v, bool empty, int base, uint32_t unit_words) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Agg o;
        o.n = __shfl_down(v.n, d, 64);
        o.lh_pos = __shfl_down(v.lh_pos, d, 64);
        o.lh_out = __shfl_down(v.lh_out, d, 64);
        o.bits = __shfl_down(v.bits, d, 64);
        const bool oe = __shfl_down((int)empty, d, 64) != 0 || lane + d >= 64;
        if ((lane & (2 * d - 1)) == 0 && !oe) {
            if (empty) { v = o; empty = false; }
            else v = agg_combine(o, v, (uint32_t)(base - lane - d + 1) * unit_words);
        }
    }
    Agg R;
    R.n = __shfl(v.n, 0, 64);
    R.lh_pos = __shfl(v.lh_pos, 0, 64);
    R.lh_out = __shfl(v.lh_out, 0, 64);
    R.bits = __shfl(v.bits, 0, 64);
    return R;
}

// Exclusive prefix of the run-structure aggregate over tiles [0, t), by decoupled
// look-back over two levels.  Round A reads the predecessors inside t's block of 64
// tiles (lane l: tile t - 1 - l); the nearest one that has published its inclusive
// prefix ends the search, the local aggregates of the tiles after it are reduced.  The
// block's last tile reads all 63 locals instead and publishes the block's aggregate.
// Round B then reads the earlier blocks, nearest first (lane l: block b - 1 - l, through
// the state of its last tile): an inclusive prefix there ends the search, otherwise the
// block aggregates are reduced.  A query of up to 4,096 tiles needs two rounds of loads,
// where one per 64 predecessors was needed before.  Tiles are taken in ticket order, so a
// tile only waits for states of tiles that started before it.  Called by one whole
// wavefront; A is the tile's own aggregate (its words start at tS).
__device__ Agg lookback(EWT_GLOBAL TileState* st, int t, const Agg& A, uint32_t tS, uint32_t epoch, uint32_t* err) {
    const int lane = __lane_id();
    const int p = t & 63, b = t >> 6;
    Agg acc;
    acc.n = 0; acc.lh_pos = 0; acc.lh_out = 0; acc.bits = 0;
    bool acc_empty = true;
    uint32_t spins = 0;
    if (p > 0) {   // round A: the block's earlier tiles
        const bool last = p == 63;   // reads every in-block local (no inclusive shortcut)
        while (true) {
            const int j = t - 1 - lane;
            const bool inb = lane < p;
            Agg vi, vl;
            bool inc = false, loc = false;
            if (inb) {
                inc = agg_fetch(st[j].incl, epoch, vi);
                loc = agg_fetch(st[j].local, epoch, vl);
            }
            const uint64_t incm = last ? 0ull : __ballot(inc);
            const int linc = incm ? (__ffsll((long long)incm) - 1) : 64;
            const bool need = inb && lane <= linc;
            const bool ok = !need || (lane == linc ? inc : loc);
            if (__ballot(!ok) != 0ull) {
                if (++spins > (1u << 22)) {
                    if (lane == 0) atomicOr(err, 1u);
                    return acc;
                }
                __builtin_amdgcn_s_sleep(2);
                continue;
            }
            Agg v;
            v.n = 0; v.lh_pos = 0; v.lh_out = 0; v.bits = 0;
            if (need) v = (lane == linc) ? vi : vl;
            acc = wave_reduce_back(v, !need, t - 1, (uint32_t)TW);
            acc_empty = false;
            if (last && lane == 0) agg_publish(st[t].blk, agg_combine(acc, A, tS), epoch);
            if (linc < 64 || b == 0) return acc;   // an inclusive prefix, or block 0 read whole
            break;
        }
    }
    // round B: earlier blocks, nearest first
    int bb = b - 1;
    while (true) {
        const int k = bb - lane;
        const int j = 64 * k + 63;
        Agg vi, vb;
        bool inc = false, blk = false;
        if (k >= 0) {
            inc = agg_fetch(st[j].incl, epoch, vi);
            blk = agg_fetch(st[j].blk, epoch, vb);
        }
        const uint64_t incm = __ballot(inc);
        const int linc = incm ? (__ffsll((long long)incm) - 1) : 64;
        const bool need = k >= 0 && lane <= linc;
        const bool ok = !need || (lane == linc ? inc : blk);
        if (__ballot(!ok) != 0ull) {
            if (++spins > (1u << 22)) {
                if (lane == 0) atomicOr(err, 1u);
                return acc;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        Agg v;
        v.n = 0; v.lh_pos = 0; v.lh_out = 0; v.bits = 0;
        if (need) v = (lane == linc) ? vi : vb;
        const Agg R = wave_reduce_back(v, !need, bb, 64u * (uint32_t)TW);
        acc = acc_empty ? R : agg_combine(R, acc, (uint32_t)(bb + 1) * 64u * (uint32_t)TW);
        acc_empty = false;
        if (linc < 64 || bb - 64 < 0) return acc;   // an inclusive prefix, or every block read
        bb -= 64;
    }
}

// ---------------------------------------------------------------- the tile

// Cooperative windows taken by one wavefront at a time (WB): all their loads are
// issued before any of them is decoded.  Single queries take WIN_BATCH; the batched
// kernel is built for WIN_BATCHES and the autotuner picks one per workload (more
// windows in flight against the registers they hold).
constexpr int WIN_BATCH = 7;

#ifdef EWT_PHASE_TIMING
// Debug builds only: per-tile timestamps of the phase boundaries.
__device__ uint64_t* ewt_phase_buf;
#define EWT_PHASE(k) do { if (threadIdx.x == 0 && ewt_phase_buf) ewt_phase_buf[(size_t)dbg_slot * 8 + (k)] = wall_clock64(); } while (0)
#else
#define EWT_PHASE(k) do { } while (0)
#endif

// Misc LDS slots.
enum { M_NDENSE = 1, M_PSUM = 2, M_ONEFULL = 4, M_NONZERO = 5, M_DFULL = 6, M_MAX = 7, M_TMP = 8, M_RMAX = 24, M_X = 32, M_TOT = 40, M_PR = 64 };
static_assert(M_PR + PMW_MAX <= MISC_WORDS, "misc slots");

// Presence group of tile-relative position rel is pruned (positions outside the
// tile are never pruned).
__device__ __forceinline__ bool pruned_at(const PMask& pm, uint32_t rel) {
    const uint32_t g = rel >> pm.sh;
    return g < pm.ng && ((pm.w[g >> 5] >> (g & 31u)) & 1u);
}

// Adds, for every 4-word group of the tile, the number of this wavefront's inputs
// (lanes with valid set) that touch it into cnt[g] (LDS).  pr: the input's
// PV_COARSE presence records.
__device__ __forceinline__ void count_presence(const uint4* pr, bool valid, uint32_t* cnt) {
    const int lane = __lane_id();
    if (__ballot(valid) == 0ull) return;
#pragma unroll
    for (int h = 0; h < NG_COARSE / 64; ++h) {   // 64 groups at a time
        const uint4 r = pr[h >> 1];
        const uint64_t m = !valid ? 0ull : (h & 1) ? ((uint64_t)r.w << 32 | r.z) : ((uint64_t)r.y << 32 | r.x);
        uint32_t c = 0;   // lane g holds the count of group 64 h + g
#pragma unroll 8
        for (int g = 0; g < 64; ++g) {
            const uint32_t a = (uint32_t)__popcll(__ballot((m >> g) & 1ull));
            c = lane == g ? a : c;
        }
        if (c) atomicAdd(&cnt[64 * h + lane], c);
    }
}

// Window list entry (16 bytes, one per 64-word window):
//   x, y  address of the window's first word; bits 16..31 of y hold flags:
//         bit 0 = aligned window of a marker-bearing range (else a block of
//         dirty words), bits 1..6 = first lane of the range inside the window,
//         bits 7..13 = end of the range inside the window;
//   z, w  aligned window: address of its skip-index entry;
//         dirty block: position of the first word (w unused).
// A dirty block is decoded as a window without markers whose first word sits
// at that position, so both kinds go through the same code.
constexpr uint32_t WF_ALIGNED = 1u;

__device__ __forceinline__ uint4 window_entry(const uint64_t* words, const uint4* desc, uint32_t bs, uint32_t be,
                                              uint32_t a_lit, uint32_t cnt, uint32_t la, uint32_t nlw, uint32_t i) {
    uint4 d;
    if (i < nlw) {
        const uint64_t a = (uint64_t)(uintptr_t)(words + a_lit + 64u * i);
        const uint32_t n = min(64u, cnt - 64u * i);
        d.x = (uint32_t)a;
        d.y = (uint32_t)(a >> 32) | ((n << 7) << 16);
        d.z = la + 64u * i;
        d.w = 0u;
    } else {
        const uint32_t c = bs / 64u + (i - nlw);
        const uint64_t a = (uint64_t)(uintptr_t)(words + 64u * c);
        const uint64_t e = (uint64_t)(uintptr_t)(desc + c);
        const uint32_t ra = max(bs, 64u * c) - 64u * c;
        const uint32_t rb = min(be, 64u * c + 64u) - 64u * c;
        d.x = (uint32_t)a;
        d.y = (uint32_t)(a >> 32) | ((WF_ALIGNED | (ra << 1) | (rb << 7)) << 16);
        d.z = (uint32_t)e;
        d.w = (uint32_t)(e >> 32);
    }
    return d;
}

// Reads the list entries of windows [w0, min(w0 + WIN_BATCH, we)) (lane g holds
// entry g), fetches the skip-index entries of aligned windows (lane g) and
// issues the data loads of all of them; empty slots read nothing and add nothing.
template <int WB>
__device__ __forceinline__ void issue_batch(const uint4* win, uint32_t w0, uint32_t we, int lane, const void* dummy,
                                            uint4& sk, uint32_t& dz, uint64_t& alm, uint64_t (&v)[WB],
                                            uint32_t (&fl)[WB]) {
    const uint32_t nb = min((uint32_t)WB, we - w0);
    uint4 d = make_uint4(0u, 0u, 0u, 0u);
    if ((uint32_t)lane < nb) d = win[w0 + (uint32_t)lane];
    // skip-index entry of an aligned window, loaded by every lane without a branch (lanes
    // of dirty blocks and empty slots read a valid dummy and are masked at decode: a dirty
    // block has no markers and its first word at position d.z).  No value of this batch is
    // used before the next decode, so nothing here waits for memory.
    const bool al = (uint32_t)lane < nb && ((d.y >> 16) & WF_ALIGNED);
    alm = __ballot(al);
    dz = d.z;
    const uint64_t sa = al ? (((uint64_t)d.w << 32) | d.z) : (uint64_t)(uintptr_t)dummy;
    sk = *(const EWT_GLOBAL uint4*)(uintptr_t)sa;
#pragma unroll
    for (int g = 0; g < WB; ++g) {
        v[g] = 0;
        fl[g] = 0;
        if ((uint32_t)g < nb) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)d.x, g);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)d.y, g);
            fl[g] = hi >> 16;
            const EWT_GLOBAL uint64_t* base =
                (const EWT_GLOBAL uint64_t*)(uintptr_t)(((uint64_t)(hi & 0xFFFFu) << 32) | lo);
            v[g] = __builtin_nontemporal_load(base + lane);
        }
    }
}

// Whether the query's predicate f takes one value v on every count in [lo, hi]
// (lo <= hi).  For the threshold this is the RBMrg case split (Section 6.4): lo >= T
// gives all ones, hi < T all zeros.
__device__ __forceinline__ bool pred_uniform(const QueryDev& q, uint32_t lo, uint32_t hi, uint32_t& v) {
    const PredDev* pd = q.pd;
    if (pd == nullptr || pd->kind == PRED_THRESHOLD) {
        if (lo >= q.T) { v = 1u; return true; }
        if (hi < q.T) { v = 0u; return true; }
        return false;
    }
    const uint32_t kind = pd->kind;
    if (kind == PRED_INTERVALS) {
        // the piece of f that holds lo: a gap before interval j, interval j, or the gap after
        // the last interval; f is constant on [lo, hi] iff hi stays in that piece
        uint32_t end = 0xFFFFFFFFu;
        v = 0u;
        const uint32_t n_iv = pd->n_iv;
        for (uint32_t j = 0; j < n_iv; ++j) {
            const uint32_t a = pd->iv[2 * j], b = pd->iv[2 * j + 1];
            if (lo < a) { end = a - 1u; break; }
            if (lo <= b) { v = 1u; end = b; break; }
        }
        return hi <= end;
    }
    if (kind == PRED_TABLE) {
        // constant iff the table's bits lo..hi are all equal to bit lo
        const EWT_GLOBAL uint32_t* tab = gp(pd->tab);
        v = (tab[lo >> 5] >> (lo & 31u)) & 1u;
        const uint32_t want = v ? ~0u : 0u;
        for (uint32_t w = lo >> 5; w <= (hi >> 5); ++w) {
            uint32_t m = ~0u;
            if (w == (lo >> 5)) m &= ~0u << (lo & 31u);
            if (w == (hi >> 5)) m &= (hi & 31u) == 31u ? ~0u : ((1u << ((hi & 31u) + 1u)) - 1u);
            if ((tab[w] ^ want) & m) return false;
        }
        return true;
    }
    // parity: constant only where every count is the same
    v = (lo & 1u) ^ (kind == PRED_EVEN ? 1u : 0u);
    return lo == hi;
}


// Per-group input counts from presence words staged in LDS word-major (word w of
// input k at w * pcap + k) for the first ns inputs.  QS lanes share a quad of groups
// (BLOCK = groups / 4 * QS), each counting every QS-th input.  A lane keeps the four
// counts in the bytes of one word: the quad's four bits are spread to bits 0, 8, 16
// and 24 by one multiply (x * (1 + 2^7 + 2^14 + 2^21): the shifted copies do not
// overlap) and added; a lane sees at most pcap / QS <= 64 inputs, so no byte
// overflows.  The counts are then widened to 16-bit halves and summed over the quad's
// lanes.
template <int QS>
__device__ __forceinline__ void count_quads(const uint32_t* prs, uint32_t pcap, uint32_t ns, uint32_t* gcnt) {
    const uint32_t tid = threadIdx.x;
    const uint32_t qd = tid / (uint32_t)QS, j = tid % (uint32_t)QS;
    const uint32_t* p32 = prs + (qd >> 3) * pcap;
    const uint32_t sh = (qd & 7u) * 4u;
    uint32_t c = 0;
#pragma unroll 4
    for (uint32_t k = j; k < ns; k += (uint32_t)QS) c += (((p32[k] >> sh) & 15u) * 0x00204081u) & 0x01010101u;
    // groups 0, 2 and 1, 3 of the quad; sums over the quad's lanes stay below 2^16
    const uint32_t c02 = group_sum_dpp<QS>(c & 0x00FF00FFu);
    const uint32_t c13 = group_sum_dpp<QS>((c >> 8) & 0x00FF00FFu);
    if (j == (uint32_t)QS - 1u) {
        gcnt[4 * qd] = c02 & 0xFFFFu;
        gcnt[4 * qd + 1] = c13 & 0xFFFFu;
        gcnt[4 * qd + 2] = c02 >> 16;
        gcnt[4 * qd + 3] = c13 >> 16;
    }
}

// Per-group bounds of a tile of a query of at most PCAP_FINE inputs, from its presence
// records (qptr[k]: input k's records, in LDS).  One pass: lane l of wavefront w adds record
// word off (the tile's part for lane l) of inputs w, w + 8, ... (32 groups; lanes with skip set read
// nothing and add zeros), eight records at a time through a carry-save-adder tree, into a
// bit-sliced counter of QP planes; the eight wavefronts' counters are summed through LDS
// (part: 7 * QP * 64 words) in three rounds, and wavefront 0 gets the groups whose sum is
// below tz.  All threads must call.
constexpr int QP = 9;

__device__ __forceinline__ void csa(uint32_t& h, uint32_t& l, uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t u = a ^ b;
    h = (a & b) | (u & c);
    l = u ^ c;
}

// Adds eight 32-bit masks into the bit-sliced counter c (QP planes): bit j of each mask adds
// one to the count of position j (a carry-save tree of the eight, then one ripple).
__device__ __forceinline__ void add8(uint32_t* c, const uint32_t* y) {
    uint32_t h1, l1, h2, l2, h3, l3, g1, m1;
    csa(h1, l1, y[0], y[1], y[2]);
    csa(h2, l2, l1, y[3], y[4]);
    csa(h3, l3, l2, y[5], y[6]);
    const uint32_t o = l3 ^ y[7], h4 = l3 & y[7];
    csa(g1, m1, h1, h2, h3);
    const uint32_t tw = m1 ^ h4, g2 = m1 & h4;
    const uint32_t f = g1 ^ g2, e = g1 & g2;
    // counter += o + 2 tw + 4 f + 8 e
    uint32_t cy = c[0] & o;
    c[0] ^= o;
    uint32_t u;
    u = c[1] ^ tw; { const uint32_t n = (c[1] & tw) | (u & cy); c[1] = u ^ cy; cy = n; }
    u = c[2] ^ f;  { const uint32_t n = (c[2] & f) | (u & cy); c[2] = u ^ cy; cy = n; }
    u = c[3] ^ e;  { const uint32_t n = (c[3] & e) | (u & cy); c[3] = u ^ cy; cy = n; }
#pragma unroll
    for (int p = 4; p < QP; ++p) {
        const uint32_t n = c[p] & cy;
        c[p] ^= cy;
        cy = n;
    }
}

// Positions whose count in the bit-sliced counter c is below tz, most significant plane first.
__device__ __forceinline__ uint32_t below(const uint32_t* c, uint32_t tz) {
    uint32_t gt = 0u, eq = ~0u;
#pragma unroll
    for (int p = QP - 1; p >= 0; --p) {
        const uint32_t tb = ((tz >> p) & 1u) ? ~0u : 0u;
        gt |= eq & c[p] & ~tb;
        eq &= ~(c[p] ^ tb);
    }
    return (tz >> QP) ? ~0u : ~(gt | eq);
}

__device__ __forceinline__ uint32_t bound_pass(const uint32_t* const* qptr, uint32_t N, uint32_t off, bool skip,
                                               uint32_t tz, uint32_t* part) {
    const int lane = __lane_id();
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t ni = N > wave ? (N - wave + 7u) / 8u : 0u;   // inputs of this wavefront (at most 32)
    uint32_t x[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) x[i] = 0u;
    // every record word is loaded before any is added
#pragma unroll
    for (int i = 0; i < 32; ++i)
        if ((uint32_t)i < ni && !skip) x[i] = gp(qptr[wave + 8u * (uint32_t)i])[off];
    uint32_t c[QP];
#pragma unroll
    for (int p = 0; p < QP; ++p) c[p] = 0u;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if ((uint32_t)(8 * g) >= ni) break;
        add8(c, x + 8 * g);
    }
    // wavefronts w + s add into w (s = 4, 2, 1), each round in its own part of the scratch
    uint32_t po = 0;
#pragma unroll
    for (uint32_t sft = 4; sft >= 1; sft >>= 1) {
        if (wave >= sft && wave < 2 * sft) {
#pragma unroll
            for (int p = 0; p < QP; ++p) part[po + ((wave - sft) * QP + (uint32_t)p) * 64u + (uint32_t)lane] = c[p];
        }
        __syncthreads();
        if (wave < sft) {
            uint32_t cy = 0;
#pragma unroll
            for (int p = 0; p < QP; ++p) {
                const uint32_t b = part[po + (wave * QP + (uint32_t)p) * 64u + (uint32_t)lane];
                const uint32_t u = c[p] ^ b;
                const uint32_t n = (c[p] & b) | (u & cy);
                c[p] = u ^ cy;
                cy = n;
            }
        }
        po += sft * QP * 64u;
    }
    return below(c, tz);   // groups below tz (wavefront 0 holds the sums)
}

// Word mask of a tile of a query of at most PCAP_FINE inputs, as bytes at pmw (byte l: words
// 8l .. 8l + 7, bit set: every row count of the word is below tz; words past nPos clear).
// First from the quarter records (16 rows per group); if that leaves words of the tile in
// play, the words still in play are bounded again from the 8-row records, which settles most
// of the tiles the quarters leave almost settled.  All threads must call.
__device__ __forceinline__ void fine_bounds(const uint32_t* const* qptr, uint32_t N, uint32_t tz, uint32_t nPos,
                                            uint32_t t, uint32_t tiles, uint32_t* part, uint32_t* pmw, uint32_t* flag) {
    const int lane = __lane_id();
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t w0 = 8u * (uint32_t)lane;
    const uint32_t vmask = (1u << (nPos > w0 ? min(nPos - w0, 8u) : 0u)) - 1u;   // words of this lane in the tile
    // pass 0: quarters (lane l holds quarters 32l .. 32l + 31, four per word); passes 1 and 2:
    // the 8-row groups of words w0 + 4h .. w0 + 4h + 3 (h = pass - 1), word l of half h of the
    // tile's 8-row bits, where some of those words are still in play
    uint32_t w8 = 0;
#pragma unroll 1
    for (uint32_t pass = 0; pass < 3; ++pass) {
        const uint32_t h = pass > 0 ? pass - 1u : 0u;
        const bool skip = pass > 0 && ((w8 | ~vmask) >> (4 * h) & 15u) == 15u;
        const uint32_t off = (pass == 0 ? pq_quarters(tiles) + t * PQ_Q_TILE : pq_octets(tiles, h) + t * PQ_O_TILE) +
                             (uint32_t)lane;
        const uint32_t lt = bound_pass(qptr, N, off, skip, tz, part);
        if (pass == 0) {
            uint32_t m = lt & (lt >> 1);
            m &= m >> 2;   // bit 4i: all four quarters of word w0 + i
#pragma unroll
            for (int i = 0; i < 8; ++i) w8 |= ((m >> (4 * i)) & 1u) << i;
            w8 &= vmask;
            // the words every lane's passes 1 and 2 start from (wavefront 0 holds the sums)
            if (wave == 0) {
                ((unsigned char*)pmw)[lane] = (unsigned char)w8;
                const bool open = __ballot(w8 != vmask) != 0ull;
                if (lane == 0) *flag = open ? 1u : 0u;
            }
            __syncthreads();
            if (*flag == 0u) return;   // nothing left in play (uniform: read from LDS after a barrier)
            w8 = ((const unsigned char*)pmw)[lane];
        } else {
            uint32_t m = lt & (lt >> 1);
            m &= m >> 2;
            m &= m >> 4;   // bit 8i: all eight 8-row groups of word w0 + 4h + i
#pragma unroll
            for (int i = 0; i < 4; ++i) w8 |= ((m >> (8 * i)) & 1u) << (4 * h + (uint32_t)i);
        }
    }
    if (wave == 0) ((unsigned char*)pmw)[lane] = (unsigned char)(w8 & vmask);
}

// Queries of up to PCAP_FINE inputs use the fine records (eight wavefronts take 32 inputs
// each in the bounds passes); wider ones stage the 4-word-group records of their first
// PCAP_COARSE inputs in the window list (16 * WCAP bytes).
constexpr uint32_t PCAP_FINE = 256u;
constexpr uint32_t PCAP_COARSE = (uint32_t)(WCAP / PV_COARSE);
static_assert((NG_COARSE / 4) * 16 == BLOCK, "lanes per quad of groups");
static_assert(PCAP_COARSE / 16 < 256u, "byte counters");
static_assert(PCAP_FINE < (1u << QP) && PCAP_FINE <= 8u * 32u, "quarter counts fit QP planes, 32 inputs per wavefront");
static_assert(7 * QP * 64 * 4 <= WCAP * 16, "quarter count scratch fits the window list");

// STAGED: the tile writes its words to the staging area and publishes its
// aggregate (a placement pass finishes the output); otherwise it finds the prefix
// over earlier tiles by look-back and writes its words in place.
// Descriptor of input k of a query: from the query's own copy (batches: one coalesced
// read) or through the slot table.
__device__ __forceinline__ BitmapDev input_of(const QueryDev& q, const BitmapDev* __restrict__ table, uint32_t k) {
    return q.bms ? gp(q.bms)[k] : gp(table)[gp(q.ids)[k]];
}

static_assert((MAXN + 1u) * 4u <= (uint32_t)WCAP * 16u, "count histogram must fit in the window list");

template <bool STAGED, bool GENERAL = false, bool MAXC = false, bool LOOPED = false, bool HIST = false,
          int WB = WIN_BATCH>
__device__ void process_tile(const QueryDev& q, const BitmapDev* __restrict__ table, uint32_t t,
                             uint32_t epoch, unsigned char* smem, uint32_t* err, uint32_t dbg_slot,
                             uint32_t pre = PRE_NONE, const uint32_t* pmask = nullptr) {
    (void)dbg_slot;   // timestamp slot of debug builds
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wavefront
    const uint32_t N = q.N, T = q.T, U = q.U, tiles = q.tiles;
    const uint32_t tS = t * (uint32_t)TW;
    const uint32_t nPos = min((uint32_t)TW, U - tS);
    const uint32_t tE = tS + nPos;
    const int P = planes_for(N);
    // levels the adds ripple through: bit planes, or count levels 1..T (unary; T <= P)
    const int PL = LOOPED ? (int)T : P;
    const uint32_t walk_max = (q.variant >> VAR_WALK_SHIFT) & 255u;
    const uint32_t litwalk_max = (q.variant >> VAR_LITWALK_SHIFT) & 255u;

    uint64_t* planes = (uint64_t*)smem;
    int32_t* diff = (int32_t*)(planes + (size_t)P * TW);
    uint4* win = (uint4*)(diff + TW + 8);
    const uint64_t** dense = (const uint64_t**)(win + WCAP);
    uint32_t* misc = (uint32_t*)(dense + BLOCK);

    EWT_PHASE(0);
    for (int i = tid; i < P * TW; i += BLOCK) planes[i] = 0;
    for (int i = tid; i < TW + 8; i += BLOCK) diff[i] = 0;
    // until the decode starts, the window list holds the 4-word-group records of the
    // first pcap inputs (word-major: word w of input k at w * pcap + k; wide queries) or
    // the wavefronts' partial counters of the bounds passes (fine records), and the
    // dense-row list the per-group counts (wide queries) or the inputs' fine records
    uint32_t* prs = (uint32_t*)win;
    uint32_t* gcnt = (uint32_t*)dense;
    const uint32_t** qptr = (const uint32_t**)dense;   // quarter records of the inputs (fine presence)
    if (tid < 8) misc[tid] = 0;
    if (tid < PMW_MAX) misc[M_PR + tid] = 0;
    // largest count: one read of the running maximum for the whole workgroup (other
    // workgroups raise it meanwhile; every wavefront must take the same early exit)
    if constexpr (MAXC && !HIST) {
        if (tid == 0) misc[M_RMAX] = (uint32_t)__hip_atomic_load(q.pd->acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();

    // ---- classify / prune (RBMrg on EWAH, cases 1 and 2, per tile)
    // f constant on every possible count (threshold: T = 0 or T > N)
    uint32_t tv = T == 0 ? 1u : 0u;
    bool trivial = (T == 0) || (T > N);
    if constexpr (GENERAL) trivial = pred_uniform(q, 0u, N, tv);
    // largest count: the running maximum over the tiles done so far bounds what is
    // worth counting (branch and bound); no tile is trivial
    uint32_t Rmax = 0;
    if constexpr (HIST) trivial = false;
    if constexpr (MAXC && !HIST) {
        trivial = false;
        Rmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)misc[M_RMAX]);   // the workgroup's one read
    }
    Seg seg;
    BitmapDev B0;
    // presence granularity: single words for queries of up to PCAP_FINE inputs, else
    // groups of 4 words
    const bool fine = N <= PCAP_FINE;
    const uint32_t gsh = fine ? 0u : 2u;   // log2 of the words per group
    const uint32_t ng = fine ? (uint32_t)NG_FINE : (uint32_t)NG_COARSE;
    const uint32_t pcap = fine ? PCAP_FINE : PCAP_COARSE;
    const uint32_t ngv = (nPos + (1u << gsh) - 1u) >> gsh;   // groups inside the tile
    // presence groups an input touching all of the tile has: quarters, or 4-word groups
    const uint32_t nfull = fine ? 4u * nPos : ngv;
    // word mask of the bounds pre-pass (stored with the classify step's counters)
    const uint32_t pmv = (pre == PRE_MASK && tid < PRE_MASK_WORDS) ? gp(pmask)[tid] : 0u;
    if (!trivial) {
        for (uint32_t kb = 0; kb < N; kb += BLOCK) {
            uint32_t k = kb + (uint32_t)tid;
            bool onefull = false, nonzero = false;
            uint32_t np = 0;
            if (k < N) {
                const BitmapDev B = input_of(q, table, k);
                // the presence count or record and both locator entries are loaded before
                // any is used, so the classify step waits for memory once
                const uint32_t* qr = B.presq;   // the tile's parts are found from t in the bounds step
                uint4 pr = make_uint4(0u, 0u, 0u, 0u);
                uint32_t qc = 0;
                static_assert(PV_COARSE == 1, "one 4-word-group record per tile");
                if (fine) {
                    if (pre == PRE_NONE) qc = gp(B.qcnt)[t];   // else the pre-pass took the bounds
                } else pr = gp(B.pres)[t];
                Seg s = locate(B, t, tS, tE, tiles);
                if (fine) {
                    // quarter counts; the records are read by the bounds step
                    np = qc;
                    qptr[k] = qr;
                } else {
                    np = (uint32_t)(__popc(pr.x) + __popc(pr.y) + __popc(pr.z) + __popc(pr.w));
                    if (k < pcap) {
                        prs[k] = pr.x;
                        prs[pcap + k] = pr.y;
                        prs[2 * pcap + k] = pr.z;
                        prs[3 * pcap + k] = pr.w;
                    }
                }
                onefull = s.onefull;
                nonzero = !s.zero;
                if (kb == 0) { seg = s; B0 = B; }
            }
            // one LDS atomic per wavefront and counter
            const uint32_t c1 = (uint32_t)__popcll(__ballot(onefull)), c2 = (uint32_t)__popcll(__ballot(nonzero));
            const uint32_t c3 = (uint32_t)__popcll(__ballot(np == nfull && k < N));
            const uint32_t c4 = wave_incl_scan(np);
            if (lane == 63) {
                if (c1) atomicAdd(&misc[M_ONEFULL], c1);
                if (c2) atomicAdd(&misc[M_NONZERO], c2);
                if (c3) atomicAdd(&misc[M_DFULL], c3);
                if (c4) atomicAdd(&misc[M_PSUM], c4);
            }
        }
    }
    if (pre == PRE_MASK && tid < PRE_MASK_WORDS) misc[M_PR + tid] = pmv;
    __syncthreads();
    EWT_PHASE(1);
    // every row count of the tile lies in [full one-fills, inputs that can hold a one]
    uint32_t mode = trivial ? (tv ? 1u : 2u)
                            : (misc[M_ONEFULL] >= T ? 1u : (misc[M_NONZERO] < T ? 2u : 0u));
    if constexpr (GENERAL) {
        uint32_t uv = 0;
        if (!trivial) mode = pred_uniform(q, misc[M_ONEFULL], max(misc[M_ONEFULL], misc[M_NONZERO]), uv) ? (uv ? 1u : 2u) : 0u;
        mode = (uint32_t)__builtin_amdgcn_readfirstlane((int)mode);   // uniform (it depends on LDS counters)
    }
    // per-group bounds: a group whose bound is below tz has every count below tz, where
    // f is v0 (for the threshold: below T, zero)
    uint32_t Tz = T, v0 = 0;
    if constexpr (GENERAL) {
        Tz = (uint32_t)__builtin_amdgcn_readfirstlane((int)q.pd->tz);
        v0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)q.pd->v0);
    }
    if constexpr (HIST) {
        // counts of zero are not tallied; a tile whose inputs that can hold a one are all
        // full one-fills has every row at that count
        const uint32_t lo = misc[M_ONEFULL], hi = misc[M_NONZERO];
        if (hi == 0) return;
        if (lo >= hi) {
            if (tid == 0) {
                const bool last = tS + nPos == U;
                const uint64_t rows = 64ull * nPos - ((last && q.tail_bits) ? 64ull - q.tail_bits : 0ull);
                atomicAdd(q.pd->acc + hi, (unsigned long long)rows);
            }
            return;
        }
        mode = 0u;
        Tz = 1u;   // groups no input touches hold counts of zero
    } else if constexpr (MAXC) {
        // every count of the tile is at most the number of inputs that can hold a one
        // there; if those are all full one-fills, every count equals it
        const uint32_t lo = misc[M_ONEFULL], hi = misc[M_NONZERO];
        if (hi <= Rmax) return;
        if (lo >= hi) {
            if (tid == 0) atomicMax(q.pd->acc, (unsigned long long)hi);
            return;
        }
        mode = 0u;
        Tz = Rmax + 1u;   // groups that cannot exceed the running maximum add nothing
    }
    // per-group bounds: counted only when fewer than T inputs touch every group and
    // T is above 11/10 of the mean bound (else few groups fall below T and the count costs more
    // than it saves)
    PMask pm;
    pm.w = misc + M_PR;
    pm.sh = gsh;
    pm.ng = ng;
    pm.on = false;
    const uint32_t gate = (q.variant >> VAR_GATE_SHIFT) & 3u;
    const uint64_t gnum = gate == GATE_1_5 ? 15ull : 11ull;
    if (pre != PRE_NONE) {
        pm.on = pre == PRE_MASK;   // bounds of the pre-pass (a tile it settled never gets here)
    } else if (mode == 0 && misc[M_DFULL] < Tz && gate != GATE_NEVER &&
               (gate == GATE_ALWAYS || 10ull * Tz * nfull > gnum * misc[M_PSUM])) {
        if (fine) fine_bounds(qptr, N, Tz, nPos, t, tiles, prs, misc + M_PR, misc + M_TMP);
        else count_quads<16>(prs, PCAP_COARSE, min(N, PCAP_COARSE), gcnt);
        if (N > pcap) {   // the rest of very wide queries (4-word groups): wavefront ballots
            __syncthreads();
            for (uint32_t kb = PCAP_COARSE; kb < N; kb += BLOCK) {
                const uint32_t k = kb + (uint32_t)tid;
                uint4 pr[PV_COARSE];
#pragma unroll
                for (int v = 0; v < PV_COARSE; ++v) pr[v] = make_uint4(0u, 0u, 0u, 0u);
                if (k < N) {
                    const uint4* src = gp(input_of(q, table, k).pres) + (size_t)t * PV_COARSE;
#pragma unroll
                    for (int v = 0; v < PV_COARSE; ++v) pr[v] = src[v];
                }
                count_presence(pr, k < N, gcnt);
            }
        }
        __syncthreads();
        if (!fine && (uint32_t)tid < ng) {
            const uint64_t m = __ballot(gcnt[tid] < Tz && (uint32_t)tid < ngv);
            if ((tid & 63) == 0) { misc[M_PR + 2 * (tid >> 6)] = (uint32_t)m; misc[M_PR + 2 * (tid >> 6) + 1] = (uint32_t)(m >> 32); }
        }
        __syncthreads();
        uint32_t npr = 0;
#pragma unroll
        for (int i = 0; i < PMW_MAX; ++i)
            if ((uint32_t)i < ng / 32u) npr += (uint32_t)__popc(misc[M_PR + i]);
        pm.on = npr != 0u;
        if (npr == ngv) mode = v0 ? 1u : 2u;
    }
    const bool prune = pm.any();

    // ---- settled batched tile: every output word of the tile is one fill, so its run
    // structure is known without compare and encode (one head at the tile's first word,
    // nothing staged; the placement pass writes the marker).  mode comes from LDS counters
    // read after the last barrier, the same for every wavefront, and the exit is taken
    // here, outside every loop that holds a barrier, so all wavefronts leave together.
    // An all-ones tile holding the last, partial word is excluded: that word is a literal.
    // Single threshold queries take the same exit: wavefront 0 publishes the aggregate,
    // looks back and writes the at most two marker words such a tile owns (closing the run
    // left open before it unless its fill continues that run; the last tile's marker).
    if constexpr (!GENERAL && !MAXC && !HIST) {
        const uint32_t umode = (uint32_t)__builtin_amdgcn_readfirstlane((int)mode);
        if (umode == 2u || (umode == 1u && !(tE == U && q.tail_bits))) {
            const uint32_t c = umode == 1u ? 1u : 0u;
            Agg A;
            A.n = 1;
            A.lh_pos = tS;
            A.lh_out = 0;
            A.bits = c | (c << 2) | (1u << 4) | (c << 5);
            EWT_GLOBAL TileState* st = gp(q.state);
            if constexpr (STAGED) {
                if (tid == 0) {
                    st[t].head[0] = 0ull;
                    st[t].head[1] = 1ull << 16;
                    agg_publish(st[t].local, A, epoch);
                }
                EWT_PHASE(7);
            } else if (wave == 0) {
                if (lane == 0) agg_publish(st[t].local, A, epoch);
                EWT_PHASE(6);
                Agg X;
                X.n = 0; X.lh_pos = 0; X.lh_out = 0; X.bits = 3u << 2;
                Agg I = A;
                if (t > 0) {
                    X = lookback(st, (int)t, A, tS, epoch, err);
                    I = agg_combine(X, A, tS);
                }
                if (lane == 0) {
                    agg_publish(st[t].incl, I, epoch);
                    const uint64_t cap = q.cap;
                    EWT_GLOBAL uint64_t* out = gp(q.out);
                    const bool merge = t > 0 && ((X.bits >> 2) & 3u) == c;
                    if (t > 0 && !merge) {   // this tile's head closes the run left open before it
                        const uint32_t K = X.n - X.lh_out - 1u;
                        const uint32_t L = (tS - X.lh_pos) - K;
                        if (X.lh_out < cap) out[X.lh_out] = ((X.bits >> 5) & 1u) | ((uint64_t)L << 1) | ((uint64_t)K << 33);
                    }
                    if (t == tiles - 1) {    // the last tile closes the last run
                        const uint32_t lpos = merge ? X.lh_pos : tS;
                        const uint32_t lout = merge ? X.lh_out : X.n;
                        const uint64_t lf = merge ? ((X.bits >> 5) & 1u) : c;
                        const uint32_t K = I.n - lout - 1u;
                        const uint32_t L = (U - lpos) - K;
                        if (lout < cap) out[lout] = lf | ((uint64_t)L << 1) | ((uint64_t)K << 33);
                        *gp(q.out_n) = I.n;
                    }
                }
                EWT_PHASE(7);
            }
            return;
        }
    }

    // ---- decode and count
    if (mode == 0) {
        for (uint32_t kb = 0; kb < N; kb += BLOCK) {
            const uint32_t k = kb + (uint32_t)tid;
            uint32_t nlw = 0, nww = 0;
            Seg s = {};
            const uint64_t* wp = nullptr;
            const uint4* dp = nullptr;
            if (k < N) {
                BitmapDev B = B0;
                if (kb != 0) B = input_of(q, table, k);
                s = (kb == 0) ? seg : locate(B, t, tS, tE, tiles);
                wp = B.words;
                dp = B.desc;
                if (s.fa < s.fb) { atomicAdd(&diff[s.fa - tS], 1); atomicAdd(&diff[s.fb - tS], -1); }
                if (s.cnt) {
                    if (!LOOPED && (q.variant & VAR_DENSE) && s.cnt == nPos) {
                        uint32_t j = atomicAdd(&misc[M_NDENSE], 1u);
                        dense[j] = wp + s.a_lit;
                    } else if (s.cnt <= litwalk_max) {
                        lit_lane<LOOPED>(gp(wp), s.a_lit, s.cnt, s.la - tS, planes, PL, pm);
                    } else {
                        nlw = (s.cnt + 63u) / 64u;
                    }
                }
                if (s.be > s.bs) {
                    if (s.be - s.bs <= walk_max) walk_lane<LOOPED>(gp(wp), s.bs, s.be, s.y0, tS, tE, planes, diff, PL, pm);
                    else nww = (s.be - 1u) / 64u - s.bs / 64u + 1u;
                }
            }
            EWT_PHASE(2);
            // window offsets of every input (block scan); the windows are then
            // listed and processed in rounds of at most WCAP
            uint32_t tot;
            const uint32_t off = block_excl_scan(nlw + nww, misc + M_TMP, tot);
            for (uint32_t j = off; j < min(off + nlw + nww, (uint32_t)WCAP); ++j)
                win[j] = window_entry(wp, dp, s.bs, s.be, s.a_lit, s.cnt, s.la, nlw, j - off);
            for (uint32_t W0 = 0; W0 < tot; W0 += (uint32_t)WCAP) {
                const uint32_t nr = min((uint32_t)WCAP, tot - W0);
                if (W0 > 0) {   // later rounds (long tiles): the segment is located again
                    const uint32_t j0 = max(off, W0), j1 = min(off + nlw + nww, W0 + nr);
                    if (j0 < j1) {
                        const BitmapDev B = input_of(q, table, k);
                        const Seg s2 = locate(B, t, tS, tE, tiles);
                        for (uint32_t j = j0; j < j1; ++j)
                            win[j - W0] = window_entry(B.words, B.desc, s2.bs, s2.be, s2.a_lit, s2.cnt, s2.la, nlw, j - off);
                    }
                }
                __syncthreads();

                // each wavefront takes a contiguous share of the round's windows
                const uint32_t wb = (nr * (uint32_t)wave) / NWAVES, we = (nr * (uint32_t)(wave + 1)) / NWAVES;
                // software pipeline: the loads of batch k + 1 are in flight while batch k
                // is added into the planes
                uint4 sk;
                uint32_t dz;
                uint64_t alm;
                uint64_t v[WB];
                uint32_t fl[WB];
                issue_batch(win, wb, we, lane, table, sk, dz, alm, v, fl);
                for (uint32_t w0 = wb; w0 < we; w0 += (uint32_t)WB) {
                    // decode, branch-free over the batch: position of every word (span = L
                    // for a marker, 1 for a dirty word)
                    uint32_t r[WB];
                    uint64_t x[WB], fills[WB], lit[WB];
                    uint32_t any_fill = 0;
                    // skip-index entries: aligned windows' loaded values, dirty blocks' defaults
                    const uint32_t skx = lane_sel(alm, 0u, sk.x), sky = lane_sel(alm, 0u, sk.y);
                    const uint32_t skz = lane_sel(alm, dz, sk.z);
#pragma unroll
                    for (int g = 0; g < WB; ++g) {
                        const uint32_t m0 = (uint32_t)__builtin_amdgcn_readlane((int)skx, g);
                        const uint32_t m1 = (uint32_t)__builtin_amdgcn_readlane((int)sky, g);
                        const uint32_t p0 = (uint32_t)__builtin_amdgcn_readlane((int)skz, g);
                        const uint64_t M = ((uint64_t)m1 << 32) | m0;
                        const uint64_t inr = lane_range((fl[g] >> 1) & 63u, (fl[g] >> 7) & 127u);
                        x[g] = v[g];
                        const uint32_t span = lane_sel(M, 1u, (uint32_t)(x[g] >> 1));
                        r[g] = p0 + wave_incl_scan_dpp(span) - span;
                        fills[g] = __ballot((uint32_t)x[g] & 1u) & M & inr;
                        lit[g] = ~M & inr & __ballot(r[g] - tS < nPos);
                        any_fill |= fills[g] ? (1u << g) : 0u;
                    }
                    // one-fills of markers in range (rare): counted through the difference array
                    if (any_fill) {
#pragma unroll
                        for (int g = 0; g < WB; ++g) {
                            if (((any_fill >> g) & 1u) && ((fills[g] >> lane) & 1ull)) {
                                const uint32_t L = (uint32_t)(x[g] >> 1);
                                const uint32_t fa = max(r[g], tS), fb = min(r[g] + L, tE);
                                if (fa < fb) { atomicAdd(&diff[fa - tS], 1); atomicAdd(&diff[fb - tS], -1); }
                            }
                        }
                    }
                    // words in pruned groups add nothing
                    if (prune) {
                        // branch-free: every lane reads a mask word (lanes outside the tile read
                        // some group's; lit already excludes them), all reads before one wait
                        uint32_t mw[WB], gi[WB];
#pragma unroll
                        for (int g = 0; g < WB; ++g) {
                            gi[g] = ((r[g] - tS) & (uint32_t)(TW - 1)) >> pm.sh;
                            mw[g] = pm.w[gi[g] >> 5];
                        }
#pragma unroll
                        for (int g = 0; g < WB; ++g) lit[g] &= ~__ballot((mw[g] >> (gi[g] & 31u)) & 1u);
                    }
                    // dirty words in range add at their tile-relative position
                    uint32_t act = 0;   // bit g: window g has a word to add
#pragma unroll
                    for (int g = 0; g < WB; ++g) {
                        // lanes without a word (x = 0) add nothing; their slot keeps the window's
                        // lane-to-position stride, so the 64 lanes fall on distinct LDS banks
                        r[g] = (r[g] - tS) & (uint32_t)(TW - 1);
                        x[g] = lane_sel64(lit[g], 0ull, x[g]);
                        if (lit[g]) act |= 1u << g;
                    }
                    // next batch's loads
                    if (w0 + (uint32_t)WB < we)
                        issue_batch(win, w0 + (uint32_t)WB, we, lane, table, sk, dz, alm, v, fl);
                    // ripple-carry adds, one plane at a time over the whole batch: all atomics
                    // of a plane are issued before any result is used, and the batch leaves
                    // once no lane carries (no per-window bookkeeping)
                    if (act) {
                        for (int p = 0; p < PL; ++p) {
                            uint64_t old[WB];
#pragma unroll
                            for (int g = 0; g < WB; ++g) {
                                old[g] = plane_add<LOOPED>(planes, (uint32_t)p, r[g], x[g]);
                            }
                            // one wait for all of them (lgkmcnt(0)); without it the compiler cannot
                            // tell that no result is still in flight and waits per atomic
                            __builtin_amdgcn_s_waitcnt(0xC07F);
                            uint64_t any = 0;
#pragma unroll
                            for (int g = 0; g < WB; ++g) {
                                x[g] &= old[g];
                                any |= x[g];
                            }
                            if (__ballot(any != 0ull) == 0ull) break;
                        }
                    }
                }
                __syncthreads();
            }

            EWT_PHASE(3);
            // dense rows: Harley-Seal carry-save-adder tree, one lane per word position
            const uint32_t n_dense = LOOPED ? 0u : misc[M_NDENSE];   // the unary counter takes no dense rows
            if (n_dense && (uint32_t)tid < nPos && !(prune && pruned_at(pm, (uint32_t)tid))) {
                uint64_t R[MAXP];
#pragma unroll
                for (int p = 0; p < MAXP; ++p) R[p] = 0;
                for (uint32_t d = 0; d < n_dense; d += 16u) {   // a short last group reads zeros
                    uint64_t x[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        x[j] = d + (uint32_t)j < n_dense ? __builtin_nontemporal_load(gp(dense[d + j]) + tid) : 0ull;
                    uint64_t twosA, twosB, foursA, foursB, eightsA, eightsB, sixteens;
                    EWT_CSA(twosA, R[0], R[0], x[0], x[1]);
                    EWT_CSA(twosB, R[0], R[0], x[2], x[3]);
                    EWT_CSA(foursA, R[1], R[1], twosA, twosB);
                    EWT_CSA(twosA, R[0], R[0], x[4], x[5]);
                    EWT_CSA(twosB, R[0], R[0], x[6], x[7]);
                    EWT_CSA(foursB, R[1], R[1], twosA, twosB);
                    EWT_CSA(eightsA, R[2], R[2], foursA, foursB);
                    EWT_CSA(twosA, R[0], R[0], x[8], x[9]);
                    EWT_CSA(twosB, R[0], R[0], x[10], x[11]);
                    EWT_CSA(foursA, R[1], R[1], twosA, twosB);
                    EWT_CSA(twosA, R[0], R[0], x[12], x[13]);
                    EWT_CSA(twosB, R[0], R[0], x[14], x[15]);
                    EWT_CSA(foursB, R[1], R[1], twosA, twosB);
                    EWT_CSA(eightsB, R[2], R[2], foursA, foursB);
                    EWT_CSA(sixteens, R[3], R[3], eightsA, eightsB);
                    uint64_t cy = sixteens;
#pragma unroll
                    for (int p = 4; p < MAXP; ++p) { uint64_t tt = R[p] & cy; R[p] ^= cy; cy = tt; }
                }
                uint64_t cy = 0;
#pragma unroll
                for (int p = 0; p < MAXP; ++p) {
                    if (p < P) {
                        uint64_t a = planes[p * TW + tid], b = R[p];
                        uint64_t u = a ^ b;
                        planes[p * TW + tid] = u ^ cy;
                        cy = (a & b) | (u & cy);
                    }
                }
            }
            __syncthreads();
            if (tid == 0) misc[M_NDENSE] = 0;
            __syncthreads();
        }
    }

    EWT_PHASE(4);
    // ---- compare: f(count) per row, where count = planes + k1 (the one-fills at the
    // position), bit-sliced; the threshold compares the planes with T - k1
    uint32_t k1tot;
    int32_t dv = tid < TW ? diff[tid] : 0;
    uint32_t k1 = block_excl_scan((uint32_t)dv, misc + M_TMP, k1tot) + (uint32_t)dv;
    if constexpr (HIST) {
        // count histogram of the tile in LDS (the window list is free now), then added
        // into acc[1..N]: the count of a row is its planes value plus the one-fills at
        // its word; rows of count zero are skipped
        uint32_t* hl = (uint32_t*)win;
        for (uint32_t i = (uint32_t)tid; i <= N; i += BLOCK) hl[i] = 0u;
        __syncthreads();
        if ((uint32_t)tid < nPos) {
            const uint64_t cand = (tS + (uint32_t)tid == U - 1u && q.tail_bits) ? ((1ull << q.tail_bits) - 1ull) : ~0ull;
            uint64_t R[MAXP];
            uint64_t any = 0;
#pragma unroll
            for (int p = 0; p < MAXP; ++p) {
                R[p] = p < P ? planes[p * TW + tid] : 0ull;
                any |= R[p];
            }
            any &= cand;
            if (k1) {
                const uint32_t c0 = (uint32_t)__popcll(cand & ~any);
                if (c0) atomicAdd(&hl[k1], c0);
            }
            while (any) {
                const int r = __builtin_ctzll(any);
                any &= any - 1ull;
                const uint32_t c = sliced_row(R, 1, MAXP, (uint32_t)r);
                atomicAdd(&hl[c + k1], 1u);
            }
        }
        __syncthreads();
        for (uint32_t i = 1u + (uint32_t)tid; i <= N; i += BLOCK)
            if (hl[i]) atomicAdd(q.pd->acc + i, (unsigned long long)hl[i]);
        return;
    } else if constexpr (MAXC) {
        // largest planes value over the word's valid rows (bit-sliced maximum: keep the
        // rows holding the highest plane bit seen so far), plus the position's one-fills
        if ((uint32_t)tid < nPos) {
            const uint64_t cand = (tS + (uint32_t)tid == U - 1u && q.tail_bits) ? ((1ull << q.tail_bits) - 1ull) : ~0ull;
            const uint32_t m = sliced_max(planes + tid, TW, P, cand);
            atomicMax(&misc[M_MAX], m + k1);
        }
        __syncthreads();
        if (tid == 0) atomicMax(q.pd->acc, (unsigned long long)misc[M_MAX]);
        return;
    }
    // a general table goes to LDS (the window list is free now): bit c of ftab is f(c)
    const uint32_t* ftab = (const uint32_t*)win;
    if constexpr (GENERAL) {
        if (mode == 0 && q.pd->kind == PRED_TABLE) {
            uint32_t* ft = (uint32_t*)win;
            const uint32_t nw = (N + 32u) / 32u;
            for (uint32_t i = (uint32_t)tid; i < nw; i += BLOCK) ft[i] = gp(q.pd->tab)[i];
        }
        __syncthreads();
    }
    uint64_t o = 0;
    if ((uint32_t)tid < nPos) {
        if (mode == 1) o = ~0ull;
        else if (mode == 2) o = 0;
        else if (GENERAL && q.pd->kind != PRED_THRESHOLD) {
            const PredDev* pd = q.pd;
            uint64_t R[MAXP];
#pragma unroll
            for (int p = 0; p < MAXP; ++p) R[p] = p < P ? planes[p * TW + tid] : 0ull;
            if (pd->kind == PRED_TABLE) {
                // per row: its count (planes value plus the word's one-fills) indexes the table
                for (uint32_t r = 0; r < 64u; ++r) {
                    const uint32_t c = k1 + sliced_row(R, 1, P, r);
                    o |= (uint64_t)((ftab[c >> 5] >> (c & 31u)) & 1u) << r;
                }
            } else if (pd->kind == PRED_INTERVALS) {
                // count in [a, b]  <=>  planes in [a - k1, b - k1]
                const uint32_t n_iv = pd->n_iv;
                for (uint32_t j = 0; j < n_iv; ++j) {
                    const int lo = (int)pd->iv[2 * j] - (int)k1, hi = (int)pd->iv[2 * j + 1] - (int)k1;
                    o |= sliced_ge(R, 1, P, lo) & ~sliced_ge(R, 1, P, hi + 1);
                }
            } else {   // parity of planes + k1: plane 0 flipped when k1 is odd
                o = R[0] ^ (((k1 & 1u) ^ (pd->kind == PRED_EVEN ? 1u : 0u)) ? ~0ull : 0ull);
            }
        } else if constexpr (LOOPED) {
            // count >= T  <=>  the literal adds reached level T - k1
            const int tp = (int)T - (int)k1;
            o = tp <= 0 ? ~0ull : planes[(tp - 1) * TW + tid];
        } else {
            // count >= T  <=>  planes >= T - k1
            o = sliced_ge(planes + tid, TW, P, (int)T - (int)k1);
        }
        if (tS + (uint32_t)tid == U - 1u && q.tail_bits) o &= (1ull << q.tail_bits) - 1ull;
    }
    if constexpr (GENERAL) {
        // output row count (one atomic per wavefront), for callers that need |result|
        const uint64_t accp = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)q.pd->acc >> 32)) << 32) |
                              (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)q.pd->acc);
        if (accp) {
            const uint32_t c = wave_incl_scan((uint32_t)__popcll(o));
            if (lane == 63 && c) atomicAdd((unsigned long long*)accp, (unsigned long long)c);
        }
    }
    __syncthreads();   // planes are reused below
    EWT_PHASE(5);

    // ---- encode: canonical EWAH by scan-and-compact with decoupled look-back
    uint8_t* clsA = (uint8_t*)smem;                        // TW
    uint16_t* hpos = (uint16_t*)(smem + TW);               // TW
    uint16_t* hout = (uint16_t*)(smem + 3 * TW);           // TW
    const bool act = (uint32_t)tid < nPos;
    const uint32_t cls = act ? (o == 0 ? 0u : (o == ~0ull ? 1u : 2u)) : 3u;
    clsA[tid] = (uint8_t)cls;
    __syncthreads();
    const uint32_t prevc = tid > 0 ? clsA[tid - 1] : 3u;
    const uint32_t hl = act && ((tid == 0) ? (t == 0 || cls != 2u) : (cls != 2u && cls != prevc)) ? 1u : 0u;
    const uint32_t emit = hl + (cls == 2u ? 1u : 0u);
    uint32_t tot;
    const uint32_t ex = block_excl_scan((emit << 16) | hl, misc + M_TMP, tot);
    const uint32_t ex_emit = ex >> 16, ex_head = ex & 0xFFFFu;
    const uint32_t n_local = tot >> 16, nheads = tot & 0xFFFFu;
    if (hl) { hpos[ex_head] = (uint16_t)tid; hout[ex_head] = (uint16_t)ex_emit; }
    __syncthreads();

    if constexpr (STAGED) {
        // ---- staged output: literals at their local output index, markers of the runs
        // that end inside the tile; the placement pass moves them to their final index
        // and writes the markers of runs that continue across tiles
        EWT_GLOBAL uint64_t* stage = gp(q.stage) + (size_t)t * STAGE_WORDS;
        if (act) {
            if (cls == 2u) stage[ex_emit + hl] = o;
            if (hl && ex_head + 1u < nheads) {
                const uint32_t nh = hpos[ex_head + 1];
                const uint32_t K = hout[ex_head + 1] - ex_emit - 1u;
                const uint32_t L = (nh - (uint32_t)tid) - K;
                stage[ex_emit] = (cls == 1u ? 1ull : 0ull) | ((uint64_t)L << 1) | ((uint64_t)K << 33);
            }
        }
        if (tid == 0) {
            Agg A;
            A.n = n_local;
            uint32_t bits = (uint32_t)clsA[0] | ((uint32_t)clsA[nPos - 1] << 2);
            if (nheads) {
                const uint32_t lh = hpos[nheads - 1];
                A.lh_pos = tS + lh;
                A.lh_out = hout[nheads - 1];
                bits |= (1u << 4) | ((clsA[lh] == 1u ? 1u : 0u) << 5);
            } else {
                A.lh_pos = 0; A.lh_out = 0;
            }
            A.bits = bits;
            EWT_GLOBAL TileState* st = gp(q.state);
            const uint64_t h0 = nheads > 0 ? ((uint64_t)hpos[0] | ((uint64_t)hout[0] << 32)) : 0ull;
            const uint64_t h1 = nheads > 1 ? ((uint64_t)hpos[1] | ((uint64_t)hout[1] << 32)) : 0ull;
            st[t].head[0] = h0;
            st[t].head[1] = h1 | ((uint64_t)min(nheads, 2u) << 16);
            agg_publish(st[t].local, A, epoch);
        }
        EWT_PHASE(6);
        __syncthreads();
    } else {
        // ---- prefix over earlier tiles by look-back, words written in place
        if (wave == 0) {
            // local aggregate of this tile (every lane of wave 0 computes it)
            Agg A;
            A.n = n_local;
            uint32_t bits = (uint32_t)clsA[0] | ((uint32_t)clsA[nPos - 1] << 2);
            if (nheads) {
                uint32_t lh = hpos[nheads - 1];
                A.lh_pos = tS + lh;
                A.lh_out = hout[nheads - 1];
                bits |= (1u << 4) | ((clsA[lh] == 1u ? 1u : 0u) << 5);
            } else {
                A.lh_pos = 0; A.lh_out = 0;
            }
            A.bits = bits;
            EWT_GLOBAL TileState* st = gp(q.state);
            Agg X;
            X.n = 0; X.lh_pos = 0; X.lh_out = 0; X.bits = 3u << 2;
            Agg I = A;
            if (lane == 0) agg_publish(st[t].local, A, epoch);   // tile 0's too: a block's last tile reads it
            if (t > 0) {
                X = lookback(st, (int)t, A, tS, epoch, err);
                I = agg_combine(X, A, tS);
            }
            if (lane == 0) {
                agg_publish(st[t].incl, I, epoch);
                misc[M_X + 0] = X.n; misc[M_X + 1] = X.lh_pos; misc[M_X + 2] = X.lh_out; misc[M_X + 3] = X.bits;
                misc[M_TOT] = I.n;
            }
        }
        __syncthreads();

        EWT_PHASE(6);
        const uint32_t Xn = misc[M_X + 0], Xlh_pos = misc[M_X + 1], Xlh_out = misc[M_X + 2], Xbits = misc[M_X + 3];
        const uint32_t total = misc[M_TOT];
        const uint32_t c0 = clsA[0];
        const uint32_t merge = (t > 0 && c0 != 2u && ((Xbits >> 2) & 3u) == c0) ? 1u : 0u;
        const uint64_t cap = q.cap;
        EWT_GLOBAL uint64_t* out = gp(q.out);
        auto out_of = [&](uint32_t i, uint32_t local_ex) -> uint32_t { return Xn + local_ex - (i > 0 ? merge : 0u); };

        if (act) {
            const uint32_t my_out = out_of((uint32_t)tid, ex_emit);
            if (cls == 2u) {
                uint32_t idx = my_out + hl;
                if (idx < cap) out[idx] = o;
            }
            if (hl && !(tid == 0 && merge)) {
                const uint32_t r = ex_head;
                if (r + 1u < nheads) {
                    uint32_t nh = hpos[r + 1];
                    uint32_t nh_out = out_of(nh, hout[r + 1]);
                    uint32_t K = nh_out - my_out - 1u;
                    uint32_t L = (nh - (uint32_t)tid) - K;
                    uint64_t f = cls == 1u ? 1ull : 0ull;
                    if (my_out < cap) out[my_out] = f | ((uint64_t)L << 1) | ((uint64_t)K << 33);
                }
                // the first actual head of the tile closes the group left open by earlier tiles
                if (t > 0 && r == merge) {
                    uint32_t K = my_out - Xlh_out - 1u;
                    uint32_t L = (tS + (uint32_t)tid - Xlh_pos) - K;
                    uint64_t f = (Xbits >> 5) & 1u;
                    if (Xlh_out < cap) out[Xlh_out] = f | ((uint64_t)L << 1) | ((uint64_t)K << 33);
                }
            }
        }
        if (t == tiles - 1 && tid == 0) {
            uint32_t lpos, lout;
            uint64_t lf;
            if (nheads > merge) {
                uint32_t h = hpos[nheads - 1];
                lpos = tS + h;
                lout = out_of(h, hout[nheads - 1]);
                lf = clsA[h] == 1u ? 1ull : 0ull;
            } else {
                lpos = Xlh_pos; lout = Xlh_out; lf = (Xbits >> 5) & 1u;
            }
            uint32_t K = total - lout - 1u;
            uint32_t L = (U - lpos) - K;
            if (lout < cap) out[lout] = lf | ((uint64_t)L << 1) | ((uint64_t)K << 33);
            *gp(q.out_n) = total;
        }
        __syncthreads();
    }
    EWT_PHASE(7);
}

// ------------------------------------------------------------ bounds pre-pass

// Adds, for every input k < N of a query, word off of its presence records into the
// bit-sliced counter c (one wavefront; lane 64 r + i of round r holds input k's record at rp[r];
// lanes with skip set load nothing).  16 loads are in flight before any is added (a smaller
// batch keeps the pass at 62 VGPRs, 8 wavefronts per SIMD).
__device__ __forceinline__ void count_records(const uint32_t* const* rp, uint32_t N, uint32_t off, bool skip,
                                              uint32_t* c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if ((uint32_t)(64 * r) >= N) break;
        const uint64_t base = (uint64_t)(uintptr_t)rp[r];
        const int blo = (int)(uint32_t)base, bhi = (int)(uint32_t)(base >> 32);
#pragma unroll 1
        for (uint32_t j0 = 0; j0 < 64u && 64u * (uint32_t)r + j0 < N; j0 += 16u) {
            const uint32_t ni = min(16u, N - 64u * (uint32_t)r - j0);
            uint32_t x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                x[i] = 0u;
                if ((uint32_t)i < ni && !skip) {
                    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(blo, (int)j0 + i);
                    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(bhi, (int)j0 + i);
                    x[i] = gp((const uint32_t*)(uintptr_t)(((uint64_t)hi << 32) | lo))[off];
                }
            }
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                if ((uint32_t)(8 * g) >= ni) break;
                add8(c, x + 8 * g);
            }
        }
    }
}

// Count bounds of one item (query q, tile t) of a batch, by one wavefront with no barrier:
// what the tile routine's classify and bounds steps take from the presence records (RBMrg's
// pruning by count bounds, Section 5.2), for threshold queries of at most PCAP_FINE inputs.
// A tile whose row counts are all below T publishes its aggregate here (a zero fill; the
// placement pass writes its marker) and never takes a workgroup of the batched launch.
// Returns PRE_*; PRE_MASK leaves the word mask at mask.  Lanes must all be active.
__device__ uint32_t pre_bounds(const QueryDev& q, uint32_t t, uint32_t epoch, uint32_t* mask) {
    const int lane = __lane_id();
    const uint32_t N = q.N, T = q.T;
    if (N > PCAP_FINE || T == 0u || T > N || q.pd || !q.bms) return PRE_NONE;
    const uint32_t tS = t * (uint32_t)TW;
    const uint32_t nPos = min((uint32_t)TW, q.U - tS);
    const uint32_t nfull = 4u * nPos;   // quarters of an input with a one in every quarter
    // input 64 r + lane: its record of the tile and how many of its quarters hold a one (all
    // loads issued before any is used)
    const uint32_t* rp[4];
    const uint16_t* cp[4];
    uint32_t qc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t k = 64u * (uint32_t)r + (uint32_t)lane;
        rp[r] = nullptr;
        cp[r] = nullptr;
        if (k < N) {
            rp[r] = gp(q.bms)[k].presq;
            cp[r] = gp(q.bms)[k].qcnt + t;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t k = 64u * (uint32_t)r + (uint32_t)lane;
        qc[r] = k < N ? (uint32_t)*gp(cp[r]) : 0u;
    }
    uint32_t psum = 0, dfull = 0, nz = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t k = 64u * (uint32_t)r + (uint32_t)lane;
        psum += qc[r];
        dfull += (uint32_t)__popcll(__ballot(k < N && qc[r] == nfull));
        nz += (uint32_t)__popcll(__ballot(qc[r] != 0u));
    }
    psum = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(psum), 63);
    const uint32_t gate = (q.variant >> VAR_GATE_SHIFT) & 3u;
    const uint64_t gnum = gate == GATE_1_5 ? 15ull : 11ull;
    bool settled = nz < T;   // fewer than T inputs have a one anywhere in the tile
    uint32_t w8 = 0, vmask = 0;
    if (!settled) {
        // the gate of the tile routine: bounds only where they are likely to prune
        if (dfull >= T || gate == GATE_NEVER || (gate != GATE_ALWAYS && 10ull * T * nfull <= gnum * psum))
            return PRE_OPEN;
        // lane l takes words 8 l .. 8 l + 7: first whole words (its byte of the tile's per-word
        // bits word l / 4), then the quarters of the words still in play (the tile's quarter word
        // l: quarters 32 l .. 32 l + 31, four per word), then their 8-row groups (word l of half h
        // of the tile's 8-row bits: words 8 l + 4 h .. 8 l + 4 h + 3)
        const uint32_t w0 = 8u * (uint32_t)lane;
        vmask = (1u << (nPos > w0 ? min(nPos - w0, 8u) : 0u)) - 1u;   // words of this lane in the tile
        uint32_t c[QP];
#pragma unroll
        for (int p = 0; p < QP; ++p) c[p] = 0u;
        const uint32_t tiles = q.tiles;
        count_records(rp, N, t * PQ_W_TILE + ((uint32_t)lane >> 2), false, c);
        w8 = (below(c, T) >> (8u * ((uint32_t)lane & 3u))) & vmask;
        if (__ballot(w8 != vmask) != 0ull) {
            const bool skip = (w8 | ~vmask | ~0xFFu) == ~0u;
#pragma unroll
            for (int p = 0; p < QP; ++p) c[p] = 0u;
            count_records(rp, N, pq_quarters(tiles) + t * PQ_Q_TILE + (uint32_t)lane, skip, c);
            uint32_t m = below(c, T);
            m &= m >> 1;
            m &= m >> 2;   // bit 4 i: all four quarters of word w0 + i
#pragma unroll
            for (int i = 0; i < 8; ++i) w8 |= ((m >> (4 * i)) & 1u) << i;
            w8 &= vmask;
        }
#pragma unroll 1
        for (uint32_t h = 0; h < 2u; ++h) {
            const bool skip = ((w8 | ~vmask) >> (4u * h) & 15u) == 15u;
            if (__ballot(!skip) == 0ull) continue;
#pragma unroll
            for (int p = 0; p < QP; ++p) c[p] = 0u;
            count_records(rp, N, pq_octets(tiles, h) + t * PQ_O_TILE + (uint32_t)lane, skip, c);
            uint32_t o = below(c, T);
            o &= o >> 1;
            o &= o >> 2;
            o &= o >> 4;   // bit 8 i: all eight 8-row groups of word w0 + 4 h + i
            if (!skip) {
#pragma unroll
                for (int i = 0; i < 4; ++i) w8 |= ((o >> (8 * i)) & 1u) << (4u * h + (uint32_t)i);
            }
        }
        w8 &= vmask;
        settled = __ballot(w8 != vmask) == 0ull;
    }
    if (settled) {
        if (lane == 0) {
            EWT_GLOBAL TileState* st = gp(q.state);
            Agg A;
            A.n = 1;
            A.lh_pos = tS;
            A.lh_out = 0;
            A.bits = 1u << 4;   // one head, a zero fill
            st[t].head[0] = 0ull;
            st[t].head[1] = 1ull << 16;
            agg_publish(st[t].local, A, epoch);
        }
        return PRE_SETTLED;
    }
    if (__ballot(w8 != 0u) == 0ull) return PRE_OPEN;
    // byte l of the mask: words 8 l .. 8 l + 7
    uint32_t v = w8 << (8u * ((uint32_t)lane & 3u));
    v |= (uint32_t)__shfl_xor((int)v, 1, 64);
    v |= (uint32_t)__shfl_xor((int)v, 2, 64);
    if ((lane & 3) == 0) gp(mask)[lane >> 2] = v;
    return PRE_MASK;
}

// ------------------------------------------------------------ output placement

// Exclusive prefix of the tile aggregates of one query (one workgroup of
// SCAN_THREADS threads, tiles in chunks): X_t = A_0 + ... + A_(t-1), written into
// the tile's state for the placement kernel.
constexpr int SCAN_THREADS = 1024;

__device__ void scan_query(const QueryDev& q, uint32_t epoch, uint32_t* err) {
    __shared__ uint32_t part[SCAN_THREADS / 64][5];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    EWT_GLOBAL TileState* st = gp(q.state);
    Agg carry;
    carry.n = 0; carry.lh_pos = 0; carry.lh_out = 0; carry.bits = 0;
    bool carry_empty = true;
    for (uint32_t base = 0; base < q.tiles; base += SCAN_THREADS) {
        const uint32_t i = base + (uint32_t)tid;
        const bool in = i < q.tiles;
        Agg v;
        v.n = 0; v.lh_pos = 0; v.lh_out = 0; v.bits = 0;
        bool valid = in;
        if (valid && !agg_fetch(st[i].local, epoch, v)) {
            atomicOr(err, 4u);
            valid = false;
        }
        // inclusive scan inside the wavefront: lane l - d holds the earlier tiles
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            Agg o;
            o.n = __shfl_up(v.n, d, 64);
            o.lh_pos = __shfl_up(v.lh_pos, d, 64);
            o.lh_out = __shfl_up(v.lh_out, d, 64);
            o.bits = __shfl_up(v.bits, d, 64);
            const bool ov = __shfl_up((int)valid, d, 64) != 0 && lane >= d;
            if (ov) {
                if (valid) v = agg_combine(o, v, (i - (uint32_t)d + 1u) * (uint32_t)TW);
                else { v = o; valid = true; }
            }
        }
        if (lane == 63) {
            part[wave][0] = v.n; part[wave][1] = v.lh_pos; part[wave][2] = v.lh_out; part[wave][3] = v.bits;
            part[wave][4] = valid ? 1u : 0u;
        }
        __syncthreads();
        // earlier wavefronts of the chunk, then the carry of earlier chunks
        Agg pre;
        pre.n = 0; pre.lh_pos = 0; pre.lh_out = 0; pre.bits = 0;
        bool pre_valid = false;
        for (int w = 0; w < wave; ++w) {
            if (!part[w][4]) continue;
            Agg b;
            b.n = part[w][0]; b.lh_pos = part[w][1]; b.lh_out = part[w][2]; b.bits = part[w][3];
            if (pre_valid) pre = agg_combine(pre, b, (base + (uint32_t)w * 64u) * (uint32_t)TW);
            else { pre = b; pre_valid = true; }
        }
        if (!carry_empty) {
            pre = pre_valid ? agg_combine(carry, pre, base * (uint32_t)TW) : carry;
            pre_valid = true;
        }
        // inclusive prefix of tile i, and the exclusive one (inclusive of tile i - 1)
        Agg inc = v;
        if (pre_valid && valid) inc = agg_combine(pre, v, (base + (uint32_t)wave * 64u) * (uint32_t)TW);
        Agg ex;
        ex.n = __shfl_up(inc.n, 1, 64);
        ex.lh_pos = __shfl_up(inc.lh_pos, 1, 64);
        ex.lh_out = __shfl_up(inc.lh_out, 1, 64);
        ex.bits = __shfl_up(inc.bits, 1, 64);
        if (lane == 0) ex = pre;
        if (in && i > 0) agg_publish(st[i].incl, ex, epoch);
        // carry: inclusive prefix of the chunk's last valid tile
        const uint32_t last = min(q.tiles - base, (uint32_t)SCAN_THREADS) - 1u;
        __syncthreads();
        if ((uint32_t)tid == last) {
            part[0][0] = inc.n; part[0][1] = inc.lh_pos; part[0][2] = inc.lh_out; part[0][3] = inc.bits;
        }
        __syncthreads();
        carry.n = part[0][0]; carry.lh_pos = part[0][1]; carry.lh_out = part[0][2]; carry.bits = part[0][3];
        carry_empty = false;
        __syncthreads();
    }
}

// Moves the staged words of tile t to their place and writes the markers of runs
// crossing into the tile (one wavefront per tile).
__device__ void place_tile(const QueryDev& q, uint32_t t, uint32_t epoch, uint32_t* err) {
    const int lane = __lane_id();
    EWT_GLOBAL TileState* st = gp(q.state);
    Agg A, X;
    if (!agg_fetch(st[t].local, epoch, A)) { if (lane == 0) atomicOr(err, 8u); return; }
    X.n = 0; X.lh_pos = 0; X.lh_out = 0; X.bits = 3u << 2;
    if (t > 0 && !agg_fetch(st[t].incl, epoch, X)) { if (lane == 0) atomicOr(err, 8u); return; }
    const uint64_t h0 = st[t].head[0], h1w = st[t].head[1];
    const uint32_t nheads = (uint32_t)(h1w >> 16) & 3u;
    const uint32_t tS = t * (uint32_t)TW;
    const uint32_t c0 = A.bits & 3u;
    const uint32_t merge = (t > 0 && c0 != 2u && ((X.bits >> 2) & 3u) == c0) ? 1u : 0u;
    const uint64_t cap = q.cap;
    EWT_GLOBAL uint64_t* out = gp(q.out);
    const EWT_GLOBAL uint64_t* stage = gp(q.stage) + (size_t)t * STAGE_WORDS;
    // the marker slot of the tile's last head stays unstaged (its run continues past
    // the tile): a later tile or the last one writes it
    const uint32_t open = ((A.bits >> 4) & 1u) ? A.lh_out : 0xFFFFFFFFu;
    for (uint32_t e = merge + (uint32_t)lane; e < A.n; e += 64u) {
        const uint32_t idx = X.n + e - merge;
        if (e != open && idx < cap) out[idx] = stage[e];
    }
    if (lane == 0) {
        // the first head of the tile that starts a run closes the run left open before it
        if (t > 0 && nheads > merge) {
            const uint64_t h = merge ? h1w : h0;
            const uint32_t hp = (uint32_t)h & 0xFFFFu, ho = (uint32_t)(h >> 32);
            const uint32_t my_out = X.n + ho - merge;
            const uint32_t K = my_out - X.lh_out - 1u;
            const uint32_t L = (tS + hp - X.lh_pos) - K;
            if (X.lh_out < cap) out[X.lh_out] = ((X.bits >> 5) & 1u) | ((uint64_t)L << 1) | ((uint64_t)K << 33);
        }
        if (t == q.tiles - 1) {   // the last tile closes the last run
            const Agg I = t > 0 ? agg_combine(X, A, tS) : A;
            uint32_t lpos, lout;
            uint64_t lf;
            if (nheads > merge) {
                lpos = A.lh_pos;
                lout = X.n + A.lh_out - (A.lh_pos > tS ? merge : 0u);
                lf = (A.bits >> 5) & 1u;
            } else {
                lpos = X.lh_pos; lout = X.lh_out; lf = (X.bits >> 5) & 1u;
            }
            const uint32_t K = I.n - lout - 1u;
            const uint32_t L = (q.U - lpos) - K;
            if (lout < cap) out[lout] = lf | ((uint64_t)L << 1) | ((uint64_t)K << 33);
            *gp(q.out_n) = I.n;
        }
    }
}

// ----------------------------------------------------------------- kernels
// Both kernels are built for four wavefronts per SIMD (at most 128 VGPRs), so a
// compute unit holds 1024 threads: one workgroup of 1024 or two of 512.

// One query, one workgroup per tile.  Tiles are taken in ticket order so that a
// tile only ever waits for tiles that are already running or done.
__global__ __launch_bounds__(BLOCK, 4) void thr_query_kernel(QueryDev q, const BitmapDev* __restrict__ table,
                                                          uint32_t* ticket, uint32_t epoch, uint32_t* err,
                                                          InlineIds ids) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) {
        uint32_t t = atomicAdd(ticket, 1u);
        if (t == q.tiles - 1) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = t;
    }
    __syncthreads();
    QueryDev qq = q;
    if (!qq.ids) qq.ids = ids.v;   // slots in the kernel arguments
    process_tile<false>(qq, table, s_t, epoch, smem, err, s_t);
}

// The same with the unary per-row counter (use_looped(q.variant, q.N, q.T) holds).
__global__ __launch_bounds__(BLOCK, 4) void thr_query_looped_kernel(QueryDev q, const BitmapDev* __restrict__ table,
                                                                 uint32_t* ticket, uint32_t epoch, uint32_t* err,
                                                                 InlineIds ids) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) {
        uint32_t t = atomicAdd(ticket, 1u);
        if (t == q.tiles - 1) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = t;
    }
    __syncthreads();
    QueryDev qq = q;
    if (!qq.ids) qq.ids = ids.v;   // slots in the kernel arguments
    process_tile<false, false, false, true>(qq, table, s_t, epoch, smem, err, s_t);
}

// The same for a general symmetric predicate (q.pd: intervals of counts or parity),
// a separate instantiation so that the threshold kernels keep their registers.
__global__ __launch_bounds__(BLOCK, 4) void thr_query_sym_kernel(QueryDev q, const BitmapDev* __restrict__ table,
                                                          uint32_t* ticket, uint32_t epoch, uint32_t* err) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) {
        uint32_t t = atomicAdd(ticket, 1u);
        if (t == q.tiles - 1) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = t;
    }
    __syncthreads();
    process_tile<false, true>(q, table, s_t, epoch, smem, err, s_t);
}

// Count histogram of a query (q.pd->kind = PRED_HIST): no output is written.
__global__ __launch_bounds__(BLOCK, 4) void thr_query_hist_kernel(QueryDev q, const BitmapDev* __restrict__ table,
                                                               uint32_t* ticket, uint32_t epoch, uint32_t* err) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) {
        uint32_t t = atomicAdd(ticket, 1u);
        if (t == q.tiles - 1) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = t;
    }
    __syncthreads();
    process_tile<false, false, true, false, true>(q, table, s_t, epoch, smem, err, s_t);
}

// Largest row count of a query (q.pd->kind = PRED_MAXCOUNT): no output is written.
__global__ __launch_bounds__(BLOCK, 4) void thr_query_max_kernel(QueryDev q, const BitmapDev* __restrict__ table,
                                                          uint32_t* ticket, uint32_t epoch, uint32_t* err) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) {
        uint32_t t = atomicAdd(ticket, 1u);
        if (t == q.tiles - 1) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = t;
    }
    __syncthreads();
    process_tile<false, false, true>(q, table, s_t, epoch, smem, err, s_t);
}

// Many queries in one persistent launch.  The (query, tile) items are split into
// NXCD contiguous ranges, one per XCD (workgroup i runs on XCD i mod NXCD), so that
// neighbouring tiles of a query, which share the compressed chunk at their boundary,
// are read through one L2.  A workgroup takes the next item of its own range from
// that range's counter and, once the range is used up, items of the other ranges in
// turn.  qtile[i] = first item of query i (qtile[nq] = total); tq[i] = query of item i.
// item_t (null: off): per item, the wall-clock ticks its workgroup spent on it, the
// measure of each query's cost inside a batch.
// Bounds pre-pass of a batch: one wavefront per item.
constexpr uint32_t PRE_WG = 4u;   // wavefronts per workgroup (2 as fast; 8 and 16 slower)
__global__ __launch_bounds__(64 * PRE_WG) void thr_bounds_kernel(const QueryDev* __restrict__ qs, const uint32_t* __restrict__ qtile,
                                                          const uint32_t* __restrict__ tq, uint32_t nq, uint32_t total,
                                                          const uint32_t* epoch_ptr, uint32_t* __restrict__ pre,
                                                          uint32_t* __restrict__ pmask, uint32_t* __restrict__ list,
                                                          uint32_t* work, uint32_t* __restrict__ item_t, uint32_t tiles) {
    // workgroup b runs on XCD b % NXCD: each XCD takes a contiguous share [a, e) of the items
    const uint32_t nwg = gridDim.x, x = blockIdx.x % (uint32_t)NXCD;
    const uint32_t per = nwg / NXCD, ext = nwg % NXCD;
    const uint32_t wg0 = x * per + min(x, ext);
    uint32_t it = (wg0 + blockIdx.x / (uint32_t)NXCD) * PRE_WG + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (it >= total) return;
    // a share of whole queries (every query of a batch has the same tiles) is taken in blocks of
    // PRE_TB tiles: block 0 of every query of the share, then block 1, and so on.  The XCDs then
    // read the same tiles of the pool's records at about the same time, and a record that many
    // queries name is more likely still cached when the next of them reads it; inside a block
    // the tiles of a query stay together (they share its descriptors and count lines)
    const uint32_t a = wg0 * PRE_WG, e = min((wg0 + per + (x < ext ? 1u : 0u)) * PRE_WG, total);
    it = pre_item_order(it, a, e, tiles);
    const uint64_t t0 = item_t ? wall_clock64() : 0ull;
    const uint32_t qi = nq > 1u ? tq[it] : 0u;
    const QueryDev q = qs[qi];
    const uint32_t r = pre_bounds(q, it - qtile[qi], *epoch_ptr, pmask + (size_t)it * PRE_MASK_WORDS);
    if (__lane_id() == 0) {
        pre[it] = r;
        if (r != PRE_SETTLED) {   // left to the tile routine: onto its XCD's list
            const uint32_t x = (uint32_t)((uint64_t)it * NXCD / total);
            const uint32_t lo = (uint32_t)(((uint64_t)total * x + NXCD - 1) / NXCD);   // first item of XCD x
            const uint32_t hi = (uint32_t)(((uint64_t)total * (x + 1u) + NXCD - 1) / NXCD);
            // wide queries' items from the front, the others from the back, so that the tile
            // routine takes the long items first and the short ones fill the end of the launch
            if (q.N >= 128u) list[lo + atomicAdd(&work[WORK_LIST + WORK_STRIDE * x], 1u)] = it;
            else list[hi - 1u - atomicAdd(&work[WORK_LIST + WORK_STRIDE * x + 1], 1u)] = it;
        }
        if (item_t) {   // ticks of the tile routine (none for a settled tile), then of this wavefront
            if (r == PRE_SETTLED) item_t[it] = 0u;
            item_t[total + it] = (uint32_t)(wall_clock64() - t0);
        }
    }
}

template <int WB>
__global__ __launch_bounds__(BLOCK, 4) void thr_batch_kernel(const QueryDev* __restrict__ qs, const uint32_t* __restrict__ qtile,
                                                          const uint32_t* __restrict__ tq, uint32_t nq,
                                                          const BitmapDev* __restrict__ table,
                                                          uint32_t* work, const uint32_t* epoch_ptr, uint32_t* err,
                                                          uint32_t* __restrict__ item_t, const uint32_t* __restrict__ pre,
                                                          const uint32_t* __restrict__ pmask,
                                                          const uint32_t* __restrict__ list) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_n, s_it[CLAIM_ITEMS], s_q[CLAIM_ITEMS], s_pre[CLAIM_ITEMS];
    const uint32_t total = qtile[nq];
    const uint32_t epoch = *epoch_ptr;
    const uint32_t x0 = blockIdx.x % (uint32_t)NXCD;
    while (true) {
        // wavefront 0 claims a run of items and reads their queries and pre-pass results: from
        // the XCD's list of items the pre-pass left, or (no pre-pass) from the XCD's range of
        // items; other XCDs' once its own is used up.  Runs are of up to CLAIM_ITEMS items where
        // an XCD's workgroups have at least 64 runs each to share, else of single items (a short
        // batch split into long runs would leave workgroups idle).
        if (threadIdx.x < 64) {
            uint32_t c = 0, n = 0, base = 0, nfront = 0, top = 0;
            if (threadIdx.x == 0) {
                const uint32_t per = (gridDim.x + NXCD - 1) / NXCD;   // workgroups per XCD
                for (uint32_t d = 0; d < (uint32_t)NXCD; ++d) {
                    const uint32_t x = (x0 + d) % (uint32_t)NXCD;
                    const uint32_t lo = (uint32_t)(((uint64_t)total * x + NXCD - 1) / NXCD);
                    const uint32_t hi = (uint32_t)(((uint64_t)total * (x + 1u) + NXCD - 1) / NXCD);
                    uint32_t len = hi - lo, nf = len;
                    if (list) {   // the list's front part, then its back part in reverse
                        nf = __hip_atomic_load(&work[WORK_LIST + WORK_STRIDE * x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        len = nf + __hip_atomic_load(&work[WORK_LIST + WORK_STRIDE * x + 1], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (len == 0) continue;
                    const uint32_t k = max(1u, min(CLAIM_ITEMS, len / (64u * per)));
                    c = atomicAdd(&work[WORK_CTR + WORK_STRIDE * x], k);
                    if (c < len) { base = lo; n = min(k, len - c); nfront = nf; top = hi; break; }
                }
            }
            c = (uint32_t)__builtin_amdgcn_readfirstlane((int)c);
            n = (uint32_t)__builtin_amdgcn_readfirstlane((int)n);
            base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
            nfront = (uint32_t)__builtin_amdgcn_readfirstlane((int)nfront);
            top = (uint32_t)__builtin_amdgcn_readfirstlane((int)top);
            const uint32_t j = threadIdx.x;
            if (j < n) {
                const uint32_t cj = c + j;
                const uint32_t it = list ? list[cj < nfront ? base + cj : top - 1u - (cj - nfront)] : base + cj;
                s_it[j] = it;
                s_q[j] = nq > 1u ? tq[it] : 0u;   // query of the item (a batch of one needs none)
                s_pre[j] = pre ? pre[it] : PRE_NONE;
            }
            if (j == 0) s_n = n;
        }
        __syncthreads();
        // uniform: the query record is then read into scalar registers
        const uint32_t n = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_n);
        if (n == 0) break;
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_it[j]);
            const uint32_t pj = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_pre[j]);
            const uint32_t qi = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_q[j]);
            const uint64_t t0 = item_t ? wall_clock64() : 0ull;
            QueryDev q = qs[qi];
            const uint32_t* pm = pmask ? pmask + (size_t)it * PRE_MASK_WORDS : nullptr;
            if (use_looped(q.variant, q.N, q.T))
                process_tile<true, false, false, true, false, WB>(q, table, it - qtile[qi], epoch, smem, err, it, pj, pm);
            else process_tile<true, false, false, false, false, WB>(q, table, it - qtile[qi], epoch, smem, err, it, pj, pm);
            if (item_t && threadIdx.x == 0) item_t[it] = (uint32_t)(wall_clock64() - t0);
        }
        __syncthreads();   // every wavefront is done with the claimed run before wavefront 0 rewrites it
    }
}

// Output placement of a batch: one workgroup per query for the prefixes, then one
// wavefront per (query, tile); tq[i] = query of item i.
__global__ __launch_bounds__(SCAN_THREADS) void scan_batch_kernel(const QueryDev* __restrict__ qs, const uint32_t* epoch_ptr,
                                                                   uint32_t* err) {
    scan_query(qs[blockIdx.x], *epoch_ptr, err);
}
__global__ __launch_bounds__(256) void place_batch_kernel(const QueryDev* __restrict__ qs, const uint32_t* __restrict__ qtile,
                                                           const uint32_t* __restrict__ tq, uint32_t total,
                                                           const uint32_t* epoch_ptr, uint32_t* err) {
    const uint32_t it = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (it >= total) return;
    const uint32_t qi = tq[it];
    const QueryDev q = qs[qi];
    place_tile(q, it - qtile[qi], *epoch_ptr, err);
}

// Next launch tag of a batch; tag 0 (the value of cleared states) is skipped.
// Every launch of a batch rewrites every tile state, so states older than the
// previous launch never survive and the 16-bit tag cycle is safe.
// Before each batched launch: advance the epoch (work[1]) and clear the item counters.
__global__ void bump_epoch_kernel(uint32_t* work) {
    uint32_t e = work[1] + 1u;
    if ((e & 0xFFFFu) == 0) e += 1u;
    work[1] = e;
    for (int x = 0; x < NXCD; ++x) {
        work[WORK_CTR + WORK_STRIDE * x] = 0u;
        work[WORK_LIST + WORK_STRIDE * x] = 0u;
        work[WORK_LIST + WORK_STRIDE * x + 1] = 0u;
    }
}

// Output for r = 0 (no words).
__global__ void zero_len_kernel(uint64_t* out_n) { *out_n = 0; }

}  // namespace ewt

// ---------------------------------------------------------------- launchers
namespace ewt {

hipError_t set_smem_limits(size_t max_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)thr_query_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)thr_query_sym_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)thr_query_max_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)thr_query_looped_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)thr_query_hist_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
    if (e != hipSuccess) return e;
    const void* batch_kernels[] = {(const void*)thr_batch_kernel<4>, (const void*)thr_batch_kernel<5>,
                                   (const void*)thr_batch_kernel<6>, (const void*)thr_batch_kernel<7>};
    for (const void* k : batch_kernels) {
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int pre_waves_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)thr_bounds_kernel, 64 * PRE_WG, 0) != hipSuccess) return (int)PRE_WG;
    return n > 0 ? (int)PRE_WG * n : (int)PRE_WG;
}

int batch_blocks_per_cu(size_t smem) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)thr_batch_kernel<WIN_BATCH>, BLOCK, smem) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

hipError_t launch_query(const QueryDev& q, const BitmapDev* table, uint32_t* ticket, uint32_t epoch, uint32_t* err,
                        hipStream_t s, uint32_t pred_kind, const InlineIds* ids) {
    size_t smem = tile_smem_bytes(q.N);
    if (!q.ids && (q.pd || !ids || q.N > IDS_INLINE)) return hipErrorInvalidValue;
    static const InlineIds none{};
    const InlineIds& iv = ids ? *ids : none;
    if (!q.pd && use_looped(q.variant, q.N, q.T))
        hipLaunchKernelGGL(thr_query_looped_kernel, dim3(q.tiles), dim3(BLOCK), smem, s, q, table, ticket, epoch, err, iv);
    else if (!q.pd)
        hipLaunchKernelGGL(thr_query_kernel, dim3(q.tiles), dim3(BLOCK), smem, s, q, table, ticket, epoch, err, iv);
    else if (pred_kind == PRED_HIST)
        hipLaunchKernelGGL(thr_query_hist_kernel, dim3(q.tiles), dim3(BLOCK), smem, s, q, table, ticket, epoch, err);
    else if (pred_kind == PRED_MAXCOUNT)
        hipLaunchKernelGGL(thr_query_max_kernel, dim3(q.tiles), dim3(BLOCK), smem, s, q, table, ticket, epoch, err);
    else hipLaunchKernelGGL(thr_query_sym_kernel, dim3(q.tiles), dim3(BLOCK), smem, s, q, table, ticket, epoch, err);
    return hipGetLastError();
}

hipError_t launch_batch(const QueryDev* qs, const uint32_t* qtile, const uint32_t* tq, uint32_t nq, uint32_t total,
                        const BitmapDev* table, uint32_t* work, const uint32_t* epoch_ptr, uint32_t* err, uint32_t grid,
                        size_t smem, hipStream_t s, uint32_t* item_t, int win_batch, uint32_t* pre, uint32_t* pmask,
                        uint32_t* list) {
    if ((pre == nullptr) != (list == nullptr) || (pre && !pmask)) return hipErrorInvalidValue;
    if (pre)
        hipLaunchKernelGGL(thr_bounds_kernel, dim3((total + PRE_WG - 1) / PRE_WG), dim3(64 * PRE_WG), 0, s, qs, qtile, tq, nq, total, epoch_ptr,
                           pre, pmask, list, work, item_t, nq ? total / nq : 0u);   // tiles per query
    switch (win_batch) {
        case 4: hipLaunchKernelGGL(thr_batch_kernel<4>, dim3(grid), dim3(BLOCK), smem, s, qs, qtile, tq, nq, table, work,
                                   epoch_ptr, err, item_t, pre, pmask, list); break;
        case 5: hipLaunchKernelGGL(thr_batch_kernel<5>, dim3(grid), dim3(BLOCK), smem, s, qs, qtile, tq, nq, table, work,
                                   epoch_ptr, err, item_t, pre, pmask, list); break;
        case 6: hipLaunchKernelGGL(thr_batch_kernel<6>, dim3(grid), dim3(BLOCK), smem, s, qs, qtile, tq, nq, table, work,
                                   epoch_ptr, err, item_t, pre, pmask, list); break;
        case 7: hipLaunchKernelGGL(thr_batch_kernel<7>, dim3(grid), dim3(BLOCK), smem, s, qs, qtile, tq, nq, table, work,
                                   epoch_ptr, err, item_t, pre, pmask, list); break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(scan_batch_kernel, dim3(nq), dim3(SCAN_THREADS), 0, s, qs, epoch_ptr, err);
    hipLaunchKernelGGL(place_batch_kernel, dim3((total + 3) / 4), dim3(256), 0, s, qs, qtile, tq, total, epoch_ptr, err);
    return hipGetLastError();
}

hipError_t launch_bump(uint32_t* work, hipStream_t s) {
    hipLaunchKernelGGL(bump_epoch_kernel, dim3(1), dim3(1), 0, s, work);
    return hipGetLastError();
}

#ifdef EWT_PHASE_TIMING
extern "C" int ewt_debug_set_phase_buffer(void* p) {
    return (int)hipMemcpyToSymbol(HIP_SYMBOL(ewt_phase_buf), &p, sizeof(p));
}
#endif

hipError_t launch_zero_len(uint64_t* out_n, hipStream_t s) {
    hipLaunchKernelGGL(zero_len_kernel, dim3(1), dim3(1), 0, s, out_n);
    return hipGetLastError();
}

}  // namespace ewt
