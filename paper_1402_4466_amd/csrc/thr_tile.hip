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

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
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
__device__ __forceinline__ void ripple_add(uint64_t* planes, uint32_t pos, uint64_t v, int P) {
    for (int p = 0; p < P && v; ++p) {
        uint64_t old = atomicXor((unsigned long long*)&planes[p * TW + pos], (unsigned long long)v);
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

__device__ __forceinline__ Seg locate(const BitmapDev& B, uint32_t t, uint32_t tS, uint32_t tE, uint32_t tiles) {
    Seg s;
    const uint2 l0 = gp(B.loc)[t];
    uint32_t pm = l0.x, um = l0.y;
    uint64_t h = gp(B.words)[pm];
    uint32_t f = (uint32_t)(h & 1u), L = (uint32_t)((h >> 1) & 0xFFFFFFFFu), K = (uint32_t)(h >> 33);
    uint32_t fa = max(um, tS), fb = min(um + L, tE);
    s.fa = fa; s.fb = (f && fa < fb) ? fb : fa;
    uint32_t la = max(um + L, tS), lb = min(um + L + K, tE);
    s.cnt = la < lb ? lb - la : 0u;
    s.la = la;
    s.a_lit = pm + 1u + (la - (um + L));
    s.bs = pm + 1u + K;
    s.y0 = um + L + K;
    s.be = s.bs;
    if (t + 1 < tiles) {
        const uint2 l1 = gp(B.loc)[t + 1];
        if (l1.x != pm) {
            uint64_t h2 = gp(B.words)[l1.x];
            uint32_t L2 = (uint32_t)((h2 >> 1) & 0xFFFFFFFFu), K2 = (uint32_t)(h2 >> 33);
            uint32_t lit_start = l1.y + L2;
            uint32_t inlit = tE > lit_start ? min(K2, tE - lit_start) : 0u;
            s.be = l1.x + 1u + inlit;
        }
    } else if (s.bs < B.n_words) {
        s.be = B.n_words;
    }
    s.onefull = f && fa == tS && fb == tE;
    s.zero = (s.fa >= s.fb) && s.cnt == 0 && s.be <= s.bs;
    return s;
}

// One lane walks the markers of [bs, be), starting at a marker whose run starts at y0.
__device__ __forceinline__ void walk_body(const EWT_GLOBAL uint64_t* words, uint32_t bs, uint32_t be,
                                          uint32_t y0, uint32_t tS, uint32_t tE, uint64_t* planes,
                                          int32_t* diff, int P) {
    uint32_t p = bs, u = y0;
    while (p < be && u < tE) {
        uint64_t h = words[p];
        uint32_t f = (uint32_t)(h & 1u), L = (uint32_t)((h >> 1) & 0xFFFFFFFFu), K = (uint32_t)(h >> 33);
        if (f) {
            uint32_t fa = max(u, tS), fb = min(u + L, tE);
            if (fa < fb) { atomicAdd(&diff[fa - tS], 1); atomicAdd(&diff[fb - tS], -1); }
        }
        uint32_t ls = u + L;
        uint32_t la = max(ls, tS), lb = min(ls + K, tE);
        for (uint32_t x = la; x < lb; ++x) ripple_add(planes, x - tS, words[p + 1u + (x - ls)], P);
        p += 1u + K;
        u += L + K;
    }
}

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

// Decode one 64-word window (chunk c) of a compressed stream with one
// wavefront.  M (bit j = word 64c + j is a marker) and uw0 (position where
// word 64c's coverage starts) come from the skip index.  A marker covers L
// fill words and is followed by its K dirty words, so with span = L for a
// marker and 1 for a dirty word, each word starts at uw0 + (exclusive scan of
// the spans): the run start for a marker, the position for a dirty word.
__device__ __forceinline__ uint32_t decode_window(uint64_t v, uint64_t M, uint32_t uw0, bool& is_marker) {
    const int lane = __lane_id();
    is_marker = (M >> lane) & 1ull;
    const uint32_t span = is_marker ? (uint32_t)((v >> 1) & 0xFFFFFFFFu) : 1u;
    return uw0 + wave_incl_scan_dpp(span) - span;
}

// Exclusive prefix of the run-structure aggregate over tiles [0, t), by
// decoupled look-back read 64 predecessors at a time: lane i looks at tile
// base - i; the nearest tile that has published its inclusive prefix ends the
// search, and the local aggregates of the tiles after it are reduced across
// the wavefront (the aggregate is associative).  Called by one whole wavefront.
__device__ Agg lookback(EWT_GLOBAL TileState* st, int t, uint32_t epoch, uint32_t* err) {
    const int lane = __lane_id();
    bool acc_empty = true;
    Agg acc;
    acc.n = 0; acc.lh_pos = 0; acc.lh_out = 0; acc.bits = 0;
    int base = t - 1;
    uint32_t spins = 0;
    while (true) {
        const int j = base - lane;
        Agg vi, vl;
        bool inc = false, loc = false;
        if (j >= 0) {
            inc = agg_fetch(st[j].incl, epoch, vi);
            loc = agg_fetch(st[j].local, epoch, vl);
        }
        const uint64_t incm = __ballot(inc);
        const int linc = incm ? (__ffsll((long long)incm) - 1) : 64;
        const bool need = j >= 0 && lane <= linc;
        const bool ok = !need || inc || loc;
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
        bool empty = !need;
        // tree reduction: lane i + d holds the lower (earlier) tiles
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
                else v = agg_combine(o, v, (uint32_t)(base - lane - d + 1) * (uint32_t)TW);
            }
        }
        Agg R;
        R.n = __shfl(v.n, 0, 64);
        R.lh_pos = __shfl(v.lh_pos, 0, 64);
        R.lh_out = __shfl(v.lh_out, 0, 64);
        R.bits = __shfl(v.bits, 0, 64);
        acc = acc_empty ? R : agg_combine(R, acc, (uint32_t)(base + 1) * (uint32_t)TW);
        acc_empty = false;
        if (linc < 64) return acc;
        base -= 64;
        if (base < 0) {   // tile 0 always publishes an inclusive value: cannot get here
            if (lane == 0) atomicOr(err, 2u);
            return acc;
        }
    }
}

// ---------------------------------------------------------------- the tile

// Misc LDS slots.
constexpr int WIN_BATCH = 8;   // windows grabbed per wavefront at a time

#ifdef EWT_PHASE_TIMING
// Debug builds only: per-tile timestamps of the phase boundaries.
__device__ uint64_t* ewt_phase_buf;
#define EWT_PHASE(k) do { if (threadIdx.x == 0 && ewt_phase_buf) ewt_phase_buf[(size_t)dbg_slot * 8 + (k)] = wall_clock64(); } while (0)
#else
#define EWT_PHASE(k) do { } while (0)
#endif

enum { M_NITEMS = 0, M_NDENSE, M_WINCTR, M_NWIN, M_ONEFULL, M_NONZERO, M_TMP = 8, M_X = 32, M_TOT = 40 };

__device__ void process_tile(const QueryDev& q, const BitmapDev* __restrict__ table, uint32_t t,
                             uint32_t epoch, unsigned char* smem, uint32_t* err, uint32_t dbg_slot) {
    (void)dbg_slot;   // timestamp slot of debug builds
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t N = q.N, T = q.T, U = q.U, tiles = q.tiles;
    const uint32_t tS = t * (uint32_t)TW;
    const uint32_t nPos = min((uint32_t)TW, U - tS);
    const uint32_t tE = tS + nPos;
    const int P = planes_for(N);
    const uint32_t nb = min(N, (uint32_t)BLOCK);
    const uint32_t walk_max = (q.variant >> VAR_WALK_SHIFT) & 255u;
    const uint32_t litwalk_max = (q.variant >> VAR_LITWALK_SHIFT) & 255u;

    uint64_t* planes = (uint64_t*)smem;
    int32_t* diff = (int32_t*)(planes + (size_t)P * TW);
    uint4* items = (uint4*)(diff + TW + 8);
    uint32_t* winp = (uint32_t*)(items + 2 * BLOCK);
    const uint64_t** dense = (const uint64_t**)(winp + 2 * BLOCK + 8);
    uint32_t* misc = (uint32_t*)(dense + BLOCK);
    (void)nb;

    EWT_PHASE(0);
    for (int i = tid; i < P * TW; i += BLOCK) planes[i] = 0;
    for (int i = tid; i < TW + 8; i += BLOCK) diff[i] = 0;
    if (tid < 8) misc[tid] = 0;
    __syncthreads();

    // ---- classify / prune (RBMrg on EWAH, cases 1 and 2, per tile)
    const bool trivial = (T == 0) || (T > N);
    Seg seg;
    if (!trivial) {
        for (uint32_t kb = 0; kb < N; kb += BLOCK) {
            uint32_t k = kb + (uint32_t)tid;
            if (k < N) {
                Seg s = locate(gp(table)[gp(q.ids)[k]], t, tS, tE, tiles);
                if (s.onefull) atomicAdd(&misc[M_ONEFULL], 1u);
                if (!s.zero) atomicAdd(&misc[M_NONZERO], 1u);
                if (kb == 0) seg = s;
            }
        }
    }
    __syncthreads();
    EWT_PHASE(1);
    const uint32_t mode = trivial ? (T == 0 ? 1u : 2u)
                                  : (misc[M_ONEFULL] >= T ? 1u : (misc[M_NONZERO] < T ? 2u : 0u));

    // ---- decode and count
    if (mode == 0) {
        for (uint32_t kb = 0; kb < N; kb += BLOCK) {
            uint32_t k = kb + (uint32_t)tid;
            if (k < N) {
                const uint32_t slot = gp(q.ids)[k];
                const BitmapDev B = gp(table)[slot];
                Seg s = (kb == 0) ? seg : locate(B, t, tS, tE, tiles);
                if (s.fa < s.fb) { atomicAdd(&diff[s.fa - tS], 1); atomicAdd(&diff[s.fb - tS], -1); }
                if (s.cnt) {
                    if ((q.variant & VAR_DENSE) && s.cnt == nPos) {
                        uint32_t j = atomicAdd(&misc[M_NDENSE], 1u);
                        dense[j] = B.words + s.a_lit;
                    } else if (s.cnt <= litwalk_max) {
                        for (uint32_t j = 0; j < s.cnt; ++j) ripple_add(planes, s.la - tS + j, gp(B.words)[s.a_lit + j], P);
                    } else {
                        uint32_t j = atomicAdd(&misc[M_NITEMS], 1u);
                        items[j] = make_uint4(slot, s.a_lit, s.a_lit + s.cnt, s.la | 0x80000000u);
                    }
                }
                if (s.be > s.bs) {
                    if (s.be - s.bs <= walk_max) {
                        walk_body(gp(B.words), s.bs, s.be, s.y0, tS, tE, planes, diff, P);
                    } else {
                        uint32_t j = atomicAdd(&misc[M_NITEMS], 1u);
                        items[j] = make_uint4(slot, s.bs, s.be, 0u);
                    }
                }
            }
            __syncthreads();
            EWT_PHASE(2);
            // window prefix over the cooperative items (two per thread)
            const uint32_t n_items = misc[M_NITEMS];
            uint32_t w2[2] = {0u, 0u};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t i = 2u * (uint32_t)tid + (uint32_t)h;
                if (i < n_items) {
                    uint4 it = items[i];
                    w2[h] = (it.w & 0x80000000u) ? (it.z - it.y + 63u) / 64u : ((it.z - 1u) / 64u - it.y / 64u + 1u);
                }
            }
            uint32_t tot;
            uint32_t ex = block_excl_scan(w2[0] + w2[1], misc + M_TMP, tot);
            if (2u * (uint32_t)tid < n_items) winp[2 * tid] = ex;
            if (2u * (uint32_t)tid + 1u < n_items) winp[2 * tid + 1] = ex + w2[0];
            if (tid == 0) { misc[M_NWIN] = tot; misc[M_WINCTR] = 0; }
            __syncthreads();

            // cooperative windows: one wavefront per 64 compressed words, WIN_BATCH
            // windows per grab, all loads issued before any decoding and the
            // ripple adds of the batch interleaved
            const uint32_t total_w = misc[M_NWIN];
            while (true) {
                uint32_t w0 = 0;
                if (lane == 0) w0 = atomicAdd(&misc[M_WINCTR], (uint32_t)WIN_BATCH);
                w0 = __builtin_amdgcn_readfirstlane(__shfl(w0, 0, 64));
                if (w0 >= total_w) break;
                uint32_t lo = 0, hi = n_items - 1;       // largest i with winp[i] <= w0
                while (lo < hi) {
                    uint32_t mid = (lo + hi + 1) >> 1;
                    if (winp[mid] <= w0) lo = mid; else hi = mid - 1;
                }
                lo = __builtin_amdgcn_readfirstlane(lo);
                uint32_t wi = __builtin_amdgcn_readfirstlane(w0 - winp[lo]);
                uint32_t lo_n = __builtin_amdgcn_readfirstlane(((lo + 1 < n_items) ? winp[lo + 1] : total_w) - winp[lo]);
                uint64_t vs[WIN_BATCH];
                uint64_t ms[WIN_BATCH];
                uint32_t ps[WIN_BATCH];
                uint4 its[WIN_BATCH];
                uint32_t qs[WIN_BATCH];
                uint32_t wis[WIN_BATCH];
                // stage 1: which item and window each batch slot is (wave-uniform)
#pragma unroll
                for (int g = 0; g < WIN_BATCH; ++g) {
                    if (g > 0) {
                        if (wi + 1u >= lo_n && lo + 1 < n_items) {
                            ++lo;
                            wi = 0;
                            lo_n = __builtin_amdgcn_readfirstlane(((lo + 1 < n_items) ? winp[lo + 1] : total_w) - winp[lo]);
                        } else {
                            ++wi;
                        }
                    }
                    uint4 it = items[lo];
                    it.x = __builtin_amdgcn_readfirstlane(it.x);
                    it.y = __builtin_amdgcn_readfirstlane(it.y);
                    it.z = __builtin_amdgcn_readfirstlane(it.z);
                    it.w = __builtin_amdgcn_readfirstlane(it.w);
                    its[g] = it;
                    wis[g] = wi;
                }
                // stage 2: descriptors of the bitmaps involved (scalar loads)
                const uint64_t* wpt[WIN_BATCH];
                const uint64_t* mpt[WIN_BATCH];
                const uint32_t* ppt[WIN_BATCH];
#pragma unroll
                for (int g = 0; g < WIN_BATCH; ++g) {
                    const EWT_GLOBAL BitmapDev* B = gp(table) + its[g].x;
                    wpt[g] = B->words;
                    mpt[g] = B->mmask;
                    ppt[g] = B->mpos;
                }
                // stage 3: all data loads of the batch
#pragma unroll
                for (int g = 0; g < WIN_BATCH; ++g) {
                    const uint4 it = its[g];
                    vs[g] = 0;
                    ms[g] = 0;
                    ps[g] = 0;
                    qs[g] = 0;
                    if (w0 + (uint32_t)g < total_w) {
                        if (it.w & 0x80000000u) {
                            const uint32_t qv = it.y + wis[g] * 64u + (uint32_t)lane;
                            qs[g] = qv;
                            if (qv < it.z) vs[g] = __builtin_nontemporal_load(gp(wpt[g]) + qv);
                        } else {
                            const uint32_t c = (it.y >> 6) + wis[g];
                            const uint32_t qv = c * 64u + (uint32_t)lane;
                            qs[g] = qv;
                            vs[g] = __builtin_nontemporal_load(gp(wpt[g]) + qv);
                            ms[g] = gp(mpt[g])[c];
                            ps[g] = gp(ppt[g])[c];
                        }
                    }
                }
                // decode: position of every dirty word in the tile (or no add)
                uint32_t rp[WIN_BATCH];
#pragma unroll
                for (int g = 0; g < WIN_BATCH; ++g) {
                    const uint4 it = its[g];
                    const uint32_t qv = qs[g];
                    uint64_t v = vs[g];
                    uint32_t r = 0;
                    if (w0 + (uint32_t)g >= total_w) {
                        v = 0;
                    } else if (it.w & 0x80000000u) {
                        if (qv < it.z) r = (it.w & 0x7FFFFFFFu) + (qv - it.y) - tS;
                        else v = 0;
                    } else {
                        bool im;
                        const uint32_t pos = decode_window(v, ms[g], ps[g], im);
                        const bool in = qv >= it.y && qv < it.z;
                        if (in && im && (v & 1ull)) {
                            const uint32_t L = (uint32_t)((v >> 1) & 0xFFFFFFFFu);
                            const uint32_t fa = max(pos, tS), fb = min(pos + L, tE);
                            if (fa < fb) { atomicAdd(&diff[fa - tS], 1); atomicAdd(&diff[fb - tS], -1); }
                        }
                        if (in && !im && pos >= tS && pos < tE) r = pos - tS;
                        else v = 0;
                    }
                    vs[g] = v;
                    rp[g] = r;
                }
                // interleaved ripple-carry adds of the batch
                for (int p = 0; p < P; ++p) {
                    uint64_t any = 0;
#pragma unroll
                    for (int g = 0; g < WIN_BATCH; ++g) {
                        if (vs[g]) {
                            const uint64_t old = atomicXor((unsigned long long*)&planes[p * TW + rp[g]],
                                                           (unsigned long long)vs[g]);
                            vs[g] &= old;
                        }
                        any |= vs[g];
                    }
                    if (!__any(any != 0)) break;
                }
            }
            __syncthreads();

            EWT_PHASE(3);
            // dense rows: Harley-Seal carry-save-adder tree, one lane per word position
            const uint32_t n_dense = misc[M_NDENSE];
            if (n_dense && (uint32_t)tid < nPos) {
                uint64_t R[MAXP];
#pragma unroll
                for (int p = 0; p < MAXP; ++p) R[p] = 0;
                uint32_t d = 0;
                for (; d + 16u <= n_dense; d += 16u) {
                    uint64_t x[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) x[j] = __builtin_nontemporal_load(gp(dense[d + j]) + tid);
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
                for (; d < n_dense; ++d) {
                    uint64_t cy = __builtin_nontemporal_load(gp(dense[d]) + tid);
#pragma unroll
                    for (int p = 0; p < MAXP; ++p) { uint64_t tt = R[p] & cy; R[p] ^= cy; cy = tt; }
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
            if (tid == 0) { misc[M_NITEMS] = 0; misc[M_NDENSE] = 0; }
            __syncthreads();
        }
    }

    EWT_PHASE(4);
    // ---- compare: count >= T - k1 per row, bit-sliced
    uint32_t k1tot;
    int32_t dv = tid < TW ? diff[tid] : 0;
    uint32_t k1 = block_excl_scan((uint32_t)dv, misc + M_TMP, k1tot) + (uint32_t)dv;
    uint64_t o = 0;
    if ((uint32_t)tid < nPos) {
        if (mode == 1) o = ~0ull;
        else if (mode == 2) o = 0;
        else {
            int tp = (int)T - (int)k1;
            if (tp <= 0) o = ~0ull;
            else if (tp >= (1 << P)) o = 0;
            else {
                uint64_t gt = 0, eq = ~0ull;
                for (int p = P - 1; p >= 0; --p) {
                    uint64_t a = planes[p * TW + tid];
                    uint64_t tb = ((tp >> p) & 1) ? ~0ull : 0ull;
                    gt |= eq & a & ~tb;
                    eq &= ~(a ^ tb);
                }
                o = gt | eq;
            }
        }
        if (tS + (uint32_t)tid == U - 1u && q.tail_bits) o &= (1ull << q.tail_bits) - 1ull;
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
        if (t > 0) {
            if (lane == 0) agg_publish(st[t].local, A, epoch);
            X = lookback(st, (int)t, epoch, err);
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
    EWT_PHASE(7);
}

// ----------------------------------------------------------------- kernels

// One query, one workgroup per tile.  Tiles are taken in ticket order so that a
// tile only ever waits for tiles that are already running or done.
__global__ __launch_bounds__(BLOCK) void thr_query_kernel(QueryDev q, const BitmapDev* __restrict__ table,
                                                          uint32_t* ticket, uint32_t epoch, uint32_t* err) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) {
        uint32_t t = atomicAdd(ticket, 1u);
        if (t == q.tiles - 1) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = t;
    }
    __syncthreads();
    process_tile(q, table, s_t, epoch, smem, err, s_t);
}

// Many queries in one persistent launch: workgroups take (query, tile) items
// from a global counter in order.  qtile[i] = first item of query i (qtile[nq] = total).
__global__ __launch_bounds__(BLOCK) void thr_batch_kernel(const QueryDev* __restrict__ qs, const uint32_t* __restrict__ qtile,
                                                          uint32_t nq, const BitmapDev* __restrict__ table,
                                                          uint32_t* work, const uint32_t* epoch_ptr, uint32_t* err) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_item, s_q;
    const uint32_t total = qtile[nq];
    const uint32_t epoch = *epoch_ptr;
    while (true) {
        if (threadIdx.x == 0) {
            uint32_t it = atomicAdd(work, 1u);
            if (it == total + gridDim.x - 1u) __hip_atomic_store(work, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t qi = 0;
            if (it < total) {
                uint32_t lo = 0, hi = nq - 1;
                while (lo < hi) {
                    uint32_t mid = (lo + hi + 1) >> 1;
                    if (qtile[mid] <= it) lo = mid; else hi = mid - 1;
                }
                qi = lo;
            }
            s_item = it;
            s_q = qi;
        }
        __syncthreads();
        const uint32_t it = s_item, qi = s_q;
        if (it >= total) break;
        QueryDev q = qs[qi];
        process_tile(q, table, it - qtile[qi], epoch, smem, err, it);
    }
}

// Next launch tag of a batch; tag 0 (the value of cleared states) is skipped.
// Every launch of a batch rewrites every tile state, so states older than the
// previous launch never survive and the 16-bit tag cycle is safe.
__global__ void bump_epoch_kernel(uint32_t* epoch) {
    uint32_t e = *epoch + 1u;
    if ((e & 0xFFFFu) == 0) e += 1u;
    *epoch = e;
}

// Output for r = 0 (no words).
__global__ void zero_len_kernel(uint64_t* out_n) { *out_n = 0; }

}  // namespace ewt

// ---------------------------------------------------------------- launchers
namespace ewt {

hipError_t set_smem_limits(size_t max_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)thr_query_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)thr_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
}

hipError_t launch_query(const QueryDev& q, const BitmapDev* table, uint32_t* ticket, uint32_t epoch, uint32_t* err,
                        hipStream_t s) {
    size_t smem = tile_smem_bytes(q.N);
    hipLaunchKernelGGL(thr_query_kernel, dim3(q.tiles), dim3(BLOCK), smem, s, q, table, ticket, epoch, err);
    return hipGetLastError();
}

hipError_t launch_batch(const QueryDev* qs, const uint32_t* qtile, uint32_t nq, const BitmapDev* table, uint32_t* work,
                        const uint32_t* epoch_ptr, uint32_t* err, uint32_t grid, size_t smem, hipStream_t s) {
    hipLaunchKernelGGL(thr_batch_kernel, dim3(grid), dim3(BLOCK), smem, s, qs, qtile, nq, table, work, epoch_ptr, err);
    return hipGetLastError();
}

hipError_t launch_bump(uint32_t* epoch, hipStream_t s) {
    hipLaunchKernelGGL(bump_epoch_kernel, dim3(1), dim3(1), 0, s, epoch);
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
