// Tile routine and kernels of the T-of-N threshold query (see thr_device.h for
// the step-by-step description and the paper passages each step follows).
#include "thr_device.h"

namespace ewt {

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

__device__ __forceinline__ void agg_store(Agg* dst, const Agg& a) {
    __hip_atomic_store(&dst->n, a.n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&dst->lh_pos, a.lh_pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&dst->lh_out, a.lh_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&dst->bits, a.bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ Agg agg_load(Agg* src) {
    Agg a;
    a.n = __hip_atomic_load(&src->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.lh_pos = __hip_atomic_load(&src->lh_pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.lh_out = __hip_atomic_load(&src->lh_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.bits = __hip_atomic_load(&src->bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return a;
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
    uint2 l0 = B.loc[t];
    uint32_t pm = l0.x, um = l0.y;
    uint64_t h = B.words[pm];
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
        uint2 l1 = B.loc[t + 1];
        if (l1.x != pm) {
            uint64_t h2 = B.words[l1.x];
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
__device__ __forceinline__ void walk_body(const uint64_t* __restrict__ words, uint32_t bs, uint32_t be,
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

// Decode one 64-word window (chunk c) of a compressed stream with one wavefront.
// Returns for this lane: whether its word is a marker, and its position (literal) or run start (marker).
__device__ __forceinline__ void decode_window(uint64_t v, uint2 sk, volatile uint8_t* wf, bool& is_marker,
                                              uint32_t& pos) {
    const int lane = __lane_id();
    const uint32_t uw0 = sk.x, m0 = sk.y;
    uint64_t M = 0;
    if (m0 < 64u) {
        // next marker offset if this word were a marker, 64 = outside the window
        uint32_t K = (uint32_t)(v >> 33);
        uint32_t nx = (uint32_t)lane + 1u + K;
        uint32_t J0 = nx > 64u ? 64u : nx;
        // pointer doubling: J_r = next^(2^r)
        uint32_t J1 = __shfl(J0, (int)(J0 & 63u), 64); J1 = J0 < 64u ? J1 : 64u;
        uint32_t J2 = __shfl(J1, (int)(J1 & 63u), 64); J2 = J1 < 64u ? J2 : 64u;
        uint32_t J3 = __shfl(J2, (int)(J2 & 63u), 64); J3 = J2 < 64u ? J3 : 64u;
        uint32_t J4 = __shfl(J3, (int)(J3 & 63u), 64); J4 = J3 < 64u ? J4 : 64u;
        uint32_t J5 = __shfl(J4, (int)(J4 & 63u), 64); J5 = J4 < 64u ? J5 : 64u;
        // chain members from m0: {c_0} -> + c_32 -> + c_16, c_48 -> ... -> all
        wf[lane] = (uint32_t)lane == m0 ? 1 : 0;
        __builtin_amdgcn_wave_barrier();
        uint32_t Js[6] = {J0, J1, J2, J3, J4, J5};
#pragma unroll
        for (int r = 5; r >= 0; --r) {
            uint8_t in = wf[lane];
            __builtin_amdgcn_wave_barrier();
            if (in && Js[r] < 64u) wf[Js[r]] = 1;
            __builtin_amdgcn_wave_barrier();
        }
        bool im = wf[lane] != 0;
        __builtin_amdgcn_wave_barrier();
        M = __ballot(im);
    }
    is_marker = (M >> lane) & 1ull;
    uint32_t L = (uint32_t)((v >> 1) & 0xFFFFFFFFu), K = (uint32_t)(v >> 33);
    uint32_t len = is_marker ? L + K : 0u;
    uint32_t ex = wave_incl_scan(len) - len;
    uint32_t um = uw0 + m0 + ex;                 // run start (meaningful for marker lanes)
    uint64_t below = lane == 0 ? 0ull : (M & (~0ull >> (64 - lane)));
    int owner = below ? 63 - __clzll((long long)below) : -1;
    uint32_t ob = __shfl(um + L, owner < 0 ? 0 : owner, 64);
    pos = is_marker ? um : (owner < 0 ? uw0 + (uint32_t)lane : ob + (uint32_t)(lane - owner - 1));
}

// ---------------------------------------------------------------- the tile

// Misc LDS slots.
enum { M_NITEMS = 0, M_NDENSE, M_WINCTR, M_NWIN, M_ONEFULL, M_NONZERO, M_TMP = 8, M_X = 32, M_TOT = 40 };

__device__ void process_tile(const QueryDev& q, const BitmapDev* __restrict__ table, uint32_t t,
                             uint32_t epoch, unsigned char* smem, uint32_t* err) {
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
    volatile uint8_t* wflags = (volatile uint8_t*)(misc + 64) + wave * 64;
    (void)nb;

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
                Seg s = locate(table[q.ids[k]], t, tS, tE, tiles);
                if (s.onefull) atomicAdd(&misc[M_ONEFULL], 1u);
                if (!s.zero) atomicAdd(&misc[M_NONZERO], 1u);
                if (kb == 0) seg = s;
            }
        }
    }
    __syncthreads();
    const uint32_t mode = trivial ? (T == 0 ? 1u : 2u)
                                  : (misc[M_ONEFULL] >= T ? 1u : (misc[M_NONZERO] < T ? 2u : 0u));

    // ---- decode and count
    if (mode == 0) {
        for (uint32_t kb = 0; kb < N; kb += BLOCK) {
            uint32_t k = kb + (uint32_t)tid;
            if (k < N) {
                uint32_t slot = q.ids[k];
                const BitmapDev& B = table[slot];
                Seg s = (kb == 0) ? seg : locate(B, t, tS, tE, tiles);
                if (s.fa < s.fb) { atomicAdd(&diff[s.fa - tS], 1); atomicAdd(&diff[s.fb - tS], -1); }
                if (s.cnt) {
                    if ((q.variant & VAR_DENSE) && s.cnt == nPos) {
                        uint32_t j = atomicAdd(&misc[M_NDENSE], 1u);
                        dense[j] = B.words + s.a_lit;
                    } else if (s.cnt <= litwalk_max) {
                        for (uint32_t j = 0; j < s.cnt; ++j) ripple_add(planes, s.la - tS + j, B.words[s.a_lit + j], P);
                    } else {
                        uint32_t j = atomicAdd(&misc[M_NITEMS], 1u);
                        items[j] = make_uint4(slot, s.a_lit, s.a_lit + s.cnt, s.la | 0x80000000u);
                    }
                }
                if (s.be > s.bs) {
                    if (s.be - s.bs <= walk_max) {
                        walk_body(B.words, s.bs, s.be, s.y0, tS, tE, planes, diff, P);
                    } else {
                        uint32_t j = atomicAdd(&misc[M_NITEMS], 1u);
                        items[j] = make_uint4(slot, s.bs, s.be, 0u);
                    }
                }
            }
            __syncthreads();
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

            // cooperative windows: one wavefront per 64 compressed words
            const uint32_t total_w = misc[M_NWIN];
            while (true) {
                uint32_t w = 0;
                if (lane == 0) w = atomicAdd(&misc[M_WINCTR], 1u);
                w = __shfl(w, 0, 64);
                if (w >= total_w) break;
                uint32_t lo = 0, hi = n_items - 1;       // largest i with winp[i] <= w
                while (lo < hi) {
                    uint32_t mid = (lo + hi + 1) >> 1;
                    if (winp[mid] <= w) lo = mid; else hi = mid - 1;
                }
                uint4 it = items[lo];
                uint32_t wi = w - winp[lo];
                const BitmapDev& B = table[it.x];
                if (it.w & 0x80000000u) {
                    uint32_t la = it.w & 0x7FFFFFFFu;
                    uint32_t qv = it.y + wi * 64u + (uint32_t)lane;
                    if (qv < it.z) ripple_add(planes, la + (qv - it.y) - tS, B.words[qv], P);
                } else {
                    uint32_t c = (it.y >> 6) + wi;
                    uint32_t qv = c * 64u + (uint32_t)lane;
                    uint64_t v = B.words[qv];
                    uint2 sk = B.skip[c];
                    bool im;
                    uint32_t pos;
                    decode_window(v, sk, wflags, im, pos);
                    if (qv >= it.y && qv < it.z) {
                        if (im) {
                            if (v & 1ull) {
                                uint32_t L = (uint32_t)((v >> 1) & 0xFFFFFFFFu);
                                uint32_t fa = max(pos, tS), fb = min(pos + L, tE);
                                if (fa < fb) { atomicAdd(&diff[fa - tS], 1); atomicAdd(&diff[fb - tS], -1); }
                            }
                        } else if (pos >= tS && pos < tE) {
                            ripple_add(planes, pos - tS, v, P);
                        }
                    }
                }
            }
            __syncthreads();

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
                    for (int j = 0; j < 16; ++j) x[j] = __builtin_nontemporal_load(dense[d + j] + tid);
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
                    uint64_t cy = __builtin_nontemporal_load(dense[d] + tid);
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

    if (tid == 0) {
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
        TileState* st = q.state;
        Agg X;
        X.n = 0; X.lh_pos = 0; X.lh_out = 0; X.bits = 3u << 2;
        Agg I = A;
        if (t > 0) {
            agg_store(&st[t].local, A);
            __hip_atomic_store(&st[t].flag_local, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            bool acc_empty = true;
            Agg acc = A;
            int j = (int)t - 1;
            uint32_t spins = 0;
            while (true) {
                uint32_t fi = __hip_atomic_load(&st[j].flag_incl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (fi == epoch) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    Agg Ij = agg_load(&st[j].incl);
                    X = acc_empty ? Ij : agg_combine(Ij, acc, (uint32_t)(j + 1) * TW);
                    break;
                }
                uint32_t fl = __hip_atomic_load(&st[j].flag_local, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (fl == epoch) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    Agg Lj = agg_load(&st[j].local);
                    acc = acc_empty ? Lj : agg_combine(Lj, acc, (uint32_t)(j + 1) * TW);
                    acc_empty = false;
                    --j;
                    if (j < 0) { atomicOr(err, 2u); break; }   // tile 0 always publishes its inclusive value
                    continue;
                }
                if (++spins > (1u << 24)) { atomicOr(err, 1u); break; }
                __builtin_amdgcn_s_sleep(2);
            }
            I = agg_combine(X, A, tS);
        }
        agg_store(&st[t].incl, I);
        __hip_atomic_store(&st[t].flag_incl, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        misc[M_X + 0] = X.n; misc[M_X + 1] = X.lh_pos; misc[M_X + 2] = X.lh_out; misc[M_X + 3] = X.bits;
        misc[M_TOT] = I.n;
    }
    __syncthreads();

    const uint32_t Xn = misc[M_X + 0], Xlh_pos = misc[M_X + 1], Xlh_out = misc[M_X + 2], Xbits = misc[M_X + 3];
    const uint32_t total = misc[M_TOT];
    const uint32_t c0 = clsA[0];
    const uint32_t merge = (t > 0 && c0 != 2u && ((Xbits >> 2) & 3u) == c0) ? 1u : 0u;
    const uint64_t cap = q.cap;
    uint64_t* out = q.out;
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
        *q.out_n = total;
    }
    __syncthreads();
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
    process_tile(q, table, s_t, epoch, smem, err);
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
        process_tile(q, table, it - qtile[qi], epoch, smem, err);
    }
}

__global__ void bump_epoch_kernel(uint32_t* epoch) { *epoch += 1u; }

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

hipError_t launch_zero_len(uint64_t* out_n, hipStream_t s) {
    hipLaunchKernelGGL(zero_len_kernel, dim3(1), dim3(1), 0, s, out_n);
    return hipGetLastError();
}

}  // namespace ewt
