// Host runtime of the threshold library: registration (validation, locator and
// skip-index construction), device bitmap table, per-stream query contexts,
// batched plans with HIP graph capture, and the C ABI of include/ewahthr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ewahthr.h"
#include "thr_device.h"

using namespace ewt;

namespace {

thread_local std::string g_err;

ewah_status fail(ewah_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(EWAH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

struct Arena {
    void* d = nullptr;
    int refs = 0;
};

}  // namespace

namespace ewt {
void set_last_error(const std::string& msg) { g_err = msg; }
}

struct ewah_bitmap {
    BitmapDev dev;        // device pointers into the arena
    uint32_t slot = 0;    // index in the device table
    ewah_stats stats{};
    Arena* arena = nullptr;
};

namespace {

struct Ctx {                       // per-stream query state
    uint32_t* d_ids = nullptr;
    size_t ids_cap = 0;
    uint32_t* h_ids = nullptr;     // pinned staging
    TileState* d_state = nullptr;
    size_t state_cap = 0;
    uint32_t* d_ticket = nullptr;  // tile order of the single-query kernel
    uint32_t epoch = 0;
    hipEvent_t ev = nullptr;       // staging buffer free once this completes
    unsigned long long* d_acc = nullptr;   // opt-threshold: largest count / output row count / histogram
    unsigned long long* h_acc = nullptr;   // pinned copy (MAXN + 1 values)
    // single threshold queries of many tiles run through the persistent batched kernel
    // (staged tiles, scan, placement) as a batch of one: its own tile states, staging area
    // and item-to-query map (all zeros); its work words (epoch, item counters) are
    // uploaded with the input slots, the epoch counted here
    TileState* d_state1 = nullptr;
    uint64_t* d_stage1 = nullptr;
    uint32_t* d_tq1 = nullptr;
    size_t tiles1_cap = 0;
    uint32_t epoch1 = 0;
};

struct Lib {
    bool ready = false;
    int device = -1;
    uint32_t n_cu = 0;
    size_t max_smem = 0;
    std::vector<BitmapDev> table;  // host mirror
    std::vector<float4> stats;     // per slot: (n_words, n_literals, popcount, run_count) for features
    std::vector<uint32_t> free_slots;
    BitmapDev* d_table = nullptr;
    float4* d_stats = nullptr;
    size_t d_table_cap = 0;
    uint32_t* d_err = nullptr;
    std::map<hipStream_t, Ctx> ctx;
    unsigned char* na_ptr = nullptr;   // device address of `scratch` (allocation-free entry point)
    uint32_t na_epoch = 0;             // launch tag of its tile states
};

Lib g;

// ------------------------------------------- scratch of the allocation-free query
// ewah_threshold_noalloc keeps its per-call device state in this file-scope array
// instead of allocating: the tile-order ticket, the input slots and one tile state
// per tile.  The host never uses the array's name as an address: ewah_init takes its
// device address with hipGetSymbolAddress (g.na_ptr) and every kernel argument and
// copy uses that.  Every call on the GPU shares it, so calls that overlap race.
constexpr uint32_t NA_MAX_TILES = 4096;   // 2^27 rows per query
constexpr size_t NA_SLOTS_OFF = 256;      // bytes; the ticket is the first word
constexpr size_t NA_STATE_OFF = NA_SLOTS_OFF + (((size_t)(MAXN + 1) * 4 + 255) & ~(size_t)255);
constexpr size_t NA_BYTES = NA_STATE_OFF + (size_t)NA_MAX_TILES * sizeof(TileState);
static __device__ __align__(256) unsigned char scratch[NA_BYTES];
static uint32_t na_host_slots[MAXN + 1];   // host staging of the input slots (static: no allocation)

// Clears n 64-bit words (used instead of hipMemsetAsync so that the call stays capturable).
__global__ void clear_words_kernel(uint64_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

ewah_status ensure_ready() {
    if (!g.ready) return fail(EWAH_EINVAL, "ewah_init() has not been called");
    return EWAH_OK;
}

// ----------------------------------------------------------- index builder

struct Built {
    std::vector<uint4> loc;    // per tile boundary: covering marker index, its run start, the marker word
    std::vector<uint4> desc;   // per CHUNK words: marker mask (lo, hi), position of the chunk's first word
    std::vector<uint4> pres;   // per tile PV_COARSE records: 4-word groups holding a dirty word or a one-fill
    std::vector<uint32_t> presq;   // pq_words(tiles) words: per-word, quarter-word and 8-row groups holding a one
    std::vector<uint16_t> qcnt;    // per tile: number of quarter-word groups holding a one
    ewah_stats st{};
};

// Sets bits [lo, hi] of a bit vector.
void set_bits(std::vector<uint64_t>& v, uint64_t lo, uint64_t hi) {
    for (uint64_t w = lo / 64; w <= hi / 64; ++w) {
        const uint64_t a = (w == lo / 64) ? lo % 64 : 0, b = (w == hi / 64) ? hi % 64 : 63;
        const uint64_t m = (b == 63 ? ~0ull : ((1ull << (b + 1)) - 1)) & (~0ull << a);
        v[w] |= m;
    }
}

inline uint64_t popc64(uint64_t x) { return (uint64_t)__builtin_popcountll(x); }

// Validates one stream and builds its locator and skip index (one pass).
ewah_status build_index(const uint64_t* w, uint64_t nw, uint64_t n_bits, Built& b) {
    const uint64_t U = (n_bits + 63) / 64;
    if (U >= (1ull << 31)) return fail(EWAH_EINVAL, "n_bits too large (U must be < 2^31 words)");
    if (nw >= (1ull << 32) - 2 * CHUNK) return fail(EWAH_EINVAL, "stream too long (n_words must be < 2^32 - 128)");
    const uint64_t tiles = (U + TW - 1) / TW;
    const uint64_t nchunks = (nw + CHUNK - 1) / CHUNK;
    b.loc.assign(tiles + 1, make_uint4(0, 0, 0, 0));
    std::vector<uint64_t> gbits((tiles * TW + 63) / 64 + 1, 0);   // words holding a dirty word or a one-fill
    std::vector<uint64_t> qbits(tiles * TW * 4 / 64 + 1, 0);       // quarter words holding a one
    std::vector<uint64_t> obits(tiles * TW * 8 / 64 + 1, 0);       // 8-row groups holding a one
    b.desc.assign(nchunks, make_uint4(0, 0, 0, 0));
    const uint64_t tailmask = (n_bits % 64) ? ((1ull << (n_bits % 64)) - 1) : ~0ull;
    ewah_stats& st = b.st;
    st = ewah_stats{};
    st.n_bits = n_bits;
    st.n_words = nw;
    uint64_t p = 0, u = 0;
    int prev_bit = -1;   // last row bit, for RunCount
    auto run_bits = [&](uint64_t v, uint64_t nbits) {  // count runs over the next nbits rows of v
        if (nbits == 0) return;
        uint64_t m = nbits == 64 ? ~0ull : ((1ull << nbits) - 1);
        uint64_t x = v & m;
        uint64_t shifted = (x << 1) | (uint64_t)(prev_bit < 0 ? (x & 1) : (uint64_t)prev_bit);
        uint64_t changes = (x ^ shifted) & m;
        st.run_count += popc64(changes) + (prev_bit < 0 ? 1 : 0);
        prev_bit = (int)((x >> (nbits - 1)) & 1);
    };
    while (p < nw) {
        const uint64_t m = w[p];
        const uint64_t f = m & 1, L = (m >> 1) & 0xFFFFFFFFull, K = m >> 33;
        if (L > U - u) return fail(EWAH_EFORMAT, "marker at word " + std::to_string(p) + ": fill run past the end");
        if (K > nw - p - 1) return fail(EWAH_EFORMAT, "marker at word " + std::to_string(p) + ": stream ends inside its literal run");
        if (K > U - u - L) return fail(EWAH_EFORMAT, "marker at word " + std::to_string(p) + ": literal run past the end");
        st.n_markers++;
        const uint64_t c = p / CHUNK;
        const uint64_t bit = p - c * CHUNK;
        if (bit < 32) b.desc[c].x |= 1u << bit;
        else b.desc[c].y |= 1u << (bit - 32);
        if (p % CHUNK == 0) b.desc[c].z = (uint32_t)u;
        if (f && L) {
            set_bits(gbits, u, u + L - 1);
            set_bits(qbits, 4 * u, 4 * (u + L) - 1);
            set_bits(obits, 8 * u, 8 * (u + L) - 1);
        }
        if (K) set_bits(gbits, u + L, u + L + K - 1);
        if (L + K > 0) {
            const uint4 e = make_uint4((uint32_t)p, (uint32_t)u, (uint32_t)m, (uint32_t)(m >> 32));
            for (uint64_t t = (u + TW - 1) / TW; t * TW < u + L + K && t < tiles; ++t) b.loc[t] = e;
        }
        // statistics over the fill run
        if (L) {
            uint64_t last_in_run = (u + L == U) ? 1 : 0;
            if (f) {
                st.one_fill_words += L;
                st.popcount += (L - last_in_run) * 64 + (last_in_run ? popc64(tailmask) : 0);
            }
            // a fill run contributes one run boundary at most
            uint64_t rows = (L - last_in_run) * 64 + (last_in_run ? (n_bits - (U - 1) * 64) : 0);
            if (rows) {
                if (prev_bit != (int)f) st.run_count++;
                prev_bit = (int)f;
            }
        }
        for (uint64_t i = 0; i < K; ++i) {
            const uint64_t q = p + 1 + i, pos = u + L + i;
            if (q % CHUNK == 0) b.desc[q / CHUNK].z = (uint32_t)pos;
            uint64_t v = w[q];
            const uint64_t nbits = (pos == U - 1) ? (n_bits - (U - 1) * 64) : 64;
            if (pos == U - 1) v &= tailmask;
            for (uint64_t j = 0; j < 4; ++j)
                if ((v >> (16 * j)) & 0xFFFFull) qbits[(4 * pos + j) / 64] |= 1ull << ((4 * pos + j) % 64);
            for (uint64_t j = 0; j < 8; ++j)
                if ((v >> (8 * j)) & 0xFFull) obits[(8 * pos + j) / 64] |= 1ull << ((8 * pos + j) % 64);
            st.popcount += popc64(v);
            run_bits(v, nbits);
        }
        st.n_literals += K;
        p += 1 + K;
        u += L + K;
    }
    if (u != U) return fail(EWAH_EFORMAT, "stream covers " + std::to_string(u) + " words, expected " + std::to_string(U));
    if (tiles) b.loc[tiles] = make_uint4((uint32_t)nw, (uint32_t)U, 0, 0);
    // per tile: the quarter bits and their count, and the word bits ORed over each group of 4 words
    b.presq.assign(pq_words((uint32_t)tiles), 0u);
    b.qcnt.assign(tiles, 0u);
    b.pres.assign(tiles * PV_COARSE, make_uint4(0, 0, 0, 0));
    static_assert(NQ_TILE < 65536, "quarter counts fit 16 bits");
    static_assert(TW % 64 == 0 && GW_COARSE == 4, "presence record packing");
    for (uint64_t t = 0; t < tiles; ++t) {
        const uint64_t* qw = qbits.data() + t * (NQ_TILE / 64);
        uint32_t* wrec = b.presq.data() + t * PQ_W_TILE;
        uint32_t* qrec = b.presq.data() + pq_quarters((uint32_t)tiles) + t * PQ_Q_TILE;
        uint32_t nq = 0;
        for (int k = 0; k < NQ_TILE / 64; ++k) {
            qrec[2 * k] = (uint32_t)qw[k];
            qrec[2 * k + 1] = (uint32_t)(qw[k] >> 32);
            nq += (uint32_t)popc64(qw[k]);
        }
        b.qcnt[t] = (uint16_t)nq;
        const uint64_t* ow = obits.data() + t * (NO_TILE / 64);
        // the 32 bits of words 4 m .. 4 m + 3 (m = 2 l + h) go to word l of half h: the halves of
        // the words of lanes l = 0 .. 63 each lie together
        for (int k = 0; k < NO_TILE / 64; ++k) {
            for (int e = 0; e < 2; ++e) {
                const int m = 2 * k + e;
                b.presq[pq_octets((uint32_t)tiles, (uint32_t)(m % 2)) + t * PQ_O_TILE + m / 2] =
                    (uint32_t)(ow[k] >> (32 * e));
            }
        }
        for (int wd = 0; wd < TW; ++wd)   // a word holds a one iff one of its quarters does
            if ((qw[wd / 16] >> (4 * (wd % 16))) & 15ull) wrec[wd / 32] |= 1u << (wd % 32);
        const uint64_t* w = gbits.data() + t * (TW / 64);
        uint32_t c[4 * PV_COARSE] = {};
        for (int k = 0; k < TW / 64; ++k) {
            uint64_t y = w[k] | (w[k] >> 1);
            y |= y >> 2;   // bit 4i: OR of bits 4i .. 4i + 3
            uint32_t q = 0;
            for (int i = 0; i < 16; ++i) q |= (uint32_t)((y >> (4 * i)) & 1u) << i;
            c[k / 2] |= q << (16 * (k % 2));
        }
        for (int v = 0; v < PV_COARSE; ++v)
            b.pres[t * PV_COARSE + v] = make_uint4(c[4 * v], c[4 * v + 1], c[4 * v + 2], c[4 * v + 3]);
    }
    st.index_bytes = (b.loc.size() + b.desc.size() + b.pres.size()) * sizeof(uint4) + b.presq.size() * 4 +
                     b.qcnt.size() * 2;
    return EWAH_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

ewah_status table_sync() {
    // grow the device table if needed and upload the host mirror
    if (g.table.size() > g.d_table_cap) {
        size_t cap = std::max<size_t>(1024, g.d_table_cap * 2);
        while (cap < g.table.size()) cap *= 2;
        HIPCHK(hipDeviceSynchronize());
        BitmapDev* nd = nullptr;
        float4* ns = nullptr;
        HIPCHK(hipMalloc(&nd, cap * sizeof(BitmapDev)));
        HIPCHK(hipMalloc(&ns, cap * sizeof(float4)));
        if (g.d_table) HIPCHK(hipFree(g.d_table));
        if (g.d_stats) HIPCHK(hipFree(g.d_stats));
        g.d_table = nd;
        g.d_stats = ns;
        g.d_table_cap = cap;
    }
    if (!g.table.empty()) {
        HIPCHK(hipMemcpy(g.d_table, g.table.data(), g.table.size() * sizeof(BitmapDev), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(g.d_stats, g.stats.data(), g.stats.size() * sizeof(float4), hipMemcpyHostToDevice));
    }
    return EWAH_OK;
}

uint32_t alloc_slot() {
    if (!g.free_slots.empty()) {
        uint32_t s = g.free_slots.back();
        g.free_slots.pop_back();
        return s;
    }
    g.table.push_back(BitmapDev{});
    g.stats.push_back(make_float4(0, 0, 0, 0));
    return (uint32_t)(g.table.size() - 1);
}

ewah_status get_ctx(hipStream_t s, Ctx** out) {
    auto it = g.ctx.find(s);
    if (it == g.ctx.end()) {
        Ctx c;
        HIPCHK(hipMalloc(&c.d_ticket, 256));
        HIPCHK(hipMemset(c.d_ticket, 0, 256));
        HIPCHK(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
        it = g.ctx.emplace(s, c).first;
    }
    *out = &it->second;
    return EWAH_OK;
}

ewah_status ctx_reserve(Ctx& c, hipStream_t s, size_t n_ids, size_t tiles) {
    if (n_ids > c.ids_cap || tiles > c.state_cap) {
        HIPCHK(hipStreamSynchronize(s));
        if (n_ids > c.ids_cap) {
            size_t cap = std::max<size_t>(n_ids, 1024);
            if (c.d_ids) HIPCHK(hipFree(c.d_ids));
            if (c.h_ids) HIPCHK(hipHostFree(c.h_ids));
            HIPCHK(hipMalloc(&c.d_ids, cap * 4));
            HIPCHK(hipHostMalloc(&c.h_ids, cap * 4, hipHostMallocDefault));
            c.ids_cap = cap;
        }
        if (tiles > c.state_cap) {
            size_t cap = std::max<size_t>(tiles, 1024);
            if (c.d_state) HIPCHK(hipFree(c.d_state));
            HIPCHK(hipMalloc(&c.d_state, cap * sizeof(TileState)));
            HIPCHK(hipMemset(c.d_state, 0, cap * sizeof(TileState)));
            c.state_cap = cap;
            c.epoch = 0;
        }
    }
    return EWAH_OK;
}

// Buffers of the one-query batched run for queries of up to `tiles` tiles.
ewah_status ctx_reserve_batched(Ctx& c, hipStream_t s, size_t tiles) {
    if (tiles > c.tiles1_cap) {
        HIPCHK(hipStreamSynchronize(s));   // earlier runs on this stream may still use the old buffers
        if (c.d_state1) HIPCHK(hipFree(c.d_state1));
        if (c.d_stage1) HIPCHK(hipFree(c.d_stage1));
        if (c.d_tq1) HIPCHK(hipFree(c.d_tq1));
        c.d_state1 = nullptr; c.d_stage1 = nullptr; c.d_tq1 = nullptr; c.tiles1_cap = 0;
        const size_t cap = std::max<size_t>(tiles, 1024);
        HIPCHK(hipMalloc(&c.d_state1, cap * sizeof(TileState)));
        HIPCHK(hipMemset(c.d_state1, 0, cap * sizeof(TileState)));
        if (hipMalloc(&c.d_stage1, cap * STAGE_WORDS * sizeof(uint64_t)) != hipSuccess)
            return fail(EWAH_ENOMEM, "staging area of " + std::to_string(cap * STAGE_WORDS * 8) + " bytes");
        HIPCHK(hipMalloc(&c.d_tq1, cap * 4));
        HIPCHK(hipMemset(c.d_tq1, 0, cap * 4));
        c.tiles1_cap = cap;
        c.epoch1 = 0;   // fresh states hold tag 0, which no epoch takes
    }
    return EWAH_OK;
}

// Resident workgroups of the batched kernel at a given LDS size (cached per size).
uint32_t batch_resident(size_t smem) {
    static std::map<size_t, uint32_t> cache;
    auto it = cache.find(smem);
    if (it != cache.end()) return it->second;
    const uint32_t r = g.n_cu * (uint32_t)batch_blocks_per_cu(smem);
    cache[smem] = r;
    return r;
}

}  // namespace

// ------------------------------------------------------------------- C ABI

extern "C" {

const char* ewah_last_error(void) { return g_err.c_str(); }

ewah_status ewah_init(int device) {
    if (g.ready) {
        if (device != g.device) return fail(EWAH_EINVAL, "library already initialised on another device");
        return EWAH_OK;
    }
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(EWAH_EINVAL, "no such device");
    HIPCHK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(EWAH_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    g.device = device;
    g.n_cu = (uint32_t)prop.multiProcessorCount;
    g.max_smem = prop.sharedMemPerBlock;
    size_t need = tile_smem_bytes(MAXN);
    if (g.max_smem < need)
        return fail(EWAH_EDEVICE, "device offers " + std::to_string(g.max_smem) + " B of LDS per workgroup, need " +
                                      std::to_string(need));
    HIPCHK(set_smem_limits(need));
    HIPCHK(hipMalloc(&g.d_err, 256));
    HIPCHK(hipMemset(g.d_err, 0, 256));
    // device address of the allocation-free entry point's scratch on this device
    void* na = nullptr;
    HIPCHK(hipGetSymbolAddress(&na, HIP_SYMBOL(scratch)));
    if (!na) return fail(EWAH_EDEVICE, "no device address for the scratch array");
    g.na_ptr = (unsigned char*)na;
    g.na_epoch = 0;
    g.ready = true;
    return EWAH_OK;
}

uint32_t ewah_num_cus(void) { return g.n_cu; }

uint64_t ewah_output_bound(uint64_t n_bits, uint64_t sum_input_words) {
    uint64_t U = (n_bits + 63) / 64;
    if (U == 0) return 0;
    return std::min<uint64_t>(U + 1, sum_input_words + 1);
}

uint32_t ewah_variant_code(int dense, uint32_t walk, uint32_t litwalk) { return var_make(dense != 0, walk, litwalk); }
uint32_t ewah_variant_code_ex(int dense, uint32_t walk, uint32_t litwalk, int looped) {
    return var_make(dense != 0, walk, litwalk, looped != 0);
}
uint32_t ewah_variant_code_full(int dense, uint32_t walk, uint32_t litwalk, int looped, uint32_t gate) {
    return var_make(dense != 0, walk, litwalk, looped != 0, gate);
}
uint32_t ewah_default_variant(void) { return var_make(true, 8, 8); }

ewah_status ewah_register_many(const ewah_view* v, uint32_t count, int on_device, ewah_bitmap** out) {
    ewah_status st = ensure_ready();
    if (st) return st;
    if (count == 0) return EWAH_OK;
    if (!v || !out) return fail(EWAH_EINVAL, "null argument");
    std::vector<Built> built(count);
    std::vector<std::vector<uint64_t>> host(count);
    std::vector<const uint64_t*> src(count);
    for (uint32_t i = 0; i < count; ++i) {
        if (v[i].n_words && !v[i].words) return fail(EWAH_EINVAL, "null words pointer");
        src[i] = v[i].words;
        if (on_device && v[i].n_words) {
            host[i].resize(v[i].n_words);
            HIPCHK(hipMemcpy(host[i].data(), v[i].words, v[i].n_words * 8, hipMemcpyDeviceToHost));
            src[i] = host[i].data();
        }
    }
    // validation and index building, one bitmap at a time on up to 16 host threads; the
    // first failing bitmap (lowest index) is reported
    {
        const uint32_t nt = std::max(1u, std::min({16u, std::thread::hardware_concurrency(), count}));
        std::atomic<uint32_t> next{0};
        std::mutex mu;
        uint32_t bad = count;
        ewah_status bad_st = EWAH_OK;
        std::string bad_msg;
        auto work = [&]() {
            for (;;) {
                const uint32_t i = next.fetch_add(1);
                if (i >= count) return;
                const ewah_status e = build_index(src[i], v[i].n_words, v[i].n_bits, built[i]);
                if (e) {
                    std::lock_guard<std::mutex> lk(mu);
                    if (i < bad) { bad = i; bad_st = e; bad_msg = g_err; }   // g_err of this thread
                }
            }
        };
        std::vector<std::thread> pool;
        for (uint32_t k = 1; k < nt; ++k) pool.emplace_back(work);
        work();
        for (auto& th : pool) th.join();
        if (bad < count) return fail(bad_st, "bitmap " + std::to_string(bad) + ": " + bad_msg);
    }
    // one device arena per call; per bitmap [words padded to CHUNK, plus CHUNK zero words |
    // skip index | locator | 4-word-group presence | quarter-word presence], each part 256-byte aligned.  The image is assembled on the host
    // and uploaded in pieces of at most kStage bytes.
    constexpr size_t kStage = 256ull << 20;
    struct Layout { size_t words, desc, loc, pres, presq, qcnt, end; };
    std::vector<Layout> lay(count);
    size_t total = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const size_t nch = std::max<size_t>(built[i].desc.size(), 1);
        Layout& l = lay[i];
        l.words = total;
        l.desc = l.words + align256((nch * CHUNK + CHUNK) * 8);
        l.loc = l.desc + align256(nch * 16);
        l.pres = l.loc + align256(built[i].loc.size() * 16);
        l.presq = l.pres + align256(std::max<size_t>(built[i].pres.size(), 1) * 16);
        l.qcnt = l.presq + align256(std::max<size_t>(built[i].presq.size(), 1) * 4);
        l.end = l.qcnt + align256(std::max<size_t>(built[i].qcnt.size(), 1) * 2);
        total = l.end;
    }
    Arena* arena = new Arena();
    if (hipMalloc(&arena->d, total) != hipSuccess) {
        delete arena;
        return fail(EWAH_ENOMEM, "device allocation of " + std::to_string(total) + " bytes failed");
    }
    if (((uintptr_t)arena->d + total) >> 48) {   // window addresses carry flags in their top 16 bits
        (void)hipFree(arena->d);
        delete arena;
        return fail(EWAH_EDEVICE, "device address above 2^48");
    }
    std::vector<char> stage;
    for (uint32_t i0 = 0; i0 < count;) {
        uint32_t i1 = i0 + 1;
        while (i1 < count && lay[i1].end - lay[i0].words <= kStage) ++i1;
        const size_t base = lay[i0].words, len = lay[i1 - 1].end - base;
        stage.assign(len, 0);
        for (uint32_t i = i0; i < i1; ++i) {
            const uint64_t* src = on_device ? host[i].data() : v[i].words;
            if (v[i].n_words) std::memcpy(stage.data() + (lay[i].words - base), src, v[i].n_words * 8);
            if (!built[i].desc.empty())
                std::memcpy(stage.data() + (lay[i].desc - base), built[i].desc.data(), built[i].desc.size() * 16);
            std::memcpy(stage.data() + (lay[i].loc - base), built[i].loc.data(), built[i].loc.size() * 16);
            if (!built[i].pres.empty())
                std::memcpy(stage.data() + (lay[i].pres - base), built[i].pres.data(), built[i].pres.size() * 16);
            if (!built[i].presq.empty())
                std::memcpy(stage.data() + (lay[i].presq - base), built[i].presq.data(), built[i].presq.size() * 4);
            if (!built[i].qcnt.empty())
                std::memcpy(stage.data() + (lay[i].qcnt - base), built[i].qcnt.data(), built[i].qcnt.size() * 2);
        }
        HIPCHK(hipMemcpy((char*)arena->d + base, stage.data(), len, hipMemcpyHostToDevice));
        i0 = i1;
    }
    for (uint32_t i = 0; i < count; ++i) {
        char* base = (char*)arena->d;
        ewah_bitmap* b = new ewah_bitmap();
        b->dev.words = (const uint64_t*)(base + lay[i].words);
        b->dev.loc = (const uint4*)(base + lay[i].loc);
        b->dev.desc = (const uint4*)(base + lay[i].desc);
        b->dev.pres = (const uint4*)(base + lay[i].pres);
        b->dev.presq = (const uint32_t*)(base + lay[i].presq);
        b->dev.qcnt = (const uint16_t*)(base + lay[i].qcnt);
        b->dev.n_words = (uint32_t)v[i].n_words;
        b->dev.U = (uint32_t)((v[i].n_bits + 63) / 64);
        b->stats = built[i].st;
        b->arena = arena;
        arena->refs++;
        b->slot = alloc_slot();
        g.table[b->slot] = b->dev;
        g.stats[b->slot] = make_float4((float)b->stats.n_words, (float)b->stats.n_literals, (float)b->stats.popcount,
                                       (float)b->stats.run_count);
        out[i] = b;
    }
    return table_sync();
}

ewah_status ewah_register(const ewah_view* v, int on_device, ewah_bitmap** out) {
    return ewah_register_many(v, 1, on_device, out);
}

void ewah_release(ewah_bitmap* b) {
    if (!b) return;
    g.table[b->slot] = BitmapDev{};
    g.stats[b->slot] = make_float4(0, 0, 0, 0);
    g.free_slots.push_back(b->slot);
    if (--b->arena->refs == 0) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b->arena->d);
        delete b->arena;
    }
    delete b;
}

ewah_status ewah_get_stats(const ewah_bitmap* b, ewah_stats* out) {
    if (!b || !out) return fail(EWAH_EINVAL, "null argument");
    *out = b->stats;
    return EWAH_OK;
}

const uint64_t* ewah_device_words(const ewah_bitmap* b) { return b ? b->dev.words : nullptr; }

}  // extern "C"

namespace {

// One query on the single-query kernel: count >= T, or the predicate pred (host copy,
// uploaded with the input slots) when it is not null.
ewah_status run_plain(const ewah_bitmap* const* in, uint32_t n, uint32_t T, const PredDev* pred,
                      uint64_t* out_words_dev, uint64_t out_cap, uint64_t* out_n_words_dev, uint32_t variant,
                      void* hip_stream, const uint32_t* tab = nullptr) {
    ewah_status st = ensure_ready();
    if (st) return st;
    // the largest-count and histogram passes write no output
    const bool writes = !pred || (pred->kind != PRED_MAXCOUNT && pred->kind != PRED_HIST);
    if ((n && !in) || (writes && !out_n_words_dev)) return fail(EWAH_EINVAL, "null argument");
    if (n > MAXN) return fail(EWAH_EINVAL, "at most " + std::to_string(MAXN) + " inputs per query");
    if (n == 0) return fail(EWAH_EINVAL, "n = 0: the number of rows is undefined without an input");
    uint64_t n_bits = 0, sum_words = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!in[i]) return fail(EWAH_EINVAL, "null bitmap at index " + std::to_string(i));
        if (i == 0) n_bits = in[i]->stats.n_bits;
        else if (in[i]->stats.n_bits != n_bits) return fail(EWAH_EINVAL, "inputs have different n_bits");
        sum_words += in[i]->stats.n_words;
    }
    const uint64_t bound = writes ? ewah_output_bound(n_bits, sum_words) : 0;
    if (out_cap < bound)
        return fail(EWAH_ENOSPC, "out_cap " + std::to_string(out_cap) + " < bound " + std::to_string(bound));
    if (bound && !out_words_dev) return fail(EWAH_EINVAL, "null output");
    hipStream_t s = (hipStream_t)hip_stream;
    const uint32_t U = (uint32_t)((n_bits + 63) / 64);
    if (U == 0) {
        if (writes) HIPCHK(launch_zero_len(out_n_words_dev, s));
        return EWAH_OK;
    }
    const uint32_t tiles = (U + TW - 1) / TW;
    // staging: the n slots, then (8-byte aligned) the predicate record
    const size_t pred_off = ((size_t)n + 1) & ~(size_t)1;
    size_t n_stage = pred ? pred_off + sizeof(PredDev) / 4 : n;
    // a general table (PRED_TABLE) follows the predicate record: bit c = f(c), c = 0..n
    const size_t tab_off = n_stage;
    const size_t tab_words = (pred && pred->kind == PRED_TABLE) ? ((size_t)n + 32) / 32 : 0;
    if (tab_words && !tab) return fail(EWAH_EINVAL, "null function table");
    n_stage += tab_words;
    // A threshold query with more tiles than resident workgroups runs as a
    // batch of one on the persistent kernel: its tiles are taken in turn from per-XCD
    // ranges and placed by a scan, instead of one workgroup per tile chained by
    // look-back.  Its query record, item range {0, tiles} and work words (epoch and
    // cleared item counters, 64-byte aligned) are staged after the slots.
    const size_t smem = tile_smem_bytes(n);
    const uint32_t resident = batch_resident(smem);
    const bool batched = !pred && tiles > resident;
    size_t q_off = 0, qt_off = 0, w_off = 0;
    if (batched) {
        q_off = (n_stage + 1) & ~(size_t)1;          // 8-byte aligned
        qt_off = q_off + sizeof(QueryDev) / 4;
        w_off = (qt_off + 2 + 15) & ~(size_t)15;     // 64-byte aligned
        n_stage = w_off + WORK_WORDS;
    }
    Ctx* c = nullptr;
    st = get_ctx(s, &c);
    if (st) return st;
    st = ctx_reserve(*c, s, n_stage, tiles);
    if (st) return st;
    if (batched) {
        st = ctx_reserve_batched(*c, s, tiles);
        if (st) return st;
    }
    QueryDev q{};
    q.ids = c->d_ids;
    q.out = out_words_dev;
    q.out_n = out_n_words_dev;
    q.state = batched ? c->d_state1 : c->d_state;
    q.stage = batched ? c->d_stage1 : nullptr;   // the single-query kernel writes its output in place
    q.cap = out_cap;
    q.N = n;
    q.T = pred ? pred->tz : T;
    q.U = U;
    q.tiles = tiles;
    q.tail_bits = (uint32_t)(n_bits % 64);
    // default variant of a single threshold query: the unary counter at T <= 2 (an add
    // stops within two levels; measured faster there), else the library default
    const uint32_t T_eff = pred ? pred->tz : T;
    q.variant = variant ? variant
                        : ((!pred && T_eff >= 1u && T_eff <= 2u) ? var_make(false, 8, 8, true) : ewah_default_variant());
    q.pd = pred ? (const PredDev*)(c->d_ids + pred_off) : nullptr;
    if (!batched && !pred && n <= IDS_INLINE) {
        // the slots travel in the kernel arguments: nothing to upload, nothing to wait for
        InlineIds iv;
        for (uint32_t i = 0; i < n; ++i) iv.v[i] = in[i]->slot;
        q.ids = nullptr;
        if ((++c->epoch & 0xFFFFu) == 0) {   // 16-bit tags wrapped: clear stale states
            hipLaunchKernelGGL(clear_words_kernel, dim3(256), dim3(256), 0, s, (uint64_t*)c->d_state,
                               c->state_cap * sizeof(TileState) / 8);
            HIPCHK(hipGetLastError());
            c->epoch = 1;
        }
        HIPCHK(launch_query(q, g.d_table, c->d_ticket, c->epoch, g.d_err, s, PRED_THRESHOLD, &iv));
        return EWAH_OK;
    }
    HIPCHK(hipEventSynchronize(c->ev));   // previous upload from the staging buffer is done
    for (uint32_t i = 0; i < n; ++i) c->h_ids[i] = in[i]->slot;
    if (pred) {
        PredDev pc = *pred;
        if (tab_words) {
            pc.tab = (const uint32_t*)(c->d_ids + tab_off);
            std::memcpy(c->h_ids + tab_off, tab, tab_words * 4);
        }
        std::memcpy(c->h_ids + pred_off, &pc, sizeof(PredDev));
    }
    if (batched) {
        std::memcpy(c->h_ids + q_off, &q, sizeof(QueryDev));
        c->h_ids[qt_off] = 0u;
        c->h_ids[qt_off + 1] = tiles;
        uint32_t e = c->epoch1 + 1u;   // 16-bit state tags: skip tag 0
        if ((e & 0xFFFFu) == 0) e += 1u;
        c->epoch1 = e;
        std::memset(c->h_ids + w_off, 0, WORK_WORDS * 4);
        c->h_ids[w_off + 1] = e;
    }
    HIPCHK(hipMemcpyAsync(c->d_ids, c->h_ids, n_stage * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(c->ev, s));
    if (batched) {
        uint32_t* work = c->d_ids + w_off;
        HIPCHK(launch_batch((const QueryDev*)(c->d_ids + q_off), c->d_ids + qt_off, c->d_tq1, 1u, tiles, g.d_table,
                            work, work + 1, g.d_err, resident, smem, s));
        return EWAH_OK;
    }
    if ((++c->epoch & 0xFFFFu) == 0) {   // 16-bit tags wrapped: clear stale states
        hipLaunchKernelGGL(clear_words_kernel, dim3(256), dim3(256), 0, s, (uint64_t*)c->d_state,
                           c->state_cap * sizeof(TileState) / 8);
        HIPCHK(hipGetLastError());
        c->epoch = 1;
    }
    HIPCHK(launch_query(q, g.d_table, c->d_ticket, c->epoch, g.d_err, s, pred ? pred->kind : (uint32_t)PRED_THRESHOLD));
    return EWAH_OK;
}

// Runs one query whose predicate record accumulates into the stream's accumulator
// (n_values words, cleared first) and returns the accumulated values (synchronous).
ewah_status run_accumulate(const ewah_bitmap* const* in, uint32_t n, PredDev& pd, uint64_t* out_words_dev,
                           uint64_t out_cap, uint64_t* out_n_words_dev, hipStream_t s, uint64_t* values,
                           uint32_t n_values = 1) {
    Ctx* c = nullptr;
    ewah_status st = get_ctx(s, &c);
    if (st) return st;
    if (n_values == 0 || n_values > MAXN + 1) return fail(EWAH_EINVAL, "accumulator size");
    if (!c->d_acc) {
        HIPCHK(hipMalloc(&c->d_acc, (MAXN + 1) * 8));
        HIPCHK(hipHostMalloc(&c->h_acc, (MAXN + 1) * 8, hipHostMallocDefault));
    }
    HIPCHK(hipMemsetAsync(c->d_acc, 0, (size_t)n_values * 8, s));
    pd.acc = c->d_acc;
    st = run_plain(in, n, pd.tz, &pd, out_words_dev, out_cap, out_n_words_dev, 0, s);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(c->h_acc, c->d_acc, (size_t)n_values * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(values, c->h_acc, (size_t)n_values * 8);
    return EWAH_OK;
}

// Count histogram: hist[c] = rows with exactly c of the n inputs set, c = 0..n (synchronous).
ewah_status count_histogram(const ewah_bitmap* const* in, uint32_t n, uint64_t* hist, hipStream_t s) {
    if (!hist) return fail(EWAH_EINVAL, "null histogram");
    if (n == 0 || !in) return fail(EWAH_EINVAL, "n = 0: the number of rows is undefined without an input");
    if (n > MAXN) return fail(EWAH_EINVAL, "at most " + std::to_string(MAXN) + " inputs per query");
    if (!in[0]) return fail(EWAH_EINVAL, "null bitmap at index 0");
    PredDev pd{};
    pd.kind = PRED_HIST;
    pd.tz = 1;
    ewah_status st = run_accumulate(in, n, pd, nullptr, 0, nullptr, s, hist, n + 1);
    if (st) return st;
    uint64_t set = 0;
    for (uint32_t c = 1; c <= n; ++c) set += hist[c];
    hist[0] = in[0]->stats.n_bits - set;
    return EWAH_OK;
}

// Device form of a symmetric function given by its table f[0..n]: the runs of counts
// giving 1 as intervals (at most MAX_IV), parity, or else the table itself as bits (tab).
ewah_status pred_from_table(const uint8_t* f, uint32_t n, PredDev& pd, std::vector<uint32_t>& tab) {
    pd = PredDev{};
    uint32_t k = 0;
    bool fits = true;
    for (uint32_t c = 0; c <= n; ++c) {
        if (!f[c] || (c > 0 && f[c - 1])) continue;
        uint32_t e = c;
        while (e < n && f[e + 1]) ++e;
        if (k == (uint32_t)MAX_IV) { fits = false; break; }
        pd.iv[2 * k] = c;
        pd.iv[2 * k + 1] = e;
        ++k;
    }
    uint32_t tz = 1;
    while (tz <= n && (f[tz] != 0) == (f[0] != 0)) ++tz;
    pd.tz = tz;
    pd.v0 = f[0] ? 1u : 0u;
    if (fits) {
        pd.kind = PRED_INTERVALS;
        pd.n_iv = k;
        return EWAH_OK;
    }
    bool odd = true, even = true;
    for (uint32_t c = 0; c <= n; ++c) {
        odd = odd && ((f[c] != 0) == ((c & 1u) != 0));
        even = even && ((f[c] != 0) == ((c & 1u) == 0));
    }
    if (odd || even) {
        pd = PredDev{};
        pd.kind = odd ? PRED_ODD : PRED_EVEN;
        pd.tz = 1;
        pd.v0 = even ? 1u : 0u;
        return EWAH_OK;
    }
    // any other table: looked up per row (bit c of the table is f(c))
    pd.kind = PRED_TABLE;
    pd.n_iv = 0;
    tab.assign(((size_t)n + 32) / 32, 0u);
    for (uint32_t c = 0; c <= n; ++c)
        if (f[c]) tab[c >> 5] |= 1u << (c & 31u);
    return EWAH_OK;
}

}  // namespace

extern "C" {

ewah_status ewah_threshold_v(const ewah_bitmap* const* in, uint32_t n, uint32_t T, uint64_t* out_words_dev,
                             uint64_t out_cap, uint64_t* out_n_words_dev, uint32_t variant, void* hip_stream) {
    return run_plain(in, n, T, nullptr, out_words_dev, out_cap, out_n_words_dev, variant, hip_stream);
}

ewah_status ewah_threshold(const ewah_bitmap* const* in, uint32_t n, uint32_t T, uint64_t* out_words_dev,
                           uint64_t out_cap, uint64_t* out_n_words_dev, void* hip_stream) {
    return run_plain(in, n, T, nullptr, out_words_dev, out_cap, out_n_words_dev, 0, hip_stream);
}

ewah_status ewah_threshold_noalloc(const ewah_bitmap* const* in, uint32_t n, uint32_t T, uint64_t* out_words_dev,
                                   uint64_t out_cap, uint64_t* out_n_words_dev, void* hip_stream) {
    ewah_status st = ensure_ready();
    if (st) return st;
    if (!in || !out_n_words_dev) return fail(EWAH_EINVAL, "null argument");
    if (n == 0) return fail(EWAH_EINVAL, "n = 0: the number of rows is undefined without an input");
    if (n > MAXN) return fail(EWAH_EINVAL, "at most " + std::to_string(MAXN) + " inputs per query");
    uint64_t n_bits = 0, sum_words = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!in[i]) return fail(EWAH_EINVAL, "null bitmap at index " + std::to_string(i));
        if (i == 0) n_bits = in[i]->stats.n_bits;
        else if (in[i]->stats.n_bits != n_bits) return fail(EWAH_EINVAL, "inputs have different n_bits");
        sum_words += in[i]->stats.n_words;
    }
    const uint64_t bound = ewah_output_bound(n_bits, sum_words);
    if (out_cap < bound)
        return fail(EWAH_ENOSPC, "out_cap " + std::to_string(out_cap) + " < bound " + std::to_string(bound));
    if (bound && !out_words_dev) return fail(EWAH_EINVAL, "null output");
    hipStream_t s = (hipStream_t)hip_stream;
    const uint64_t U = (n_bits + 63) / 64;
    if (U == 0) {
        HIPCHK(launch_zero_len(out_n_words_dev, s));
        return EWAH_OK;
    }
    const uint64_t tiles = (U + TW - 1) / TW;
    if (tiles > NA_MAX_TILES)
        return fail(EWAH_EINVAL, "ewah_threshold_noalloc: " + std::to_string(tiles) + " tiles of " + std::to_string(TW) +
                                     " words; its static scratch holds at most " + std::to_string(NA_MAX_TILES) +
                                     " (n_bits <= " + std::to_string((uint64_t)NA_MAX_TILES * TW * 64) + ")");
    uint32_t* d_ticket = (uint32_t*)g.na_ptr;
    uint32_t* d_slots = (uint32_t*)(g.na_ptr + NA_SLOTS_OFF);
    TileState* d_state = (TileState*)(g.na_ptr + NA_STATE_OFF);
    // tile states carry a 16-bit launch tag; on a wrap the stale states are cleared
    if ((++g.na_epoch & 0xFFFFu) == 0) {
        hipLaunchKernelGGL(clear_words_kernel, dim3(256), dim3(256), 0, s, (uint64_t*)d_state,
                           (size_t)NA_MAX_TILES * sizeof(TileState) / 8);
        HIPCHK(hipGetLastError());
        g.na_epoch = 1;
    }
    // input slots: in the kernel arguments for up to IDS_INLINE inputs, else a pageable
    // copy, staged by the runtime before the call returns, so the static host buffer is
    // free for the next call
    InlineIds iv;
    if (n <= IDS_INLINE) {
        for (uint32_t i = 0; i < n; ++i) iv.v[i] = in[i]->slot;
    } else {
        for (uint32_t i = 0; i < n; ++i) na_host_slots[i] = in[i]->slot;
        HIPCHK(hipMemcpyAsync(d_slots, na_host_slots, (size_t)n * 4, hipMemcpyHostToDevice, s));
    }
    QueryDev q{};
    q.ids = n <= IDS_INLINE ? nullptr : d_slots;
    q.out = out_words_dev;
    q.out_n = out_n_words_dev;
    q.state = d_state;
    q.stage = nullptr;
    q.cap = out_cap;
    q.N = n;
    q.T = T;
    q.U = (uint32_t)U;
    q.tiles = (uint32_t)tiles;
    q.tail_bits = (uint32_t)(n_bits % 64);
    q.variant = (T >= 1u && T <= 2u) ? var_make(false, 8, 8, true) : ewah_default_variant();
    q.pd = nullptr;
    q.bms = nullptr;
    HIPCHK(launch_query(q, g.d_table, d_ticket, g.na_epoch, g.d_err, s, PRED_THRESHOLD, &iv));
    return EWAH_OK;
}

ewah_status ewah_opt_threshold(const ewah_bitmap* const* in, uint32_t n, uint64_t K, uint64_t* out_words_dev,
                               uint64_t out_cap, uint64_t* out_n_words_dev, uint32_t* T_out, void* hip_stream) {
    if (!T_out) return fail(EWAH_EINVAL, "null T_out");
    if (n && in && in[0] && (K == 0 || K > in[0]->stats.n_bits))
        return fail(EWAH_EINVAL, "K must be in [1, n_bits]");
    hipStream_t s = (hipStream_t)hip_stream;
    ewah_status st;
    uint32_t best = 0;
    if (K == 1) {
        // the largest row count M (one pass, branch and bound over the tiles): the rows of
        // count M exist (T = 0 if no row is set)
        PredDev pd{};
        pd.kind = PRED_MAXCOUNT;
        pd.tz = 1;
        uint64_t M = 0;
        st = run_accumulate(in, n, pd, out_words_dev, out_cap, out_n_words_dev, s, &M);
        if (st) return st;
        best = (uint32_t)M;
    } else {
        // the count histogram (one pass): the largest T whose suffix sum reaches K; T = 0
        // gives all n_bits >= K rows
        if (n > MAXN) return fail(EWAH_EINVAL, "at most " + std::to_string(MAXN) + " inputs per query");
        std::vector<uint64_t> hist((size_t)n + 1);
        st = count_histogram(in, n, hist.data(), s);
        if (st) return st;
        uint64_t above = 0;
        for (uint32_t T = n; T >= 1; --T) {
            above += hist[T];
            if (above >= K) { best = T; break; }
        }
    }
    *T_out = best;
    return run_plain(in, n, best, nullptr, out_words_dev, out_cap, out_n_words_dev, 0, hip_stream);
}

ewah_status ewah_count_histogram(const ewah_bitmap* const* in, uint32_t n, uint64_t* hist, void* hip_stream) {
    ewah_status st = ensure_ready();
    if (st) return st;
    return count_histogram(in, n, hist, (hipStream_t)hip_stream);
}

ewah_status ewah_symmetric(const ewah_bitmap* const* in, uint32_t n, const uint8_t* f, uint32_t f_len,
                           uint64_t* out_words_dev, uint64_t out_cap, uint64_t* out_n_words_dev, void* hip_stream) {
    if (!f) return fail(EWAH_EINVAL, "null function table");
    if (f_len != n + 1) return fail(EWAH_EINVAL, "the function table needs n + 1 entries (counts 0..n)");
    if (n > MAXN) return fail(EWAH_EINVAL, "at most " + std::to_string(MAXN) + " inputs per query");
    PredDev pd;
    std::vector<uint32_t> tab;
    ewah_status st = pred_from_table(f, n, pd, tab);
    if (st) return st;
    return run_plain(in, n, pd.tz, &pd, out_words_dev, out_cap, out_n_words_dev, 0, hip_stream,
                     tab.empty() ? nullptr : tab.data());
}

ewah_status ewah_device_errors(uint32_t* flags) {
    ewah_status st = ensure_ready();
    if (st) return st;
    HIPCHK(hipDeviceSynchronize());
    uint32_t v = 0;
    HIPCHK(hipMemcpy(&v, g.d_err, 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemset(g.d_err, 0, 4));
    if (flags) *flags = v;
    return EWAH_OK;
}

}  // extern "C"

// ------------------------------------------------------------------- batches

struct ewah_batch {
    std::vector<QueryDev> h_qs;
    QueryDev* d_qs = nullptr;
    uint32_t* d_qtile = nullptr;
    uint32_t* d_ids = nullptr;
    BitmapDev* d_bms = nullptr;    // every query's input descriptors, in the order of d_ids
    TileState* d_state = nullptr;
    uint64_t* d_stage = nullptr;   // STAGE_WORDS per tile of every query
    uint32_t* d_tq = nullptr;      // query of every (query, tile) item
    uint32_t total = 0;            // (query, tile) items
    uint32_t* d_work = nullptr;    // WORK_WORDS words: epoch at [1], per-XCD item counters
    uint32_t* d_codes = nullptr;   // variant codes for ewah_batch_select
    float* d_feat = nullptr;       // features [nq][16] and predictions [nq][16] of ewah_batch_select_model
    float* d_pred = nullptr;
    uint32_t* d_itemt = nullptr;   // per-item busy ticks of ewah_batch_time_queries
    uint32_t* d_pre = nullptr;     // per item: result of the bounds pre-pass (PRE_*)
    uint32_t* d_pmask = nullptr;   // per item: PRE_MASK_WORDS words of its word mask
    uint32_t* d_list = nullptr;    // the items the pre-pass leaves to the tile routine, per XCD
    std::vector<uint32_t> h_codes; // their host copy (upload only on change)
    uint64_t n_bits = 0;
    uint32_t nq = 0;
    uint32_t grid = 0;
    int win_batch = 6;             // windows per wavefront batch of the persistent kernel (4..7)
    int prepass = 1;               // bounds pre-pass before the persistent launch
    size_t smem = 0;
    int use_graph = 1;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// pre-pass buffers of a batch's launches (null: no pre-pass)
uint32_t* pre_of(const ewah_batch* b) { return b->prepass ? b->d_pre : nullptr; }
uint32_t* list_of(const ewah_batch* b) { return b->prepass ? b->d_list : nullptr; }
constexpr uint32_t PRE_MIN_ITEMS = 65536;   // default: the pre-pass for batches of at least this many items

ewah_status batch_build_graph(ewah_batch* b) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    if (!b->use_graph) return EWAH_OK;
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = launch_bump(b->d_work, b->cap_stream);
    hipError_t e2 = launch_batch(b->d_qs, b->d_qtile, b->d_tq, b->nq, b->total, g.d_table, b->d_work, b->d_work + 1,
                                 g.d_err, b->grid, b->smem, b->cap_stream, nullptr, b->win_batch, pre_of(b), b->d_pmask,
                                 list_of(b));
    hipError_t e3 = hipStreamEndCapture(b->cap_stream, &b->graph);
    HIPCHK(e1);
    HIPCHK(e2);
    HIPCHK(e3);
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return EWAH_OK;
}

}  // namespace

extern "C" {

ewah_status ewah_batch_plan(const ewah_bitmap* const* pool, uint32_t pool_n, const ewah_query* q, uint32_t nq,
                            const ewah_batch_config* cfg, ewah_batch** out) {
    ewah_status st = ensure_ready();
    if (st) return st;
    if (!pool || !q || !out || nq == 0) return fail(EWAH_EINVAL, "null argument or empty batch");
    uint64_t n_bits = 0;
    for (uint32_t i = 0; i < pool_n; ++i) {
        if (!pool[i]) return fail(EWAH_EINVAL, "null pool bitmap");
        if (i == 0) n_bits = pool[i]->stats.n_bits;
        else if (pool[i]->stats.n_bits != n_bits) return fail(EWAH_EINVAL, "pool bitmaps have different n_bits");
    }
    const uint32_t U = (uint32_t)((n_bits + 63) / 64);
    if (U == 0) return fail(EWAH_EINVAL, "batched queries need n_bits > 0");
    const uint32_t tiles = (U + TW - 1) / TW;
    std::unique_ptr<ewah_batch> b(new ewah_batch());
    b->nq = nq;
    std::vector<uint32_t> ids;
    std::vector<uint32_t> qtile(nq + 1, 0);
    std::vector<size_t> id_off(nq);
    uint32_t maxN = 1;
    uint64_t items = 0;   // (query, tile) items, summed in 64 bits and checked before anything is allocated
    for (uint32_t i = 0; i < nq; ++i) {
        if (q[i].n == 0 || q[i].n > MAXN || !q[i].idx || !q[i].out_n_words_dev || !q[i].out_words_dev)
            return fail(EWAH_EINVAL, "query " + std::to_string(i) + ": bad arguments");
        uint64_t sum = 0;
        id_off[i] = ids.size();
        for (uint32_t k = 0; k < q[i].n; ++k) {
            uint32_t j = q[i].idx[k];
            if (j >= pool_n) return fail(EWAH_EINVAL, "query " + std::to_string(i) + ": pool index out of range");
            ids.push_back(pool[j]->slot);
            sum += pool[j]->stats.n_words;
        }
        uint64_t bound = ewah_output_bound(n_bits, sum);
        if (q[i].out_cap < bound)
            return fail(EWAH_ENOSPC, "query " + std::to_string(i) + ": out_cap below bound " + std::to_string(bound));
        maxN = std::max(maxN, q[i].n);
        items += tiles;
        if (items >= (1ull << 31))
            return fail(EWAH_EINVAL, "too many tiles in one batch (at most 2^31 - 1 (query, tile) items)");
        qtile[i + 1] = (uint32_t)items;
    }
    HIPCHK(hipMalloc(&b->d_ids, ids.size() * 4));
    HIPCHK(hipMemcpy(b->d_ids, ids.data(), ids.size() * 4, hipMemcpyHostToDevice));
    {
        std::vector<BitmapDev> bmsv(ids.size());
        for (size_t k = 0; k < ids.size(); ++k) bmsv[k] = g.table[ids[k]];
        HIPCHK(hipMalloc(&b->d_bms, std::max<size_t>(bmsv.size(), 1) * sizeof(BitmapDev)));
        HIPCHK(hipMemcpy(b->d_bms, bmsv.data(), bmsv.size() * sizeof(BitmapDev), hipMemcpyHostToDevice));
    }
    HIPCHK(hipMalloc(&b->d_state, (size_t)qtile[nq] * sizeof(TileState)));
    HIPCHK(hipMemset(b->d_state, 0, (size_t)qtile[nq] * sizeof(TileState)));
    if (hipMalloc(&b->d_stage, (size_t)qtile[nq] * STAGE_WORDS * sizeof(uint64_t)) != hipSuccess)
        return fail(EWAH_ENOMEM, "staging area of " + std::to_string((size_t)qtile[nq] * STAGE_WORDS * 8) + " bytes");
    {
        std::vector<uint32_t> tq(qtile[nq]);
        for (uint32_t i = 0; i < nq; ++i)
            for (uint32_t j = qtile[i]; j < qtile[i + 1]; ++j) tq[j] = i;
        HIPCHK(hipMalloc(&b->d_tq, std::max<size_t>(tq.size(), 1) * 4));
        if (!tq.empty()) HIPCHK(hipMemcpy(b->d_tq, tq.data(), tq.size() * 4, hipMemcpyHostToDevice));
        b->total = qtile[nq];
    }
    HIPCHK(hipMalloc(&b->d_qtile, (nq + 1) * 4));
    HIPCHK(hipMemcpy(b->d_qtile, qtile.data(), (nq + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&b->d_pre, (size_t)qtile[nq] * 4));
    HIPCHK(hipMalloc(&b->d_pmask, (size_t)qtile[nq] * PRE_MASK_WORDS * 4));
    HIPCHK(hipMalloc(&b->d_list, (size_t)qtile[nq] * 4));
    HIPCHK(hipMalloc(&b->d_work, WORK_WORDS * 4));
    HIPCHK(hipMemset(b->d_work, 0, WORK_WORDS * 4));
    HIPCHK(hipMalloc(&b->d_codes, 64 * 4));
    b->n_bits = n_bits;
    b->h_qs.resize(nq);
    for (uint32_t i = 0; i < nq; ++i) {
        QueryDev& d = b->h_qs[i];
        d.ids = b->d_ids + id_off[i];
        d.bms = b->d_bms + id_off[i];
        d.out = q[i].out_words_dev;
        d.out_n = q[i].out_n_words_dev;
        d.state = b->d_state + qtile[i];
        d.stage = b->d_stage + (size_t)qtile[i] * STAGE_WORDS;
        d.cap = q[i].out_cap;
        d.N = q[i].n;
        d.T = q[i].T;
        d.U = U;
        d.tiles = tiles;
        d.tail_bits = (uint32_t)(n_bits % 64);
        d.variant = q[i].variant ? q[i].variant : ewah_default_variant();
        d.pd = nullptr;   // batches hold threshold queries
    }
    HIPCHK(hipMalloc(&b->d_qs, nq * sizeof(QueryDev)));
    HIPCHK(hipMemcpy(b->d_qs, b->h_qs.data(), nq * sizeof(QueryDev), hipMemcpyHostToDevice));
    b->smem = tile_smem_bytes(maxN);
    b->prepass = b->total >= PRE_MIN_ITEMS ? 1 : 0;
    b->grid = (cfg && cfg->grid) ? cfg->grid : g.n_cu * (uint32_t)batch_blocks_per_cu(b->smem);
    b->use_graph = cfg ? cfg->use_graph : 1;
    st = batch_build_graph(b.get());
    if (st) return st;
    *out = b.release();
    return EWAH_OK;
}

ewah_status ewah_batch_run(ewah_batch* b, void* hip_stream) {
    if (!b) return fail(EWAH_EINVAL, "null batch");
    hipStream_t s = (hipStream_t)hip_stream;
    if (b->exec) {
        HIPCHK(hipGraphLaunch(b->exec, s));
    } else {
        HIPCHK(launch_bump(b->d_work, s));
        HIPCHK(launch_batch(b->d_qs, b->d_qtile, b->d_tq, b->nq, b->total, g.d_table, b->d_work, b->d_work + 1, g.d_err,
                            b->grid, b->smem, s, nullptr, b->win_batch, pre_of(b), b->d_pmask, list_of(b)));
    }
    return EWAH_OK;
}

ewah_status ewah_batch_set_variants(ewah_batch* b, const uint32_t* variants) {
    if (!b || !variants) return fail(EWAH_EINVAL, "null argument");
    for (uint32_t i = 0; i < b->nq; ++i) b->h_qs[i].variant = variants[i] ? variants[i] : ewah_default_variant();
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(b->d_qs, b->h_qs.data(), b->nq * sizeof(QueryDev), hipMemcpyHostToDevice));
    return EWAH_OK;
}

ewah_status ewah_batch_set_grid(ewah_batch* b, uint32_t grid) {
    if (!b || grid == 0) return fail(EWAH_EINVAL, "bad argument");
    HIPCHK(hipDeviceSynchronize());
    b->grid = grid;
    return batch_build_graph(b);
}

ewah_status ewah_batch_set_win_batch(ewah_batch* b, uint32_t win_batch) {
    if (!b || win_batch < 4 || win_batch > 7) return fail(EWAH_EINVAL, "win_batch must be in 4..7");
    HIPCHK(hipDeviceSynchronize());
    b->win_batch = (int)win_batch;
    return batch_build_graph(b);
}

ewah_status ewah_batch_set_prepass(ewah_batch* b, int on) {
    if (!b) return fail(EWAH_EINVAL, "null batch");
    HIPCHK(hipDeviceSynchronize());
    b->prepass = on ? 1 : 0;
    return batch_build_graph(b);
}

void ewah_batch_free(ewah_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    (void)hipFree(b->d_qs);
    (void)hipFree(b->d_qtile);
    (void)hipFree(b->d_ids);
    (void)hipFree(b->d_bms);
    (void)hipFree(b->d_state);
    (void)hipFree(b->d_stage);
    (void)hipFree(b->d_tq);
    (void)hipFree(b->d_work);
    (void)hipFree(b->d_codes);
    if (b->d_feat) (void)hipFree(b->d_feat);
    if (b->d_pred) (void)hipFree(b->d_pred);
    if (b->d_itemt) (void)hipFree(b->d_itemt);
    (void)hipFree(b->d_pre);
    (void)hipFree(b->d_pmask);
    (void)hipFree(b->d_list);
    delete b;
}

}  // extern "C"

// --------------------------------------------------------- learned selection

extern "C" {

ewah_status ewah_query_features(const ewah_bitmap* const* pool, uint32_t pool_n, const uint32_t* idx,
                                const uint32_t* offs, const uint32_t* T, uint32_t nq, float* feat_dev,
                                void* hip_stream) {
    ewah_status st = ensure_ready();
    if (st) return st;
    if (nq == 0) return EWAH_OK;
    if (!pool || !idx || !offs || !T || !feat_dev || pool_n == 0) return fail(EWAH_EINVAL, "null argument");
    const uint64_t n_bits = pool[0]->stats.n_bits;
    const uint32_t total = offs[nq];
    std::vector<uint32_t> slots(total);
    for (uint32_t i = 0; i < total; ++i) {
        if (idx[i] >= pool_n || !pool[idx[i]]) return fail(EWAH_EINVAL, "pool index out of range");
        slots[i] = pool[idx[i]]->slot;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    uint32_t* d_slots = nullptr;
    QueryDev* d_q = nullptr;
    HIPCHK(hipMalloc(&d_slots, std::max<size_t>(total, 1) * 4));
    HIPCHK(hipMalloc(&d_q, (size_t)nq * sizeof(QueryDev)));
    std::vector<QueryDev> hq(nq);
    for (uint32_t q = 0; q < nq; ++q) {
        QueryDev d{};
        d.ids = d_slots + offs[q];
        d.N = offs[q + 1] - offs[q];
        d.T = T[q];
        hq[q] = d;
    }
    HIPCHK(hipMemcpy(d_slots, slots.data(), (size_t)total * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_q, hq.data(), (size_t)nq * sizeof(QueryDev), hipMemcpyHostToDevice));
    HIPCHK(launch_features(d_q, nq, g.d_stats, (float)n_bits, feat_dev, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipFree(d_slots));
    HIPCHK(hipFree(d_q));
    return EWAH_OK;
}

ewah_status ewah_batch_features(ewah_batch* b, float* feat_dev, void* hip_stream) {
    if (!b || !feat_dev) return fail(EWAH_EINVAL, "null argument");
    HIPCHK(launch_features(b->d_qs, b->nq, g.d_stats, (float)b->n_bits, feat_dev, (hipStream_t)hip_stream));
    return EWAH_OK;
}

ewah_status ewah_batch_select(ewah_batch* b, const float* pred_dev, uint32_t n_arms, const uint32_t* arm_codes,
                              void* hip_stream) {
    if (!b || !pred_dev || !arm_codes || n_arms == 0 || n_arms > 64) return fail(EWAH_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    if (b->h_codes.size() != n_arms || std::memcmp(b->h_codes.data(), arm_codes, n_arms * 4) != 0) {
        HIPCHK(hipStreamSynchronize(s));   // d_codes may still be read by an earlier selection
        HIPCHK(hipMemcpy(b->d_codes, arm_codes, n_arms * 4, hipMemcpyHostToDevice));
        b->h_codes.assign(arm_codes, arm_codes + n_arms);
    }
    HIPCHK(launch_select(pred_dev, b->nq, n_arms, b->d_codes, b->d_qs, s));
    return EWAH_OK;
}

ewah_status ewah_batch_select_model(ewah_batch* b, const ewah_selector* sel, int mode, void* hip_stream) {
    if (!b || !sel) return fail(EWAH_EINVAL, "null argument");
    const uint32_t K = ewah_selector_num_arms(sel);
    if (K == 0 || K > 16) return fail(EWAH_EINVAL, "selector has no arms");
    if (!b->d_feat) {
        HIPCHK(hipMalloc(&b->d_feat, (size_t)b->nq * 16 * sizeof(float)));
        HIPCHK(hipMalloc(&b->d_pred, (size_t)b->nq * 16 * sizeof(float)));
    }
    uint32_t codes[16];
    ewah_status st = ewah_selector_arm_codes(sel, codes);
    if (st) return st;
    st = ewah_batch_features(b, b->d_feat, hip_stream);
    if (st) return st;
    st = ewah_selector_predict(sel, mode, b->d_feat, b->nq, b->d_pred, hip_stream);
    if (st) return st;
    return ewah_batch_select(b, b->d_pred, K, codes, hip_stream);
}

ewah_status ewah_batch_time_queries(ewah_batch* b, uint32_t reps, float* busy_us, void* hip_stream) {
    if (!b || !busy_us || reps == 0) return fail(EWAH_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    if (!b->d_itemt) {
        HIPCHK(hipMalloc(&b->d_itemt, std::max<size_t>(2 * (size_t)b->total, 1) * 4));
        HIPCHK(hipMemset(b->d_itemt, 0, std::max<size_t>(2 * (size_t)b->total, 1) * 4));
    }
    int khz = 0;
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g.device));
    if (khz <= 0) return fail(EWAH_EDEVICE, "device reports no wall-clock rate");
    std::vector<uint32_t> qtile(b->nq + 1);
    HIPCHK(hipMemcpy(qtile.data(), b->d_qtile, (b->nq + 1) * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> ticks(2 * (size_t)b->total);
    std::vector<double> best(b->nq, 1e300);
    // a pre-pass wavefront holds 1 / pre_waves_per_cu of a CU, a workgroup of the tile routine
    // 1 / batch_blocks_per_cu: its ticks count at that ratio (none without the pre-pass)
    const double wpre = b->prepass ? (double)batch_blocks_per_cu(b->smem) / (double)pre_waves_per_cu() : 0.0;
    for (uint32_t r = 0; r < reps; ++r) {
        HIPCHK(launch_bump(b->d_work, s));
        HIPCHK(launch_batch(b->d_qs, b->d_qtile, b->d_tq, b->nq, b->total, g.d_table, b->d_work, b->d_work + 1, g.d_err,
                            b->grid, b->smem, s, b->d_itemt, b->win_batch, pre_of(b), b->d_pmask, list_of(b)));
        HIPCHK(hipMemcpyAsync(ticks.data(), b->d_itemt, 2 * (size_t)b->total * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (uint32_t q = 0; q < b->nq; ++q) {
            double t = 0, tp = 0;
            for (uint32_t i = qtile[q]; i < qtile[q + 1]; ++i) {
                t += ticks[i];
                tp += ticks[(size_t)b->total + i];
            }
            best[q] = std::min(best[q], t + wpre * tp);
        }
    }
    for (uint32_t q = 0; q < b->nq; ++q) busy_us[q] = (float)(best[q] * 1e3 / khz);
    return EWAH_OK;
}

ewah_status ewah_batch_get_variants(ewah_batch* b, uint32_t* variants_host) {
    if (!b || !variants_host) return fail(EWAH_EINVAL, "null argument");
    HIPCHK(hipDeviceSynchronize());
    std::vector<QueryDev> hq(b->nq);
    HIPCHK(hipMemcpy(hq.data(), b->d_qs, b->nq * sizeof(QueryDev), hipMemcpyDeviceToHost));
    for (uint32_t i = 0; i < b->nq; ++i) {
        variants_host[i] = hq[i].variant;
        b->h_qs[i].variant = hq[i].variant;
    }
    return EWAH_OK;
}

}  // extern "C"
