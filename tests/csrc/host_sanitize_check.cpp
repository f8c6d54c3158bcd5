// Drives the library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
// without a GPU: the registration-time validation and index builder (reached here by
// including the runtime's source, since it is internal to it) on well-formed streams and
// on random word sequences, the output bound, the variant codes, and the selector's
// model-file reader on valid, truncated and corrupted files.  Built for the host only.
#include "../../paper_1402_4466_amd/csrc/thr_api.cpp"

#include <cstdio>
#include <string>

static uint64_t st_ = 0x1402446614024466ull;
static uint64_t rnd() {   // SplitMix64
    uint64_t z = (st_ += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A well-formed (not necessarily canonical) stream over U words: runs of fills and
// literal blocks, split at random.
static std::vector<uint64_t> stream(uint64_t U) {
    std::vector<uint64_t> s;
    uint64_t u = 0;
    while (u < U) {
        const uint64_t L = std::min<uint64_t>(rnd() % 1500, U - u);
        const uint64_t K = std::min<uint64_t>(rnd() % 70, U - u - L);
        s.push_back((rnd() & 1) | (L << 1) | (K << 33));
        for (uint64_t k = 0; k < K; ++k) s.push_back(rnd());
        u += L + K;
    }
    if (s.empty()) s.push_back(0);
    return s;
}

int main() {
    for (int it = 0; it < 300; ++it) {
        const uint64_t n_bits = 1 + rnd() % (3 * 512 * 64 * 4), U = (n_bits + 63) / 64;
        std::vector<uint64_t> s = stream(U);
        Built b;
        if (build_index(s.data(), s.size(), n_bits, b) != EWAH_OK) {
            std::printf("FAIL well-formed stream rejected: %s\n", ewah_last_error());
            return 1;
        }
        if (b.st.n_words != s.size() || b.loc.size() != (U + 511) / 512 + 1) {
            std::printf("FAIL index sizes\n");
            return 1;
        }
        // corrupt: random words, a truncated stream, a marker whose run overshoots
        std::vector<uint64_t> junk(rnd() % 50);
        for (auto& w : junk) w = (rnd() % 3) ? ((rnd() & 1) | ((rnd() % (U + 3)) << 1) | ((rnd() % 5) << 33)) : rnd();
        Built j;
        (void)build_index(junk.data(), junk.size(), n_bits, j);
        if (s.size() > 1) {
            Built t;
            if (build_index(s.data(), s.size() - 1, n_bits, t) == EWAH_OK) {
                // a shorter stream can only be valid if the dropped word was a run-free marker
                const uint64_t last = s.back();
                if (((last >> 1) & 0xFFFFFFFFull) != 0 || (last >> 33) != 0) {
                    std::printf("FAIL truncated stream accepted\n");
                    return 1;
                }
            }
        }
        if (ewah_output_bound(n_bits, s.size()) != std::min<uint64_t>(U + 1, s.size() + 1)) {
            std::printf("FAIL output bound\n");
            return 1;
        }
    }
    const uint32_t v = ewah_variant_code_full(1, 8, 8, 1, 3);
    if (!(v & 1u) || ((v >> 8) & 255u) != 8 || !(v & (1u << 24)) || ((v >> 25) & 3u) != 3) {
        std::printf("FAIL variant code\n");
        return 1;
    }
    // model files: a valid one (two arms), then truncations and byte flips of it
    std::string good = "{\"kind\":\"mlp\",\"n_out\":2,\"arm_codes\":[5,6],\"mu\":[";
    for (int i = 0; i < 16; ++i) good += (i ? ",0.5" : "0.5");
    good += "],\"sigma\":[";
    for (int i = 0; i < 16; ++i) good += (i ? ",2" : "2");
    good += "],\"params_raw\":[";
    const uint64_t np = ewah_mlp_num_params(2);
    for (uint64_t i = 0; i < np; ++i) good += (i ? ",-0.25e-1" : "0.125");
    good += "],\"eval\":{\"s\":\"a\\\"b\\u00e9\",\"x\":[true,false,null,{}]}}";
    const char* path = "host_sanitize_model.json";
    auto load = [&](const std::string& text) {
        FILE* f = std::fopen(path, "wb");
        std::fwrite(text.data(), 1, text.size(), f);
        std::fclose(f);
        ewah_selector* s = nullptr;
        const ewah_status e = ewah_selector_load(path, &s);
        if (s) ewah_selector_free(s);
        return e;
    };
    if (load(good) != EWAH_OK) {
        std::printf("FAIL valid model rejected: %s\n", ewah_last_error());
        return 1;
    }
    for (size_t cut = 0; cut < good.size(); cut += 1 + good.size() / 300)
        if (load(good.substr(0, cut)) == EWAH_OK) {
            std::printf("FAIL truncated model accepted at %zu\n", cut);
            return 1;
        }
    for (int k = 0; k < 400; ++k) {
        std::string t = good;
        t[rnd() % t.size()] = (char)(rnd() & 0xFF);
        (void)load(t);
    }
    std::remove(path);
    std::printf("ok\n");
    return 0;
}
