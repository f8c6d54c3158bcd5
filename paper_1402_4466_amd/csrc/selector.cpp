// The selector of the batched path as a library object: the learned cost model
// (FP32 MLP predicting the log-time of every kernel variant, trained by the
// library's own HIP kernels) and the paper-style rule set (one running-time model
// per variant fitted by least squares, Section 8.1; the variant with the smallest
// estimate is taken, as hybrid H does, Section 8.2).  Machine-learned selection
// is the paper's stated future work (Section 9).
//
// Model files are JSON objects; the keys read here are
//   "n_out" (variants K), "arm_codes" [K], "mu" [16], "sigma" [16],
//   "params_raw" [P] (network on standardised features), "params_folded" [P]
//   (the same with the standardisation folded into the first layer), and,
//   optionally, "rules_coef" [5][K] and "arm_names" [K].
// Other keys (evaluation reports written by the training driver) are ignored.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ewahthr.h"

namespace {

ewah_status sfail(ewah_status s, const std::string& msg);

// ------------------------------------------------------------ a small JSON reader

struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<JVal> arr;
    std::map<std::string, JVal> obj;
};

struct JParser {
    const char* p;
    const char* e;
    std::string err;
    void ws() { while (p < e && std::isspace((unsigned char)*p)) ++p; }
    bool lit(const char* s) {
        const size_t n = std::strlen(s);
        if ((size_t)(e - p) < n || std::strncmp(p, s, n) != 0) return false;
        p += n;
        return true;
    }
    bool str(std::string& out) {
        if (p >= e || *p != '"') return false;
        ++p;
        while (p < e && *p != '"') {
            if (*p == '\\') {
                if (++p >= e) return false;
                const char c = *p++;
                switch (c) {
                    case 'n': out += '\n'; break;
                    case 't': out += '\t'; break;
                    case 'r': out += '\r'; break;
                    case 'b': out += '\b'; break;
                    case 'f': out += '\f'; break;
                    case 'u':   // kept as '?': names are informational only
                        if (e - p < 4) return false;
                        p += 4;
                        out += '?';
                        break;
                    default: out += c;
                }
            } else {
                out += *p++;
            }
        }
        if (p >= e) return false;
        ++p;
        return true;
    }
    bool value(JVal& v, int depth) {
        if (depth > 64) { err = "nesting too deep"; return false; }
        ws();
        if (p >= e) { err = "unexpected end"; return false; }
        const char c = *p;
        if (c == '{') {
            ++p;
            v.kind = JVal::OBJ;
            ws();
            if (p < e && *p == '}') { ++p; return true; }
            for (;;) {
                ws();
                std::string k;
                if (!str(k)) { err = "bad key"; return false; }
                ws();
                if (p >= e || *p != ':') { err = "expected ':'"; return false; }
                ++p;
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.obj[k] = std::move(x);
                ws();
                if (p < e && *p == ',') { ++p; continue; }
                if (p < e && *p == '}') { ++p; return true; }
                err = "expected ',' or '}'";
                return false;
            }
        }
        if (c == '[') {
            ++p;
            v.kind = JVal::ARR;
            ws();
            if (p < e && *p == ']') { ++p; return true; }
            for (;;) {
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.arr.push_back(std::move(x));
                ws();
                if (p < e && *p == ',') { ++p; continue; }
                if (p < e && *p == ']') { ++p; return true; }
                err = "expected ',' or ']'";
                return false;
            }
        }
        if (c == '"') {
            v.kind = JVal::STR;
            if (!str(v.str)) { err = "bad string"; return false; }
            return true;
        }
        if (lit("true")) { v.kind = JVal::BOOL; v.b = true; return true; }
        if (lit("false")) { v.kind = JVal::BOOL; v.b = false; return true; }
        if (lit("null")) { v.kind = JVal::NUL; return true; }
        if (lit("NaN")) { v.kind = JVal::NUM; v.num = std::nan(""); return true; }
        if (lit("Infinity")) { v.kind = JVal::NUM; v.num = HUGE_VAL; return true; }
        if (lit("-Infinity")) { v.kind = JVal::NUM; v.num = -HUGE_VAL; return true; }
        char* end = nullptr;
        const std::string tok(p, (size_t)std::min<ptrdiff_t>(e - p, 64));
        const double d = std::strtod(tok.c_str(), &end);
        if (end == tok.c_str()) { err = "bad value"; return false; }
        p += end - tok.c_str();
        v.kind = JVal::NUM;
        v.num = d;
        return true;
    }
};

bool num_array(const JVal& root, const char* key, std::vector<double>& out, size_t want, std::string& why) {
    auto it = root.obj.find(key);
    if (it == root.obj.end()) { why = std::string("missing \"") + key + "\""; return false; }
    const JVal& a = it->second;
    if (a.kind != JVal::ARR) { why = std::string("\"") + key + "\" is not an array"; return false; }
    out.clear();
    for (const JVal& x : a.arr) {
        if (x.kind == JVal::NUM) { out.push_back(x.num); continue; }
        if (x.kind == JVal::ARR) {   // one level of nesting (rules_coef is [5][K])
            for (const JVal& y : x.arr) {
                if (y.kind != JVal::NUM) { why = std::string("\"") + key + "\" holds a non-number"; return false; }
                out.push_back(y.num);
            }
            continue;
        }
        why = std::string("\"") + key + "\" holds a non-number";
        return false;
    }
    if (want && out.size() != want) {
        why = std::string("\"") + key + "\" has " + std::to_string(out.size()) + " values, expected " +
              std::to_string(want);
        return false;
    }
    return true;
}

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

constexpr int NF = 16;   // features
constexpr int NH = 64;   // hidden width
constexpr int NR = 5;    // rule-set regressors

// Regressors of the paper-style running-time model from the features: the compressed
// size (EWAHSize in words), EWAHSize * ln N (RBMrg / BSTM form), N * tiles (the per-tile
// fixed work of each input), T * EWAHSize (Looped form) and the dirty-word count.
void rule_regressors(const float* f, double* x) {
    const double ewah = std::exp2((double)f[10]) - 1.0;
    const double N = std::exp2((double)f[0]);
    const double T = std::exp2((double)f[1]);
    const double tiles = std::max(std::exp2((double)f[13]) / 65536.0, 1.0);
    x[0] = ewah;
    x[1] = ewah * std::log(std::max(N, 1.0));
    x[2] = N * tiles;
    x[3] = T * ewah;
    x[4] = (double)f[12] * ewah;
}

}  // namespace

struct ewah_selector {
    uint32_t K = 0;
    std::vector<uint32_t> codes;
    std::vector<double> mu, sigma;         // standardisation of the features
    std::vector<float> raw, folded;        // network parameters (raw: on standardised features)
    std::vector<double> coef;              // rule set [NR][K], empty if absent
    std::vector<std::string> names;
    mutable ewah_mlp* net = nullptr;       // device copy of the folded parameters (made on first use)
    mutable float* d_coef = nullptr;       // rule coefficients on the device (float)
    float final_loss = 0.f;
};

namespace {

// W1' = W1 / sigma (per input row), b1' = b1 - sum_i (mu_i / sigma_i) W1[i]: the exact
// identity that lets raw features go straight into the first layer.
std::vector<float> fold(const std::vector<float>& raw, const std::vector<double>& mu, const std::vector<double>& sd) {
    std::vector<float> f(raw);
    for (int a = 0; a < NH; ++a) {
        double b = raw[(size_t)NF * NH + a];
        for (int i = 0; i < NF; ++i) {
            const double w = raw[(size_t)i * NH + a];
            f[(size_t)i * NH + a] = (float)(w / sd[i]);
            b -= mu[i] / sd[i] * w;
        }
        f[(size_t)NF * NH + a] = (float)b;
    }
    return f;
}

ewah_status upload(const ewah_selector* s) {
    if (!s->net) {
        ewah_status st = ewah_mlp_create(s->K, 1, &s->net);
        if (st) return sfail(st, std::string("mlp_create: ") + ewah_mlp_last_error());
    }
    ewah_status st = ewah_mlp_set_params(s->net, s->folded.data(), s->folded.size());
    if (st) return sfail(st, std::string("mlp_set_params: ") + ewah_mlp_last_error());
    if (!s->coef.empty()) {
        std::vector<float> c(s->coef.begin(), s->coef.end());
        if (!s->d_coef && hipMalloc(&s->d_coef, c.size() * sizeof(float)) != hipSuccess)
            return sfail(EWAH_ENOMEM, "device allocation of the rule coefficients failed");
        if (hipMemcpy(s->d_coef, c.data(), c.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return sfail(EWAH_EDEVICE, "upload of the rule coefficients failed");
    }
    return EWAH_OK;
}

// Least squares through the origin per variant (normal equations on columns scaled to
// unit RMS, solved by Gaussian elimination with partial pivoting in FP64).
void fit_rules(const std::vector<float>& feat, const std::vector<double>& t_us, uint32_t n, uint32_t K,
               std::vector<double>& coef) {
    std::vector<double> X((size_t)n * NR);
    for (uint32_t i = 0; i < n; ++i) rule_regressors(&feat[(size_t)i * NF], &X[(size_t)i * NR]);
    double scale[NR];
    for (int j = 0; j < NR; ++j) {
        double s = 0;
        for (uint32_t i = 0; i < n; ++i) s += X[(size_t)i * NR + j] * X[(size_t)i * NR + j];
        scale[j] = s > 0 ? std::sqrt(s / n) : 1.0;
    }
    coef.assign((size_t)NR * K, 0.0);
    for (uint32_t k = 0; k < K; ++k) {
        double A[NR][NR + 1] = {};
        for (uint32_t i = 0; i < n; ++i) {
            double x[NR];
            for (int j = 0; j < NR; ++j) x[j] = X[(size_t)i * NR + j] / scale[j];
            const double y = t_us[(size_t)i * K + k];
            for (int a = 0; a < NR; ++a) {
                for (int b = 0; b < NR; ++b) A[a][b] += x[a] * x[b];
                A[a][NR] += x[a] * y;
            }
        }
        for (int a = 0; a < NR; ++a) A[a][a] += 1e-12 * (A[a][a] + 1.0);   // keeps singular columns at zero
        for (int c = 0; c < NR; ++c) {
            int piv = c;
            for (int r = c + 1; r < NR; ++r)
                if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
            if (piv != c)
                for (int j = 0; j <= NR; ++j) std::swap(A[c][j], A[piv][j]);
            if (A[c][c] == 0) continue;
            for (int r = 0; r < NR; ++r) {
                if (r == c) continue;
                const double m = A[r][c] / A[c][c];
                for (int j = c; j <= NR; ++j) A[r][j] -= m * A[c][j];
            }
        }
        for (int j = 0; j < NR; ++j) coef[(size_t)j * K + k] = A[j][j] != 0 ? A[j][NR] / A[j][j] / scale[j] : 0.0;
    }
}

void write_array(FILE* f, const char* key, const std::vector<double>& v, bool last = false) {
    std::fprintf(f, "\"%s\":[", key);
    for (size_t i = 0; i < v.size(); ++i) std::fprintf(f, "%s%.17g", i ? "," : "", v[i]);
    std::fprintf(f, "]%s", last ? "" : ",");
}

}  // namespace

namespace ewt {
hipError_t launch_rules(const float* feat, uint32_t nq, const float* coef, uint32_t K, float* pred, hipStream_t s);
void set_last_error(const std::string& msg);   // the library's ewah_last_error channel
}

namespace {
ewah_status sfail(ewah_status s, const std::string& msg) {
    ewt::set_last_error(msg);
    return s;
}
}  // namespace

extern "C" {

void ewah_selector_free(ewah_selector* s) {
    if (!s) return;
    if (s->net) ewah_mlp_free(s->net);
    if (s->d_coef) { (void)hipDeviceSynchronize(); (void)hipFree(s->d_coef); }
    delete s;
}

ewah_status ewah_selector_load(const char* path, ewah_selector** out) {
    if (!path || !out) return sfail(EWAH_EINVAL, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return sfail(EWAH_EINVAL, std::string("cannot open ") + path);
    std::string text;
    char buf[1 << 16];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    JParser P{text.data(), text.data() + text.size(), {}};
    JVal root;
    if (!P.value(root, 0) || root.kind != JVal::OBJ) return sfail(EWAH_EFORMAT, std::string(path) + ": " + P.err);
    std::unique_ptr<ewah_selector> s(new ewah_selector());
    std::string why;
    std::vector<double> v;
    auto kind = root.obj.find("kind");
    if (kind != root.obj.end() && (kind->second.kind != JVal::STR || kind->second.str != "mlp"))
        return sfail(EWAH_EFORMAT, std::string(path) + ": not an MLP selector model");
    if (!num_array(root, "arm_codes", v, 0, why)) return sfail(EWAH_EFORMAT, std::string(path) + ": " + why);
    if (v.empty() || v.size() > 16) return sfail(EWAH_EFORMAT, std::string(path) + ": 1..16 arms");
    s->K = (uint32_t)v.size();
    for (double c : v) s->codes.push_back((uint32_t)c);
    auto nout = root.obj.find("n_out");
    if (nout != root.obj.end() && (nout->second.kind != JVal::NUM || (uint32_t)nout->second.num != s->K))
        return sfail(EWAH_EFORMAT, std::string(path) + ": n_out differs from the number of arm codes");
    const size_t np = (size_t)ewah_mlp_num_params(s->K);
    if (!num_array(root, "mu", s->mu, NF, why) || !num_array(root, "sigma", s->sigma, NF, why))
        return sfail(EWAH_EFORMAT, std::string(path) + ": " + why);
    for (double sd : s->sigma)
        if (!(sd > 0)) return sfail(EWAH_EFORMAT, std::string(path) + ": sigma must be positive");
    if (!num_array(root, "params_raw", v, np, why)) return sfail(EWAH_EFORMAT, std::string(path) + ": " + why);
    s->raw.assign(v.begin(), v.end());
    if (root.obj.count("params_folded")) {
        if (!num_array(root, "params_folded", v, np, why)) return sfail(EWAH_EFORMAT, std::string(path) + ": " + why);
        s->folded.assign(v.begin(), v.end());
    } else {
        s->folded = fold(s->raw, s->mu, s->sigma);
    }
    if (root.obj.count("rules_coef")) {
        if (!num_array(root, "rules_coef", s->coef, (size_t)NR * s->K, why))
            return sfail(EWAH_EFORMAT, std::string(path) + ": " + why);
    }
    auto names = root.obj.find("arm_names");
    if (names != root.obj.end() && names->second.kind == JVal::ARR)
        for (const JVal& x : names->second.arr) s->names.push_back(x.kind == JVal::STR ? x.str : std::string());
    *out = s.release();   // the device copy is made on first use
    return EWAH_OK;
}

ewah_status ewah_selector_save(const ewah_selector* s, const char* path) {
    if (!s || !path) return sfail(EWAH_EINVAL, "null argument");
    FILE* f = std::fopen(path, "wb");
    if (!f) return sfail(EWAH_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "{\"kind\":\"mlp\",\"n_out\":%u,", s->K);
    std::vector<double> codes(s->codes.begin(), s->codes.end());
    write_array(f, "arm_codes", codes);
    if (!s->names.empty()) {
        std::fprintf(f, "\"arm_names\":[");
        for (size_t i = 0; i < s->names.size(); ++i) std::fprintf(f, "%s\"%s\"", i ? "," : "", s->names[i].c_str());
        std::fprintf(f, "],");
    }
    write_array(f, "mu", s->mu);
    write_array(f, "sigma", s->sigma);
    write_array(f, "params_raw", std::vector<double>(s->raw.begin(), s->raw.end()));
    if (!s->coef.empty()) write_array(f, "rules_coef", s->coef);
    write_array(f, "params_folded", std::vector<double>(s->folded.begin(), s->folded.end()), true);
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? EWAH_OK : sfail(EWAH_EINVAL, std::string("write failed: ") + path);
}

uint32_t ewah_selector_num_arms(const ewah_selector* s) { return s ? s->K : 0u; }

ewah_status ewah_selector_arm_codes(const ewah_selector* s, uint32_t* codes) {
    if (!s || !codes) return sfail(EWAH_EINVAL, "null argument");
    std::memcpy(codes, s->codes.data(), s->K * sizeof(uint32_t));
    return EWAH_OK;
}

ewah_status ewah_selector_train(const float* feat, const float* log2_time, uint32_t n, uint32_t n_arms,
                                const uint32_t* arm_codes, const ewah_train_config* cfg, ewah_selector** out) {
    if (!feat || !log2_time || !arm_codes || !out) return sfail(EWAH_EINVAL, "null argument");
    if (n == 0 || n_arms == 0 || n_arms > 16) return sfail(EWAH_EINVAL, "need n >= 1 samples and 1..16 arms");
    const uint32_t epochs = cfg && cfg->epochs ? cfg->epochs : 80;
    const uint32_t bs = cfg && cfg->batch ? cfg->batch : 1024;
    const float lr = cfg && cfg->lr > 0 ? cfg->lr : 2e-3f;
    const uint64_t seed = cfg && cfg->seed ? cfg->seed : 1;
    std::unique_ptr<ewah_selector> s(new ewah_selector());
    s->K = n_arms;
    s->codes.assign(arm_codes, arm_codes + n_arms);
    // standardisation (the constant last feature stays 1)
    s->mu.assign(NF, 0.0);
    s->sigma.assign(NF, 1.0);
    for (int j = 0; j < NF; ++j) {
        double m = 0, q = 0;
        for (uint32_t i = 0; i < n; ++i) m += feat[(size_t)i * NF + j];
        m /= n;
        for (uint32_t i = 0; i < n; ++i) {
            const double d = feat[(size_t)i * NF + j] - m;
            q += d * d;
        }
        const double sd = std::sqrt(q / n);
        s->mu[j] = m;
        s->sigma[j] = sd < 1e-6 ? 1.0 : sd;
    }
    s->mu[NF - 1] = 0.0;
    s->sigma[NF - 1] = 1.0;
    std::vector<float> Xs((size_t)n * NF), Y((size_t)n * n_arms);
    double ymean = 0;
    for (uint32_t i = 0; i < n; ++i) {
        for (int j = 0; j < NF; ++j)
            Xs[(size_t)i * NF + j] = j == NF - 1 ? 1.f : (float)((feat[(size_t)i * NF + j] - s->mu[j]) / s->sigma[j]);
        // relative costs: each arm's log-time minus the sample's mean over the arms, so the
        // network models how the arms differ rather than how large the query is
        double rm = 0;
        for (uint32_t k = 0; k < n_arms; ++k) {
            const float t = log2_time[(size_t)i * n_arms + k];
            if (!std::isfinite(t)) return sfail(EWAH_EINVAL, "non-finite label at sample " + std::to_string(i));
            rm += t;
        }
        rm /= n_arms;
        for (uint32_t k = 0; k < n_arms; ++k) {
            Y[(size_t)i * n_arms + k] = (float)(log2_time[(size_t)i * n_arms + k] - rm);
            ymean += Y[(size_t)i * n_arms + k];
        }
    }
    ymean /= (double)n * n_arms;
    for (float& y : Y) y = (float)(y - ymean);
    ewah_mlp* net = nullptr;
    ewah_status st = ewah_mlp_create(n_arms, seed, &net);
    if (st) return sfail(st, std::string("mlp_create: ") + ewah_mlp_last_error());
    float *dX = nullptr, *dY = nullptr, *dL = nullptr;
    auto cleanup = [&]() {
        (void)hipDeviceSynchronize();
        if (dX) (void)hipFree(dX);
        if (dY) (void)hipFree(dY);
        if (dL) (void)hipFree(dL);
        ewah_mlp_free(net);
    };
    if (hipMalloc(&dX, Xs.size() * 4) != hipSuccess || hipMalloc(&dY, Y.size() * 4) != hipSuccess ||
        hipMalloc(&dL, 4) != hipSuccess) {
        cleanup();
        return sfail(EWAH_ENOMEM, "device allocation of the training set failed");
    }
    std::vector<uint32_t> perm(n);
    std::vector<float> pX(Xs.size()), pY(Y.size());
    float loss = 0.f;
    for (uint32_t ep = 0; ep < epochs; ++ep) {
        // Fisher-Yates shuffle from a counter-based SplitMix64 stream keyed by (seed, epoch)
        for (uint32_t i = 0; i < n; ++i) perm[i] = i;
        const uint64_t key = mix64(seed * 0x9E3779B97F4A7C15ULL + ep);
        for (uint32_t i = n - 1; i > 0; --i) {
            const uint64_t r = mix64(key + (uint64_t)i * 0x9E3779B97F4A7C15ULL);
            const uint32_t j = (uint32_t)((r >> 11) % ((uint64_t)i + 1));
            std::swap(perm[i], perm[j]);
        }
        for (uint32_t i = 0; i < n; ++i) {
            std::memcpy(&pX[(size_t)i * NF], &Xs[(size_t)perm[i] * NF], NF * 4);
            std::memcpy(&pY[(size_t)i * n_arms], &Y[(size_t)perm[i] * n_arms], n_arms * 4);
        }
        if (hipMemcpy(dX, pX.data(), pX.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dY, pY.data(), pY.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
            cleanup();
            return sfail(EWAH_EDEVICE, "upload of the training set failed");
        }
        for (uint32_t s0 = 0; s0 < n; s0 += bs) {
            const uint32_t b = std::min(bs, n - s0);
            st = ewah_mlp_train_step(net, dX + (size_t)s0 * NF, dY + (size_t)s0 * n_arms, b, lr, dL, nullptr);
            if (st) {
                cleanup();
                return sfail(st, std::string("mlp_train_step: ") + ewah_mlp_last_error());
            }
        }
        if (ep + 1 == epochs && hipMemcpy(&loss, dL, 4, hipMemcpyDeviceToHost) != hipSuccess) {
            cleanup();
            return sfail(EWAH_EDEVICE, "loss readback failed");
        }
    }
    s->raw.resize((size_t)ewah_mlp_num_params(n_arms));
    st = ewah_mlp_get_params(net, s->raw.data(), s->raw.size());
    cleanup();
    if (st) return sfail(st, std::string("mlp_get_params: ") + ewah_mlp_last_error());
    s->folded = fold(s->raw, s->mu, s->sigma);
    s->final_loss = loss;
    // the rule set on the same labels, in microseconds
    std::vector<float> fv(feat, feat + (size_t)n * NF);
    std::vector<double> t_us((size_t)n * n_arms);
    for (size_t i = 0; i < t_us.size(); ++i) t_us[i] = std::exp2((double)log2_time[i]);
    fit_rules(fv, t_us, n, n_arms, s->coef);
    *out = s.release();
    return EWAH_OK;
}

float ewah_selector_train_loss(const ewah_selector* s) { return s ? s->final_loss : 0.f; }

ewah_status ewah_selector_predict(const ewah_selector* s, int mode, const float* feat_dev, uint32_t n, float* pred_dev,
                                  void* hip_stream) {
    if (!s || (n && (!feat_dev || !pred_dev))) return sfail(EWAH_EINVAL, "null argument");
    if (n == 0) return EWAH_OK;
    if (!s->net) {
        ewah_status st = upload(s);
        if (st) return st;
    }
    if (mode == EWAH_SELECT_MLP) {
        ewah_status st = ewah_mlp_forward(s->net, feat_dev, n, pred_dev, hip_stream);
        return st ? sfail(st, std::string("mlp_forward: ") + ewah_mlp_last_error()) : EWAH_OK;
    }
    if (mode == EWAH_SELECT_RULES) {
        if (!s->d_coef) return sfail(EWAH_EINVAL, "the model holds no rule set");
        if (ewt::launch_rules(feat_dev, n, s->d_coef, s->K, pred_dev, (hipStream_t)hip_stream) != hipSuccess)
            return sfail(EWAH_EDEVICE, "rule-set kernel launch failed");
        return EWAH_OK;
    }
    return sfail(EWAH_EINVAL, "mode must be EWAH_SELECT_MLP or EWAH_SELECT_RULES");
}

}  // extern "C"
