// Device-side feature extraction and variant selection for batched queries.
// Features come from the registration catalog of each input (compressed
// size, dirty words, cardinality, RunCount), the statistics the paper's hybrid
// assumes a database maintains (Section 8.1); the selection takes, per query,
// the variant with the smallest predicted cost (the rule of hybrid H, Section
// 8.2, applied to the learned cost model's predictions).
#include "thr_device.h"

namespace ewt {

// One wavefront per query; lanes stride over the query's inputs.
__global__ __launch_bounds__(256) void features_kernel(const QueryDev* __restrict__ qs, uint32_t nq,
                                                       const float4* __restrict__ stats, float r,
                                                       float* __restrict__ feat) {
    const uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= nq) return;
    const QueryDev Q = qs[q];
    const uint32_t N = Q.N;
    float s_ld = 0.f, s_ld2 = 0.f, mx_ld = -1e30f, mn_ld = 1e30f;
    float s_runs = 0.f, mx_runs = 0.f, s_words = 0.f, mx_words = 0.f, s_lits = 0.f, s_dens = 0.f;
    for (uint32_t k = (uint32_t)lane; k < N; k += 64) {
        const float4 st = stats[Q.ids[k]];            // (n_words, n_literals, popcount, run_count)
        const float dens = fmaxf(st.z / r, 1e-9f);
        const float ld = log2f(dens);
        s_ld += ld;
        s_ld2 += ld * ld;
        mx_ld = fmaxf(mx_ld, ld);
        mn_ld = fminf(mn_ld, ld);
        s_runs += st.w;
        mx_runs = fmaxf(mx_runs, st.w);
        s_words += st.x;
        mx_words = fmaxf(mx_words, st.x);
        s_lits += st.y;
        s_dens += dens;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        s_ld += __shfl_xor(s_ld, d, 64);
        s_ld2 += __shfl_xor(s_ld2, d, 64);
        mx_ld = fmaxf(mx_ld, __shfl_xor(mx_ld, d, 64));
        mn_ld = fminf(mn_ld, __shfl_xor(mn_ld, d, 64));
        s_runs += __shfl_xor(s_runs, d, 64);
        mx_runs = fmaxf(mx_runs, __shfl_xor(mx_runs, d, 64));
        s_words += __shfl_xor(s_words, d, 64);
        mx_words = fmaxf(mx_words, __shfl_xor(mx_words, d, 64));
        s_lits += __shfl_xor(s_lits, d, 64);
        s_dens += __shfl_xor(s_dens, d, 64);
    }
    if (lane == 0) {
        const float n = (float)max(N, 1u);
        const float T = (float)Q.T;
        const float Tc = fminf(T, n);
        const float mean = s_ld / n;
        const float var = fmaxf(s_ld2 / n - mean * mean, 0.f);
        float* f = feat + (size_t)q * 16;
        f[0] = log2f(n);
        f[1] = log2f(fmaxf(T, 1.f));
        f[2] = T / n;
        f[3] = log2f(n - Tc + 1.f);
        f[4] = mean;
        f[5] = mx_ld;
        f[6] = mn_ld;
        f[7] = sqrtf(var);
        f[8] = log2f(s_runs + 1.f);
        f[9] = log2f(mx_runs + 1.f);
        f[10] = log2f(s_words + 1.f);
        f[11] = log2f(mx_words + 1.f);
        f[12] = s_lits / fmaxf(s_words, 1.f);
        f[13] = log2f(r);
        f[14] = s_dens / fmaxf(T, 1.f);
        f[15] = 1.f;
    }
}

// Per query: argmin over the predicted costs, written as the query's variant.
__global__ void select_kernel(const float* __restrict__ pred, uint32_t nq, uint32_t n_arms,
                              const uint32_t* __restrict__ codes, QueryDev* __restrict__ qs) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    uint32_t best = 0;
    float bv = pred[(size_t)q * n_arms];
    for (uint32_t k = 1; k < n_arms; ++k) {
        const float v = pred[(size_t)q * n_arms + k];
        if (v < bv) { bv = v; best = k; }
    }
    qs[q].variant = codes[best];
}

// Rule set (Section 8.1 model forms): predicted time of arm k = sum_j x_j coef[j][k], with
// x the five regressors of the paper-style running-time model computed from the features:
// EWAHSize (compressed words), EWAHSize ln N, N times tiles, T EWAHSize, dirty words.
__global__ void rules_kernel(const float* __restrict__ feat, uint32_t nq, const float* __restrict__ coef, uint32_t K,
                             float* __restrict__ pred) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const float* f = feat + (size_t)q * 16;
    const float ewah = exp2f(f[10]) - 1.f;
    const float N = exp2f(f[0]);
    const float T = exp2f(f[1]);
    const float tiles = fmaxf(exp2f(f[13]) / 65536.f, 1.f);
    const float x[5] = {ewah, ewah * logf(fmaxf(N, 1.f)), N * tiles, T * ewah, f[12] * ewah};
    for (uint32_t k = 0; k < K; ++k) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < 5; ++j) s = fmaf(x[j], coef[(size_t)j * K + k], s);
        pred[(size_t)q * K + k] = s;
    }
}

hipError_t launch_rules(const float* feat, uint32_t nq, const float* coef, uint32_t K, float* pred, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(rules_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, feat, nq, coef, K, pred);
    return hipGetLastError();
}

hipError_t launch_features(const QueryDev* qs, uint32_t nq, const float4* stats, float r, float* feat, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3((nq + 3) / 4), dim3(256), 0, s, qs, nq, stats, r, feat);
    return hipGetLastError();
}

hipError_t launch_select(const float* pred, uint32_t nq, uint32_t n_arms, const uint32_t* codes, QueryDev* qs,
                         hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(select_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, pred, nq, n_arms, codes, qs);
    return hipGetLastError();
}

}  // namespace ewt
