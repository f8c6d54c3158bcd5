// Small FP32 multilayer perceptron used as the cost model of the kernel-variant
// selector: 16 inputs -> 64 -> 64 (ReLU) -> K outputs (predicted log-time of
// each variant).  Machine-learned algorithm selection is the paper's stated
// future work for choosing among threshold algorithms (Section 9); the
// paper's own hybrid picks the algorithm with the lowest fitted running-time
// estimate (Section 8).  Selection never changes query results.
//
// Kernels: inference (one lane per sample), fused forward + backward over 64
// samples per workgroup with activations in LDS and gradient accumulation
// into a global buffer, and an Adam update.  Loss: mean squared error over
// samples and outputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ewahthr.h"

namespace ewm {

constexpr int NI = 16;    // inputs
constexpr int H = 64;     // hidden width (both layers)
constexpr int NOMAX = 16; // outputs (variants) at most
constexpr int SB = 64;    // samples per workgroup in the gradient kernel

// Parameter layout (floats): W1[NI][H], b1[H], W2[H][H], b2[H], W3[H][no], b3[no].
__host__ __device__ inline size_t off_b1() { return (size_t)NI * H; }
__host__ __device__ inline size_t off_W2() { return off_b1() + H; }
__host__ __device__ inline size_t off_b2() { return off_W2() + (size_t)H * H; }
__host__ __device__ inline size_t off_W3() { return off_b2() + H; }
__host__ __device__ inline size_t off_b3(int no) { return off_W3() + (size_t)H * no; }
__host__ __device__ inline size_t n_params(int no) { return off_b3(no) + no; }

__device__ inline void load_params(float* sp, const float* __restrict__ p, int no) {
    const size_t n = n_params(no);
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
}

// y[b][k] for every sample b; one lane per sample, parameters in LDS.
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ x, const float* __restrict__ p,
                                                          float* __restrict__ y, uint32_t batch, int no) {
    extern __shared__ float sp[];
    load_params(sp, p, no);
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    float xi[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) xi[i] = x[(size_t)b * NI + i];
    float h1[H];
#pragma unroll
    for (int a = 0; a < H; ++a) {
        float s = sp[off_b1() + a];
#pragma unroll
        for (int i = 0; i < NI; ++i) s = fmaf(xi[i], sp[(size_t)i * H + a], s);
        h1[a] = s > 0.f ? s : 0.f;
    }
    float out[NOMAX];
#pragma unroll
    for (int k = 0; k < NOMAX; ++k) out[k] = k < no ? sp[off_b3(no) + k] : 0.f;
    for (int j = 0; j < H; ++j) {
        float s = sp[off_b2() + j];
#pragma unroll
        for (int a = 0; a < H; ++a) s = fmaf(h1[a], sp[off_W2() + (size_t)a * H + j], s);
        const float h2 = s > 0.f ? s : 0.f;
#pragma unroll
        for (int k = 0; k < NOMAX; ++k)
            if (k < no) out[k] = fmaf(h2, sp[off_W3() + (size_t)j * no + k], out[k]);
    }
    for (int k = 0; k < no; ++k) y[(size_t)b * no + k] = out[k];
}

// Forward + backward of the mean squared error for SB samples per workgroup
// (one wave, one lane per sample); gradients summed into g (zeroed by the
// caller), loss sum into *loss.  scale = 1 / (batch * no).
__global__ __launch_bounds__(SB) void mlp_grad_kernel(const float* __restrict__ x, const float* __restrict__ t,
                                                      const float* __restrict__ p, float* __restrict__ g,
                                                      float* __restrict__ loss, uint32_t batch, int no, float scale) {
    extern __shared__ float lds[];
    float* sp = lds;                                  // parameters
    float* sx = sp + n_params(no);                    // [SB][NI]
    float* s1 = sx + SB * NI;                         // h1 [SB][H + 1]
    float* s2 = s1 + SB * (H + 1);                    // h2 [SB][H + 1]
    float* sdy = s2 + SB * (H + 1);                   // dy [SB][NOMAX]
    float* sd2 = sdy + SB * NOMAX;                    // dh2 [SB][H + 1]
    float* sd1 = sd2 + SB * (H + 1);                  // dh1 [SB][H + 1]
    load_params(sp, p, no);
    const int tid = threadIdx.x;
    const uint32_t b = blockIdx.x * SB + tid;
    const bool live = b < batch;
    // forward
    float xi[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        xi[i] = live ? x[(size_t)b * NI + i] : 0.f;
        sx[tid * NI + i] = xi[i];
    }
    for (int a = 0; a < H; ++a) {
        float s = sp[off_b1() + a];
#pragma unroll
        for (int i = 0; i < NI; ++i) s = fmaf(xi[i], sp[(size_t)i * H + a], s);
        s1[tid * (H + 1) + a] = s > 0.f ? s : 0.f;
    }
    for (int j = 0; j < H; ++j) {
        float s = sp[off_b2() + j];
        for (int a = 0; a < H; ++a) s = fmaf(s1[tid * (H + 1) + a], sp[off_W2() + (size_t)a * H + j], s);
        s2[tid * (H + 1) + j] = s > 0.f ? s : 0.f;
    }
    float lsum = 0.f;
    for (int k = 0; k < no; ++k) {
        float s = sp[off_b3(no) + k];
        for (int j = 0; j < H; ++j) s = fmaf(s2[tid * (H + 1) + j], sp[off_W3() + (size_t)j * no + k], s);
        const float d = live ? s - t[(size_t)b * no + k] : 0.f;
        lsum += d * d;
        sdy[tid * NOMAX + k] = 2.f * d * scale;
    }
    // backward through the layers (per sample)
    for (int j = 0; j < H; ++j) {
        float s = 0.f;
        for (int k = 0; k < no; ++k) s = fmaf(sdy[tid * NOMAX + k], sp[off_W3() + (size_t)j * no + k], s);
        sd2[tid * (H + 1) + j] = s2[tid * (H + 1) + j] > 0.f ? s : 0.f;
    }
    for (int a = 0; a < H; ++a) {
        float s = 0.f;
        for (int j = 0; j < H; ++j) s = fmaf(sd2[tid * (H + 1) + j], sp[off_W2() + (size_t)a * H + j], s);
        sd1[tid * (H + 1) + a] = s1[tid * (H + 1) + a] > 0.f ? s : 0.f;
    }
    __syncthreads();
    // parameter gradients: sums over the workgroup's samples, lane = row
    const int nb = (int)min((uint32_t)SB, batch - blockIdx.x * SB);
    {   // W1[i][a], b1[a]: lane a
        const int a = tid;
        float gb = 0.f;
        float gw[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) gw[i] = 0.f;
        for (int s = 0; s < nb; ++s) {
            const float d = sd1[s * (H + 1) + a];
            gb += d;
#pragma unroll
            for (int i = 0; i < NI; ++i) gw[i] = fmaf(sx[s * NI + i], d, gw[i]);
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) atomicAdd(&g[(size_t)i * H + a], gw[i]);
        atomicAdd(&g[off_b1() + a], gb);
    }
    {   // W2[a][j], b2[j]: lane a, loop over j
        const int a = tid;
        for (int j = 0; j < H; ++j) {
            float acc = 0.f;
            for (int s = 0; s < nb; ++s) acc = fmaf(s1[s * (H + 1) + a], sd2[s * (H + 1) + j], acc);
            atomicAdd(&g[off_W2() + (size_t)a * H + j], acc);
        }
        float gb = 0.f;
        for (int s = 0; s < nb; ++s) gb += sd2[s * (H + 1) + a];
        atomicAdd(&g[off_b2() + a], gb);
    }
    {   // W3[j][k], b3[k]: lane j
        const int j = tid;
        for (int k = 0; k < no; ++k) {
            float acc = 0.f;
            for (int s = 0; s < nb; ++s) acc = fmaf(s2[s * (H + 1) + j], sdy[s * NOMAX + k], acc);
            atomicAdd(&g[off_W3() + (size_t)j * no + k], acc);
        }
        if (j < no) {
            float gb = 0.f;
            for (int s = 0; s < nb; ++s) gb += sdy[s * NOMAX + j];
            atomicAdd(&g[off_b3(no) + j], gb);
        }
    }
    // loss
    float l = lsum;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) l += __shfl_xor(l, d, 64);
    if (tid == 0) atomicAdd(loss, l * scale);
}

// Adam (Kingma & Ba) on every parameter; gradients are zeroed afterwards.
__global__ void mlp_adam_kernel(float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, uint32_t n, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    g[i] = 0.f;
}

__global__ void fill_zero_kernel(float* __restrict__ a, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.f;
}

size_t grad_smem(int no) {
    return (n_params(no) + (size_t)SB * NI + 4 * (size_t)SB * (H + 1) + (size_t)SB * NOMAX) * sizeof(float);
}

}  // namespace ewm

// ------------------------------------------------------------------- C ABI

struct ewah_mlp {
    int no = 0;
    size_t n = 0;
    float* d_p = nullptr;
    float* d_g = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    uint64_t step = 0;
};

namespace {
thread_local std::string m_err;
ewah_status mfail(ewah_status s, const std::string& msg) {
    m_err = msg;
    return s;
}
#define MCHK(expr)                                                                               \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return mfail(EWAH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
}  // namespace

extern "C" {

const char* ewah_mlp_last_error(void) { return m_err.c_str(); }

uint64_t ewah_mlp_num_params(uint32_t n_out) { return (uint64_t)ewm::n_params((int)n_out); }

ewah_status ewah_mlp_create(uint32_t n_out, uint64_t seed, ewah_mlp** out) {
    if (!out || n_out == 0 || n_out > (uint32_t)ewm::NOMAX) return mfail(EWAH_EINVAL, "n_out must be in 1..16");
    ewah_mlp* m = new ewah_mlp();
    m->no = (int)n_out;
    m->n = ewm::n_params(m->no);
    // He-uniform initialisation from a counter-based SplitMix64 stream; biases zero
    std::vector<float> h(m->n, 0.f);
    uint64_t ctr = 0;
    auto uni = [&]() {
        ctr += 1;
        return (double)(mix64(seed + ctr * 0x9E3779B97F4A7C15ULL) >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](size_t off, int fan_in, size_t count) {
        const double lim = std::sqrt(6.0 / fan_in);
        for (size_t i = 0; i < count; ++i) h[off + i] = (float)((2.0 * uni() - 1.0) * lim);
    };
    fill(0, ewm::NI, (size_t)ewm::NI * ewm::H);
    fill(ewm::off_W2(), ewm::H, (size_t)ewm::H * ewm::H);
    fill(ewm::off_W3(), ewm::H, (size_t)ewm::H * m->no);
    const size_t bytes = m->n * sizeof(float);
    if (hipMalloc(&m->d_p, bytes) != hipSuccess || hipMalloc(&m->d_g, bytes) != hipSuccess ||
        hipMalloc(&m->d_m, bytes) != hipSuccess || hipMalloc(&m->d_v, bytes) != hipSuccess) {
        delete m;
        return mfail(EWAH_ENOMEM, "device allocation failed");
    }
    MCHK(hipMemcpy(m->d_p, h.data(), bytes, hipMemcpyHostToDevice));
    MCHK(hipMemset(m->d_g, 0, bytes));
    MCHK(hipMemset(m->d_m, 0, bytes));
    MCHK(hipMemset(m->d_v, 0, bytes));
    MCHK(hipFuncSetAttribute((const void*)ewm::mlp_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ewm::grad_smem(ewm::NOMAX)));
    *out = m;
    return EWAH_OK;
}

void ewah_mlp_free(ewah_mlp* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(m->d_p);
    (void)hipFree(m->d_g);
    (void)hipFree(m->d_m);
    (void)hipFree(m->d_v);
    delete m;
}

ewah_status ewah_mlp_get_params(const ewah_mlp* m, float* host, uint64_t n) {
    if (!m || !host || n != m->n) return mfail(EWAH_EINVAL, "bad arguments");
    MCHK(hipDeviceSynchronize());
    MCHK(hipMemcpy(host, m->d_p, n * sizeof(float), hipMemcpyDeviceToHost));
    return EWAH_OK;
}

ewah_status ewah_mlp_set_params(ewah_mlp* m, const float* host, uint64_t n) {
    if (!m || !host || n != m->n) return mfail(EWAH_EINVAL, "bad arguments");
    MCHK(hipDeviceSynchronize());
    MCHK(hipMemcpy(m->d_p, host, n * sizeof(float), hipMemcpyHostToDevice));
    MCHK(hipMemset(m->d_m, 0, n * sizeof(float)));
    MCHK(hipMemset(m->d_v, 0, n * sizeof(float)));
    m->step = 0;
    return EWAH_OK;
}

ewah_status ewah_mlp_forward(ewah_mlp* m, const float* x_dev, uint32_t batch, float* y_dev, void* stream) {
    if (!m || (batch && (!x_dev || !y_dev))) return mfail(EWAH_EINVAL, "bad arguments");
    if (!batch) return EWAH_OK;
    hipLaunchKernelGGL(ewm::mlp_forward_kernel, dim3((batch + 255) / 256), dim3(256), m->n * sizeof(float),
                       (hipStream_t)stream, x_dev, m->d_p, y_dev, batch, m->no);
    MCHK(hipGetLastError());
    return EWAH_OK;
}

ewah_status ewah_mlp_grad(ewah_mlp* m, const float* x_dev, const float* t_dev, uint32_t batch, float* grad_dev,
                          float* loss_dev, void* stream) {
    if (!m || !x_dev || !t_dev || !grad_dev || !loss_dev || batch == 0) return mfail(EWAH_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t n = (uint32_t)m->n;
    hipLaunchKernelGGL(ewm::fill_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, grad_dev, n);
    hipLaunchKernelGGL(ewm::fill_zero_kernel, dim3(1), dim3(1), 0, s, loss_dev, 1u);
    hipLaunchKernelGGL(ewm::mlp_grad_kernel, dim3((batch + ewm::SB - 1) / ewm::SB), dim3(ewm::SB), ewm::grad_smem(m->no),
                       s, x_dev, t_dev, m->d_p, grad_dev, loss_dev, batch, m->no, 1.f / ((float)batch * (float)m->no));
    MCHK(hipGetLastError());
    return EWAH_OK;
}

ewah_status ewah_mlp_train_step(ewah_mlp* m, const float* x_dev, const float* t_dev, uint32_t batch, float lr,
                                float* loss_dev, void* stream) {
    if (!m || !x_dev || !t_dev || !loss_dev || batch == 0) return mfail(EWAH_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t n = (uint32_t)m->n;
    hipLaunchKernelGGL(ewm::fill_zero_kernel, dim3(1), dim3(1), 0, s, loss_dev, 1u);
    hipLaunchKernelGGL(ewm::mlp_grad_kernel, dim3((batch + ewm::SB - 1) / ewm::SB), dim3(ewm::SB), ewm::grad_smem(m->no),
                       s, x_dev, t_dev, m->d_p, m->d_g, loss_dev, batch, m->no, 1.f / ((float)batch * (float)m->no));
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
    hipLaunchKernelGGL(ewm::mlp_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m->d_p, m->d_g, m->d_m, m->d_v,
                       n, lr, b1, b2, 1e-8f, c1, c2);
    MCHK(hipGetLastError());
    return EWAH_OK;
}

}  // extern "C"
