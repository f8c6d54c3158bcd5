// Streaming-read ceiling of the device for the access shape of the tile
// kernel: every wavefront reads 512-byte chunks (64 lanes x 8 bytes), B chunks
// in flight per wavefront, over a 4 GiB buffer; chunks taken in order (stride
// 1) or scattered (a large odd stride modulo the buffer).  Prints GB/s, best
// of 4 runs.  Measurement tool: not part of the query path.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

template <int B>
__global__ __launch_bounds__(1024) void read_chunks(const uint64_t* __restrict__ p, size_t nchunks, uint64_t* out,
                                                    uint32_t stride) {
    const int lane = threadIdx.x & 63;
    const size_t nw = (size_t)gridDim.x * (blockDim.x / 64);
    const size_t wid = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const size_t per = (nchunks + nw - 1) / nw;
    const size_t beg = wid * per, end = beg + per < nchunks ? beg + per : nchunks;
    uint64_t acc = 0;
    for (size_t c0 = beg; c0 < end; c0 += B) {
        uint64_t v[B];
#pragma unroll
        for (int g = 0; g < B; ++g) {
            const size_t c = ((c0 + g) * stride) % nchunks;
            v[g] = (c0 + g < end) ? __builtin_nontemporal_load(p + c * 64 + lane) : 0;
        }
#pragma unroll
        for (int g = 0; g < B; ++g) acc ^= v[g];
    }
    if (acc == 0x123456789ull) out[0] = acc;   // keeps the loads
}

int main() {
    const size_t bytes = (size_t)4 << 30;
    uint64_t *p = nullptr, *o = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || hipMalloc(&o, 64) != hipSuccess) return 1;
    if (hipMemset(p, 1, bytes) != hipSuccess) return 1;
    const size_t nchunks = bytes / 512;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1;
    for (uint32_t stride : {1u, 7919u}) {
        for (int batch : {4, 8, 16}) {
            float best = 1e30f;
            for (int rep = 0; rep < 4; ++rep) {
                (void)hipEventRecord(a);
                if (batch == 4) hipLaunchKernelGGL(read_chunks<4>, dim3(512), dim3(1024), 0, 0, p, nchunks, o, stride);
                if (batch == 8) hipLaunchKernelGGL(read_chunks<8>, dim3(512), dim3(1024), 0, 0, p, nchunks, o, stride);
                if (batch == 16) hipLaunchKernelGGL(read_chunks<16>, dim3(512), dim3(1024), 0, 0, p, nchunks, o, stride);
                (void)hipEventRecord(b);
                (void)hipEventSynchronize(b);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, a, b);
                if (ms < best) best = ms;
            }
            printf("%s 512-byte chunks, %2d per wavefront in flight: %.1f GB/s\n", stride == 1 ? "sequential" : "scattered ",
                   batch, bytes / best / 1e6);
        }
    }
    return 0;
}
