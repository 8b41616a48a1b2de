// Calibration kernels: register-only and copy-only loops that measure the
// roofline denominators of this device (the peaks the transform kernels are
// reported against).  They do no transform work.
#pragma once

#include "tft_device.hpp"

namespace tft {

constexpr int kCalThreads = 256;

// 32-bit VALU: eight independent chains of a = (a ^ b) + s per lane (one
// v_xad_u32 each).
__global__ __launch_bounds__(kCalThreads) void k_cal_valu(uint32_t* out, uint32_t s, int iters) {
    uint32_t a[8];
#pragma unroll
    for (int i = 0; i < 8; i++) a[i] = s * (threadIdx.x + 7 * i + 1);
    for (int r = 0; r < iters; r++) {
#pragma unroll
        for (int i = 0; i < 8; i++) a[i] = (a[i] ^ a[(i + 1) & 7]) + s;
    }
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) x ^= a[i];
    out[blockIdx.x * kCalThreads + threadIdx.x] = x;
}

// 32 x 32 + 64 -> 64 multiply-add (v_mad_u64_u32), eight chains per lane.
__global__ __launch_bounds__(kCalThreads) void k_cal_mad64(uint32_t* out, uint32_t s, int iters) {
    uint64_t b[8];
#pragma unroll
    for (int i = 0; i < 8; i++) b[i] = (uint64_t)(s + threadIdx.x + i) * 0x9E3779B97F4A7C15ull;
    for (int r = 0; r < iters; r++) {
#pragma unroll
        for (int i = 0; i < 8; i++) b[i] = (uint64_t)(uint32_t)b[i] * (uint32_t)(b[(i + 3) & 7] >> 32) + b[i];
    }
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) x ^= (uint32_t)b[i] ^ (uint32_t)(b[i] >> 32);
    out[blockIdx.x * kCalThreads + threadIdx.x] = x;
}

// Butterflies in registers: radix-8 units (12 butterflies each) with the
// device arithmetic of the transforms, no memory traffic in the loop.
template <class Mod>
__global__ __launch_bounds__(kCalThreads) void k_cal_bfly(Mod md, typename Mod::Word* x,
                                                         const typename Mod::Word* tw, int iters) {
    using Word = typename Mod::Word;
    const uint32_t id = blockIdx.x * kCalThreads + threadIdx.x;
    Word v[8], w[7];
#pragma unroll
    for (int t = 0; t < 8; t++) v[t] = x[id * 8 + t];
#pragma unroll
    for (int t = 0; t < 7; t++) w[t] = tw[t];
    for (int r = 0; r < iters; r++) {
#pragma unroll
        for (int s = 0; s < 3; s++) {
            const int dist = 8 >> (s + 1);
#pragma unroll
            for (int q = 0; q < (1 << s); q++) {
#pragma unroll
                for (int t = 0; t < dist; t++) {
                    const int a = q * 2 * dist + t, b = a + dist;
                    const Word u = v[a], m = md.mul_tw(v[b], w[(1 << s) - 1 + q]);
                    v[a] = md.add(u, m);
                    v[b] = md.sub(u, m);
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 8; t++) x[id * 8 + t] = v[t];
}

// HBM copy, 16 bytes per lane per step.
__global__ __launch_bounds__(kCalThreads) void k_cal_copy(uint4* dst, const uint4* src, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * kCalThreads + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kCalThreads)
        dst[i] = src[i];
}

}  // namespace tft
