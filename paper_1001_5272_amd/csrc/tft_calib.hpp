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

// A word of the lane (lane ^ s), s = 1, 2 or 4, by cross-lane data movement
// without LDS memory: DPP quad permutations for s = 1, 2, ds_swizzle (xor
// mode inside 32 lanes) for s = 4; 64-bit words as two 32-bit moves.
template <int S>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v) {
    if constexpr (S == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    else if constexpr (S == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // 2,3,0,1
    else return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (4 << 10) | 0x1F);   // xor 4, and 0x1f
}
template <int S, class Word>
__device__ __forceinline__ Word xor_lane(Word v) {
    if constexpr (sizeof(Word) == 8)
        return ((uint64_t)xor_lane32<S>((uint32_t)(v >> 32)) << 32) | xor_lane32<S>((uint32_t)v);
    else
        return xor_lane32<S>(v);
}

// The radix-8 units of k_cal_bfly, each followed by the exchange a pass needs
// between its units: an 8 x 8 transpose inside every group of eight lanes
// (lane i of a group then holds word i of each of the group's units).
// XCHG 0: through LDS, as the pass kernels do it (each lane writes its eight
// words, a barrier, each lane reads its column, a barrier); 1: lane shuffles
// (ds_bpermute); 2: DPP and ds_swizzle.  1 and 2 run three xor stages that
// each move 4 of the 8 words.  All three leave the same values; they measure
// the cost of the ways to exchange.
template <int S, int XCHG, class Word>
__device__ __forceinline__ void xchg_stage(Word (&v)[8], uint32_t lane8) {
    const bool up = (lane8 & (uint32_t)S) != 0;
#pragma unroll
    for (int t = 0; t < 8; t++) {
        if (t & S) continue;
        const Word send = up ? v[t] : v[t | S];
        const Word recv = XCHG == 1 ? shfl_xor_word(send, S) : xor_lane<S>(send);
        if (up)
            v[t] = recv;
        else
            v[t | S] = recv;
    }
}
template <class Mod, int XCHG>
__global__ __launch_bounds__(kCalThreads) void k_cal_xchg(Mod md, typename Mod::Word* x,
                                                         const typename Mod::Word* tw, int iters) {
    using Word = typename Mod::Word;
    __shared__ Word sh[kCalThreads * 8 + kCalThreads / 4];
    const uint32_t id = blockIdx.x * kCalThreads + threadIdx.x;
    const uint32_t lane8 = threadIdx.x & 7, base = threadIdx.x & ~7u;
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
        if constexpr (XCHG == 0) {
#pragma unroll
            for (int t = 0; t < 8; t++) sh[pad(threadIdx.x * 8 + t)] = v[t];
            lds_sync();
#pragma unroll
            for (int t = 0; t < 8; t++) v[t] = sh[pad((base + t) * 8 + lane8)];
            lds_sync();
        } else {
            xchg_stage<1, XCHG>(v, lane8);
            xchg_stage<2, XCHG>(v, lane8);
            xchg_stage<4, XCHG>(v, lane8);
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
