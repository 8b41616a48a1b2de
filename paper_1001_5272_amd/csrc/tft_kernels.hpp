// Kernels of the in-place truncated Fourier transform (Harvey & Roche 2010).
//
// Two schedules compute the same map X_s = F(w_s), s < n:
//
// 1. Single workgroup (n fits in LDS): the whole length-n transform runs in one
//    LDS block of 2^ceil(lg n) words (the block is on-chip scratch; HBM holds
//    exactly n words).
//
// 2. Two passes over HBM with n = a W + b, W = 2^R, 0 <= b < W.  Column c < W is
//    the tree node (c, R) of section 3 (the strided subarray F_{c + d W}), of
//    length a + 1 for c < b and a for c >= b.  Writing P_c(x) = sum_d F_{c+dW} x^d,
//    the identities w_s^{2^R} = w_{s >> R} and w_{u+e} = w_u w_e for e < 2^R | u
//    (section 2.2) give
//          X_{jW+e} = sum_c w_{jW+e}^c P_c(w_j),
//    i.e. row j is the length-W transform, at global block index j, of the
//    column values P_c(w_j).  The column pass evaluates every column at
//    w_0..w_a in place.  Full rows j < a then need only their own slots.  The
//    partial last row j = a has b slots but needs P_c(w_a) of every column:
//    columns c < b store it in their own last slot; columns c >= b have no slot
//    for it, so the column pass emits it as an extra value V_c.  This is the
//    paper's odd-length correction (Algorithm 1, the value v evaluated at
//    w_{(m-1)/2} and added into S_{m-1}) lifted to the W-way split: the last
//    row's transform combines its own b values with the W - b values V_c and
//    keeps b outputs.  The V_c live in a fixed context scratch of at most W
//    words, independent of n.  The inverse runs the passes backwards: full
//    rows, then columns c >= b (which also re-derive V_c from the restored
//    coefficients), then the last row with the V_c as known coefficients, then
//    columns c < b (section 4: the correction is removed after the subtree it
//    reads is restored).
#pragma once
#include "tft_device.hpp"

namespace tft {

constexpr int kThreads = 256;        // elementwise kernels and the persistent batch kernel
constexpr int kColThreads = 512;     // column passes: 8 waves per workgroup (measured best)
constexpr int kRowThreads = 1024;    // row passes: 16 waves per workgroup (measured best)

template <class Word>
__device__ __forceinline__ Word* lds_buf() {
    extern __shared__ __align__(16) unsigned char tft_smem[];
    return reinterpret_cast<Word*>(tft_smem);
}

// Workgroup ids are dealt round-robin to the 8 XCDs; map consecutive logical
// tiles (which share 128-byte HBM lines) onto the same XCD so they share L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t x, uint32_t tiles) {
    if (tiles < 16 || (tiles & 7u)) return x;
    return (x & 7u) * (tiles >> 3) + (x >> 3);
}

// The same for a work list of n items (adjacent items are neighbouring tiles
// of one transform): a bijection on [0, n), identity on the last n mod 8.
__device__ __forceinline__ uint32_t xcd_remap_list(uint32_t x, uint32_t n) {
    const uint32_t full = n & ~7u;
    if (full < 16 || x >= full) return x;
    return (x & 7u) * (full >> 3) + (x >> 3);
}

// ------------------------------------------------------ single workgroup
template <class Mod>
__device__ __forceinline__ void small_forward_body(const Mod& md, const Tables<typename Mod::Word>& T0, typename Mod::Word* X,
                                   uint32_t n, uint32_t M, uint64_t g0 = 0) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    const Tables<Word> L = local_tables(T0, buf + padded_words(M), M / 2);
    for (uint32_t i = threadIdx.x; i < M; i += nthreads()) buf[pad(i)] = i < n ? X[i] : Word(0);
    __syncthreads();
    dif_forward(md, L, buf, 0, M, 0, n, g0);
    for (uint32_t i = threadIdx.x; i < n; i += nthreads()) X[i] = buf[pad(i)];
}

template <class Mod>
__device__ __forceinline__ void small_inverse_body(const Mod& md, const Tables<typename Mod::Word>& T0, typename Mod::Word* X,
                                   uint32_t n, uint32_t M) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    const Tables<Word> L = local_tables(T0, buf + padded_words(M), M / 2);
    for (uint32_t i = threadIdx.x; i < M; i += nthreads()) buf[pad(i)] = i < n ? X[i] : Word(0);
    __syncthreads();
    gitft(md, L, buf, 0, M, n, 0);
    for (uint32_t i = threadIdx.x; i < n; i += nthreads()) X[i] = buf[pad(i)];
}

// Whole product in one workgroup: both operands zero-extended to M words of
// LDS (M = 2^ceil(lg r), on-chip scratch; X in HBM holds only the r words of
// the product), full M-point forward transforms, pointwise product and full
// M-point inverse: the product has degree < r <= M, so the cyclic product of
// length M is the product itself.  The full inverse (one scaling by 1/M on the
// store) replaces the truncated inverse's dependent walk, the longest part of
// a single-workgroup product.
template <class Mod>
__device__ __forceinline__ void small_mul_body(const Mod& md, const Tables<typename Mod::Word>& T0, const typename Mod::Word* A,
                               uint32_t m, const typename Mod::Word* B, uint32_t nb, typename Mod::Word* X,
                               uint32_t M) {
    using Word = typename Mod::Word;
    Word* ba = lds_buf<Word>();
    Word* bb = ba + padded_words(M);
    const Tables<Word> L = local_tables(T0, ba + 2 * padded_words(M), M / 2);
    const uint32_t r = m + nb - 1;
    for (uint32_t i = threadIdx.x; i < M; i += nthreads()) {
        ba[pad(i)] = i < m ? A[i] : Word(0);
        bb[pad(i)] = i < nb ? B[i] : Word(0);
    }
    __syncthreads();
    dif_forward(md, L, ba, 0, M, 0, M, 0);
    dif_forward(md, L, bb, 0, M, 0, M, 0);
    // the products up to the factor that the store's scaling takes back
    for (uint32_t i = threadIdx.x; i < M; i += nthreads()) ba[pad(i)] = md.mul_scaled(ba[pad(i)], bb[pad(i)]);
    __syncthreads();
    full_inverse<Mod, false>(md, L, ba, 0, 0, M, 0);
    const Word sc = md.tw_mul_tw(inv_pow2_tw(md, __builtin_ctz(M)), md.kappa_tw());
    for (uint32_t i = threadIdx.x; i < r; i += nthreads()) X[i] = md.mul_tw(ba[pad(i)], sc);
}

// Single-instance single-workgroup kernels are latency-bound: run 16 waves.
constexpr int kSmallThreads = 1024;

template <class Mod>
__global__ __launch_bounds__(kSmallThreads) void k_small_fwd(Mod md, Tables<typename Mod::Word> T,
                                                        typename Mod::Word* X, uint32_t n, uint32_t M, uint64_t g0,
                                                        uint64_t stride) {
    // workgroup b transforms X + b stride (several blocks of one length)
    small_forward_body(md, T, X + blockIdx.x * stride, n, M, g0);
}

template <class Mod>
__global__ __launch_bounds__(kSmallThreads) void k_small_inv(Mod md, Tables<typename Mod::Word> T,
                                                        typename Mod::Word* X, uint32_t n, uint32_t M) {
    small_inverse_body(md, T, X, n, M);
}

template <class Mod>
__global__ __launch_bounds__(kSmallThreads) void k_small_mul(Mod md, Tables<typename Mod::Word> T,
                                                        const typename Mod::Word* A, uint32_t m,
                                                        const typename Mod::Word* B, uint32_t nb,
                                                        typename Mod::Word* X, uint32_t M) {
    small_mul_body(md, T, A, m, B, nb, X, M);
}

// ------------------------------------------------------------ two passes
// One in-place two-pass transform of length n = a W + b (W = 2^logW): the data
// X, the column-pass source (X itself, or a shorter read-only operand that is
// implicitly zero-extended to n), the W-word area V for the extra column
// evaluations, and an optional pointwise multiplier Y applied on the first
// inverse load.
template <class Word>
struct TwoPass {
    Word* X;
    const Word* src;
    const Word* Y;
    Word* V;
    uint64_t n_src, n;
    uint32_t logW, a, b, Lout, M;
    uint32_t split;   // 1: Lout = M + 1 with M a power of two (see col_fwd_body)
    uint32_t early;   // inverse with b > 0: 0 columns c < b after the last row; 1 split mode, 2 general
                      // (columns c < b run with phase 0, see col_inv_body and last_inv_body);
                      // 3 b = W - 1 with a + 1 a power of two (see tail_inv_body)
    Word* Q;          // early == 2: Q_0..Q_a at Q, scratch at Q + kQStride, 1 / Q(w_a) at Q[2 kQStride]
    uint64_t g0;      // forward of a whole block (n = a W, b = 0): the block's global index, else 0
    uint32_t nparts;  // inverse with b = 1: column tiles leaving a partial last-row sum at Q + kQStride, or 0
    uint32_t ldstw;   // 1: column tiles copy their block-0 twiddles to LDS; 0: read them from the table in memory
                      // (when the copy would cost a tile per CU)
    uint64_t inst;    // forward over whole blocks (b = 0) with gridDim.y > 1: instance y at X + y inst (and src + y inst)
};
constexpr uint32_t kQStride = (1u << 16) + 64;

constexpr int kMaxC = 16;   // widest column tile
constexpr int kLastThreads = 1024;   // the last-row inverse is one workgroup: give it many waves

// A column transform of len values, len not a power of two, may split at H,
// the largest power of two below len: with R = len - H it needs a block of
// S = 2^ceil(lg R) words besides the H-word block, and is used when
// H/32 <= S <= H/4 (then H + S words of LDS per column instead of 2H; see
// col_fwd_body and col_inv_body).
__host__ __device__ inline bool col_split(uint32_t len, uint32_t* H, uint32_t* S) {
    uint32_t h = 1;
    while (2 * h < len) h <<= 1;   // h < len <= 2h
    if (h == len || h < 64) return false;
    uint32_t s = 1;
    while (s < len - h) s <<= 1;
    // S <= H/4 saves a quarter of the LDS or more (at S = H/2 the unfused
    // passes cost more than the smaller tile gains, measured at a = 768);
    // S >= H/32 keeps the fold (H/S terms per word, one dependent chain per
    // thread) short
    if (4 * s > h || 32 * s < h) return false;
    *H = h;
    *S = s;
    return true;
}

// Forward column pass over the tile of C columns starting at column tile*C:
// evaluates each column polynomial at w_0..w_{Lout-1} (Lout = a + (b > 0)) in
// an LDS block of M = 2^ceil(lg Lout) words per column, writes the outputs
// that have a slot and the extra value P_c(w_a) of columns c >= b to V[c].
template <class Mod, int LOGC, bool HS = false>
__device__ __forceinline__ void col_fwd_body(const Mod& md, const Tables<typename Mod::Word>& T0,
                             const TwoPass<typename Mod::Word>& P, uint32_t tile) {
    using Word = typename Mod::Word;
    constexpr uint32_t C = 1u << LOGC;
    __shared__ Word red[(kColThreads / 64) * C];
    __shared__ Word extra[C], hi0[C];
    Word* buf = lds_buf<Word>();
    uint32_t Hs = 0, Ss = 0;
    const bool hs = HS && !P.split && P.g0 == 0 && P.Lout != P.M && col_split(P.Lout, &Hs, &Ss);
    const Tables<Word> T = hs ? local_tables<Word, true, false>(T0, buf + padded_words((Hs + Ss) << LOGC),
                                                                P.ldstw ? Hs / 2 : 0u)
                              : local_tables<Word, true, false>(T0, buf + padded_words(P.M << LOGC),
                                                                P.ldstw ? P.M / 2 : 0u);
    const uint32_t c0 = tile * C;
    const uint64_t W = 1ull << P.logW;
    // b = 1 (P.nparts): the tile's share sum_c Z_c w_{aW}^c of the last row's
    // one output, Z_c = P_c(w_a) being output a of column c (slot or V_c)
    __shared__ Word ypow[C], zterm[C];
    const bool share = P.b == 1 && P.nparts;
    if (share && threadIdx.x < C) ypow[threadIdx.x] = pow_tw(md, tw_fwd(md, T, (uint64_t)P.a << P.logW), c0 + threadIdx.x);
    auto put_share = [&]() {
        __syncthreads();
        if (threadIdx.x == 0) {
            Word sum = 0;
            for (uint32_t c = 0; c < C; c++) sum = md.add(sum, zterm[c]);
            P.Q[kQStride + tile] = sum;
        }
    };
    if (P.split) {
        // Lout = H + 1 with H = P.M a power of two, and every column has at
        // most H + 1 coefficients.  Outputs s < H are the H-point transform of
        // P_c mod (x^H - 1) = lo + hi (hi is only the coefficient x_H); output
        // H is P_c(w_H) = (lo - hi)(w_H) = (lo + hi)(w_H) - 2 x_H, one
        // evaluation of the folded block taken before its transform.
        const uint32_t H = P.M;
        __shared__ Word zp[kColThreads >> LOGC];   // one power per thread of a lane
        for (uint32_t c = threadIdx.x; c < C; c += nthreads()) {
            const uint64_t idx = (c0 + c) + (uint64_t)H * W;
            hi0[c] = idx < P.n_src ? P.src[idx] : Word(0);
        }
        if (H >= 16) {
            // the first radix-8 group straight from HBM (as below), each unit
            // also adding its share of the evaluation at z = w_H: the rows
            // u + t H/8 contribute z^u sum_t x_t (z^(H/8))^t
            __syncthreads();
            const uint32_t M8 = H >> 3, maskK = (1u << T.K) - 1;
            const uint32_t EH = __builtin_bitreverse32(H) >> (32 - T.K);   // w_H = w[K]^EH
            const Word z8 = root_pow(md, T, (M8 * EH) & maskK);
            Unit<Mod, 3> top;
            top.load0(T.lf, 0, 0);
            Word acc = 0;
            for (uint32_t it = threadIdx.x; it < M8 * C; it += nthreads()) {
                const uint32_t c = it & (C - 1), u = it >> LOGC;
                Word x[8];
#pragma unroll
                for (int t = 0; t < 8; t++) {
                    const uint64_t idx = (c0 + c) + (uint64_t)(u + t * M8) * W;
                    x[t] = idx < P.n_src ? P.src[idx] : Word(0);
                }
                if (u == 0) x[0] = md.add(x[0], hi0[c]);
                Word e = x[7];
#pragma unroll
                for (int t = 6; t >= 0; t--) e = md.add(md.mul_tw(e, z8), x[t]);
                acc = md.add(acc, md.mul_tw(e, root_pow(md, T, (u * EH) & maskK)));
                top.template forward<true>(md, x);
#pragma unroll
                for (int t = 0; t < 8; t++) buf[pad(u * C + c) + pad_step(t, M8 * C)] = x[t];
            }
            reduce_lanes(md, acc, LOGC, red, extra);   // its barriers also publish the tile
            if (H >= 64) {
                // the last group straight to HBM (outputs d < H), then output H
                dif_stages(md, T, buf, LOGC, H, H >> 4, 8, 0, H, 0);
                for (uint32_t it = threadIdx.x; it < M8 * C; it += nthreads()) {
                    const uint32_t c = it & (C - 1), i = it >> LOGC;
                    Word x[8];
#pragma unroll
                    for (int t = 0; t < 8; t++) x[t] = buf[pad(8 * i * C + c) + pad_step(t, C)];
                    Unit<Mod, 3> un;
                    un.load0(T.lf, 0, i);
                    un.forward(md, x);
#pragma unroll
                    for (int t = 0; t < 8; t++) {
                        const uint64_t idx = (c0 + c) + (uint64_t)(8 * i + t) * W;
                        if (idx < P.n) P.X[idx] = x[t];
                    }
                }
                for (uint32_t c = threadIdx.x; c < C; c += nthreads()) {
                    const uint64_t idx = (c0 + c) + (uint64_t)H * W;
                    const Word v = md.sub(md.sub(extra[c], hi0[c]), hi0[c]);
                    if (idx < P.n)
                        P.X[idx] = v;
                    else if (P.b && H == P.a)
                        P.V[c0 + c] = v;
                    if (share) zterm[c] = md.mul_tw(v, ypow[c]);
                }
                if (share) put_share();
                return;
            }
            dif_stages(md, T, buf, LOGC, H, H >> 4, 1, 0, H, 0);
        } else {
            eval_scales(md, LOGC, H, tw_fwd(md, T, H), zp);
            __syncthreads();
            for (uint32_t it = threadIdx.x; it < H * C; it += nthreads()) {
                const uint32_t c = it & (C - 1), d = it >> LOGC;
                const uint64_t idx = (c0 + c) + (uint64_t)d * W;
                Word v = idx < P.n_src ? P.src[idx] : Word(0);
                if (d == 0) v = md.add(v, hi0[c]);
                buf[pad(it)] = v;
            }
            __syncthreads();
            eval_lanes(md, buf, LOGC, H, tw_fwd(md, T, H), red, extra, zp);
            dif_forward(md, T, buf, LOGC, H, 0, H, 0);
        }
        for (uint32_t it = threadIdx.x; it < (H + 1) * C; it += nthreads()) {
            const uint32_t c = it & (C - 1), d = it >> LOGC;
            const uint64_t idx = (c0 + c) + (uint64_t)d * W;
            const Word v = d < H ? buf[pad(it)] : md.sub(md.sub(extra[c], hi0[c]), hi0[c]);
            if (idx < P.n)
                P.X[idx] = v;
            else if (P.b && d == P.a)
                P.V[c0 + c] = v;
            if (share && d == H) zterm[c] = md.mul_tw(v, ypow[c]);
        }
        if (share) put_share();
        return;
    }
    if constexpr (HS) if (hs) {
        // Lout = H + R outputs, R <= S <= H/4, and every column has at most
        // Lout coefficients: P = lo + x^H hi (hi: R coefficients at most).
        // Outputs s < H are the block-0 transform of A = P mod (x^H - 1)
        // = lo + hi; outputs H .. H + R - 1 lie in the block of size S at
        // global index H/S, which holds (lo - hi) mod (x^S - w_{H/S}):
        // F_j = sum_k A_{j + k S} w_{H/S}^k - 2 hi_j.  H + S words of LDS per
        // column instead of 2H.
        const uint32_t H = Hs, S = Ss, R = P.Lout - Hs;
        Word* fb = buf + pad(H << LOGC);   // the block of S words (H C is a multiple of 32)
        staged_copy<8>(H * C, [&](uint32_t it) {
            const uint32_t c = it & (C - 1), d = it >> LOGC;
            const uint64_t idx = (c0 + c) + (uint64_t)d * W;
            return idx < P.n_src ? P.src[idx] : Word(0);
        }, [&](uint32_t it, Word v) { buf[pad(it)] = v; });
        staged_copy<8>(S * C, [&](uint32_t it) {
            const uint32_t c = it & (C - 1), j = it >> LOGC;
            const uint64_t idx = (c0 + c) + (uint64_t)(H + j) * W;
            return (j < R && idx < P.n_src) ? P.src[idx] : Word(0);
        }, [&](uint32_t it, Word v) { fb[pad(it)] = v; });
        __syncthreads();
        for (uint32_t it = threadIdx.x; it < (R << LOGC); it += nthreads()) buf[pad(it)] = md.add(buf[pad(it)], fb[pad(it)]);
        __syncthreads();
        const Word cf = tw_fwd(md, T, H / S);
        for (uint32_t it = threadIdx.x; it < (S << LOGC); it += nthreads()) {
            const uint32_t c = it & (C - 1), j = it >> LOGC;
            Word acc = 0;
            for (uint32_t k = H / S; k-- > 0;) acc = md.add(md.mul_tw(acc, cf), buf[pad((j + k * S) * C + c)]);
            const Word h = fb[pad(it)];
            fb[pad(it)] = md.sub(md.sub(acc, h), h);
        }
        __syncthreads();
        dif_forward(md, T, buf, LOGC, H, 0, H, 0);       // outputs 0 .. H-1
        dif_forward(md, T, fb, LOGC, S, 0, R, H / S);    // outputs H .. H+R-1
        staged_copy<8>(P.Lout * C, [&](uint32_t it) { return buf[pad(it)]; }, [&](uint32_t it, Word v) {
            const uint32_t c = it & (C - 1), d = it >> LOGC;
            const uint64_t idx = (c0 + c) + (uint64_t)d * W;
            if (idx < P.n)
                P.X[idx] = v;
            else if (P.b && d == P.a)
                P.V[c0 + c] = v;
            if (share && d == P.a) zterm[c] = md.mul_tw(v, ypow[c]);
        });
        if (share) put_share();
        return;
    }
    // A zero-extended source (a product's operand) may fill only the first zr
    // rows of the tile's columns.  With Z = 2^ceil(lg zr), the stages of block
    // size above Z pair every value with a zero (the high half), so each only
    // copies a block into both children: after them every block of size Z
    // holds the same Z values.  Those stages are skipped by writing the Z rows
    // into every block that meets [0, Lout) and running the stages below.
    uint32_t zr = P.M, Z = P.M;
    if (P.g0 == 0 && P.n_src < P.n) {
        const uint64_t rows = P.n_src > c0 ? (P.n_src - c0 + W - 1) / W : 0;
        zr = (uint32_t)(rows < P.Lout ? rows : P.Lout);
        Z = 1;
        while (Z < zr) Z <<= 1;
    }
    if (8 * Z <= P.M) {
        const uint32_t live = (P.Lout + Z - 1) / Z * Z;   // rows of the blocks that meet [0, Lout), <= M
        for (uint32_t it = threadIdx.x; it < (Z << LOGC); it += nthreads()) {
            const uint32_t c = it & (C - 1), d = it >> LOGC;
            const uint64_t idx = (c0 + c) + (uint64_t)d * W;
            const Word v = (d < zr && idx < P.n_src) ? P.src[idx] : Word(0);
            for (uint32_t k = d; k < live; k += Z) buf[pad((k << LOGC) + c)] = v;
        }
        __syncthreads();
        if (Z >= 2) dif_stages(md, T, buf, LOGC, P.M, Z >> 1, 1, 0, P.Lout, 0);
    } else if (P.g0 == 0 && P.M >= 16) {
        // the first radix-8 group (stages M/2, M/4, M/8 of block 0) straight
        // from HBM: the unit of lane c at u holds rows u + t M/8
        const uint32_t M8 = P.M >> 3;
        Unit<Mod, 3> top;
        top.load0(T.lf, 0, 0);
        for (uint32_t it = threadIdx.x; it < M8 * C; it += nthreads()) {
            const uint32_t c = it & (C - 1), u = it >> LOGC;
            Word x[8];
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const uint32_t d = u + t * M8;
                const uint64_t idx = (c0 + c) + (uint64_t)d * W;
                x[t] = (d < P.Lout && idx < P.n_src) ? P.src[idx] : Word(0);
            }
            top.template forward<true>(md, x);
#pragma unroll
            for (int t = 0; t < 8; t++) buf[pad(u * C + c) + pad_step(t, M8 * C)] = x[t];
        }
        __syncthreads();
        if (P.M >= 64) {
            // the last group (stages 4, 2, 1 on eight consecutive rows) straight
            // to HBM, for the blocks of eight that meet [0, Lout)
            dif_stages(md, T, buf, LOGC, P.M, P.M >> 4, 8, 0, P.Lout, 0);
            const uint32_t blocks = (P.Lout + 7) >> 3;
            for (uint32_t it = threadIdx.x; it < blocks * C; it += nthreads()) {
                const uint32_t c = it & (C - 1), i = it >> LOGC;
                Word x[8];
#pragma unroll
                for (int t = 0; t < 8; t++) x[t] = buf[pad(8 * i * C + c) + pad_step(t, C)];
                Unit<Mod, 3> un;
                un.load0(T.lf, 0, i);
                un.forward(md, x);
#pragma unroll
                for (int t = 0; t < 8; t++) {
                    const uint32_t d = 8 * i + t;
                    const uint64_t idx = (c0 + c) + (uint64_t)d * W;
                    if (d >= P.Lout) break;
                    if (idx < P.n)
                        P.X[idx] = x[t];
                    else if (P.b && d == P.a)
                        P.V[c0 + c] = x[t];
                    if (share && d == P.a) zterm[c] = md.mul_tw(x[t], ypow[c]);
                }
            }
            if (share) put_share();
            return;
        }
        dif_stages(md, T, buf, LOGC, P.M, P.M >> 4, 1, 0, P.Lout, 0);
    } else {
        staged_copy<8>(P.M * C, [&](uint32_t it) {
            const uint32_t c = it & (C - 1), d = it >> LOGC;
            const uint64_t idx = (c0 + c) + (uint64_t)d * W;
            return (d < P.Lout && idx < P.n_src) ? P.src[idx] : Word(0);
        }, [&](uint32_t it, Word v) { buf[pad(it)] = v; });
        __syncthreads();
        dif_forward(md, T, buf, LOGC, P.M, 0, P.Lout, P.g0);
    }
    staged_copy<8>(P.Lout * C, [&](uint32_t it) { return buf[pad(it)]; }, [&](uint32_t it, Word v) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        const uint64_t idx = (c0 + c) + (uint64_t)d * W;
        if (idx < P.n)
            P.X[idx] = v;
        else if (P.b && d == P.a)
            P.V[c0 + c] = v;
        if (share && d == P.a) zterm[c] = md.mul_tw(v, ypow[c]);
    });
    if (share) put_share();
}

// Full rows of W = 2^logW words, logW >= 6, with the first and last radix-8
// groups fused with the HBM transfers: a unit of the first forward group
// (stages W/2, W/4, W/8) holds words u + t W/8, t < 8 -- one coalesced load
// per t -- and a unit of the last group (stages 4, 2, 1) holds eight
// consecutive words; the inverse runs the same groups in the other order.
// Each unit works on its own loads as soon as they land, and the row makes
// two LDS round trips and two barriers fewer than a load / transform / store
// sequence.  Twiddles of block 0: w_{2x} = tab[x << sh].

// 8 consecutive words at p (p 64-byte aligned)
template <class Word>
__device__ __forceinline__ void load8(const Word* p, Word (&x)[8]) {
#pragma unroll
    for (int t = 0; t < 8; t++) x[t] = p[t];
}
template <class Word>
__device__ __forceinline__ void store8(Word* p, const Word (&x)[8]) {
#pragma unroll
    for (int t = 0; t < 8; t++) p[t] = x[t];
}

// Forward transform of row g (block F mod (x^W - w_g)) from row into buf
// (padded, published by the last barrier), twisted to block index 0 as
// described in row_fwd_body.
template <class Mod>
__device__ __forceinline__ void row_fwd_lds(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf,
                                            const typename Mod::Word* row, uint32_t logW, uint64_t g) {
    using Word = typename Mod::Word;
    const uint32_t W = 1u << logW, W8 = W >> 3, nt = nthreads(), maskK = (1u << T.K) - 1;
    const Word* tab = T.f1;   // w_{2x} = f1[2x], x < W/2 <= 2^(B1-1)
    const uint32_t E = __builtin_bitreverse32((uint32_t)(g << logW)) >> (32 - T.K);
    const Word z8 = root_pow(md, T, (W8 * E) & maskK);   // z^(W/8)
    Unit<Mod, 3> top;
    top.load0(tab, 1, 0);
    for (uint32_t u = threadIdx.x; u < W8; u += nt) {
        Word x[8];
#pragma unroll
        for (int t = 0; t < 8; t++) x[t] = row[u + t * W8];
        Word f = root_pow(md, T, (u * E) & maskK);         // z^u, then z^(u + t W/8)
        x[0] = md.mul_tw(x[0], f);
#pragma unroll
        for (int t = 1; t < 8; t++) {
            f = md.tw_mul_tw(f, z8);
            x[t] = md.mul_tw(x[t], f);
        }
        top.template forward<true>(md, x);
#pragma unroll
        for (int t = 0; t < 8; t++) buf[pad(u) + pad_step(t, W8)] = x[t];
    }
    __syncthreads();
    dif_stages(md, T, buf, 0, W, W >> 4, 1, 0, W, 0);
}
// The same, in place at row.
template <class Mod>
__device__ __forceinline__ void row_fwd_fused(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf,
                              typename Mod::Word* row, uint32_t logW, uint64_t g) {
    using Word = typename Mod::Word;
    row_fwd_lds(md, T, buf, row, logW, g);
    staged_copy<8>(1u << logW, [&](uint32_t i) { return buf[pad(i)]; }, [&](uint32_t i, Word v) { row[i] = v; });
}

// Inverse of row_fwd_fused: coefficients of row g from its W values, stored
// at row.  load(i, x) gives the values 8 i .. 8 i + 7 (it may read buf at
// those positions only: the first group writes them back in place).
// PART: only words below lim < W are stored at row; the coefficient at index
// lim goes to *beyond.
template <class Mod, bool PART, class Load>
__device__ __forceinline__ void row_inv_run(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf,
                                            typename Mod::Word* row, uint32_t logW, uint64_t g, uint32_t lim,
                                            typename Mod::Word* beyond, Load load) {
    using Word = typename Mod::Word;
    const uint32_t W = 1u << logW, W8 = W >> 3, nt = nthreads(), maskK = (1u << T.K) - 1;
    const Word* tab = T.i1;
    for (uint32_t i = threadIdx.x; i < W8; i += nt) {
        Word x[8];
        load(i, x);
        Unit<Mod, 3> un;
        un.load0(tab, 1, i);
        un.template inverse<false>(md, x);
#pragma unroll
        for (int t = 0; t < 8; t++) buf[pad(8 * i) + t] = x[t];
    }
    __syncthreads();
    if (logW > 6) dit_stages<Mod, false>(md, T, buf, 0, 0, W, 3, (int)logW - 3, 0);
    // the last group, then z^-i / W on the store (z = w_{gW} = w[K]^E)
    const uint32_t E = __builtin_bitreverse32((uint32_t)(g << logW)) >> (32 - T.K);
    const Word z8 = root_pow_inv(md, T, (W8 * E) & maskK);
    const Word sc = inv_pow2_tw(md, (int)logW);
    Unit<Mod, 3> top;
    top.load0(tab, 1, 0);
    for (uint32_t u = threadIdx.x; u < W8; u += nt) {
        Word x[8];
#pragma unroll
        for (int t = 0; t < 8; t++) x[t] = buf[pad(u) + pad_step(t, W8)];
        top.template inverse<false, true>(md, x);
        Word f = md.tw_mul_tw(sc, root_pow_inv(md, T, (u * E) & maskK));
#pragma unroll
        for (int t = 0; t < 8; t++) {
            if (t) f = md.tw_mul_tw(f, z8);
            const uint32_t idx = u + t * W8;
            const Word v = md.mul_tw(x[t], f);
            if (!PART || idx < lim)
                row[idx] = v;
            else if (idx == lim)
                *beyond = v;
        }
    }
}

// row_inv_run on the W values at row (times Y pointwise first when yr is
// set); PART: only the words below lim exist at row and yr, the others enter
// as 0.
template <class Mod, bool PART = false>
__device__ __forceinline__ void row_inv_fused(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf,
                              typename Mod::Word* row, const typename Mod::Word* yr, uint32_t logW, uint64_t g,
                              uint32_t lim = 0, typename Mod::Word* beyond = nullptr) {
    using Word = typename Mod::Word;
    row_inv_run<Mod, PART>(md, T, buf, row, logW, g, lim, beyond, [&](uint32_t i, Word (&x)[8]) {
        if (PART) {
#pragma unroll
            for (int t = 0; t < 8; t++) x[t] = 8 * i + t < lim ? row[8 * i + t] : Word(0);
        } else {
            load8(row + 8 * i, x);
        }
        if (yr) {
            Word y[8];
            if (PART) {
#pragma unroll
                for (int t = 0; t < 8; t++) y[t] = 8 * i + t < lim ? yr[8 * i + t] : Word(0);
            } else {
                load8(yr + 8 * i, y);
            }
#pragma unroll
            for (int t = 0; t < 8; t++) x[t] = md.mul(x[t], y[t]);
        }
    });
}

// Forward row pass: row j < a is transformed in full (global block index j at
// size W); row a (when b > 0) is built from its b slots and V_c (c >= b) and
// keeps b outputs.
template <class Mod>
__device__ __forceinline__ void row_fwd_body(const Mod& md, const Tables<typename Mod::Word>& T,
                             const TwoPass<typename Mod::Word>& P, uint32_t j) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    const uint32_t W = 1u << P.logW;
    Word* row = P.X + (uint64_t)j * W;
    if (j < P.a && P.logW >= 6) {
        row_fwd_fused(md, T, buf, row, P.logW, P.g0 * P.a + j);
    } else if (j < P.a) {
        // Row j holds F mod (x^W - w_g), g its global block index; its outputs
        // are F(w_{gW + r}) = F(z w_r) with z = w_{gW} (disjoint bits), i.e. the
        // transform at block index 0 of G(x) = F(z x) mod (x^W - 1).  Twisting
        // coefficient i by z^i costs one product each (z^i = w[K]^(i E) with
        // z = w[K]^E), and the block-0 transform takes every twiddle straight
        // from the table and skips the unit twiddles of its first group.
        const uint64_t g = P.g0 * P.a + j;
        const uint32_t nt = nthreads(), maskK = (1u << T.K) - 1;
        const uint32_t E = __builtin_bitreverse32((uint32_t)(g << P.logW)) >> (32 - T.K);
        const Word step = root_pow(md, T, (nt * E) & maskK);
        Word f = root_pow(md, T, (threadIdx.x * E) & maskK);
        staged_copy<8>(W, [&](uint32_t i) { return row[i]; }, [&](uint32_t i, Word v) {
            buf[pad(i)] = md.mul_tw(v, f);
            f = md.tw_mul_tw(f, step);
        });
        __syncthreads();
        dif_forward(md, T, buf, 0, W, 0, W, 0);
        staged_copy<8>(W, [&](uint32_t i) { return buf[pad(i)]; }, [&](uint32_t i, Word v) { row[i] = v; });
    } else {
        for (uint32_t i = threadIdx.x; i < W; i += nthreads()) buf[pad(i)] = i < P.b ? row[i] : P.V[i];
        __syncthreads();
        dif_forward(md, T, buf, 0, W, 0, P.b, P.a);
        for (uint32_t i = threadIdx.x; i < P.b; i += nthreads()) row[i] = buf[pad(i)];
    }
}

// Inverse row pass, item k: k < a inverts full row k (global block index k at
// size W); k >= a inverts piece k - a of the partial last row -- the dyadic
// blocks of its b known outputs that the last-row inverse would otherwise
// invert one after another (they read only known outputs, so they run here,
// in parallel with the rows).  With P.Y set, values are first multiplied
// pointwise by Y (the product step fused into the load).
template <class Mod>
__device__ __forceinline__ void row_inv_body(const Mod& md, const Tables<typename Mod::Word>& T,
                             const TwoPass<typename Mod::Word>& P, uint32_t k) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    const uint32_t W = 1u << P.logW;
    if (P.early == 3 && k == P.a) {
        // the last row with one value missing (b = W - 1): its full inverse
        // with that value 0; tail_inv_body adds the missing value's share
        row_inv_fused<Mod, true>(md, T, buf, P.X + (uint64_t)P.a * W, P.Y ? P.Y + (uint64_t)P.a * W : nullptr, P.logW,
                                 P.a, P.b, P.V + (W - 1));
        return;
    }
    uint64_t start, g;
    uint32_t len;
    if (k < P.a) {
        start = (uint64_t)k * W;
        len = W;
        g = k;
    } else {
        const Piece pc = gitft_piece(W, P.b, P.a, (int)(k - P.a));
        start = (uint64_t)P.a * W + pc.off;
        len = pc.size;
        g = pc.g;
    }
    Word* row = P.X + start;
    if (k < P.a && P.logW >= 6) {
        row_inv_fused(md, T, buf, row, P.Y ? P.Y + start : nullptr, P.logW, g);
        return;
    }
    if (P.Y) {
        const Word* yr = P.Y + start;
        struct Two { Word x, y; };
        staged_copy<4>(len, [&](uint32_t i) { return Two{row[i], yr[i]}; },
                       [&](uint32_t i, Two v) { buf[pad(i)] = md.mul(v.x, v.y); });
    } else {
        staged_copy<8>(len, [&](uint32_t i) { return row[i]; }, [&](uint32_t i, Word v) { buf[pad(i)] = v; });
    }
    __syncthreads();
    const Word sc = inv_pow2_tw(md, __builtin_ctz(len));
    const uint32_t nt = nthreads();
    if (k < P.a) {
        // A full row inverts at block index 0 (the twist of row_fwd_body):
        // the result is len G_i with G_i = c_i z^i, so the store multiplies
        // by z^-i / len, z = w_{gW} = w[K]^E
        full_inverse<Mod, false>(md, T, buf, 0, 0, len, 0);
        const uint32_t maskK = (1u << T.K) - 1;
        const uint32_t E = __builtin_bitreverse32((uint32_t)(g << P.logW)) >> (32 - T.K);
        const Word step = root_pow_inv(md, T, (nt * E) & maskK);
        Word f = md.tw_mul_tw(sc, root_pow_inv(md, T, (threadIdx.x * E) & maskK));
        staged_copy<8>(len, [&](uint32_t i) { return buf[pad(i)]; }, [&](uint32_t i, Word v) {
            row[i] = md.mul_tw(v, f);
            f = md.tw_mul_tw(f, step);
        });
        return;
    }
    // no halvings in the butterflies, one scaling by 2^-lg len on the store
    full_inverse<Mod, false>(md, T, buf, 0, 0, len, g);
    for (uint32_t i = threadIdx.x; i < len; i += nt) row[i] = md.mul_tw(buf[pad(i)], sc);
}

// Row pass of a batched product whose inverse keeps the columns c < b for
// after the last row (early == 0), records with g0 = 0.  Item k < a takes row
// k of both operands' column-pass outputs (P.X and Q.X, W >= 64), transforms
// both in LDS, multiplies them pointwise and inverts the row, storing the
// coefficients over P's row: forward row pass, product and inverse row pass
// in one HBM round trip.  Item a (b > 0) builds the partial last row of both
// operands (b slots and V_c), keeps the product of their b outputs and
// inverts its dyadic pieces, which read only those values (the inverse row
// pass's piece items).
template <class Mod>
__device__ __forceinline__ void row_mul_body(const Mod& md, const Tables<typename Mod::Word>& T,
                                             const TwoPass<typename Mod::Word>& P,
                                             const TwoPass<typename Mod::Word>& Q, uint32_t k) {
    using Word = typename Mod::Word;
    const uint32_t W = 1u << P.logW;
    Word* ba = lds_buf<Word>();
    Word* bb = ba + padded_words(W);
    Word* row = P.X + (uint64_t)k * W;
    const Word* rb = Q.X + (uint64_t)k * W;
    if (k < P.a) {
        row_fwd_lds(md, T, ba, row, P.logW, k);
        row_fwd_lds(md, T, bb, rb, P.logW, k);
        row_inv_run<Mod, false>(md, T, ba, row, P.logW, k, 0, nullptr, [&](uint32_t i, Word (&x)[8]) {
#pragma unroll
            for (int t = 0; t < 8; t++) x[t] = md.mul(ba[pad(8 * i) + t], bb[pad(8 * i) + t]);
        });
        return;
    }
    for (uint32_t i = threadIdx.x; i < W; i += nthreads()) {
        ba[pad(i)] = i < P.b ? row[i] : P.V[i];
        bb[pad(i)] = i < P.b ? rb[i] : Q.V[i];
    }
    __syncthreads();
    dif_forward(md, T, ba, 0, W, 0, P.b, P.a);
    dif_forward(md, T, bb, 0, W, 0, P.b, P.a);
    for (uint32_t i = threadIdx.x; i < P.b; i += nthreads()) ba[pad(i)] = md.mul(ba[pad(i)], bb[pad(i)]);
    __syncthreads();
    // 0 < b < W: the pieces are the dyadic blocks of [0, b), one per set bit
    const int np = __popc(P.b);
    for (int q = 0; q < np; q++) {
        const Piece pc = gitft_piece(W, P.b, P.a, q);
        full_inverse<Mod, false>(md, T, ba, 0, pc.off, pc.size, pc.g);
        const Word sc = inv_pow2_tw(md, __builtin_ctz(pc.size));
        for (uint32_t i = threadIdx.x; i < pc.size; i += nthreads()) row[pc.off + i] = md.mul_tw(ba[pad(pc.off + i)], sc);
    }
}

// The same for R = 2^logR consecutive full rows j0 .. j0 + R - 1 (those below
// a) at once, for rows too short to fill the workgroup: after the twist to
// block index 0 every row takes the same twiddles, so the rows sit in LDS as
// R interleaved columns (word i of row q at i R + q) and go through the
// block-0 forward, the product and the block-0 inverse together, every
// thread busy.
template <class Mod>
__device__ __forceinline__ void row_mul_rows(const Mod& md, const Tables<typename Mod::Word>& T,
                                             const TwoPass<typename Mod::Word>& P,
                                             const TwoPass<typename Mod::Word>& Q, uint32_t j0, int logR) {
    using Word = typename Mod::Word;
    const uint32_t logW = P.logW, W = 1u << logW, W8 = W >> 3, R = 1u << logR;
    const uint32_t nt = nthreads(), maskK = (1u << T.K) - 1;
    const uint32_t cnt = min(R, P.a - j0);
    Word* ba = lds_buf<Word>();
    Word* bb = ba + padded_words(R * W);
    // unit (q, u): words u + t W/8 of row j0 + q, coalesced over u
    for (uint32_t it = threadIdx.x; it < (R << (logW - 3)); it += nt) {
        const uint32_t q = it >> (logW - 3), u = it & (W8 - 1);
        const uint32_t j = j0 + q;
        const uint32_t E = __builtin_bitreverse32(j << logW) >> (32 - T.K);
        const Word z8 = root_pow(md, T, (W8 * E) & maskK);
        Word f = root_pow(md, T, (u * E) & maskK);
        const uint64_t base = (uint64_t)j * W + u;
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const uint32_t d = ((u + t * W8) << logR) + q;
            Word xa = 0, xb = 0;
            if (q < cnt) {
                xa = P.X[base + t * W8];
                xb = Q.X[base + t * W8];
            }
            ba[pad(d)] = md.mul_tw(xa, f);
            bb[pad(d)] = md.mul_tw(xb, f);
            f = md.tw_mul_tw(f, z8);
        }
    }
    __syncthreads();
    dif_forward(md, T, ba, logR, W, 0, W, 0);
    dif_forward(md, T, bb, logR, W, 0, W, 0);
    // the products up to the factor that the store's scaling takes back
    for (uint32_t i = threadIdx.x; i < (R << logW); i += nt) ba[pad(i)] = md.mul_scaled(ba[pad(i)], bb[pad(i)]);
    __syncthreads();
    // block-0 inverse (values times W), then z^-i / W on the store
    full_inverse<Mod, false>(md, T, ba, logR, 0, W, 0);
    const Word sc = md.tw_mul_tw(inv_pow2_tw(md, (int)logW), md.kappa_tw());
    for (uint32_t it = threadIdx.x; it < (R << (logW - 3)); it += nt) {
        const uint32_t q = it >> (logW - 3), u = it & (W8 - 1);
        if (q >= cnt) continue;
        const uint32_t j = j0 + q;
        const uint32_t E = __builtin_bitreverse32(j << logW) >> (32 - T.K);
        const Word z8 = root_pow_inv(md, T, (W8 * E) & maskK);
        Word f = md.tw_mul_tw(sc, root_pow_inv(md, T, (u * E) & maskK));
        const uint64_t base = (uint64_t)j * W + u;
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const uint32_t d = ((u + t * W8) << logR) + q;
            P.X[base + t * W8] = md.mul_tw(ba[pad(d)], f);
            f = md.tw_mul_tw(f, z8);
        }
    }
}

// Rows per row-product item: R W = 8 threads (one radix-8 unit per thread),
// at least one row.
__host__ __device__ inline int row_mul_log_rows(uint32_t logW, uint32_t threads) {
    const int lt = 31 - __builtin_clz(threads) + 3;
    return lt > (int)logW ? lt - (int)logW : 0;
}

// Number of inverse-row items: a rows plus the last row's pieces.
__host__ __device__ inline uint32_t row_inv_items(uint32_t W, uint32_t a, uint32_t b) {
    if (!b) return a;
    Piece pcs[kMaxPieces];
    return a + (uint32_t)gitft_pieces(W, b, a, pcs);
}

// Inverse column pass over one tile for one class of columns: phase 0 handles
// c >= b (length a) and, when b > 0, re-evaluates V_c = P_c(w_a) from the
// restored coefficients; phase 1 handles c < b (length a + 1).  Columns of the
// other class inside the tile are skipped.
template <class Mod, int LOGC, bool HS = false>
__device__ __forceinline__ void col_inv_body(const Mod& md, const Tables<typename Mod::Word>& T0,
                             const TwoPass<typename Mod::Word>& P, int phase, uint32_t tile) {
    using Word = typename Mod::Word;
    constexpr uint32_t C = 1u << LOGC;
    __shared__ Word red[(kColThreads / 64) * C];
    __shared__ Word extra[C], last[C];
    Word* buf = lds_buf<Word>();
    const uint32_t c0 = tile * C;
    const uint64_t W = 1ull << P.logW;
    const uint32_t len = phase ? P.a + 1 : P.a;
    uint32_t Mg = 1;
    while (Mg < len) Mg <<= 1;
    const bool top = P.split && len == P.M + 1;   // one coefficient above the H-point block
    uint32_t Hs = 0, Ss = 0;
    const bool hs = HS && !top && len != Mg && col_split(len, &Hs, &Ss);
    // the LDS twiddle table sits after the block this class uses (H + S words
    // when split, else the Mg- or M-word block), inside the launch's tile
    const uint32_t blk = top ? P.M : Mg;
    const Tables<Word> T = hs ? local_tables<Word, false, true>(T0, buf + padded_words((Hs + Ss) << LOGC),
                                                                P.ldstw ? Hs / 2 : 0u)
                              : local_tables<Word, false, true>(T0, buf + padded_words(blk << LOGC),
                                                                P.ldstw ? blk / 2 : 0u);
    const uint32_t Mb = top ? P.M : Mg;            // block inverted in LDS
    // the columns of the tile in this class; in early modes phase 0 takes
    // every column with its first a values, and the last-row inverse (and, in
    // general, k_col_fix) finishes the columns c < b
    const bool every = P.early && phase == 0;
    auto mine_col = [&](uint32_t col) { return every || (phase ? (col < P.b) : (col >= P.b)); };
    // powers for the evaluations at the end, computed first (few waves, and
    // nothing else is live yet); the next barrier publishes them
    __shared__ Word ypow[C], zp[kColThreads >> LOGC];   // zp: one power per thread of a lane
    if (phase == 0 && P.b == 1 && P.nparts && threadIdx.x < C)   // w_{aW}^c
        ypow[threadIdx.x] = pow_tw(md, tw_fwd(md, T, (uint64_t)P.a << P.logW), c0 + threadIdx.x);
    // the extra values V_c = P_c(w_a) of the restored columns (sums in
    // extra[c]) and, with b = 1, this tile's share sum_{c >= 1} V_c w_{aW}^c
    // of the last-row evaluation (last_inv_body adds the tiles' shares)
    auto put_extra = [&]() {
        for (uint32_t c = threadIdx.x; c < C; c += nthreads())
            if (mine_col(c0 + c)) P.V[c0 + c] = extra[c];
        if (P.nparts) {
            if (threadIdx.x < C) {
                const uint32_t c = c0 + threadIdx.x;
                last[threadIdx.x] = c >= 1 ? md.mul_tw(extra[threadIdx.x], ypow[threadIdx.x]) : Word(0);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                Word sum = 0;
                for (uint32_t c = 0; c < C; c++) sum = md.add(sum, last[c]);
                P.Q[kQStride + tile] = sum;
            }
        }
    };
    if (!top && len == Mg && Mg >= 64) {
        // whole columns: the first radix-8 group (stages 1, 2, 4 on eight
        // consecutive rows) straight from HBM, the last (stages Mg/8, Mg/4,
        // Mg/2) straight to HBM, scaled by 1/Mg; with b > 0 in phase 0 the last
        // group's units also add their shares of V_c = P_c(w_a), w_a = w[K]^Ea
        const bool ev = phase == 0 && P.b;
        const uint32_t M8 = Mg >> 3;
        for (uint32_t it = threadIdx.x; it < M8 * C; it += nthreads()) {
            const uint32_t c = it & (C - 1), i = it >> LOGC;
            const uint32_t col = c0 + c;
            const bool mine = mine_col(col);
            Word x[8];
#pragma unroll
            for (int t = 0; t < 8; t++) x[t] = mine ? P.X[col + (uint64_t)(8 * i + t) * W] : Word(0);
            Unit<Mod, 3> un;
            un.load0(T.li, 0, i);
            un.template inverse<false>(md, x);
#pragma unroll
            for (int t = 0; t < 8; t++) buf[pad(8 * i * C + c) + pad_step(t, C)] = x[t];
        }
        __syncthreads();
        const int L = __builtin_ctz(Mg);
        dit_stages<Mod, false>(md, T, buf, LOGC, 0, Mg, 3, L - 3, 0);
        const Word sc = inv_pow2_tw(md, L);
        const uint32_t maskK = (1u << T.K) - 1;
        const uint32_t Ea = __builtin_bitreverse32(P.a) >> (32 - T.K);
        const Word z8 = ev ? root_pow(md, T, (M8 * Ea) & maskK) : Word(0);
        Unit<Mod, 3> lastg;
        lastg.load0(T.li, 0, 0);
        Word acc = 0;
        for (uint32_t it = threadIdx.x; it < M8 * C; it += nthreads()) {
            const uint32_t c = it & (C - 1), u = it >> LOGC;
            const uint32_t col = c0 + c;
            Word x[8];
#pragma unroll
            for (int t = 0; t < 8; t++) x[t] = buf[pad(u * C + c) + pad_step(t, M8 * C)];
            lastg.template inverse<false, true>(md, x);
            if (mine_col(col)) {
#pragma unroll
                for (int t = 0; t < 8; t++) P.X[col + (uint64_t)(u + t * M8) * W] = md.mul_tw(x[t], sc);
            }
            if (ev) {
                Word e = x[7];
#pragma unroll
                for (int t = 6; t >= 0; t--) e = md.add(md.mul_tw(e, z8), x[t]);
                acc = md.add(acc, md.mul_tw(e, root_pow(md, T, (u * Ea) & maskK)));
            }
        }
        if (ev) {
            reduce_lanes(md, md.mul_tw(acc, sc), LOGC, red, extra);
            put_extra();
        }
        return;
    }
    if constexpr (HS) if (hs) {
        // len = H + R values, R <= S <= H/4.  A = P mod (x^H - 1) from the
        // first H values (a full inverse); P = A + (x^H - 1) Q with
        // deg Q < R, and at the last R points z = w_{H+t} (z^H = -1)
        // Q(z) = (A(z) - P(z)) / 2.  A(w_{H+t}) for t < R: A folded modulo
        // x^S - w_{H/S} (the block of size S at global index H/S holds those
        // points) and transformed there.  Q~(x) = Q(w_H x) takes those values
        // at w_0 .. w_{R-1} (w_{H+t} = w_H w_t), so Q~ is the truncated
        // inverse of length R in a block of S words, and Q_i = Q~_i w_H^-i.
        // The full inverse leaves H A (no halvings), so the block of S words
        // holds 2H Q~ and the coefficients are (2 H A_i - 2H Q_i) / 2H,
        // H A_i / H and 2H Q_i / 2H.
        const uint32_t H = Hs, S = Ss, R = len - Hs;
        Word* fb = buf + pad(H << LOGC);   // the block of S words (H C is a multiple of 32)
        const int lgH = __builtin_ctz(H);
        const uint32_t maskK = (1u << T.K) - 1;
        if (phase == 0 && P.b) eval_scales(md, LOGC, P.a, tw_fwd(md, T, P.a), zp);
        staged_copy<8>(H * C, [&](uint32_t it) {
            const uint32_t c = it & (C - 1), d = it >> LOGC;
            const uint32_t col = c0 + c;
            return mine_col(col) ? P.X[col + (uint64_t)d * W] : Word(0);
        }, [&](uint32_t it, Word v) { buf[pad(it)] = v; });
        __syncthreads();
        full_inverse<Mod, false>(md, T, buf, LOGC, 0, H, 0);
        // fold: F_j = sum_k (H A)_{j + k S} c^k, c = w_{H/S}
        const Word cf = tw_fwd(md, T, H / S);
        for (uint32_t it = threadIdx.x; it < (S << LOGC); it += nthreads()) {
            const uint32_t c = it & (C - 1), j = it >> LOGC;
            Word acc = 0;
            for (uint32_t k = H / S; k-- > 0;) acc = md.add(md.mul_tw(acc, cf), buf[pad((j + k * S) * C + c)]);
            fb[pad(it)] = acc;
        }
        lds_sync();
        dif_forward(md, T, fb, LOGC, S, 0, R, H / S);   // H A(w_{H+t}), t < R
        Word htw = md.one_tw();   // H in twiddle form
        for (int i = 0; i < lgH; i++) htw = md.add(htw, htw);
        for (uint32_t it = threadIdx.x; it < (S << LOGC); it += nthreads()) {
            const uint32_t c = it & (C - 1), t = it >> LOGC;
            const uint32_t col = c0 + c;
            Word v = 0;
            if (t < R) {
                const Word y = mine_col(col) ? P.X[col + (uint64_t)(H + t) * W] : Word(0);
                v = md.sub(fb[pad(it)], md.mul_tw(y, htw));   // 2H Q~(w_t)
            }
            fb[pad(it)] = v;
        }
        lds_sync();
        if (S > 1) gitft(md, T, fb, LOGC, S, R, 0);   // 2H Q~ (coefficients R .. S-1 are 0)
        lds_sync();
        const Word sH = inv_pow2_tw(md, lgH), s2H = inv_pow2_tw(md, lgH + 1);
        const uint32_t EH = __builtin_bitreverse32(H) >> (32 - T.K);   // w_H = w[K]^EH
        for (uint32_t it = threadIdx.x; it < (H << LOGC); it += nthreads()) {
            const uint32_t i = it >> LOGC;
            const Word a2 = buf[pad(it)];
            if (i < R) {
                const Word q = md.mul_tw(fb[pad(it)], root_pow_inv(md, T, (i * EH) & maskK));   // 2H Q_i
                buf[pad(it)] = md.mul_tw(md.sub(md.add(a2, a2), q), s2H);
                fb[pad(it)] = md.mul_tw(q, s2H);
            } else {
                buf[pad(it)] = md.mul_tw(a2, sH);
            }
        }
        __syncthreads();
        staged_copy<8>(len * C, [&](uint32_t it) { return buf[pad(it)]; }, [&](uint32_t it, Word v) {
            const uint32_t c = it & (C - 1), d = it >> LOGC;
            const uint32_t col = c0 + c;
            if (mine_col(col)) P.X[col + (uint64_t)d * W] = v;
        });
        if (phase == 0 && P.b) {
            eval_lanes(md, buf, LOGC, P.a, tw_fwd(md, T, P.a), red, extra, zp);
            put_extra();
        }
        return;
    }
    if (phase == 0 && P.b) eval_scales(md, LOGC, P.a, tw_fwd(md, T, P.a), zp);
    staged_copy<8>(Mb * C, [&](uint32_t it) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        const uint32_t col = c0 + c;
        return (mine_col(col) && d < len) ? P.X[col + (uint64_t)d * W] : Word(0);
    }, [&](uint32_t it, Word v) { buf[pad(it)] = v; });
    if (top) {
        for (uint32_t c = threadIdx.x; c < C; c += nthreads()) {
            const uint32_t col = c0 + c;
            last[c] = mine_col(col) ? P.X[col + (uint64_t)P.M * W] : Word(0);
        }
    }
    __syncthreads();
    if (top) {
        // outputs 0..H-1 are the transform of C0 = lo + hi, output H is
        // C0(w_H) - 2 x_H (see col_fwd_body): invert the H-point block, then
        // x_H = (C0(w_H) - y_H) / 2 and x_0 = C0_0 - x_H
        const uint32_t H = P.M;
        full_inverse(md, T, buf, LOGC, 0, H, 0);
        eval_lanes(md, buf, LOGC, H, tw_fwd(md, T, H), red, extra);
        if (threadIdx.x < C) {
            const Word xh = md.half(md.sub(extra[threadIdx.x], last[threadIdx.x]));
            last[threadIdx.x] = xh;
            buf[pad(threadIdx.x)] = md.sub(buf[pad(threadIdx.x)], xh);
        }
        __syncthreads();
    } else if (len == Mg) {
        // whole columns: no halvings in the butterflies, one scaling by
        // 2^-lg Mg afterwards -- on the store, unless the evaluation below
        // reads the coefficients from LDS
        full_inverse<Mod, false>(md, T, buf, LOGC, 0, Mg, 0);
        const Word sc = inv_pow2_tw(md, __builtin_ctz(Mg));
        if (!(phase == 0 && P.b)) {
            staged_copy<8>(len * C, [&](uint32_t it) { return buf[pad(it)]; }, [&](uint32_t it, Word v) {
                const uint32_t c = it & (C - 1), d = it >> LOGC;
                const uint32_t col = c0 + c;
                if (mine_col(col)) P.X[col + (uint64_t)d * W] = md.mul_tw(v, sc);
            });
            return;
        }
        for (uint32_t it = threadIdx.x; it < Mg * C; it += nthreads()) buf[pad(it)] = md.mul_tw(buf[pad(it)], sc);
        __syncthreads();
    } else if (!(phase == 0 && P.b)) {
        // nothing is evaluated afterwards: the walk's last upward pass writes
        // the column values straight to HBM
        auto out = [&](uint32_t d, uint32_t c, Word v) {
            const uint32_t col = c0 + c;
            if (d < len && mine_col(col)) P.X[col + (uint64_t)d * W] = v;
        };
        gitft(md, T, buf, LOGC, Mg, len, 0, false, &out);
        return;
    } else {
        gitft(md, T, buf, LOGC, Mg, len, 0);
    }
    staged_copy<8>(len * C, [&](uint32_t it) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        return d < Mb ? buf[pad(it)] : last[c];
    }, [&](uint32_t it, Word v) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        const uint32_t col = c0 + c;
        if (mine_col(col)) P.X[col + (uint64_t)d * W] = v;
    });
    if (phase == 0 && P.b) {
        // the extra value V_c = P_c(w_a) of the restored column (early mode:
        // for c < b the same evaluation gives C0(w_H), H = a)
        eval_lanes(md, buf, LOGC, P.a, tw_fwd(md, T, P.a), red, extra, zp);
        put_extra();
    }
}

// Inverse with b = W - 1 and a + 1 = Mg a power of two (early mode 3): column
// W - 1 is the only one with a values, every other column has a + 1 = Mg, and
// the last row lacks only the value at s = W - 1.  With ones missing value set
// to 0, each of the two is a full inverse of block size (done in LDS here for
// the column, by the row pass for the row); the missing value is fixed by a
// known coefficient, and its share is a rank-one term -- the inverse of a unit
// vector at point z of a block of size N is (z^-d / N)_d (Lagrange basis).
//  * column W - 1: coefficient a of P_c is 0, so with B = N x (the full
//    inverse of (y, 0), unscaled) the missing value is t = -B_a w_a^a,
//    P_c(w_a) = t, and the coefficients are (B_d - B_a w_a^(a-d)) / Mg;
//  * last row: its coefficient W - 1 is t, the row pass left r' (inverse of
//    (y, 0)) in X and r'_{W-1} in V[W - 1], and the coefficients are
//    r'_d + (t - r'_{W-1}) z^(W-1-d) with z = w_{aW + W - 1}.
// The columns c < b then invert in full (phase 1).
template <class Mod>
__device__ __forceinline__ void tail_inv_body(const Mod& md, const Tables<typename Mod::Word>& T0,
                              const TwoPass<typename Mod::Word>& P) {
    using Word = typename Mod::Word;
    constexpr uint32_t kRowPer = 8;   // last-row words per thread held from the start
    __shared__ Word tsh;
    Word* buf = lds_buf<Word>();
    const uint32_t Mg = P.a + 1, W = 1u << P.logW, nt = nthreads();
    const uint32_t maskK = (1u << T0.K) - 1;
    const uint64_t c = W - 1;
    Word* row = P.X + (uint64_t)P.a * W;
    // everything that does not depend on the column's inverse is loaded first,
    // so that its memory latency overlaps the column work: the last row's
    // words, r'_{W-1}, and the powers used below
    const uint32_t Ea = __builtin_bitreverse32(P.a) >> (32 - T0.K);                   // w_a = w[K]^Ea
    const uint64_t zi = (uint64_t)P.a * W + (W - 1);
    const uint32_t Ez = __builtin_bitreverse32((uint32_t)zi) >> (32 - T0.K);          // z = w[K]^Ez
    const bool held = W - 1 <= kRowPer * nt;
    Word rv[kRowPer];
    if (held) {
#pragma unroll
        for (uint32_t k = 0; k < kRowPer; k++) {
            const uint32_t d = threadIdx.x + k * nt;
            rv[k] = d + 1 < W ? row[d] : Word(0);
        }
    }
    const Word rlast = P.V[W - 1];
    const Word waa = root_pow(md, T0, (P.a * Ea) & maskK);                               // w_a^a
    Word f = root_pow(md, T0, ((P.a - threadIdx.x) * Ea) & maskK);                      // w_a^(a-d)
    const Word fs = root_pow(md, T0, ((0u - nt) * Ea) & maskK);                         // w_a^-nt
    const Word gz = root_pow(md, T0, ((W - 1 - threadIdx.x) * Ez) & maskK);             // z^(W-1-d)
    const Word gs = root_pow(md, T0, ((0u - nt) * Ez) & maskK);                         // z^-nt
    const Tables<Word> T = local_tables<Word, false, true>(T0, buf + padded_words(Mg), Mg / 2);
    staged_copy<8>(Mg, [&](uint32_t d) { return d < P.a ? P.X[c + (uint64_t)d * W] : Word(0); },
                   [&](uint32_t d, Word v) { buf[pad(d)] = v; });
    __syncthreads();
    full_inverse<Mod, false, true>(md, T, buf, 0, 0, Mg, 0);
    if (threadIdx.x == 0) tsh = buf[pad(P.a)];
    __syncthreads();
    const Word Ba = tsh;
    const Word sc = inv_pow2_tw(md, __builtin_ctz(Mg));
    for (uint32_t d = threadIdx.x; d < P.a; d += nt) {
        P.X[c + (uint64_t)d * W] = md.mul_tw(md.sub(buf[pad(d)], md.mul_tw(Ba, f)), sc);
        f = md.tw_mul_tw(f, fs);
    }
    const Word t = md.sub(Word(0), md.mul_tw(Ba, waa));
    const Word D = md.sub(t, rlast);
    Word g = md.mul_tw(D, gz);                                                          // D z^(W-1-d)
    if (held) {
#pragma unroll
        for (uint32_t k = 0; k < kRowPer; k++) {
            const uint32_t d = threadIdx.x + k * nt;
            if (d + 1 < W) row[d] = md.add(rv[k], g);
            g = md.mul_tw(g, gs);
        }
    } else {
        staged_copy<8>(W - 1, [&](uint32_t d) { return row[d]; }, [&](uint32_t d, Word v) {
            row[d] = md.add(v, g);
            g = md.mul_tw(g, gs);
        });
    }
}

// Inverse of the last row after its pieces were inverted by the row pass: the
// b slots hold the pieces' coefficients and the W - b values V_c are the known
// coefficients of the block; the remaining (elementwise) steps of the
// truncated inverse recover the b column values P_c(w_a), c < b.  With one
// unknown (b = 1) the slot holds the value of the row polynomial at w_{aW},
// so P_0(w_a) is that value minus sum_{c >= 1} V_c w_{aW}^c: one evaluation.
// With P.early the columns c < b were inverted before (split mode, see
// col_inv_body): their top coefficient is x_H = (C0(w_H) - P_c(w_a)) / 2, with
// C0(w_H) left in V[c], and x_0 = C0_0 - x_H.
template <class Mod>
__device__ __forceinline__ void last_inv_body(const Mod& md, const Tables<typename Mod::Word>& T,
                              const TwoPass<typename Mod::Word>& P) {
    using Word = typename Mod::Word;
    __shared__ Word red[kLastThreads / 64], val[1];
    Word* buf = lds_buf<Word>();
    const uint32_t W = 1u << P.logW;
    Word* row = P.X + (uint64_t)P.a * W;
    if (P.b == 1 && P.nparts) {
        // the column tiles left their shares of sum_{c >= 1} V_c w_{aW}^c
        Word s = 0;
        for (uint32_t i = threadIdx.x; i < P.nparts; i += nthreads()) s = md.add(s, P.Q[kQStride + i]);
        for (int o = 1; o < 64; o <<= 1) s = md.add(s, shfl_xor_word(s, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            Word t = 0;
            for (uint32_t w = 0; w < (nthreads() >> 6); w++) t = md.add(t, red[w]);
            buf[pad(0)] = md.sub(row[0], t);
        }
        __syncthreads();
    } else if (P.b == 1) {
        for (uint32_t i = threadIdx.x; i < W; i += nthreads()) buf[pad(i)] = i == 0 ? Word(0) : P.V[i];
        __syncthreads();
        eval_lanes(md, buf, 0, W, tw_fwd(md, T, (uint64_t)P.a * W), red, val);
        if (threadIdx.x == 0) buf[pad(0)] = md.sub(row[0], val[0]);
        __syncthreads();
    } else {
        for (uint32_t i = threadIdx.x; i < W; i += nthreads()) buf[pad(i)] = i < P.b ? row[i] : P.V[i];
        __syncthreads();
        gitft(md, T, buf, 0, W, P.b, P.a, /*skip_full=*/true);
    }
    for (uint32_t i = threadIdx.x; i < P.b; i += nthreads()) {
        if (P.early == 1) {
            const Word xh = md.half(md.sub(P.V[i], buf[pad(i)]));
            row[i] = xh;
            P.X[i] = md.sub(P.X[i], xh);
        } else if (P.early == 2) {
            // the column's top coefficient t_c = (P_c(w_a) - P'_c(w_a)) / Q(w_a)
            row[i] = md.mul(md.sub(buf[pad(i)], P.V[i]), P.Q[2 * kQStride]);
        } else {
            row[i] = buf[pad(i)];
        }
    }
}

// The columns c < b hold a + 1 transform values; the column pass inverted only
// the first a of them, giving the polynomial P'_c of degree < a through those
// values and P'_c(w_a) (in V[c]).  The true column is P_c = P'_c + t_c Q with
// Q = prod_{i < a} (x - w_i) (monic, degree a) and t_c = (P_c(w_a) -
// P'_c(w_a)) / Q(w_a), P_c(w_a) being the last-row value.  The points w_0 ..
// w_{a-1} are the dyadic pieces of [0, a) (one per set bit e of a: the roots of
// x^(2^e) - w_{o_e / 2^e}, o_e = a with bits 0..e cleared), so Q is a product of
// popcount(a) binomials; Q(w_a) = prod_e (w_{a >> e} - w_{o_e / 2^e}) since
// w_s^(2^e) = w_{s >> e}.  One workgroup builds Q in the scratch area beside
// the row pass.
template <class Mod>
__device__ typename Mod::Word pow_normal(const Mod& md, typename Mod::Word x, uint64_t e) {
    typename Mod::Word r = 1;
    while (e) {
        if (e & 1) r = md.mul(r, x);
        x = md.mul(x, x);
        e >>= 1;
    }
    return r;
}

template <class Mod>
__device__ __forceinline__ void col_poly_body(const Mod& md, const Tables<typename Mod::Word>& T,
                              const TwoPass<typename Mod::Word>& P, uint64_t p) {
    using Word = typename Mod::Word;
    const uint32_t a = P.a;
    Word* cur = (__builtin_popcount(a) & 1) ? P.Q + kQStride : P.Q;   // ends in P.Q
    Word* nxt = cur == P.Q ? P.Q + kQStride : P.Q;
    if (threadIdx.x == 0) cur[0] = 1;
    __syncthreads();
    uint32_t deg = 0;
    for (int e = 31; e >= 0; e--) {
        if (!((a >> e) & 1u)) continue;
        const uint32_t s = 1u << e;
        const uint32_t o = (a >> (e + 1)) << (e + 1);
        const Word ce = md.mul_tw(Word(1), tw_fwd(md, T, o >> e));
        for (uint32_t d = threadIdx.x; d <= deg + s; d += nthreads()) {
            Word v = d >= s ? cur[d - s] : Word(0);
            if (d <= deg) v = md.sub(v, md.mul(ce, cur[d]));
            nxt[d] = v;
        }
        __syncthreads();
        Word* t = cur;
        cur = nxt;
        nxt = t;
        deg += s;
    }
    if (threadIdx.x == 0) {
        Word q = 1;
        for (int e = 31; e >= 0; e--) {
            if (!((a >> e) & 1u)) continue;
            const uint32_t o = (a >> (e + 1)) << (e + 1);
            const Word ce = md.mul_tw(Word(1), tw_fwd(md, T, o >> e));
            const Word we = md.mul_tw(Word(1), tw_fwd(md, T, a >> e));
            q = md.mul(q, md.sub(we, ce));
        }
        P.Q[2 * kQStride] = pow_normal(md, q, p - 2);
    }
}

// ---- single transform: one launch per pass, geometry by value
// HS: the column transforms of the launch split at a power of two (col_split);
// a separate instantiation, so that the others keep their register budget
template <class Mod, int LOGC, bool HS = false>
__global__ __launch_bounds__(kColThreads) void k_col_fwd(Mod md, Tables<typename Mod::Word> T,
                                                      TwoPass<typename Mod::Word> P, uint32_t tiles) {
    if (blockIdx.y) {
        P.X += blockIdx.y * P.inst;
        P.src += blockIdx.y * P.inst;
    }
    col_fwd_body<Mod, LOGC, HS>(md, T, P, xcd_remap(blockIdx.x, tiles));
}
template <class Mod>
__global__ __launch_bounds__(kRowThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_row_fwd(Mod md, Tables<typename Mod::Word> T,
                                                      TwoPass<typename Mod::Word> P) {
    using Word = typename Mod::Word;
    if (blockIdx.y) P.X += blockIdx.y * P.inst;
    if (P.b == 1 && P.nparts) {
        // one output in the last row: the sum of the column tiles' shares,
        // added by workgroup 0 before its own row (no workgroup of its own)
        if (blockIdx.x == 0) {
            __shared__ Word red[kRowThreads / 64];
            Word s = 0;
            for (uint32_t i = threadIdx.x; i < P.nparts; i += nthreads()) s = md.add(s, P.Q[kQStride + i]);
            for (int o = 1; o < 64; o <<= 1) s = md.add(s, shfl_xor_word(s, o));
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
            __syncthreads();
            if (threadIdx.x == 0) {
                Word t = 0;
                for (uint32_t w = 0; w < (nthreads() >> 6); w++) t = md.add(t, red[w]);
                P.X[(uint64_t)P.a << P.logW] = t;
            }
        }
        row_fwd_body(md, T, P, blockIdx.x);
        return;
    }
    // the partial last row (item a) goes first: dispatched last, it would run
    // alone after the full rows whenever they fill every slot of the device
    const uint32_t k = P.b ? (blockIdx.x == 0 ? P.a : blockIdx.x - 1) : blockIdx.x;
    row_fwd_body(md, T, P, k);
}
// Forward row pass of two instances of a whole block (b = 0, W >= 64) at X
// and X + inst, multiplied: workgroup j transforms row j of both in LDS and
// stores their pointwise product over the first instance's row (the
// space-restricted product's blocks, no pointwise launch of their own).
template <class Mod>
__global__ __launch_bounds__(kRowThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_row_fwd_mul(
    Mod md, Tables<typename Mod::Word> T, TwoPass<typename Mod::Word> P) {
    using Word = typename Mod::Word;
    const uint32_t W = 1u << P.logW;
    Word* ba = lds_buf<Word>();
    Word* bb = ba + padded_words(W);
    const uint32_t j = blockIdx.x;
    const uint64_t g = P.g0 * P.a + j;
    Word* ra = P.X + (uint64_t)j * W;
    row_fwd_lds(md, T, ba, ra, P.logW, g);
    row_fwd_lds(md, T, bb, ra + P.inst, P.logW, g);
    staged_copy<8>(W, [&](uint32_t i) { return md.mul(ba[pad(i)], bb[pad(i)]); }, [&](uint32_t i, Word v) { ra[i] = v; });
}
// Rows of a product of two transforms of length n = a W + b (W >= 64,
// records with g0 = 0; b = 0, or b = W - 1 with a + 1 a power of two):
// workgroup j takes row j of the first operand's column-pass output at P.X,
// transforms it in LDS, multiplies it by row j of the second operand's
// transform (P.Y) and inverts the row, storing the coefficients over P.X's
// row.  With b = W - 1 workgroup 0 takes the partial last row: its b
// outputs (b slots and V_{W-1}), their product with Y's, and the inverse of
// the full row with the missing value 0, whose coefficient W - 1 goes to
// V[W - 1] (the one-short inverse's row, completed by k_tail_inv).
template <class Mod>
__global__ __launch_bounds__(kRowThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_row_fwd_mul_inv(
    Mod md, Tables<typename Mod::Word> T, TwoPass<typename Mod::Word> P) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    if (P.b && blockIdx.x == 0) {
        const uint32_t W = 1u << P.logW;
        Word* row = P.X + (uint64_t)P.a * W;
        const Word* yr = P.Y + (uint64_t)P.a * W;
        for (uint32_t i = threadIdx.x; i < W; i += nthreads()) buf[pad(i)] = i < P.b ? row[i] : P.V[i];
        __syncthreads();
        dif_forward(md, T, buf, 0, W, 0, P.b, P.a);
        row_inv_run<Mod, true>(md, T, buf, row, P.logW, P.a, P.b, P.V + (W - 1), [&](uint32_t i, Word (&x)[8]) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const uint32_t idx = 8 * i + t;
                x[t] = idx < P.b ? md.mul(buf[pad(8 * i) + t], yr[idx]) : Word(0);
            }
        });
        return;
    }
    const uint32_t j = blockIdx.x - (P.b ? 1u : 0u);
    Word* row = P.X + ((uint64_t)j << P.logW);
    const Word* yr = P.Y + ((uint64_t)j << P.logW);
    row_fwd_lds(md, T, buf, row, P.logW, j);
    row_inv_run<Mod, false>(md, T, buf, row, P.logW, j, 0, nullptr, [&](uint32_t i, Word (&x)[8]) {
        Word y[8];
        load8(yr + 8 * i, y);
#pragma unroll
        for (int t = 0; t < 8; t++) x[t] = md.mul(buf[pad(8 * i) + t], y[t]);
    });
}
// With P.early == 2 workgroup 0 builds Q (col_poly_body; dispatched first, it
// runs beside the rows).  The last row's pieces come next, the full rows last.
template <class Mod>
__global__ __launch_bounds__(kRowThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_row_inv(Mod md, Tables<typename Mod::Word> T,
                                                      TwoPass<typename Mod::Word> P, uint64_t p) {
    const bool q = P.early == 2;
    if (q && blockIdx.x == 0) {
        col_poly_body(md, T, P, p);
        return;
    }
    if (P.early == 3) {   // the last row (item a) first, then rows 0 .. a-1
        row_inv_body(md, T, P, blockIdx.x == 0 ? P.a : blockIdx.x - 1);
        return;
    }
    // then the last row's pieces (items a ..), then the full rows
    const uint32_t r = blockIdx.x - (q ? 1u : 0u);
    const uint32_t np = __builtin_popcount(P.b);   // the pieces of [0, b): one per set bit
    row_inv_body(md, T, P, r < np ? P.a + r : r - np);
}
template <class Mod, int LOGC, bool HS = false>
__global__ __launch_bounds__(kColThreads) void k_col_inv(Mod md, Tables<typename Mod::Word> T,
                                                      TwoPass<typename Mod::Word> P, int phase, uint32_t tile0,
                                                      uint32_t tiles) {
    col_inv_body<Mod, LOGC, HS>(md, T, P, phase, tile0 + xcd_remap(blockIdx.x, tiles));
}
template <class Mod>
__global__ __launch_bounds__(kLastThreads) void k_last_inv(Mod md, Tables<typename Mod::Word> T,
                                                           TwoPass<typename Mod::Word> P) {
    last_inv_body(md, T, P);
}
template <class Mod>
__global__ __launch_bounds__(kLastThreads) void k_tail_inv(Mod md, Tables<typename Mod::Word> T,
                                                           TwoPass<typename Mod::Word> P) {
    tail_inv_body(md, T, P);
}
// The folding step of the space-restricted product (section 5, Algorithm 3):
// out[j] = sum_t c^t A[j + t L] for j < L with c = w_g (in twiddle form), the
// coefficients of A mod (x^L - w_g), i.e. of the block at global index g and
// size L.  Thread (k, j) runs Horner over the k-th chunk of T consecutive t
// and scales by c^(k T); with K chunks the K partial vectors go to part
// (k_fold_sum adds them), with K = 1 straight to out.  blockIdx.y selects the
// operand (both operands of a block in one launch).
template <class Word>
struct FoldArgs {
    const Word* A[2];
    uint64_t m[2];
    Word* out[2];   // K == 1: the block; else the partial area of the operand
};
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_fold(Mod md, Tables<typename Mod::Word> T,
                                                  FoldArgs<typename Mod::Word> F, uint32_t logL, uint32_t K,
                                                  uint64_t chunk, uint64_t g) {
    using Word = typename Mod::Word;
    const uint64_t idx = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= ((uint64_t)K << logL)) return;
    const Word* A = F.A[blockIdx.y];
    const uint64_t m = F.m[blockIdx.y];
    const uint64_t L = 1ull << logL;
    const uint64_t j = idx & (L - 1), k = idx >> logL;
    const uint64_t terms = j < m ? (m - 1 - j) / L + 1 : 0;   // t with j + t L < m
    const uint64_t t0 = k * chunk;
    const uint64_t t1 = t0 + chunk < terms ? t0 + chunk : terms;
    const Word c = tw_fwd(md, T, g);
    Word acc = 0;
    // Horner from the top term down, eight terms' loads in flight at a time
    uint64_t t = t1;
    for (; t >= t0 + 8; t -= 8) {
        Word v[8];
#pragma unroll
        for (int k8 = 0; k8 < 8; k8++) v[k8] = A[j + (t - 1 - k8) * L];
#pragma unroll
        for (int k8 = 0; k8 < 8; k8++) acc = md.add(md.mul_tw(acc, c), v[k8]);
    }
    for (; t > t0; t--) acc = md.add(md.mul_tw(acc, c), A[j + (t - 1) * L]);
    if (t0 > 0 && t0 < t1) {
        // c^t0 by square and multiply over the bits of t0
        Word z = c, e = md.one_tw();
        for (uint64_t b = t0; b; b >>= 1) {
            if (b & 1) e = md.tw_mul_tw(e, z);
            z = md.tw_mul_tw(z, z);
        }
        acc = md.mul_tw(acc, e);
    }
    F.out[blockIdx.y][idx] = acc;
}

// out[b L + j] = sum_{k in span b} part[k L + j], span b = [b S, (b+1) S) with
// S = kFoldSpan: workgroup (j, b, operand), eight independent loads per
// thread, then lane exchanges and the workgroup.  One span per j gives the
// final sums.
constexpr uint32_t kFoldSpan = 8 * kThreads;
template <class Word>
struct SumArgs {
    const Word* part[2];
    Word* out[2];
};
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_fold_sum(Mod md, SumArgs<typename Mod::Word> S, uint32_t logL,
                                                      uint32_t K) {
    using Word = typename Mod::Word;
    __shared__ Word red[kThreads / 64];
    const Word* part = S.part[blockIdx.z];
    const uint64_t j = blockIdx.x;
    const uint32_t k0 = blockIdx.y * kFoldSpan;
    Word v[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint32_t k = k0 + threadIdx.x + i * kThreads;
        v[i] = k < K ? part[((uint64_t)k << logL) + j] : Word(0);
    }
    Word s = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) s = md.add(s, v[i]);
    for (int o = 1; o < 64; o <<= 1) s = md.add(s, shfl_xor_word(s, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        Word t = 0;
        for (int w = 0; w < kThreads / 64; w++) t = md.add(t, red[w]);
        S.out[blockIdx.z][((uint64_t)blockIdx.y << logL) + j] = t;
    }
}

// out[j] = sum_{k < K} part[k L + j] for few partials (K <= kFoldFewK): one
// thread per word j and operand (grid y), the K loads of a thread independent.
constexpr uint32_t kFoldFewK = 64;
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_fold_sum_few(Mod md, SumArgs<typename Mod::Word> S, uint32_t logL,
                                                          uint32_t K) {
    using Word = typename Mod::Word;
    const uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >> logL) return;
    const Word* part = S.part[blockIdx.y];
    Word s = 0;
#pragma unroll 8
    for (uint32_t k = 0; k < K; k++) s = md.add(s, part[((uint64_t)k << logL) + j]);
    S.out[blockIdx.y][j] = s;
}

// The last blocks of the space-restricted product (section 5, Algorithm 3),
// those of fewer than S = 2^logS points, all lie in at most two aligned nodes
// of size S of the transform tree, [g S, (g + 1) S) for g = G0 and G0 + 1.
// For each node (workgroup x): A mod (x^S - w_g) at N + x S and B mod
// (x^S - w_g) at N + (2 + x) S (folded beforehand) are transformed at block
// index g, and the products A(w_s) B(w_s) of the positions s < r of the node
// are written to X[s].  The same values as the blocks one at a time, without a
// pass over A and B per block.
template <class Mod>
__global__ __launch_bounds__(kSmallThreads) void k_restr_tail(Mod md, Tables<typename Mod::Word> T,
                                                             const typename Mod::Word* N, uint32_t logS, uint64_t G0,
                                                             uint64_t r, typename Mod::Word* X) {
    using Word = typename Mod::Word;
    const uint32_t S = 1u << logS;
    const uint64_t g = G0 + blockIdx.x;
    const uint64_t base = g << logS;
    const uint32_t need = r - base < S ? (uint32_t)(r - base) : S;
    Word* ba = lds_buf<Word>();
    Word* bb = ba + padded_words(S);
    const Word* na = N + ((uint64_t)blockIdx.x << logS);
    const Word* nb = N + ((uint64_t)(2 + blockIdx.x) << logS);
    for (uint32_t i = threadIdx.x; i < S; i += nthreads()) {
        ba[pad(i)] = na[i];
        bb[pad(i)] = nb[i];
    }
    __syncthreads();
    dif_forward(md, T, ba, 0, S, 0, need, g);
    dif_forward(md, T, bb, 0, S, 0, need, g);
    for (uint32_t i = threadIdx.x; i < need; i += nthreads()) X[base + i] = md.mul(ba[pad(i)], bb[pad(i)]);
}

// The space-restricted product's last positions q <= s < r from at most two
// nodes of size S = 2^logS, [q + j S, q + (j + 1) S): node j holds A's values
// at N + 2 j S and B's at N + (2 j + 1) S (transformed beforehand), and
// X[s] = A(w_s) B(w_s).
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_restr_nodes_mul(Mod md, const typename Mod::Word* N, uint32_t logS,
                                                             uint64_t q, uint64_t r, typename Mod::Word* X) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= r - q) return;
    const uint64_t j = i >> logS, k = i & ((1ull << logS) - 1);
    X[q + i] = md.mul(N[((2 * j) << logS) + k], N[((2 * j + 1) << logS) + k]);
}

// X[i] = i mod p (canonical residues for timing runs).
template <class Word>
__global__ __launch_bounds__(kThreads) void k_fill_index(Word* X, uint64_t n, uint64_t p) {
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        X[i] = (Word)(i % p);
}

// X[c + d W] += t_c Q_d for c < b, d < a (t_c in the last-row slot of column c);
// grid: x over columns (kThreads each), y over groups of kFixRows rows, whose
// loads a thread issues together.
constexpr uint32_t kFixRows = 8;
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_col_fix(Mod md, TwoPass<typename Mod::Word> P) {
    using Word = typename Mod::Word;
    const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= P.b) return;
    const uint64_t W = 1ull << P.logW;
    const Word t = P.X[(uint64_t)P.a * W + c];
    const uint32_t d0 = blockIdx.y * kFixRows;
    Word x[kFixRows];
#pragma unroll
    for (uint32_t k = 0; k < kFixRows; k++)
        if (d0 + k < P.a) x[k] = P.X[c + (uint64_t)(d0 + k) * W];
#pragma unroll
    for (uint32_t k = 0; k < kFixRows; k++)
        if (d0 + k < P.a) P.X[c + (uint64_t)(d0 + k) * W] = md.add(x[k], md.mul(t, P.Q[d0 + k]));
}

// ---- batches: every workgroup takes one (record, index) item of a work list
// for one pass; records are the geometries of the batch's transforms.
struct Item {
    uint32_t rec;
    uint32_t idx;
};
template <class Mod, int LOGC>
__global__ __launch_bounds__(kColThreads) void k_col_fwd_list(Mod md, Tables<typename Mod::Word> T,
                                                           const TwoPass<typename Mod::Word>* recs,
                                                           const Item* items, uint32_t spread) {
    // spread: neighbouring tiles on one XCD (its L2 holds the shared lines)
    const Item it = items[spread ? xcd_remap_list(blockIdx.x, gridDim.x) : blockIdx.x];
    col_fwd_body<Mod, LOGC>(md, T, recs[it.rec], it.idx);
}
template <class Mod>
__global__ __launch_bounds__(kRowThreads) void k_row_fwd_list(Mod md, Tables<typename Mod::Word> T,
                                                           const TwoPass<typename Mod::Word>* recs,
                                                           const Item* items) {
    const Item it = items[blockIdx.x];
    row_fwd_body(md, T, recs[it.rec], it.idx);
}
template <class Mod>
__global__ __launch_bounds__(kRowThreads) void k_row_inv_list(Mod md, Tables<typename Mod::Word> T,
                                                           const TwoPass<typename Mod::Word>* recs,
                                                           const Item* items) {
    const Item it = items[blockIdx.x];
    row_inv_body(md, T, recs[it.rec], it.idx);
}
// Item (rec, k) of a batched product: records rec (first operand, result)
// and rec + 1 (second operand); k < a: the rows from k (row_mul_rows, or
// row_mul_body for one row per item), k = a: the partial last row.
template <class Mod>
__global__ __launch_bounds__(kRowThreads) void k_row_mul_list(Mod md, Tables<typename Mod::Word> T,
                                                           const TwoPass<typename Mod::Word>* recs,
                                                           const Item* items) {
    const Item it = items[blockIdx.x];
    const TwoPass<typename Mod::Word>& P = recs[it.rec];
    const int logR = row_mul_log_rows(P.logW, nthreads());
    if (it.idx < P.a && logR > 0)
        row_mul_rows(md, T, P, recs[it.rec + 1], it.idx, logR);
    else
        row_mul_body(md, T, P, recs[it.rec + 1], it.idx);
}
template <class Mod, int LOGC>
__global__ __launch_bounds__(kColThreads) void k_col_inv_list(Mod md, Tables<typename Mod::Word> T,
                                                           const TwoPass<typename Mod::Word>* recs,
                                                           const Item* items, int phase, uint32_t spread) {
    const Item it = items[spread ? xcd_remap_list(blockIdx.x, gridDim.x) : blockIdx.x];
    col_inv_body<Mod, LOGC>(md, T, recs[it.rec], phase, it.idx);
}
template <class Mod>
__global__ __launch_bounds__(kLastThreads) void k_last_inv_list(Mod md, Tables<typename Mod::Word> T,
                                                            const TwoPass<typename Mod::Word>* recs,
                                                            const Item* items) {
    last_inv_body(md, T, recs[items[blockIdx.x].rec]);
}

// ---- batches of single-workgroup instances: a persistent kernel.  Each
// workgroup repeatedly takes the next instance from an atomic counter (the
// list is sorted by decreasing size, so the longest instances start first) and
// runs it entirely in LDS: a product when B is set, else a forward transform.
template <class Word>
struct SmallJob {
    const Word* A;
    const Word* B;
    Word* X;
    uint32_t m, nb, M;
};
template <class Mod, int NT = kThreads>
__global__ __launch_bounds__(NT) void k_small_list(Mod md, Tables<typename Mod::Word> T,
                                                         const SmallJob<typename Mod::Word>* jobs, uint32_t count,
                                                         uint32_t* counter) {
    __shared__ uint32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t k = next;
        __syncthreads();
        if (k >= count) break;
        const SmallJob<typename Mod::Word> J = jobs[k];
        if (J.B)
            small_mul_body(md, T, J.A, J.m, J.B, J.nb, J.X, J.M);
        else
            small_forward_body(md, T, J.X, J.m, J.M);
        __syncthreads();
    }
}

// Reset of the work counters (two words), as a kernel so that a captured
// graph replays it.
__global__ void k_reset_counter(uint32_t* counter) {
    if (threadIdx.x < 2 && blockIdx.x == 0) counter[threadIdx.x] = 0u;
}

// ---------------------------------------------------------- elementwise
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_pointwise(Mod md, typename Mod::Word* X, const typename Mod::Word* Y,
                                                        uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)nthreads() + threadIdx.x; i < n; i += (uint64_t)gridDim.x * nthreads())
        X[i] = md.mul(X[i], Y[i]);
}

// dst[i] = i < n_src ? src[i] : 0 for i < n_dst
template <class Word>
__global__ __launch_bounds__(kThreads) void k_copy_pad(Word* dst, uint64_t n_dst, const Word* src, uint64_t n_src) {
    for (uint64_t i = blockIdx.x * (uint64_t)nthreads() + threadIdx.x; i < n_dst;
         i += (uint64_t)gridDim.x * nthreads())
        dst[i] = i < n_src ? src[i] : Word(0);
}

// Signed integers to residues: dst[i] = src[i] mod p in [0, p).
template <class Word>
__global__ __launch_bounds__(kThreads) void k_from_signed(Word* dst, const int64_t* src, uint64_t n, uint64_t p) {
    for (uint64_t i = blockIdx.x * (uint64_t)nthreads() + threadIdx.x; i < n; i += (uint64_t)gridDim.x * nthreads()) {
        const int64_t v = src[i];
        uint64_t r;
        if (v >= 0)
            r = (uint64_t)v % p;
        else
            r = (p - ((uint64_t)(-(v + 1)) % p) - 1) % p;   // -(v+1) avoids overflow at INT64_MIN
        dst[i] = (Word)r;
    }
}

// The same for primes below 2^31 without 64-bit division: |v| = hi 2^32 + lo,
// hi 2^32 mod p = mont(hi, 2^64 mod p), lo mod p by a 32-bit Barrett step
// (barrett32, b = floor(2^32 / p)), then the sign.
// x mod p for x < 2^32, p < 2^31, b = floor(2^32 / p): the quotient estimate
// floor(x b / 2^32) is at most one short, so one conditional subtraction.
__device__ __forceinline__ uint32_t barrett32(uint32_t x, uint32_t p, uint32_t b) {
    const uint32_t r = x - __umulhi(x, b) * p;
    return r >= p ? r - p : r;
}
__global__ __launch_bounds__(kThreads) void k_from_signed32(ModU32 md, uint32_t b, uint32_t* dst, const int64_t* src,
                                                           uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)nthreads() + threadIdx.x; i < n; i += (uint64_t)gridDim.x * nthreads()) {
        const int64_t v = src[i];
        const uint64_t u = v >= 0 ? (uint64_t)v : 0u - (uint64_t)v;   // |v| (2^63 for INT64_MIN)
        const uint32_t r = md.add(md.mont((uint32_t)(u >> 32), md.r2), barrett32((uint32_t)u, md.p, b));
        dst[i] = v >= 0 ? r : md.sub(0u, r);
    }
}

// Chinese remaindering of three residue vectors (Garner's mixed-radix form):
// x = r1 + p1 t2 + p1 p2 t3 with t2 = (r2 - r1) p1^-1 mod p2 and
// t3 = (r3 - (r1 + p1 t2)) (p1 p2)^-1 mod p3, so 0 <= x < M = p1 p2 p3; the
// output is the signed representative in [-M/2, M/2), little-endian 128-bit.
struct Crt3 {
    uint64_t p1, p2, p3;
    ModU32 m2, m3;              // 32-bit Montgomery arithmetic modulo p2 and p3
    uint32_t inv12_m;           // p1^-1 mod p2, Montgomery form (x 2^32 mod p2)
    uint32_t inv123_m;          // (p1 p2)^-1 mod p3, Montgomery form
    uint32_t b2, b3;            // floor(2^32 / p2), floor(2^32 / p3)
    uint64_t p1p2;              // p1 p2 < 2^62
    unsigned __int128 M, half_M;
};
// Garner's mixed-radix reconstruction, one coefficient per thread:
// x = a1 + p1 t2 + p1 p2 t3 with t2 = (a2 - a1) / p1 mod p2 and
// t3 = (a3 - (a1 + p1 t2)) / (p1 p2) mod p3, then the signed representative in
// (-M/2, M/2].  Every reduction is a 32-bit Barrett step or a Montgomery
// product (no 64- or 128-bit division).
__global__ __launch_bounds__(kThreads) void k_crt3(Crt3 c, const uint32_t* r1, const uint32_t* r2, const uint32_t* r3,
                                                  uint64_t* out, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)nthreads() + threadIdx.x; i < n; i += (uint64_t)gridDim.x * nthreads()) {
        const uint32_t a1 = r1[i], a2 = r2[i], a3 = r3[i];
        const uint32_t d2 = c.m2.sub(a2, barrett32(a1, (uint32_t)c.p2, c.b2));
        const uint32_t t2 = c.m2.mont(d2, c.inv12_m);
        const uint64_t x12 = a1 + c.p1 * t2;                                  // < p1 p2 < 2^62
        // x12 mod p3 = (hi 2^32 + lo) mod p3, hi < 2^30: mont(hi, 2^64 mod p3) = hi 2^32 mod p3
        const uint32_t hi = (uint32_t)(x12 >> 32), lo = (uint32_t)x12;
        const uint32_t x12m = c.m3.add(c.m3.mont(hi, c.m3.r2), barrett32(lo, (uint32_t)c.p3, c.b3));
        const uint32_t t3 = c.m3.mont(c.m3.sub(a3, x12m), c.inv123_m);
        unsigned __int128 x = (unsigned __int128)x12 + (unsigned __int128)c.p1p2 * t3;
        if (x >= c.half_M) x -= c.M;                                          // two's complement wrap to signed
        out[2 * i] = (uint64_t)x;
        out[2 * i + 1] = (uint64_t)(x >> 64);
    }
}

// ---- the paper's Algorithms 1 and 2, one wavefront per instance ---------
// Sections 3 and 4 compute the TFT and ITFT in place on the even/odd tree with
// a constant number of scalars.  A node (q, r) is the strided subarray
// S_i = X_{q + i 2^r} of length ceil((n - q) / 2^r); its even child is
// (q, r + 1), its odd child (q + 2^r, r + 1), and its parent (q with bit r - 1
// cleared, r - 1) -- the node is the odd child exactly when that bit is set --
// so the walk keeps only the current node and how it got there (just entered,
// back from the even child, back from the odd child).  Forward at a node of
// length m > 1: enter the even child; back from it, if m is odd add
// w_{m-1} H(w_{(m-1)/2}) into S_{m-1} (H: the odd child's raw coefficients as
// a polynomial) and enter the odd child; back from the odd child, apply the
// butterflies of eq. (1) and return.  Inverse: on entering, the inverse
// butterflies, then the odd child; back from it, remove the correction and
// enter the even child; back from the even child, return.  Every lane of a
// wavefront holds the same state; the 64 lanes share each node's butterflies
// and the correction's sum; the instance sits in the wavefront's LDS slice
// (at most kWalkMax words), loaded and stored once.
constexpr uint32_t kWalkMax = 1024;
constexpr uint32_t kWalkWaves = 4;   // wavefronts (instances) per workgroup

__device__ __forceinline__ uint32_t walk_len(uint32_t n, uint32_t q, uint32_t r) { return (n - q + (1u << r) - 1) >> r; }
// orders the wavefront's LDS accesses across lanes (one wavefront, no barrier)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// w_{m-1} H(w_{(m-1)/2}), H(y) = sum_{i <= (m-3)/2} S_{2i+1} y^i over the lanes (every lane gets it)
template <class Mod>
__device__ __forceinline__ typename Mod::Word walk_correction(const Mod& md, const Tables<typename Mod::Word>& T,
                                                             const typename Mod::Word* x, uint32_t q, uint32_t r,
                                                             uint32_t m, uint32_t lane) {
    using Word = typename Mod::Word;
    const uint32_t maskK = (1u << T.K) - 1;
    const uint32_t e = __builtin_bitreverse32((m - 1) >> 1) >> (32 - T.K);   // w_{(m-1)/2} = w[K]^e
    Word acc = 0;
    for (uint32_t i = lane; 2 * i + 1 < m - 1; i += 64)
        acc = md.add(acc, md.mul_tw(x[q + ((2 * i + 1) << r)], root_pow(md, T, (i * e) & maskK)));
    for (int o = 1; o < 64; o <<= 1) acc = md.add(acc, shfl_xor_word(acc, o));
    return md.mul_tw(acc, tw_fwd(md, T, m - 1));
}

template <class Mod, bool INV>
__global__ __launch_bounds__(64 * kWalkWaves) void k_walk(Mod md, Tables<typename Mod::Word> T,
                                                         typename Mod::Word* const* X, const uint64_t* lens,
                                                         uint32_t count) {
    using Word = typename Mod::Word;
    __shared__ Word slice[kWalkWaves][kWalkMax];
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t inst = blockIdx.x * kWalkWaves + wv;
    if (inst >= count) return;   // whole wavefront
    const uint32_t n = (uint32_t)lens[inst];
    Word* g = X[inst];
    Word* x = slice[wv];
    for (uint32_t i = lane; i < n; i += 64) x[i] = g[i];
    wave_sync();
    enum { kEnter, kFromEven, kFromOdd };
    uint32_t q = 0, r = 0;
    int how = kEnter;
    for (;;) {
        const uint32_t m = walk_len(n, q, r), st = 1u << r;
        if (how == kEnter && m > 1) {
            if (INV) {
                for (uint32_t j = lane; j < (m >> 1); j += 64) {
                    const Word th = tw_inv(md, T, 2 * (uint64_t)j);
                    Word& a = x[q + ((2 * j) << r)];
                    Word& b = x[q + ((2 * j + 1) << r)];
                    const Word u = a, w = b;
                    a = md.half(md.add(u, w));
                    b = md.mul_tw(md.half(md.sub(u, w)), th);
                }
                wave_sync();
                q += st;   // the odd child next
            }
            r++;           // forward: the even child next
            continue;
        }
        if ((!INV && how == kFromEven) || (INV && how == kFromOdd)) {
            if (m & 1u) {
                const Word v = walk_correction(md, T, x, q, r, m, lane);
                if (lane == 0) {
                    Word& last = x[q + ((m - 1) << r)];
                    last = INV ? md.sub(last, v) : md.add(last, v);
                }
                wave_sync();
            }
            if (!INV) q += st;   // forward: the odd child next; inverse: the even child
            r++;
            how = kEnter;
            continue;
        }
        if (!INV && how == kFromOdd) {
            for (uint32_t j = lane; j < (m >> 1); j += 64) {
                const Word th = tw_fwd(md, T, 2 * (uint64_t)j);
                Word& a = x[q + ((2 * j) << r)];
                Word& b = x[q + ((2 * j + 1) << r)];
                const Word t = md.mul_tw(b, th), u = a;
                a = md.add(u, t);
                b = md.sub(u, t);
            }
            wave_sync();
        }
        // the node is finished: back to its parent
        if (r == 0) break;
        const uint32_t bit = 1u << (r - 1);
        how = (q & bit) ? kFromOdd : kFromEven;
        q &= ~bit;
        r--;
    }
    for (uint32_t i = lane; i < n; i += 64) g[i] = x[i];
}

}  // namespace tft
