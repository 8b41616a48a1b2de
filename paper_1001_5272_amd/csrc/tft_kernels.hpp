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

constexpr int kThreads = 256;

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

// ------------------------------------------------------ single workgroup
template <class Mod>
__device__ void small_forward_body(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* X,
                                   uint32_t n, uint32_t M) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) buf[i] = i < n ? X[i] : Word(0);
    __syncthreads();
    dif_forward(md, T, buf, 0, M, 0, n, 0);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) X[i] = buf[i];
}

template <class Mod>
__device__ void small_inverse_body(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* X,
                                   uint32_t n, uint32_t M) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) buf[i] = i < n ? X[i] : Word(0);
    __syncthreads();
    gitft(md, T, buf, 0, M, n, 0);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) X[i] = buf[i];
}

// Whole product in one workgroup: both operands zero-extended to M words of
// LDS, forward transforms truncated to r outputs, pointwise product, inverse.
template <class Mod>
__device__ void small_mul_body(const Mod& md, const Tables<typename Mod::Word>& T, const typename Mod::Word* A,
                               uint32_t m, const typename Mod::Word* B, uint32_t nb, typename Mod::Word* X,
                               uint32_t M) {
    using Word = typename Mod::Word;
    Word* ba = lds_buf<Word>();
    Word* bb = ba + M;
    const uint32_t r = m + nb - 1;
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
        ba[i] = i < m ? A[i] : Word(0);
        bb[i] = i < nb ? B[i] : Word(0);
    }
    __syncthreads();
    dif_forward(md, T, ba, 0, M, 0, r, 0);
    dif_forward(md, T, bb, 0, M, 0, r, 0);
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) ba[i] = i < r ? md.mul(ba[i], bb[i]) : Word(0);
    __syncthreads();
    gitft(md, T, ba, 0, M, r, 0);
    for (uint32_t i = threadIdx.x; i < r; i += blockDim.x) X[i] = ba[i];
}

template <class Mod>
__global__ __launch_bounds__(kThreads) void k_small_fwd(Mod md, Tables<typename Mod::Word> T,
                                                        typename Mod::Word* X, uint32_t n, uint32_t M) {
    small_forward_body(md, T, X, n, M);
}

template <class Mod>
__global__ __launch_bounds__(kThreads) void k_small_inv(Mod md, Tables<typename Mod::Word> T,
                                                        typename Mod::Word* X, uint32_t n, uint32_t M) {
    small_inverse_body(md, T, X, n, M);
}

template <class Mod>
__global__ __launch_bounds__(kThreads) void k_small_mul(Mod md, Tables<typename Mod::Word> T,
                                                        const typename Mod::Word* A, uint32_t m,
                                                        const typename Mod::Word* B, uint32_t nb,
                                                        typename Mod::Word* X, uint32_t M) {
    small_mul_body(md, T, A, m, B, nb, X, M);
}

// ------------------------------------------------------------ column pass
// Forward column pass.  Reads columns from src (n_src words; src may equal dst,
// or be a shorter read-only operand that is implicitly zero-extended to n),
// evaluates each column polynomial at w_0..w_{Lout-1} (Lout = a + (b > 0)) in
// an LDS block of M = 2^ceil(lg Lout) words per column, writes outputs that
// have a slot in dst and the extra value P_c(w_a) of columns c >= b to V[c].
template <class Mod, int LOGC>
__global__ __launch_bounds__(kThreads) void k_col_fwd(Mod md, Tables<typename Mod::Word> T,
                                                      const typename Mod::Word* src, uint64_t n_src,
                                                      typename Mod::Word* dst, uint64_t n, uint32_t logW,
                                                      uint32_t a, uint32_t b, uint32_t Lout, uint32_t M,
                                                      typename Mod::Word* V, uint32_t tiles) {
    using Word = typename Mod::Word;
    constexpr uint32_t C = 1u << LOGC;
    Word* buf = lds_buf<Word>();
    const uint32_t c0 = xcd_remap(blockIdx.x, tiles) * C;
    const uint64_t W = 1ull << logW;
    for (uint32_t it = threadIdx.x; it < M * C; it += blockDim.x) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        const uint64_t idx = (c0 + c) + (uint64_t)d * W;
        buf[it] = (d < Lout && idx < n_src) ? src[idx] : Word(0);
    }
    __syncthreads();
    dif_forward(md, T, buf, LOGC, M, 0, Lout, 0);
    for (uint32_t it = threadIdx.x; it < Lout * C; it += blockDim.x) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        const uint64_t idx = (c0 + c) + (uint64_t)d * W;
        if (idx < n)
            dst[idx] = buf[it];
        else if (b && d == a)
            V[c0 + c] = buf[it];
    }
}

// Inverse column pass for one class of columns: phase 0 handles c >= b (length
// a) and, when b > 0, re-evaluates V_c = P_c(w_a) from the restored
// coefficients; phase 1 handles c < b (length a + 1).  Tiles [tile0, tile0 +
// tiles) are covered; columns of the other class inside a tile are skipped.
template <class Mod, int LOGC>
__global__ __launch_bounds__(kThreads) void k_col_inv(Mod md, Tables<typename Mod::Word> T, typename Mod::Word* X,
                                                      uint32_t logW, uint32_t a, uint32_t b, uint32_t M,
                                                      typename Mod::Word* V, int phase, uint32_t tile0,
                                                      uint32_t tiles) {
    using Word = typename Mod::Word;
    constexpr uint32_t C = 1u << LOGC;
    Word* buf = lds_buf<Word>();
    const uint32_t c0 = (tile0 + xcd_remap(blockIdx.x, tiles)) * C;
    const uint64_t W = 1ull << logW;
    const uint32_t len = phase ? a + 1 : a;
    uint32_t Mg = 1;
    while (Mg < len) Mg <<= 1;
    for (uint32_t it = threadIdx.x; it < M * C; it += blockDim.x) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        const uint32_t col = c0 + c;
        const bool mine = phase ? (col < b) : (col >= b);
        buf[it] = (mine && d < len) ? X[col + (uint64_t)d * W] : Word(0);
    }
    __syncthreads();
    gitft(md, T, buf, LOGC, Mg, len, 0);
    for (uint32_t it = threadIdx.x; it < len * C; it += blockDim.x) {
        const uint32_t c = it & (C - 1), d = it >> LOGC;
        const uint32_t col = c0 + c;
        const bool mine = phase ? (col < b) : (col >= b);
        if (mine) X[col + (uint64_t)d * W] = buf[it];
    }
    if (phase == 0 && b) {
        __syncthreads();
        dif_forward(md, T, buf, LOGC, M, a, a + 1, 0);
        for (uint32_t c = threadIdx.x; c < C; c += blockDim.x)
            if (c0 + c >= b) V[c0 + c] = buf[a * C + c];
    }
}

// --------------------------------------------------------------- row pass
// Forward row pass: workgroup j < a transforms full row j (global block index
// j at size W); workgroup a (when b > 0) builds the last row from its b slots
// and V_c (c >= b) and keeps b outputs.
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_row_fwd(Mod md, Tables<typename Mod::Word> T, typename Mod::Word* X,
                                                      uint32_t logW, uint32_t a, uint32_t b,
                                                      const typename Mod::Word* V) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    const uint32_t j = blockIdx.x;
    const uint32_t W = 1u << logW;
    Word* row = X + (uint64_t)j * W;
    if (j < a) {
        for (uint32_t i = threadIdx.x; i < W; i += blockDim.x) buf[i] = row[i];
        __syncthreads();
        dif_forward(md, T, buf, 0, W, 0, W, j);
        for (uint32_t i = threadIdx.x; i < W; i += blockDim.x) row[i] = buf[i];
    } else {
        for (uint32_t i = threadIdx.x; i < W; i += blockDim.x) buf[i] = i < b ? row[i] : V[i];
        __syncthreads();
        dif_forward(md, T, buf, 0, W, 0, b, a);
        for (uint32_t i = threadIdx.x; i < b; i += blockDim.x) row[i] = buf[i];
    }
}

// Inverse row pass.  Workgroups j < a invert full row j (global block index j
// at size W).  Workgroups a + k invert piece k of the partial last row: the
// dyadic blocks of its b known outputs that the last-row inverse would
// otherwise invert one after another (they read only known outputs, so they
// run here, in parallel with the rows).  With Y non-null, values are first
// multiplied pointwise by Y (the product step fused into the load).
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_row_inv(Mod md, Tables<typename Mod::Word> T, typename Mod::Word* X,
                                                      const typename Mod::Word* Y, uint32_t logW, uint32_t a,
                                                      PieceList pieces) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    const uint32_t W = 1u << logW;
    uint64_t start;
    uint32_t len;
    uint64_t g;
    if (blockIdx.x < a) {
        start = (uint64_t)blockIdx.x * W;
        len = W;
        g = blockIdx.x;
    } else {
        const Piece pc = pieces.p[blockIdx.x - a];
        start = (uint64_t)a * W + pc.off;
        len = pc.size;
        g = pc.g;
    }
    Word* row = X + start;
    if (Y) {
        const Word* yr = Y + start;
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) buf[i] = md.mul(row[i], yr[i]);
    } else {
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) buf[i] = row[i];
    }
    __syncthreads();
    full_inverse(md, T, buf, 0, 0, len, g);
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) row[i] = buf[i];
}

// Inverse of the last row after its pieces were inverted by k_row_inv: the b
// slots now hold the pieces' coefficients and the W - b values V_c are the
// known coefficients of the block; the remaining (elementwise) steps of the
// truncated inverse recover the b column values P_c(w_a), c < b.
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_last_inv(Mod md, Tables<typename Mod::Word> T, typename Mod::Word* X,
                                                       uint32_t logW, uint32_t a, uint32_t b,
                                                       const typename Mod::Word* V) {
    using Word = typename Mod::Word;
    Word* buf = lds_buf<Word>();
    const uint32_t W = 1u << logW;
    Word* row = X + (uint64_t)a * W;
    for (uint32_t i = threadIdx.x; i < W; i += blockDim.x) buf[i] = i < b ? row[i] : V[i];
    __syncthreads();
    gitft(md, T, buf, 0, W, b, a, /*skip_full=*/true);
    for (uint32_t i = threadIdx.x; i < b; i += blockDim.x) row[i] = buf[i];
}

// ---------------------------------------------------------- elementwise
template <class Mod>
__global__ __launch_bounds__(kThreads) void k_pointwise(Mod md, typename Mod::Word* X, const typename Mod::Word* Y,
                                                        uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        X[i] = md.mul(X[i], Y[i]);
}

// dst[i] = i < n_src ? src[i] : 0 for i < n_dst
template <class Word>
__global__ __launch_bounds__(kThreads) void k_copy_pad(Word* dst, uint64_t n_dst, const Word* src, uint64_t n_src) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_dst;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = i < n_src ? src[i] : Word(0);
}

}  // namespace tft
