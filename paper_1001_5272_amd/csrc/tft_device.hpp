// Device-side arithmetic and in-LDS transform routines for the in-place
// truncated Fourier transform (Harvey & Roche 2010) on gfx950.
//
// Notation follows section 2.2 of the paper: w[k] is a primitive 2^k-th root
// of unity with w[k+1]^2 = w[k]; w_s = w[k]^(rev_k s); the transform of F is
// F^_s = F(w_s).  Every routine below computes exactly these values (all
// arithmetic is exact modulo p), so results are bit-identical to any other
// correct implementation.
//
// Transforms inside LDS use the "modular splitting" form of the radix-2 FFT:
// a block of size 2h at global block index i holds F mod (x^{2h} - w_i), and
// because x^{2h} - w_i = (x^h - w_{2i})(x^h + w_{2i}) with w_{2i+1} = -w_{2i}
// (section 2.2 identities) one stage maps (lo, hi) to (lo + w_{2i} hi,
// lo - w_{2i} hi).  After the last stage position s holds F(w_s).  This is the
// same output the paper's even/odd recursion (eq. 1) produces; it is chosen
// here because its stages are layer-parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tft {

// ----------------------------------------------------------------- tables
// Two-level root tables, independent of the transform length:
//   w_s    = f1[s mod 2^B1] * f2[s >> B1]
//   w_s^-1 = i1[s mod 2^B1] * i2[s >> B1]
// For 31-bit primes the entries are stored in Montgomery form (x 2^32).
constexpr int kB1 = 15;
constexpr uint32_t kMask1 = (1u << kB1) - 1;

template <class Word>
struct Tables {
    const Word* f1;
    const Word* f2;
    const Word* i1;
    const Word* i2;
    // optional LDS copies of the small-index twiddles: lf[i] = w_{2i} for
    // i < nlf, li[i] = w_{2i}^-1 for i < nli (every twiddle of a block at
    // global index 0 below that size)
    const Word* lf = nullptr;
    const Word* li = nullptr;
    uint32_t nlf = 0, nli = 0;
    // w_s = w[K]^(rev_K s): K is the order (log 2) of the root the tables
    // expand, so w[K]^e = w_{rev_K e} for 0 <= e < 2^K
    uint32_t K = 0;
    // most stages per LDS round trip (1..3), a tuning parameter of the plan
    uint32_t smax = 3;
};

// Threads in the workgroup.  Every launch here has uniform workgroups, so the
// size comes from the kernel's hidden arguments through one scalar load;
// blockDim.x also allows for a partial last workgroup and compiles to a
// vector load of the dispatch data that is repeated after every barrier.
__device__ __forceinline__ uint32_t nthreads() { return __builtin_amdgcn_workgroup_size_x(); }

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations, not for its global loads and stores, so those stay in
// flight across it (__syncthreads also drains the vector memory counter).
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------- 31-bit primes
// Residues in [0, p), p < 2^31 odd.  Twiddles are kept in Montgomery form
// (w 2^32 mod p) so that mul_tw(x, w 2^32) = x w mod p.
struct ModU32 {
    using Word = uint32_t;
    uint32_t p;        // modulus
    uint32_t pneg;     // -p^-1 mod 2^32
    uint32_t r2;       // 2^64 mod p
    uint32_t halfp1;   // (p + 1) / 2

    __device__ __forceinline__ Word add(Word a, Word b) const {
        Word s = a + b;                      // < 2p < 2^32
        return s < s - p ? s : s - p;        // min(s, s - p) as unsigned
    }
    __device__ __forceinline__ Word sub(Word a, Word b) const {
        Word d = a - b;
        Word e = d + p;
        return d < e ? d : e;
    }
    // Montgomery product a b 2^-32 mod p for a < 2^32, b < p: t = a b and
    // m = t pneg mod 2^32 make t + m p a multiple of 2^32 below 2p 2^32 <
    // 2^64, so its high word is the product in [0, 2p).  Written as two
    // 32 x 32 -> 64 multiply-adds and one low multiply (v_mad_u64_u32,
    // v_mul_lo_u32): five VALU instructions, against eight with separate
    // low and high products and the carry of the low words.
    __device__ __forceinline__ Word mont(Word a, Word b) const {
        const uint64_t t = (uint64_t)a * b;
        const uint32_t m = (uint32_t)t * pneg;
        const uint32_t u = (uint32_t)((t + (uint64_t)m * p) >> 32);
        const uint32_t v = u - p;
        return u < v ? u : v;
    }
    __device__ __forceinline__ Word mul_tw(Word a, Word twm) const { return mont(a, twm); }
    __device__ __forceinline__ Word tw_mul_tw(Word t1, Word t2) const { return mont(t1, t2); }
    // plain product of two residues
    __device__ __forceinline__ Word mul(Word a, Word b) const { return mont(mont(a, b), r2); }
    __device__ __forceinline__ Word half(Word x) const { return (x >> 1) + ((x & 1u) ? halfp1 : 0u); }
    __device__ __forceinline__ Word one_tw() const { return mont(1u, r2); }   // 1 in twiddle (Montgomery) form
    // a b / R: the product of two residues up to a constant factor 1/R, which
    // a later scaling by a twiddle takes back with kappa_tw() (R in twiddle
    // form, R^2 mod p): one Montgomery reduction instead of mul's two
    __device__ __forceinline__ Word mul_scaled(Word a, Word b) const { return mont(a, b); }
    __device__ __forceinline__ Word kappa_tw() const { return r2; }
};

// ------------------------------------------------ other primes p < 2^63
// Residues in [0, p), 2^31 < p < 2^63 odd: 64-bit Montgomery arithmetic
// (R = 2^64), twiddles in Montgomery form (w 2^64 mod p), as ModU32 with
// words of 64 bits.  p < 2^63 keeps a + b and the reduction's (t + m p) / R
// below 2^64.
struct ModM64 {
    using Word = uint64_t;
    uint64_t p;        // modulus
    uint64_t pneg;     // -p^-1 mod 2^64
    uint64_t r2;       // 2^128 mod p
    uint64_t halfp1;   // (p + 1) / 2

    __device__ __forceinline__ Word add(Word a, Word b) const {
        const Word s = a + b;                 // < 2p < 2^64
        return s >= p ? s - p : s;
    }
    __device__ __forceinline__ Word sub(Word a, Word b) const {
        const Word d = a - b;
        return a < b ? d + p : d;
    }
    // Montgomery product a b 2^-64 mod p for a < 2^64, b < p: with
    // m = (a b mod 2^64) pneg mod 2^64, a b + m p is a multiple of 2^64 and
    // (a b + m p) / 2^64 < 2p.
    __device__ __forceinline__ Word mont(Word a, Word b) const {
        const unsigned __int128 t = (unsigned __int128)a * b;
        const uint64_t lo = (uint64_t)t, hi = (uint64_t)(t >> 64);
        const uint64_t m = lo * pneg;
        const uint64_t mh = (uint64_t)(((unsigned __int128)m * p) >> 64);
        const uint64_t u = hi + mh + (lo != 0u ? 1u : 0u);   // the low words sum to 0 or 2^64
        return u >= p ? u - p : u;
    }
    __device__ __forceinline__ Word mul_tw(Word a, Word twm) const { return mont(a, twm); }
    __device__ __forceinline__ Word tw_mul_tw(Word t1, Word t2) const { return mont(t1, t2); }
    // plain product of two residues
    __device__ __forceinline__ Word mul(Word a, Word b) const { return mont(mont(a, b), r2); }
    __device__ __forceinline__ Word half(Word x) const { return (x >> 1) + ((x & 1u) ? halfp1 : 0u); }
    __device__ __forceinline__ Word one_tw() const { return mont(1u, r2); }   // 2^64 mod p
    // a b / R and R in twiddle form (R^2 mod p), as ModU32
    __device__ __forceinline__ Word mul_scaled(Word a, Word b) const { return mont(a, b); }
    __device__ __forceinline__ Word kappa_tw() const { return r2; }
};

// ------------------------------------------------- p = 2^64 - 2^32 + 1
// Residues in [0, p).  2^64 = 2^32 - 1 and 2^96 = -1 modulo p, so a 128-bit
// product reduces with shifts, adds and subtracts only.
struct ModGL {
    using Word = uint64_t;
    static constexpr uint64_t P = 0xFFFFFFFF00000001ull;
    static constexpr uint64_t EPS = 0xFFFFFFFFull;       // 2^64 mod p
    static constexpr uint64_t HALF = 0x7FFFFFFF80000001ull; // (p + 1) / 2

    __device__ __forceinline__ Word add(Word a, Word b) const {
        Word s = a + b;
        return (s < a || s >= P) ? s - P : s;   // wraps: s + 2^64 - p when carried
    }
    __device__ __forceinline__ Word sub(Word a, Word b) const {
        Word d = a - b;
        return (a < b) ? d + P : d;
    }
    __device__ __forceinline__ Word reduce128(uint64_t lo, uint64_t hi) const {
        uint64_t hh = hi >> 32, hl = hi & EPS;
        uint64_t t0 = lo - hh;
        if (lo < hh) t0 -= EPS;                  // borrow: add p
        uint64_t t1 = (hl << 32) - hl;           // hl (2^32 - 1)
        uint64_t r = t0 + t1;
        if (r < t0) r += EPS;                    // carry: add 2^64 mod p
        return r >= P ? r - P : r;
    }
    __device__ __forceinline__ Word mul(Word a, Word b) const {
        unsigned __int128 t = (unsigned __int128)a * b;
        return reduce128((uint64_t)t, (uint64_t)(t >> 64));
    }
    __device__ __forceinline__ Word mul_tw(Word a, Word tw) const { return mul(a, tw); }
    __device__ __forceinline__ Word tw_mul_tw(Word t1, Word t2) const { return mul(t1, t2); }
    __device__ __forceinline__ Word half(Word x) const { return (x >> 1) + ((x & 1ull) ? HALF : 0ull); }
    __device__ __forceinline__ Word one_tw() const { return 1ull; }
    // twiddles are plain residues: no constant factor
    __device__ __forceinline__ Word mul_scaled(Word a, Word b) const { return mul(a, b); }
    __device__ __forceinline__ Word kappa_tw() const { return 1ull; }
};

template <class Mod>
__device__ __forceinline__ typename Mod::Word tw_fwd(const Mod& md, const Tables<typename Mod::Word>& T,
                                                      uint64_t s) {
    if ((s >> 1) < T.nlf && !(s & 1)) return T.lf[s >> 1];
    typename Mod::Word t = T.f1[s & kMask1];
    const uint64_t h = s >> kB1;
    if (h) t = md.tw_mul_tw(t, T.f2[h]);
    return t;
}

template <class Mod>
__device__ __forceinline__ typename Mod::Word tw_inv(const Mod& md, const Tables<typename Mod::Word>& T,
                                                      uint64_t s) {
    if ((s >> 1) < T.nli && !(s & 1)) return T.li[s >> 1];
    typename Mod::Word t = T.i1[s & kMask1];
    const uint64_t h = s >> kB1;
    if (h) t = md.tw_mul_tw(t, T.i2[h]);
    return t;
}

// w[K]^e and w[K]^-e (0 <= e < 2^K) in twiddle form: the tables index roots
// by bit-reversed exponent.
template <class Mod>
__device__ __forceinline__ typename Mod::Word root_pow(const Mod& md, const Tables<typename Mod::Word>& T,
                                                       uint32_t e) {
    return tw_fwd(md, T, (uint64_t)(__builtin_bitreverse32(e) >> (32 - T.K)));
}
template <class Mod>
__device__ __forceinline__ typename Mod::Word root_pow_inv(const Mod& md, const Tables<typename Mod::Word>& T,
                                                           uint32_t e) {
    return tw_inv(md, T, (uint64_t)(__builtin_bitreverse32(e) >> (32 - T.K)));
}

// Copy w_{2i} and w_{2i}^-1 (i < nl, 2 nl <= 2^B1) into LDS at dst (2 nl
// words) and return tables that read them from there.  One coalesced pass
// replaces a dependent global load at the start of every stage group.
// FWD / INV: copy only that direction's table (nl words).
template <class Word, bool FWD = true, bool INV = true>
__device__ __forceinline__ Tables<Word> local_tables(const Tables<Word>& T, Word* dst, uint32_t nl) {
    Tables<Word> L = T;
    for (uint32_t i = threadIdx.x; i < nl; i += nthreads()) {
        if (FWD) dst[i] = T.f1[2 * i];
        if (INV) dst[(FWD ? nl : 0) + i] = T.i1[2 * i];
    }
    lds_sync();
    if (FWD) {
        L.lf = dst;
        L.nlf = nl;
    }
    if (INV) {
        L.li = dst + (FWD ? nl : 0);
        L.nli = nl;
    }
    return L;
}

// z^e for z in twiddle form (square and multiply).
template <class Mod>
__device__ __forceinline__ typename Mod::Word pow_tw(const Mod& md, typename Mod::Word z, uint32_t e) {
    typename Mod::Word r = md.one_tw();
    while (e) {
        if (e & 1u) r = md.tw_mul_tw(r, z);
        z = md.tw_mul_tw(z, z);
        e >>= 1;
    }
    return r;
}

// Workgroup-strided loop over items it < count (it = threadIdx.x + k
// nthreads()) doing put(it, load(it)).  Each thread issues the loads of U
// items before it consumes any, so U memory requests per thread are in flight
// at once rather than one round trip per item.
template <int U, class Load, class Put>
__device__ __forceinline__ void staged_copy(uint32_t count, Load&& load, Put&& put) {
    const uint32_t nt = nthreads();
    uint32_t it = threadIdx.x;
    for (; it + (U - 1) * nt < count; it += U * nt) {
        decltype(load(it)) v[U];
#pragma unroll
        for (int m = 0; m < U; m++) v[m] = load(it + m * nt);
#pragma unroll
        for (int m = 0; m < U; m++) put(it + m * nt, v[m]);
    }
    for (; it < count; it += nt) put(it, load(it));
}

// ------------------------------------------------------- register units
// A radix-2^S unit holds 2^S values x[t] taken at a fixed stride inside one
// block of size 2h (global block index G) and applies the S stages h, h/2,
// ..., h/2^(S-1) to them in registers.  At stage s the unit meets 2^s
// sub-blocks, with global indices G 2^s + q, whose twiddle is w_{2(G 2^s + q)}.
template <class Mod, int S>
struct Unit {
    using Word = typename Mod::Word;
    static constexpr int R = 1 << S;
    Word tw[R - 1];     // twiddle of sub-block q at stage s is tw[(1 << s) - 1 + q]
    uint64_t G = ~0ull;

    __device__ __forceinline__ void load_fwd(const Mod& md, const Tables<Word>& T, uint64_t g) {
        if (g == G) return;
        G = g;
#pragma unroll
        for (int s = 0; s < S; s++)
#pragma unroll
            for (int q = 0; q < (1 << s); q++) tw[(1 << s) - 1 + q] = tw_fwd(md, T, 2 * ((g << s) + q));
    }
    __device__ __forceinline__ void load_inv(const Mod& md, const Tables<Word>& T, uint64_t g) {
        if (g == G) return;
        G = g;
#pragma unroll
        for (int s = 0; s < S; s++)
#pragma unroll
            for (int q = 0; q < (1 << s); q++) tw[(1 << s) - 1 + q] = tw_inv(md, T, 2 * ((g << s) + q));
    }
    // Inside a block at global index 0 the sub-block indices are small, and
    // w_{2x} = tab[x << sh] (tab = lf or li with sh = 0, f1 or i1 with sh = 1):
    // one load per twiddle, with no branch, so all of them are in flight at once.
    __device__ __forceinline__ void load0(const Word* tab, uint32_t sh, uint32_t i) {
#pragma unroll
        for (int s = 0; s < S; s++)
#pragma unroll
            for (int q = 0; q < (1 << s); q++) tw[(1 << s) - 1 + q] = tab[((i << s) + q) << sh];
    }
    // forward: (a, b) -> (a + w b, a - w b), stages s = 0 .. S-1.  TOP: the
    // unit sits in the block at global index 0 (G = 0), where every
    // sub-block q = 0 has twiddle w_0 = 1 and its products are left out.
    template <bool TOP = false>
    __device__ __forceinline__ void forward(const Mod& md, Word (&x)[R]) const {
#pragma unroll
        for (int s = 0; s < S; s++) {
            const int dist = R >> (s + 1);
#pragma unroll
            for (int q = 0; q < (1 << s); q++) {
                const Word w = tw[(1 << s) - 1 + q];
#pragma unroll
                for (int t = 0; t < dist; t++) {
                    const int a = q * 2 * dist + t, b = a + dist;
                    const Word v = (TOP && q == 0) ? x[b] : md.mul_tw(x[b], w);
                    const Word u = x[a];
                    x[a] = md.add(u, v);
                    x[b] = md.sub(u, v);
                }
            }
        }
    }
    // inverse: (a, b) -> ((a + b)/2, (a - b) w^-1 / 2), stages s = S-1 .. 0;
    // HALF = false leaves out the halvings (the caller scales by 2^-stages);
    // TOP as in forward
    template <bool HALF = true, bool TOP = false>
    __device__ __forceinline__ void inverse(const Mod& md, Word (&x)[R]) const {
#pragma unroll
        for (int s = S - 1; s >= 0; s--) {
            const int dist = R >> (s + 1);
#pragma unroll
            for (int q = 0; q < (1 << s); q++) {
                const Word w = tw[(1 << s) - 1 + q];
#pragma unroll
                for (int t = 0; t < dist; t++) {
                    const int a = q * 2 * dist + t, b = a + dist;
                    const Word u = x[a], v = x[b];
                    const bool one = TOP && q == 0;
                    if (HALF) {
                        x[a] = md.half(md.add(u, v));
                        const Word d = md.half(md.sub(u, v));
                        x[b] = one ? d : md.mul_tw(d, w);
                    } else {
                        x[a] = md.add(u, v);
                        const Word d = md.sub(u, v);
                        x[b] = one ? d : md.mul_tw(d, w);
                    }
                }
            }
        }
    }
};

// ------------------------------------------------------- LDS block views
// LDS data tiles are addressed through pad(): one unused word after every 32,
// which spreads the strided accesses of the radix-8 units over the banks (a
// row tile without it meets 16-way bank conflicts in its lowest stages).
__host__ __device__ __forceinline__ uint32_t pad(uint32_t x) { return x + (x >> 5); }
// pad(x + t s) - pad(x) for the elements x + t s (t < R) of a unit at stride s,
// a power of two, when x mod (R s) < s (the unit lies in one aligned block of
// R s words): t s + (t s >> 5), the same in every lane, so a unit computes
// one padded address and adds a wave-uniform offset per element.
__host__ __device__ __forceinline__ uint32_t pad_step(uint32_t t, uint32_t s) { return t * s + ((t * s) >> 5); }
// words of LDS a padded tile of n words occupies
__host__ __device__ __forceinline__ uint32_t padded_words(uint32_t n) { return n + (n >> 5) + 1; }

// A tile in LDS holds C interleaved vectors ("lanes"): element d of lane c is
// buf[d * C + c].  Rows use C = 1.  All routines are called by every thread of
// the workgroup and end with a barrier.

// One group of S forward stages starting at half-size h over the blocks of
// size 2h that meet the wanted outputs [out_lo, out_hi).
// Z: the block is at global index 0 and its twiddles come from tab (see
// Unit::load0); TOP (with Z): this is its first group.
template <class Mod, int S, bool Z = false, bool TOP = false>
__device__ __forceinline__ void dif_group(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf,
                                          int logC, uint32_t M, uint32_t h, uint32_t out_lo, uint32_t out_hi,
                                          uint64_t g0, const typename Mod::Word* tab = nullptr, uint32_t sh = 0) {
    using Word = typename Mod::Word;
    constexpr int R = 1 << S;
    const uint32_t C = 1u << logC;
    const uint32_t q = h >> (S - 1);            // element stride inside a unit = units per block
    const uint32_t logq = __builtin_ctz(q);
    const uint32_t two_h = h << 1;
    const uint32_t i_lo = out_lo / two_h, i_hi = (out_hi - 1) / two_h;
    const uint32_t items = ((i_hi - i_lo + 1) << logq) << logC;
    const uint64_t gbase = g0 * (uint64_t)(M / two_h);
    Unit<Mod, S> un;
    for (uint32_t it = threadIdx.x; it < items; it += nthreads()) {
        const uint32_t c = it & (C - 1);
        const uint32_t u = it >> logC;
        const uint32_t i = i_lo + (u >> logq);
        const uint32_t j = u & (q - 1);
        const uint32_t base = i * two_h + j;
        const uint32_t a0 = pad(base * C + c), st = q << logC;   // (base C + c) mod (2h C) < q C
        Word x[R];
#pragma unroll
        for (int t = 0; t < R; t++) x[t] = buf[a0 + pad_step(t, st)];
        if (Z) un.load0(tab, sh, i);
        else un.load_fwd(md, T, gbase + i);
        un.template forward<TOP>(md, x);
#pragma unroll
        for (int t = 0; t < R; t++) buf[a0 + pad_step(t, st)] = x[t];
    }
    lds_sync();
}

// Lane exchange of one word across the wavefront (64-bit words as two halves).
template <class Word>
__device__ __forceinline__ Word shfl_xor_word(Word v, int mask) {
    if constexpr (sizeof(Word) == 8) {
        const uint32_t lo = __shfl_xor((uint32_t)v, mask), hi = __shfl_xor((uint32_t)(v >> 32), mask);
        return ((uint64_t)hi << 32) | lo;
    } else {
        return __shfl_xor(v, mask);
    }
}

// res[c] = sum of acc over the threads of lane c (thread t is in lane t mod C,
// C <= 64): lane exchanges across each wavefront, then the wavefronts' sums
// through red (LDS, (nthreads() / 64) C words).  Ends with a barrier.
template <class Mod>
__device__ __forceinline__ void reduce_lanes(const Mod& md, typename Mod::Word acc, int logC, typename Mod::Word* red,
                                             typename Mod::Word* res) {
    using Word = typename Mod::Word;
    const uint32_t C = 1u << logC;
    for (uint32_t o = C; o < 64; o <<= 1) acc = md.add(acc, shfl_xor_word(acc, (int)o));
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < C) red[wave * C + lane] = acc;
    lds_sync();
    if (threadIdx.x < C) {
        Word sum = 0;
        for (uint32_t k = 0; k < (nthreads() >> 6); k++) sum = md.add(sum, red[k * C + threadIdx.x]);
        res[threadIdx.x] = sum;
    }
    lds_sync();
}

// Evaluation at one point for every lane of a tile: res[c] = sum_{d < len}
// buf[d C + c] z^d (z in twiddle form).  The nthreads() / C threads of a lane
// each run Horner over one chunk of d and scale by z^(chunk start); the chunk
// values are summed across each wavefront by lane exchanges (threads of one
// lane sit C apart), then across wavefronts.  red is LDS scratch of
// (nthreads() / 64) C words, res of C words; C <= 64.
// The scale factors z^(t chunk) of eval_lanes for the threads t < nthreads() /
// C of a lane, into zp (LDS, written by those threads; the caller's next
// barrier publishes them).  Called early, their power chains overlap the
// caller's loads instead of lengthening the evaluation.
template <class Mod>
__device__ __forceinline__ void eval_scales(const Mod& md, int logC, uint32_t len, typename Mod::Word z,
                                            typename Mod::Word* zp) {
    const uint32_t tpc = nthreads() >> logC;
    const uint32_t chunk = (len + tpc - 1) / tpc;
    if (threadIdx.x < tpc) zp[threadIdx.x] = pow_tw(md, z, threadIdx.x * chunk);
}

template <class Mod>
__device__ __forceinline__ void eval_lanes(const Mod& md, const typename Mod::Word* buf, int logC, uint32_t len, typename Mod::Word z,
                           typename Mod::Word* red, typename Mod::Word* res, const typename Mod::Word* zp = nullptr) {
    using Word = typename Mod::Word;
    const uint32_t C = 1u << logC;
    const uint32_t tpc = nthreads() >> logC;
    const uint32_t c = threadIdx.x & (C - 1), t = threadIdx.x >> logC;
    const uint32_t chunk = (len + tpc - 1) / tpc;
    const uint32_t lo = t * chunk;
    const uint32_t hi = lo + chunk < len ? lo + chunk : len;
    Word acc = 0;
    for (uint32_t d = hi; d > lo; d--) acc = md.add(md.mul_tw(acc, z), buf[pad((d - 1) * C + c)]);
    if (lo > 0 && lo < hi) acc = md.mul_tw(acc, zp ? zp[t] : pow_tw(md, z, lo));
    reduce_lanes(md, acc, logC, red, res);
}

// Stages per LDS round trip (1..3, at most `left`) for a pass over `words`
// words.  Radix-8 units do the least work per butterfly, but a unit is a long
// dependent chain for one lane: when the radix-8 units would leave more than
// half of the workgroup idle (a block that alone occupies the CU), smaller
// units give more lanes shorter chains.
__device__ __forceinline__ int group_stages(uint32_t words, int left, uint32_t smax = 3) {
    const uint32_t half = nthreads() >> 1;
    int S = (int)smax;
    while (S > 1 && (words >> S) < half) S--;
    return S < left ? S : left;
}

// Forward transform of the block of size M at global index g0 (the block is
// F mod (x^M - w_{g0})); only blocks meeting [out_lo, out_hi) are computed, so
// positions outside that range end with unspecified values.
// Stages h_hi, h_hi/2, ..., h_lo (powers of two, h_lo <= h_hi <= M/2) of the
// forward transform of that block, in groups of at most three.
template <class Mod>
__device__ __forceinline__ void dif_stages(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf, int logC,
                           uint32_t M, uint32_t h_hi, uint32_t h_lo, uint32_t out_lo, uint32_t out_hi, uint64_t g0) {
    const uint32_t words = M << logC;
    const int lo = __builtin_ctz(h_lo);
    if (g0 == 0) {
        // block 0: twiddles w_{2x}, x < M/2, from the LDS copy when it reaches
        // that far, else read in place from f1 (x < 2^(B1-1) for M <= 2^B1)
        const bool lds = T.nlf >= (M >> 1);
        const typename Mod::Word* tab = lds ? T.lf : T.f1;
        const uint32_t sh = lds ? 0u : 1u;
        for (uint32_t h = h_hi; h >= h_lo;) {
            const int S = group_stages(words, __builtin_ctz(h) - lo + 1, T.smax);
            if (h == M >> 1) {   // the first group: sub-blocks q = 0 have twiddle 1
                if (S == 3) dif_group<Mod, 3, true, true>(md, T, buf, logC, M, h, out_lo, out_hi, 0, tab, sh);
                else if (S == 2) dif_group<Mod, 2, true, true>(md, T, buf, logC, M, h, out_lo, out_hi, 0, tab, sh);
                else dif_group<Mod, 1, true, true>(md, T, buf, logC, M, h, out_lo, out_hi, 0, tab, sh);
            } else {
                if (S == 3) dif_group<Mod, 3, true>(md, T, buf, logC, M, h, out_lo, out_hi, 0, tab, sh);
                else if (S == 2) dif_group<Mod, 2, true>(md, T, buf, logC, M, h, out_lo, out_hi, 0, tab, sh);
                else dif_group<Mod, 1, true>(md, T, buf, logC, M, h, out_lo, out_hi, 0, tab, sh);
            }
            h >>= S;
        }
        return;
    }
    for (uint32_t h = h_hi; h >= h_lo;) {
        const int S = group_stages(words, __builtin_ctz(h) - lo + 1, T.smax);
        if (S == 3) dif_group<Mod, 3>(md, T, buf, logC, M, h, out_lo, out_hi, g0);
        else if (S == 2) dif_group<Mod, 2>(md, T, buf, logC, M, h, out_lo, out_hi, g0);
        else dif_group<Mod, 1>(md, T, buf, logC, M, h, out_lo, out_hi, g0);
        h >>= S;
    }
}

// Forward transform of the block of size M at global index g0 (the block is
// F mod (x^M - w_{g0})); only blocks meeting [out_lo, out_hi) are computed, so
// positions outside that range end with unspecified values.
template <class Mod>
__device__ __forceinline__ void dif_forward(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf, int logC,
                            uint32_t M, uint32_t out_lo, uint32_t out_hi, uint64_t g0) {
    if (M >= 2) dif_stages(md, T, buf, logC, M, M >> 1, 1, out_lo, out_hi, g0);
}

// One group of S inverse stages ending at half-size h (stages h/2^(S-1) .. h)
// over every block of size 2h inside [off, off + Sz).
// Z and TOP as in dif_group (TOP: the last group of a block at index 0).
template <class Mod, int S, bool SYNC = true, bool HALF = true, bool Z = false, bool TOP = false>
__device__ __forceinline__ void dit_group(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf,
                                          int logC, uint32_t off, uint32_t Sz, uint32_t h, uint64_t g,
                                          const typename Mod::Word* tab = nullptr, uint32_t sh = 0) {
    using Word = typename Mod::Word;
    constexpr int R = 1 << S;
    const uint32_t C = 1u << logC;
    const uint32_t q = h >> (S - 1);
    const uint32_t logq = __builtin_ctz(q);
    const uint32_t two_h = h << 1;
    const uint32_t items = (Sz >> S) << logC;   // one unit per R elements
    const uint64_t gbase = g * (uint64_t)(Sz / two_h);
    Unit<Mod, S> un;
    for (uint32_t it = threadIdx.x; it < items; it += nthreads()) {
        const uint32_t c = it & (C - 1);
        const uint32_t u = it >> logC;
        const uint32_t i = u >> logq;
        const uint32_t j = u & (q - 1);
        const uint32_t base = off + i * two_h + j;
        const uint32_t a0 = pad(base * C + c), st = q << logC;   // off is a multiple of Sz >= 2h
        Word x[R];
#pragma unroll
        for (int t = 0; t < R; t++) x[t] = buf[a0 + pad_step(t, st)];
        if (Z) un.load0(tab, sh, i);
        else un.load_inv(md, T, gbase + i);
        un.template inverse<HALF, TOP>(md, x);
#pragma unroll
        for (int t = 0; t < R; t++) buf[a0 + pad_step(t, st)] = x[t];
    }
    if (SYNC) lds_sync();
}

// Inverse stages 2^d0 .. 2^(d1-1) (0 <= d0 < d1 <= lg Sz) of the block of size
// Sz at offset off with global block index g, in groups of at most three.
// RADIX8: always three stages per pass (a latency-bound single workgroup
// prefers fewer barriers to more busy lanes).
template <class Mod, bool HALF = true, bool RADIX8 = false>
__device__ __forceinline__ void dit_stages(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf, int logC,
                           uint32_t off, uint32_t Sz, int d0, int d1, uint64_t g) {
    const int L = __builtin_ctz(Sz);
    const uint32_t words = Sz << logC;
    for (int done = d0; done < d1;) {    // stages 2^d0 .. 2^(done-1) finished
        const int S = RADIX8 ? (d1 - done < 3 ? d1 - done : 3) : group_stages(words, d1 - done, T.smax);
        const uint32_t h = 1u << (done + S - 1);
        if (g == 0) {   // block 0: twiddles as in dif_stages; the last group skips twiddle 1
            const bool lds = T.nli >= (Sz >> 1);
            const typename Mod::Word* tab = lds ? T.li : T.i1;
            const uint32_t sh = lds ? 0u : 1u;
            if (done + S == L) {
                if (S == 3) dit_group<Mod, 3, true, HALF, true, true>(md, T, buf, logC, off, Sz, h, 0, tab, sh);
                else if (S == 2) dit_group<Mod, 2, true, HALF, true, true>(md, T, buf, logC, off, Sz, h, 0, tab, sh);
                else dit_group<Mod, 1, true, HALF, true, true>(md, T, buf, logC, off, Sz, h, 0, tab, sh);
            } else {
                if (S == 3) dit_group<Mod, 3, true, HALF, true>(md, T, buf, logC, off, Sz, h, 0, tab, sh);
                else if (S == 2) dit_group<Mod, 2, true, HALF, true>(md, T, buf, logC, off, Sz, h, 0, tab, sh);
                else dit_group<Mod, 1, true, HALF, true>(md, T, buf, logC, off, Sz, h, 0, tab, sh);
            }
        } else {
            if (S == 3) dit_group<Mod, 3, true, HALF>(md, T, buf, logC, off, Sz, h, g);
            else if (S == 2) dit_group<Mod, 2, true, HALF>(md, T, buf, logC, off, Sz, h, g);
            else dit_group<Mod, 1, true, HALF>(md, T, buf, logC, off, Sz, h, g);
        }
        done += S;
    }
}

// Full inverse of the forward stages on the block of size Sz at offset off with
// global block index g: stages 1, 2, ..., Sz/2.  HALF = false leaves every
// value multiplied by Sz (the caller scales by 1/Sz, e.g. on its store).
template <class Mod, bool HALF = true, bool RADIX8 = false>
__device__ __forceinline__ void full_inverse(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf, int logC,
                             uint32_t off, uint32_t Sz, uint64_t g) {
    if (Sz >= 2) dit_stages<Mod, HALF, RADIX8>(md, T, buf, logC, off, Sz, 0, __builtin_ctz(Sz), g);
}

// 2^-L in twiddle form.
template <class Mod>
__device__ __forceinline__ typename Mod::Word inv_pow2_tw(const Mod& md, int L) {
    typename Mod::Word s = md.one_tw();
    for (int i = 0; i < L; i++) s = md.half(s);   // halving commutes with the twiddle form's constant factor
    return s;
}

// Generalised inverse truncated transform of one block.
//
// On entry, a block of size M (power of two) at global index g0 has its first
// m positions holding transform values (the polynomial B of degree < M taken
// at w_{g0 M + s}, s < m) and positions [m, M) holding the coefficients
// B_m..B_{M-1}, which are known.  On exit all M positions hold B's
// coefficients.  (For an ordinary inverse TFT of length m the known
// coefficients are zeros.)
//
// The recursion follows the truncation boundary down the splitting tree.  At
// a block of size 2h with twiddle w = w_{2g}, writing C0 = lo + w hi and
// C1 = lo - w hi for its children:
//   m >= h: C0's h values are all known, so C0 is recovered by a full inverse;
//           for j >= m - h the coefficient hi_j is known, so C1_j = C0_j - 2 w hi_j
//           becomes a known coefficient of the right child, which is solved
//           recursively with m - h known values; then (lo, hi) follow from
//           (C0, C1) by the inverse butterfly.
//   m <  h: for j >= m both lo_j and hi_j are known, so C0_j = lo_j + w hi_j is
//           a known coefficient of the left child, which is solved
//           recursively; then lo_j = C0_j - w hi_j.
// The schedule here is not recursive.  The full inverses act on the dyadic
// pieces of [0, m) and read only given values, so they all run first
// (pieces_inverse).  The downward steps then touch only positions >= m, and
// the upward steps follow; both are taken three levels at a time in
// registers (walk_group), so a block of size 2^L needs about L barriers in all
// rather than one per level.  A caller that has already inverted the pieces
// (elsewhere, in parallel) passes skip_full = true.
constexpr int kMaxLevels = 24;   // log2 of the largest LDS block, with room

// Level d of gitft's walk along the truncation boundary: offset, half size
// and global index of the block met there, the number m of transform values
// it holds, and whether the walk goes on to its right child.
struct Level {
    uint32_t off, h, m;
    uint64_t g;
    bool right;
};
__device__ __forceinline__ Level gitft_level(uint32_t M, uint32_t m, uint64_t g0, int d) {
    uint32_t off = 0, size = M;
    uint64_t g = g0;
    for (int i = 0;; i++) {
        const uint32_t h = size >> 1;
        const bool right = m >= h;
        if (i == d) return Level{off, h, m, g, right};
        if (right) {
            off += h;
            g = 2 * g + 1;
            m -= h;
        } else {
            g = 2 * g;
        }
        size = h;
    }
}

// Number of levels of the walk (blocks with 0 < m < size).
__host__ __device__ __forceinline__ int gitft_depth(uint32_t M, uint32_t m) {
    int d = 0;
    while (M > 1 && m > 0 && m < M) {
        M >>= 1;
        if (m >= M) m -= M;
        d++;
    }
    return d;
}

// The full inverses of all pieces of [0, m) inside the block (size M, global
// index g0).  The pieces are the dyadic blocks given by the set bits of m (bit
// e: the block of size 2^e at offset m with bits 0..e cleared).  A pass takes
// stages 2^s0 .. 2^(s0+S-1) (S from group_stages): the pieces of size at least
// 2^(s0+S) are unions of aligned blocks of that size, which together fill
// [0, mS) (m rounded down to a multiple of 2^(s0+S)) and take radix-2^S
// units, while the pieces for bits s0+2 and s0+1 of m (below s0+S) take their
// last two or one stages here.  One barrier per pass.  The butterflies leave
// out the halvings: a unit whose piece this pass completes (piece size
// 2^(s0+S), 2^(s0+2) or 2^(s0+1)) scales its values by 2^-e from scale[e].
// With tab set the block sits at global index 0 and its twiddles come from tab
// (see Unit::load0).
template <class Mod, int S>
__device__ __forceinline__ void pieces_pass(const Mod& md, const Tables<typename Mod::Word>& T,
                                            typename Mod::Word* buf, int logC, uint32_t m, uint64_t gbase,
                                            uint32_t s0, const typename Mod::Word* scale,
                                            const typename Mod::Word* tab, uint32_t sh) {
    using Word = typename Mod::Word;
    constexpr int R = 1 << S;
    const uint32_t C = 1u << logC;
    const uint32_t q = 1u << s0;
    const uint32_t mS = (m >> (s0 + S)) << (s0 + S);
    const uint32_t nS = mS >> S;
    const uint32_t n4 = S == 3 ? ((m >> (s0 + 2)) & 1u) << s0 : 0u;
    const uint32_t n2 = S >= 2 ? ((m >> (s0 + 1)) & 1u) << s0 : 0u;
    const uint32_t off4 = mS, off2 = mS + (n4 << 2);
    const uint32_t items = (nS + n4 + n2) << logC;
    Unit<Mod, S> uS;
    Unit<Mod, 2> u4;
    Unit<Mod, 1> u2;
    if (tab) {
        if (n4) u4.load0(tab, sh, off4 >> (s0 + 2));
        if (n2) u2.load0(tab, sh, off2 >> (s0 + 1));
    } else {
        if (n4) u4.load_inv(md, T, (gbase + off4) >> (s0 + 2));
        if (n2) u2.load_inv(md, T, (gbase + off2) >> (s0 + 1));
    }
    for (uint32_t it = threadIdx.x; it < items; it += nthreads()) {
        const uint32_t c = it & (C - 1);
        const uint32_t u = it >> logC;
        if (u < nS) {
            const uint32_t i = u >> s0, j = u & (q - 1);
            const uint32_t base = (i << (s0 + S)) + j;
            Word x[R];
#pragma unroll
            for (int t = 0; t < R; t++) x[t] = buf[pad((base + t * q) * C + c)];
            if (tab) uS.load0(tab, sh, i);
            else uS.load_inv(md, T, (gbase >> (s0 + S)) + i);
            uS.template inverse<false>(md, x);
            if (31 - __builtin_clz(base ^ m) == (int)(s0 + S)) {   // the unit's piece is complete
                const Word sc = scale[s0 + S];
#pragma unroll
                for (int t = 0; t < R; t++) x[t] = md.mul_tw(x[t], sc);
            }
#pragma unroll
            for (int t = 0; t < R; t++) buf[pad((base + t * q) * C + c)] = x[t];
        } else if (u < nS + n4) {
            const uint32_t base = off4 + (u - nS);
            Word x[4];
#pragma unroll
            for (int t = 0; t < 4; t++) x[t] = buf[pad((base + t * q) * C + c)];
            u4.template inverse<false>(md, x);
            const Word sc = scale[s0 + 2];
#pragma unroll
            for (int t = 0; t < 4; t++) buf[pad((base + t * q) * C + c)] = md.mul_tw(x[t], sc);
        } else {
            const uint32_t base = off2 + (u - nS - n4);
            Word x[2];
#pragma unroll
            for (int t = 0; t < 2; t++) x[t] = buf[pad((base + t * q) * C + c)];
            u2.template inverse<false>(md, x);
            const Word sc = scale[s0 + 1];
#pragma unroll
            for (int t = 0; t < 2; t++) buf[pad((base + t * q) * C + c)] = md.mul_tw(x[t], sc);
        }
    }
    lds_sync();
}

// The full inverses of the pieces (see pieces_pass), each scaled by 2^-e for
// its size 2^e in the pass that completes it.
template <class Mod>
__device__ __forceinline__ void pieces_inverse(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf, int logC,
                               uint32_t M, uint32_t m, uint64_t g0) {
    using Word = typename Mod::Word;
    __shared__ Word scale[32];
    const uint64_t gbase = g0 << __builtin_ctz(M);   // global position of the block's first word
    const int top = 31 - __builtin_clz(m);            // largest piece: 2^top
    if (top == 0) return;
    if (threadIdx.x <= (uint32_t)top) scale[threadIdx.x] = inv_pow2_tw(md, (int)threadIdx.x);
    lds_sync();
    // block 0: twiddles w_{2x}^-1 from the LDS copy or read in place from i1
    const Word* tab = nullptr;
    uint32_t sh = 0;
    if (g0 == 0) {
        tab = T.nli >= (M >> 1) ? T.li : T.i1;
        sh = T.nli >= (M >> 1) ? 0u : 1u;
    }
    for (int s0 = 0; s0 < top;) {
        const int S = group_stages(m << logC, top - s0, T.smax);
        if (S == 3) pieces_pass<Mod, 3>(md, T, buf, logC, m, gbase, (uint32_t)s0, scale, tab, sh);
        else if (S == 2) pieces_pass<Mod, 2>(md, T, buf, logC, m, gbase, (uint32_t)s0, scale, tab, sh);
        else pieces_pass<Mod, 1>(md, T, buf, logC, m, gbase, (uint32_t)s0, scale, tab, sh);
        s0 += S;
    }
}

// Per-level data of gitft's walk, filled once per call (one thread per level)
// so that the passes below read it from LDS instead of re-walking the tree in
// every wave.
template <class Word>
struct WalkTable {
    uint32_t off[kMaxLevels];   // block offset
    uint32_t h[kMaxLevels];     // half size
    uint32_t lb[kMaxLevels];    // first j of the downward step's range, top bit = walk goes right
    Word w[kMaxLevels], wi[kMaxLevels];
};
constexpr uint32_t kRightBit = 1u << 31;

// S consecutive levels d0 .. d0+S-1 of gitft's walk in one pass.  With u the
// half size of the deepest of them, the values at positions j + t u (t < 2^S)
// of the level-d0 block contain every pair that the S levels combine, so one
// unit per j < u does all S levels in registers.  Slot k of the unit holds
// position t = k ^ rmask (rmask = the S walk directions, level d0 in the top
// bit): at level d0+s the unit's part of the current block is slots
// k < 2^(S-s), its child half slots k < 2^(S-s-1) and the sibling half the
// rest, whatever the directions.
//   down = true: the known-coefficient steps (C1_j = C0_j - 2 w hi_j on the
//     right, C0_j = lo_j + w hi_j on the left) for j in the level's range;
//   down = false: the upward steps, deepest level first.
// The upward steps write their results through sink(position, lane, value)
// (LdsSink: back into the tile).
template <class Word>
struct LdsSink {
    Word* buf;
    uint32_t C;
    __device__ __forceinline__ void operator()(uint32_t p, uint32_t c, Word v) const { buf[pad(p * C + c)] = v; }
};
template <class Mod, int S, class Sink>
__device__ __forceinline__ void walk_group(const Mod& md, typename Mod::Word* buf, int logC, int d0,
                           const WalkTable<typename Mod::Word>& L, bool down, const Sink& sink) {
    using Word = typename Mod::Word;
    constexpr int R = 1 << S;
    const uint32_t C = 1u << logC;
    uint32_t lb[S];
    bool rt[S];
    Word w[S], wi[S];
    uint32_t rmask = 0;
    const uint32_t off = L.off[d0];
    const uint32_t u = L.h[d0 + S - 1];
#pragma unroll
    for (int s = 0; s < S; s++) {
        const uint32_t v = L.lb[d0 + s];
        rt[s] = (v & kRightBit) != 0;
        lb[s] = v & ~kRightBit;
        rmask |= (rt[s] ? 1u : 0u) << (S - 1 - s);
        w[s] = L.w[d0 + s];
        wi[s] = L.wi[d0 + s];
    }
    const uint32_t items = u << logC;
    for (uint32_t it = threadIdx.x; it < items; it += nthreads()) {
        const uint32_t c = it & (C - 1);
        const uint32_t j = it >> logC;
        if (down) {
            // a unit with no position in range at any level has nothing to do
            bool any = false;
#pragma unroll
            for (int s = 0; s < S; s++) any |= j + ((R >> (s + 1)) - 1) * u >= lb[s];
            if (!any) continue;
        }
        Word x[R];
#pragma unroll
        for (int k = 0; k < R; k++) x[k] = buf[pad((off + j + (k ^ rmask) * u) * C + c)];
        if (down) {
#pragma unroll
            for (int s = 0; s < S; s++) {
                const int half = R >> (s + 1);
#pragma unroll
                for (int k = 0; k < half; k++) {
                    const uint32_t jj = j + ((k ^ rmask) & (half - 1)) * u;
                    if (jj >= lb[s]) {
                        const Word child = x[k], other = x[k + half];
                        if (rt[s]) {
                            const Word t = md.mul_tw(child, w[s]);
                            x[k] = md.sub(md.sub(other, t), t);
                        } else {
                            x[k] = md.add(child, md.mul_tw(other, w[s]));
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < R / 2; k++) buf[pad((off + j + (k ^ rmask) * u) * C + c)] = x[k];
        } else {
#pragma unroll
            for (int s = S - 1; s >= 0; s--) {
                const int half = R >> (s + 1);
#pragma unroll
                for (int k = 0; k < half; k++) {
                    const Word child = x[k], other = x[k + half];
                    if (rt[s]) {   // lo = other, hi = child
                        x[k + half] = md.half(md.add(other, child));
                        x[k] = md.mul_tw(md.half(md.sub(other, child)), wi[s]);
                    } else {       // lo = child, hi = other
                        x[k] = md.sub(child, md.mul_tw(other, w[s]));
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < R; k++) sink(off + j + (k ^ rmask) * u, c, x[k]);
        }
    }
    lds_sync();
}

template <class Mod, class Sink>
__device__ __forceinline__ void walk_levels(const Mod& md, typename Mod::Word* buf, int logC, int d0, int S,
                            const WalkTable<typename Mod::Word>& L, bool down, const Sink& sink) {
    if (S == 3) walk_group<Mod, 3>(md, buf, logC, d0, L, down, sink);
    else if (S == 2) walk_group<Mod, 2>(md, buf, logC, d0, L, down, sink);
    else walk_group<Mod, 1>(md, buf, logC, d0, L, down, sink);
}

// final (optional): where the last upward pass writes the finished block
// (position, lane, value) instead of the tile; without a walk the block is
// copied to it from the tile.
template <class Mod, class Sink = LdsSink<typename Mod::Word>>
__device__ __forceinline__ void gitft(const Mod& md, const Tables<typename Mod::Word>& T, typename Mod::Word* buf, int logC,
                      uint32_t M, uint32_t m, uint64_t g0, bool skip_full = false, const Sink* final = nullptr) {
    using Word = typename Mod::Word;
    __shared__ WalkTable<Word> L;
    const int depth = gitft_depth(M, m);
    if (threadIdx.x < (uint32_t)depth) {
        const int d = (int)threadIdx.x;
        const Level v = gitft_level(M, m, g0, d);
        L.off[d] = v.off;
        L.h[d] = v.h;
        L.lb[d] = v.right ? (v.m - v.h) | kRightBit : v.m;
        L.w[d] = tw_fwd(md, T, 2 * v.g);
        L.wi[d] = tw_inv(md, T, 2 * v.g);
    }
    if (!skip_full && (m >> 1) != 0) pieces_inverse(md, T, buf, logC, M, m, g0);   // ends with a barrier
    else lds_sync();
    const LdsSink<Word> tile{buf, 1u << logC};
    for (int d = 0; d < depth; d += 3) walk_levels(md, buf, logC, d, depth - d < 3 ? depth - d : 3, L, true, tile);
    for (int e = depth; e > 0; e -= 3) {
        const int S = e < 3 ? e : 3;
        if (final && e == S) walk_levels(md, buf, logC, e - S, S, L, false, *final);
        else walk_levels(md, buf, logC, e - S, S, L, false, tile);
    }
    if (final && depth == 0) {
        for (uint32_t it = threadIdx.x; it < (M << logC); it += nthreads())
            (*final)(it >> logC, it & ((1u << logC) - 1), buf[pad(it)]);
    }
}

// The full-inverse pieces of gitft(M, m, g0): dyadic blocks (offset, size,
// global index) that partition [0, m) (a final piece may have size 1, whose
// inverse is the identity).  Returns the count (at most 1 + log2 M).
struct Piece {
    uint32_t off, size;
    uint64_t g;
};
constexpr int kMaxPieces = 20;

// The piece number `want` of gitft_pieces(M, m, g0) (same walk, no array).
__host__ __device__ inline Piece gitft_piece(uint32_t M, uint32_t m, uint64_t g0, int want) {
    int k = 0;
    uint32_t off = 0, size = M;
    uint64_t g = g0;
    while (size > 1 && m > 0 && m < size) {
        const uint32_t h = size >> 1;
        if (m >= h) {
            if (k++ == want) return Piece{off, h, 2 * g};
            off += h;
            g = 2 * g + 1;
            m -= h;
        } else {
            g = 2 * g;
        }
        size = h;
    }
    return Piece{off, size, g};
}
struct PieceList {
    int count;
    Piece p[kMaxPieces];
};
__host__ __device__ inline int gitft_pieces(uint32_t M, uint32_t m, uint64_t g0, Piece* out) {
    int k = 0;
    uint32_t off = 0, size = M;
    uint64_t g = g0;
    while (size > 1 && m > 0 && m < size) {
        const uint32_t h = size >> 1;
        if (m >= h) {
            out[k++] = Piece{off, h, 2 * g};
            off += h;
            g = 2 * g + 1;
            m -= h;
        } else {
            g = 2 * g;
        }
        size = h;
    }
    if (m > 0 && m == size) out[k++] = Piece{off, size, g};   // may be a single element
    return k;
}

}  // namespace tft
