// Host side of libtft: contexts (prime, roots, tables), the planner that picks
// the schedule for a length n, and the C entry points declared in
// include/libtft.h.  All device work is in tft_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "libtft.h"
#include "tft_kernels.hpp"

using tft::kB1;
using tft::kThreads;

namespace {

constexpr uint64_t kGoldilocks = 0xFFFFFFFF00000001ull;
constexpr unsigned kMaxLog2 = 28;               // longest transform supported by the tables
constexpr size_t kScratchWords = size_t(1) << 16;   // V_c area: one word per column, W <= 2^16
constexpr size_t kLdsSoft = 64 * 1024;          // preferred LDS per workgroup
constexpr size_t kLdsHard = 160 * 1024;         // gfx950 LDS per workgroup

typedef unsigned __int128 u128;

uint64_t mulmod_h(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }
uint64_t powmod_h(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulmod_h(r, a, p);
        a = mulmod_h(a, a, p);
        e >>= 1;
    }
    return r;
}
uint64_t rev_bits(uint64_t s, unsigned k) {
    uint64_t r = 0;
    for (unsigned i = 0; i < k; i++) { r = (r << 1) | (s & 1); s >>= 1; }
    return r;
}
uint64_t pow2ceil(uint64_t x) {
    uint64_t m = 1;
    while (m < x) m <<= 1;
    return m;
}
unsigned log2u(uint64_t x) {
    unsigned k = 0;
    while ((1ull << k) < x) k++;
    return k;
}

struct Plan {
    int kind;            // 0 single workgroup, 1 two-pass
    uint64_t n;
    unsigned logW;
    uint64_t W, a, b;
    uint32_t Lout, M;    // column outputs and column LDS block (kind 1); LDS block (kind 0)
    int logC;
    size_t lds_col, lds_row;
};

}  // namespace

struct tft_ctx {
    int device;
    uint64_t p, g;
    unsigned v;          // usable log2 length
    unsigned wbytes;     // 4 or 8
    unsigned override_logW;
    tft::ModU32 m32;
    tft::ModGL m64;
    void* tables;        // f1 | f2 | i1 | i2
    size_t n1, n2;       // entries per level
    void* scratch;       // V_c area
    // measurement mode (tft_timing_*): events bracketing each launch
    bool timing;
    struct Rec { int kid; hipEvent_t e0, e1; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    uint64_t launches[TFT_K_COUNT];
    double total_ms[TFT_K_COUNT];
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline tft_status launch_status() { return hipGetLastError() == hipSuccess ? TFT_OK : TFT_EDEVICE; }

hipEvent_t take_event(tft_ctx* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Every kernel goes through here; in measurement mode the launch is bracketed
// by two events on its stream.
template <typename Kernel, typename... Args>
void launch(tft_ctx* ctx, int kid, Kernel kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st,
            Args... args) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        e0 = take_event(ctx);
        e1 = take_event(ctx);
        if (e0 && e1) (void)hipEventRecord(e0, st);
    }
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
    if (e0 && e1) {
        (void)hipEventRecord(e1, st);
        ctx->recs.push_back({kid, e0, e1});
    }
}

unsigned small_max_log2(unsigned wbytes) { return wbytes == 4 ? 13 : 12; }

Plan make_plan(const tft_ctx* ctx, uint64_t n) {
    Plan P{};
    P.n = n;
    const unsigned w = ctx->wbytes;
    if (log2u(n) <= small_max_log2(w) && !(ctx->override_logW && (1ull << ctx->override_logW) < n)) {
        P.kind = 0;
        P.M = (uint32_t)pow2ceil(n);
        P.lds_row = (size_t)P.M * w;
        return P;
    }
    P.kind = 1;
    P.logC = (w == 4) ? 4 : 3;   // 64-byte segments per column tile row
    auto fill = [&](unsigned logW) {
        P.logW = logW;
        P.W = 1ull << logW;
        P.a = n >> logW;
        P.b = n & (P.W - 1);
        P.Lout = (uint32_t)(P.a + (P.b ? 1 : 0));
        P.M = (uint32_t)pow2ceil(P.Lout);
        P.lds_col = ((size_t)P.M << P.logC) * w;
        P.lds_row = (size_t)P.W * w;
    };
    const unsigned logC = (unsigned)P.logC;
    if (ctx->override_logW) {
        fill(ctx->override_logW);
        if (P.W < (1ull << logC) || P.a < 1 || P.lds_col > kLdsHard || P.lds_row > kLdsHard) P.kind = -1;
        return P;
    }
    for (size_t lim : {kLdsSoft, kLdsHard - 32 * 1024}) {
        for (unsigned logW = logC; logW <= 16 && (1ull << logW) <= n; logW++) {
            fill(logW);
            if (P.lds_col <= lim && P.lds_row <= lim) return P;
        }
    }
    P.kind = -1;   // beyond this build's two-pass limit
    return P;
}

template <class Word>
tft::Tables<Word> tables_of(const tft_ctx* ctx) {
    const Word* base = reinterpret_cast<const Word*>(ctx->tables);
    tft::Tables<Word> T;
    T.f1 = base;
    T.f2 = base + ctx->n1;
    T.i1 = base + ctx->n1 + ctx->n2;
    T.i2 = base + 2 * ctx->n1 + ctx->n2;
    return T;
}

template <class Mod>
const Mod& mod_of(const tft_ctx* ctx);
template <>
const tft::ModU32& mod_of<tft::ModU32>(const tft_ctx* ctx) { return ctx->m32; }
template <>
const tft::ModGL& mod_of<tft::ModGL>(const tft_ctx* ctx) { return ctx->m64; }

template <class Mod>
void set_lds_limits() {
    const int lim = (int)kLdsHard;
    (void)hipFuncSetAttribute((const void*)tft::k_small_fwd<Mod>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_small_inv<Mod>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_small_mul<Mod>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_col_fwd<Mod, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_col_fwd<Mod, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_col_inv<Mod, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_col_inv<Mod, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_row_fwd<Mod>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_row_inv<Mod>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)tft::k_last_inv<Mod>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

// -------------------------------------------------------------- forward
template <class Mod>
tft_status forward_impl(tft_ctx* ctx, const typename Mod::Word* src, uint64_t n_src, typename Mod::Word* X,
                        uint64_t n, hipStream_t st) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const auto T = tables_of<Word>(ctx);
    const Plan P = make_plan(ctx, n);
    if (P.kind < 0) return TFT_ERANGE;
    if (P.kind == 0) {
        if (src != X) {
            launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3(1), dim3(kThreads), 0, st, X, n, src, n_src);
        }
        launch(ctx, TFT_K_SMALL_FWD, tft::k_small_fwd<Mod>, dim3(1), dim3(kThreads), P.lds_row, st, md, T, X, (uint32_t)n,
                           P.M);
        return launch_status();
    }
    Word* V = reinterpret_cast<Word*>(ctx->scratch);
    const uint32_t tiles = (uint32_t)(P.W >> P.logC);
    if (P.logC == 3)
        launch(ctx, TFT_K_COL_FWD, tft::k_col_fwd<Mod, 3>, dim3(tiles), dim3(kThreads), P.lds_col, st, md, T, src, n_src, X,
                           n, P.logW, (uint32_t)P.a, (uint32_t)P.b, P.Lout, P.M, V, tiles);
    else
        launch(ctx, TFT_K_COL_FWD, tft::k_col_fwd<Mod, 4>, dim3(tiles), dim3(kThreads), P.lds_col, st, md, T, src, n_src, X,
                           n, P.logW, (uint32_t)P.a, (uint32_t)P.b, P.Lout, P.M, V, tiles);
    launch(ctx, TFT_K_ROW_FWD, tft::k_row_fwd<Mod>, dim3((uint32_t)(P.a + (P.b ? 1 : 0))), dim3(kThreads), P.lds_row, st, md,
                       T, X, P.logW, (uint32_t)P.a, (uint32_t)P.b, V);
    return launch_status();
}

// -------------------------------------------------------------- inverse
template <class Mod>
tft_status inverse_impl(tft_ctx* ctx, typename Mod::Word* X, const typename Mod::Word* Y, uint64_t n,
                        hipStream_t st) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const auto T = tables_of<Word>(ctx);
    const Plan P = make_plan(ctx, n);
    if (P.kind < 0) return TFT_ERANGE;
    if (P.kind == 0) {
        if (Y) launch(ctx, TFT_K_POINTWISE, tft::k_pointwise<Mod>, dim3(1), dim3(kThreads), 0, st, md, X, Y, n);
        launch(ctx, TFT_K_SMALL_INV, tft::k_small_inv<Mod>, dim3(1), dim3(kThreads), P.lds_row, st, md, T, X, (uint32_t)n,
                           P.M);
        return launch_status();
    }
    Word* V = reinterpret_cast<Word*>(ctx->scratch);
    const uint32_t C = 1u << P.logC;
    const uint32_t tiles_all = (uint32_t)(P.W >> P.logC);
    tft::PieceList pieces{};
    pieces.count = P.b ? tft::gitft_pieces((uint32_t)P.W, (uint32_t)P.b, P.a, pieces.p) : 0;
    launch(ctx, TFT_K_ROW_INV, tft::k_row_inv<Mod>, dim3((uint32_t)P.a + pieces.count), dim3(kThreads), P.lds_row, st,
           md, T, X, Y, P.logW, (uint32_t)P.a, pieces);
    // columns c >= b
    {
        const uint32_t t0 = (uint32_t)(P.b / C);
        const uint32_t nt = tiles_all - t0;
        auto kern = P.logC == 3 ? tft::k_col_inv<Mod, 3> : tft::k_col_inv<Mod, 4>;
        launch(ctx, TFT_K_COL_INV_SHORT, kern, dim3(nt), dim3(kThreads), P.lds_col, st, md, T, X, P.logW,
               (uint32_t)P.a, (uint32_t)P.b, P.M, V, 0, t0, nt);
    }
    if (P.b) {
        launch(ctx, TFT_K_LAST_INV, tft::k_last_inv<Mod>, dim3(1), dim3(kThreads), P.lds_row, st, md, T, X, P.logW,
               (uint32_t)P.a, (uint32_t)P.b, (const Word*)V);
        const uint32_t nt = (uint32_t)((P.b + C - 1) / C);
        auto kern = P.logC == 3 ? tft::k_col_inv<Mod, 3> : tft::k_col_inv<Mod, 4>;
        launch(ctx, TFT_K_COL_INV_LONG, kern, dim3(nt), dim3(kThreads), P.lds_col, st, md, T, X, P.logW,
               (uint32_t)P.a, (uint32_t)P.b, P.M, V, 1, 0u, nt);
    }
    return launch_status();
}

template <class Mod>
tft_status pointwise_impl(tft_ctx* ctx, typename Mod::Word* X, const typename Mod::Word* Y, uint64_t n,
                          hipStream_t st) {
    const Mod& md = mod_of<Mod>(ctx);
    uint64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    launch(ctx, TFT_K_POINTWISE, tft::k_pointwise<Mod>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, md, X, Y, n);
    return launch_status();
}

template <class Mod>
tft_status mul_impl(tft_ctx* ctx, const typename Mod::Word* A, uint64_t m, const typename Mod::Word* B, uint64_t nb,
                    typename Mod::Word* X, typename Mod::Word* Y, hipStream_t st) {
    const uint64_t r = m + nb - 1;
    const Plan P = make_plan(ctx, r);
    if (P.kind < 0) return TFT_ERANGE;
    if (P.kind == 0 && 2 * P.lds_row <= kLdsHard - 32 * 1024) {
        const Mod& md = mod_of<Mod>(ctx);
        const auto T = tables_of<typename Mod::Word>(ctx);
        launch(ctx, TFT_K_SMALL_MUL, tft::k_small_mul<Mod>, dim3(1), dim3(kThreads), 2 * P.lds_row, st, md, T, A, (uint32_t)m,
                           B, (uint32_t)nb, X, P.M);
        return launch_status();
    }
    if (!Y) return TFT_EINVAL;
    tft_status s = forward_impl<Mod>(ctx, A, m, X, r, st);
    if (s != TFT_OK) return s;
    s = forward_impl<Mod>(ctx, B, nb, Y, r, st);
    if (s != TFT_OK) return s;
    return inverse_impl<Mod>(ctx, X, Y, r, st);
}

template <class Mod>
tft_status padded_forward_impl(tft_ctx* ctx, typename Mod::Word* X, uint64_t n, typename Mod::Word* Xp,
                               hipStream_t st) {
    using Word = typename Mod::Word;
    const uint64_t N = pow2ceil(n);
    uint64_t blocks = (N + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, Xp, N, (const Word*)X, n);
    tft_status s = forward_impl<Mod>(ctx, Xp, N, Xp, N, st);
    if (s != TFT_OK) return s;
    blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, X, n, (const Word*)Xp, n);
    return launch_status();
}

template <class Mod>
tft_status padded_inverse_impl(tft_ctx* ctx, typename Mod::Word* X, uint64_t n, typename Mod::Word* Xp,
                               hipStream_t st) {
    using Word = typename Mod::Word;
    const uint64_t N = pow2ceil(n);
    tft_status s = inverse_impl<Mod>(ctx, Xp, nullptr, N, st);
    if (s != TFT_OK) return s;
    uint64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, X, n, (const Word*)Xp, n);
    return launch_status();
}

template <class Mod>
tft_status padded_mul_impl(tft_ctx* ctx, const typename Mod::Word* A, uint64_t m, const typename Mod::Word* B,
                           uint64_t nb, typename Mod::Word* X, typename Mod::Word* Ap, typename Mod::Word* Bp,
                           hipStream_t st) {
    using Word = typename Mod::Word;
    const uint64_t r = m + nb - 1;
    const uint64_t N = pow2ceil(r);
    uint64_t blocks = (N + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, Ap, N, A, m);
    launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, Bp, N, B, nb);
    tft_status s = forward_impl<Mod>(ctx, Ap, N, Ap, N, st);
    if (s == TFT_OK) s = forward_impl<Mod>(ctx, Bp, N, Bp, N, st);
    if (s == TFT_OK) s = inverse_impl<Mod>(ctx, Ap, Bp, N, st);
    if (s != TFT_OK) return s;
    blocks = (r + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, X, r, (const Word*)Ap, r);
    return launch_status();
}

// -------------------------------------------------------------- tables
template <class Word>
std::vector<Word> build_tables(uint64_t p, uint64_t g, unsigned v, size_t n1, size_t n2, bool montgomery) {
    // f1[s] = w_s (s < n1), f2[h] = w_{h 2^B1} (h < n2), i1[s] = w_s^-1, i2[h] = w_{h 2^B1}^-1
    std::vector<Word> out(2 * (n1 + n2), Word(0));
    auto root = [&](unsigned k) { return powmod_h(g, (p - 1) >> k, p); };
    auto enc = [&](uint64_t x) -> Word {
        return montgomery ? (Word)(((u128)x << 32) % p) : (Word)x;
    };
    const unsigned k1 = v < (unsigned)kB1 ? v : (unsigned)kB1;
    const uint64_t lim1 = 1ull << k1;
    {
        // w_s = w[k1]^(rev_k1 s): walk powers of w[k1]
        std::vector<uint64_t> pw(lim1);
        const uint64_t r = root(k1);
        uint64_t x = 1;
        for (uint64_t e = 0; e < lim1; e++) { pw[e] = x; x = mulmod_h(x, r, p); }
        for (uint64_t s = 0; s < lim1; s++) {
            const uint64_t w = pw[rev_bits(s, k1)];
            out[s] = enc(w);
            out[n1 + n2 + s] = enc(powmod_h(w, p - 2, p));
        }
    }
    if (n2 > 1) {
        const unsigned k2 = log2u(n2);           // w_{h 2^B1} = w[B1+k2]^(rev_k2 h)
        std::vector<uint64_t> pw(n2);
        const uint64_t r = root(kB1 + k2);
        uint64_t x = 1;
        for (uint64_t e = 0; e < n2; e++) { pw[e] = x; x = mulmod_h(x, r, p); }
        for (uint64_t h = 0; h < n2; h++) {
            const uint64_t w = pw[rev_bits(h, k2)];
            out[n1 + h] = enc(w);
            out[2 * n1 + n2 + h] = enc(powmod_h(w, p - 2, p));
        }
    } else {
        out[n1] = enc(1);
        out[2 * n1 + n2] = enc(1);
    }
    return out;
}

bool is_probable_prime(uint64_t n) {
    if (n < 2) return false;
    for (uint64_t q : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        if (n % q == 0) return n == q;
    }
    uint64_t d = n - 1;
    unsigned s = 0;
    while (!(d & 1)) { d >>= 1; s++; }
    for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        uint64_t x = powmod_h(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (unsigned r = 1; r < s; r++) {
            x = mulmod_h(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

template <class F>
tft_status dispatch(tft_ctx* ctx, F&& f) {
    if (!ctx) return TFT_EINVAL;
    DeviceGuard guard(ctx->device);
    return f();
}

}  // namespace

// ============================================================== C entry points
extern "C" {

const char* tft_strerror(tft_status s) {
    switch (s) {
        case TFT_OK: return "ok";
        case TFT_EINVAL: return "invalid argument";
        case TFT_ERANGE: return "length or prime out of range";
        case TFT_ENOMEM: return "out of memory";
        case TFT_EDEVICE: return "device error";
        case TFT_EAGAIN: return "queue full, try again";
    }
    return "unknown status";
}

tft_status tft_ctx_create(uint64_t p, uint64_t g, int device, tft_ctx** out) {
    if (!out) return TFT_EINVAL;
    *out = nullptr;
    const bool wide = (p == kGoldilocks);
    if (!wide && (p >= (1ull << 31) || p < 3 || !(p & 1) || !is_probable_prime(p))) return TFT_ERANGE;
    unsigned v = 0;
    while (!(((p - 1) >> v) & 1)) v++;
    if (v < 1) return TFT_ERANGE;
    if (g % p == 0 || powmod_h(g, (p - 1) / 2, p) != p - 1) return TFT_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TFT_EDEVICE;
    tft_ctx* c = new (std::nothrow) tft_ctx();
    if (!c) return TFT_ENOMEM;
    c->device = device;
    c->p = p;
    c->g = g;
    c->v = v < kMaxLog2 ? v : kMaxLog2;
    c->wbytes = wide ? 8 : 4;
    c->override_logW = 0;
    c->timing = false;
    for (int i = 0; i < TFT_K_COUNT; i++) { c->launches[i] = 0; c->total_ms[i] = 0.0; }
    if (!wide) {
        uint32_t inv = 1;                          // p^-1 mod 2^32 by Newton iteration
        for (int i = 0; i < 5; i++) inv *= 2u - (uint32_t)p * inv;
        c->m32.p = (uint32_t)p;
        c->m32.pneg = (uint32_t)(0u - inv);
        c->m32.r2 = (uint32_t)(((u128)1 << 64) % p);
        c->m32.halfp1 = (uint32_t)((p + 1) / 2);
    }
    c->n1 = size_t(1) << kB1;
    c->n2 = c->v > (unsigned)kB1 ? size_t(1) << (c->v - kB1) : 1;
    DeviceGuard guard(device);
    size_t bytes = 0;
    hipError_t e;
    if (wide) {
        auto t = build_tables<uint64_t>(p, g, c->v, c->n1, c->n2, false);
        bytes = t.size() * 8;
        e = hipMalloc(&c->tables, bytes);
        if (e == hipSuccess) e = hipMemcpy(c->tables, t.data(), bytes, hipMemcpyHostToDevice);
        set_lds_limits<tft::ModGL>();
    } else {
        auto t = build_tables<uint32_t>(p, g, c->v, c->n1, c->n2, true);
        bytes = t.size() * 4;
        e = hipMalloc(&c->tables, bytes);
        if (e == hipSuccess) e = hipMemcpy(c->tables, t.data(), bytes, hipMemcpyHostToDevice);
        set_lds_limits<tft::ModU32>();
    }
    if (e == hipSuccess) e = hipMalloc(&c->scratch, kScratchWords * c->wbytes);
    if (e != hipSuccess) {
        if (c->tables) (void)hipFree(c->tables);
        delete c;
        return e == hipErrorOutOfMemory ? TFT_ENOMEM : TFT_EDEVICE;
    }
    *out = c;
    return TFT_OK;
}

void tft_ctx_destroy(tft_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard guard(ctx->device);
    (void)hipFree(ctx->tables);
    (void)hipFree(ctx->scratch);
    for (auto& r : ctx->recs) { (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
}

unsigned tft_ctx_max_log2(const tft_ctx* ctx) { return ctx ? ctx->v : 0; }
unsigned tft_ctx_word_bytes(const tft_ctx* ctx) { return ctx ? ctx->wbytes : 0; }

static tft_status check_len(const tft_ctx* ctx, size_t n) {
    if (n == 0) return TFT_EINVAL;
    if (log2u(n) > ctx->v) return TFT_ERANGE;
    return TFT_OK;
}

tft_status tft_forward(tft_ctx* ctx, void* X, size_t n, void* stream) {
    if (!ctx || !X) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&] {
        if (ctx->wbytes == 4) {
            auto* x = (uint32_t*)X;
            return forward_impl<tft::ModU32>(ctx, x, n, x, n, st);
        }
        auto* x = (uint64_t*)X;
        return forward_impl<tft::ModGL>(ctx, x, n, x, n, st);
    });
}

tft_status tft_inverse(tft_ctx* ctx, void* X, size_t n, void* stream) {
    if (!ctx || !X) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&] {
        if (ctx->wbytes == 4) return inverse_impl<tft::ModU32>(ctx, (uint32_t*)X, nullptr, n, st);
        return inverse_impl<tft::ModGL>(ctx, (uint64_t*)X, nullptr, n, st);
    });
}

tft_status tft_pointwise_mul(tft_ctx* ctx, void* X, const void* Y, size_t n, void* stream) {
    if (!ctx || !X || !Y || n == 0) return TFT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&] {
        if (ctx->wbytes == 4) return pointwise_impl<tft::ModU32>(ctx, (uint32_t*)X, (const uint32_t*)Y, n, st);
        return pointwise_impl<tft::ModGL>(ctx, (uint64_t*)X, (const uint64_t*)Y, n, st);
    });
}

tft_status poly_mul(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X, void* Y, void* stream) {
    if (!ctx || !A || !B || !X || m == 0 || nb == 0) return TFT_EINVAL;
    tft_status s = check_len(ctx, m + nb - 1);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&] {
        if (ctx->wbytes == 4)
            return mul_impl<tft::ModU32>(ctx, (const uint32_t*)A, m, (const uint32_t*)B, nb, (uint32_t*)X, (uint32_t*)Y,
                                         st);
        return mul_impl<tft::ModGL>(ctx, (const uint64_t*)A, m, (const uint64_t*)B, nb, (uint64_t*)X, (uint64_t*)Y, st);
    });
}

tft_status tft_padded_forward(tft_ctx* ctx, void* X, size_t n, void* Xpad, void* stream) {
    if (!ctx || !X || !Xpad) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&] {
        if (ctx->wbytes == 4) return padded_forward_impl<tft::ModU32>(ctx, (uint32_t*)X, n, (uint32_t*)Xpad, st);
        return padded_forward_impl<tft::ModGL>(ctx, (uint64_t*)X, n, (uint64_t*)Xpad, st);
    });
}

tft_status tft_padded_inverse(tft_ctx* ctx, void* X, size_t n, void* Xpad, void* stream) {
    if (!ctx || !X || !Xpad) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&] {
        if (ctx->wbytes == 4) return padded_inverse_impl<tft::ModU32>(ctx, (uint32_t*)X, n, (uint32_t*)Xpad, st);
        return padded_inverse_impl<tft::ModGL>(ctx, (uint64_t*)X, n, (uint64_t*)Xpad, st);
    });
}

tft_status poly_mul_padded(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X, void* Apad,
                           void* Bpad, void* stream) {
    if (!ctx || !A || !B || !X || !Apad || !Bpad || m == 0 || nb == 0) return TFT_EINVAL;
    tft_status s = check_len(ctx, m + nb - 1);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&] {
        if (ctx->wbytes == 4)
            return padded_mul_impl<tft::ModU32>(ctx, (const uint32_t*)A, m, (const uint32_t*)B, nb, (uint32_t*)X,
                                                (uint32_t*)Apad, (uint32_t*)Bpad, st);
        return padded_mul_impl<tft::ModGL>(ctx, (const uint64_t*)A, m, (const uint64_t*)B, nb, (uint64_t*)X,
                                           (uint64_t*)Apad, (uint64_t*)Bpad, st);
    });
}

tft_status tft_plan_info(tft_ctx* ctx, size_t n, tft_plan_desc* out) {
    if (!ctx || !out || n == 0) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    const Plan P = make_plan(ctx, n);
    if (P.kind < 0) return TFT_ERANGE;
    std::memset(out, 0, sizeof(*out));
    out->kind = P.kind;
    out->logW = P.logW;
    out->W = P.W;
    out->a = P.a;
    out->b = P.b;
    out->col_block = P.M;
    out->cols_per_tile = P.kind == 1 ? (1u << P.logC) : 0;
    out->lds_bytes_col = P.lds_col;
    out->lds_bytes_row = P.lds_row;
    return TFT_OK;
}

tft_status tft_set_plan_override(tft_ctx* ctx, unsigned logW) {
    if (!ctx || logW > 16) return TFT_EINVAL;
    ctx->override_logW = logW;
    return TFT_OK;
}

tft_status tft_timing_enable(tft_ctx* ctx, int on) {
    if (!ctx) return TFT_EINVAL;
    ctx->timing = on != 0;
    return TFT_OK;
}

static tft_status timing_collect(tft_ctx* ctx) {
    tft_status s = TFT_OK;
    for (auto& r : ctx->recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
            s = TFT_EDEVICE;
        ctx->launches[r.kid] += 1;
        ctx->total_ms[r.kid] += ms;
        ctx->pool.push_back(r.e0);
        ctx->pool.push_back(r.e1);
    }
    ctx->recs.clear();
    return s;
}

tft_status tft_timing_read(tft_ctx* ctx, int id, uint64_t* launches, double* total_ms) {
    if (!ctx || id < 0 || id >= TFT_K_COUNT || !launches || !total_ms) return TFT_EINVAL;
    DeviceGuard guard(ctx->device);
    tft_status s = timing_collect(ctx);
    *launches = ctx->launches[id];
    *total_ms = ctx->total_ms[id];
    return s;
}

tft_status tft_timing_reset(tft_ctx* ctx) {
    if (!ctx) return TFT_EINVAL;
    DeviceGuard guard(ctx->device);
    tft_status s = timing_collect(ctx);
    for (int i = 0; i < TFT_K_COUNT; i++) { ctx->launches[i] = 0; ctx->total_ms[i] = 0.0; }
    return s;
}

const char* tft_kernel_name(int id) {
    static const char* names[TFT_K_COUNT] = {"small_fwd", "small_inv", "small_mul", "col_fwd", "row_fwd",
                                             "row_inv", "col_inv_short", "last_inv", "col_inv_long",
                                             "pointwise", "copy_pad"};
    return (id >= 0 && id < TFT_K_COUNT) ? names[id] : "unknown";
}

}  // extern "C"
