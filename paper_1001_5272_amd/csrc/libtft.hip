// Host side of libtft: contexts (prime, roots, tables), the planner that picks
// the schedule for a length n, and the C entry points declared in
// include/libtft.h.  All device work is in tft_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <type_traits>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "libtft.h"
#include "tft_kernels.hpp"
#include "tft_calib.hpp"

using tft::kB1;
using tft::kThreads;

// Workspace of poly_mul_noalloc: B's transform (the r words that poly_mul takes
// from the caller) lives in this fixed device array instead.  Every device the
// library runs on holds its own copy from module load until the process ends.
// In host code the name is only a handle: the array's address on a device
// comes from hipGetSymbolAddress with that device current (noalloc_setup).
constexpr size_t kNoAllocBytes = size_t(32) << 20;   // 32 MiB: 2^22 words of 8 bytes, 2^23 of 4
static __device__ __align__(256) uint64_t scratch[kNoAllocBytes / 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
std::atomic<void*> g_noalloc_ptr[kMaxDevices];

// Once per device, with that device current: the device address of scratch.
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipSuccess;   // poly_mul_noalloc reports TFT_EDEVICE
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device].load(std::memory_order_acquire)) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[device].store(ptr, std::memory_order_release);
    return hipSuccess;
}
}  // namespace

namespace {

constexpr uint64_t kGoldilocks = 0xFFFFFFFF00000001ull;
constexpr unsigned kMaxLog2 = 28;               // longest transform supported by the tables
// plan cache: quarter octaves of n, then one slot per power of two
constexpr unsigned kPow2Buckets = 4 * kMaxLog2 + 4;
constexpr unsigned kPlanBuckets = kPow2Buckets + kMaxLog2 + 1;
constexpr size_t kVWords = size_t(1) << 16;          // V_c area: one word per column, W <= 2^16
// V_c area, then the column polynomial Q of the general last-row step (two
// buffers of kQStride words and 1 / Q(w_a))
constexpr size_t kScratchWords = kVWords + 2 * size_t(tft::kQStride) + 64;
// the space-restricted product's fold partials: two areas of kFoldItems words
// (about that many threads per operand read it at once), then kFoldSpare words
// for sums of spans
constexpr size_t kFoldItems = size_t(1) << 18;
constexpr size_t kFoldSpare = size_t(1) << 10;
// the restricted product's last positions (fewer than 2^(kRestrLog + 1)) come
// from node folds of at most 2^kRestrLog words, four of them (two nodes, two
// operands) after the partials in the fold area
constexpr unsigned kRestrLog = 17;
constexpr size_t kFoldWords = 2 * kFoldItems + kFoldSpare + (size_t(4) << kRestrLog);
constexpr size_t kLdsSoft = 76 * 1024;          // preferred LDS per workgroup (two per CU)
constexpr size_t kLdsHard = 160 * 1024;         // gfx950 LDS per workgroup
constexpr size_t kLdsDynMax = 144 * 1024;       // dynamic LDS any launch may request
constexpr uint32_t kRowMulThreads = 128;          // fused row-product workgroups of a batch (at least)
constexpr int kBigJobThreads = 1024;              // single-workgroup batch jobs alone on a CU
constexpr uint32_t kListColThreads = 128;         // column-list workgroups of a standalone batch (at most)
constexpr uint64_t kFewColumns = 128;   // classes this narrow run one column per workgroup

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
    uint32_t split;      // kind 1: Lout = M + 1, the column block holds M words (see col_fwd_body)
    int logC;            // columns per tile 2^logC
    unsigned rlog;       // words per row thread 2^rlog (one or two radix-8 units)
    unsigned smax;       // most stages per LDS round trip
    unsigned ldstw;      // column tiles copy their twiddles to LDS (1) or read them from memory (0)
    unsigned hs;         // column transforms may split at a power of two (single transforms; not batches)
    size_t lds_col, lds_row;
};

// A tuned plan as one word (the plan cache's entries): bits 0-4 log2 W
// (0: the planner's width), bits 5-7 log2 columns per tile, bits 8-10 log2
// words per row thread, bits 11-12 stages per LDS round trip (0 in a field:
// the default).
struct PlanCode {
    unsigned logW, logC, rlog, smax;
};
inline PlanCode decode_plan(unsigned code) {
    return PlanCode{code & 31u, (code >> 5) & 7u, (code >> 8) & 7u, (code >> 11) & 3u};
}
inline unsigned encode_plan(const PlanCode& c) {
    return (c.logW & 31u) | ((c.logC & 7u) << 5) | ((c.rlog & 7u) << 8) | ((c.smax & 3u) << 11);
}

}  // namespace

// Memory and streams that consecutive batches reuse (each slot of the serving
// queue, the convenience batch calls): a device area and a pinned host
// staging area that grow geometrically and are kept, so that a batch in steady
// state allocates nothing, uploads its work lists with an asynchronous copy on
// its own stream and never waits on a free.  One batch at a time uses an
// arena, and only once the batch before it has finished on the device.
struct BatchArena {
    void* dmem = nullptr;
    size_t dcap = 0;
    void* hmem = nullptr;   // pinned
    size_t hcap = 0;
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, done = nullptr;
};

struct tft_ctx {
    int device;
    uint64_t p, g;
    unsigned v;          // usable log2 length
    unsigned wbytes;     // 4 or 8
    // plan state, read by every caller's thread and the serving queue's worker
    std::atomic<unsigned> override_logW;
    std::atomic<unsigned> tuned_logW[kPlanBuckets];   // plan cache by floor(4 lg n): plan codes, 0 = planner's choice
    std::atomic<unsigned> batch_widen;                // batches: rows this many steps wider than balanced (0..2)
    std::atomic<unsigned> batch_col_thr;              // standalone batches: column-list workgroup size (at most)
    std::atomic<unsigned> batch_rowmul_thr;           // and fused row-product workgroup size (at least)
    tft::ModU32 m32;
    tft::ModGL m64;
    tft::ModM64 mm64;    // 8-byte words, p other than 2^64 - 2^32 + 1
    void* tables;        // f1 | f2 | i1 | i2
    size_t n1, n2;       // entries per level
    void* varea;         // V_c area and column polynomial (kScratchWords words)
    void* fold;          // the space-restricted product's fold partials and node folds (kFoldWords words)
    // measurement mode (tft_timing_*): events bracketing each launch of the
    // kernels selected in timing_mask (bit = tft_kernel_id)
    std::atomic<bool> timing;
    std::atomic<uint32_t> timing_mask;
    std::mutex timing_mu;   // recs, pool, launches, total_ms (launches from several threads)
    struct Rec { int kid; hipEvent_t e0, e1; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    uint64_t launches[TFT_K_COUNT];
    double total_ms[TFT_K_COUNT];
    struct tft_batch* last_batch;   // kept alive for the convenience batch calls
    hipEvent_t last_done;
    BatchArena once_arena;          // reused by the convenience batch calls
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
    if (!(ctx->timing.load(std::memory_order_relaxed) && ((ctx->timing_mask.load(std::memory_order_relaxed) >> kid) & 1u))) {
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
        return;
    }
    std::lock_guard<std::mutex> lk(ctx->timing_mu);
    hipEvent_t e0 = take_event(ctx), e1 = take_event(ctx);
    if (e0 && e1) (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
    if (e0 && e1) {
        (void)hipEventRecord(e1, st);
        ctx->recs.push_back({kid, e0, e1});
    } else {
        if (e0) ctx->pool.push_back(e0);
        if (e1) ctx->pool.push_back(e1);
    }
}

unsigned small_max_log2(unsigned wbytes) { return wbytes == 4 ? 13 : 12; }

// Plan-cache bucket of a length: floor(4 lg n) (quarter octaves), exactly;
// a power of two 2^e has a slot of its own, kPow2Buckets + e: with b = 0 its
// passes have no partial last row, and the plan that suits it is not the one
// that suits the truncated lengths just above it.
unsigned plan_bucket(uint64_t n) {
    const unsigned e = 63u - (unsigned)__builtin_clzll(n);
    if ((n & (n - 1)) == 0) return kPow2Buckets + e;
    const u128 n4 = (u128)n * n * n * n;
    unsigned j = 0;
    while (j < 3 && n4 >= ((u128)1 << (4 * e + j + 1))) j++;
    return 4 * e + j;
}

// Columns per tile, 2^logC: a tile row is one 64-byte segment (16 words of 4
// bytes, 8 of 8 bytes).  Narrower tiles (4 words of 8 bytes) fit more tiles on
// a CU but measured slower: half-used segments and no gain in occupancy, which
// the column kernels' registers already bound.
constexpr int col_log_width(unsigned w) { return w == 4 ? 4 : 3; }

// Column-tile kernels by tile width (2^3 or 2^4 columns) and by whether the
// columns of the launch split at a power of two (tft::col_split): the split
// is a separate instantiation so that the other launches keep the registers
// (and occupancy) of the plain column transform.
template <class Mod>
auto col_fwd_kernel(int logC, bool hs) {
    if (hs) return logC == 3 ? tft::k_col_fwd<Mod, 3, true> : tft::k_col_fwd<Mod, 4, true>;
    return logC == 3 ? tft::k_col_fwd<Mod, 3, false> : tft::k_col_fwd<Mod, 4, false>;
}
template <class Mod>
auto col_inv_kernel(int logC, bool hs) {
    if (hs) return logC == 3 ? tft::k_col_inv<Mod, 3, true> : tft::k_col_inv<Mod, 4, true>;
    return logC == 3 ? tft::k_col_inv<Mod, 3, false> : tft::k_col_inv<Mod, 4, false>;
}
template <class Mod>
auto col_fwd_list_kernel(int logC) {
    return logC == 3 ? tft::k_col_fwd_list<Mod, 3> : tft::k_col_fwd_list<Mod, 4>;
}
template <class Mod>
auto col_inv_list_kernel(int logC) {
    return logC == 3 ? tft::k_col_inv_list<Mod, 3> : tft::k_col_inv_list<Mod, 4>;
}

// wide: prefer rows one step wider than the balanced split (W = 2^(floor(k/2)+1)
// rather than 2^floor(k/2) at k = floor(lg n) even); the batches use it: with
// longer rows and shorter columns their many small column tiles each finish
// sooner (a batch of 4096 products with lengths up to 2^16 measured 20 %
// faster).
// LDS of a column tile (data and one twiddle table) for len values, as the
// kernels lay it out: the forward (len = Lout) and the inverse of a class of
// len values split at H when tft::col_split allows (H + S words per column),
// else use the power-of-two block (the forward P.M; the inverse 2^ceil(lg len),
// or P.M for the split mode's long class).
// The forward's columns (Lout values) split at a power of two; the kernels
// take the same decision (col_fwd_body, with the split instantiation).
bool fwd_splits(const Plan& P, uint32_t* H, uint32_t* S) {
    return P.hs && !P.split && P.Lout != P.M && tft::col_split(P.Lout, H, S);
}
// The inverse's class of len values splits at a power of two (col_inv_body).
bool inv_splits(const Plan& P, uint32_t len, uint32_t* H, uint32_t* S) {
    const bool top = P.split && len == P.M + 1;
    return P.hs && !top && len != pow2ceil(len) && tft::col_split(len, H, S);
}
bool inv_splits(const Plan& P, uint32_t len) {
    uint32_t H, S;
    return inv_splits(P, len, &H, &S);
}

size_t col_tile_lds(const Plan& P, uint32_t len, bool fwd, unsigned w) {
    uint32_t H = 0, S = 0;
    uint32_t blk;
    const uint32_t tw = P.ldstw ? 1u : 0u;
    if (fwd ? fwd_splits(P, &H, &S) : inv_splits(P, len, &H, &S))
        return ((size_t)tft::padded_words((H + S) << P.logC) + tw * (H / 2)) * w;
    if (fwd) {
        blk = P.M;
    } else {
        const bool top = P.split && len == P.M + 1;
        blk = top ? P.M : (uint32_t)pow2ceil(len);
    }
    return ((size_t)tft::padded_words(blk << P.logC) + tw * (blk / 2)) * w;
}

// The autotuner times candidate widths on its own thread: a width forced here
// applies to that thread's calls only, so other threads (the serving queue's
// worker, other callers) keep planning from the context's state meanwhile.
thread_local unsigned tl_force_code = 0;      // 0: none
thread_local bool tl_ignore_cache = false;   // plan without the tuned widths
thread_local int tl_batch_widen = -1;        // the batch tuner's candidate (-1: the context's setting)
thread_local int tl_batch_col_thr = -1;      // its thread-count candidates (-1: the context's settings)
thread_local int tl_batch_rowmul_thr = -1;

Plan make_plan(const tft_ctx* ctx, uint64_t n, bool wide = false) {
    Plan P{};
    P.n = n;
    const unsigned w = ctx->wbytes;
    const PlanCode force = decode_plan(tl_force_code);
    const unsigned ovr = force.logW ? force.logW
                                    : (tl_ignore_cache ? 0u : ctx->override_logW.load(std::memory_order_relaxed));
    P.smax = 3;
    P.rlog = 3;
    P.hs = wide ? 0 : 1;
    if (log2u(n) <= small_max_log2(w) && !(ovr && (1ull << ovr) < n)) {
        P.kind = 0;
        P.M = (uint32_t)pow2ceil(n);
        P.lds_row = (size_t)tft::padded_words(P.M) * w;   // data tile; the kernels add M words of twiddles
        return P;
    }
    P.kind = 1;
    P.logC = col_log_width(w);
    // tile width, row threads and stages of a forced or tuned plan (single
    // transforms only: a batch shares one tile width and one launch shape)
    auto knobs = [&](const PlanCode& c) {
        if (wide) return;
        if (c.logC == 3 || c.logC == 4) P.logC = (int)c.logC;
        if (c.rlog == 3 || c.rlog == 4) P.rlog = c.rlog;
        if (c.smax >= 1 && c.smax <= 3) P.smax = c.smax;
    };
    knobs(force);
    auto fill = [&](unsigned logW) {
        P.logW = logW;
        P.W = 1ull << logW;
        P.a = n >> logW;
        P.b = n & (P.W - 1);
        P.Lout = (uint32_t)(P.a + (P.b ? 1 : 0));
        P.M = (uint32_t)pow2ceil(P.Lout);
        P.split = (P.M >= 4 && P.Lout == P.M / 2 + 1) ? 1 : 0;
        if (P.split) P.M /= 2;
        // the largest column tile of the forward and of both inverse classes;
        // the twiddle copy is left out when two tiles per CU fit only without it
        auto tile = [&]() {
            size_t l = col_tile_lds(P, P.Lout, true, w);
            if (P.a) l = std::max(l, col_tile_lds(P, (uint32_t)P.a, false, w));
            if (P.b) l = std::max(l, col_tile_lds(P, (uint32_t)P.a + 1, false, w));
            return l;
        };
        P.ldstw = 1;
        P.lds_col = tile();
        if (P.lds_col > kLdsSoft) {
            P.ldstw = 0;
            const size_t bare = tile();
            if (bare <= kLdsSoft) P.lds_col = bare;
            else P.ldstw = 1;
        }
        P.lds_row = (size_t)tft::padded_words((uint32_t)P.W) * w;
    };
    const unsigned logC = (unsigned)P.logC;
    if (ovr) {
        fill(ovr);
        if (P.W < (1ull << logC) || P.a < 1 || P.lds_col > kLdsDynMax || P.lds_row > kLdsDynMax) P.kind = -1;
        return P;
    }
    const unsigned k = log2u(n);
    const unsigned bk = plan_bucket(n);
    const PlanCode tuned = decode_plan((bk < kPlanBuckets && !tl_ignore_cache && !wide && !tl_force_code)
                                           ? ctx->tuned_logW[bk].load(std::memory_order_relaxed) : 0u);
    if (tuned.logW && (1ull << tuned.logW) < n) {   // tft_autotune
        const int logC0 = P.logC;
        knobs(tuned);
        fill(tuned.logW);
        if (P.W >= (1ull << P.logC) && P.a >= 1 && P.lds_col <= kLdsDynMax && P.lds_row <= kLdsDynMax) return P;
        P.logC = logC0;
        P.rlog = 3;
        P.smax = 3;
    }
    // balanced split: W close to sqrt(n), within the LDS budget (preferred
    // budget first, then the larger one)
    for (size_t lim : {kLdsSoft, kLdsDynMax}) {
        int best = -1;
        for (unsigned logW = logC; logW <= 16 && (1ull << logW) < n; logW++) {
            fill(logW);
            if (P.lds_col > lim || P.lds_row > lim) continue;
            const int widen = !wide ? 0
                              : tl_batch_widen >= 0 ? tl_batch_widen : (int)ctx->batch_widen.load(std::memory_order_relaxed);
            const int t = (int)k + widen;
            if (best < 0 || std::abs(2 * (int)logW - t) <= std::abs(2 * best - t)) best = (int)logW;
        }
        if (best >= 0) {
            fill((unsigned)best);
            return P;
        }
    }
    P.kind = -1;   // beyond the two-pass limit of the library
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
    T.K = ctx->v;
    return T;
}

template <class Mod>
const Mod& mod_of(const tft_ctx* ctx);
template <>
const tft::ModU32& mod_of<tft::ModU32>(const tft_ctx* ctx) { return ctx->m32; }
template <>
const tft::ModGL& mod_of<tft::ModGL>(const tft_ctx* ctx) { return ctx->m64; }
template <>
const tft::ModM64& mod_of<tft::ModM64>(const tft_ctx* ctx) { return ctx->mm64; }

// Allow each kernel the dynamic LDS the planner may give it (the largest tile
// plus headroom, below the 160 KiB per workgroup minus static LDS).
template <class Mod>
bool set_lds_limits() {
    const int lim = (int)kLdsDynMax;
    const void* ks[] = {
        (const void*)tft::k_small_fwd<Mod>,       (const void*)tft::k_small_inv<Mod>,
        (const void*)tft::k_small_mul<Mod>,       (const void*)tft::k_small_list<Mod>,
        (const void*)tft::k_small_list<Mod, kBigJobThreads>,
        (const void*)tft::k_restr_tail<Mod>,
        (const void*)tft::k_col_fwd<Mod, 3>,      (const void*)tft::k_col_fwd<Mod, 4>,
        (const void*)tft::k_col_inv<Mod, 3>,      (const void*)tft::k_col_inv<Mod, 4>,
        (const void*)tft::k_col_fwd<Mod, 3, true>, (const void*)tft::k_col_fwd<Mod, 4, true>,
        (const void*)tft::k_col_inv<Mod, 3, true>, (const void*)tft::k_col_inv<Mod, 4, true>,
        (const void*)tft::k_col_inv<Mod, 0>,
        (const void*)tft::k_row_fwd<Mod>,         (const void*)tft::k_row_inv<Mod>,
        (const void*)tft::k_row_fwd_mul<Mod>,     (const void*)tft::k_row_fwd_mul_inv<Mod>,
        (const void*)tft::k_last_inv<Mod>,        (const void*)tft::k_tail_inv<Mod>,
        (const void*)tft::k_col_fwd_list<Mod, 3>,
        (const void*)tft::k_col_fwd_list<Mod, 4>, (const void*)tft::k_col_inv_list<Mod, 3>,
        (const void*)tft::k_col_inv_list<Mod, 4>, (const void*)tft::k_row_fwd_list<Mod>,
        (const void*)tft::k_row_inv_list<Mod>,    (const void*)tft::k_last_inv_list<Mod>,
        (const void*)tft::k_row_mul_list<Mod>,
    };
    for (const void* k : ks) {
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) return false;
    }
    return true;
}

// Threads of a row workgroup: one radix-8 unit per thread (W / 8, 64 ..
// 1024), so that idle threads of a wider workgroup do not hold wave slots.
uint32_t row_threads(const Plan& P) {
    return (uint32_t)std::min<uint64_t>(tft::kRowThreads, std::max<uint64_t>(64, P.W >> (P.rlog ? P.rlog : 3)));
}

// Threads of a column-tile workgroup: one radix-8 unit per thread (M C / 8,
// 64 .. kColThreads).
uint32_t col_threads(const Plan& P) {
    return (uint32_t)std::min<uint64_t>(tft::kColThreads, std::max<uint64_t>(64, ((uint64_t)P.M << P.logC) >> 3));
}

template <class Word>
tft::TwoPass<Word> two_pass_of(const Plan& P, Word* X, const Word* src, uint64_t n_src, const Word* Y, Word* V) {
    tft::TwoPass<Word> G;
    G.X = X;
    G.src = src;
    G.Y = Y;
    G.V = V;
    G.n_src = n_src;
    G.n = P.n;
    G.logW = P.logW;
    G.a = (uint32_t)P.a;
    G.b = (uint32_t)P.b;
    G.Lout = P.Lout;
    G.M = P.M;
    G.split = P.split;
    G.early = 0;
    G.Q = nullptr;
    G.g0 = 0;
    G.nparts = 0;
    G.ldstw = P.ldstw;
    G.inst = 0;
    return G;
}

// -------------------------------------------------------------- forward
template <class Mod>
// buffered (comparator): the extra evaluations of the partial last row go to
// X + a W, inside X's buffer of 2^ceil(lg n) words, instead of the context's
// area
// rows = false: the column pass only (the caller runs the rows; b = 0 or
// the product's one-short plans)
tft_status forward_impl(tft_ctx* ctx, const typename Mod::Word* src, uint64_t n_src, typename Mod::Word* X,
                        uint64_t n, hipStream_t st, uint64_t g0 = 0, uint32_t copies = 1,
                        bool buffered = false, bool rows = true) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const Plan P = make_plan(ctx, n);
    if (P.kind < 0) return TFT_ERANGE;
    auto T = tables_of<Word>(ctx);
    T.smax = P.smax;
    if (P.kind == 0) {
        if (src != X) {
            launch(ctx, TFT_K_COPY, tft::k_copy_pad<Word>, dim3(1), dim3(kThreads), 0, st, X, n, src, n_src);
        }
        launch(ctx, TFT_K_SMALL_FWD, tft::k_small_fwd<Mod>, dim3(copies), dim3(tft::kSmallThreads),
               P.lds_row + (size_t)P.M * ctx->wbytes, st, md, T, X, (uint32_t)n, P.M, g0, (uint64_t)n);
        return launch_status();
    }
    // a block at g0 != 0, and each of several instances, is a whole power-of-two block
    if ((g0 || copies > 1) && P.b) return TFT_EINVAL;
    Word* V = reinterpret_cast<Word*>(ctx->varea);
    auto G = two_pass_of<Word>(P, X, src, n_src, nullptr, buffered ? X + P.a * P.W : V);
    G.g0 = g0;
    G.inst = n;   // copies > 1: instance y at X + y n (src + y n), at the same block index
    const uint32_t tiles = (uint32_t)(P.W >> P.logC);
    // b = 1: the column tiles leave shares of the last row's one output
    // (scratch after V), and the row pass needs no workgroup for that row
    G.Q = V + kVWords;
    if (P.b == 1) G.nparts = tiles;
    uint32_t Hs, Ss;
    const bool hs = g0 == 0 && fwd_splits(P, &Hs, &Ss);
    if (!rows && P.b && !(P.b + 1 == P.W && !buffered && g0 == 0 && copies == 1)) return TFT_EINVAL;
    launch(ctx, TFT_K_COL_FWD, col_fwd_kernel<Mod>(P.logC, hs), dim3(tiles, copies), dim3(col_threads(P)), P.lds_col, st,
           md, T, G, tiles);
    if (rows)
        launch(ctx, TFT_K_ROW_FWD, tft::k_row_fwd<Mod>, dim3((uint32_t)(P.a + (P.b > 1 ? 1 : 0)), copies),
               dim3(row_threads(P)), P.lds_row, st, md, T, G);
    return launch_status();
}

// -------------------------------------------------------------- inverse
// b = W - 1 with a + 1 a power of two, rows of at least 64 words and the
// tail's LDS within the limit: the inverse's early mode 3 (k_tail_inv)
bool one_short_plan(const Plan& P, unsigned wbytes) {
    const bool full_long = P.b && ((P.a + 1) & P.a) == 0;
    const size_t lds_tail = ((size_t)tft::padded_words((uint32_t)P.a + 1) + (P.a + 1) / 2) * wbytes;
    return full_long && P.b + 1 == P.W && P.logW >= 6 && lds_tail <= kLdsDynMax;
}

template <class Mod>
// buffered (comparator): the extra evaluations live in X's buffer beyond n
// (X + a W, a buffer of 2^ceil(lg n) words) and the columns c < b wait for
// the last row (no early modes: those keep per-column values in the area too)
// rows = false: without the row pass (the caller ran it; b = 0 or early mode 3)
tft_status inverse_impl(tft_ctx* ctx, typename Mod::Word* X, const typename Mod::Word* Y, uint64_t n,
                        hipStream_t st, bool buffered = false, bool rows = true) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const Plan P = make_plan(ctx, n);
    if (P.kind < 0) return TFT_ERANGE;
    auto T = tables_of<Word>(ctx);
    T.smax = P.smax;
    if (P.kind == 0) {
        if (Y) launch(ctx, TFT_K_POINTWISE, tft::k_pointwise<Mod>, dim3(1), dim3(kThreads), 0, st, md, X, Y, n);
        launch(ctx, TFT_K_SMALL_INV, tft::k_small_inv<Mod>, dim3(1), dim3(tft::kSmallThreads), P.lds_row + (size_t)P.M * ctx->wbytes, st, md, T, X, (uint32_t)n,
                           P.M);
        return launch_status();
    }
    Word* V = reinterpret_cast<Word*>(ctx->varea);
    auto G = two_pass_of<Word>(P, X, X, n, Y, buffered ? X + P.a * P.W : V);
    // With b > 0 the columns c < b (a + 1 values) run with the columns c >= b on
    // their first a values and are finished after the last row: in split mode
    // by the last-row inverse alone (two coefficients change), otherwise by a
    // rank-one update with the column polynomial Q (k_col_fix).  When a + 1 is
    // a power of two the columns c < b are full inverses and the columns c >= b
    // the truncated ones, so the two classes keep their own passes.
    const bool full_long = P.b && ((P.a + 1) & P.a) == 0;
    // b = W - 1 as well: the one short column and the last row are full
    // inverses with one value missing (k_tail_inv), no truncated walks
    const size_t lds_tail = ((size_t)tft::padded_words((uint32_t)P.a + 1) + (P.a + 1) / 2) * ctx->wbytes;
    const bool one_short = !buffered && one_short_plan(P, ctx->wbytes);
    G.early = buffered ? 0u : one_short ? 3u : (P.b && !full_long) ? (P.split ? 1u : 2u) : 0u;
    G.Q = V + kVWords;
    const uint32_t C = 1u << P.logC;
    const uint32_t tiles_all = (uint32_t)(P.W >> P.logC);
    const uint32_t nrows = one_short ? (uint32_t)P.a + 1 : tft::row_inv_items((uint32_t)P.W, (uint32_t)P.a, (uint32_t)P.b);
    if (!rows && P.b && !one_short) return TFT_EINVAL;
    if (rows)
        launch(ctx, TFT_K_ROW_INV, tft::k_row_inv<Mod>, dim3(nrows + (G.early == 2 ? 1u : 0u)), dim3(row_threads(P)),
               P.lds_row, st, md, T, G, ctx->p);
    auto kern = [&](uint32_t len) { return col_inv_kernel<Mod>(P.logC, inv_splits(P, len)); };
    // LDS of a column tile inverting len values (as the kernel lays it out)
    auto col_lds = [&](uint32_t len) -> size_t { return col_tile_lds(P, len, false, ctx->wbytes); };
    if (one_short) {
        launch(ctx, TFT_K_LAST_INV, tft::k_tail_inv<Mod>, dim3(1), dim3(tft::kLastThreads), lds_tail, st, md, T, G);
        const uint32_t nt = (uint32_t)((P.b + C - 1) / C);   // columns c < b, in full
        launch(ctx, TFT_K_COL_INV_LONG, kern((uint32_t)P.a + 1), dim3(nt), dim3(col_threads(P)),
               col_lds((uint32_t)P.a + 1), st, md, T, G, 1, 0u, nt);
        return launch_status();
    }
    // A class with only a few columns runs one column per workgroup, so that a
    // tile does not transform C - 1 skipped columns on one CU.
    const size_t lds_one = ((size_t)tft::padded_words(P.M) + P.M) * ctx->wbytes;
    {   // columns c >= b (early modes: every column)
        const uint64_t ncols = G.early ? P.W : P.W - P.b;
        const uint32_t t0 = G.early ? 0u : (uint32_t)(P.b / C);
        if (ncols <= kFewColumns) {
            launch(ctx, TFT_K_COL_INV_SHORT, tft::k_col_inv<Mod, 0>, dim3((uint32_t)ncols), dim3(tft::kColThreads),
                   lds_one, st, md, T, G, 0, (uint32_t)(P.W - ncols), (uint32_t)ncols);
        } else {
            const uint32_t nt = tiles_all - t0;
            if (P.b == 1 && t0 == 0) G.nparts = nt;   // every tile leaves its share of the last-row sum
            launch(ctx, TFT_K_COL_INV_SHORT, kern((uint32_t)P.a), dim3(nt), dim3(col_threads(P)), col_lds((uint32_t)P.a),
                   st, md, T, G, 0, t0, nt);
        }
    }
    if (P.b) {
        launch(ctx, TFT_K_LAST_INV, tft::k_last_inv<Mod>, dim3(1), dim3(tft::kLastThreads), P.lds_row, st, md, T, G);
        if (G.early == 2) {
            const uint32_t gx = (uint32_t)((P.b + kThreads - 1) / kThreads);
            const uint32_t gy = (uint32_t)((P.a + tft::kFixRows - 1) / tft::kFixRows);
            launch(ctx, TFT_K_COL_FIX, tft::k_col_fix<Mod>, dim3(gx, gy), dim3(kThreads), 0, st, md, G);
        } else if (!G.early) {   // columns c < b, after the last row
            if (P.b <= kFewColumns) {
                launch(ctx, TFT_K_COL_INV_LONG, tft::k_col_inv<Mod, 0>, dim3((uint32_t)P.b), dim3(tft::kColThreads),
                       lds_one, st, md, T, G, 1, 0u, (uint32_t)P.b);
            } else {
                const uint32_t nt = (uint32_t)((P.b + C - 1) / C);
                launch(ctx, TFT_K_COL_INV_LONG, kern((uint32_t)P.a + 1), dim3(nt), dim3(col_threads(P)),
                       col_lds((uint32_t)P.a + 1), st, md, T, G, 1, 0u, nt);
            }
        }
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

// A product of length n = a W (b = 0, W >= 64), or with the one-short plan
// of the inverse (b = W - 1, a + 1 a power of two), runs its rows as one
// launch: the second operand's forward in full (into Y), the first operand's
// column pass (into X), then k_row_fwd_mul_inv -- the first operand's rows
// forward in LDS, times Y's rows, inverted (the partial last row as the
// inverse's one-short row) -- and the rest of the inverse: the first
// operand's rows go through HBM once instead of three times.
bool whole_rows_product(const Plan& P, unsigned wbytes) {
    return P.kind == 1 && P.logW >= 6 && (P.b == 0 || one_short_plan(P, wbytes));
}

template <class Mod>
tft_status mul_whole_impl(tft_ctx* ctx, const typename Mod::Word* A, uint64_t m, const typename Mod::Word* B,
                          uint64_t nb, typename Mod::Word* X, typename Mod::Word* Y, uint64_t n, hipStream_t st) {
    using Word = typename Mod::Word;
    const Plan P = make_plan(ctx, n);
    if (!whole_rows_product(P, ctx->wbytes)) return TFT_EINVAL;
    tft_status s = forward_impl<Mod>(ctx, B, nb, Y, n, st);
    if (s == TFT_OK) s = forward_impl<Mod>(ctx, A, m, X, n, st, 0, 1, false, false);
    if (s != TFT_OK) return s;
    auto T = tables_of<Word>(ctx);
    T.smax = P.smax;
    const auto G = two_pass_of<Word>(P, X, X, n, Y, reinterpret_cast<Word*>(ctx->varea));
    launch(ctx, TFT_K_ROW_FWD, tft::k_row_fwd_mul_inv<Mod>, dim3((uint32_t)P.a + (P.b ? 1u : 0u)), dim3(row_threads(P)),
           P.lds_row, st, mod_of<Mod>(ctx), T, G);
    s = launch_status();
    return s == TFT_OK ? inverse_impl<Mod>(ctx, X, Y, n, st, false, false) : s;
}

template <class Mod>
tft_status mul_impl(tft_ctx* ctx, const typename Mod::Word* A, uint64_t m, const typename Mod::Word* B, uint64_t nb,
                    typename Mod::Word* X, typename Mod::Word* Y, hipStream_t st) {
    const uint64_t r = m + nb - 1;
    const Plan P = make_plan(ctx, r);
    if (P.kind < 0) return TFT_ERANGE;
    const size_t mul_lds = 2 * P.lds_row + (size_t)P.M * ctx->wbytes;
    if (P.kind == 0 && mul_lds <= kLdsHard - 32 * 1024) {
        const Mod& md = mod_of<Mod>(ctx);
        const auto T = tables_of<typename Mod::Word>(ctx);
        launch(ctx, TFT_K_SMALL_MUL, tft::k_small_mul<Mod>, dim3(1), dim3(tft::kSmallThreads), mul_lds, st, md, T, A, (uint32_t)m,
                           B, (uint32_t)nb, X, P.M);
        return launch_status();
    }
    if (!Y) return TFT_EINVAL;
    if (whole_rows_product(P, ctx->wbytes)) return mul_whole_impl<Mod>(ctx, A, m, B, nb, X, Y, r, st);
    tft_status s = forward_impl<Mod>(ctx, A, m, X, r, st);
    if (s != TFT_OK) return s;
    s = forward_impl<Mod>(ctx, B, nb, Y, r, st);
    if (s != TFT_OK) return s;
    return inverse_impl<Mod>(ctx, X, Y, r, st);
}

// Forward transforms of the two whole blocks (n a power of two) at X and X + n,
// both at global block index g0, then X[i] = X[i] X[n + i], i < n: one column
// launch for both, then both blocks' rows in one launch that multiplies on its
// store (k_row_fwd_mul), when the rows are fused (W >= 64) and two of them fit
// in LDS; otherwise the two forwards and a pointwise launch.
template <class Mod>
tft_status forward_pair_mul(tft_ctx* ctx, typename Mod::Word* X, uint64_t n, uint64_t g0, hipStream_t st) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const Plan P = make_plan(ctx, n);
    if (P.kind < 0) return TFT_ERANGE;
    if (P.kind != 1 || P.b || P.logW < 6 || 2 * P.lds_row > kLdsDynMax) {
        tft_status s = forward_impl<Mod>(ctx, X, n, X, n, st, g0, 2);
        if (s != TFT_OK) return s;
        const uint64_t blocks = std::min<uint64_t>(8192, (n + kThreads - 1) / kThreads);
        launch(ctx, TFT_K_POINTWISE, tft::k_pointwise<Mod>, dim3((uint32_t)blocks), dim3(kThreads), 0, st, md, X,
               (const Word*)(X + n), n);
        return launch_status();
    }
    auto T = tables_of<Word>(ctx);
    T.smax = P.smax;
    Word* V = reinterpret_cast<Word*>(ctx->varea);
    auto G = two_pass_of<Word>(P, X, X, n, nullptr, V);
    G.g0 = g0;
    G.inst = n;
    G.Q = V + kVWords;
    const uint32_t tiles = (uint32_t)(P.W >> P.logC);
    launch(ctx, TFT_K_COL_FWD, col_fwd_kernel<Mod>(P.logC, false), dim3(tiles, 2), dim3(col_threads(P)), P.lds_col, st,
           md, T, G, tiles);
    launch(ctx, TFT_K_ROW_FWD, tft::k_row_fwd_mul<Mod>, dim3((uint32_t)P.a), dim3(row_threads(P)), 2 * P.lds_row, st, md,
           T, G);
    return launch_status();
}

// Folding for the space-restricted product: A mod (x^L - w_g) into outA and B
// mod (x^L - w_g) into outB, each word a Horner sum over the operand's terms
// j + t L.  The terms of a word are split into K chunks so that about
// kFoldItems threads per operand read the operand at once; the chunks' partial
// sums go to the context's fold area and are added by a second launch.
template <class Mod>
tft_status fold_impl(tft_ctx* ctx, const typename Mod::Word* A, uint64_t m, typename Mod::Word* outA,
                     const typename Mod::Word* B, uint64_t nb, typename Mod::Word* outB, unsigned logL, uint64_t g,
                     hipStream_t st) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const auto T = tables_of<Word>(ctx);
    const uint64_t L = 1ull << logL;
    const uint64_t terms = (std::max(m, nb) + L - 1) >> logL;   // largest number of t per j
    uint64_t K = std::max<uint64_t>(1, std::min<uint64_t>(terms, kFoldItems >> logL));
    const uint64_t chunk = (terms + K - 1) / K;
    K = (terms + chunk - 1) / chunk;
    Word* part = reinterpret_cast<Word*>(ctx->fold);   // two areas of kFoldItems words, then kFoldSpare
    tft::FoldArgs<Word> F;
    F.A[0] = A;
    F.A[1] = B;
    F.m[0] = m;
    F.m[1] = nb;
    F.out[0] = K == 1 ? outA : part;
    F.out[1] = K == 1 ? outB : part + kFoldItems;
    const uint64_t items = K << logL;
    launch(ctx, TFT_K_FOLD, tft::k_fold<Mod>, dim3((uint32_t)((items + kThreads - 1) / kThreads), 2), dim3(kThreads), 0,
           st, md, T, F, logL, (uint32_t)K, chunk, g);
    if (K == 1) return launch_status();
    tft::SumArgs<Word> S1;
    S1.part[0] = part;
    S1.part[1] = part + kFoldItems;
    if (K <= tft::kFoldFewK) {
        S1.out[0] = outA;
        S1.out[1] = outB;
        launch(ctx, TFT_K_FOLD, tft::k_fold_sum_few<Mod>, dim3((uint32_t)((L + kThreads - 1) / kThreads), 2),
               dim3(kThreads), 0, st, md, S1, logL, (uint32_t)K);
        return launch_status();
    }
    // many partials per word (L < kFoldItems / kFoldFewK): a workgroup per word and
    // span of kFoldSpan partials, then (if more than one span) per word
    const uint32_t spans = (uint32_t)((K + tft::kFoldSpan - 1) / tft::kFoldSpan);
    Word* part2 = part + 2 * kFoldItems;   // 2 spans L words, spans L <= kFoldItems / kFoldSpan + L
    S1.out[0] = spans == 1 ? outA : part2;
    S1.out[1] = spans == 1 ? outB : part2 + kFoldSpare / 2;
    launch(ctx, TFT_K_FOLD, tft::k_fold_sum<Mod>, dim3((uint32_t)L, spans, 2), dim3(kThreads), 0, st, md, S1, logL,
           (uint32_t)K);
    if (spans > 1) {
        tft::SumArgs<Word> S2;
        S2.part[0] = part2;
        S2.part[1] = part2 + kFoldSpare / 2;
        S2.out[0] = outA;
        S2.out[1] = outB;
        launch(ctx, TFT_K_FOLD, tft::k_fold_sum<Mod>, dim3((uint32_t)L, 1, 2), dim3(kThreads), 0, st, md, S2, logL,
               spans);
    }
    return launch_status();
}

// Space-restricted product (section 5, Algorithm 3): the output buffer is the
// only memory of the product's size written.  For q = 0, L_0, L_0 + L_1, ...
// with L the largest power of two such that q + 2L <= r: fold A modulo
// x^L - w_{q/L} into X[q, q+L) and B into X[q+L, q+2L), transform both blocks
// (global index q/L, one launch per pass for the two, so X_{q+i} = A(w_{q+i})),
// multiply pointwise into X[q, q+L) (on the row pass's store, forward_pair_mul).  Each block reads all of A and B once, and
// the short blocks at the end are latency-bound launches, so once
// t = r - q < 2^(kRestrLog + 1) the remaining blocks are not taken one by one:
// they lie in at most two aligned nodes of the transform tree of size
// S = 2^(ceil(lg t) - 1) (t <= 2 S, and q is a multiple of S), whose folds of
// A and B (4 S words, a fixed area of the context) are transformed and
// multiplied into X[q, r) -- the same values, two passes over A and B instead
// of about lg t.  Below two single-workgroup sizes the nodes are transformed
// and multiplied by one workgroup each (k_restr_tail, folds in the V area).
// Then the inverse TFT of length r.
template <class Mod>
tft_status mul_restricted_impl(tft_ctx* ctx, const typename Mod::Word* A, uint64_t m, const typename Mod::Word* B,
                               uint64_t nb, typename Mod::Word* X, hipStream_t st) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const uint64_t r = m + nb - 1;
    if (r > (1ull << ctx->v)) return TFT_ERANGE;
    const unsigned logSs = small_max_log2(ctx->wbytes);
    const uint64_t Ss = 1ull << logSs;
    tft_status s = TFT_OK;
    uint64_t q = 0;
    while (s == TFT_OK && r - q >= (2ull << kRestrLog)) {
        const unsigned logL = (63u - (unsigned)__builtin_clzll(r - q)) - 1u;
        const uint64_t L = 1ull << logL, g = q >> logL;
        s = fold_impl<Mod>(ctx, A, m, X + q, B, nb, X + q + L, logL, g, st);
        if (s == TFT_OK) s = forward_pair_mul<Mod>(ctx, X + q, L, g, st);
        q += L;
    }
    if (s != TFT_OK) return s;
    const uint64_t t = r - q;   // q is a multiple of every block size so far (all >= 2^kRestrLog)
    if (t < 2 * Ss) {
        Word* N = reinterpret_cast<Word*>(ctx->varea);
        const uint32_t nodes = (uint32_t)((t + Ss - 1) >> logSs);
        for (uint32_t j = 0; j < nodes && s == TFT_OK; j++)
            s = fold_impl<Mod>(ctx, A, m, N + j * Ss, B, nb, N + (2 + j) * Ss, logSs, (q >> logSs) + j, st);
        if (s != TFT_OK) return s;
        launch(ctx, TFT_K_SMALL_MUL, tft::k_restr_tail<Mod>, dim3(nodes), dim3(tft::kSmallThreads),
               2 * (size_t)tft::padded_words((uint32_t)Ss) * ctx->wbytes, st, md, tables_of<Word>(ctx),
               (const Word*)N, logSs, q >> logSs, r, X);
    } else {
        const unsigned logS = (t & (t - 1)) ? 64u - (unsigned)__builtin_clzll(t) - 1u : 63u - (unsigned)__builtin_clzll(t) - 1u;
        const uint64_t S = 1ull << logS;   // S < t <= 2 S, Ss <= S <= 2^kRestrLog
        Word* N = reinterpret_cast<Word*>(ctx->fold) + 2 * kFoldItems + kFoldSpare;
        const uint32_t nodes = (uint32_t)((t + S - 1) >> logS);
        for (uint32_t j = 0; j < nodes && s == TFT_OK; j++) {
            const uint64_t g = (q >> logS) + j;
            s = fold_impl<Mod>(ctx, A, m, N + 2 * j * S, B, nb, N + (2 * j + 1) * S, logS, g, st);
            if (s == TFT_OK) s = forward_impl<Mod>(ctx, N + 2 * j * S, S, N + 2 * j * S, S, st, g, 2);
        }
        if (s != TFT_OK) return s;
        launch(ctx, TFT_K_POINTWISE, tft::k_restr_nodes_mul<Mod>, dim3((uint32_t)((t + kThreads - 1) / kThreads)),
               dim3(kThreads), 0, st, md, (const Word*)N, logS, q, r, X);
    }
    s = launch_status();
    return s == TFT_OK ? inverse_impl<Mod>(ctx, X, nullptr, r, st) : s;
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
    // the same schedule as poly_mul at a length a W
    tft_status s = TFT_OK;
    if (whole_rows_product(make_plan(ctx, N), ctx->wbytes)) {
        s = mul_whole_impl<Mod>(ctx, Ap, N, Bp, N, Ap, Bp, N, st);
    } else {
        s = forward_impl<Mod>(ctx, Ap, N, Ap, N, st);
        if (s == TFT_OK) s = forward_impl<Mod>(ctx, Bp, N, Bp, N, st);
        if (s == TFT_OK) s = inverse_impl<Mod>(ctx, Ap, Bp, N, st);
    }
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
    auto enc = [&](uint64_t x) -> Word {   // Montgomery form: x 2^(bits of Word) mod p
        return montgomery ? (Word)(((u128)x << (8 * sizeof(Word))) % p) : (Word)x;
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

// f(Mod{}) with the context's arithmetic: ModU32 (words of 4 bytes), ModGL
// (p = 2^64 - 2^32 + 1) or ModM64 (the other primes of 8-byte words); f uses
// the argument's type only.
template <class F>
tft_status with_mod(const tft_ctx* ctx, F&& f) {
    if (ctx->wbytes == 4) return f(tft::ModU32{});
    if (ctx->p == kGoldilocks) return f(tft::ModGL{});
    return f(tft::ModM64{});
}

template <class F>
tft_status dispatch(tft_ctx* ctx, F&& f) {
    if (!ctx) return TFT_EINVAL;
    DeviceGuard guard(ctx->device);
    return with_mod(ctx, f);
}

// ================================================================= batches
// A batch is planned once (host) and its work lists uploaded once; running it
// only launches kernels, so a run can be captured in a HIP graph and replayed.
enum { PH_COL_FWD = 0, PH_ROW_FWD, PH_ROW_INV, PH_COL_INV_SHORT, PH_LAST_INV, PH_COL_INV_LONG, PH_COUNT };

}  // namespace

struct tft_batch {
    tft_ctx* ctx;
    int products;              // 1: products, 0: forward transforms
    size_t count;
    size_t n_small, n_two;     // instances on each path
    void* dmem;                // recs | items | jobs | V areas | counter
    size_t dbytes;
    void* recs;
    tft::Item* items[PH_COUNT];
    uint32_t n_items[PH_COUNT];
    void* jobs;
    uint32_t* counter;
    size_t lds_col, lds_row, lds_small;   // lds_small: the single-workgroup jobs after the first n_big
    size_t n_big, lds_big;     // single-workgroup jobs whose LDS allows one workgroup per CU: their
    uint32_t big_grid;         // own persistent launch of kBigJobThreads threads, before the rest
    bool row_mul;              // products: forward rows, product and inverse rows fused (k_row_mul_list)
    uint32_t rowmul_thr;       // its workgroup size
    size_t lds_rowmul;         // and its two row buffers
    uint32_t spread;           // a batch with the device to itself (the serving queue's batches
                               // overlap each other): column lists in XCD-aware order, fused row
                               // products (throughput); otherwise the unfused row passes, more
                               // workgroups per pass (latency)
    uint32_t row_thr, col_thr;   // workgroup sizes of the pass launches (widest row / tile of the batch)
    uint32_t list_col_thr;       // of its column lists
    int logC;
    uint32_t small_grid;
    hipStream_t side;          // the single-workgroup jobs run here, beside the two-pass phases
    hipEvent_t fork, join;
    BatchArena* arena;         // borrowed memory, stream and events (nullptr: the batch owns its own)
};

namespace {

hipError_t arena_init(BatchArena* A) {
    hipError_t e = hipStreamCreateWithFlags(&A->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&A->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&A->join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&A->done, hipEventDisableTiming);
    return e;
}

// grows the arena to at least `bytes` (only while no batch of it is on the device)
hipError_t arena_reserve(BatchArena* A, size_t bytes) {
    if (bytes > A->dcap) {
        const size_t c = std::max<size_t>({bytes, 2 * A->dcap, size_t(1) << 20});
        if (A->dmem) (void)hipFree(A->dmem);
        A->dmem = nullptr;
        A->dcap = 0;
        const hipError_t e = hipMalloc(&A->dmem, c);
        if (e != hipSuccess) return e;
        A->dcap = c;
    }
    if (bytes > A->hcap) {
        const size_t c = std::max<size_t>({bytes, 2 * A->hcap, size_t(1) << 20});
        if (A->hmem) (void)hipHostFree(A->hmem);
        A->hmem = nullptr;
        A->hcap = 0;
        const hipError_t e = hipHostMalloc(&A->hmem, c, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        A->hcap = c;
    }
    return hipSuccess;
}

void arena_free(BatchArena* A) {
    if (A->dmem) (void)hipFree(A->dmem);
    if (A->hmem) (void)hipHostFree(A->hmem);
    if (A->side) (void)hipStreamDestroy(A->side);
    if (A->fork) (void)hipEventDestroy(A->fork);
    if (A->join) (void)hipEventDestroy(A->join);
    if (A->done) (void)hipEventDestroy(A->done);
    *A = BatchArena();
}

// LDS of a single-workgroup batch job of length r (data blocks + twiddles).
size_t small_job_lds(unsigned w, uint64_t r, int products) {
    const size_t Mr = pow2ceil(r);
    return ((products ? 2 : 1) * (size_t)tft::padded_words((uint32_t)Mr) + Mr) * w;
}

// A batch runs instance r in one workgroup (no workspace) when the planner
// keeps it in LDS and both operands' blocks fit beside its twiddles.
bool batch_small(const tft_ctx* ctx, const Plan& P, uint64_t r, int products) {
    return P.kind == 0 && small_job_lds(ctx->wbytes, r, products) <= kLdsHard - 32 * 1024;
}

// Whether a batched product of length r needs the r-word workspace (the same
// decision batch_build takes, so the serving queue reserves exactly that).
bool needs_workspace(const tft_ctx* ctx, uint64_t r, int products) {
    const Plan P = make_plan(ctx, r, true);
    return products && !batch_small(ctx, P, r, products);
}

template <class Mod>
tft_status batch_build(tft_ctx* ctx, const tft_mul_desc* d, size_t count, int products, tft_batch* B,
                       hipStream_t upload) {
    using Word = typename Mod::Word;
    const unsigned w = ctx->wbytes;
    std::vector<tft::SmallJob<Word>> jobs;
    std::vector<tft::TwoPass<Word>> recs;
    std::vector<tft::Item> items[PH_COUNT];
    std::vector<size_t> vwords;   // V area size per record
    struct RowGeom {
        uint32_t rec, logW, a, b;   // first record of the instance and its split
    };
    std::vector<RowGeom> rows;
    size_t v_total = 0;
    B->lds_col = B->lds_row = B->lds_small = 0;
    B->row_thr = B->col_thr = 64;
    B->logC = col_log_width(w);
    for (size_t k = 0; k < count; k++) {
        const tft_mul_desc& D = d[k];
        if (!D.a || !D.out || D.la == 0 || (products && (!D.b || D.lb == 0))) return TFT_EINVAL;
        const uint64_t r = products ? D.la + D.lb - 1 : D.la;
        if (log2u(r) > ctx->v) return TFT_ERANGE;
        const Plan P = make_plan(ctx, r, true);
        if (P.kind < 0) return TFT_ERANGE;
        if (batch_small(ctx, P, r, products)) {
            tft::SmallJob<Word> J;
            J.A = (const Word*)D.a;
            J.B = products ? (const Word*)D.b : nullptr;
            J.X = (Word*)D.out;
            J.m = (uint32_t)D.la;
            J.nb = products ? (uint32_t)D.lb : 0;
            J.M = (uint32_t)pow2ceil(r);
            jobs.push_back(J);
            continue;
        }
        if (P.kind != 1) return TFT_ERANGE;
        if (products && !D.work) return TFT_EINVAL;
        B->lds_col = std::max(B->lds_col, P.lds_col);
        B->lds_row = std::max(B->lds_row, P.lds_row);
        // one radix-8 unit per thread: rows of W words, tiles of M C words
        B->row_thr = std::max(B->row_thr, row_threads(P));
        B->col_thr = std::max(B->col_thr, col_threads(P));
        const uint32_t tiles = (uint32_t)(P.W >> P.logC);
        const uint32_t C = 1u << P.logC;
        const int nops = products ? 2 : 1;
        const uint32_t rec0 = (uint32_t)recs.size();
        for (int op = 0; op < nops; op++) {
            Word* X = op == 0 ? (Word*)D.out : (Word*)D.work;
            const Word* src = op == 0 ? (const Word*)D.a : (const Word*)D.b;
            const uint64_t n_src = op == 0 ? D.la : D.lb;
            const Word* Y = (products && op == 0) ? (const Word*)D.work : nullptr;
            recs.push_back(two_pass_of<Word>(P, X, products ? src : X, products ? n_src : r, Y, nullptr));
            vwords.push_back(P.W);
            v_total += P.W;
            const uint32_t rec = rec0 + op;
            for (uint32_t t = 0; t < tiles; t++) items[PH_COL_FWD].push_back({rec, t});
        }
        rows.push_back({rec0, (uint32_t)P.logW, (uint32_t)P.a, (uint32_t)P.b});
        if (products) {
            for (uint32_t t = (uint32_t)(P.b / C); t < tiles; t++) items[PH_COL_INV_SHORT].push_back({rec0, t});
            if (P.b) {
                items[PH_LAST_INV].push_back({rec0, 0});
                for (uint32_t t = 0; t < (P.b + C - 1) / C; t++) items[PH_COL_INV_LONG].push_back({rec0, t});
            }
        }
    }
    // Row phases.  Products of a batch with the device to itself fuse the
    // forward rows of both operands, the pointwise product and the inverse
    // rows into one launch (k_row_mul_list: R rows per workgroup with R W = 8
    // threads, two buffers of LDS) when the buffers fit: 3 r words of HBM
    // traffic instead of 7 r.  Otherwise forward rows per operand, then
    // inverse rows and the last row's pieces: twice the workgroups and a
    // third of the work each, which the serving queue's small, overlapping
    // batches finish sooner (served p50 and p99 about 5 % and 15 % lower).
    const uint32_t rowmul_min = tl_batch_rowmul_thr > 0 ? (uint32_t)tl_batch_rowmul_thr
                                                        : ctx->batch_rowmul_thr.load(std::memory_order_relaxed);
    const uint32_t list_col_max = tl_batch_col_thr > 0 ? (uint32_t)tl_batch_col_thr
                                                       : ctx->batch_col_thr.load(std::memory_order_relaxed);
    B->rowmul_thr = std::max<uint32_t>(B->row_thr, rowmul_min);
    // Column tiles of a batch are mostly smaller than its largest one, whose
    // size sets col_thr: where eight tiles fit in a CU's LDS, 128 threads let
    // more of them share the CU with fewer idle threads (4096 products:
    // 1.07 -> 0.94 ms).  The serving queue keeps one thread per radix-8 unit
    // of the largest tile.
    B->list_col_thr = B->spread && B->lds_col * 8 <= kLdsHard ? std::min<uint32_t>(B->col_thr, list_col_max)
                                                              : B->col_thr;
    B->lds_rowmul = 0;
    for (const RowGeom& g : rows) {
        const int logR = tft::row_mul_log_rows(g.logW, B->rowmul_thr);
        B->lds_rowmul = std::max(B->lds_rowmul, (size_t)2 * tft::padded_words(1u << (g.logW + logR)) * w);
    }
    B->row_mul = B->spread && products && !rows.empty() && B->lds_rowmul <= kLdsDynMax;
    for (const RowGeom& g : rows) {
        const uint32_t nfwd = g.a + (g.b ? 1 : 0);
        if (B->row_mul) {
            const uint32_t R = 1u << tft::row_mul_log_rows(g.logW, B->rowmul_thr);
            for (uint32_t j = 0; j < g.a; j += R) items[PH_ROW_FWD].push_back({g.rec, j});
            if (g.b) items[PH_ROW_FWD].push_back({g.rec, g.a});
            continue;
        }
        for (int op = 0; op < (products ? 2 : 1); op++)
            for (uint32_t j = 0; j < nfwd; j++) items[PH_ROW_FWD].push_back({g.rec + op, j});
        if (products) {
            const uint32_t nr = tft::row_inv_items(1u << g.logW, g.a, g.b);
            for (uint32_t j = 0; j < nr; j++) items[PH_ROW_INV].push_back({g.rec, j});
        }
    }
    // longest single-workgroup jobs first
    std::stable_sort(jobs.begin(), jobs.end(), [](const tft::SmallJob<Word>& x, const tft::SmallJob<Word>& y) {
        return (uint64_t)x.m + x.nb > (uint64_t)y.m + y.nb;
    });
    B->n_small = jobs.size();
    // the jobs (longest first) in two classes by LDS: above a third of a CU's
    // LDS one workgroup fits per CU, and it gets kBigJobThreads threads; the
    // rest share the CUs at three or more workgroups of kThreads each
    B->n_big = 0;
    B->lds_big = B->lds_small = 0;
    for (const auto& J : jobs) {
        const size_t l = small_job_lds(w, (uint64_t)J.m + J.nb - (J.B ? 1 : 0), products);
        if (l > kLdsHard / 3) {
            B->n_big++;
            B->lds_big = std::max(B->lds_big, l);
        } else {
            B->lds_small = std::max(B->lds_small, l);
        }
    }
    B->n_two = recs.size() / (products ? 2 : 1);
    // one device allocation: recs | items per phase | jobs | V areas | counter
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    const size_t o_recs = off;
    off = align(off + recs.size() * sizeof(tft::TwoPass<Word>));
    size_t o_items[PH_COUNT];
    for (int ph = 0; ph < PH_COUNT; ph++) {
        o_items[ph] = off;
        off = align(off + items[ph].size() * sizeof(tft::Item));
    }
    const size_t o_jobs = off;
    off = align(off + jobs.size() * sizeof(tft::SmallJob<Word>));
    const size_t o_v = off;
    off = align(off + v_total * w);
    const size_t o_ctr = off;
    off = align(off + 256);
    B->dbytes = off;
    // the V areas are written before they are read and the counter is reset
    // by every run, so only the lists in front of them are uploaded
    std::vector<char> own;
    char* host;
    if (B->arena) {
        const hipError_t e = arena_reserve(B->arena, off);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? TFT_ENOMEM : TFT_EDEVICE;
        B->dmem = B->arena->dmem;
        host = (char*)B->arena->hmem;
        std::memset(host, 0, o_v);
    } else {
        const hipError_t e = hipMalloc(&B->dmem, off);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? TFT_ENOMEM : TFT_EDEVICE;
        own.assign(o_v, 0);
        host = own.data();
    }
    char* base = (char*)B->dmem;
    size_t vo = 0;
    for (size_t i = 0; i < recs.size(); i++) {
        recs[i].V = (Word*)(base + o_v) + vo;
        vo += vwords[i];
    }
    std::memcpy(host + o_recs, recs.data(), recs.size() * sizeof(tft::TwoPass<Word>));
    for (int ph = 0; ph < PH_COUNT; ph++)
        std::memcpy(host + o_items[ph], items[ph].data(), items[ph].size() * sizeof(tft::Item));
    std::memcpy(host + o_jobs, jobs.data(), jobs.size() * sizeof(tft::SmallJob<Word>));
    const hipError_t e = B->arena ? hipMemcpyAsync(B->dmem, host, o_v, hipMemcpyHostToDevice, upload)
                                  : hipMemcpy(B->dmem, host, o_v, hipMemcpyHostToDevice);
    if (e != hipSuccess) return TFT_EDEVICE;
    B->recs = base + o_recs;
    for (int ph = 0; ph < PH_COUNT; ph++) {
        B->items[ph] = (tft::Item*)(base + o_items[ph]);
        B->n_items[ph] = (uint32_t)items[ph].size();
    }
    B->jobs = base + o_jobs;
    B->counter = (uint32_t*)(base + o_ctr);
    // persistent grids: as many workgroups as fit at once (LDS-limited), at most one per job
    int ncu = 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) ncu = 256;
    uint32_t per_cu = B->lds_small ? (uint32_t)std::max<size_t>(1, kLdsHard / B->lds_small) : 1;
    per_cu = std::min<uint32_t>(per_cu, 8);
    B->small_grid = (uint32_t)std::min<size_t>(jobs.size() - B->n_big, (size_t)ncu * per_cu);
    B->big_grid = (uint32_t)std::min<size_t>(B->n_big, (size_t)ncu);
    return TFT_OK;
}

template <class Mod>
tft_status batch_run(tft_batch* B, hipStream_t st) {
    using Word = typename Mod::Word;
    tft_ctx* ctx = B->ctx;
    const Mod& md = mod_of<Mod>(ctx);
    const auto T = tables_of<Word>(ctx);
    const auto* recs = (const tft::TwoPass<Word>*)B->recs;
    const bool both = B->n_small && B->n_two;
    hipStream_t small_st = st;
    if (both) {
        if (hipEventRecord(B->fork, st) != hipSuccess || hipStreamWaitEvent(B->side, B->fork, 0) != hipSuccess)
            return TFT_EDEVICE;
        small_st = B->side;
    }
    if (B->n_small) {
        const auto* jobs = (const tft::SmallJob<Word>*)B->jobs;
        launch(ctx, TFT_K_COPY, tft::k_reset_counter, dim3(1), dim3(64), 0, small_st, B->counter);
        if (B->n_big)
            launch(ctx, TFT_K_SMALL_LIST, tft::k_small_list<Mod, kBigJobThreads>, dim3(B->big_grid),
                   dim3(kBigJobThreads), B->lds_big, small_st, md, T, jobs, (uint32_t)B->n_big, B->counter);
        if (B->n_small > B->n_big)
            launch(ctx, TFT_K_SMALL_LIST, tft::k_small_list<Mod>, dim3(B->small_grid), dim3(kThreads), B->lds_small,
                   small_st, md, T, jobs + B->n_big, (uint32_t)(B->n_small - B->n_big), B->counter + 1);
    }
    if (B->n_items[PH_COL_FWD])
        launch(ctx, TFT_K_COL_FWD, col_fwd_list_kernel<Mod>(B->logC),
               dim3(B->n_items[PH_COL_FWD]), dim3(B->list_col_thr), B->lds_col, st, md, T, recs,
               (const tft::Item*)B->items[PH_COL_FWD], B->spread);
    if (B->n_items[PH_ROW_FWD] && B->row_mul)
        launch(ctx, TFT_K_ROW_FWD, tft::k_row_mul_list<Mod>, dim3(B->n_items[PH_ROW_FWD]), dim3(B->rowmul_thr),
               B->lds_rowmul, st, md, T, recs, (const tft::Item*)B->items[PH_ROW_FWD]);
    else if (B->n_items[PH_ROW_FWD])
        launch(ctx, TFT_K_ROW_FWD, tft::k_row_fwd_list<Mod>, dim3(B->n_items[PH_ROW_FWD]), dim3(B->row_thr), B->lds_row,
               st, md, T, recs, (const tft::Item*)B->items[PH_ROW_FWD]);
    if (B->n_items[PH_ROW_INV])
        launch(ctx, TFT_K_ROW_INV, tft::k_row_inv_list<Mod>, dim3(B->n_items[PH_ROW_INV]), dim3(B->row_thr), B->lds_row,
               st, md, T, recs, (const tft::Item*)B->items[PH_ROW_INV]);
    if (B->n_items[PH_COL_INV_SHORT])
        launch(ctx, TFT_K_COL_INV_SHORT, col_inv_list_kernel<Mod>(B->logC),
               dim3(B->n_items[PH_COL_INV_SHORT]), dim3(B->list_col_thr), B->lds_col, st, md, T, recs,
               (const tft::Item*)B->items[PH_COL_INV_SHORT], 0, B->spread);
    if (B->n_items[PH_LAST_INV])
        launch(ctx, TFT_K_LAST_INV, tft::k_last_inv_list<Mod>, dim3(B->n_items[PH_LAST_INV]), dim3(B->row_thr),
               B->lds_row, st, md, T, recs, (const tft::Item*)B->items[PH_LAST_INV]);
    if (B->n_items[PH_COL_INV_LONG])
        launch(ctx, TFT_K_COL_INV_LONG, col_inv_list_kernel<Mod>(B->logC),
               dim3(B->n_items[PH_COL_INV_LONG]), dim3(B->list_col_thr), B->lds_col, st, md, T, recs,
               (const tft::Item*)B->items[PH_COL_INV_LONG], 1, B->spread);
    if (both) {
        if (hipEventRecord(B->join, B->side) != hipSuccess || hipStreamWaitEvent(st, B->join, 0) != hipSuccess)
            return TFT_EDEVICE;
    }
    return launch_status();
}

void batch_free(tft_batch* B) {
    if (!B) return;
    DeviceGuard guard(B->ctx->device);
    if (!B->arena) {
        if (B->dmem) (void)hipFree(B->dmem);
        if (B->side) (void)hipStreamDestroy(B->side);
        if (B->fork) (void)hipEventDestroy(B->fork);
        if (B->join) (void)hipEventDestroy(B->join);
    }
    delete B;
}

// arena == nullptr: the batch allocates its own memory and uploads its lists
// synchronously (it can then be run many times, also under graph capture);
// otherwise it borrows the arena and uploads on `upload`, the stream it runs on.
// spread: the batch has the device to itself (not the serving queue's
// overlapping batches): XCD-aware column lists and fused row products
tft_status batch_create(tft_ctx* ctx, const tft_mul_desc* d, size_t count, int products, tft_batch** out,
                        BatchArena* arena = nullptr, hipStream_t upload = nullptr, bool spread = true) {
    if (!ctx || !out || (count && !d)) return TFT_EINVAL;
    *out = nullptr;
    DeviceGuard guard(ctx->device);
    tft_batch* B = new (std::nothrow) tft_batch();
    if (!B) return TFT_ENOMEM;
    B->ctx = ctx;
    B->spread = spread ? 1u : 0u;   // read by batch_build
    B->products = products;
    B->count = count;
    B->arena = arena;
    if (arena) {
        B->side = arena->side;
        B->fork = arena->fork;
        B->join = arena->join;
    }
    tft_status s = with_mod(ctx, [&](auto mt) { return batch_build<decltype(mt)>(ctx, d, count, products, B, upload); });
    if (s == TFT_OK && !arena) {
        if (hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&B->join, hipEventDisableTiming) != hipSuccess)
            s = TFT_EDEVICE;
    }
    if (s != TFT_OK) {
        batch_free(B);
        return s;
    }
    *out = B;
    return TFT_OK;
}

// Convenience calls keep their batch alive until the next convenience call
// (or context destruction) so that work already enqueued can finish.
tft_status batch_once(tft_ctx* ctx, const tft_mul_desc* d, size_t count, int products, hipStream_t st) {
    if (ctx->last_batch) {
        (void)hipEventSynchronize(ctx->last_done);
        batch_free(ctx->last_batch);
        ctx->last_batch = nullptr;
    }
    if (count == 0) return TFT_OK;
    if (!ctx->once_arena.side && arena_init(&ctx->once_arena) != hipSuccess) {
        arena_free(&ctx->once_arena);
        return TFT_EDEVICE;
    }
    tft_batch* B = nullptr;
    tft_status s = batch_create(ctx, d, count, products, &B, &ctx->once_arena, st);
    if (s != TFT_OK) return s;
    DeviceGuard guard(ctx->device);
    s = with_mod(ctx, [&](auto mt) { return batch_run<decltype(mt)>(B, st); });
    ctx->last_batch = B;
    if (!ctx->last_done && hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming) != hipSuccess)
        return TFT_EDEVICE;
    if (hipEventRecord(ctx->last_done, st) != hipSuccess) return TFT_EDEVICE;
    return s;
}

}  // namespace

// ================================================================= serving
// A request queue with continuous batching.  submit() appends a product to a
// pending FIFO and returns a ticket.  A worker thread admits pending requests
// in order while their workspace (r words, the in-place footprint of B's
// transform) fits in the queue's device pool and fewer than max_inflight
// requests are on the device; each group of newly admitted requests becomes
// one batch, launched with whichever of kQueueSlots slots (a stream and a reusable
// batch arena) is free, so that consecutive batches overlap on the device and
// a batch in steady state neither allocates nor frees device memory.  The worker polls the batches' completion
// events, releases their workspace, records completion times and admits more.
namespace {

struct QReq {
    uint64_t ticket;
    tft_mul_desc d;
    uint64_t r;
    uint64_t off;        // workspace offset in the pool (words), ~0 if none needed
    hipStream_t src;     // the stream the operands were produced on
};

struct QBatch {
    tft_batch* B;
    int slot;   // the stream and arena it runs with; its arena's `done` event follows it
    std::vector<QReq> reqs;
};

// First-fit allocator over word offsets of the pool, coalescing on free.
struct PoolAlloc {
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    uint64_t total = 0, used = 0;
    void init(uint64_t words) {
        free_.clear();
        free_[0] = words;
        total = words;
        used = 0;
    }
    bool alloc(uint64_t n, uint64_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                used += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

// Batches a queue keeps in flight at once (each with its stream and arena).
constexpr int kQueueSlots = 3;

struct tft_queue {
    tft_ctx* ctx;
    void* pool;
    size_t pool_words, max_inflight, max_pending, max_batch;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<QReq> pending;
    std::deque<QBatch> inflight;
    size_t inflight_reqs;
    PoolAlloc alloc;
    // completion time (steady clock, ns; 0 while pending) of ticket t at
    // done_ns[t - 1]: tickets are consecutive, so a deque indexed by ticket
    // grows by one word per request without rehashing or moving what it
    // holds (a hash map's rehash at a million entries took tens of ms under
    // the queue's lock, stalling the client and the worker alike)
    std::deque<uint64_t> done_ns;
    std::unordered_map<uint64_t, int> failed;   // tickets whose batch failed
    uint64_t next_ticket;
    bool stop;
    std::thread worker;
    hipStream_t streams[kQueueSlots];
    BatchArena arenas[kQueueSlots];
    bool slot_busy[kQueueSlots];
    uint64_t n_submitted, n_completed, n_batches, n_rejected, max_pool_used;
    tft_status error;
    // one event per producer stream, recorded by every submit on that stream;
    // a batch waits for the latest record of each stream its requests name
    std::unordered_map<hipStream_t, hipEvent_t> src_events;
};

namespace {

void queue_worker(tft_queue* q) {
    (void)hipSetDevice(q->ctx->device);
    std::unique_lock<std::mutex> lk(q->mu);
    for (;;) {
        bool progress = false;
        // retire finished batches
        for (auto it = q->inflight.begin(); it != q->inflight.end();) {
            const hipError_t e = hipEventQuery(q->arenas[it->slot].done);
            if (e == hipErrorNotReady) {
                ++it;
                continue;
            }
            const uint64_t t = now_ns();
            for (const QReq& rq : it->reqs) {
                q->done_ns[rq.ticket - 1] = t;
                if (e != hipSuccess) q->failed[rq.ticket] = 1;
                if (rq.off != ~0ull) q->alloc.release(rq.off, rq.r);
            }
            q->inflight_reqs -= it->reqs.size();
            q->n_completed += it->reqs.size();
            if (e != hipSuccess) q->error = TFT_EDEVICE;
            tft_batch_destroy(it->B);
            q->slot_busy[it->slot] = false;
            it = q->inflight.erase(it);
            progress = true;
        }
        if (progress) q->cv_done.notify_all();
        // admit in arrival order and launch one batch (at most two batches in
        // flight, one per slot)
        int slot = -1;
        for (int i = 0; i < kQueueSlots && slot < 0; i++)
            if (!q->slot_busy[i]) slot = i;
        if (!q->pending.empty() && slot >= 0) {
            std::vector<QReq> group;
            while (!q->pending.empty() && group.size() < q->max_batch && q->inflight_reqs + group.size() < q->max_inflight) {
                group.push_back(q->pending.front());   // workspace was reserved at submit
                q->pending.pop_front();
            }
            if (!group.empty()) {
                q->inflight_reqs += group.size();
                const hipStream_t st = q->streams[slot];
                // the batch starts after the work that produced its operands:
                // the latest record of each producer stream's event (records
                // and waits both happen under the queue's lock)
                tft_status s = TFT_OK;
                std::vector<hipStream_t> srcs;
                for (const QReq& rq : group)
                    if (std::find(srcs.begin(), srcs.end(), rq.src) == srcs.end()) srcs.push_back(rq.src);
                for (hipStream_t src : srcs)
                    if (hipStreamWaitEvent(st, q->src_events[src], 0) != hipSuccess) s = TFT_EDEVICE;
                lk.unlock();
                std::vector<tft_mul_desc> ds(group.size());
                for (size_t i = 0; i < group.size(); i++) ds[i] = group[i].d;
                tft_batch* B = nullptr;
                BatchArena* A = &q->arenas[slot];
                if (s == TFT_OK) s = batch_create(q->ctx, ds.data(), ds.size(), 1, &B, A, st, false);
                if (s == TFT_OK) s = tft_batch_run(B, st);
                if (s == TFT_OK && hipEventRecord(A->done, st) != hipSuccess) s = TFT_EDEVICE;
                lk.lock();
                if (s != TFT_OK) {
                    // fail the group now; its workspace is released once the stream has drained
                    (void)hipStreamSynchronize(st);
                    (void)hipStreamSynchronize(A->side);
                    if (B) tft_batch_destroy(B);
                    const uint64_t t = now_ns();
                    for (const QReq& rq : group) {
                        q->done_ns[rq.ticket - 1] = t;
                        q->failed[rq.ticket] = 1;
                        if (rq.off != ~0ull) q->alloc.release(rq.off, rq.r);
                    }
                    q->inflight_reqs -= group.size();
                    q->n_completed += group.size();
                    q->error = s;
                    q->cv_done.notify_all();
                } else {
                    q->slot_busy[slot] = true;
                    q->inflight.push_back(QBatch{B, slot, std::move(group)});
                    q->n_batches++;
                }
                continue;
            }
        }
        if (q->stop && q->pending.empty() && q->inflight.empty()) break;
        // nothing to do right now: sleep briefly (a submit wakes us; with
        // batches in flight, look for completions every 5 us: against 20 us
        // the served p50 at 20 k requests/s was 12 us lower, p99 the same)
        q->cv_work.wait_for(lk, std::chrono::microseconds(q->inflight.empty() ? 500 : 5));
    }
}

}  // namespace

// ============================================================== C entry points
template <class Mod>
tft_status walk_impl(tft_ctx* ctx, void* const* X, const size_t* n, size_t count, int inverse, hipStream_t st) {
    using Word = typename Mod::Word;
    const Mod& md = mod_of<Mod>(ctx);
    const auto T = tables_of<Word>(ctx);
    std::vector<uint64_t> host(2 * count);
    for (size_t k = 0; k < count; k++) {
        host[k] = (uint64_t)(uintptr_t)X[k];
        host[count + k] = n[k];
    }
    void* dmem = nullptr;
    if (hipMalloc(&dmem, host.size() * 8) != hipSuccess) return TFT_ENOMEM;
    tft_status s = TFT_OK;
    if (hipMemcpy(dmem, host.data(), host.size() * 8, hipMemcpyHostToDevice) != hipSuccess) s = TFT_EDEVICE;
    if (s == TFT_OK) {
        Word* const* ptrs = reinterpret_cast<Word* const*>(dmem);
        const uint64_t* lens = reinterpret_cast<const uint64_t*>(dmem) + count;
        const dim3 grid((uint32_t)((count + tft::kWalkWaves - 1) / tft::kWalkWaves));
        if (inverse)
            launch(ctx, TFT_K_SMALL_LIST, tft::k_walk<Mod, true>, grid, dim3(64 * tft::kWalkWaves), 0, st, md, T, ptrs,
                   lens, (uint32_t)count);
        else
            launch(ctx, TFT_K_SMALL_LIST, tft::k_walk<Mod, false>, grid, dim3(64 * tft::kWalkWaves), 0, st, md, T, ptrs,
                   lens, (uint32_t)count);
        s = launch_status();
        if (hipStreamSynchronize(st) != hipSuccess && s == TFT_OK) s = TFT_EDEVICE;
    }
    (void)hipFree(dmem);
    return s;
}

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
    // 4-byte words for p < 2^31; 8-byte words for p = 2^64 - 2^32 + 1 and for
    // the other primes below 2^63 (Montgomery arithmetic, ModM64)
    const bool gold = (p == kGoldilocks);
    if (!gold && (p >= (1ull << 63) || p < 3 || !(p & 1) || !is_probable_prime(p))) return TFT_ERANGE;
    const bool wide = gold || p >= (1ull << 31);
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
    c->override_logW.store(0);
    c->batch_widen.store(1);
    c->batch_col_thr.store(kListColThreads);
    c->batch_rowmul_thr.store(kRowMulThreads);
    for (unsigned i = 0; i < kPlanBuckets; i++) c->tuned_logW[i].store(0);
    c->timing.store(false);
    c->timing_mask.store(~0u);
    c->last_batch = nullptr;
    c->last_done = nullptr;
    for (int i = 0; i < TFT_K_COUNT; i++) { c->launches[i] = 0; c->total_ms[i] = 0.0; }
    if (!wide) {
        uint32_t inv = 1;                          // p^-1 mod 2^32 by Newton iteration
        for (int i = 0; i < 5; i++) inv *= 2u - (uint32_t)p * inv;
        c->m32.p = (uint32_t)p;
        c->m32.pneg = (uint32_t)(0u - inv);
        c->m32.r2 = (uint32_t)(((u128)1 << 64) % p);
        c->m32.halfp1 = (uint32_t)((p + 1) / 2);
    } else if (!gold) {
        uint64_t inv = 1;                          // p^-1 mod 2^64 by Newton iteration
        for (int i = 0; i < 6; i++) inv *= 2u - p * inv;
        c->mm64.p = p;
        c->mm64.pneg = 0u - inv;
        const uint64_t r1 = (uint64_t)(((u128)1 << 64) % p);
        c->mm64.r2 = (uint64_t)((u128)r1 * r1 % p);
        c->mm64.halfp1 = (p + 1) / 2;
    }
    c->n1 = size_t(1) << kB1;
    c->n2 = c->v > (unsigned)kB1 ? size_t(1) << (c->v - kB1) : 1;
    DeviceGuard guard(device);
    size_t bytes = 0;
    hipError_t e = noalloc_setup(device);
    if (e != hipSuccess) {
        delete c;
        return TFT_EDEVICE;
    }
    if (wide) {
        auto t = build_tables<uint64_t>(p, g, c->v, c->n1, c->n2, !gold);
        bytes = t.size() * 8;
        e = hipMalloc(&c->tables, bytes);
        if (e == hipSuccess) e = hipMemcpy(c->tables, t.data(), bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess && !(gold ? set_lds_limits<tft::ModGL>() : set_lds_limits<tft::ModM64>()))
            e = hipErrorInvalidValue;
    } else {
        auto t = build_tables<uint32_t>(p, g, c->v, c->n1, c->n2, true);
        bytes = t.size() * 4;
        e = hipMalloc(&c->tables, bytes);
        if (e == hipSuccess) e = hipMemcpy(c->tables, t.data(), bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess && !set_lds_limits<tft::ModU32>()) e = hipErrorInvalidValue;
    }
    c->varea = c->fold = nullptr;
    if (e == hipSuccess) e = hipMalloc(&c->varea, kScratchWords * c->wbytes);
    if (e == hipSuccess) e = hipMalloc(&c->fold, kFoldWords * c->wbytes);
    if (e != hipSuccess) {
        if (c->tables) (void)hipFree(c->tables);
        if (c->varea) (void)hipFree(c->varea);
        delete c;
        return e == hipErrorOutOfMemory ? TFT_ENOMEM : TFT_EDEVICE;
    }
    *out = c;
    return TFT_OK;
}

void tft_ctx_destroy(tft_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard guard(ctx->device);
    if (ctx->last_batch) {
        (void)hipEventSynchronize(ctx->last_done);
        batch_free(ctx->last_batch);
    }
    if (ctx->last_done) (void)hipEventDestroy(ctx->last_done);
    arena_free(&ctx->once_arena);
    (void)hipFree(ctx->tables);
    (void)hipFree(ctx->varea);
    (void)hipFree(ctx->fold);
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
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        auto* x = (typename Mod::Word*)X;
        return forward_impl<Mod>(ctx, x, n, x, n, st);
    });
}

tft_status tft_inverse(tft_ctx* ctx, void* X, size_t n, void* stream) {
    if (!ctx || !X) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        return inverse_impl<Mod>(ctx, (typename Mod::Word*)X, nullptr, n, st);
    });
}

tft_status tft_pointwise_mul(tft_ctx* ctx, void* X, const void* Y, size_t n, void* stream) {
    if (!ctx || !X || !Y || n == 0) return TFT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        using Word = typename Mod::Word;
        return pointwise_impl<Mod>(ctx, (Word*)X, (const Word*)Y, n, st);
    });
}

tft_status poly_mul(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X, void* Y, void* stream) {
    if (!ctx || !A || !B || !X || m == 0 || nb == 0) return TFT_EINVAL;
    tft_status s = check_len(ctx, m + nb - 1);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        using Word = typename Mod::Word;
        return mul_impl<Mod>(ctx, (const Word*)A, m, (const Word*)B, nb, (Word*)X, (Word*)Y, st);
    });
}

tft_status poly_mul_noalloc(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X,
                            void* stream) {
    if (!ctx || !A || !B || !X || m == 0 || nb == 0) return TFT_EINVAL;
    const size_t r = m + nb - 1;
    tft_status s = check_len(ctx, r);
    if (s != TFT_OK) return s;
    if (r > kNoAllocBytes / ctx->wbytes) return TFT_ERANGE;   // beyond the fixed workspace
    void* Y = ctx->device < kMaxDevices ? g_noalloc_ptr[ctx->device].load(std::memory_order_acquire) : nullptr;
    if (!Y) return TFT_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        using Word = typename Mod::Word;
        return mul_impl<Mod>(ctx, (const Word*)A, m, (const Word*)B, nb, (Word*)X, (Word*)Y, st);
    });
}

tft_status tft_padded_forward(tft_ctx* ctx, void* X, size_t n, void* Xpad, void* stream) {
    if (!ctx || !X || !Xpad) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        using Word = typename Mod::Word;
        return padded_forward_impl<Mod>(ctx, (Word*)X, n, (Word*)Xpad, st);
    });
}

tft_status tft_padded_inverse(tft_ctx* ctx, void* X, size_t n, void* Xpad, void* stream) {
    if (!ctx || !X || !Xpad) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        using Word = typename Mod::Word;
        return padded_inverse_impl<Mod>(ctx, (Word*)X, n, (Word*)Xpad, st);
    });
}

tft_status tft_buffered_forward(tft_ctx* ctx, void* Xbuf, size_t n, void* stream) {
    if (!ctx || !Xbuf) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        auto* x = (typename Mod::Word*)Xbuf;
        return forward_impl<Mod>(ctx, x, n, x, n, st, 0, 1, true);
    });
}

tft_status tft_buffered_inverse(tft_ctx* ctx, void* Xbuf, size_t n, void* stream) {
    if (!ctx || !Xbuf) return TFT_EINVAL;
    tft_status s = check_len(ctx, n);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        return inverse_impl<Mod>(ctx, (typename Mod::Word*)Xbuf, nullptr, n, st, true);
    });
}

tft_status poly_mul_padded(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X, void* Apad,
                           void* Bpad, void* stream) {
    if (!ctx || !A || !B || !X || !Apad || !Bpad || m == 0 || nb == 0) return TFT_EINVAL;
    tft_status s = check_len(ctx, m + nb - 1);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        using Word = typename Mod::Word;
        return padded_mul_impl<Mod>(ctx, (const Word*)A, m, (const Word*)B, nb, (Word*)X, (Word*)Apad, (Word*)Bpad, st);
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
    out->row_threads = P.kind == 1 ? row_threads(P) : 0;
    out->stages_per_pass = P.smax;
    return TFT_OK;
}

tft_status tft_set_plan_override(tft_ctx* ctx, unsigned logW) {
    if (!ctx || logW > 16) return TFT_EINVAL;
    ctx->override_logW = logW;
    return TFT_OK;
}

tft_status tft_batch_create(tft_ctx* ctx, const tft_mul_desc* d, size_t count, int products, tft_batch** out) {
    return batch_create(ctx, d, count, products ? 1 : 0, out);
}

tft_status tft_batch_run(tft_batch* B, void* stream) {
    if (!B) return TFT_EINVAL;
    DeviceGuard guard(B->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    return with_mod(B->ctx, [&](auto mt) { return batch_run<decltype(mt)>(B, st); });
}

tft_status tft_batch_info(const tft_batch* B, tft_batch_desc* out) {
    if (!B || !out) return TFT_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->count = B->count;
    out->single_workgroup = B->n_small;
    out->two_pass = B->n_two;
    out->device_bytes = B->dbytes;
    uint32_t launches = B->n_small ? 1 + (B->n_big ? 1 : 0) + (B->n_small > B->n_big ? 1 : 0) : 0;
    for (int ph = 0; ph < PH_COUNT; ph++) launches += B->n_items[ph] ? 1 : 0;
    out->launches = launches;
    return TFT_OK;
}

void tft_batch_destroy(tft_batch* B) { batch_free(B); }

tft_status poly_mul_batch(tft_ctx* ctx, const tft_mul_desc* d, size_t count, void* stream) {
    if (!ctx || (count && !d)) return TFT_EINVAL;
    DeviceGuard guard(ctx->device);
    return batch_once(ctx, d, count, 1, (hipStream_t)stream);
}

tft_status tft_forward_batch(tft_ctx* ctx, void* const* X, const size_t* n, size_t count, void* stream) {
    if (!ctx || (count && (!X || !n))) return TFT_EINVAL;
    std::vector<tft_mul_desc> d(count);
    for (size_t k = 0; k < count; k++) {
        d[k] = tft_mul_desc{X[k], n[k], nullptr, 0, X[k], nullptr};
    }
    DeviceGuard guard(ctx->device);
    return batch_once(ctx, d.data(), count, 0, (hipStream_t)stream);
}

tft_status tft_walk_batch(tft_ctx* ctx, void* const* X, const size_t* n, size_t count, int inverse, void* stream) {
    if (!ctx || (count && (!X || !n)) || count > (size_t)UINT32_MAX) return TFT_EINVAL;
    for (size_t k = 0; k < count; k++) {
        if (!X[k] || n[k] == 0) return TFT_EINVAL;
        if (n[k] > tft::kWalkMax || n[k] > (size_t(1) << ctx->v)) return TFT_ERANGE;
    }
    if (!count) return TFT_OK;
    DeviceGuard guard(ctx->device);
    return with_mod(ctx, [&](auto mt) {
        return walk_impl<decltype(mt)>(ctx, X, n, count, inverse, (hipStream_t)stream);
    });
}

tft_status tft_from_signed(tft_ctx* ctx, const int64_t* src, size_t n, void* dst, void* stream) {
    if (!ctx || !src || !dst || n == 0) return TFT_EINVAL;
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    uint64_t blocks = std::min<uint64_t>((n + kThreads - 1) / kThreads, 8192);
    if (ctx->wbytes == 4)
        launch(ctx, TFT_K_COPY, tft::k_from_signed32, dim3((uint32_t)blocks), dim3(kThreads), 0, st, ctx->m32,
               (uint32_t)((1ull << 32) / ctx->p), (uint32_t*)dst, src, (uint64_t)n);
    else
        launch(ctx, TFT_K_COPY, tft::k_from_signed<uint64_t>, dim3((uint32_t)blocks), dim3(kThreads), 0, st,
               (uint64_t*)dst, src, (uint64_t)n, ctx->p);
    return launch_status();
}

tft_status tft_crt3(tft_ctx* const ctxs[3], const void* r1, const void* r2, const void* r3, size_t n, void* out,
                    void* stream) {
    if (!ctxs || !ctxs[0] || !ctxs[1] || !ctxs[2] || !r1 || !r2 || !r3 || !out || n == 0) return TFT_EINVAL;
    for (int i = 0; i < 3; i++)
        if (ctxs[i]->wbytes != 4 || ctxs[i]->device != ctxs[0]->device) return TFT_EINVAL;
    const uint64_t p1 = ctxs[0]->p, p2 = ctxs[1]->p, p3 = ctxs[2]->p;
    if (p1 == p2 || p1 == p3 || p2 == p3) return TFT_EINVAL;
    tft::Crt3 c;
    c.p1 = p1;
    c.p2 = p2;
    c.p3 = p3;
    c.m2 = ctxs[1]->m32;
    c.m3 = ctxs[2]->m32;
    const uint64_t inv12 = powmod_h(p1 % p2, p2 - 2, p2);
    const uint64_t inv123 = powmod_h(mulmod_h(p1 % p3, p2 % p3, p3), p3 - 2, p3);
    c.inv12_m = (uint32_t)(((u128)inv12 << 32) % p2);
    c.inv123_m = (uint32_t)(((u128)inv123 << 32) % p3);
    c.b2 = (uint32_t)((1ull << 32) / p2);
    c.b3 = (uint32_t)((1ull << 32) / p3);
    c.p1p2 = p1 * p2;
    c.M = (u128)p1 * p2 * p3;
    c.half_M = (c.M + 1) / 2;
    tft_ctx* ctx = ctxs[0];
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    uint64_t blocks = std::min<uint64_t>((n + kThreads - 1) / kThreads, 16384);
    launch(ctx, TFT_K_CRT, tft::k_crt3, dim3((uint32_t)blocks), dim3(kThreads), 0, st, c, (const uint32_t*)r1,
           (const uint32_t*)r2, (const uint32_t*)r3, (uint64_t*)out, (uint64_t)n);
    return launch_status();
}

tft_status tft_queue_create(tft_ctx* ctx, size_t pool_words, size_t max_inflight, tft_queue** out) {
    if (!ctx || !out || pool_words == 0 || max_inflight == 0) return TFT_EINVAL;
    *out = nullptr;
    DeviceGuard guard(ctx->device);
    tft_queue* q = new (std::nothrow) tft_queue();
    if (!q) return TFT_ENOMEM;
    q->ctx = ctx;
    q->pool_words = pool_words;
    q->max_inflight = max_inflight;
    q->max_pending = 1u << 20;
    q->max_batch = 1024;
    q->inflight_reqs = 0;
    q->next_ticket = 1;
    q->stop = false;
    for (int i = 0; i < kQueueSlots; i++) q->slot_busy[i] = false;
    q->n_submitted = q->n_completed = q->n_batches = q->n_rejected = q->max_pool_used = 0;
    q->error = TFT_OK;
    q->alloc.init(pool_words);
    hipError_t e = hipMalloc(&q->pool, pool_words * ctx->wbytes);
    for (int i = 0; i < kQueueSlots; i++) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->streams[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = arena_init(&q->arenas[i]);
    }
    if (e != hipSuccess) {
        if (q->pool) (void)hipFree(q->pool);
        for (int i = 0; i < kQueueSlots; i++) {
            if (q->streams[i]) (void)hipStreamDestroy(q->streams[i]);
            arena_free(&q->arenas[i]);
        }
        delete q;
        return e == hipErrorOutOfMemory ? TFT_ENOMEM : TFT_EDEVICE;
    }
    q->worker = std::thread(queue_worker, q);
    *out = q;
    return TFT_OK;
}

tft_status tft_queue_submit(tft_queue* q, const tft_mul_desc* d, void* hip_stream, uint64_t* ticket) {
    if (!q || !d || !ticket || !d->a || !d->b || !d->out || d->la == 0 || d->lb == 0) return TFT_EINVAL;
    const uint64_t r = d->la + d->lb - 1;
    if (log2u(r) > q->ctx->v) return TFT_ERANGE;
    const bool need_ws = needs_workspace(q->ctx, r, true);
    if (need_ws && r > q->pool_words) return TFT_ERANGE;   // could never be admitted
    const hipStream_t src = (hipStream_t)hip_stream;
    DeviceGuard guard(q->ctx->device);
    std::lock_guard<std::mutex> lk(q->mu);
    if (q->pending.size() >= q->max_pending) return TFT_EAGAIN;
    QReq rq;
    rq.d = *d;
    rq.r = r;
    rq.off = ~0ull;
    rq.src = src;
    rq.d.work = nullptr;
    // admission by in-place footprint: the r words of B's transform, reserved
    // now or refused
    if (need_ws) {
        uint64_t off;
        if (!q->alloc.alloc(r, &off)) {
            q->n_rejected++;
            return TFT_EAGAIN;
        }
        rq.off = off;
        rq.d.work = (char*)q->pool + off * q->ctx->wbytes;
        q->max_pool_used = std::max<uint64_t>(q->max_pool_used, q->alloc.used);
    }
    hipEvent_t& ev = q->src_events[src];
    hipError_t e = hipSuccess;
    if (!ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, src);
    if (e != hipSuccess) {
        if (rq.off != ~0ull) q->alloc.release(rq.off, r);
        return TFT_EDEVICE;
    }
    rq.ticket = q->next_ticket++;
    q->done_ns.push_back(0);
    q->pending.push_back(rq);
    q->n_submitted++;
    *ticket = rq.ticket;
    q->cv_work.notify_one();
    return TFT_OK;
}

tft_status tft_queue_poll(tft_queue* q, uint64_t ticket, int* done) {
    if (!q || !done) return TFT_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    *done = ticket >= 1 && ticket <= q->done_ns.size() && q->done_ns[ticket - 1] != 0;
    if (*done && q->failed.count(ticket)) return TFT_EDEVICE;
    return TFT_OK;
}

tft_status tft_queue_wait(tft_queue* q, uint64_t ticket) {
    if (!q || ticket == 0) return TFT_EINVAL;
    std::unique_lock<std::mutex> lk(q->mu);
    if (ticket >= q->next_ticket) return TFT_EINVAL;
    q->cv_done.wait(lk, [&] { return q->done_ns[ticket - 1] != 0; });
    return q->failed.count(ticket) ? TFT_EDEVICE : TFT_OK;
}

tft_status tft_queue_completion_ns(tft_queue* q, uint64_t ticket, uint64_t* ns) {
    if (!q || !ns) return TFT_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    *ns = ticket >= 1 && ticket <= q->done_ns.size() ? q->done_ns[ticket - 1] : 0;
    return TFT_OK;
}

tft_status tft_queue_stats(tft_queue* q, tft_queue_desc* out) {
    if (!q || !out) return TFT_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    out->submitted = q->n_submitted;
    out->completed = q->n_completed;
    out->batches = q->n_batches;
    out->rejected = q->n_rejected;
    out->pending = q->pending.size();
    out->inflight = q->inflight_reqs;
    out->pool_words = q->pool_words;
    out->pool_used_max = q->max_pool_used;
    return q->error;
}

void tft_queue_destroy(tft_queue* q) {
    if (!q) return;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->stop = true;
        q->cv_work.notify_one();
    }
    if (q->worker.joinable()) q->worker.join();
    DeviceGuard guard(q->ctx->device);
    for (int i = 0; i < kQueueSlots; i++) {
        (void)hipStreamDestroy(q->streams[i]);
        arena_free(&q->arenas[i]);
    }
    for (auto& kv : q->src_events)
        if (kv.second) (void)hipEventDestroy(kv.second);
    (void)hipFree(q->pool);
    delete q;
}

tft_status tft_timing_enable(tft_ctx* ctx, int on) {
    if (!ctx) return TFT_EINVAL;
    ctx->timing = on != 0;
    return TFT_OK;
}

tft_status tft_timing_select(tft_ctx* ctx, uint32_t kernel_mask) {
    if (!ctx) return TFT_EINVAL;
    ctx->timing_mask = kernel_mask;
    return TFT_OK;
}

static tft_status timing_collect(tft_ctx* ctx) {   // with timing_mu held
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
    std::lock_guard<std::mutex> lk(ctx->timing_mu);
    tft_status s = timing_collect(ctx);
    *launches = ctx->launches[id];
    *total_ms = ctx->total_ms[id];
    return s;
}

tft_status tft_timing_reset(tft_ctx* ctx) {
    if (!ctx) return TFT_EINVAL;
    DeviceGuard guard(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->timing_mu);
    tft_status s = timing_collect(ctx);
    for (int i = 0; i < TFT_K_COUNT; i++) { ctx->launches[i] = 0; ctx->total_ms[i] = 0.0; }
    return s;
}

tft_status poly_mul_restricted(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X, void* stream) {
    if (!ctx || !A || !B || !X || m == 0 || nb == 0) return TFT_EINVAL;
    tft_status s = check_len(ctx, m + nb - 1);
    if (s != TFT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    return dispatch(ctx, [&](auto mt) {
        using Mod = decltype(mt);
        using Word = typename Mod::Word;
        return mul_restricted_impl<Mod>(ctx, (const Word*)A, m, (const Word*)B, nb, (Word*)X, st);
    });
}

tft_status tft_autotune(tft_ctx* ctx, size_t n, tft_plan_desc* chosen) {
    if (!ctx || n == 0) return TFT_EINVAL;
    if (n > (1ull << ctx->v)) return TFT_ERANGE;
    DeviceGuard dg(ctx->device);
    const unsigned k = plan_bucket(n);
    const unsigned saved_tuned = ctx->tuned_logW[k].load();
    tl_ignore_cache = true;   // the planner's own choice, whatever the context holds
    const Plan base = make_plan(ctx, n);
    tft_status st = TFT_OK;
    unsigned best_code = 0;
    if (base.kind == 1) {
        void* X = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipMalloc(&X, n * ctx->wbytes) != hipSuccess) st = TFT_ENOMEM;
        if (st == TFT_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = TFT_EDEVICE;
        // canonical residues (i mod p), so that the timed kernels see real data
        if (st == TFT_OK) {
            if (ctx->wbytes == 8)
                tft::k_fill_index<uint64_t><<<1024, kThreads>>>((uint64_t*)X, n, ctx->p);
            else
                tft::k_fill_index<uint32_t><<<1024, kThreads>>>((uint32_t*)X, n, ctx->p);
            if (hipGetLastError() != hipSuccess) st = TFT_EDEVICE;
        }
        // median of five timed round trips of a candidate plan (after one
        // warm-up); +inf if the candidate is not a valid plan
        auto time_plan = [&](const PlanCode& c) -> float {
            tl_force_code = encode_plan(c);
            const Plan P = make_plan(ctx, n);
            if (P.kind != 1 || P.logW != c.logW) return 1e30f;
            float t[6];
            for (int rep = 0; rep < 6 && st == TFT_OK; rep++) {
                t[rep] = 0.f;
                if (hipEventRecord(e0, nullptr) != hipSuccess) { st = TFT_EDEVICE; break; }
                tft_status a = tft_forward(ctx, X, n, nullptr);
                tft_status b = tft_inverse(ctx, X, n, nullptr);
                if (a != TFT_OK || b != TFT_OK) { st = a != TFT_OK ? a : b; break; }
                if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    st = TFT_EDEVICE;
                    break;
                }
                (void)hipEventElapsedTime(&t[rep], e0, e1);
            }
            if (st != TFT_OK) return 1e30f;
            std::sort(t + 1, t + 6);   // t[0] is the warm-up
            return t[3];
        };
        // 1. the column width (logW) within two of the planner's, each with one
        //    and with two radix-8 units per row thread (how many rows share a
        //    CU decides whether the row pass takes one round of workgroups or
        //    two); another choice replaces the planner's only when 3 % faster,
        //    so that run-to-run noise does not move the plan
        PlanCode best{base.logW, (unsigned)base.logC, 3u, 3u};
        float best_ms = time_plan(best);
        const float base_ms = best_ms;
        const int lo = std::max<int>((int)base.logW - 2, 3), hi = std::min<int>((int)base.logW + 2, 16);
        for (int lw = lo; lw <= hi && st == TFT_OK; lw++) {
            if ((1ull << lw) >= n) continue;
            for (unsigned rl = 3; rl <= 4 && st == TFT_OK; rl++) {
                if ((unsigned)lw == base.logW && rl == 3) continue;
                PlanCode c = best;
                c.logW = (unsigned)lw;
                c.rlog = rl;
                const float ms = time_plan(c);
                if (ms < 0.97f * best_ms) {
                    best = c;
                    best_ms = ms;
                }
            }
        }
        // 2. at that width, one knob at a time: columns per tile (8 or 16),
        //    stages per LDS round trip (3 or 2); each kept only when 3 % faster
        for (int knob = 0; knob < 3 && st == TFT_OK; knob++) {
            if (knob == 1) continue;   // words per row thread: searched with the width
            PlanCode c = best;
            if (knob == 0) c.logC = c.logC == 3 ? 4u : 3u;
            if (knob == 2) c.smax = c.smax == 3 ? 2u : 3u;
            const float ms = time_plan(c);
            if (ms < 0.97f * best_ms) {
                best = c;
                best_ms = ms;
            }
        }
        (void)base_ms;
        best_code = encode_plan(best);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (X) (void)hipFree(X);
    }
    tl_force_code = 0;
    tl_ignore_cache = false;
    ctx->tuned_logW[k].store(st == TFT_OK ? best_code : saved_tuned);
    if (st == TFT_OK && chosen) st = tft_plan_info(ctx, n, chosen);
    return st;
}

tft_status tft_autotune_batch(tft_ctx* ctx, const tft_mul_desc* d, size_t count, int products, unsigned* widen) {
    if (!ctx || !d || count == 0) return TFT_EINVAL;
    DeviceGuard dg(ctx->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tft_status st = TFT_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = TFT_EDEVICE;
    // median of five timed runs of a candidate (after one warm-up run), with
    // the candidate set through the thread-local overrides
    auto time_candidate = [&](int w, int col, int rowmul, float* out) {
        tl_batch_widen = w;
        tl_batch_col_thr = col;
        tl_batch_rowmul_thr = rowmul;
        tft_batch* B = nullptr;
        st = tft_batch_create(ctx, d, count, products, &B);
        tl_batch_widen = tl_batch_col_thr = tl_batch_rowmul_thr = -1;
        if (st != TFT_OK) return;
        float t[6];
        for (int rep = 0; rep < 6 && st == TFT_OK; rep++) {
            if (hipEventRecord(e0, nullptr) != hipSuccess) st = TFT_EDEVICE;
            if (st == TFT_OK) st = tft_batch_run(B, nullptr);
            if (st == TFT_OK && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                st = TFT_EDEVICE;
            t[rep] = 0.f;
            if (st == TFT_OK) (void)hipEventElapsedTime(&t[rep], e0, e1);
        }
        tft_batch_destroy(B);
        std::sort(t + 1, t + 6);
        *out = t[3];
    };
    // first the row width at the default thread counts; another width
    // replaces the default (one step wider) only when 3 % faster
    float ms[3] = {0.f, 0.f, 0.f};
    for (int w = 0; w < 3 && st == TFT_OK; w++) time_candidate(w, (int)kListColThreads, (int)kRowMulThreads, &ms[w]);
    unsigned best = 1;
    if (st == TFT_OK)
        for (unsigned w = 0; w < 3; w++)
            if (ms[w] < 0.97f * ms[best]) best = w;
    // then, at that width, the column-list and fused-row workgroup sizes
    // (likewise kept only when 3 % faster than the defaults)
    static const int kCols[] = {128, 256}, kRows[] = {128, 256};
    int best_col = (int)kListColThreads, best_row = (int)kRowMulThreads;
    float best_ms = ms[best];
    for (int c : kCols)
        for (int r : kRows) {
            if (st != TFT_OK || (c == (int)kListColThreads && r == (int)kRowMulThreads)) continue;
            float t = 0.f;
            time_candidate((int)best, c, r, &t);
            if (st == TFT_OK && t < 0.97f * ms[best] && t < best_ms) {
                best_ms = t;
                best_col = c;
                best_row = r;
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != TFT_OK) return st;
    ctx->batch_widen.store(best);
    ctx->batch_col_thr.store((unsigned)best_col);
    ctx->batch_rowmul_thr.store((unsigned)best_row);
    if (widen) *widen = best;
    return TFT_OK;
}

tft_status tft_batch_tuning_get(const tft_ctx* ctx, tft_batch_tuning* out) {
    if (!ctx || !out) return TFT_EINVAL;
    out->widen = ctx->batch_widen.load();
    out->list_col_threads = ctx->batch_col_thr.load();
    out->row_mul_threads = ctx->batch_rowmul_thr.load();
    return TFT_OK;
}

tft_status tft_plan_cache_get(tft_ctx* ctx, unsigned bucket, unsigned* code) {
    if (!ctx || !code || bucket >= kPlanBuckets) return TFT_EINVAL;
    *code = ctx->tuned_logW[bucket];
    return TFT_OK;
}

tft_status tft_plan_cache_set(tft_ctx* ctx, unsigned bucket, unsigned code) {
    if (!ctx || bucket >= kPlanBuckets || (code & 31u) > 16 || code >> 13) return TFT_EINVAL;
    ctx->tuned_logW[bucket] = code;
    return TFT_OK;
}

unsigned tft_plan_bucket(size_t n) { return n ? plan_bucket(n) : 0u; }

tft_status tft_calibrate(tft_ctx* ctx, tft_calibration* out) {
    if (!ctx || !out) return TFT_EINVAL;
    DeviceGuard dg(ctx->device);
    const uint32_t blocks = 8192;
    const size_t lanes = (size_t)blocks * tft::kCalThreads;
    const uint64_t copy_words = uint64_t(1) << 24;   // 256 MiB each way in 16-byte words
    void *o = nullptr, *x = nullptr, *tw = nullptr, *src = nullptr, *dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tft_status st = TFT_OK;
    auto ok = [&](hipError_t e) { if (e != hipSuccess && st == TFT_OK) st = TFT_EDEVICE; return st == TFT_OK; };
    ok(hipMalloc(&o, lanes * 4));
    ok(hipMalloc(&x, lanes * 8 * ctx->wbytes));
    ok(hipMalloc(&tw, 8 * ctx->wbytes));
    ok(hipMalloc(&src, copy_words * 16));
    ok(hipMalloc(&dst, copy_words * 16));
    ok(hipEventCreate(&e0));
    ok(hipEventCreate(&e1));
    if (st == TFT_OK) {
        ok(hipMemset(x, 1, lanes * 8 * ctx->wbytes));   // residues 0x0101.. < p for both word sizes
        ok(hipMemset(tw, 3, 8 * ctx->wbytes));
        ok(hipMemset(src, 7, copy_words * 16));
    }
    // time one launch (after one warm-up launch of the same kernel)
    auto timed = [&](auto&& run) -> double {
        if (st != TFT_OK) return 0.0;
        run();
        ok(hipEventRecord(e0, nullptr));
        run();
        ok(hipEventRecord(e1, nullptr));
        ok(hipEventSynchronize(e1));
        float ms = 0.f;
        ok(hipEventElapsedTime(&ms, e0, e1));
        ok(hipGetLastError());
        return ms > 0.f ? ms * 1e-3 : 0.0;
    };
    const int it_alu = 4000, it_bf = 400;
    const double t_valu = timed([&] { tft::k_cal_valu<<<blocks, tft::kCalThreads>>>((uint32_t*)o, 3u, it_alu); });
    const double t_mad = timed([&] { tft::k_cal_mad64<<<blocks, tft::kCalThreads>>>((uint32_t*)o, 3u, it_alu); });
    const double t_bf = timed([&] {
        (void)with_mod(ctx, [&](auto mt) {
            using Mod = decltype(mt);
            using Word = typename Mod::Word;
            tft::k_cal_bfly<Mod><<<blocks, tft::kCalThreads>>>(mod_of<Mod>(ctx), (Word*)x, (const Word*)tw, it_bf);
            return TFT_OK;
        });
    });
    auto xchg = [&](auto mode) {
        return timed([&] {
            (void)with_mod(ctx, [&](auto mt) {
                using Mod = decltype(mt);
                using Word = typename Mod::Word;
                tft::k_cal_xchg<Mod, decltype(mode)::value><<<blocks, tft::kCalThreads>>>(
                    mod_of<Mod>(ctx), (Word*)x, (const Word*)tw, it_bf);
                return TFT_OK;
            });
        });
    };
    const double t_xl = xchg(std::integral_constant<int, 0>{});
    const double t_xb = xchg(std::integral_constant<int, 1>{});
    const double t_xd = xchg(std::integral_constant<int, 2>{});
    const double t_copy = timed([&] {
        tft::k_cal_copy<<<2048, tft::kCalThreads>>>((uint4*)dst, (const uint4*)src, copy_words);
    });
    if (st == TFT_OK && t_valu > 0 && t_mad > 0 && t_bf > 0 && t_xl > 0 && t_xb > 0 && t_xd > 0 && t_copy > 0) {
        out->valu_tops = (double)lanes * it_alu * 8 / t_valu / 1e12;
        out->mad64_tops = (double)lanes * it_alu * 8 / t_mad / 1e12;
        out->butterflies_g = (double)lanes * it_bf * 12 / t_bf / 1e9;
        out->butterflies_lds_xchg_g = (double)lanes * it_bf * 12 / t_xl / 1e9;
        out->butterflies_bpermute_xchg_g = (double)lanes * it_bf * 12 / t_xb / 1e9;
        out->butterflies_dpp_xchg_g = (double)lanes * it_bf * 12 / t_xd / 1e9;
        out->copy_gbs = 2.0 * 16.0 * (double)copy_words / t_copy / 1e9;
    } else if (st == TFT_OK) {
        st = TFT_EDEVICE;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void* q : {o, x, tw, src, dst})
        if (q) (void)hipFree(q);
    return st;
}

const char* tft_kernel_name(int id) {
    static const char* names[TFT_K_COUNT] = {"small_fwd", "small_inv", "small_mul", "col_fwd", "row_fwd",
                                             "row_inv", "col_inv_short", "last_inv", "col_inv_long",
                                             "pointwise", "copy_pad", "small_list", "crt3", "col_fix", "fold"};
    return (id >= 0 && id < TFT_K_COUNT) ? names[id] : "unknown";
}

}  // extern "C"
