/*
 * libtft — in-place truncated Fourier transform over Z/pZ on one AMD MI355X
 * (gfx950) GPU, after D. Harvey and D. S. Roche, "An in-place truncated
 * Fourier transform and applications to polynomial multiplication" (2010).
 *
 * Notation (paper, section 2.2): w[k] is a primitive 2^k-th root of unity and
 * the roots are compatible, w[k+1]^2 = w[k]; here w[k] = g^((p-1)/2^k) for
 * the generator g given at context creation.  w_s = w[k]^(rev_k s) for any
 * k >= bitlen(s), and the transform of a polynomial F of degree < n is
 * F^_s = F(w_s), 0 <= s < n: the first n outputs of the length-2^ceil(lg n)
 * DFT in bit-reversed order (section 1.2).
 *
 * Words.  A context for a prime p < 2^31 works on uint32_t words; the context
 * for p = 2^64 - 2^32 + 1 works on uint64_t words.  Every data argument is a
 * device pointer to canonical residues in [0, p); results are canonical.
 * Results are exact (no rounding), so they are bit-identical to any other
 * correct implementation.
 *
 * Memory.  The caller owns every data buffer.  The transforms run in place on
 * the n words given: there is no padding to 2^ceil(lg n) and no per-call
 * allocation.  A context owns only constant tables (two-level root tables,
 * independent of n) and one fixed scratch area (the "extra evaluations" of the
 * partial last row, at most 2^16 words, independent of n).  Calls that share
 * a context must therefore be ordered: issue them on one stream, or
 * synchronise between streams.  All work is enqueued on the caller's stream
 * (a hipStream_t passed as void*; NULL is the default stream) and the calls
 * return without waiting for it.
 *
 * Errors.  Functions return a tft_status and never throw.  Argument errors are
 * detected on the host before anything is enqueued; a launch failure reports
 * TFT_EDEVICE.  Asynchronous device faults surface at the caller's next
 * synchronisation, as for any HIP kernel.
 */
#ifndef LIBTFT_H
#define LIBTFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TFT_OK = 0,
    TFT_EINVAL = -1,   /* null pointer, zero length, bad generator */
    TFT_ERANGE = -2,   /* length above 2^v (v = 2-adic order of p-1) or above the library's limit; unsupported p */
    TFT_ENOMEM = -3,   /* context or queue allocation failed */
    TFT_EDEVICE = -4,  /* a HIP call failed */
    TFT_EAGAIN = -5    /* queue: the request does not fit the free pool now (or the pending list is full) */
} tft_status;

typedef struct tft_ctx tft_ctx;

/* Create a context for prime p with generator g of (Z/pZ)^* on HIP device
 * `device` (section 2.1: the ring needs 2^k-th roots of unity and 2 must be a
 * unit).  Supported: odd primes p < 2^31 (words of 4 bytes, 32-bit
 * Montgomery arithmetic), p = 2^64-2^32+1 (8-byte words, reduction by
 * 2^64 = 2^32 - 1 and 2^96 = -1), and the other odd primes 2^31 < p < 2^63
 * (8-byte words, 64-bit Montgomery arithmetic); any other p is TFT_ERANGE.
 * g must generate the 2-part of the group: g^((p-1)/2) = -1.  On success
 * *out owns device tables of about 1 MiB; release it with tft_ctx_destroy. */
tft_status tft_ctx_create(uint64_t p, uint64_t g, int device, tft_ctx** out);
void tft_ctx_destroy(tft_ctx* ctx);

/* v = 2-adic order of p-1, capped at 28 (the library's limit): every length n must
 * satisfy n <= 2^v (section 6: a root of order 2^ceil(lg n) is needed). */
unsigned tft_ctx_max_log2(const tft_ctx* ctx);
/* 4 (uint32_t words) or 8 (uint64_t words). */
unsigned tft_ctx_word_bytes(const tft_ctx* ctx);

/* InplaceTFT (section 3, Algorithm 1; Proposition 3.2): X[0..n) holds F_0..F_{n-1}
 * on entry and F^_0..F^_{n-1} on exit.  X is a device pointer to n words. */
tft_status tft_forward(tft_ctx* ctx, void* X, size_t n, void* hip_stream);

/* InplaceITFT (section 4, Algorithm 2; Proposition 4.2): the inverse map,
 * X[0..n) holds F^_0..F^_{n-1} on entry and F_0..F_{n-1} on exit. */
tft_status tft_inverse(tft_ctx* ctx, void* X, size_t n, void* hip_stream);

/* X[i] <- X[i] * Y[i] mod p for i < n (the pointwise step of section 5). */
tft_status tft_pointwise_mul(tft_ctx* ctx, void* X, const void* Y, size_t n, void* hip_stream);

/* Product C = A B (section 5: A has m coefficients, B has nb; the output has
 * r = m + nb - 1 coefficients).  A and B are read only.  X (r words) receives
 * C; Y (r words) is caller-owned workspace holding B's transform, required
 * unless r fits the single-workgroup path (then it may be NULL).  The path is
 * transform A and B in r slots each, multiply pointwise, inverse-transform X. */
tft_status poly_mul(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X, void* Y,
                    void* hip_stream);

/* poly_mul for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product C = A B into X (r = m + nb - 1 words), bit-identical to
 * poly_mul's, with B's transform held in a fixed library-owned device array
 * of 32 MiB per device (allocated when the library is loaded, kept until the
 * process ends) instead of the caller's workspace Y.  The call allocates and
 * frees nothing (outside measurement mode, tft_timing_enable).  Limit: r <= 2^22 words for 8-byte contexts and r <= 2^23
 * for 4-byte contexts; a longer product returns TFT_ERANGE before any work is
 * enqueued.  Every call on one device shares that device's array and leaves
 * its contents behind (each call overwrites the r words it uses before reading
 * them): calls on one device must not overlap -- issue them on one stream, or
 * synchronise between streams; overlapping calls race and give wrong results.
 * TFT_EDEVICE if the array's device address could not be obtained when the
 * context was created.  Other errors as for poly_mul. */
tft_status poly_mul_noalloc(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X,
                            void* hip_stream);

/* Space-restricted product (section 5, Algorithm 3; Proposition 5.1): the same
 * C = A B with X (r = m + nb - 1 words) as the only memory of the product's
 * size written -- no workspace.  For q = 0, L_0, L_0 + L_1, ... (L the largest
 * power of two with q + 2L <= r) A and B are folded modulo x^L - w_{q/L} into
 * X[q, q+L) and X[q+L, q+2L), both blocks are transformed (their values are
 * A^_{q+i} and B^_{q+i}) and multiplied into X[q, q+L).  Once fewer than 2^18
 * positions remain, they lie in at most two aligned nodes of the transform
 * tree; A and B are folded once per node into a fixed area of the context
 * (four nodes of at most 2^17 words, allocated with the context) and the
 * node values are multiplied into X[q, r).  Then the inverse TFT of length r.
 * Each fold reads a whole operand, so this path moves more memory than
 * poly_mul in exchange for the r-word footprint.  Calls on one context share
 * its fold area: issue them on one stream.  Errors as for poly_mul. */
tft_status poly_mul_restricted(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X,
                               void* hip_stream);

/* Comparator, not the method: the ordinary padded radix-2 transform
 * (section 1.1) that the TFT smooths.  With N = 2^ceil(lg n):
 * tft_padded_forward copies X[0..n) into Xpad (N caller-owned words),
 * zero-fills Xpad[n..N), runs the length-N transform in Xpad and copies the
 * first n outputs back to X (the same values tft_forward produces), leaving
 * all N outputs in Xpad.  tft_padded_inverse takes those N outputs in Xpad,
 * runs the length-N inverse there and copies the first n coefficients to X.
 * Time and memory jump at powers of two, which is what it is measured for. */
tft_status tft_padded_forward(tft_ctx* ctx, void* X, size_t n, void* Xpad, void* hip_stream);
tft_status tft_padded_inverse(tft_ctx* ctx, void* X, size_t n, void* Xpad, void* hip_stream);

/* Comparator, not the method: van der Hoeven's buffered TFT and ITFT (section
 * 1.2), which compute the same map as tft_forward / tft_inverse but operate in
 * a buffer of 2^ceil(lg n) words and keep intermediate results in its
 * 2^ceil(lg n) - n cells beyond the data.  Here the buffer holds the row /
 * column schedule's extra evaluations of the partial last row (at
 * Xbuf + a W, the cells after the data) instead of the context's area, and
 * the inverse finishes the columns c < b after the last row.  Xbuf is a device
 * pointer to 2^ceil(lg n) words: the first n hold the input on entry and the
 * result on exit, the others are working space (unspecified on exit).
 * Results are bit-identical to tft_forward / tft_inverse; the point of
 * comparison is the memory (2^ceil(lg n) words instead of n). */
tft_status tft_buffered_forward(tft_ctx* ctx, void* Xbuf, size_t n, void* hip_stream);
tft_status tft_buffered_inverse(tft_ctx* ctx, void* Xbuf, size_t n, void* hip_stream);

/* Padded product for comparison: A and B zero-extended to N = 2^ceil(lg r)
 * words in Apad and Bpad (caller-owned), N-point transforms, pointwise
 * product, N-point inverse, first r coefficients to X. */
tft_status poly_mul_padded(tft_ctx* ctx, const void* A, size_t m, const void* B, size_t nb, void* X, void* Apad,
                           void* Bpad, void* hip_stream);

/* ---------------------------------------------------------------- batches
 * Many independent products (or forward transforms) of uneven lengths.  A
 * descriptor names one product C = A B as in poly_mul: a (la words) and b (lb
 * words) read only, out (la + lb - 1 words) receives C, work (la + lb - 1
 * words) is caller workspace, required only when the product is too long for
 * the single-workgroup path (NULL otherwise).  For forward transforms a
 * descriptor names X = a = out with n = la; b, lb and work are ignored.
 *
 * tft_batch_create plans the batch and uploads its work lists (it allocates
 * device memory and waits for the upload); tft_batch_run only enqueues kernels
 * on the stream -- products short enough for LDS run as a persistent kernel
 * that takes the next instance (longest first) from an atomic counter, the
 * others as one launch per pass over a work list of (instance, tile) items --
 * so a run can be captured in a HIP graph and replayed.  The descriptors'
 * buffers must stay valid while runs are in flight; one batch must not run
 * concurrently with itself.  poly_mul_batch and tft_forward_batch plan and
 * run in one call, with work-list memory the context keeps and grows (each
 * call first waits for the previous such call's batch to finish on the
 * device); the batch is kept by the context until its next such call. */
typedef struct {
    const void* a;
    size_t la;
    const void* b;
    size_t lb;
    void* out;
    void* work;
} tft_mul_desc;
typedef struct tft_batch tft_batch;
typedef struct {
    size_t count, single_workgroup, two_pass, device_bytes;
    unsigned launches;
} tft_batch_desc;
tft_status tft_batch_create(tft_ctx* ctx, const tft_mul_desc* d, size_t count, int products, tft_batch** out);
tft_status tft_batch_run(tft_batch* batch, void* hip_stream);
tft_status tft_batch_info(const tft_batch* batch, tft_batch_desc* out);
void tft_batch_destroy(tft_batch* batch);
tft_status poly_mul_batch(tft_ctx* ctx, const tft_mul_desc* d, size_t count, void* hip_stream);
tft_status tft_forward_batch(tft_ctx* ctx, void* const* X, const size_t* n, size_t count, void* hip_stream);

/* The paper's Algorithm 1 (inverse = 0) or Algorithm 2 (inverse = 1) as a
 * sequential walk (section 3: the in-place TFT visits the even/odd tree in
 * post order with a constant number of scalars, applying the odd-length
 * correction before each odd child of an odd-length node; section 4: the ITFT
 * undoes the same steps in reverse order), one wavefront per instance: every
 * lane follows the same node and the 64 lanes share each node's butterflies
 * and the correction's sum.  An alternative to the layer-parallel
 * small-instance kernels for batches of short instances.
 * X[k] (device, n[k] words, in place), 1 <= n[k] <= 1024 and n[k] <= 2^v, else
 * TFT_EINVAL / TFT_ERANGE before any work.  The call uploads the two arrays,
 * enqueues one kernel on hip_stream and waits for it (synchronous).  Results
 * equal tft_forward / tft_inverse bit for bit. */
tft_status tft_walk_batch(tft_ctx* ctx, void* const* X, const size_t* n, size_t count, int inverse, void* hip_stream);

/* ---------------------------------------------------------------- serving
 * A request queue with continuous batching (products as in poly_mul, section
 * 5, arriving one at a time).  tft_queue_create allocates a device pool of
 * pool_words words and starts a worker thread.
 *
 * tft_queue_submit offers a product (a tft_mul_desc; its work field is
 * ignored: workspace comes from the pool).  Admission is by in-place
 * footprint: a product that needs workspace (one too long for the
 * single-workgroup path) reserves r = la + lb - 1 words of the pool -- not
 * 2^ceil(lg r) -- at submit, and submit returns TFT_EAGAIN at once, leaving
 * nothing queued, when those words do not fit in the pool's free space now
 * (retry after earlier tickets complete), TFT_ERANGE when they could never
 * fit (r > pool_words) or r > 2^v, and TFT_EAGAIN also when 2^20 requests are
 * pending.  On success it returns a ticket without waiting.  hip_stream is
 * the stream that produces the operands (NULL: the default stream): submit
 * records an event on it, and the batch that runs the request waits for that
 * event on the device, so operands still being written by earlier work on
 * that stream are read only once it has finished.  A, B and out must stay
 * valid and untouched by other work until the ticket completes.
 *
 * The worker takes pending requests in arrival order while fewer than
 * max_inflight are on the device; each group taken together runs as one
 * batch, and up to three consecutive batches run on their own streams so
 * that they overlap on the device; each stream keeps the device and pinned
 * host memory of its
 * batches' work lists, grown as needed, so a batch in steady state allocates
 * and frees nothing.  poll reports completion without blocking; wait blocks;
 * completion_ns gives the steady-clock time (ns) at which the worker saw the
 * request complete (0 while pending); the queue keeps that time, 8 bytes per
 * request ever submitted, until it is destroyed.  A request whose batch
 * failed reports TFT_EDEVICE.  stats: `rejected` counts submits refused for
 * footprint.  destroy waits for all submitted requests. */
typedef struct tft_queue tft_queue;
typedef struct {
    uint64_t submitted, completed, batches, rejected, pending, inflight, pool_words, pool_used_max;
} tft_queue_desc;
tft_status tft_queue_create(tft_ctx* ctx, size_t pool_words, size_t max_inflight, tft_queue** out);
tft_status tft_queue_submit(tft_queue* q, const tft_mul_desc* d, void* hip_stream, uint64_t* ticket);
tft_status tft_queue_poll(tft_queue* q, uint64_t ticket, int* done);
tft_status tft_queue_wait(tft_queue* q, uint64_t ticket);
tft_status tft_queue_completion_ns(tft_queue* q, uint64_t ticket, uint64_t* ns);
tft_status tft_queue_stats(tft_queue* q, tft_queue_desc* out);
void tft_queue_destroy(tft_queue* q);

/* ------------------------------------------------ exact integer products
 * tft_from_signed: dst[i] = src[i] mod p in [0, p) for n signed 64-bit inputs
 * (src on the device, dst n words of ctx's width).
 * tft_crt3: Chinese remaindering of three residue vectors r1, r2, r3 (n words
 * each, modulo the primes of ctxs[0..2], all 31-bit word contexts on one
 * device) into the signed representatives in [-M/2, M/2), M = p1 p2 p3, as
 * n little-endian 128-bit integers (16 n bytes at out).  With products of
 * signed inputs whose exact coefficients lie in that range this recovers the
 * integer product exactly. */
tft_status tft_from_signed(tft_ctx* ctx, const int64_t* src, size_t n, void* dst, void* hip_stream);
tft_status tft_crt3(tft_ctx* const ctxs[3], const void* r1, const void* r2, const void* r3, size_t n, void* out,
                    void* hip_stream);

/* Schedule chosen for length n (for tests and benchmarks).  kind 0: the
 * single-workgroup path (whole transform in LDS); kind 1: the two-pass path
 * with n = a W + b, W = 2^logW columns of the tree at depth logW (paper,
 * section 3: node (c, logW) is the strided subarray X_{c + i W}). */
typedef struct {
    int kind;
    unsigned logW;
    size_t W, a, b;
    size_t col_block;      /* power-of-two LDS block per column */
    unsigned cols_per_tile;
    size_t lds_bytes_col, lds_bytes_row;
    unsigned row_threads;      /* threads of a row workgroup (W/8: one radix-8 unit each; W/16: two) */
    unsigned stages_per_pass;  /* most butterfly stages per LDS round trip (1..3) */
} tft_plan_desc;
tft_status tft_plan_info(tft_ctx* ctx, size_t n, tft_plan_desc* out);

/* Force the two-pass path with column width 2^logW for every length n > 2^logW
 * (0 restores the planner's choice).  Used by the tuner and by tests that
 * exercise many tiles at small n; any valid choice gives the same result.
 * Lengths whose tiles would not fit in LDS then return TFT_ERANGE. */
tft_status tft_set_plan_override(tft_ctx* ctx, unsigned logW);

/* Autotuner.  Times forward + inverse round trips of length n on the device
 * (on a buffer of n words the call allocates and frees, filled with i mod p;
 * synchronous; median of five after a warm-up) for candidate plans, and
 * records the fastest in the context's plan cache for every length in the
 * same bucket, floor(4 lg n) (quarter octaves).  Candidates: first the column
 * width 2^logW within two of the planner's choice, then, at that width, one
 * knob at a time -- columns per tile (8 or 16), words per row thread (8 or 16:
 * one or two radix-8 units, which changes how many rows share a CU) and
 * butterfly stages per LDS round trip (3 or 2).  A candidate replaces the
 * current choice only when it is 3 % faster.  Later single-transform calls
 * (tft_forward, tft_inverse, poly_mul and the products built on them) plan
 * with the cached choice; batches and the serving queue keep their own
 * shape.  Any plan gives the same results.  Lengths the planner runs in one
 * workgroup are left to the planner (cache entry 0).  `chosen` (may be NULL)
 * receives the resulting plan.  The cache is plain data: tft_plan_cache_get /
 * set read and write the entry of a bucket, a plan code with log2 W in bits
 * 0-4 (0: the planner's choice), log2 columns per tile in bits 5-7, log2 words
 * per row thread in bits 8-10 and stages per LDS round trip in bits 11-12 (0
 * in a field: the default), so that a caller can store tuned plans and load
 * them into a new context; tft_plan_bucket gives the bucket of a length:
 * floor(4 lg n) (quarter octaves), and 4 * 28 + 4 + k for n = 2^k (a power
 * of two has no partial last row, so it keeps a plan of its own). */
tft_status tft_autotune(tft_ctx* ctx, size_t n, tft_plan_desc* chosen);
/* Batch autotuner.  Runs the batch of `count` descriptors (as tft_batch_create
 * and tft_batch_run would: products if `products`, else forward transforms)
 * with the rows of its two-pass instances at the balanced split of each
 * length, one step wider (the default) and two steps wider, timing each (median
 * of five runs after a warm-up; synchronous), and keeps the fastest -- a change
 * from the default only when 3 % faster -- for every later batch of the context,
 * the serving queue's included.  Then, at that width, it times the workgroup
 * sizes of a standalone batch's column lists (at most 128 or 256 threads;
 * default 128) and fused row products (at least 128 or 256; default 128) and
 * keeps the fastest pair on the same 3 % rule.  The descriptors' outputs are
 * written by the runs (products: the products themselves; forward transforms:
 * transformed several times over, so pass scratch copies).  *widen (may be
 * NULL) receives the width choice, 0..2; tft_batch_tuning_get reports all
 * three.  Any choice gives the same results. */
tft_status tft_autotune_batch(tft_ctx* ctx, const tft_mul_desc* d, size_t count, int products, unsigned* widen);
typedef struct {
    unsigned widen;              /* rows this many steps wider than balanced, 0..2 */
    unsigned list_col_threads;   /* column-list workgroups of a standalone batch, at most */
    unsigned row_mul_threads;    /* fused row-product workgroups of a standalone batch, at least */
} tft_batch_tuning;
/* The context's current batch settings (the defaults until tft_autotune_batch
 * changes them).  EINVAL for NULL arguments. */
tft_status tft_batch_tuning_get(const tft_ctx* ctx, tft_batch_tuning* out);
tft_status tft_plan_cache_get(tft_ctx* ctx, unsigned bucket, unsigned* code);
tft_status tft_plan_cache_set(tft_ctx* ctx, unsigned bucket, unsigned code);
unsigned tft_plan_bucket(size_t n);

/* Measurement mode.  While enabled, each kernel a context launches is
 * bracketed by two HIP events recorded on the caller's stream, so that a
 * benchmark can report per-kernel durations measured live (the events are
 * created on first use and kept by the context; this mode is for
 * measurement, not for production loops).  tft_timing_read waits for the
 * events recorded so far and returns, for kernel `id`, the number of launches
 * and their summed duration in milliseconds since the last tft_timing_reset. */
typedef enum {
    TFT_K_SMALL_FWD = 0,   /* single-workgroup forward */
    TFT_K_SMALL_INV,       /* single-workgroup inverse */
    TFT_K_SMALL_MUL,       /* single-workgroup product */
    TFT_K_COL_FWD,         /* forward column pass (large-stride layers) */
    TFT_K_ROW_FWD,         /* forward row pass (small-stride layers) and last row; in batched
                              products, forward rows of both operands, product and inverse rows */
    TFT_K_ROW_INV,         /* inverse row pass */
    TFT_K_COL_INV_SHORT,   /* inverse columns c >= b (single transforms with b > 0: every column on
                              its first a values), re-deriving the extra evaluations */
    TFT_K_LAST_INV,        /* inverse of the partial last row (or, for b = W - 1 with a + 1 a
                              power of two, the one short column and the last row's fix) */
    TFT_K_COL_INV_LONG,    /* inverse columns c < b (batches) */
    TFT_K_POINTWISE,       /* pointwise product */
    TFT_K_COPY,            /* zero-extending copy, counter reset, signed-to-residue */
    TFT_K_SMALL_LIST,      /* persistent single-workgroup jobs of a batch */
    TFT_K_CRT,             /* three-prime Chinese remaindering */
    TFT_K_COL_FIX,         /* inverse: rank-one completion of the columns c < b */
    TFT_K_FOLD,            /* space-restricted product: operand folding */
    TFT_K_COUNT
} tft_kernel_id;
tft_status tft_timing_enable(tft_ctx* ctx, int on);
/* Restrict measurement mode to the kernels whose bit (1u << tft_kernel_id)
 * is set in kernel_mask (default: every kernel).  Each bracketed launch adds
 * two event records to the stream, which cost time of their own; a benchmark
 * that times one kernel class brackets only that one. */
tft_status tft_timing_select(tft_ctx* ctx, uint32_t kernel_mask);
tft_status tft_timing_read(tft_ctx* ctx, int id, uint64_t* launches, double* total_ms);
tft_status tft_timing_reset(tft_ctx* ctx);
const char* tft_kernel_name(int id);

/* Roofline denominators measured on the context's device.  Not an operation
 * of the paper: the peaks that benchmarks report the transform kernels
 * against, each from a register-only or copy-only kernel timed with HIP
 * events (the call allocates and frees its own buffers, about 0.5 GiB, and
 * waits for the device; a few tens of milliseconds):
 *   valu_tops      32-bit integer VALU operations per second / 10^12
 *                  (chains of v_xad_u32);
 *   mad64_tops     32 x 32 + 64 -> 64 multiply-adds per second / 10^12;
 *   butterflies_g  butterflies per second / 10^9 with the context's modular
 *                  arithmetic, in registers (radix-8 units, no memory traffic);
 *   copy_gbs       HBM copy bandwidth, bytes read + written per second / 10^9;
 *   butterflies_lds_xchg_g, butterflies_bpermute_xchg_g, butterflies_dpp_xchg_g
 *                  the butterfly rate of butterflies_g when every radix-8 unit
 *                  is followed by an 8 x 8 transpose among eight lanes: through
 *                  LDS (as the pass kernels exchange values between their
 *                  units), with lane shuffles (ds_bpermute), or with DPP quad
 *                  permutations and ds_swizzle.
 * Returns TFT_EDEVICE if a kernel or allocation fails. */
typedef struct {
    double valu_tops, mad64_tops, butterflies_g, copy_gbs;
    double butterflies_lds_xchg_g, butterflies_bpermute_xchg_g, butterflies_dpp_xchg_g;
} tft_calibration;
tft_status tft_calibrate(tft_ctx* ctx, tft_calibration* out);

/* Human-readable name of a status code. */
const char* tft_strerror(tft_status s);

#ifdef __cplusplus
}
#endif
#endif /* LIBTFT_H */
