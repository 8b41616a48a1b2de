/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously correct CPU implementation of what the in-place
 * truncated Fourier transform (Harvey & Roche, "An in-place truncated Fourier
 * transform and applications to polynomial multiplication", 2010) computes,
 * plus the polynomial product built on it and the exact integer product used
 * by the three-prime CRT path.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the GPU product
 * path never calls, links or includes anything from this directory, and this
 * file includes nothing from the product.
 *
 * All arithmetic is exact: residues are kept in [0, p) as 64-bit words and
 * every product is reduced with a 128-bit remainder.  Nothing here is blocked,
 * fused or reordered beyond what the cited definitions state.
 *
 * Conventions (paper, section 2.2 "DFT notation"):
 *   w[j]  = a primitive 2^j-th root of unity, chosen compatibly
 *           (w[j+1]^2 = w[j]); here w[j] = g^((p-1)/2^j) for a generator g.
 *   w_s   = w[k]^(rev_k s) for any k >= bitlen(s)   (rev_k = k-bit reversal)
 *   F^_s  = F(w_s)                                  (the transform)
 * The TFT of length n maps F_0..F_{n-1} to F^_0..F^_{n-1}.
 *
 * Every function returns 0 on success and a negative value on a bad argument.
 * Parity status of each function (what pins it) is listed in its comment; the
 * pins live in tests/test_oracle_*.py.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;
typedef __int128 i128;

/* ---------------------------------------------------------------- ring ops */
/* Section 2.1: the ring is Z/pZ with p prime, 2^v | p-1, so 2 is a unit and
 * 2^k-th roots of unity exist for k <= v.  Pinned against Python integers. */
u64 or_mulmod(u64 a, u64 b, u64 p) { return (u64)(((u128)a * (u128)b) % p); }
u64 or_addmod(u64 a, u64 b, u64 p) { return (u64)(((u128)a + (u128)b) % p); }
u64 or_submod(u64 a, u64 b, u64 p) { return (u64)(((u128)a + (u128)(p - b)) % p); }

u64 or_powmod(u64 a, u64 e, u64 p)
{
    u64 r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = or_mulmod(r, a, p);
        a = or_mulmod(a, a, p);
        e >>= 1;
    }
    return r;
}

/* Inverse by Fermat's little theorem (p prime). */
u64 or_invmod(u64 a, u64 p) { return or_powmod(a, p - 2, p); }

/* v = 2-adic valuation of p-1: the largest k with 2^k | p-1. */
unsigned or_two_adic(u64 p)
{
    u64 q = p - 1;
    unsigned v = 0;
    while (q && !(q & 1)) { q >>= 1; v++; }
    return v;
}

/* -------------------------------------------------------------- roots */
/* Section 2.2: w[j] = g^((p-1)/2^j), 0 <= j <= v.  Pinned: w[1] = p-1,
 * w[j+1]^2 = w[j], w[v] has order exactly 2^v. */
u64 or_root_chain(u64 p, u64 g, unsigned j) { return or_powmod(g, (p - 1) >> j, p); }

/* k-bit reversal of s (s < 2^k). */
u64 or_rev(u64 s, unsigned k)
{
    u64 r = 0;
    for (unsigned i = 0; i < k; i++) {
        r = (r << 1) | (s & 1);
        s >>= 1;
    }
    return r;
}

unsigned or_bitlen(u64 s)
{
    unsigned k = 0;
    while (s) { k++; s >>= 1; }
    return k;
}

/* Section 2.2: w_s = w[k]^(rev_k s) with k = bitlen(s) (k = 0 gives w_0 = 1).
 * Pinned against the table printed in section 2.2 (w_0..w_7) and the
 * identities w_{2s+1} = -w_{2s}, w_{2s}^2 = w_s. */
u64 or_omega(u64 p, u64 g, u64 s)
{
    unsigned k = or_bitlen(s);
    return or_powmod(or_root_chain(p, g, k), or_rev(s, k), p);
}

/* Same root with an explicit, possibly larger, k (compatibility check). */
u64 or_omega_k(u64 p, u64 g, u64 s, unsigned k)
{
    return or_powmod(or_root_chain(p, g, k), or_rev(s, k), p);
}

/* Table w_0..w_{n-1}. */
int or_omega_table(u64 p, u64 g, u64 n, u64 *out)
{
    if (!out && n) return -1;
    for (u64 s = 0; s < n; s++) out[s] = or_omega(p, g, s);
    return 0;
}

static int n_ok(u64 p, u64 n)
{
    /* the transform needs a root of order 2^ceil(lg n) (section 6) */
    if (n == 0) return 0;
    unsigned k = or_bitlen(n - 1);
    return k <= or_two_adic(p);
}

/* Horner evaluation F(z) = sum_{t<n} F_t z^t.  Pinned against Python. */
u64 or_eval(u64 p, const u64 *F, u64 n, u64 z)
{
    u64 acc = 0;
    for (u64 t = n; t-- > 0;) acc = or_addmod(or_mulmod(acc, z, p), F[t] % p, p);
    return acc;
}

/* ----------------------------------------------------- O3: direct TFT */
/* The definition itself (section 2.2, the transform F^_s = F(w_s)) for the
 * output indices s < n: one Horner evaluation per output, O(n^2).  Pinned by
 * hand-computed examples (tests/golden), monomial inputs, the convolution
 * theorem against numpy.convolve and the zero-padded DFT prefix property of
 * section 1.2. */
int or_tft_direct(u64 p, u64 g, const u64 *F, u64 n, u64 *X)
{
    if (!n_ok(p, n) || !F || !X || F == X) return -1;
    for (u64 s = 0; s < n; s++) X[s] = or_eval(p, F, n, or_omega(p, g, s));
    return 0;
}

/* Direct evaluation of a sample of outputs: X[i] = F(w_{idx[i]}). */
int or_tft_sample(u64 p, u64 g, const u64 *F, u64 n, const u64 *idx, u64 cnt, u64 *X)
{
    if (!n_ok(p, n) || !F || (cnt && (!idx || !X))) return -1;
    for (u64 i = 0; i < cnt; i++) {
        if (idx[i] >= n) return -2;
        X[i] = or_eval(p, F, n, or_omega(p, g, idx[i]));
    }
    return 0;
}

/* ------------------------------------------ O4: interpolation (inverse TFT) */
/* The inverse transform (section 4) recovers the unique F of degree < n with
 * F(w_s) = Y_s for s < n.  The points w_0..w_{n-1} are distinct (rev_k is a
 * bijection and w[k] is primitive), so Lagrange interpolation defines it:
 *   M(x) = prod_s (x - w_s),  M_s(x) = M(x)/(x - w_s),
 *   F = sum_s Y_s * M_s(x) / M_s(w_s).   O(n^2). */
int or_itft_lagrange(u64 p, u64 g, const u64 *Y, u64 n, u64 *F)
{
    if (!n_ok(p, n) || !Y || !F || Y == F) return -1;
    u64 *w = (u64 *)malloc(n * sizeof(u64));
    u64 *M = (u64 *)calloc(n + 1, sizeof(u64)); /* M_0 + M_1 x + ... + M_n x^n */
    u64 *Q = (u64 *)malloc(n * sizeof(u64));
    if (!w || !M || !Q) { free(w); free(M); free(Q); return -3; }
    for (u64 s = 0; s < n; s++) w[s] = or_omega(p, g, s);
    M[0] = 1;
    for (u64 s = 0; s < n; s++) {                 /* M <- M * (x - w_s) */
        for (u64 d = s + 1; d > 0; d--)
            M[d] = or_submod(M[d - 1], or_mulmod(M[d], w[s], p), p);
        M[0] = or_submod(0, or_mulmod(M[0], w[s], p), p);
    }
    memset(F, 0, n * sizeof(u64));
    for (u64 s = 0; s < n; s++) {
        /* synthetic division: Q = M / (x - w_s), exact since M(w_s) = 0 */
        u64 carry = M[n];
        for (u64 d = n; d-- > 0;) {
            Q[d] = carry;
            carry = or_addmod(M[d], or_mulmod(carry, w[s], p), p);
        }
        u64 den = or_eval(p, Q, n, w[s]);
        u64 c = or_mulmod(Y[s] % p, or_invmod(den, p), p);
        for (u64 d = 0; d < n; d++) F[d] = or_addmod(F[d], or_mulmod(c, Q[d], p), p);
    }
    free(w); free(M); free(Q);
    return 0;
}

/* ----------------------------------------------- O5: padded radix-2 FFT */
/* Section 1.1/1.2: pad to N = 2^k >= n with zeros, take an ordinary DFT of
 * length N, keep the first n outputs in bit-reversed order.  Written as the
 * textbook iterative radix-2 FFT (bit-reversal copy, then log2 N butterfly
 * stages) producing the natural-order DFT A_j = sum_t a_t w^(j t) with
 * w = w[k]; then X_s = A_{rev_k s} because w_s = w[k]^(rev_k s).  Shares no
 * code path with or_tft_direct beyond the ring ops.  O(N log N). */
static void dft_natural(u64 p, u64 *a, u64 N, unsigned k, u64 w)
{
    /* bit-reversal permutation of the input */
    for (u64 i = 0; i < N; i++) {
        u64 j = or_rev(i, k);
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (u64 len = 2; len <= N; len <<= 1) {
        u64 wl = or_powmod(w, N / len, p);      /* primitive len-th root */
        for (u64 base = 0; base < N; base += len) {
            u64 t = 1;
            for (u64 j = 0; j < len / 2; j++) {
                u64 u = a[base + j];
                u64 v = or_mulmod(a[base + j + len / 2], t, p);
                a[base + j] = or_addmod(u, v, p);
                a[base + j + len / 2] = or_submod(u, v, p);
                t = or_mulmod(t, wl, p);
            }
        }
    }
}

/* Forward: X_s = F(w_s) for s < n via the padded length-2^k DFT, where
 * k = max(ceil(lg n), kmin) (kmin lets a test ask for a longer padding). */
int or_fft_padded(u64 p, u64 g, const u64 *F, u64 n, unsigned kmin, u64 *X)
{
    if (!n_ok(p, n) || !F || !X) return -1;
    unsigned k = or_bitlen(n - 1);
    if (kmin > k) k = kmin;
    if (k > or_two_adic(p)) return -2;
    u64 N = (u64)1 << k;
    u64 *a = (u64 *)calloc(N, sizeof(u64));
    if (!a) return -3;
    for (u64 t = 0; t < n; t++) a[t] = F[t] % p;
    dft_natural(p, a, N, k, or_root_chain(p, g, k));
    for (u64 s = 0; s < n; s++) X[s] = a[or_rev(s, k)];
    free(a);
    return 0;
}

/* Inverse for n = N = 2^k only: F_t = N^-1 sum_s X_s w_s^-t. */
int or_ifft_pow2(u64 p, u64 g, const u64 *X, u64 N, u64 *F)
{
    if (!n_ok(p, N) || (N & (N - 1)) || !X || !F) return -1;
    unsigned k = or_bitlen(N - 1);
    u64 *a = (u64 *)malloc(N * sizeof(u64));
    if (!a) return -3;
    for (u64 s = 0; s < N; s++) a[or_rev(s, k)] = X[s] % p; /* natural order */
    dft_natural(p, a, N, k, or_invmod(or_root_chain(p, g, k), p));
    u64 ninv = or_invmod(N % p, p);
    for (u64 t = 0; t < N; t++) F[t] = or_mulmod(a[t], ninv, p);
    free(a);
    return 0;
}

/* ------------------------------------------------------- O6: products */
/* C = A B, C_s = sum_{i+j=s} A_i B_j mod p (section 5: the product is unique).
 * Pinned against numpy.convolve on small values. */
int or_mul_schoolbook(u64 p, const u64 *A, u64 m, const u64 *B, u64 nb, u64 *C)
{
    if (!m || !nb || !A || !B || !C) return -1;
    memset(C, 0, (m + nb - 1) * sizeof(u64));
    for (u64 i = 0; i < m; i++)
        for (u64 j = 0; j < nb; j++)
            C[i + j] = or_addmod(C[i + j], or_mulmod(A[i] % p, B[j] % p, p), p);
    return 0;
}

/* One coefficient of the product, O(min(m, nb)). */
u64 or_mul_coeff(u64 p, const u64 *A, u64 m, const u64 *B, u64 nb, u64 s)
{
    u64 acc = 0;
    u64 lo = s + 1 > nb ? s + 1 - nb : 0;
    for (u64 i = lo; i < m && i <= s; i++)
        acc = or_addmod(acc, or_mulmod(A[i] % p, B[s - i] % p, p), p);
    return acc;
}

/* Product through a zero-padded power-of-two DFT (large-size reference):
 * N = 2^ceil(lg(m+nb-1)); forward DFT of both, pointwise, inverse. */
int or_mul_padded(u64 p, u64 g, const u64 *A, u64 m, const u64 *B, u64 nb, u64 *C)
{
    if (!m || !nb || !A || !B || !C) return -1;
    u64 r = m + nb - 1;
    if (!n_ok(p, r)) return -2;
    unsigned k = or_bitlen(r - 1);
    u64 N = (u64)1 << k;
    u64 *a = (u64 *)calloc(N, sizeof(u64));
    u64 *b = (u64 *)calloc(N, sizeof(u64));
    if (!a || !b) { free(a); free(b); return -3; }
    for (u64 i = 0; i < m; i++) a[i] = A[i] % p;
    for (u64 i = 0; i < nb; i++) b[i] = B[i] % p;
    u64 w = or_root_chain(p, g, k);
    dft_natural(p, a, N, k, w);
    dft_natural(p, b, N, k, w);
    for (u64 i = 0; i < N; i++) a[i] = or_mulmod(a[i], b[i], p);
    dft_natural(p, a, N, k, or_invmod(w, p));
    u64 ninv = or_invmod(N % p, p);
    for (u64 s = 0; s < r; s++) C[s] = or_mulmod(a[s], ninv, p);
    free(a); free(b);
    return 0;
}

/* ---------------------------------------------- O7: exact integer product */
/* Exact signed convolution in 128-bit integers; the result is written as
 * little-endian (lo, hi) 64-bit pairs.  Pinned against Python integers. */
int or_conv_i128(const int64_t *a, u64 m, const int64_t *b, u64 nb, u64 *out_lohi)
{
    if (!m || !nb || !a || !b || !out_lohi) return -1;
    u64 r = m + nb - 1;
    i128 *c = (i128 *)calloc(r, sizeof(i128));
    if (!c) return -3;
    for (u64 i = 0; i < m; i++)
        for (u64 j = 0; j < nb; j++) c[i + j] += (i128)a[i] * (i128)b[j];
    for (u64 s = 0; s < r; s++) {
        u128 u = (u128)c[s];
        out_lohi[2 * s] = (u64)u;
        out_lohi[2 * s + 1] = (u64)(u >> 64);
    }
    free(c);
    return 0;
}

/* One exact coefficient c_s, O(min(m, nb)). */
int or_conv_coeff_i128(const int64_t *a, u64 m, const int64_t *b, u64 nb, u64 s, u64 *lohi)
{
    if (!a || !b || !lohi || s >= m + nb - 1) return -1;
    i128 acc = 0;
    u64 lo = s + 1 > nb ? s + 1 - nb : 0;
    for (u64 i = lo; i < m && i <= s; i++) acc += (i128)a[i] * (i128)b[s - i];
    u128 u = (u128)acc;
    lohi[0] = (u64)u;
    lohi[1] = (u64)(u >> 64);
    return 0;
}

/* ------------------------------- the paper's in-place algorithms (CPU) */
/* Algorithms 1 and 2 (sections 3 and 4) written as the recursion their
 * Lemmas 3.1 and 4.1 describe, on the tree of nodes (q, r): the node is the
 * strided subarray S_i = X_{q + i 2^r} of length ceil((n - q) / 2^r); its even
 * child is (q, r+1) and its odd child (q + 2^r, r+1).  Forward at a node of
 * length m > 1: transform the even child; if m is odd, evaluate the still-raw
 * odd coefficients at w_{(m-1)/2} and add w_{m-1} times that value into
 * S_{m-1}; transform the odd child; then apply the butterflies (eq. 1)
 * S_{2j}, S_{2j+1} <- S_{2j} +/- w_{2j} S_{2j+1}.  The inverse undoes these
 * steps in the opposite order.  The recursion depth is O(log n); the paper's
 * O(1)-space iterative walk visits the same nodes in the same order.  This is
 * the "plain CPU TFT" baseline; it must agree with or_tft_direct. */
typedef struct {
    u64 p, n, inv2;
    const u64 *w;   /* w_s, s < n */
    const u64 *wi;  /* w_s^-1, s < n */
    u64 *X;
} paper_ctx;

u64 or_node_len(u64 n, u64 q, unsigned r)
{
    u64 st = (u64)1 << r;
    return q >= n ? 0 : (n - q + st - 1) / st;
}

static u64 correction_value(const paper_ctx *c, u64 q, unsigned r, u64 m)
{
    /* v = H(w_{(m-1)/2}), H(y) = sum_i S_{2i+1} y^i over the raw odd entries */
    u64 st = (u64)1 << r;
    u64 z = c->w[(m - 1) / 2];
    u64 v = 0;
    for (u64 i = (m - 1) / 2; i-- > 0;)
        v = or_addmod(or_mulmod(v, z, c->p), c->X[q + (2 * i + 1) * st], c->p);
    return or_mulmod(v, c->w[m - 1], c->p);
}

static void paper_tft_node(paper_ctx *c, u64 q, unsigned r)
{
    u64 m = or_node_len(c->n, q, r);
    if (m <= 1) return;
    u64 st = (u64)1 << r, p = c->p;
    paper_tft_node(c, q, r + 1);
    if (m & 1) {
        u64 *last = &c->X[q + (m - 1) * st];
        *last = or_addmod(*last, correction_value(c, q, r, m), p);
    }
    paper_tft_node(c, q + st, r + 1);
    for (u64 j = 0; j < m / 2; j++) {
        u64 *e = &c->X[q + 2 * j * st], *o = &c->X[q + (2 * j + 1) * st];
        u64 t = or_mulmod(c->w[2 * j], *o, p);
        u64 a = *e;
        *e = or_addmod(a, t, p);
        *o = or_submod(a, t, p);
    }
}

static void paper_itft_node(paper_ctx *c, u64 q, unsigned r)
{
    u64 m = or_node_len(c->n, q, r);
    if (m <= 1) return;
    u64 st = (u64)1 << r, p = c->p;
    for (u64 j = 0; j < m / 2; j++) {
        u64 *e = &c->X[q + 2 * j * st], *o = &c->X[q + (2 * j + 1) * st];
        u64 a = *e, b = *o;
        *e = or_mulmod(or_addmod(a, b, p), c->inv2, p);
        *o = or_mulmod(or_mulmod(or_submod(a, b, p), c->inv2, p), c->wi[2 * j], p);
    }
    paper_itft_node(c, q + st, r + 1);
    if (m & 1) {
        u64 *last = &c->X[q + (m - 1) * st];
        *last = or_submod(*last, correction_value(c, q, r, m), p);
    }
    paper_itft_node(c, q, r + 1);
}

static int paper_run(u64 p, u64 g, u64 *X, u64 n, int inverse)
{
    if (!n_ok(p, n) || !X) return -1;
    u64 *w = (u64 *)malloc(n * sizeof(u64));
    u64 *wi = (u64 *)malloc(n * sizeof(u64));
    if (!w || !wi) { free(w); free(wi); return -3; }
    for (u64 s = 0; s < n; s++) { w[s] = or_omega(p, g, s); wi[s] = or_invmod(w[s], p); }
    for (u64 s = 0; s < n; s++) X[s] %= p;
    paper_ctx c = { p, n, (p + 1) / 2, w, wi, X };
    if (inverse) paper_itft_node(&c, 0, 0); else paper_tft_node(&c, 0, 0);
    free(w); free(wi);
    return 0;
}

int or_tft_paper(u64 p, u64 g, u64 *X, u64 n) { return paper_run(p, g, X, n, 0); }
int or_itft_paper(u64 p, u64 g, u64 *X, u64 n) { return paper_run(p, g, X, n, 1); }

/* Counts of the paper's forward walk: butterflies and correction mulmods
 * (Horner terms plus the final multiply), for the operation-count report. */
static void count_node(u64 n, u64 q, unsigned r, u64 *bf, u64 *corr)
{
    u64 m = or_node_len(n, q, r);
    if (m <= 1) return;
    u64 st = (u64)1 << r;
    count_node(n, q, r + 1, bf, corr);
    if (m & 1) *corr += (m - 1) / 2 + 1;
    count_node(n, q + st, r + 1, bf, corr);
    *bf += m / 2;
}

int or_paper_counts(u64 n, u64 *butterflies, u64 *corrections)
{
    if (!n || !butterflies || !corrections) return -1;
    *butterflies = 0;
    *corrections = 0;
    count_node(n, 0, 0, butterflies, corrections);
    return 0;
}

/* ------------------- the paper's algorithms with O(1) auxiliary space (CPU) */
/* The same transforms as or_tft_paper / or_itft_paper (sections 3 and 4), now
 * with a constant number of scalars besides X: no root table and no
 * recursion.  This is the plain CPU TFT that the benchmark times beside the
 * GPU path; it must agree with or_tft_direct and or_itft_lagrange.
 *
 * Roots on the fly.  From w_s = w[k]^(rev_k s) (section 2.2) and
 * w[k]^(2^(k-1-i)) = w[i+1], a root is the product over the set bits i of s of
 * w[i+1].  The butterflies of a node need w_{2j} for j = 0, 1, ...: stepping
 * j -> j+1 clears the trailing ones of j (bits 0..t-1) and sets bit t, so
 * w_{2j+2} = w_{2j} w[t+2] / (w[2] ... w[t+1]): amortised O(1) products from
 * the chain w[1..v] and its inverses (at most 65 words each, independent of
 * n).
 *
 * Traversal.  A node (q, r) of the tree of section 3 has length
 * ceil((n - q) / 2^r); its parent is (q with bit r-1 cleared, r-1), and it is
 * the odd child exactly when bit r-1 of q is set, so the walk needs no stack:
 * the state is the current node and whether it was just entered or just
 * returned to from its even or its odd child.  Forward: enter a node of
 * length m > 1 -> enter its even child; back from the even child -> if m is
 * odd apply the correction (the raw odd coefficients evaluated at
 * w_{(m-1)/2}, times w_{m-1}, added into S_{m-1}) and enter the odd child;
 * back from the odd child -> the butterflies of eq. (1), then return to the
 * parent.  Inverse (section 4): enter -> inverse butterflies, then enter the
 * odd child; back from the odd child -> remove the correction (its odd
 * coefficients are raw again) and enter the even child; back from the even
 * child -> return to the parent. */
typedef struct {
    u64 p;
    unsigned v;
    u64 w[65], wi[65];   /* w[j], w[j]^-1, j <= v */
} chain_ctx;

static void chain_init(chain_ctx *c, u64 p, u64 g)
{
    c->p = p;
    c->v = or_two_adic(p);
    for (unsigned j = 0; j <= c->v && j <= 64; j++) {
        c->w[j] = or_root_chain(p, g, j);
        c->wi[j] = or_invmod(c->w[j], p);
    }
}

/* w_s (inverse: w_s^-1) from the set bits of s */
static u64 chain_root(const chain_ctx *c, u64 s, int inverse)
{
    u64 r = 1 % c->p;
    for (unsigned i = 0; s; i++, s >>= 1)
        if (s & 1) r = or_mulmod(r, inverse ? c->wi[i + 1] : c->w[i + 1], c->p);
    return r;
}

/* the odd-length correction of node (q, r), length m odd: w_{m-1} H(w_{(m-1)/2})
 * with H(y) = sum_i S_{2i+1} y^i over the node's (raw) odd entries */
static u64 inplace_correction(const chain_ctx *c, const u64 *X, u64 q, unsigned r, u64 m)
{
    const u64 st = (u64)1 << r, p = c->p;
    const u64 z = chain_root(c, (m - 1) / 2, 0);
    u64 h = 0;
    for (u64 i = (m - 1) / 2; i-- > 0;) h = or_addmod(or_mulmod(h, z, p), X[q + (2 * i + 1) * st], p);
    return or_mulmod(h, chain_root(c, m - 1, 0), p);
}

/* eq. (1) at node (q, r) of length m: S_{2j}, S_{2j+1} <- S_{2j} +/- w_{2j} S_{2j+1};
 * inverse: S_{2j}, S_{2j+1} <- (S_{2j} + S_{2j+1}) / 2, w_{2j}^-1 (S_{2j} - S_{2j+1}) / 2.
 * w_{2j} runs over the even indices: the product over the set bits i of j of w[i+2]. */
static void inplace_butterflies(const chain_ctx *c, u64 *X, u64 q, unsigned r, u64 m, int inverse)
{
    const u64 st = (u64)1 << r, p = c->p, half = (p + 1) / 2;
    u64 tw = 1 % p;   /* w_{2j} (inverse: its inverse) */
    for (u64 j = 0; j < m / 2; j++) {
        u64 *e = &X[q + 2 * j * st], *o = &X[q + (2 * j + 1) * st];
        if (!inverse) {
            u64 t = or_mulmod(tw, *o, p), a = *e;
            *e = or_addmod(a, t, p);
            *o = or_submod(a, t, p);
        } else {
            u64 a = *e, b = *o;
            *e = or_mulmod(or_addmod(a, b, p), half, p);
            *o = or_mulmod(or_mulmod(or_submod(a, b, p), half, p), tw, p);
        }
        /* w_{2(j+1)}: step j -> j+1 in the chain shifted by one level */
        unsigned t = 0;
        while ((j >> t) & 1) {
            tw = or_mulmod(tw, inverse ? c->w[t + 2] : c->wi[t + 2], p);
            t++;
        }
        if (j + 1 < m / 2) tw = or_mulmod(tw, inverse ? c->wi[t + 2] : c->w[t + 2], p);
    }
}

enum { ENTER = 0, FROM_EVEN = 1, FROM_ODD = 2 };

static void inplace_walk(const chain_ctx *c, u64 *X, u64 n, int inverse)
{
    const u64 p = c->p;
    u64 q = 0;
    unsigned r = 0;
    int state = ENTER;
    for (;;) {
        const u64 m = or_node_len(n, q, r), st = (u64)1 << r;
        if (state == ENTER && m > 1) {
            if (!inverse) {
                r++;                              /* even child (q, r+1) */
                continue;
            }
            inplace_butterflies(c, X, q, r, m, 1);
            q += st;                              /* odd child (q + 2^r, r+1) */
            r++;
            continue;
        }
        if (state == FROM_EVEN && !inverse) {
            if (m & 1) {
                u64 *last = &X[q + (m - 1) * st];
                *last = or_addmod(*last, inplace_correction(c, X, q, r, m), p);
            }
            q += st;
            r++;
            state = ENTER;
            continue;
        }
        if (state == FROM_ODD && inverse) {
            if (m & 1) {
                u64 *last = &X[q + (m - 1) * st];
                *last = or_submod(*last, inplace_correction(c, X, q, r, m), p);
            }
            r++;                                  /* even child */
            state = ENTER;
            continue;
        }
        if (state == FROM_ODD && !inverse) inplace_butterflies(c, X, q, r, m, 0);
        /* this node is finished (a leaf, or its last step is done): back to the parent */
        if (r == 0) return;
        const u64 bit = (u64)1 << (r - 1);
        state = (q & bit) ? FROM_ODD : FROM_EVEN;
        q &= ~bit;
        r--;
    }
}

static int inplace_run(u64 p, u64 g, u64 *X, u64 n, int inverse)
{
    if (!n_ok(p, n) || !X) return -1;
    chain_ctx c;
    chain_init(&c, p, g);
    for (u64 s = 0; s < n; s++) X[s] %= p;
    inplace_walk(&c, X, n, inverse);
    return 0;
}

int or_tft_inplace(u64 p, u64 g, u64 *X, u64 n) { return inplace_run(p, g, X, n, 0); }
int or_itft_inplace(u64 p, u64 g, u64 *X, u64 n) { return inplace_run(p, g, X, n, 1); }

/* Section 5, Algorithm 3 (Proposition 5.1): C = A B into X (r = m + nb - 1
 * words) with X the only memory written besides O(1) scalars.  The blocks:
 * q = 0, then q += L, with L the largest power of two such that q + 2L <= r
 * (so L | q).  For each block the coefficients of A(w_q x) mod x^L - 1 (the
 * terms w_q^i A_i summed into slot i mod L) are transformed in
 * X[q, q+L): since L | q, w_q w_i = w_{q+i}, so the slots then hold
 * A(w_{q+i}); the same for B in X[q+L, q+2L); the products go to X[q, q+L).
 * The last point w_{r-1} has no room for two values: X[r-1] = A(w_{r-1})
 * B(w_{r-1}) by direct evaluation.  Then the in-place inverse of length r. */
int or_mul_restricted(u64 p, u64 g, const u64 *A, u64 m, const u64 *B, u64 nb, u64 *X)
{
    if (!A || !B || !X || m == 0 || nb == 0) return -1;
    const u64 r = m + nb - 1;
    if (!n_ok(p, r)) return -2;
    chain_ctx c;
    chain_init(&c, p, g);
    u64 q = 0;
    while (q + 1 < r) {
        unsigned l = 0;
        while (q + ((u64)4 << l) <= r) l++;    /* largest L = 2^l with q + 2L <= r */
        const u64 L = (u64)1 << l;
        const u64 wq = chain_root(&c, q, 0);
        for (int side = 0; side < 2; side++) {
            const u64 *P = side ? B : A;
            const u64 len = side ? nb : m;
            u64 *blk = X + q + (side ? L : 0);
            for (u64 i = 0; i < L; i++) blk[i] = 0;
            u64 zi = 1 % p;   /* w_q^i */
            for (u64 i = 0; i < len; i++) {
                blk[i % L] = or_addmod(blk[i % L], or_mulmod(zi, P[i] % p, p), p);
                zi = or_mulmod(zi, wq, p);
            }
            inplace_walk(&c, blk, L, 0);     /* a full transform: L is a power of two */
        }
        for (u64 i = 0; i < L; i++) X[q + i] = or_mulmod(X[q + i], X[q + L + i], p);
        q += L;
    }
    const u64 z = chain_root(&c, r - 1, 0);
    u64 a = 0, b = 0;
    for (u64 i = m; i-- > 0;) a = or_addmod(or_mulmod(a, z, p), A[i] % p, p);
    for (u64 i = nb; i-- > 0;) b = or_addmod(or_mulmod(b, z, p), B[i] % p, p);
    X[r - 1] = or_mulmod(a, b, p);
    inplace_walk(&c, X, r, 1);
    return 0;
}
