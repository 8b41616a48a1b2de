"""Planted mistakes: each case copies the oracle source, plants one plausible
mistake (a dropped term, a wrong sign, a wrong index, a transposed operand),
compiles the copy on the CPU and checks that the pins reject it.  This shows
the pins are strong enough to catch such errors in the oracle itself."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "tft_oracle.c")

MUTATIONS = {
    # natural-order root index instead of the bit-reversed one
    "omega_not_reversed": ("return or_powmod(or_root_chain(p, g, k), or_rev(s, k), p);\n}\n\n/* Same root",
                           "return or_powmod(or_root_chain(p, g, k), s, p);\n}\n\n/* Same root"),
    # Horner evaluation drops the constant term
    "eval_drops_term": ("for (u64 t = n; t-- > 0;)", "for (u64 t = n; t-- > 1;)"),
    # paper TFT: the odd-length correction is skipped
    "paper_no_correction": ("*last = or_addmod(*last, correction_value(c, q, r, m), p);", "(void)last;"),
    # paper TFT: butterfly sign flipped
    "paper_sign": ("*o = or_submod(a, t, p);\n    }\n}", "*o = or_addmod(a, t, p);\n    }\n}"),
    # paper TFT: twiddle index off (w_j instead of w_{2j})
    "paper_twiddle_index": ("u64 t = or_mulmod(c->w[2 * j], *o, p);", "u64 t = or_mulmod(c->w[j], *o, p);"),
    # padded FFT: output not permuted
    "padded_no_permutation": ("for (u64 s = 0; s < n; s++) X[s] = a[or_rev(s, k)];", "for (u64 s = 0; s < n; s++) X[s] = a[s];"),
    # schoolbook: transposed index
    "schoolbook_index": ("C[i + j] = or_addmod(C[i + j], or_mulmod(A[i] % p, B[j] % p, p), p);",
                         "C[i + j] = or_addmod(C[i + j], or_mulmod(A[j % m] % p, B[i % nb] % p, p), p);"),
    # operation counts: the final multiply of the correction is not counted
    "counts_drop_final_multiply": ("if (m & 1) *corr += (m - 1) / 2 + 1;", "if (m & 1) *corr += (m - 1) / 2;"),
    # operation counts: a node of length m counts ceil(m/2) butterflies
    "counts_butterfly_ceil": ("*bf += m / 2;", "*bf += (m + 1) / 2;"),
    # in-place walk (O(1) space): the odd-length correction is skipped
    "inplace_no_correction": ("*last = or_addmod(*last, inplace_correction(c, X, q, r, m), p);", "(void)last;"),
    # in-place walk: the on-the-fly root steps one level too low (w_j instead of w_{2j})
    "inplace_root_step": ("if (j + 1 < m / 2) tw = or_mulmod(tw, inverse ? c->wi[t + 2] : c->w[t + 2], p);",
                          "if (j + 1 < m / 2) tw = or_mulmod(tw, inverse ? c->wi[t + 1] : c->w[t + 1], p);"),
    # in-place inverse: the correction is added back instead of removed
    "inplace_inverse_sign": ("*last = or_submod(*last, inplace_correction(c, X, q, r, m), p);",
                             "*last = or_addmod(*last, inplace_correction(c, X, q, r, m), p);"),
    # Algorithm 3: the fold leaves out the twist by w_q
    "restricted_no_twist": ("                zi = or_mulmod(zi, wq, p);\n", ""),
    # Algorithm 3: the last point keeps only A's value
    "restricted_last_point": ("X[r - 1] = or_mulmod(a, b, p);", "X[r - 1] = a;"),
    # interpolation: sign slip in building M
    "lagrange_sign": ("M[0] = or_submod(0, or_mulmod(M[0], w[s], p), p);", "M[0] = or_mulmod(M[0], w[s], p);"),
}


def build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(path)], check=True)
    return so


def pins_pass(so):
    """A compact subset of the pins of tests/test_oracle_*.py, run against a
    library at an arbitrary path.  Returns False on the first failing pin."""
    import json
    L = ctypes.CDLL(str(so))
    u64, P = ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)
    for f in ("or_tft_direct", "or_itft_lagrange", "or_tft_paper", "or_mul_schoolbook", "or_tft_inplace",
              "or_itft_inplace", "or_mul_restricted"):
        getattr(L, f).restype = ctypes.c_int
    L.or_fft_padded.restype = ctypes.c_int
    L.or_fft_padded.argtypes = [u64, u64, P, u64, ctypes.c_uint, P]
    L.or_omega.restype = u64
    L.or_omega.argtypes = [u64, u64, u64]

    def arr(v):
        return np.ascontiguousarray(np.asarray(v, dtype=np.uint64))

    def call(fn, p, g, F, out_len=None):
        F = arr(F)
        X = np.zeros(out_len or len(F), dtype=np.uint64)
        getattr(L, fn)(u64(p), u64(g), F.ctypes.data_as(P), u64(len(F)), X.ctypes.data_as(P))
        return [int(x) for x in X]

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tft_p17.json")))
    if [int(L.or_omega(17, 3, s)) for s in range(16)] != gold["omega"]:
        return False
    for c in gold["cases"]:
        if call("or_tft_direct", 17, 3, c["F"]) != c["X"]:
            return False
        if call("or_itft_lagrange", 17, 3, c["X"]) != c["F"]:
            return False
        X = arr(c["F"]).copy()
        L.or_tft_paper(u64(17), u64(3), X.ctypes.data_as(P), u64(len(X)))
        if [int(x) for x in X] != c["X"]:
            return False
        X = arr(c["F"]).copy()
        L.or_tft_inplace(u64(17), u64(3), X.ctypes.data_as(P), u64(len(X)))
        if [int(x) for x in X] != c["X"]:
            return False
        L.or_itft_inplace(u64(17), u64(3), X.ctypes.data_as(P), u64(len(X)))
        if [int(x) for x in X] != c["F"]:
            return False
        Xp = np.zeros(len(c["F"]), dtype=np.uint64)
        L.or_fft_padded(17, 3, arr(c["F"]).ctypes.data_as(P), len(c["F"]), 0, Xp.ctypes.data_as(P))
        if [int(x) for x in Xp] != c["X"]:
            return False
    # operation counts of Algorithm 1 derived by hand (tests/test_oracle_transform.py)
    L.or_paper_counts.restype = ctypes.c_int
    L.or_paper_counts.argtypes = [u64, P, P]
    for n, want in ((3, (2, 2)), (5, (5, 5)), (6, (7, 4)), (7, (9, 6))):
        bf, corr = np.zeros(1, dtype=np.uint64), np.zeros(1, dtype=np.uint64)
        L.or_paper_counts(u64(n), bf.ctypes.data_as(P), corr.ctypes.data_as(P))
        if (int(bf[0]), int(corr[0])) != want:
            return False
    rng = np.random.default_rng(0)
    A, B = rng.integers(0, 1000, 9), rng.integers(0, 1000, 5)
    C = np.zeros(13, dtype=np.uint64)
    L.or_mul_schoolbook(u64(998244353), arr(A).ctypes.data_as(P), u64(9), arr(B).ctypes.data_as(P), u64(5),
                        C.ctypes.data_as(P))
    if [int(c) for c in C] != [int(x) for x in np.convolve(A, B) % 998244353]:
        return False
    for m, nb in ((1, 1), (2, 1), (3, 4), (9, 5), (7, 7), (16, 17)):   # r = 1 .. 32: one to five blocks
        A, B = rng.integers(0, 1000, m), rng.integers(0, 1000, nb)
        C = np.zeros(m + nb - 1, dtype=np.uint64)
        L.or_mul_restricted(u64(998244353), u64(3), arr(A).ctypes.data_as(P), u64(m), arr(B).ctypes.data_as(P),
                            u64(nb), C.ctypes.data_as(P))
        if [int(c) for c in C] != [int(x) for x in np.convolve(A, B) % 998244353]:
            return False
    return True


def test_unmutated_oracle_passes(tmp_path):
    so = build_variant(tmp_path, "clean", "/* k-bit reversal of s (s < 2^k). */", "/* k-bit reversal of s (s < 2^k). */")
    assert pins_pass(so)


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    so = build_variant(tmp_path, name, old, new)
    assert not pins_pass(so), f"planted mistake {name} was not caught by the pins"
