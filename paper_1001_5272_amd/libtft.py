"""Thin Python binding of libtft (include/libtft.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels of ``libtft.so``.  PyTorch supplies device memory (tensors) and
streams; tensors must be contiguous ``torch.uint32`` (primes below 2^31) or
``torch.uint64`` (p = 2^64 - 2^32 + 1 and the other primes below 2^63) on the
context's device.  Functions
carry the names of the C entry points; a failing status raises ``TftError``.

There is no fallback: if ``libtft.so`` has not been built, or no GPU is
visible, using the library raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library shares)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libtft.so")

TFT_OK, TFT_EINVAL, TFT_ERANGE, TFT_ENOMEM, TFT_EDEVICE, TFT_EAGAIN = 0, -1, -2, -3, -4, -5

_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_st = ctypes.c_int

# name -> (restype, argtypes); must list every function of include/libtft.h
class PlanDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("logW", ctypes.c_uint), ("W", _sz), ("a", _sz), ("b", _sz),
                ("col_block", _sz), ("cols_per_tile", ctypes.c_uint), ("lds_bytes_col", _sz),
                ("lds_bytes_row", _sz), ("row_threads", ctypes.c_uint), ("stages_per_pass", ctypes.c_uint)]


class _Calibration(ctypes.Structure):
    _fields_ = [("valu_tops", ctypes.c_double), ("mad64_tops", ctypes.c_double),
                ("butterflies_g", ctypes.c_double), ("copy_gbs", ctypes.c_double),
                ("butterflies_lds_xchg_g", ctypes.c_double), ("butterflies_bpermute_xchg_g", ctypes.c_double),
                ("butterflies_dpp_xchg_g", ctypes.c_double)]


SIGNATURES = {
    "tft_ctx_create": (_st, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_vp)]),
    "tft_ctx_destroy": (None, [_vp]),
    "tft_ctx_max_log2": (ctypes.c_uint, [_vp]),
    "tft_ctx_word_bytes": (ctypes.c_uint, [_vp]),
    "tft_forward": (_st, [_vp, _vp, _sz, _vp]),
    "tft_inverse": (_st, [_vp, _vp, _sz, _vp]),
    "tft_pointwise_mul": (_st, [_vp, _vp, _vp, _sz, _vp]),
    "poly_mul": (_st, [_vp, _vp, _sz, _vp, _sz, _vp, _vp, _vp]),
    "poly_mul_restricted": (_st, [_vp, _vp, _sz, _vp, _sz, _vp, _vp]),
    "poly_mul_noalloc": (_st, [_vp, _vp, _sz, _vp, _sz, _vp, _vp]),
    "tft_padded_forward": (_st, [_vp, _vp, _sz, _vp, _vp]),
    "tft_padded_inverse": (_st, [_vp, _vp, _sz, _vp, _vp]),
    "tft_buffered_forward": (_st, [_vp, _vp, _sz, _vp]),
    "tft_buffered_inverse": (_st, [_vp, _vp, _sz, _vp]),
    "poly_mul_padded": (_st, [_vp, _vp, _sz, _vp, _sz, _vp, _vp, _vp, _vp]),
    "tft_plan_info": (_st, [_vp, _sz, _vp]),
    "tft_set_plan_override": (_st, [_vp, ctypes.c_uint]),
    "tft_batch_create": (_st, [_vp, _vp, _sz, ctypes.c_int, ctypes.POINTER(_vp)]),
    "tft_batch_run": (_st, [_vp, _vp]),
    "tft_batch_info": (_st, [_vp, _vp]),
    "tft_batch_destroy": (None, [_vp]),
    "poly_mul_batch": (_st, [_vp, _vp, _sz, _vp]),
    "tft_forward_batch": (_st, [_vp, _vp, _vp, _sz, _vp]),
    "tft_from_signed": (_st, [_vp, _vp, _sz, _vp, _vp]),
    "tft_crt3": (_st, [_vp, _vp, _vp, _vp, _sz, _vp, _vp]),
    "tft_queue_create": (_st, [_vp, _sz, _sz, ctypes.POINTER(_vp)]),
    "tft_queue_submit": (_st, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "tft_queue_poll": (_st, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
    "tft_queue_wait": (_st, [_vp, ctypes.c_uint64]),
    "tft_queue_completion_ns": (_st, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    "tft_queue_stats": (_st, [_vp, _vp]),
    "tft_queue_destroy": (None, [_vp]),
    "tft_calibrate": (_st, [_vp, ctypes.POINTER(_Calibration)]),
    "tft_autotune": (_st, [_vp, _sz, ctypes.POINTER(PlanDesc)]),
    "tft_autotune_batch": (_st, [_vp, _vp, _sz, ctypes.c_int, ctypes.POINTER(ctypes.c_uint)]),
    "tft_batch_tuning_get": (_st, [_vp, ctypes.c_void_p]),
    "tft_plan_cache_get": (_st, [_vp, ctypes.c_uint, ctypes.POINTER(ctypes.c_uint)]),
    "tft_plan_cache_set": (_st, [_vp, ctypes.c_uint, ctypes.c_uint]),
    "tft_plan_bucket": (ctypes.c_uint, [_sz]),
    "tft_timing_enable": (_st, [_vp, ctypes.c_int]),
    "tft_timing_select": (_st, [_vp, ctypes.c_uint32]),
    "tft_walk_batch": (_st, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_sz), _sz, ctypes.c_int, _vp]),
    "tft_timing_read": (_st, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)]),
    "tft_timing_reset": (_st, [_vp]),
    "tft_kernel_name": (ctypes.c_char_p, [ctypes.c_int]),
    "tft_strerror": (ctypes.c_char_p, [_st]),
}

KERNEL_NAMES = ["small_fwd", "small_inv", "small_mul", "col_fwd", "row_fwd", "row_inv", "col_inv_short",
                "last_inv", "col_inv_long", "pointwise", "copy_pad", "small_list", "crt3", "col_fix", "fold"]


class TftError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class MulDesc(ctypes.Structure):
    _fields_ = [("a", _vp), ("la", _sz), ("b", _vp), ("lb", _sz), ("out", _vp), ("work", _vp)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("count", _sz), ("single_workgroup", _sz), ("two_pass", _sz), ("device_bytes", _sz),
                ("launches", ctypes.c_uint)]


class QueueDesc(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("submitted", "completed", "batches", "rejected", "pending",
                                                 "inflight", "pool_words", "pool_used_max")]


_lib = None


def load():
    """Load libtft.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1001_5272_amd/build.py "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return load().tft_strerror(status).decode()


def _check(status: int, what: str):
    if status != TFT_OK:
        raise TftError(status, what)


def _stream(stream):
    if stream is None:
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return _vp(stream.cuda_stream)
    return _vp(int(stream))


class Context:
    """A context for one prime on one device (tft_ctx_create)."""

    def __init__(self, p: int, g: int, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libtft needs a GPU; none is visible")
        h = _vp()
        _check(load().tft_ctx_create(p, g, device, ctypes.byref(h)), "tft_ctx_create")
        self.handle = h
        self.p, self.g, self.device = p, g, device
        self.word_bytes = load().tft_ctx_word_bytes(h)
        self.max_log2 = load().tft_ctx_max_log2(h)
        self.dtype = torch.uint32 if self.word_bytes == 4 else torch.uint64

    def close(self):
        if self.handle:
            load().tft_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, x, name):
        if not isinstance(x, torch.Tensor) or x.dtype != self.dtype or not x.is_cuda or not x.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {self.dtype} CUDA tensor")
        return _vp(x.data_ptr())


def tft_ctx_create(p: int, g: int, device: int = 0) -> Context:
    return Context(p, g, device)


def tft_ctx_destroy(ctx: Context):
    ctx.close()


def tft_forward(ctx: Context, X, n: int | None = None, stream=None):
    n = X.numel() if n is None else n
    _check(load().tft_forward(ctx.handle, ctx._t(X, "X"), n, _stream(stream)), "tft_forward")
    return X


def tft_inverse(ctx: Context, X, n: int | None = None, stream=None):
    n = X.numel() if n is None else n
    _check(load().tft_inverse(ctx.handle, ctx._t(X, "X"), n, _stream(stream)), "tft_inverse")
    return X


def tft_pointwise_mul(ctx: Context, X, Y, n: int | None = None, stream=None):
    n = X.numel() if n is None else n
    _check(load().tft_pointwise_mul(ctx.handle, ctx._t(X, "X"), ctx._t(Y, "Y"), n, _stream(stream)),
           "tft_pointwise_mul")
    return X


def poly_mul(ctx: Context, A, B, X, Y=None, stream=None):
    y = ctx._t(Y, "Y") if Y is not None else _vp(0)
    _check(load().poly_mul(ctx.handle, ctx._t(A, "A"), A.numel(), ctx._t(B, "B"), B.numel(), ctx._t(X, "X"), y,
                           _stream(stream)), "poly_mul")
    return X


def poly_mul_noalloc(ctx: Context, A, B, X, stream=None):
    """poly_mul with B's transform in the library's fixed device array (no
    workspace argument, nothing allocated; r <= 2^22 words of 8 bytes or 2^23
    of 4).  Calls on one device must not overlap."""
    _check(load().poly_mul_noalloc(ctx.handle, ctx._t(A, "A"), A.numel(), ctx._t(B, "B"), B.numel(),
                                   ctx._t(X, "X"), _stream(stream)), "poly_mul_noalloc")
    return X


def poly_mul_restricted(ctx: Context, A, B, X, stream=None):
    """Space-restricted product (Algorithm 3): X (len(A) + len(B) - 1 words) is
    the only memory written."""
    _check(load().poly_mul_restricted(ctx.handle, ctx._t(A, "A"), A.numel(), ctx._t(B, "B"), B.numel(),
                                      ctx._t(X, "X"), _stream(stream)), "poly_mul_restricted")
    return X


def tft_padded_forward(ctx: Context, X, Xpad, n: int | None = None, stream=None):
    n = X.numel() if n is None else n
    _check(load().tft_padded_forward(ctx.handle, ctx._t(X, "X"), n, ctx._t(Xpad, "Xpad"), _stream(stream)),
           "tft_padded_forward")
    return X


def tft_padded_inverse(ctx: Context, X, Xpad, n: int | None = None, stream=None):
    n = X.numel() if n is None else n
    _check(load().tft_padded_inverse(ctx.handle, ctx._t(X, "X"), n, ctx._t(Xpad, "Xpad"), _stream(stream)),
           "tft_padded_inverse")
    return X


def tft_buffered_forward(ctx: Context, Xbuf, n: int, stream=None):
    """Van der Hoeven-style buffered TFT (comparator): Xbuf holds 2^ceil(lg n)
    words, the first n of them the input and, on return, the transform."""
    if Xbuf.numel() < (1 << (n - 1).bit_length()):
        raise ValueError("Xbuf needs 2^ceil(lg n) words")
    _check(load().tft_buffered_forward(ctx.handle, ctx._t(Xbuf, "Xbuf"), n, _stream(stream)), "tft_buffered_forward")
    return Xbuf


def tft_buffered_inverse(ctx: Context, Xbuf, n: int, stream=None):
    """Inverse of tft_buffered_forward in the same 2^ceil(lg n)-word buffer."""
    if Xbuf.numel() < (1 << (n - 1).bit_length()):
        raise ValueError("Xbuf needs 2^ceil(lg n) words")
    _check(load().tft_buffered_inverse(ctx.handle, ctx._t(Xbuf, "Xbuf"), n, _stream(stream)), "tft_buffered_inverse")
    return Xbuf


def poly_mul_padded(ctx: Context, A, B, X, Apad, Bpad, stream=None):
    _check(load().poly_mul_padded(ctx.handle, ctx._t(A, "A"), A.numel(), ctx._t(B, "B"), B.numel(),
                                  ctx._t(X, "X"), ctx._t(Apad, "Apad"), ctx._t(Bpad, "Bpad"), _stream(stream)),
           "poly_mul_padded")
    return X


def tft_plan_info(ctx: Context, n: int) -> dict:
    d = PlanDesc()
    _check(load().tft_plan_info(ctx.handle, n, ctypes.byref(d)), "tft_plan_info")
    return {f: getattr(d, f) for f, _ in PlanDesc._fields_}


def tft_autotune(ctx: Context, n: int) -> dict:
    """Time candidate plans for length n (column width W = 2^logW near the
    planner's choice, then columns per tile, threads per row and stages per
    LDS round trip) and cache the fastest for every length in the same
    quarter octave (or, for a power of two, its own slot: tft_plan_bucket);
    returns the resulting plan."""
    d = PlanDesc()
    _check(load().tft_autotune(ctx.handle, n, ctypes.byref(d)), "tft_autotune")
    return {f: getattr(d, f) for f, _ in PlanDesc._fields_}


def tft_autotune_batch(ctx: Context, jobs, products=True) -> int:
    """Time the batch of jobs (as Batch would run it) with the two-pass rows at
    the balanced split, one step wider and two steps wider, then the column-list
    and fused-row workgroup sizes at the chosen width; keep the fastest for the
    context's later batches and return the width (0..2; tft_batch_tuning_get
    gives all three).  Runs the batch."""
    arr = _descs(ctx, jobs, products)
    w = ctypes.c_uint()
    _check(load().tft_autotune_batch(ctx.handle, arr, len(jobs), 1 if products else 0, ctypes.byref(w)),
           "tft_autotune_batch")
    return int(w.value)


class BatchTuning(ctypes.Structure):
    _fields_ = [("widen", ctypes.c_uint), ("list_col_threads", ctypes.c_uint), ("row_mul_threads", ctypes.c_uint)]


def tft_batch_tuning_get(ctx: Context) -> dict:
    """The context's batch settings: row width (steps wider than balanced) and
    the workgroup sizes of a standalone batch's column lists and fused rows."""
    t = BatchTuning()
    _check(load().tft_batch_tuning_get(ctx.handle, ctypes.byref(t)), "tft_batch_tuning_get")
    return {f: getattr(t, f) for f, _ in BatchTuning._fields_}


def tft_plan_cache_get(ctx: Context, bucket: int) -> int:
    """The plan code cached for a bucket (0: the planner's choice)."""
    v = ctypes.c_uint()
    _check(load().tft_plan_cache_get(ctx.handle, bucket, ctypes.byref(v)), "tft_plan_cache_get")
    return int(v.value)


def tft_plan_cache_set(ctx: Context, bucket: int, logW: int):
    _check(load().tft_plan_cache_set(ctx.handle, bucket, logW), "tft_plan_cache_set")


def tft_plan_bucket(n: int) -> int:
    """Plan-cache bucket of a length: floor(4 lg n), or 4 * 28 + 4 + k for
    n = 2^k."""
    return int(load().tft_plan_bucket(n))


def plan_cache_dump(ctx: Context) -> dict:
    """The context's tuned plans as {bucket: plan code} (JSON-ready)."""
    out = {}
    for k in range(0, 4 * 28 + 4 + 29):   # quarter octaves, then one slot per power of two
        v = tft_plan_cache_get(ctx, k)
        if v:
            out[k] = v
    return out


def plan_cache_load(ctx: Context, plans: dict):
    for k, v in plans.items():
        tft_plan_cache_set(ctx, int(k), int(v))


def tft_set_plan_override(ctx: Context, logW: int):
    _check(load().tft_set_plan_override(ctx.handle, logW), "tft_set_plan_override")


def tft_calibrate(ctx: Context) -> dict:
    """Measured roofline denominators of the context's device (see the header)."""
    c = _Calibration()
    _check(load().tft_calibrate(ctx.handle, ctypes.byref(c)), "tft_calibrate")
    return {f: getattr(c, f) for f, _ in _Calibration._fields_}


def tft_timing_enable(ctx: Context, on: bool = True):
    _check(load().tft_timing_enable(ctx.handle, 1 if on else 0), "tft_timing_enable")


def tft_timing_select(ctx: Context, names=None):
    """Bracket only the launches of the named kernels (None: every kernel)."""
    mask = 0xFFFFFFFF if names is None else sum(1 << KERNEL_NAMES.index(n) for n in names)
    _check(load().tft_timing_select(ctx.handle, mask), "tft_timing_select")


def tft_timing_reset(ctx: Context):
    _check(load().tft_timing_reset(ctx.handle), "tft_timing_reset")


def tft_timing_read(ctx: Context) -> dict:
    """{kernel name: (launches, total_ms)} for kernels launched since the last reset."""
    out = {}
    for i, name in enumerate(KERNEL_NAMES):
        cnt, ms = ctypes.c_uint64(), ctypes.c_double()
        _check(load().tft_timing_read(ctx.handle, i, ctypes.byref(cnt), ctypes.byref(ms)), "tft_timing_read")
        if cnt.value:
            out[name] = (int(cnt.value), float(ms.value))
    return out


def tft_kernel_name(i: int) -> str:
    return load().tft_kernel_name(i).decode()


def _descs(ctx, jobs, products=True):
    """jobs: list of (A, B, X, Y) tensors (Y may be None) for products, or of
    X tensors for forward transforms."""
    arr = (MulDesc * len(jobs))()
    for i, j in enumerate(jobs):
        if products:
            A, B, X, Y = j
            arr[i] = MulDesc(ctx._t(A, "A").value, A.numel(), ctx._t(B, "B").value, B.numel(), ctx._t(X, "X").value,
                             ctx._t(Y, "Y").value if Y is not None else None)
        else:
            arr[i] = MulDesc(ctx._t(j, "X").value, j.numel(), None, 0, ctx._t(j, "X").value, None)
    return arr


class Batch:
    """A planned batch (tft_batch_create); run() enqueues it (tft_batch_run)."""

    def __init__(self, ctx: Context, jobs, products=True):
        self.ctx = ctx
        self._keep = list(jobs)
        arr = _descs(ctx, jobs, products)
        h = _vp()
        _check(load().tft_batch_create(ctx.handle, arr, len(jobs), 1 if products else 0, ctypes.byref(h)),
               "tft_batch_create")
        self.handle = h

    def run(self, stream=None):
        _check(load().tft_batch_run(self.handle, _stream(stream)), "tft_batch_run")

    def info(self) -> dict:
        d = BatchDesc()
        _check(load().tft_batch_info(self.handle, ctypes.byref(d)), "tft_batch_info")
        return {f: getattr(d, f) for f, _ in BatchDesc._fields_}

    def close(self):
        if self.handle:
            load().tft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tft_batch_create(ctx: Context, jobs, products=True) -> Batch:
    return Batch(ctx, jobs, products)


def tft_batch_run(batch: Batch, stream=None):
    batch.run(stream)


def tft_batch_info(batch: Batch) -> dict:
    return batch.info()


def tft_batch_destroy(batch: Batch):
    batch.close()


def poly_mul_batch(ctx: Context, jobs, stream=None):
    """jobs: list of (A, B, X, Y) tensors; Y may be None for short products."""
    arr = _descs(ctx, jobs, True)
    _check(load().poly_mul_batch(ctx.handle, arr, len(jobs), _stream(stream)), "poly_mul_batch")


def tft_forward_batch(ctx: Context, xs, stream=None):
    ptrs = (_vp * len(xs))(*[ctx._t(x, "X").value for x in xs])
    ns = (_sz * len(xs))(*[x.numel() for x in xs])
    _check(load().tft_forward_batch(ctx.handle, ptrs, ns, len(xs), _stream(stream)), "tft_forward_batch")


def tft_walk_batch(ctx: Context, xs, inverse: bool = False, stream=None):
    """The paper's Algorithm 1 (or 2 with inverse) on each tensor of xs in place,
    one wavefront per instance (at most 1024 words each); synchronous."""
    ptrs = (_vp * len(xs))(*[ctx._t(x, "X").value for x in xs])
    ns = (_sz * len(xs))(*[x.numel() for x in xs])
    _check(load().tft_walk_batch(ctx.handle, ptrs, ns, len(xs), 1 if inverse else 0, _stream(stream)),
           "tft_walk_batch")


def tft_from_signed(ctx: Context, src, dst, stream=None):
    if src.dtype != torch.int64 or not src.is_cuda or not src.is_contiguous():
        raise TypeError("src must be a contiguous int64 CUDA tensor")
    _check(load().tft_from_signed(ctx.handle, _vp(src.data_ptr()), src.numel(), ctx._t(dst, "dst"), _stream(stream)),
           "tft_from_signed")
    return dst


def tft_crt3(ctxs, r1, r2, r3, out, stream=None):
    """out: int64 tensor of 2 n entries (little-endian 128-bit values)."""
    hs = (_vp * 3)(*[c.handle.value for c in ctxs])
    n = r1.numel()
    if out.dtype != torch.int64 or out.numel() != 2 * n or not out.is_contiguous():
        raise TypeError("out must be a contiguous int64 tensor of 2 n entries")
    _check(load().tft_crt3(hs, ctxs[0]._t(r1, "r1"), ctxs[1]._t(r2, "r2"), ctxs[2]._t(r3, "r3"), n,
                           _vp(out.data_ptr()), _stream(stream)), "tft_crt3")
    return out


class Queue:
    """Serving queue with continuous batching (tft_queue_*).

    The queue holds a reference to each request's tensors until poll() or
    wait() reports the ticket complete (or the queue is closed), so that
    torch's allocator cannot hand their memory to other tensors while the
    device may still read or write them."""

    def __init__(self, ctx: Context, pool_words: int, max_inflight: int = 4096):
        self.ctx = ctx
        h = _vp()
        _check(load().tft_queue_create(ctx.handle, pool_words, max_inflight, ctypes.byref(h)), "tft_queue_create")
        self.handle = h
        self._live = {}

    def try_submit(self, A, B, X, stream=None):
        """Submit C = A B into X; the operands are produced on `stream` (default:
        the current stream).  Returns the ticket, or None when the request's
        footprint does not fit the pool's free space now (TFT_EAGAIN)."""
        d = MulDesc(self.ctx._t(A, "A").value, A.numel(), self.ctx._t(B, "B").value, B.numel(),
                    self.ctx._t(X, "X").value, None)
        t = ctypes.c_uint64()
        st = load().tft_queue_submit(self.handle, ctypes.byref(d), _stream(stream), ctypes.byref(t))
        if st == TFT_EAGAIN:
            return None
        _check(st, "tft_queue_submit")
        self._live[int(t.value)] = (A, B, X)
        return int(t.value)

    def submit(self, A, B, X, stream=None) -> int:
        """As try_submit, raising TftError(TFT_EAGAIN) when the request does not fit now."""
        t = self.try_submit(A, B, X, stream)
        if t is None:
            raise TftError(TFT_EAGAIN, "tft_queue_submit")
        return t

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int()
        st = load().tft_queue_poll(self.handle, ticket, ctypes.byref(done))
        if done.value:
            self._live.pop(ticket, None)
        _check(st, "tft_queue_poll")
        return bool(done.value)

    def wait(self, ticket: int):
        st = load().tft_queue_wait(self.handle, ticket)
        self._live.pop(ticket, None)
        _check(st, "tft_queue_wait")

    def completion_ns(self, ticket: int) -> int:
        ns = ctypes.c_uint64()
        _check(load().tft_queue_completion_ns(self.handle, ticket, ctypes.byref(ns)), "tft_queue_completion_ns")
        return int(ns.value)

    def stats(self) -> dict:
        d = QueueDesc()
        _check(load().tft_queue_stats(self.handle, ctypes.byref(d)), "tft_queue_stats")
        return {f: int(getattr(d, f)) for f, _ in QueueDesc._fields_}

    def close(self):
        if self.handle:
            load().tft_queue_destroy(self.handle)   # waits for every submitted request
            self.handle = None
        self._live = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tft_queue_create(ctx: Context, pool_words: int, max_inflight: int = 4096) -> Queue:
    return Queue(ctx, pool_words, max_inflight)


def tft_queue_submit(q: Queue, A, B, X, stream=None) -> int:
    return q.submit(A, B, X, stream)


def tft_queue_poll(q: Queue, ticket: int) -> bool:
    return q.poll(ticket)


def tft_queue_wait(q: Queue, ticket: int):
    q.wait(ticket)


def tft_queue_completion_ns(q: Queue, ticket: int) -> int:
    return q.completion_ns(ticket)


def tft_queue_stats(q: Queue) -> dict:
    return q.stats()


def tft_queue_destroy(q: Queue):
    q.close()
