"""Thin ctypes binding of ``libgf2x.so`` (the C ABI in ``include/gf2x.h``).

Only argument marshalling happens here: every step of a product runs in the
library's HIP kernels.  Device buffers are torch tensors (any 8-byte dtype,
typically ``torch.int64`` holding the uint64 words); streams are torch CUDA
streams or raw ``hipStream_t`` integers.  If the library is not built, every
entry point raises -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf2x.so")
# Schedule table measured on MI355X by ``python -m paper_2201_10473_amd.tune``.
DEFAULT_TUNE_CACHE = os.path.join(_HERE, "tune_gfx950.txt")

GF2X_OK = 0
GF2X_EINVAL = -1
GF2X_ENOMEM = -2
GF2X_EDEVICE = -3
GF2X_EAGAIN = -4
GF2X_ENOTSUP = -5
GF2X_MAX_BITS = 131072

KIND_CYCLIC = 0
KIND_FULL = 1
KIND_SPARSE = 2
GF2X_SPARSE_MAX_BITS = 65504


def sparse_kind(weight):
    """Kind of a dense x sparse ring product whose sparse operand has `weight`
    positions (uint32 values at the item's b offset)."""
    if not 0 <= int(weight) < (1 << 24):
        raise ValueError("weight must be below 2^24")
    return KIND_SPARSE | (int(weight) << 8)

ITEMS_ON_DEVICE = 0x1
SHARED_A = 0x2
FORCE_PACKED = 0x4
FORCE_TOEPLITZ = 0x8
USE_GRAPH = 0x10
FUSED = 0x20

# Layout of struct gf2x_item.
ITEM_DTYPE = np.dtype(
    [("n_bits", "<u4"), ("kind", "<u4"), ("a_off", "<u8"), ("b_off", "<u8"), ("c_off", "<u8")], align=True
)
assert ITEM_DTYPE.itemsize == 32

_lib = None


class Gf2xError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        msg = lib.gf2x_strerror(code).decode()
        dev = lib.gf2x_last_device_error().decode()
        super().__init__("%s failed: %s (%d)%s" % (where, msg, code, (" [" + dev + "]") if dev else ""))
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("tune_cache", ctypes.c_char_p),
        ("flags", ctypes.c_uint32),
    ]


class _SrvOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("streams", ctypes.c_uint32),
        ("max_bits", ctypes.c_uint32),
        ("max_batch", ctypes.c_uint32),
        ("max_pending", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


class SrvStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("refused", ctypes.c_uint64),
        ("pending", ctypes.c_uint64),
        ("batches", ctypes.c_uint64),
        ("launches", ctypes.c_uint64),
        ("max_batch", ctypes.c_uint32),
        ("max_batch_seen", ctypes.c_uint32),
        ("max_slots_busy", ctypes.c_uint32),
        ("hbm_bytes", ctypes.c_uint64),
        ("phased_batches", ctypes.c_uint64),
        ("host_pack_ns", ctypes.c_uint64),
        ("host_issue_ns", ctypes.c_uint64),
        ("host_retire_ns", ctypes.c_uint64),
        ("host_pack_max_ns", ctypes.c_uint64),
        ("host_issue_max_ns", ctypes.c_uint64),
        ("host_retire_max_ns", ctypes.c_uint64),
        ("device_max_ns", ctypes.c_uint64),
        ("batch_max_ns", ctypes.c_uint64),
        ("loop_busy_max_ns", ctypes.c_uint64),
        ("wake_late_max_ns", ctypes.c_uint64),
        ("loop_busy_max_at_ns", ctypes.c_uint64),
        ("host_issue_copy_max_ns", ctypes.c_uint64),
        ("host_issue_launch_max_ns", ctypes.c_uint64),
        ("host_issue_tail_max_ns", ctypes.c_uint64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def load():
    """Load the built library (raises if it is missing: no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libgf2x.so is not built (expected at %s); build it with "
            "paper_2201_10473_amd.build.build_library()" % LIB_PATH
        )
    # torch bundles its own HIP runtime under the same soname as the system
    # one.  Importing torch first makes the library bind to that runtime, so
    # the process has one HIP runtime and torch's device pointers and streams
    # are valid in the library.  (Loaded the other way round, two runtimes
    # would compete for the device.)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    lib.gf2x_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Opts)]
    lib.gf2x_create.restype = ctypes.c_int
    lib.gf2x_destroy.argtypes = [vp]
    lib.gf2x_destroy.restype = None
    for name in ("gf2x_mul", "gf2x_mul_cyclic"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, vp, vp, u32, vp]
        fn.restype = ctypes.c_int
    lib.gf2x_mul_batched.argtypes = [vp, vp, u32, vp, vp, vp, u32, vp]
    lib.gf2x_mul_batched.restype = ctypes.c_int
    lib.gf2x_mul_batched_noalloc.argtypes = [vp, vp, u32, vp, vp, vp, vp]
    lib.gf2x_mul_batched_noalloc.restype = ctypes.c_int
    lib.gf2x_device_item_errors.argtypes = [vp, ctypes.POINTER(u64)]
    lib.gf2x_device_item_errors.restype = ctypes.c_int
    lib.gf2x_plan_create.argtypes = [ctypes.POINTER(vp), vp, vp, u32, vp, vp, vp, u32]
    lib.gf2x_plan_create.restype = ctypes.c_int
    lib.gf2x_plan_launch.argtypes = [vp, vp]
    lib.gf2x_plan_launch.restype = ctypes.c_int
    lib.gf2x_plan_destroy.argtypes = [vp]
    lib.gf2x_plan_destroy.restype = None
    lib.gf2x_inv_cyclic_batched.argtypes = [vp, vp, u32, vp, vp, u32, vp]
    lib.gf2x_inv_cyclic_batched.restype = ctypes.c_int
    lib.gf2x_schedule_info.argtypes = [
        vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.c_char_p, sz
    ]
    lib.gf2x_schedule_info.restype = ctypes.c_int
    lib.gf2x_tune.argtypes = [vp, ctypes.POINTER(u32), u32, u32, ctypes.c_char_p]
    lib.gf2x_tune.restype = ctypes.c_int
    lib.gf2x_srv_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(_SrvOpts)]
    lib.gf2x_srv_create.restype = ctypes.c_int
    lib.gf2x_srv_submit.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(u64)]
    lib.gf2x_srv_submit.restype = ctypes.c_int
    lib.gf2x_srv_completion.argtypes = [vp, u64, u32, vp]
    lib.gf2x_srv_completion.restype = ctypes.c_int
    lib.gf2x_srv_drain.argtypes = [vp, u64]
    lib.gf2x_srv_drain.restype = ctypes.c_int
    lib.gf2x_srv_get_stats.argtypes = [vp, ctypes.POINTER(SrvStats)]
    lib.gf2x_srv_get_stats.restype = ctypes.c_int
    lib.gf2x_srv_now_ns.argtypes = []
    lib.gf2x_srv_now_ns.restype = u64
    lib.gf2x_srv_destroy.argtypes = [vp]
    lib.gf2x_srv_destroy.restype = None
    lib.gf2x_strerror.argtypes = [ctypes.c_int]
    lib.gf2x_strerror.restype = ctypes.c_char_p
    lib.gf2x_last_device_error.argtypes = []
    lib.gf2x_last_device_error.restype = ctypes.c_char_p
    lib.gf2x_version.argtypes = []
    lib.gf2x_version.restype = ctypes.c_int
    _lib = lib
    return lib


def words(n):
    return (int(n) + 63) // 64


def _ptr(x):
    """Device address of a torch tensor, or an int address as given."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc, where):
    if rc != GF2X_OK:
        raise Gf2xError(rc, where)


class Context:
    """A library context bound to one HIP device."""

    def __init__(self, device=0, hbm_budget_bytes=0, tune_cache="default"):
        """tune_cache: path of a schedule table, "default" for the packaged
        MI355X table (if present), or None for the built-in cost model."""
        lib = load()
        if tune_cache == "default":
            tune_cache = DEFAULT_TUNE_CACHE if os.path.exists(DEFAULT_TUNE_CACHE) else None
        self._lib = lib
        opts = _Opts(device, hbm_budget_bytes, tune_cache.encode() if tune_cache else None, 0)
        h = ctypes.c_void_p()
        _check(lib.gf2x_create(ctypes.byref(h), ctypes.byref(opts)), "gf2x_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gf2x_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def mul(self, c, a, b, n, stream=None):
        """c (2*W(n) words) = a * b in F2[X]."""
        _check(self._lib.gf2x_mul(self._h, _ptr(c), _ptr(a), _ptr(b), int(n), _stream(stream)), "gf2x_mul")

    def mul_cyclic(self, c, a, b, n, stream=None):
        """c (W(n) words) = a * b mod (X^n - 1)."""
        _check(
            self._lib.gf2x_mul_cyclic(self._h, _ptr(c), _ptr(a), _ptr(b), int(n), _stream(stream)),
            "gf2x_mul_cyclic",
        )

    def mul_batched(self, items, c_base, a_base, b_base, flags=0, stream=None, count=None):
        """Batch of products.  ``items``: numpy array of ITEM_DTYPE (host), or a
        device tensor of the same bytes with ITEMS_ON_DEVICE (then ``count``)."""
        if flags & ITEMS_ON_DEVICE:
            if count is None:
                raise ValueError("count is required with device items")
            items_ptr = _ptr(items)
        else:
            items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
            count = len(items)
            items_ptr = items.ctypes.data
        _check(
            self._lib.gf2x_mul_batched(
                self._h, items_ptr, int(count), _ptr(c_base), _ptr(a_base), _ptr(b_base), int(flags),
                _stream(stream),
            ),
            "gf2x_mul_batched",
        )

    def device_item_errors(self):
        """Device-resident descriptors skipped as invalid since the last call
        (waits for the device)."""
        v = ctypes.c_uint64()
        _check(self._lib.gf2x_device_item_errors(self._h, ctypes.byref(v)), "gf2x_device_item_errors")
        return v.value

    def mul_batched_noalloc(self, items, c_base, a_base, b_base, stream=None):
        """mul_batched with host items, using the library's static scratch
        array instead of allocated workspace (no device allocation)."""
        items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
        _check(
            self._lib.gf2x_mul_batched_noalloc(
                self._h, items.ctypes.data, len(items), _ptr(c_base), _ptr(a_base), _ptr(b_base), _stream(stream)
            ),
            "gf2x_mul_batched_noalloc",
        )

    def plan(self, items, c_base, a_base, b_base, flags=0):
        """Record a batch (host items) once for replays with constant host work."""
        return Plan(self, items, c_base, a_base, b_base, flags)

    def inv_cyclic_batched(self, items, c_base, a_base, stream=None):
        """Inverses in F2[X]/(X^n - 1) (n an odd prime; all items of one n) of
        the items' operands a_base + a_off, written at c_base + c_off.  For an
        operand that is not invertible the result is a_i^(2^(n-1) - 2), not an
        inverse."""
        items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
        _check(
            self._lib.gf2x_inv_cyclic_batched(
                self._h, items.ctypes.data, len(items), _ptr(c_base), _ptr(a_base), 0, _stream(stream)
            ),
            "gf2x_inv_cyclic_batched",
        )

    def tune(self, sizes, batch=4096, out_path=None):
        """Measure every candidate schedule for each size; keep the fastest."""
        arr = (ctypes.c_uint32 * len(sizes))(*[int(x) for x in sizes])
        _check(
            self._lib.gf2x_tune(self._h, arr, len(sizes), int(batch), out_path.encode() if out_path else None),
            "gf2x_tune",
        )

    def schedule_info(self, n):
        """(padded 32-bit words, base 32x32 products, algorithmic lane-ops, name) for n."""
        s = ctypes.c_uint32()
        base = ctypes.c_uint64()
        ops = ctypes.c_uint64()
        name = ctypes.create_string_buffer(64)
        _check(
            self._lib.gf2x_schedule_info(
                self._h, int(n), ctypes.byref(s), ctypes.byref(base), ctypes.byref(ops), name, 64
            ),
            "gf2x_schedule_info",
        )
        return s.value, base.value, ops.value, name.value.decode()


class Plan:
    """A recorded batch (gf2x_plan_* in the C ABI); launch() replays it."""

    def __init__(self, ctx, items, c_base, a_base, b_base, flags=0):
        self._lib = load()
        self._ctx = ctx
        items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
        h = ctypes.c_void_p()
        _check(
            self._lib.gf2x_plan_create(ctypes.byref(h), ctx._h, items.ctypes.data, len(items), _ptr(c_base),
                                       _ptr(a_base), _ptr(b_base), int(flags)),
            "gf2x_plan_create",
        )
        self._h = h

    def launch(self, stream=None):
        _check(self._lib.gf2x_plan_launch(self._h, _stream(stream)), "gf2x_plan_launch")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gf2x_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over a Context (gf2x_srv_* in the C ABI).
    Operands and results are host numpy uint64 arrays with word offsets; the
    server keeps references to them until drain() returns."""

    def __init__(self, ctx, hbm_budget_bytes=0, streams=0, max_bits=0, max_batch=0, max_pending=0):
        self._lib = load()
        self._ctx = ctx
        opts = _SrvOpts(hbm_budget_bytes, streams, max_bits, max_batch, max_pending, 0)
        h = ctypes.c_void_p()
        _check(self._lib.gf2x_srv_create(ctypes.byref(h), ctx._h, ctypes.byref(opts)), "gf2x_srv_create")
        self._h = h
        self._keep = []

    def now_ns(self):
        return self._lib.gf2x_srv_now_ns()

    def submit(self, n_bits, a, a_off, b, b_off, c, c_off, arrival_ns=None):
        """Queue requests; returns the first ticket (tickets are consecutive)."""
        arrs = [np.ascontiguousarray(n_bits, dtype=np.uint32)]
        for x in (a_off, b_off, c_off):
            arrs.append(np.ascontiguousarray(x, dtype=np.uint64))
        arr_ns = None if arrival_ns is None else np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        for buf in (a, b, c):
            if buf.dtype != np.uint64 or not buf.flags.c_contiguous:
                raise ValueError("operand and result buffers must be contiguous uint64 arrays")
        count = len(arrs[0])
        first = ctypes.c_uint64()
        rc = self._lib.gf2x_srv_submit(
            self._h, count, arrs[0].ctypes.data, a.ctypes.data, arrs[1].ctypes.data, b.ctypes.data,
            arrs[2].ctypes.data, c.ctypes.data, arrs[3].ctypes.data,
            None if arr_ns is None else arr_ns.ctypes.data, ctypes.byref(first))
        _check(rc, "gf2x_srv_submit")
        self._keep.append((arrs, arr_ns, a, b, c))
        return first.value

    def completion(self, first, count):
        out = np.zeros(count, dtype=np.uint64)
        _check(self._lib.gf2x_srv_completion(self._h, first, count, out.ctypes.data), "gf2x_srv_completion")
        return out

    def drain(self, timeout_ms=0):
        _check(self._lib.gf2x_srv_drain(self._h, timeout_ms), "gf2x_srv_drain")
        self._keep = []

    def stats(self):
        st = SrvStats()
        _check(self._lib.gf2x_srv_get_stats(self._h, ctypes.byref(st)), "gf2x_srv_get_stats")
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gf2x_srv_destroy(self._h)
            self._h = None
            self._keep = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_items(n_bits, kinds, a_off, b_off, c_off):
    """Pack per-item arrays (broadcast) into a numpy array of ITEM_DTYPE."""
    count = max(np.size(x) for x in (n_bits, kinds, a_off, b_off, c_off))
    it = np.zeros(count, dtype=ITEM_DTYPE)
    it["n_bits"] = n_bits
    it["kind"] = kinds
    it["a_off"] = a_off
    it["b_off"] = b_off
    it["c_off"] = c_off
    return it


def version():
    return load().gf2x_version()
