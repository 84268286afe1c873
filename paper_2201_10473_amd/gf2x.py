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
GF2X_ENOTSUP = -5
GF2X_MAX_BITS = 131072

KIND_CYCLIC = 0
KIND_FULL = 1

ITEMS_ON_DEVICE = 0x1
SHARED_A = 0x2
FORCE_PACKED = 0x4
FORCE_TOEPLITZ = 0x8
USE_GRAPH = 0x10

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


def load():
    """Load the built library (raises if it is missing: no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libgf2x.so is not built (expected at %s); run __graft_entry__.build()" % LIB_PATH
        )
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
    lib.gf2x_schedule_info.argtypes = [
        vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.c_char_p, sz
    ]
    lib.gf2x_schedule_info.restype = ctypes.c_int
    lib.gf2x_tune.argtypes = [vp, ctypes.POINTER(u32), u32, u32, ctypes.c_char_p]
    lib.gf2x_tune.restype = ctypes.c_int
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
