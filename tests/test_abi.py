"""The C-ABI library: it loads, exports every entry point the header declares,
and its host-side argument checks and schedule table behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2201_10473_amd import gf2x

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gf2x.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf2x_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = gf2x.load()
    names = _declared_functions()
    assert "gf2x_mul" in names and "gf2x_mul_cyclic" in names and "gf2x_mul_batched" in names
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_strerror():
    lib = gf2x.load()
    assert gf2x.version() == 10000
    for code in (0, -1, -2, -3, -5, -99):
        assert lib.gf2x_strerror(code)
    assert lib.gf2x_strerror(-1) != lib.gf2x_strerror(-2)


def test_null_context_is_rejected_without_touching_a_device():
    lib = gf2x.load()
    p = 4096  # never dereferenced: the check fails first
    assert lib.gf2x_mul(None, p, p + 8 * 1024, p + 16 * 1024, 17669, None) == gf2x.GF2X_EINVAL
    assert lib.gf2x_mul_cyclic(None, p, p, p, 17669, None) == gf2x.GF2X_EINVAL
    assert lib.gf2x_mul_batched(None, p, 1, p, p, p, 0, None) == gf2x.GF2X_EINVAL
    assert lib.gf2x_create(None, None) == gf2x.GF2X_EINVAL


def _info(n):
    lib = gf2x.load()
    s = ctypes.c_uint32()
    base = ctypes.c_uint64()
    ops = ctypes.c_uint64()
    name = ctypes.create_string_buffer(64)
    rc = lib.gf2x_schedule_info(None, n, ctypes.byref(s), ctypes.byref(base), ctypes.byref(ops), name, 64)
    return rc, s.value, base.value, ops.value, name.value.decode()


def test_schedule_table_covers_every_size():
    prev_ops = 0
    for n in list(range(1, 300)) + list(range(300, gf2x.GF2X_MAX_BITS + 1, 997)) + [gf2x.GF2X_MAX_BITS]:
        rc, s, base, ops, name = _info(n)
        assert rc == 0
        assert s * 32 >= n
        assert base > 0 and ops > base and name
    assert _info(0)[0] == gf2x.GF2X_EINVAL
    assert _info(gf2x.GF2X_MAX_BITS + 1)[0] == gf2x.GF2X_EINVAL


@pytest.mark.parametrize("n", [12323, 17669, 24659, 35851, 40973, 57637])
def test_schedule_for_ring_sizes_is_subquadratic(n):
    rc, s, base, ops, name = _info(n)
    w32 = (n + 31) // 32
    assert rc == 0 and s >= w32
    # far fewer base products than the w32^2 of a word schoolbook
    assert base < 0.3 * w32 * w32
    assert "T3" in name or "K2" in name


def test_server_rejects_null_context():
    lib = gf2x.load()
    h = ctypes.c_void_p()
    assert lib.gf2x_srv_create(ctypes.byref(h), None, None) == gf2x.GF2X_EINVAL
    assert lib.gf2x_srv_drain(None, 1) == gf2x.GF2X_EINVAL
    assert lib.gf2x_srv_now_ns() > 0
    lib.gf2x_srv_destroy(None)


def test_plan_entry_points_reject_null_arguments():
    lib = gf2x.load()
    p = 4096  # never dereferenced: the checks fail first
    assert lib.gf2x_plan_create(None, None, p, 1, p, p, p, 0) == gf2x.GF2X_EINVAL
    out = ctypes.c_void_p()
    assert lib.gf2x_plan_create(ctypes.byref(out), None, p, 1, p, p, p, 0) == gf2x.GF2X_EINVAL
    assert out.value is None
    assert lib.gf2x_plan_launch(None, None) == gf2x.GF2X_EINVAL
    lib.gf2x_plan_destroy(None)
