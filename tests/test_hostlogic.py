"""CPU tests of the library's host logic: the pool sub-allocator and the
field cache (LRU spill to the pinned host area, fill on use, pinning, pool
limit, fault injection), driven through the library's own headers with a
fake mover that copies between host byte arrays."""

import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1111_5596_amd", "csrc")

OK, ERR_NOMEM, ERR_STATE = 0, -4, -8


@pytest.fixture(scope="module")
def hl(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("hostlogic") / "libhostlogic.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-shared", "-fPIC", "-Wall", "-I", CSRC,
                    os.path.join(ROOT, "tests", "hostlogic", "capi.cpp"), "-o", out], check=True)
    lib = ctypes.CDLL(out)
    u64, sz, vp = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p
    for name, res, args in [
        ("hl_create", vp, [sz, sz]), ("hl_destroy", None, [vp]),
        ("hl_create_field", ctypes.c_int, [vp, u64, sz]), ("hl_destroy_field", ctypes.c_int, [vp, u64]),
        ("hl_acquire", ctypes.c_int, [vp, u64, ctypes.c_int]), ("hl_release", None, [vp, u64]),
        ("hl_evict", ctypes.c_int, [vp, u64]), ("hl_evict_all", ctypes.c_int, [vp]),
        ("hl_set_limit", ctypes.c_int, [vp, sz]), ("hl_fault_after", None, [vp, ctypes.c_int64]),
        ("hl_swap", ctypes.c_int, [vp, u64, u64]), ("hl_write", ctypes.c_int, [vp, u64, ctypes.c_uint8]),
        ("hl_verify", ctypes.c_int, [vp, u64, ctypes.c_uint8]),
        ("hl_info", ctypes.c_int, [vp, u64, ctypes.POINTER(ctypes.c_int64)]),
        ("hl_counters", None, [vp, ctypes.POINTER(ctypes.c_uint64)]), ("hl_check", ctypes.c_int, [vp]),
        ("pl_create", vp, [sz]), ("pl_destroy", None, [vp]), ("pl_alloc", ctypes.c_int64, [vp, sz]),
        ("pl_release", ctypes.c_int, [vp, sz]), ("pl_check", ctypes.c_int, [vp]), ("pl_used", sz, [vp]),
        ("pl_largest", sz, [vp]), ("pl_set_limit", None, [vp, sz])]:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


class Cache:
    def __init__(self, lib, dev, host):
        self.lib, self.h = lib, lib.hl_create(dev, host)

    def __getattr__(self, name):
        fn = getattr(self.lib, "hl_" + name)
        return lambda *a: fn(self.h, *a)

    def info(self, i):
        out = (ctypes.c_int64 * 6)()
        assert self.lib.hl_info(self.h, i, out) == 0
        return dict(zip(["on_device", "dev_off", "on_host", "host_off", "pins", "bytes"], out))

    def counters(self):
        out = (ctypes.c_uint64 * 11)()
        self.lib.hl_counters(self.h, out)
        return dict(zip(["hits", "misses", "spills", "fills", "bytes_spilled", "bytes_filled", "used",
                         "high_water", "host_used", "limit", "copies"], out))


def test_pool_first_fit_coalescing_and_limit(hl):
    p = hl.pl_create(1 << 20)
    rng = np.random.default_rng(0)
    live = {}
    for step in range(2000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            assert hl.pl_release(p, off) == 0
            del live[off]
        else:
            n = int(rng.integers(1, 40000))
            off = hl.pl_alloc(p, n)
            if off >= 0:
                assert off % 256 == 0
                for o, m in live.items():  # no overlap
                    assert off + n <= o or o + m <= off
                live[off] = n
        assert hl.pl_check(p) == 0
    for off in list(live):
        hl.pl_release(p, off)
    assert hl.pl_used(p) == 0 and hl.pl_largest(p) == 1 << 20 and hl.pl_check(p) == 0
    assert hl.pl_release(p, 12345) == -1  # unknown block
    hl.pl_set_limit(p, 4096)
    assert hl.pl_alloc(p, 8192) == -1 and hl.pl_alloc(p, 4096) == 0
    hl.pl_destroy(p)


def test_lru_spill_and_fill_preserve_contents(hl):
    c = Cache(hl, 4096 * 4, 4096 * 8)
    for i in range(1, 5):
        assert c.create_field(i, 4000) == OK
        assert c.write(i, i) == 0
    # touching 1 makes 2 the least recently used
    assert c.acquire(1, 1) == OK
    c.release(1)
    assert c.create_field(5, 4000) == OK  # must spill exactly field 2
    assert not c.info(2)["on_device"] and c.info(2)["on_host"]
    assert all(c.info(i)["on_device"] for i in (1, 3, 4, 5))
    k = c.counters()
    assert k["spills"] == 1 and k["bytes_spilled"] == 4000
    # using 2 again fills it (spilling the LRU among 1, 3, 4, 5, i.e. 3)
    assert c.acquire(2, 1) == OK
    assert c.verify(2, 2) == 0
    c.release(2)
    assert not c.info(3)["on_device"]
    k = c.counters()
    assert k["fills"] == 1 and k["misses"] == 1 and k["spills"] == 2
    assert c.acquire(3, 1) == OK and c.verify(3, 3) == 0
    c.release(3)
    assert c.check() == 0


def test_pinned_fields_are_never_evicted(hl):
    c = Cache(hl, 4096 * 2, 4096 * 4)
    c.create_field(1, 4096)
    c.create_field(2, 4096)
    assert c.acquire(1, 1) == OK and c.acquire(2, 1) == OK
    assert c.create_field(3, 4096) == ERR_NOMEM  # everything pinned
    c.release(1)
    assert c.create_field(3, 4096) == OK
    assert not c.info(1)["on_device"] and c.info(2)["on_device"]
    assert c.evict(2) == ERR_STATE  # still pinned
    c.release(2)
    assert c.evict(2) == OK
    assert c.check() == 0


def test_acquire_without_contents_skips_copy(hl):
    c = Cache(hl, 4096, 4096)
    c.create_field(1, 4096)
    c.write(1, 9)
    assert c.evict(1) == OK
    before = c.counters()["copies"]
    assert c.acquire(1, 0) == OK  # overwrite-only use: no host->device copy
    assert c.counters()["copies"] == before and c.counters()["fills"] == 0
    assert c.info(1)["on_device"] and not c.info(1)["on_host"] and c.counters()["host_used"] == 0


def test_nomem_when_spill_area_full_and_no_spill_area(hl):
    c = Cache(hl, 4096 * 2, 4096)
    c.create_field(1, 4096)
    c.create_field(2, 4096)
    assert c.create_field(3, 4096) == OK  # spills 1 into the only host slot
    assert c.create_field(4, 4096) == ERR_NOMEM  # host area full
    assert c.info(2)["on_device"] and c.info(3)["on_device"]
    c2 = Cache(hl, 4096, 0)
    c2.create_field(1, 4096)
    assert c2.create_field(2, 4096) == ERR_NOMEM
    assert c.check() == 0 and c2.check() == 0


def test_pool_limit_moves_or_spills(hl):
    c = Cache(hl, 4096 * 4, 4096 * 4)
    for i in range(1, 5):
        c.create_field(i, 4096)
        c.write(i, 10 * i)
    c.destroy_field(1)  # hole at the bottom
    assert c.set_limit(4096 * 2) == OK
    used = [i for i in (2, 3, 4) if c.info(i)["on_device"]]
    assert len(used) == 2 and all(c.info(i)["dev_off"] + 4096 <= 8192 for i in used)
    for i in (2, 3, 4):
        assert c.acquire(i, 1) == OK and c.verify(i, 10 * i) == 0
        c.release(i)
    assert c.counters()["limit"] == 8192 and c.check() == 0


def test_fault_injection_and_swap(hl):
    c = Cache(hl, 4096 * 8, 0)
    c.fault_after(2)
    assert c.create_field(1, 100) == OK
    assert c.create_field(2, 100) == ERR_NOMEM  # injected, nothing leaked
    assert c.create_field(2, 100) == OK
    assert c.counters()["used"] == 512
    c.write(1, 1)
    c.write(2, 2)
    assert c.swap(1, 2) == OK
    assert c.verify(1, 2) == 0 and c.verify(2, 1) == 0
    assert c.destroy_field(1) == OK and c.destroy_field(1) == ERR_STATE
    assert c.check() == 0


def test_external_block_spills_fields_and_pins_the_limit(hl):
    """An external allocation (pinned for life, as qdp_pool_malloc makes it)
    spills LRU fields to make room, is never chosen as a victim, and a pool
    limit below its end is refused without changing anything."""
    c = Cache(hl, 4096 * 4, 4096 * 4)
    for i in range(1, 4):
        assert c.create_field(i, 4096) == OK
        c.write(i, i)
    assert c.create_field(100, 4096 * 2) == OK and c.acquire(100, 0) == OK  # the external block
    k = c.counters()
    # 1 and 2, the least recently used, made a contiguous hole
    assert k["spills"] == 2 and not c.info(1)["on_device"] and not c.info(2)["on_device"]
    # more demand spills fields, never the block
    for i in (1, 2, 3):
        assert c.acquire(i, 1) == OK and c.verify(i, i) == 0
        c.release(i)
        assert c.info(100)["on_device"] and c.info(100)["pins"] == 1
    before = (c.counters()["limit"], [c.info(i)["dev_off"] for i in (100,)])
    end = c.info(100)["dev_off"] + 4096 * 2
    assert c.set_limit(end - 4096) == ERR_STATE
    assert (c.counters()["limit"], [c.info(i)["dev_off"] for i in (100,)]) == before
    assert c.create_field(101, 4096 * 3) == ERR_NOMEM  # cannot fit beside the pinned block
    c.release(100)
    assert c.destroy_field(100) == OK and c.check() == 0
