"""Host logic of the request server that runs without a GPU: admission by budget and slot layout.

ipls_server_reserve only does arena bookkeeping, so it is exercised here with an arena address
that is never dereferenced (nothing is submitted, so no lane touches memory).
"""
import ctypes as C
import os

import pytest

import paper_2208_06902_amd as ipls

pytestmark = pytest.mark.skipif(not os.path.exists(ipls.LIB_PATH), reason="libipls.so not built")

FAKE_ARENA = 1 << 40  # 256-byte aligned, never dereferenced


def make_server(arena_bytes, **kw):
    L = ipls.load()
    cfg = ipls.server_config(**kw)
    h = C.c_void_p()
    assert L.ipls_server_create(C.c_void_p(FAKE_ARENA), arena_bytes, C.byref(cfg), C.byref(h)) == 0
    return L, h


def reserve(L, h, n, dtype, pay=False):
    rid, kp, pp = C.c_uint64(), C.c_void_p(), C.c_void_p()
    st = L.ipls_server_reserve(h, n, dtype, int(pay), C.byref(rid), C.byref(kp), C.byref(pp))
    return st, rid.value, kp.value, pp.value


def test_small_requests_share_a_contiguous_batch_buffer():
    L, h = make_server(1 << 30, batch_max_keys=1000, batch_keys=10_000, lanes=1)
    try:
        st0, r0, k0, p0 = reserve(L, h, 100, ipls.F64, True)
        st1, r1, k1, p1 = reserve(L, h, 250, ipls.F64, True)
        st2, r2, k2, p2 = reserve(L, h, 7, ipls.F64, True)
        assert (st0, st1, st2) == (0, 0, 0) and r0 < r1 < r2
        assert k1 == k0 + 100 * 8 and k2 == k1 + 250 * 8  # keys of one batch are contiguous
        assert p1 == p0 + 100 * 4 and p2 == p1 + 250 * 4
        # another class (fp32, no payload) opens its own batch buffer
        st3, _, k3, p3 = reserve(L, h, 100, ipls.F32, False)
        assert st3 == 0 and p3 is None and not (k0 <= k3 < k0 + 10_000 * 8)
    finally:
        L.ipls_server_destroy(h)


def test_full_batch_opens_a_new_one():
    L, h = make_server(1 << 30, batch_max_keys=1000, batch_keys=2000, lanes=1)
    try:
        _, _, k0, _ = reserve(L, h, 1000, ipls.U64)
        _, _, k1, _ = reserve(L, h, 1000, ipls.U64)
        _, _, k2, _ = reserve(L, h, 1, ipls.U64)  # does not fit the first buffer
        assert k1 == k0 + 8000
        assert not (k0 <= k2 < k0 + 2000 * 8)
    finally:
        L.ipls_server_destroy(h)


def test_large_requests_get_own_slots_and_the_budget_is_enforced():
    n = 1_000_000
    per_request = 2 * n * 8  # slot + ping-pong workspace
    L, h = make_server(3 * per_request + 4096, batch_max_keys=1000, batch_keys=2000, lanes=2)
    try:
        slots = [reserve(L, h, n, ipls.F64) for _ in range(3)]
        assert all(s[0] == 0 for s in slots)
        keys = sorted(s[2] for s in slots)
        assert all(b - a >= per_request for a, b in zip(keys, keys[1:]))
        st, *_ = reserve(L, h, n, ipls.F64)
        assert st == 3  # IPLS_ERR_OOM: not now
        stats = ipls.ServerStats()
        assert L.ipls_server_stats_get(h, C.byref(stats)) == 0
        assert stats.admitted == 3 and stats.rejected == 1 and stats.bytes_in_use >= 3 * per_request
    finally:
        L.ipls_server_destroy(h)


def test_invalid_config_and_unknown_request():
    L = ipls.load()
    h = C.c_void_p()
    bad = ipls.server_config(lanes=0)
    assert L.ipls_server_create(C.c_void_p(FAKE_ARENA), 1 << 20, C.byref(bad), C.byref(h)) == 1
    bad = ipls.server_config(batch_max_keys=10, batch_keys=5)
    assert L.ipls_server_create(C.c_void_p(FAKE_ARENA), 1 << 20, C.byref(bad), C.byref(h)) == 1
    assert L.ipls_server_create(C.c_void_p(FAKE_ARENA + 8), 1 << 20, None, C.byref(h)) == 1  # misaligned
    L, h = make_server(1 << 20, lanes=1)
    try:
        assert L.ipls_server_release(h, 12345) == 1
        with pytest.raises(TypeError):
            ipls.server_config(lane=2)
    finally:
        L.ipls_server_destroy(h)
