"""Host-side checks of the C ABI that need no GPU: the library loads, exports every entry point
the header declares, sizes storage as documented, and rejects bad arguments before touching a
device."""
import ctypes
import os

import numpy as np
import pytest

from paper_1710_11246_amd import slabhash as S


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(S.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return S.lib()


def test_exports_every_declared_symbol(lib):
    declared = S.declared_symbols()
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(S._SIGS), "binding and header disagree"


def test_storage_bytes(lib):
    p = S.ShParams(4096, 4 * 2048, 12345, 678)
    hdr = 4096  # header + counter slots
    want = hdr + 4096 * 256 + 4 * 2048 * 256 + 4 * 256
    assert S.sh_storage_bytes(p) == want
    assert S.sh_storage_bytes(S.ShParams(1, 0, 1, 0)) == hdr + 256
    # invalid: zero buckets, pool not a multiple of 2048, a = 0, a >= p, b >= p, B + P too big
    assert S.sh_storage_bytes(S.ShParams(16, 0, 3, 5, 3)) == S.sh_storage_bytes(S.ShParams(16, 0, 3, 5))
    for bad in [S.ShParams(0, 0, 1, 0), S.ShParams(8, 100, 1, 0), S.ShParams(8, 0, 0, 0),
                S.ShParams(8, 0, 1, 0, 4), S.ShParams(8, 0, 1, 0, 0x80000000),
                S.ShParams(8, 0, S.SH_HASH_PRIME, 0), S.ShParams(8, 0, 1, S.SH_HASH_PRIME),
                S.ShParams(0xFFFFFFFF - 2048, 2048, 1, 0)]:
        assert S.sh_storage_bytes(bad) == 0


def test_argument_errors_before_any_device_call(lib):
    p = S.ShParams(16, 0, 3, 5)
    out = ctypes.c_void_p()
    # null storage, too small, misaligned, null out: all EINVAL without a device
    assert lib.sh_create(ctypes.byref(p), None, 1 << 20, None, ctypes.byref(out)) == S.SH_EINVAL
    assert lib.sh_create(ctypes.byref(p), 256, 16, None, ctypes.byref(out)) == S.SH_EINVAL
    assert lib.sh_create(ctypes.byref(p), 257, 1 << 20, None, ctypes.byref(out)) == S.SH_EINVAL
    assert lib.sh_create(ctypes.byref(p), 256, 1 << 20, None, None) == S.SH_EINVAL
    bad = S.ShParams(0, 0, 1, 0)
    assert lib.sh_create(ctypes.byref(bad), 256, 1 << 20, None, ctypes.byref(out)) == S.SH_EINVAL
    # null table handle
    assert lib.sh_build(None, 256, 256, 10, None, None) == S.SH_EINVAL
    assert lib.sh_search(None, 256, 10, 256, None, None) == S.SH_EINVAL
    assert lib.sh_delete(None, 256, 10, None, None) == S.SH_EINVAL
    assert lib.sh_mixed(None, 256, 256, 256, 10, 256, 256, None) == S.SH_EINVAL
    assert lib.sh_stats(None, None, None) == S.SH_EINVAL
    assert lib.sh_dump(None, None, None, None, 0, None, None, None, None) == S.SH_EINVAL
    assert lib.sh_reset(None, None) == S.SH_EINVAL
    assert lib.sh_flush(None, 0, 1, None) == S.SH_EINVAL
    assert lib.sh_alloc_slabs(None, 10, 256, None) == S.SH_EINVAL
    assert lib.sh_free_slabs(None, 256, 10, None) == S.SH_EINVAL
    assert lib.sh_destroy(None) == S.SH_EINVAL
    assert lib.sh_set_launch(None, None) == S.SH_EINVAL
    w, c = ctypes.c_uint32(), ctypes.c_uint32()
    assert lib.sh_launch_shape(None, 0, 10, ctypes.byref(w), ctypes.byref(c)) == S.SH_EINVAL


def test_strerror(lib):
    assert S.sh_strerror(S.SH_OK) == "ok"
    assert S.sh_strerror(S.SH_EINVAL) == "invalid argument"
    assert S.sh_strerror(99) == "unknown status"


def test_pool_bound_holds_worst_case():
    # one bucket holding every key needs ceil(n/31) - 1 pool slabs
    for n in [1, 31, 32, 1000, 2048 * 31 + 5]:
        assert S.pool_slabs_bound(n, 0) >= -(-n // 31) - 1
        assert S.pool_slabs_bound(n) % 2048 == 0


def test_multi_argument_errors(lib):
    p = (S.ShParams * 2)(S.ShParams(16, 0, 3, 5), S.ShParams(100, 2048, 7, 9))
    one = S.sh_storage_bytes(S.ShParams(16, 0, 3, 5))
    two = S.sh_storage_bytes(S.ShParams(100, 2048, 7, 9))
    rnd = lambda x: (x + 255) // 256 * 256
    assert lib.sh_multi_storage_bytes(2, p) == rnd(2 * 64) + rnd(one) + rnd(two)
    assert lib.sh_multi_storage_bytes(0, p) == 0
    bad = (S.ShParams * 2)(S.ShParams(16, 0, 3, 5), S.ShParams(0, 0, 1, 0))
    assert lib.sh_multi_storage_bytes(2, bad) == 0
    out = ctypes.c_void_p()
    assert lib.sh_multi_create(2, p, 257, 1 << 30, None, ctypes.byref(out)) == S.SH_EINVAL
    assert lib.sh_multi_create(2, p, 256, 16, None, ctypes.byref(out)) == S.SH_EINVAL
    assert lib.sh_multi_create(0, p, 256, 1 << 30, None, ctypes.byref(out)) == S.SH_EINVAL
    assert lib.sh_multi_mixed(None, 256, 1, 256, 256, 256, 256, 256, 10, None) == S.SH_EINVAL
    assert lib.sh_multi_graph(None, 256, 1, 256, 256, 256, 256, 256, 10, None) == S.SH_EINVAL
    assert lib.sh_multi_mixed_each(None, 256, 1, 256, 256, 256, 256, 256, 10, None) == S.SH_EINVAL
    assert lib.sh_multi_table(None, 0, ctypes.byref(out)) == S.SH_EINVAL
    assert lib.sh_multi_set_launch(None, None) == S.SH_EINVAL
    assert lib.sh_graph_launch(None, None) == S.SH_EINVAL
    assert lib.sh_graph_destroy(None) == S.SH_EINVAL
    assert lib.sh_multi_destroy(None) == S.SH_EINVAL
    d = S.pack_batch_descs([0, 7], [7, 3], [1, 2]).view(np.uint8).reshape(2, 16)
    assert int.from_bytes(bytes(d[1, :8]), "little") == 7
    assert int.from_bytes(bytes(d[1, 8:12]), "little") == 3
    assert int.from_bytes(bytes(d[1, 12:16]), "little") == 2


def test_server_argument_errors(lib):
    assert S.sh_server_scratch_bytes() == 256 + 4 * 4096 * 16
    assert S.sh_server_scratch_bytes(S.ShServerCfg(8, 0, 0, 0, 0)) == 256 + 8 * 4096 * 16
    assert S.sh_server_scratch_bytes(S.ShServerCfg(9, 0, 0, 0, 0)) == 0
    out = ctypes.c_void_p()
    assert lib.sh_server_start(None, None, 256, 256, 256, 256, 256, 10, 256, 1 << 20, None,
                               ctypes.byref(out)) == S.SH_EINVAL
    req = S.ShRequest(0, 1, 0)
    tk = ctypes.c_uint64()
    assert lib.sh_server_submit(None, ctypes.byref(req), ctypes.byref(tk)) == S.SH_EINVAL
    assert lib.sh_server_poll(None, 0, None, None, None) == S.SH_EINVAL
    assert lib.sh_server_replay(None, None, None, 0, None, None) == S.SH_EINVAL
    assert lib.sh_server_stop(None) == S.SH_EINVAL
    a, b = S.sh_clock_ns(), S.sh_clock_ns()
    assert 0 < a <= b


def test_roofs_library_exports_and_argument_errors():
    from paper_1710_11246_amd import roofs as R
    if not os.path.exists(R.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    rl = R.lib()
    declared = R.declared_symbols()
    assert declared == ["sh_roof_insert", "sh_roof_run", "sh_roof_search"]
    assert set(declared) == set(R._SIGS) and all(hasattr(rl, d) for d in declared)
    buf = ctypes.c_void_p(1 << 20)  # aligned stand-in; every call below fails before using it
    bad = [(7, buf, 1 << 20, 10, 0, 0), (-1, buf, 1 << 20, 10, 0, 0),
           (0, None, 1 << 20, 10, 0, 0), (0, ctypes.c_void_p((1 << 20) + 8), 1 << 20, 10, 0, 0),
           (0, buf, 100, 10, 0, 0), (0, buf, 300, 10, 0, 0), (0, buf, 1 << 20, 1 << 32, 0, 0),
           (0, buf, 1 << 20, (1 << 32) - 64, 0, 0), (0, buf, 1 << 20, 10, 65, 0),
           (0, buf, 1 << 20, 10, 0, 3), (0, buf, 1 << 20, 10, 0, 32)]
    for kind, p, nbytes, n, wpc, depth in bad:
        assert rl.sh_roof_run(kind, p, nbytes, n, wpc, depth, 1, None) == S.SH_EINVAL
    # no operations: nothing is enqueued and no device is touched
    assert rl.sh_roof_run(1, buf, 1 << 20, 0, 0, 0, 1, None) == S.SH_OK
    arr = ctypes.c_void_p(1 << 24)  # stand-in key and result arrays, never used either
    bad = [(None, 1 << 20, arr, 10, arr, arr, 0, 0), (ctypes.c_void_p((1 << 20) + 8), 1 << 20,
           arr, 10, arr, arr, 0, 0), (buf, 300, arr, 10, arr, arr, 0, 0),
           (buf, 1 << 20, arr, (1 << 32) - 64, arr, arr, 0, 0), (buf, 1 << 20, None, 10, arr, arr,
           0, 0), (buf, 1 << 20, arr, 10, None, arr, 0, 0), (buf, 1 << 20, arr, 10, arr, None, 0,
           0), (buf, 1 << 20, arr, 10, arr, arr, 65, 0), (buf, 1 << 20, arr, 10, arr, arr, 0, 2)]
    for p, nbytes, k, n, v, f, wpc, depth in bad:
        assert rl.sh_roof_search(p, nbytes, k, n, v, f, wpc, depth, None) == S.SH_EINVAL
    assert rl.sh_roof_search(buf, 1 << 20, None, 0, None, None, 0, 0, None) == S.SH_OK
    bad = [(None, 1 << 20, arr, arr, 10, arr, 0, 0), (buf, 300, arr, arr, 10, arr, 0, 0),
           (buf, 1 << 20, None, arr, 10, arr, 0, 0), (buf, 1 << 20, arr, None, 10, arr, 0, 0),
           (buf, 1 << 20, arr, arr, 10, None, 0, 0), (buf, 1 << 20, arr, arr, 10, arr, 65, 0),
           (buf, 1 << 20, arr, arr, 10, arr, 0, 3), (buf, 1 << 20, arr, arr, 1 << 32, arr, 0, 0)]
    for p, nbytes, k, v, n, st, wpc, depth in bad:
        assert rl.sh_roof_insert(p, nbytes, k, v, n, st, wpc, depth, None) == S.SH_EINVAL
    assert rl.sh_roof_insert(buf, 1 << 20, None, None, 0, None, 0, 0, None) == S.SH_OK


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message before touching a
    device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
