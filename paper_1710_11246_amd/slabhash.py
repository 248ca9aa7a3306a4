"""Python binding of libslabhash.so (include/slabhash.h): argument marshalling only.

Every function here has the name of the C entry point it calls and only converts arguments:
torch tensors (device memory) become pointers, a torch stream becomes a hipStream_t. All work
runs in the HIP kernels of the library. The library is loaded on first use and a missing or
unloadable library raises immediately; there is no other code path.

Keys and values are uint32 bit patterns carried in torch.int32 tensors (torch has no general
uint32 support); ops, statuses and found flags are torch.uint8.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libslabhash.so")
HEADER_PATH = os.path.join(os.path.dirname(PKG), "include", "slabhash.h")

SH_OK, SH_EINVAL, SH_ENOMEM, SH_EHIP, SH_EBUSY = 0, 1, 2, 3, 4
SH_OP_SEARCH, SH_OP_INSERT, SH_OP_DELETE = 0, 1, 2
SH_KIND_MIXED = 3
SH_ERR_RESERVED_KEY, SH_ERR_POOL_EXHAUSTED = 1, 2
SH_EMPTY_KEY = 0xFFFFFFFF
SH_HASH_PRIME = 4294967291
SH_SLAB_BYTES = 256
SH_SLAB_PAIRS = 31
SH_BLOCK_SLABS = 2048
SH_MAX_BATCHES = 4096


SH_TABLE_DUPLICATES, SH_TABLE_KEYS_ONLY = 1, 2


class ShParams(ctypes.Structure):
    _fields_ = [("num_buckets", ctypes.c_uint32), ("pool_slabs", ctypes.c_uint32),
                ("hash_a", ctypes.c_uint32), ("hash_b", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


SH_LAUNCH_COUNTERS = 1


class ShLaunch(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_uint32), ("ops_per_wave", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ShStats(ctypes.Structure):
    _fields_ = [("live", ctypes.c_uint64), ("tombstones", ctypes.c_uint64),
                ("slabs_total", ctypes.c_uint64), ("pool_allocated", ctypes.c_uint64),
                ("pool_capacity", ctypes.c_uint64), ("error_word", ctypes.c_uint32),
                ("violations", ctypes.c_uint32), ("num_buckets", ctypes.c_uint32),
                ("hash_a", ctypes.c_uint32), ("hash_b", ctypes.c_uint32),
                ("hash_p", ctypes.c_uint32), ("rounds", ctypes.c_uint64),
                ("cas_lost", ctypes.c_uint64), ("allocs", ctypes.c_uint64),
                ("link_lost", ctypes.c_uint64), ("block_moves", ctypes.c_uint64),
                ("alloc_lost", ctypes.c_uint64)]


class ShServerCfg(ctypes.Structure):
    _fields_ = [("max_launches", ctypes.c_uint32), ("max_batch_ops", ctypes.c_uint32),
                ("max_requests", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
                ("reserve_slabs", ctypes.c_uint64)]


class ShRequest(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint64), ("length", ctypes.c_uint32),
                ("inserts", ctypes.c_uint32)]


class SlabHashError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__("%s failed: %s (%d)" % (fn, sh_strerror(code), code))
        self.code = code


_P, _U32, _U64, _SZ = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
_SIGS = {
    "sh_storage_bytes": ([_P], _SZ),
    "sh_create": ([_P, _P, _SZ, _P, _P], ctypes.c_int),
    "sh_reset": ([_P, _P], ctypes.c_int),
    "sh_flush": ([_P, _U32, _U32, _P], ctypes.c_int),
    "sh_alloc_slabs": ([_P, _U64, _P, _P], ctypes.c_int),
    "sh_search_all": ([_P, _P, _U64, _P, _P, _P, _U64, _P], ctypes.c_int),
    "sh_super_block_bytes": ([_U32], _SZ),
    "sh_add_super_block": ([_P, _P, _SZ, _P], ctypes.c_int),
    "sh_delete_all": ([_P, _P, _U64, _P, _P], ctypes.c_int),
    "sh_free_slabs": ([_P, _P, _U64, _P], ctypes.c_int),
    "sh_destroy": ([_P], ctypes.c_int),
    "sh_set_launch": ([_P, _P], ctypes.c_int),
    "sh_launch_shape": ([_P, ctypes.c_int, ctypes.c_uint64, _P, _P], ctypes.c_int),
    "sh_build": ([_P, _P, _P, _U64, _P, _P], ctypes.c_int),
    "sh_insert": ([_P, _P, _P, _U64, _P, _P], ctypes.c_int),
    "sh_delete": ([_P, _P, _U64, _P, _P], ctypes.c_int),
    "sh_search": ([_P, _P, _U64, _P, _P, _P], ctypes.c_int),
    "sh_mixed": ([_P, _P, _P, _P, _U64, _P, _P, _P], ctypes.c_int),
    "sh_stats": ([_P, _P, _P], ctypes.c_int),
    "sh_dump": ([_P, _P, _P, _P, _U64, _P, _P, _P, _P], ctypes.c_int),
    "sh_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "sh_multi_storage_bytes": ([_U32, _P], _SZ),
    "sh_multi_create": ([_U32, _P, _P, _SZ, _P, _P], ctypes.c_int),
    "sh_multi_table": ([_P, _U32, _P], ctypes.c_int),
    "sh_multi_set_launch": ([_P, _P], ctypes.c_int),
    "sh_multi_mixed": ([_P, _P, _U32, _P, _P, _P, _P, _P, _U64, _P], ctypes.c_int),
    "sh_multi_graph": ([_P, _P, _U32, _P, _P, _P, _P, _P, _U64, _P], ctypes.c_int),
    "sh_multi_mixed_each": ([_P, _P, _U32, _P, _P, _P, _P, _P, _U64, _P], ctypes.c_int),
    "sh_server_scratch_bytes": ([_P], _SZ),
    "sh_server_start": ([_P, _P, _P, _P, _P, _P, _P, _U64, _P, _SZ, _P, _P], ctypes.c_int),
    "sh_server_submit": ([_P, _P, _P], ctypes.c_int),
    "sh_server_poll": ([_P, _U64, _P, _P, _P], ctypes.c_int),
    "sh_server_replay": ([_P, _P, _P, _U64, _P, _P], ctypes.c_int),
    "sh_server_stop": ([_P], ctypes.c_int),
    "sh_clock_ns": ([], _U64),
    "sh_capture_begin": ([_P], ctypes.c_int),
    "sh_capture_end": ([_P, _P], ctypes.c_int),
    "sh_graph_launch": ([_P, _P], ctypes.c_int),
    "sh_graph_destroy": ([_P], ctypes.c_int),
    "sh_multi_destroy": ([_P], ctypes.c_int),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libslabhash.so (built by paper_1710_11246_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libslabhash.so is not built (%s); run "
                               "`python -m paper_1710_11246_amd.build` or __graft_entry__.build()"
                               % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def declared_symbols() -> list[str]:
    """Entry points declared in include/slabhash.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(sh_\w+)\s*\(", text, re.M)))


def _check(fn: str, code: int) -> None:
    if code != SH_OK:
        raise SlabHashError(fn, code)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


_U32_TYPES = (torch.int32,) + ((torch.uint32,) if hasattr(torch, "uint32") else ())


def _dev(t, name: str, dtypes, n: int | None = None, allow_none: bool = False):
    if t is None:
        if allow_none:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype not in dtypes:
        raise ValueError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n is not None and t.numel() < n:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), n))
    return t.data_ptr()


def sh_strerror(code: int) -> str:
    return lib().sh_strerror(int(code)).decode()


def sh_storage_bytes(params: ShParams) -> int:
    return int(lib().sh_storage_bytes(ctypes.byref(params)))


def sh_create(params: ShParams, storage: torch.Tensor, stream=None) -> ctypes.c_void_p:
    if not isinstance(storage, torch.Tensor) or not storage.is_cuda or \
            not storage.is_contiguous():
        raise ValueError("storage must be a contiguous CUDA tensor")
    out = ctypes.c_void_p()
    nbytes = storage.numel() * storage.element_size()
    _check("sh_create", lib().sh_create(ctypes.byref(params), storage.data_ptr(), nbytes,
                                        _stream(stream), ctypes.byref(out)))
    return out


def sh_reset(t, stream=None) -> None:
    _check("sh_reset", lib().sh_reset(t, _stream(stream)))


def sh_flush(t, first_bucket: int, num_buckets: int, stream=None) -> None:
    _check("sh_flush", lib().sh_flush(t, int(first_bucket), int(num_buckets), _stream(stream)))


def sh_super_block_bytes(slabs: int) -> int:
    return int(lib().sh_super_block_bytes(int(slabs)))


def sh_add_super_block(t, mem: torch.Tensor, stream=None) -> None:
    if not isinstance(mem, torch.Tensor) or not mem.is_cuda or not mem.is_contiguous():
        raise ValueError("mem must be a contiguous CUDA tensor")
    _check("sh_add_super_block", lib().sh_add_super_block(
        t, mem.data_ptr(), mem.numel() * mem.element_size(), _stream(stream)))


def sh_search_all(t, keys: torch.Tensor, counts: torch.Tensor, offsets=None, vals=None,
                  stream=None) -> None:
    n = keys.numel()
    k = _dev(keys, "keys", _U32_TYPES, n)
    c = _dev(counts, "counts", _U32_TYPES, n)
    o = _dev(offsets, "offsets", (torch.int64,), n, allow_none=True)
    v = _dev(vals, "vals", _U32_TYPES, None, allow_none=True)
    cap = vals.numel() if vals is not None else 0
    _check("sh_search_all", lib().sh_search_all(t, k, n, c, o, v, cap, _stream(stream)))


def sh_delete_all(t, keys: torch.Tensor, counts=None, stream=None) -> None:
    n = keys.numel()
    k = _dev(keys, "keys", _U32_TYPES, n)
    c = _dev(counts, "counts", _U32_TYPES, n, allow_none=True)
    _check("sh_delete_all", lib().sh_delete_all(t, k, n, c, _stream(stream)))


def sh_alloc_slabs(t, n: int, out: torch.Tensor, stream=None) -> None:
    o = _dev(out, "out", _U32_TYPES, n)
    _check("sh_alloc_slabs", lib().sh_alloc_slabs(t, int(n), o, _stream(stream)))


def sh_free_slabs(t, idx: torch.Tensor, stream=None) -> None:
    n = idx.numel()
    p = _dev(idx, "idx", _U32_TYPES, n)
    _check("sh_free_slabs", lib().sh_free_slabs(t, p, int(n), _stream(stream)))


def sh_destroy(t) -> None:
    _check("sh_destroy", lib().sh_destroy(t))


def sh_set_launch(t, waves_per_cu: int = 0, ops_per_wave: int = 0, flags: int = 0) -> None:
    shape = ShLaunch(int(waves_per_cu), int(ops_per_wave), int(flags))
    _check("sh_set_launch", lib().sh_set_launch(t, ctypes.byref(shape)))


def sh_launch_shape(t, kind: int, n: int) -> tuple[int, int]:
    """(waves per CU, ops per wavefront) that a call of n ops of `kind` would use now."""
    w, c = ctypes.c_uint32(), ctypes.c_uint32()
    _check("sh_launch_shape", lib().sh_launch_shape(t, int(kind), int(n), ctypes.byref(w),
                                                    ctypes.byref(c)))
    return int(w.value), int(c.value)


def sh_build(t, keys, vals, status=None, stream=None) -> None:
    """vals may be None for a key-only table (the library rejects it for key-value tables)."""
    n = keys.numel()
    _check("sh_build", lib().sh_build(
        t, _dev(keys, "keys", _U32_TYPES), _dev(vals, "vals", _U32_TYPES, n, True), n,
        _dev(status, "status", (torch.uint8,), n, True), _stream(stream)))


def sh_insert(t, keys, vals, status=None, stream=None) -> None:
    n = keys.numel()
    _check("sh_insert", lib().sh_insert(
        t, _dev(keys, "keys", _U32_TYPES), _dev(vals, "vals", _U32_TYPES, n, True), n,
        _dev(status, "status", (torch.uint8,), n, True), _stream(stream)))


def sh_delete(t, keys, status=None, stream=None) -> None:
    n = keys.numel()
    _check("sh_delete", lib().sh_delete(
        t, _dev(keys, "keys", _U32_TYPES), n, _dev(status, "status", (torch.uint8,), n, True),
        _stream(stream)))


def sh_search(t, keys, vals_out, found=None, stream=None) -> None:
    n = keys.numel()
    _check("sh_search", lib().sh_search(
        t, _dev(keys, "keys", _U32_TYPES), n, _dev(vals_out, "vals_out", _U32_TYPES, n),
        _dev(found, "found", (torch.uint8,), n, True), _stream(stream)))


def sh_mixed(t, ops, keys, vals_in, vals_out, status, stream=None) -> None:
    n = keys.numel()
    _check("sh_mixed", lib().sh_mixed(
        t, _dev(ops, "ops", (torch.uint8,), n), _dev(keys, "keys", _U32_TYPES),
        _dev(vals_in, "vals_in", _U32_TYPES, n, True), n,
        _dev(vals_out, "vals_out", _U32_TYPES, n),
        _dev(status, "status", (torch.uint8,), n), _stream(stream)))


def sh_stats(t, stream=None) -> dict:
    st = ShStats()
    _check("sh_stats", lib().sh_stats(t, ctypes.byref(st), _stream(stream)))
    return {name: int(getattr(st, name)) for name, _ in ShStats._fields_}


def sh_dump(t, bucket, key, val, bucket_counts, count, violations, stream=None) -> None:
    cap = 0 if key is None else key.numel()
    _check("sh_dump", lib().sh_dump(
        t, _dev(bucket, "bucket", _U32_TYPES, cap, True), _dev(key, "key", _U32_TYPES, cap, True),
        _dev(val, "val", _U32_TYPES, cap, True), cap,
        _dev(bucket_counts, "bucket_counts", _U32_TYPES, None, True),
        _dev(count, "count", (torch.int64,), 1), _dev(violations, "violations", _U32_TYPES, 1, True),
        _stream(stream)))


# ---------------------------------------------------------------------------------------------
# Batched form

def _params_array(params):
    arr = (ShParams * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def sh_multi_storage_bytes(params) -> int:
    return int(lib().sh_multi_storage_bytes(len(params), _params_array(params)))


def sh_multi_create(params, storage: torch.Tensor, stream=None) -> ctypes.c_void_p:
    if not isinstance(storage, torch.Tensor) or not storage.is_cuda or \
            not storage.is_contiguous():
        raise ValueError("storage must be a contiguous CUDA tensor")
    out = ctypes.c_void_p()
    nbytes = storage.numel() * storage.element_size()
    _check("sh_multi_create", lib().sh_multi_create(len(params), _params_array(params),
                                                    storage.data_ptr(), nbytes, _stream(stream),
                                                    ctypes.byref(out)))
    return out


def sh_multi_table(m, t: int) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    _check("sh_multi_table", lib().sh_multi_table(m, int(t), ctypes.byref(out)))
    return out


def sh_multi_set_launch(m, waves_per_cu: int = 0, ops_per_wave: int = 0, flags: int = 0):
    shape = ShLaunch(int(waves_per_cu), int(ops_per_wave), int(flags))
    _check("sh_multi_set_launch", lib().sh_multi_set_launch(m, ctypes.byref(shape)))


def _multi_args(desc, nb, ops, keys, vals_in, vals_out, status):
    n = keys.numel()
    if nb > SH_MAX_BATCHES:
        raise ValueError("at most %d batches per launch" % SH_MAX_BATCHES)
    return (_dev(desc, "desc", (torch.int64,), 2 * nb), nb, _dev(ops, "ops", (torch.uint8,), n),
            _dev(keys, "keys", _U32_TYPES), _dev(vals_in, "vals_in", _U32_TYPES, n),
            _dev(vals_out, "vals_out", _U32_TYPES, n), _dev(status, "status", (torch.uint8,), n))


def sh_multi_mixed(m, desc, nb, ops, keys, vals_in, vals_out, status, stream=None) -> None:
    """desc: int64 device tensor of 2*nb words (see pack_batch_descs); the op arrays' length
    is keys.numel()."""
    _check("sh_multi_mixed", lib().sh_multi_mixed(
        m, *_multi_args(desc, nb, ops, keys, vals_in, vals_out, status), keys.numel(),
        _stream(stream)))


def sh_multi_mixed_each(m, h_desc: np.ndarray, ops, keys, vals_in, vals_out, status,
                        stream=None) -> None:
    """The plain form: one sh_mixed launch per descriptor, issued from C. h_desc is the host
    int64 array from pack_batch_descs."""
    h = np.ascontiguousarray(h_desc, dtype=np.int64)
    nb = h.size // 2
    n = keys.numel()
    _check("sh_multi_mixed_each", lib().sh_multi_mixed_each(
        m, h.ctypes.data, nb, _dev(ops, "ops", (torch.uint8,), n), _dev(keys, "keys", _U32_TYPES),
        _dev(vals_in, "vals_in", _U32_TYPES, n), _dev(vals_out, "vals_out", _U32_TYPES, n),
        _dev(status, "status", (torch.uint8,), n), n, _stream(stream)))


def sh_multi_graph(m, desc, nb, ops, keys, vals_in, vals_out, status) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    _check("sh_multi_graph", lib().sh_multi_graph(
        m, *_multi_args(desc, nb, ops, keys, vals_in, vals_out, status), keys.numel(),
        ctypes.byref(out)))
    return out


def sh_capture_begin(stream) -> None:
    """Start capturing the work later calls enqueue on `stream` (a non-default stream)."""
    _check("sh_capture_begin", lib().sh_capture_begin(_stream(stream)))


def sh_capture_end(stream) -> ctypes.c_void_p:
    """Finish the capture on `stream`; returns the graph (replay with sh_graph_launch)."""
    out = ctypes.c_void_p()
    _check("sh_capture_end", lib().sh_capture_end(_stream(stream), ctypes.byref(out)))
    return out


def sh_graph_launch(g, stream=None) -> None:
    _check("sh_graph_launch", lib().sh_graph_launch(g, _stream(stream)))


def sh_graph_destroy(g) -> None:
    _check("sh_graph_destroy", lib().sh_graph_destroy(g))


def sh_multi_destroy(m) -> None:
    _check("sh_multi_destroy", lib().sh_multi_destroy(m))


# ---------------------------------------------------------------------------------------------
# Served form

def sh_server_scratch_bytes(cfg: ShServerCfg | None = None) -> int:
    return int(lib().sh_server_scratch_bytes(ctypes.byref(cfg) if cfg is not None else None))


def sh_server_start(t, cfg, ops, keys, vals_in, vals_out, status, scratch: torch.Tensor,
                    stream=None) -> ctypes.c_void_p:
    n = keys.numel()
    out = ctypes.c_void_p()
    _check("sh_server_start", lib().sh_server_start(
        t, ctypes.byref(cfg) if cfg is not None else None, _dev(ops, "ops", (torch.uint8,), n),
        _dev(keys, "keys", _U32_TYPES), _dev(vals_in, "vals_in", _U32_TYPES, n),
        _dev(vals_out, "vals_out", _U32_TYPES, n), _dev(status, "status", (torch.uint8,), n), n,
        _dev(scratch, "scratch", (torch.uint8,)), scratch.numel(), _stream(stream),
        ctypes.byref(out)))
    return out


def sh_server_submit(srv, offset: int, length: int, inserts: int):
    """Returns (status code, ticket): SH_OK, SH_EBUSY or SH_ENOMEM are returned, not raised."""
    req = ShRequest(int(offset), int(length), int(inserts))
    tk = ctypes.c_uint64()
    code = lib().sh_server_submit(srv, ctypes.byref(req), ctypes.byref(tk))
    if code not in (SH_OK, SH_EBUSY, SH_ENOMEM):
        raise SlabHashError("sh_server_submit", code)
    return code, int(tk.value)


def sh_server_poll(srv, ticket: int):
    """Returns (done, t_admit_ns, t_done_ns)."""
    d = ctypes.c_int()
    ta, td = ctypes.c_uint64(), ctypes.c_uint64()
    _check("sh_server_poll", lib().sh_server_poll(srv, int(ticket), ctypes.byref(d),
                                                  ctypes.byref(ta), ctypes.byref(td)))
    return bool(d.value), int(ta.value), int(td.value)


def sh_server_replay(srv, offsets, lengths, inserts, arrival_ns):
    """Submit request i (ops [offsets[i], offsets[i] + lengths[i])) at arrival_ns[i] after the
    call's start. Returns (admit_ns, done_ns) arrays relative to that start."""
    n = len(offsets)
    reqs = np.zeros(n, dtype=[("offset", "<u8"), ("length", "<u4"), ("inserts", "<u4")])
    reqs["offset"], reqs["length"], reqs["inserts"] = offsets, lengths, inserts
    arr = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
    adm = np.zeros(n, dtype=np.uint64)
    done = np.zeros(n, dtype=np.uint64)
    _check("sh_server_replay", lib().sh_server_replay(srv, reqs.ctypes.data, arr.ctypes.data, n,
                                                      adm.ctypes.data, done.ctypes.data))
    return adm, done


def sh_server_stop(srv) -> None:
    _check("sh_server_stop", lib().sh_server_stop(srv))


def sh_clock_ns() -> int:
    return int(lib().sh_clock_ns())


def pack_batch_descs(offsets, lengths, tables) -> np.ndarray:
    """sh_batch_desc_t records {uint64 offset; uint32 length; uint32 table} as int64 pairs."""
    off = np.asarray(offsets, dtype=np.uint64)
    ln = np.asarray(lengths, dtype=np.uint64)
    tb = np.asarray(tables, dtype=np.uint64)
    out = np.empty((off.size, 2), dtype=np.uint64)
    out[:, 0] = off
    out[:, 1] = ln | (tb << np.uint64(32))
    return out.reshape(-1).view(np.int64)


# ---------------------------------------------------------------------------------------------
# Conveniences for tests and the benchmark (still only marshalling).

def to_dev(a: np.ndarray, device="cuda") -> torch.Tensor:
    """uint32/uint8 numpy array -> device tensor (int32 bit pattern for uint32)."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(device)


def to_host_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def pool_slabs_bound(n_inserts: int, concurrency_slack_blocks: int = 4) -> int:
    """A pool size (multiple of 2048) that holds every slab n_inserts new keys can need: a
    bucket with c occupied slots uses ceil(c / 31) - 1 pool slabs <= c / 31, plus blocks of
    slack for slabs held briefly by wavefronts that lose a link race."""
    need = -(-int(n_inserts) // SH_SLAB_PAIRS)
    blocks = -(-need // SH_BLOCK_SLABS) + concurrency_slack_blocks
    return blocks * SH_BLOCK_SLABS


class SlabHash:
    """A table plus the torch tensor that holds its device storage (or, with `handle`, a view of
    a table owned by a MultiSlabHash)."""

    def __init__(self, num_buckets: int, pool_slabs: int, hash_a: int, hash_b: int,
                 device="cuda", stream=None, handle=None, owner=None, duplicates: bool = False,
                 keys_only: bool = False):
        self.params = ShParams(int(num_buckets), int(pool_slabs), int(hash_a), int(hash_b),
                               (SH_TABLE_DUPLICATES if duplicates else 0)
                               | (SH_TABLE_KEYS_ONLY if keys_only else 0))
        self.device = device
        self.owner = owner
        self.supers = []  # device memory of registered super blocks, in order
        if handle is not None:
            self.storage = None
            self.handle = handle
            return
        nbytes = sh_storage_bytes(self.params)
        if nbytes == 0:
            raise ValueError("invalid table parameters")
        self.storage = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.handle = sh_create(self.params, self.storage, stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and getattr(self, "owner", None) is None:
            try:
                sh_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def num_buckets(self) -> int:
        """Bucket count B."""
        return self.params.num_buckets

    def add_super_block(self, slabs: int, stream=None) -> torch.Tensor:
        """Register a further super block of `slabs` slabs (a multiple of 2048) in new device
        memory, which this object keeps; returns that memory."""
        nbytes = sh_super_block_bytes(slabs)
        if nbytes == 0:
            raise ValueError("slabs must be a positive multiple of 2048, at most 2^27 - 2048")
        mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        sh_add_super_block(self.handle, mem, stream)
        self.supers.append(mem)
        return mem

    def reset(self, stream=None):
        """Re-initialise the table in place: every slot and next index empty, every pool slab free
        (the storage ends byte for byte as a fresh table's)."""
        sh_reset(self.handle, stream)

    def set_launch(self, waves_per_cu: int = 0, ops_per_wave: int = 0, flags: int = 0):
        """Launch shape of later calls (0 = the operation kind's default); `flags` may hold
        SH_LAUNCH_COUNTERS to accumulate the operation counters `stats()` reports."""
        sh_set_launch(self.handle, waves_per_cu, ops_per_wave, flags)

    def launch_shape(self, kind: int, n: int) -> tuple[int, int]:
        """(waves per CU, ops per wavefront) a call of n ops of `kind` (an SH_OP_* code or
        SH_KIND_MIXED) would use now."""
        return sh_launch_shape(self.handle, kind, n)

    def search_all(self, keys, stream=None):
        """SEARCHALL of each key: (counts, offsets, values) as device tensors, query i's values
        (in list order) being values[offsets[i] : offsets[i] + counts[i]]. Two calls: counts,
        then the values into an output sized from them."""
        n = keys.numel()
        counts = torch.empty(n, dtype=torch.int32, device=keys.device)
        sh_search_all(self.handle, keys, counts, stream=stream)
        c64 = counts.to(torch.int64)
        offsets = torch.zeros(n, dtype=torch.int64, device=keys.device)
        if n > 1:
            offsets[1:] = torch.cumsum(c64[:-1], 0)
        total = int(c64.sum().item()) if n else 0
        vals = torch.empty(max(total, 1), dtype=torch.int32, device=keys.device)
        sh_search_all(self.handle, keys, counts, offsets, vals[:total] if total else vals[:1],
                      stream=stream)
        return counts, offsets, vals[:total]

    def delete_all(self, keys, stream=None):
        """DELETEALL of each key; the number of elements each removed (device tensor)."""
        counts = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
        sh_delete_all(self.handle, keys, counts, stream=stream)
        return counts

    def flush(self, first: int = 0, count: int | None = None, stream=None):
        """FLUSH of buckets [first, first + count) (every bucket from `first` by default)."""
        if count is None:
            count = self.num_buckets - first
        sh_flush(self.handle, first, count, stream)

    def insert(self, keys, vals=None, stream=None, status=True):
        """REPLACE each (key, value) pair (INSERT with duplicates; keys alone on a key-only
        table). Returns the per-op status tensor (1 new, 2 replaced, 0 failed), or None with
        status=False."""
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device) if status else None
        sh_insert(self.handle, keys, vals, st, stream)
        return st

    def build(self, keys, vals=None, stream=None, status=True):
        """Bulk build: the same operation as `insert`, named after the paper's bulk benchmark."""
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device) if status else None
        sh_build(self.handle, keys, vals, st, stream)
        return st

    def delete(self, keys, stream=None):
        """DELETE each key; returns the per-op status tensor (1 deleted, 0 absent)."""
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        sh_delete(self.handle, keys, st, stream)
        return st

    def search(self, keys, stream=None):
        """SEARCH each key; returns (values, found) device tensors (value 0xFFFFFFFF when
        absent; `found` is authoritative)."""
        v = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
        f = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        sh_search(self.handle, keys, v, f, stream)
        return v, f

    def mixed(self, ops, keys, vals, stream=None):
        """One concurrent batch of SH_OP_SEARCH / SH_OP_INSERT / SH_OP_DELETE ops (uint8);
        returns (values, status) device tensors. The outcome is linearizable."""
        vo = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        sh_mixed(self.handle, ops, keys, vals, vo, st, stream)
        return vo, st

    def stats(self, stream=None) -> dict:
        """Walk the table: live and deleted counts, slabs, pool use, error word, invariant
        violations, hash constants and the operation counters, as a dict. Synchronises."""
        return sh_stats(self.handle, stream)

    def dump(self, stream=None):
        """Returns numpy (bucket, key, value) sorted by (bucket, key, value), per-bucket counts
        [B, 3] (live, deleted, slabs), and the violation count."""
        dev = self.device
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        viol = torch.zeros(1, dtype=torch.int32, device=dev)
        counts = torch.empty(3 * self.num_buckets, dtype=torch.int32, device=dev)
        sh_dump(self.handle, None, None, None, counts, count, viol, stream)
        n = int(count.item())
        b = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        k = torch.empty_like(b)
        v = torch.empty_like(b)
        sh_dump(self.handle, b, k, v, counts, count, viol, stream)
        torch.cuda.synchronize()
        b, k, v = to_host_u32(b)[:n], to_host_u32(k)[:n], to_host_u32(v)[:n]
        order = np.lexsort((v, k, b))
        return (b[order], k[order], v[order], to_host_u32(counts).reshape(-1, 3),
                int(viol.item()))


class MultiSlabHash:
    """T tables in one device allocation, driven by one launch per round of batches."""

    def __init__(self, params, device="cuda", stream=None):
        self.params = list(params)
        nbytes = sh_multi_storage_bytes(self.params)
        if nbytes == 0:
            raise ValueError("invalid multi-table parameters")
        self.storage = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.handle = sh_multi_create(self.params, self.storage, stream)
        self.device = device
        self.tables = [SlabHash(p.num_buckets, p.pool_slabs, p.hash_a, p.hash_b, device,
                                handle=sh_multi_table(self.handle, t), owner=self)
                       for t, p in enumerate(self.params)]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                sh_multi_destroy(h)
            except Exception:
                pass
            self.handle = None

    def set_launch(self, waves_per_cu: int = 0, ops_per_wave: int = 0, flags: int = 0):
        """Launch shape of later batched launches (same fields as SlabHash.set_launch)."""
        sh_multi_set_launch(self.handle, waves_per_cu, ops_per_wave, flags)

    def mixed(self, desc, nb, ops, keys, vals, stream=None):
        """One launch over `nb` batches: `desc` holds sh_batch_desc_t records (offset, length,
        table) into the shared op arrays. Returns (values, status) device tensors."""
        vo = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        sh_multi_mixed(self.handle, desc, nb, ops, keys, vals, vo, st, stream)
        return vo, st


class Server:
    """A running server on `table` over device op arrays; stop() (or leaving a with-block)
    finishes all admitted work."""

    def __init__(self, table: SlabHash, ops, keys, vals, max_launches=0, max_batch_ops=0,
                 max_requests=0, reserve_slabs=0, stream=None):
        self.cfg = ShServerCfg(int(max_launches), int(max_batch_ops), int(max_requests), 0,
                               int(reserve_slabs))
        self.table = table
        self.ops, self.keys, self.vals = ops, keys, vals
        self.vals_out = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
        self.status = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        nbytes = sh_server_scratch_bytes(self.cfg)
        if nbytes == 0:
            raise ValueError("invalid server configuration")
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=keys.device)
        torch.cuda.synchronize()
        self.handle = sh_server_start(table.handle, self.cfg, ops, keys, vals, self.vals_out,
                                      self.status, self.scratch, stream)

    def submit(self, offset, length, inserts):
        """Offer the request for ops [offset, offset + length) with `inserts` inserts among
        them. Returns (code, ticket): SH_OK with the ticket, SH_EBUSY when it must wait, SH_ENOMEM
        when it can never fit; other codes raise SlabHashError."""
        return sh_server_submit(self.handle, offset, length, inserts)

    def poll(self, ticket):
        """(done, admit time, done time) of a ticket, in sh_clock_ns nanoseconds."""
        return sh_server_poll(self.handle, ticket)

    def replay(self, offsets, lengths, inserts, arrival_ns):
        """Submit request i (offsets[i], lengths[i], inserts[i]) at arrival_ns[i] after the
        call's start and wait for all; returns (admit_ns, done_ns) arrays relative to that start."""
        return sh_server_replay(self.handle, offsets, lengths, inserts, arrival_ns)

    def stop(self):
        """Finish admitted work, stop the server thread and free its host resources."""
        if self.handle is not None:
            h, self.handle = self.handle, None
            sh_server_stop(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
