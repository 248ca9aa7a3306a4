"""CPU oracle for the slab hash -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, the package smoke check (`__graft_entry__.smoke`) and the benchmark's
`cpu_baseline` leg may import this package. The product path never does: it shares no code with
this oracle, and it fails loudly when its own GPU library is missing.

`slab_oracle.c` is a sequential chained hash map with the paper's operation semantics (see its
header for the passages it follows); this module is a ctypes wrapper over it taking numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slab_oracle.c")
LIB_PATH = os.path.join(_HERE, "_build", "libslab_oracle.so")

#: The prime of the universal hash (largest prime below 2^32); the oracle's own copy.
PRIME = 4294967291
RESERVED = 0xFFFFFFFF
ERR_RESERVED = 1
ERR_NOMEM = 2
UNBOUNDED = 0xFFFFFFFFFFFFFFFF


def build(force: bool = False) -> str:
    """Compile slab_oracle.c with gcc into oracle/_build/ (always when force)."""
    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall",
                               "-Werror", _SRC, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P, U32, U64, D = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        sig = {
            "om_create": ([U32, U32, U64, U64, U64], P),
            "om_destroy": ([P], None),
            "om_error": ([P], U32),
            "om_bucket_of": ([P, U32], U32),
            "om_bucket_of_batch": ([P, P, U64, P], None),
            "om_replace": ([P, U32, U32], ctypes.c_int),
            "om_delete": ([P, U32], ctypes.c_int),
            "om_replace_batch": ([P, P, P, U64, P], None),
            "om_delete_batch": ([P, P, U64, P], None),
            "om_search_batch": ([P, P, U64, P, P, P], None),
            "om_mixed_batch": ([P, P, P, P, U64, P, P], None),
            "om_bucket_stats": ([P, P, P, P], U64),
            "om_total_slabs": ([P], U64),
            "om_pool_used": ([P], U64),
            "om_utilisation": ([P, D, D], D),
            "om_dump": ([P, P, P, P, U64], U64),
            "om_flush_all": ([P], None),
            "om_flush_buckets": ([P, U32, U32], None),
            "om_set_duplicates": ([P, U32], None),
            "om_delete_all_batch": ([P, P, U64, P], None),
            "om_search_all_batch": ([P, P, U64, P, P, P], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


class Oracle:
    """Sequential slab-hash map: B buckets, M elements per slab, hash multipliers (a, b)."""

    def __init__(self, num_buckets: int, slab_elems: int, hash_a: int, hash_b: int,
                 pool_slabs: int | None = None, duplicates: bool = False):
        self._l = _load()
        self.B, self.M = int(num_buckets), int(slab_elems)
        self.a, self.b = int(hash_a), int(hash_b)
        cap = UNBOUNDED if pool_slabs is None else int(pool_slabs)
        self._t = self._l.om_create(self.B, self.M, self.a, self.b, cap)
        if not self._t:
            raise ValueError("invalid oracle parameters")
        self.duplicates = bool(duplicates)
        self._l.om_set_duplicates(self._t, int(self.duplicates))

    def __del__(self):
        t = getattr(self, "_t", None)
        if t:
            self._l.om_destroy(t)
            self._t = None

    @property
    def error(self) -> int:
        return int(self._l.om_error(self._t))

    def bucket_of(self, keys) -> np.ndarray:
        k = _u32(keys)
        out = np.empty(k.size, np.uint32)
        self._l.om_bucket_of_batch(self._t, _ptr(k), k.size, _ptr(out))
        return out

    def replace(self, keys, vals) -> np.ndarray:
        k, v = _u32(keys), _u32(vals)
        assert k.size == v.size
        st = np.empty(k.size, np.uint8)
        self._l.om_replace_batch(self._t, _ptr(k), _ptr(v), k.size, _ptr(st))
        return st

    def delete(self, keys) -> np.ndarray:
        k = _u32(keys)
        st = np.empty(k.size, np.uint8)
        self._l.om_delete_batch(self._t, _ptr(k), k.size, _ptr(st))
        return st

    def search(self, keys):
        """Returns (values, found, slabs_visited)."""
        k = _u32(keys)
        v = np.empty(k.size, np.uint32)
        f = np.empty(k.size, np.uint8)
        s = np.empty(k.size, np.uint32)
        self._l.om_search_batch(self._t, _ptr(k), k.size, _ptr(v), _ptr(f), _ptr(s))
        return v, f, s

    def mixed(self, ops, keys, vals):
        """Apply ops (0 search, 1 replace, 2 delete) in array order. Returns (vals_out, status)."""
        o = np.ascontiguousarray(ops, dtype=np.uint8)
        k, v = _u32(keys), _u32(vals)
        vo = np.empty(k.size, np.uint32)
        st = np.empty(k.size, np.uint8)
        self._l.om_mixed_batch(self._t, _ptr(o), _ptr(k), _ptr(v), k.size, _ptr(vo), _ptr(st))
        return vo, st

    def bucket_stats(self):
        """Per-bucket (live, deleted, slabs) arrays."""
        live = np.empty(self.B, np.uint32)
        tomb = np.empty(self.B, np.uint32)
        slabs = np.empty(self.B, np.uint32)
        self._l.om_bucket_stats(self._t, _ptr(live), _ptr(tomb), _ptr(slabs))
        return live, tomb, slabs

    @property
    def total_slabs(self) -> int:
        return int(self._l.om_total_slabs(self._t))

    @property
    def pool_used(self) -> int:
        return int(self._l.om_pool_used(self._t))

    def utilisation(self, elem_bytes: float, overhead_bytes: float) -> float:
        return float(self._l.om_utilisation(self._t, elem_bytes, overhead_bytes))

    def dump(self):
        """Live (bucket, key, value) triples, bucket-major, insertion order within a bucket."""
        n = int(self._l.om_dump(self._t, None, None, None, 0))
        b = np.empty(n, np.uint32)
        k = np.empty(n, np.uint32)
        v = np.empty(n, np.uint32)
        self._l.om_dump(self._t, _ptr(b), _ptr(k), _ptr(v), n)
        return b, k, v

    def delete_all(self, keys) -> np.ndarray:
        """DELETEALL of each key in order; the number of elements each removed."""
        k = _u32(keys)
        c = np.empty(k.size, np.uint32)
        self._l.om_delete_all_batch(self._t, _ptr(k), k.size, _ptr(c))
        return c

    def search_all(self, keys):
        """SEARCHALL of each key: (counts, offsets, values), query i's values (in list order)
        being values[offsets[i] : offsets[i] + counts[i]]."""
        k = _u32(keys)
        c = np.empty(k.size, np.uint32)
        self._l.om_search_all_batch(self._t, _ptr(k), k.size, _ptr(c), None, None)
        off = np.zeros(k.size, np.uint64)
        if k.size:
            off[1:] = np.cumsum(c[:-1], dtype=np.uint64)
        v = np.empty(max(1, int(c.sum(dtype=np.uint64))), np.uint32)
        self._l.om_search_all_batch(self._t, _ptr(k), k.size, _ptr(c), _ptr(off), _ptr(v))
        return c, off, v[: int(c.sum(dtype=np.uint64))]

    def flush_all(self) -> None:
        self._l.om_flush_all(self._t)

    def flush(self, first: int = 0, count: int | None = None) -> None:
        """FLUSH of buckets [first, first + count) (all from `first` if count is None)."""
        if count is None:
            count = max(0, self.B - first)
        self._l.om_flush_buckets(self._t, int(first), int(count))
