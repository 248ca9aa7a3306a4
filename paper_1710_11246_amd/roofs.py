"""ctypes binding of libslabhash_roofs.so (include/slabhash_roofs.h): microbenchmarks of the slab
hash's memory access patterns, used to measure the ceilings its kernels run against. Argument
marshalling only; every pattern runs in the library's kernels."""
from __future__ import annotations

import ctypes
import os
import re

import torch

from .slabhash import SH_OK, SlabHashError, _stream

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libslabhash_roofs.so")
HEADER_PATH = os.path.join(os.path.dirname(PKG), "include", "slabhash_roofs.h")

SH_ROOF_SLAB_LOAD, SH_ROOF_CAS, SH_ROOF_LOAD_CAS = 0, 1, 2

_SIGS = {
    "sh_roof_run": ([ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64,
                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p],
                    ctypes.c_int),
    "sh_roof_search": ([ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint64,
                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                        ctypes.c_void_p], ctypes.c_int),
    "sh_roof_insert": ([ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                        ctypes.c_void_p], ctypes.c_int),
}
_lib = None


def lib() -> ctypes.CDLL:
    """Load libslabhash_roofs.so (built by paper_1710_11246_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libslabhash_roofs.so is not built (%s); run "
                               "`python -m paper_1710_11246_amd.build`" % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def declared_symbols() -> list[str]:
    """Entry points declared in include/slabhash_roofs.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(sh_\w+)\s*\(", text, re.M)))


def sh_roof_run(kind: int, buf: torch.Tensor, n_ops: int, waves_per_cu: int = 0, seed: int = 1,
                stream=None, depth: int = 0) -> None:
    """Enqueue n_ops operations of pattern `kind` over the device tensor `buf` (its bytes,
    rounded down to whole 256-byte slabs)."""
    if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.is_contiguous()):
        raise ValueError("buf must be a contiguous device tensor")
    nbytes = (buf.numel() * buf.element_size()) // 256 * 256
    code = lib().sh_roof_run(int(kind), ctypes.c_void_p(buf.data_ptr()), nbytes, int(n_ops),
                             int(waves_per_cu), int(depth), int(seed) & 0xFFFFFFFF,
                             ctypes.c_void_p(_stream(stream)))
    if code != SH_OK:
        raise SlabHashError("sh_roof_run", code)


def sh_roof_search(buf: torch.Tensor, keys: torch.Tensor, vals: torch.Tensor, found: torch.Tensor,
                   waves_per_cu: int = 0, depth: int = 0, stream=None) -> None:
    """Enqueue keys.numel() one-slab searches over the device tensor `buf` (its bytes, rounded
    down to whole 256-byte slabs): vals (32-bit) and found (uint8) receive the results."""
    if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.is_contiguous()):
        raise ValueError("buf must be a contiguous device tensor")
    n = keys.numel()
    for name, x, dts in (("keys", keys, (torch.int32, torch.uint32)),
                         ("vals", vals, (torch.int32, torch.uint32)),
                         ("found", found, (torch.uint8,))):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.is_contiguous()
                and x.dtype in dts and x.numel() == n):
            raise ValueError("%s must be a contiguous device tensor of %d elements of %s"
                             % (name, n, dts))
    nbytes = (buf.numel() * buf.element_size()) // 256 * 256
    code = lib().sh_roof_search(ctypes.c_void_p(buf.data_ptr()), nbytes,
                                ctypes.c_void_p(keys.data_ptr()), n,
                                ctypes.c_void_p(vals.data_ptr()),
                                ctypes.c_void_p(found.data_ptr()), int(waves_per_cu), int(depth),
                                ctypes.c_void_p(_stream(stream)))
    if code != SH_OK:
        raise SlabHashError("sh_roof_search", code)


def sh_roof_insert(buf: torch.Tensor, keys: torch.Tensor, vals: torch.Tensor,
                   status: torch.Tensor, waves_per_cu: int = 0, depth: int = 0,
                   stream=None) -> None:
    """Enqueue keys.numel() one-slab inserts over the device tensor `buf` (its bytes, rounded
    down to whole 256-byte slabs): status (uint8) receives 1 where the op's swap won."""
    if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.is_contiguous()):
        raise ValueError("buf must be a contiguous device tensor")
    n = keys.numel()
    for name, x, dts in (("keys", keys, (torch.int32, torch.uint32)),
                         ("vals", vals, (torch.int32, torch.uint32)),
                         ("status", status, (torch.uint8,))):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.is_contiguous()
                and x.dtype in dts and x.numel() == n):
            raise ValueError("%s must be a contiguous device tensor of %d elements of %s"
                             % (name, n, dts))
    nbytes = (buf.numel() * buf.element_size()) // 256 * 256
    code = lib().sh_roof_insert(ctypes.c_void_p(buf.data_ptr()), nbytes,
                                ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                                n, ctypes.c_void_p(status.data_ptr()), int(waves_per_cu),
                                int(depth), ctypes.c_void_p(_stream(stream)))
    if code != SH_OK:
        raise SlabHashError("sh_roof_insert", code)
