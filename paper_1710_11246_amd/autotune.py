"""Table sizing and launch-shape tuning for the slab hash.

Sizing follows the paper's own rule for choosing the bucket count ("Bulk benchmarks": pick the
average slab count beta for a target memory utilisation, then B = n / (M beta)), evaluated
here with the exact Binomial distribution of bucket loads under a uniform hash: a bucket holding
X of n keys uses max(1, ceil(X / M)) slabs, and memory utilisation is
u = (x / (M x + y)) * n / sum_i k_i ("Slab Hash" subsection) with x = 8 bytes per pair and
y = 8 bytes of auxiliary word and next index per 256-byte slab.

Launch shapes (waves per CU, ops per wavefront) never change results; `tune_launch` times
candidate shapes on the device with a caller-supplied runner and keeps the fastest, cached in a
JSON file keyed by device name, operation kind and size class.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

SLAB_PAIRS = 31
SLAB_BYTES = 256
PAIR_BYTES = 8
BLOCK_SLABS = 2048


def _binom_pmf(n: int, B: int, xs: np.ndarray) -> np.ndarray:
    from scipy.stats import binom
    return binom.pmf(xs, n, 1.0 / B)


def slab_moments(n: int, B: int, M: int = SLAB_PAIRS):
    """E and Var of the slab count of one bucket when n keys hash uniformly over B buckets."""
    if B == 1:
        s = max(1, -(-n // M))
        return float(s), 0.0
    lam = n / B
    hi = int(lam + 12 * math.sqrt(lam) + 4 * M + 64)
    xs = np.arange(0, min(n, hi) + 1)
    pmf = _binom_pmf(n, B, xs)
    slabs = np.maximum(1, -(-xs // M))
    e = float((pmf * slabs).sum())
    v = float((pmf * slabs * slabs).sum()) - e * e
    return e, max(v, 0.0)


def utilisation(n: int, B: int, M: int = SLAB_PAIRS) -> float:
    """Expected memory utilisation of n keys in B buckets."""
    e, _ = slab_moments(n, B, M)
    return PAIR_BYTES * n / (SLAB_BYTES * B * e)


def buckets_for_utilisation(n: int, target: float, M: int = SLAB_PAIRS) -> int:
    """Largest bucket count whose expected utilisation reaches `target`.

    Utilisation rises as B falls while most buckets fit in one slab, peaks (about 0.71 for
    M = 31 near beta = 0.85), dips as second slabs appear, and rises again towards the 31/32
    limit. Targets up to the first peak are met on the first rise; higher ones further out."""
    if n <= 0:
        return 1
    lo_beta_B = max(1, int(n / (M * 0.85)))  # B at the first peak
    if utilisation(n, lo_beta_B, M) >= target:
        lo, hi = lo_beta_B, max(lo_beta_B, n)  # u(lo) >= target; search the largest such B
        if utilisation(n, hi, M) >= target:
            return hi
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if utilisation(n, mid, M) >= target:
                lo = mid
            else:
                hi = mid
        return lo
    # beyond the first peak: scan down geometrically, then bisect the last bracket
    B = lo_beta_B
    prev = B
    while B > 1 and utilisation(n, B, M) < target:
        prev = B
        B = max(1, int(B / 1.05))
    if utilisation(n, B, M) < target:
        return 1
    lo, hi = B, prev
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if utilisation(n, mid, M) >= target:
            lo = mid
        else:
            hi = mid
    return lo


def pool_slabs_for(n_occupied: int, B: int, M: int = SLAB_PAIRS, sigmas: float = 8.0,
                   slack_blocks: int = 4) -> int:
    """Pool size (a multiple of 2048 slabs) for n_occupied slots (live plus deleted) over B
    buckets: the expected number of overflow slabs plus `sigmas` standard deviations and
    `slack_blocks` blocks for slabs held briefly by wavefronts that lose a link race, never
    more than the hard bound ceil(n/M) that holds for any distribution."""
    e, v = slab_moments(n_occupied, B, M)
    expect = B * (e - 1.0) + sigmas * math.sqrt(B * v) + 1
    hard = -(-n_occupied // M)
    need = int(min(expect, hard))
    return (-(-need // BLOCK_SLABS) + slack_blocks) * BLOCK_SLABS


# ---------------------------------------------------------------------------------------------
# Launch shapes

DEFAULT_CANDIDATES = [(wpc, c) for wpc in (8, 16, 24, 32) for c in (16, 32, 64)]


def size_class(n_ops: int) -> str:
    return "2^%d" % max(0, int(round(math.log2(max(1, n_ops)))))


def _cache_path() -> str:
    return os.environ.get("SLABHASH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "slabhash_mi355x",
                                       "launch.json"))


def load_cache() -> dict:
    try:
        return json.load(open(_cache_path()))
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        json.dump(cache, open(tmp, "w"), indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune_launch(kind: str, n_ops: int, run, device_name: str = "", candidates=None,
                reps: int = 3, use_cache: bool = True):
    """Time run(waves_per_cu, ops_per_wave) -> seconds for each candidate (median of `reps`)
    and return (best_shape, timings). `run` must leave the device in the same state for every
    call (for example by resetting and rebuilding the tables it times)."""
    key = "%s|%s|%s" % (device_name, kind, size_class(n_ops))
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        return tuple(cache[key]["shape"]), cache[key].get("timings", {})
    timings = {}
    for shape in (candidates or DEFAULT_CANDIDATES):
        ts = sorted(run(*shape) for _ in range(reps))
        timings["%d,%d" % shape] = ts[len(ts) // 2]
    best = min(timings, key=timings.get)
    shape = tuple(int(x) for x in best.split(","))
    if use_cache:
        cache[key] = {"shape": list(shape), "timings": timings}
        save_cache(cache)
    return shape, timings
