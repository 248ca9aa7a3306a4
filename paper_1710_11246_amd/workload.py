"""Seeded synthetic inputs for the slab hash: keys, values, queries, op batches, request streams.

This module holds none of the hash table's own arithmetic (no bucket hash, no slab or allocator
logic). It only draws random numbers, so the CPU oracle tests and the GPU path can share it.

Randomness is SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), used as a counter-based generator: output i (1-based) of a stream with seed s is
mix(s + i * 0x9E3779B97F4A7C15 mod 2^64). The paper evaluates on uniformly random keys only
(Performance Evaluation, bulk and concurrent benchmarks), so these inputs are the workload itself.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

#: The one reserved 32-bit key (the empty sentinel); never drawn as a key.
RESERVED_KEY = 0xFFFFFFFF

OP_SEARCH, OP_INSERT, OP_DELETE = 0, 1, 2


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Counter-based SplitMix64 stream; `next(n)` returns the next n uint64 outputs."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.count = 0

    def next(self, n: int) -> np.ndarray:
        out = np.empty(n, dtype=np.uint64)
        step = 1 << 22  # chunks keep the temporaries in cache
        with np.errstate(over="ignore"):
            for a in range(0, n, step):
                b = min(n, a + step)
                idx = np.arange(self.count + 1 + a, self.count + 1 + b, dtype=np.uint64)
                out[a:b] = splitmix64_mix(self.seed + idx * GOLDEN)
        self.count += n
        return out

    def uniform(self, n: int) -> np.ndarray:
        """n doubles in [0, 1) from the top 53 bits."""
        return (self.next(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def below(self, n: int, bound: int) -> np.ndarray:
        """n integers in [0, bound) by Lemire's multiply-shift on the high 32 bits (bound < 2^32)."""
        assert 0 < bound <= 1 << 32
        hi = (self.next(n) >> np.uint64(32)).astype(np.uint64)
        with np.errstate(over="ignore"):
            return ((hi * np.uint64(bound)) >> np.uint64(32)).astype(np.int64)

    def permutation(self, n: int) -> np.ndarray:
        """A uniformly random permutation of range(n) (sort by 64-bit random tags)."""
        return np.argsort(self.next(n), kind="stable")


def value_of(keys: np.ndarray) -> np.ndarray:
    """Value stored with each key: low 32 bits of the SplitMix64 finaliser of the key."""
    return (splitmix64_mix(np.asarray(keys, dtype=np.uint64)) & np.uint64(0xFFFFFFFF)).astype(
        np.uint32)


def unique_keys(rng: SplitMix64, n: int, exclude: np.ndarray | None = None) -> np.ndarray:
    """n distinct uint32 keys in [0, 2^32-2] in stream order (high 32 bits of each output),
    skipping the reserved key, repeats, and anything in `exclude`."""
    out = np.empty(0, dtype=np.uint32)
    excl = np.unique(np.asarray(exclude, dtype=np.uint32)) if exclude is not None else None
    while out.size < n:
        need = n - out.size
        cand = (rng.next(need + need // 16 + 64) >> np.uint64(32)).astype(np.uint32)
        cand = cand[cand != np.uint32(RESERVED_KEY)]
        if excl is not None and excl.size:
            cand = cand[~np.isin(cand, excl, assume_unique=False)]
        allc = np.concatenate([out, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        out = allc[first]
    return out[:n].copy()


def _fmix32(h: np.ndarray) -> np.ndarray:
    """MurmurHash3's 32-bit finaliser (Appleby), a bijection of the 32-bit integers."""
    h = h ^ (h >> np.uint32(16))
    h = h * np.uint32(0x85EBCA6B)
    h = h ^ (h >> np.uint32(13))
    h = h * np.uint32(0xC2B2AE35)
    return h ^ (h >> np.uint32(16))


def _perm32(seed: int, x: np.ndarray) -> np.ndarray:
    s = splitmix64_mix(np.array([seed], dtype=np.uint64))[0]
    s1, s2 = np.uint32(int(s) & 0xFFFFFFFF), np.uint32(int(s) >> 32)
    with np.errstate(over="ignore"):
        return _fmix32(_fmix32(x ^ s1) ^ s2)


def distinct_keys(seed: int, start: int, n: int) -> np.ndarray:
    """n distinct keys: a seeded bijection of the 32-bit integers applied to the counters
    start, start + 1, ..., so calls with non-overlapping counter ranges (and the same seed)
    give disjoint key sets; no sorting is needed. The reserved key is replaced by the image of
    counter 2^32 - 1, which no range below it uses."""
    assert 0 <= start and start + n < 0xFFFFFFFF
    x = np.arange(start, start + n, dtype=np.uint64).astype(np.uint32)
    k = _perm32(seed, x)
    bad = k == np.uint32(RESERVED_KEY)
    if bad.any():
        k[bad] = _perm32(seed, np.array([0xFFFFFFFF], dtype=np.uint32))[0]
    return k


def log_uniform_ints(rng: SplitMix64, n: int, lo: int, hi: int) -> np.ndarray:
    """n integers, log-uniform on [lo, hi]: floor(exp(ln lo + U (ln(hi+1) - ln lo)))."""
    u = rng.uniform(n)
    v = np.floor(np.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))).astype(np.int64)
    return np.clip(v, lo, hi)


def hash_params(rng: SplitMix64, prime: int) -> tuple[int, int]:
    """The random multipliers of a universal hash modulo `prime`: a in [1, prime-1], b in
    [0, prime-1]. The prime itself is a parameter of the table, not drawn here."""
    r = rng.next(2)
    a = 1 + int(r[0]) % (prime - 1)
    b = int(r[1]) % prime
    return a, b


def zipf_ranks(rng: SplitMix64, n: int, num: int, s: float) -> np.ndarray:
    """n ranks in [1, num] with P(r) proportional to r^-s (s > 1), by rejection-inversion
    (Hormann & Derflinger, ACM TOMACS 1996)."""
    assert s > 1.0 and num >= 1

    def H(x):  # integral of (x)^-s
        return (np.power(x, 1.0 - s) - 1.0) / (1.0 - s)

    def Hinv(y):
        return np.power(1.0 + y * (1.0 - s), 1.0 / (1.0 - s))

    h_x1 = H(1.5) - 1.0
    h_n = H(num + 0.5)
    sconst = 2.0 - Hinv(H(2.5) - math.pow(2.0, -s))
    out = np.empty(n, dtype=np.int64)
    filled = 0
    while filled < n:
        m = (n - filled) + (n - filled) // 8 + 64  # acceptance is above 0.9 for s > 1
        u = h_n + rng.uniform(m) * (h_x1 - h_n)
        x = Hinv(u)
        k = np.clip(np.floor(x + 0.5), 1, num)
        acc = (k - x <= sconst) | (u >= H(k + 0.5) - np.power(k, -s))
        got = k[acc].astype(np.int64)
        take = min(got.size, n - filled)
        out[filled:filled + take] = got[:take]
        filled += take
    return out


# --------------------------------------------------------------------------------------------
# Workloads. Each returns plain numpy arrays; the table geometry (bucket count, pool size) is
# chosen by the caller.

@dataclass
class Workload:
    name: str
    seed: int
    hash_a: int = 0
    hash_b: int = 0
    arrays: dict = field(default_factory=dict)

    def __getitem__(self, k):
        return self.arrays[k]

    def checksum(self) -> int:
        h = np.uint64(self.seed)
        for name in sorted(self.arrays):
            a = np.ascontiguousarray(self.arrays[name]).view(np.uint8).astype(np.uint64)
            with np.errstate(over="ignore"):
                h = splitmix64_mix(np.array([h ^ np.uint64(int(a.sum()) & 0xFFFFFFFFFFFFFFFF)
                                             ^ np.uint64(a.size)]))[0]
        return int(h)


def phased(seed: int, n: int, n_queries: int, hit_fraction: float, delete_fraction: float,
           prime: int) -> Workload:
    """Build n unique keys (value = value_of(key)); queries with the given hit fraction,
    shuffled; and a random subset of the keys to delete."""
    rng = SplitMix64(seed)
    a, b = hash_params(rng, prime)
    keys = unique_keys(rng, n)
    vals = value_of(keys)
    n_hit = int(round(n_queries * hit_fraction))
    hit = keys[rng.permutation(n)[:n_hit]] if n_hit else np.empty(0, np.uint32)
    miss = unique_keys(rng, n_queries - n_hit, exclude=keys)
    q = np.concatenate([hit, miss])
    q = q[rng.permutation(q.size)]
    n_del = int(round(n * delete_fraction))
    dels = keys[rng.permutation(n)[:n_del]]
    return Workload("phased", seed, a, b, dict(keys=keys, vals=vals, queries=q, deletes=dels,
                                               miss=miss, hit=hit))


def bulk(seed: int, n: int, prime: int) -> Workload:
    """n unique keys/values; an all-hit query set (a random permutation of the keys) and an
    all-miss set (n fresh keys)."""
    rng = SplitMix64(seed)
    a, b = hash_params(rng, prime)
    keys = unique_keys(rng, n)
    vals = value_of(keys)
    q_hit = keys[rng.permutation(n)]
    q_miss = unique_keys(rng, n, exclude=keys)
    return Workload("bulk", seed, a, b, dict(keys=keys, vals=vals, q_hit=q_hit, q_miss=q_miss))


def mixed_batch(rng: SplitMix64, present: np.ndarray, fresh: np.ndarray, absent: np.ndarray,
                n_ins: int, n_del: int, n_hit: int, n_miss: int):
    """One concurrent batch: n_ins inserts of `fresh` keys, n_del deletes of distinct present
    keys, n_hit searches of present keys, n_miss searches of `absent` keys, shuffled.
    Returns (ops uint8, keys uint32, vals uint32)."""
    assert fresh.size >= n_ins and absent.size >= n_miss
    pi = rng.permutation(present.size)
    dels = present[pi[:n_del]]
    hits = present[rng.below(n_hit, present.size)] if n_hit else np.empty(0, np.uint32)
    miss = absent[rng.below(n_miss, absent.size)] if n_miss else np.empty(0, np.uint32)
    ins = fresh[:n_ins]
    keys = np.concatenate([ins, dels, hits, miss]).astype(np.uint32)
    ops = np.concatenate([np.full(n_ins, OP_INSERT), np.full(n_del, OP_DELETE),
                          np.full(n_hit + n_miss, OP_SEARCH)]).astype(np.uint8)
    perm = rng.permutation(keys.size)
    keys, ops = keys[perm], ops[perm]
    vals = value_of(keys)
    return ops, keys, vals


def gamma_counts(length: int, fractions) -> tuple[int, int, int, int]:
    """Split a batch length over (insert new, delete existing, search existing, search absent)
    as in the paper's operation distribution Gamma = (a, b, c, d)."""
    a, b, c, d = fractions
    n_ins = int(math.floor(a * length))
    n_del = int(math.floor(b * length))
    rest = length - n_ins - n_del
    if c + d > 0:
        n_hit = int(round(rest * c / (c + d)))
    else:
        n_hit = 0
    return n_ins, n_del, n_hit, rest - n_hit


#: The paper's three operation distributions of the concurrent benchmark ("Concurrent
#: benchmarks"): (insert new, delete existing, search existing, search absent).
GAMMAS = {"gamma0": (0.5, 0.5, 0.0, 0.0), "gamma1": (0.2, 0.2, 0.3, 0.3),
          "gamma2": (0.1, 0.1, 0.4, 0.4)}


@dataclass
class Growth:
    """Incremental growth with concurrent batches at checkpoints. The table receives `keys` in
    insert-only batches of `batch`; when it has received checkpoints[c] of them, the batches of
    mixed[c] run in order: a list of (gamma name, [(ops, keys, vals), ...])."""
    seed: int
    hash_a: int
    hash_b: int
    keys: np.ndarray
    vals: np.ndarray
    batch: int
    checkpoints: list
    mixed: list
    mixed_inserts: int


def growth_checkpoints(seed: int, total: int, batch: int, checkpoints, per_gamma: int,
                       length: int, prime: int, gammas=GAMMAS) -> Growth:
    """Keys for growth to `total` in batches of `batch`, and at each checkpoint `per_gamma`
    mixed batches of `length` ops for every operation distribution in `gammas`. A mixed batch
    inserts fresh keys, deletes distinct keys present at its start, searches present keys
    (uniformly, with repeats) and searches keys never inserted, shuffled. Keys come from
    `distinct_keys` ranges, so growth keys, fresh keys and absent keys are pairwise disjoint."""
    assert all(0 < c <= total for c in checkpoints) and list(checkpoints) == sorted(checkpoints)
    rng = SplitMix64(seed)
    a, b = hash_params(rng, prime)
    keys = distinct_keys(seed, 0, total)
    counts = {g: gamma_counts(length, f) for g, f in gammas.items()}
    n_fresh = len(checkpoints) * per_gamma * sum(c[0] for c in counts.values())
    n_absent = max(1, max(c[3] for c in counts.values()))
    fresh = distinct_keys(seed, total, n_fresh)
    absent = distinct_keys(seed, total + n_fresh, 4 * n_absent)
    present = np.empty(0, dtype=np.uint32)
    grown, fi, mixed = 0, 0, []
    for cp in checkpoints:
        present = np.concatenate([present, keys[grown:cp]])
        grown = cp
        per_cp = []
        for g in gammas:
            n_ins, n_del, n_hit, n_miss = counts[g]
            bl = []
            for _ in range(per_gamma):
                dpos = sample_distinct(rng, n_del, present.size)
                dels = present[dpos]
                hits = present[rng.below(n_hit, present.size)] if n_hit else present[:0]
                miss = absent[rng.below(n_miss, absent.size)] if n_miss else absent[:0]
                ins = fresh[fi:fi + n_ins]
                fi += n_ins
                k = np.concatenate([ins, dels, hits, miss]).astype(np.uint32)
                o = np.concatenate([np.full(n_ins, OP_INSERT), np.full(n_del, OP_DELETE),
                                    np.full(n_hit + n_miss, OP_SEARCH)]).astype(np.uint8)
                perm = rng.permutation(k.size)
                k, o = k[perm], o[perm]
                bl.append((o, k, value_of(k)))
                present = np.concatenate([np.delete(present, dpos), ins])
            per_cp.append((g, bl))
        mixed.append(per_cp)
    return Growth(seed, a, b, keys, value_of(keys), batch, list(checkpoints), mixed, fi)


def sample_distinct(rng: SplitMix64, k: int, n: int, ok: np.ndarray | None = None) -> np.ndarray:
    """k distinct indices in [0, n) (optionally only where ok[idx]), in draw order."""
    avail = n if ok is None else int(np.count_nonzero(ok[:n]))
    if k > avail:
        raise ValueError("cannot draw %d distinct indices from %d" % (k, avail))
    out = np.empty(0, dtype=np.int64)
    while out.size < k:
        need = k - out.size
        cand = rng.below(need + need // 4 + 16, n)
        if ok is not None:
            cand = cand[ok[cand]]
        allc = np.concatenate([out, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        out = allc[first]
    return out[:k]


@dataclass
class MultiRounds:
    """Batched workload: T tables, each bulk-built with n[t] keys, then `rounds` rounds in which
    every table receives one mixed batch. Round r's ops are concatenated table by table; batch
    (r, t) is ops [offsets[r][t], offsets[r][t] + lengths[r][t]) of the round's arrays."""
    seed: int
    hash_a: np.ndarray
    hash_b: np.ndarray
    init_keys: list
    init_vals: list
    ops: list
    keys: list
    vals: list
    offsets: list
    lengths: list
    final_occupancy: np.ndarray


def multi_rounds(seed: int, T: int, n_lo: int, n_hi: int, len_lo: int, len_hi: int,
                 rounds: int, fractions, prime: int) -> MultiRounds:
    """Tables with log-uniform sizes in [n_lo, n_hi] and per-round batch lengths log-uniform in
    [len_lo, len_hi]. fractions = (insert new, delete existing, search existing, search absent)
    of each batch (the paper's operation distribution). Keys are unique within a table; at
    most one mutation per key per batch; searches of existing keys and deletes draw from the
    keys live at the start of the round. A batch never deletes more keys than are live: the
    shortfall (and all existing-key searches of a table with no live key) become searches of
    absent keys, so every batch keeps its length."""
    rng = SplitMix64(seed)
    n = log_uniform_ints(rng, T, n_lo, n_hi)
    lens = log_uniform_ints(rng, rounds * T, len_lo, len_hi).reshape(rounds, T)
    counts = [[list(gamma_counts(int(lens[r, t]), fractions)) for t in range(T)]
              for r in range(rounds)]
    ha = np.empty(T, np.int64)
    hb = np.empty(T, np.int64)
    universe, alive, nxt, absent = [], [], [], []
    init_keys, init_vals = [], []
    for t in range(T):
        ha[t], hb[t] = hash_params(rng, prime)
        n_ins = sum(counts[r][t][0] for r in range(rounds))
        n_abs = max(counts[r][t][3] + counts[r][t][1] + counts[r][t][2]
                    for r in range(rounds)) + 1
        u = unique_keys(rng, int(n[t]) + n_ins + n_abs)
        universe.append(u[: int(n[t]) + n_ins])
        absent.append(u[int(n[t]) + n_ins:])
        a = np.zeros(int(n[t]) + n_ins, dtype=bool)
        a[: int(n[t])] = True
        alive.append(a)
        nxt.append(int(n[t]))
        init_keys.append(u[: int(n[t])])
        init_vals.append(value_of(u[: int(n[t])]))
    occ = n.astype(np.int64).copy()
    R_ops, R_keys, R_vals, R_off, R_len = [], [], [], [], []
    for r in range(rounds):
        parts_o, parts_k, offs, lns = [], [], [], []
        off = 0
        for t in range(T):
            n_ins, n_del, n_hit, n_miss = counts[r][t]
            live_idx_ok = alive[t].copy()
            n_live = int(np.count_nonzero(live_idx_ok[: nxt[t]]))
            if n_del > n_live:
                n_miss += n_del - n_live
                n_del = n_live
            if n_live == 0:
                n_miss += n_hit
                n_hit = 0
            dels = sample_distinct(rng, n_del, nxt[t], live_idx_ok[: nxt[t]]) if n_del else \
                np.empty(0, np.int64)
            hits = np.empty(0, np.int64)
            if n_hit:
                hits = rng.below(n_hit * 2 + 16, nxt[t])
                hits = hits[live_idx_ok[hits]][:n_hit]
                while hits.size < n_hit:
                    h2 = rng.below(n_hit, nxt[t])
                    hits = np.concatenate([hits, h2[live_idx_ok[h2]]])[:n_hit]
            ins = universe[t][nxt[t]: nxt[t] + n_ins]
            miss = absent[t][rng.below(n_miss, absent[t].size)] if n_miss else \
                np.empty(0, np.uint32)
            k = np.concatenate([ins, universe[t][dels], universe[t][hits], miss]).astype(np.uint32)
            o = np.concatenate([np.full(n_ins, OP_INSERT), np.full(n_del, OP_DELETE),
                                np.full(n_hit + n_miss, OP_SEARCH)]).astype(np.uint8)
            perm = rng.permutation(k.size)
            parts_k.append(k[perm])
            parts_o.append(o[perm])
            offs.append(off)
            lns.append(k.size)
            off += k.size
            alive[t][dels] = False
            alive[t][nxt[t]: nxt[t] + n_ins] = True
            nxt[t] += n_ins
            occ[t] += n_ins
        keys = np.concatenate(parts_k)
        R_keys.append(keys)
        R_ops.append(np.concatenate(parts_o))
        R_vals.append(value_of(keys) ^ np.uint32(r + 1))
        R_off.append(np.asarray(offs, dtype=np.int64))
        R_len.append(np.asarray(lns, dtype=np.int64))
    return MultiRounds(seed, ha, hb, init_keys, init_vals, R_ops, R_keys, R_vals, R_off, R_len, occ)


@dataclass
class ServedRequests:
    """Requests for a served table: request i is ops [offsets[i], offsets[i] + lengths[i]) of
    the concatenated arrays; inserts[i] counts its insert ops."""
    ops: np.ndarray
    keys: np.ndarray
    vals: np.ndarray
    offsets: np.ndarray
    lengths: np.ndarray
    inserts: np.ndarray
    mut_keys: np.ndarray = None  # keys some request mutates (each exactly once)
    mut_req: np.ndarray = None   # the request mutating mut_keys[i]

    def mutator_of(self, keys: np.ndarray) -> np.ndarray:
        """For each key, the index of the request that mutates it, or -1 if none does."""
        keys = np.asarray(keys, dtype=np.uint32)
        out = np.full(keys.shape, -1, dtype=np.int64)
        if self.mut_keys is None or self.mut_keys.size == 0:
            return out
        order = np.argsort(self.mut_keys, kind="stable")
        sk = self.mut_keys[order]
        pos = np.minimum(np.searchsorted(sk, keys), sk.size - 1)
        hit = sk[pos] == keys
        out[hit] = self.mut_req[order][pos[hit]]
        return out


def served_requests(seed: int, initial: np.ndarray, n_req: int, len_lo: int, len_hi: int,
                    fractions=(0.10, 0.05, 0.85), zipf_s: float | None = 1.1,
                    disjoint: bool = False, absent_frac: float = 0.0,
                    shuffle_ranking: bool = True,
                    fresh_keys: np.ndarray | None = None) -> ServedRequests:
    """n_req requests with lengths log-uniform in [len_lo, len_hi] and i.i.d. op kinds with
    probabilities fractions = (insert, delete, search). Inserts use fresh keys (each once over
    all requests); deletes use distinct initial keys (each at most once over all requests);
    searches draw initial keys, Zipf(zipf_s) over a seeded ranking (uniform if zipf_s is None),
    plus a fraction `absent_frac` of never-inserted keys. With `disjoint`, request i only
    touches initial keys of its own slice of the initial set (no key is shared between
    requests). Without `shuffle_ranking` the initial keys' own order (their random draw order)
    serves as the Zipf ranking, which saves a sort for very large tables. `fresh_keys`, if
    given, supplies keys known to be absent from `initial` (inserts, then absent searches)."""
    rng = SplitMix64(seed)
    initial = np.asarray(initial, dtype=np.uint32)
    lens = log_uniform_ints(rng, n_req, len_lo, len_hi)
    total = int(lens.sum())
    u = rng.uniform(total)
    kind = np.where(u < fractions[0], OP_INSERT,
                    np.where(u < fractions[0] + fractions[1], OP_DELETE, OP_SEARCH)).astype(
        np.uint8)
    n_ins = int((kind == OP_INSERT).sum())
    n_srch = int((kind == OP_SEARCH).sum())
    n_fresh = n_ins + (n_srch + 16 if absent_frac > 0 else 0)
    if fresh_keys is not None:
        assert fresh_keys.size >= n_fresh
        fresh = np.asarray(fresh_keys[:n_fresh], dtype=np.uint32)
    else:
        fresh = unique_keys(rng, n_fresh, exclude=initial)
    keys = np.empty(total, dtype=np.uint32)
    keys[kind == OP_INSERT] = fresh[:n_ins]
    absent = fresh[n_ins:]
    offsets = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    rank_key = initial[rng.permutation(initial.size)] if shuffle_ranking else initial
    if disjoint:
        per = initial.size // n_req
        assert per >= 1, "not enough initial keys for disjoint requests"
        for i in range(n_req):
            a, n = int(offsets[i]), int(lens[i])
            own = rank_key[i * per:(i + 1) * per]
            k = kind[a:a + n]
            d = np.flatnonzero(k == OP_DELETE)
            if d.size > own.size:          # not enough own keys to delete: search instead
                kind[a + d[own.size:]] = OP_SEARCH
                d = d[:own.size]
            dk = own[sample_distinct(rng, d.size, own.size)] if d.size else own[:0]
            keys[a + d] = dk
            s_idx = np.flatnonzero(kind[a:a + n] == OP_SEARCH)
            keys[a + s_idx] = own[rng.below(s_idx.size, own.size)] if s_idx.size else keys[:0]
    else:
        d = np.flatnonzero(kind == OP_DELETE)
        if d.size > initial.size:
            kind[d[initial.size:]] = OP_SEARCH
            d = d[:initial.size]
        keys[d] = rank_key[sample_distinct(rng, d.size, initial.size)]
        s_idx = np.flatnonzero(kind == OP_SEARCH)
        if zipf_s is None:
            keys[s_idx] = rank_key[rng.below(s_idx.size, rank_key.size)]
        else:
            keys[s_idx] = rank_key[zipf_ranks(rng, s_idx.size, rank_key.size, zipf_s) - 1]
    if absent_frac > 0:
        s_idx = np.flatnonzero(kind == OP_SEARCH)
        pick = s_idx[rng.uniform(s_idx.size) < absent_frac]
        keys[pick] = absent[rng.below(pick.size, absent.size)] if pick.size else keys[:0]
    vals = value_of(keys) ^ np.uint32(0x9E3779B9)
    ins_per = np.add.reduceat((kind == OP_INSERT).astype(np.int64), offsets) if total else \
        np.zeros(n_req, np.int64)
    mut = np.flatnonzero(kind != OP_SEARCH)
    req_of = np.searchsorted(offsets, mut, side="right") - 1
    return ServedRequests(kind, keys, vals, offsets, lens.astype(np.int64), ins_per, keys[mut],
                          req_of)


def poisson_arrivals(rng: SplitMix64, n: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (ns, from 0) of a Poisson process with the given rate."""
    gaps = -np.log1p(-rng.uniform(n)) / rate_per_s
    return np.round(np.cumsum(gaps) * 1e9).astype(np.uint64)
