#!/usr/bin/env python3
"""Slab-hash benchmark on one MI355X.

One step is one pass of the whole hot path over one batch of synthetic input:
  reset the table (initialise base slabs, pool and bitmaps),
  bulk build of 2^22 unique uniform uint32 key/value pairs (value = SplitMix64 finaliser of the
  key) into B buckets, 2^22 all-hit searches (a permutation of the keys), 2^22 all-miss searches
  (fresh keys), then 16 concurrent mixed batches of 2^16 ops with the paper's operation
  distribution Gamma1 = (0.2 insert new, 0.2 delete existing, 0.3 search existing, 0.3 search
  absent), shuffled.
value = all ops of a step / step time, in M ops/s. Per-kernel durations come from HIP events
on the launch stream inside the timed region; the roofline entry uses the algorithmic bytes of
the kernel that takes most of the step.

python bench.py [--steps K] [--warmup W] [--util 0.6] [--no-cpu-baseline] [--sweep]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_KEYS = 1 << 22
MIX_BATCH = 1 << 16
MIX_BATCHES = 16
GAMMA1 = (0.2, 0.2, 0.3, 0.3)
# Largest bucket counts whose Binomial-model utilisation reaches each target for n = 2^22 and
# 31 pairs per 256-byte slab (the same model the autotuner evaluates).
B_FOR_UTIL = {0.2: 654181, 0.3: 436670, 0.4: 327431, 0.5: 261962, 0.6: 217316, 0.7: 176200,
              0.8: 55174}


# Bytes per launch beyond L2 (reads + writes), from rocprofv3 FETCH_SIZE/WRITE_SIZE runs scaled by
# a 1 GiB device copy; see profiles/slabhash_step_2p22_traffic.md. Valid only for the kernel
# source they were measured on (sha256 prefix of csrc/slabhash.hip); otherwise reported as null.
TRAFFIC_SRC_SHA = "f87bfcd2f0d57c57"
# Per launch, from rocprofv3 TCC_HIT_sum/TCC_MISS_sum and TCC_ATOMIC_sum/TCC_EA0_ATOMIC_sum runs
# of the same source (profiles/slabhash_step_2p22_l2.md): (L2 hit rate, atomics, atomics that
# reached memory).
L2_STATS = {"build": (0.3684, 4693064, 4693064), "search_hit": (0.0938, 0, 0),
            "search_miss": (0.0938, 0, 0), "mixed": (0.3149, 26728, 26728),
            "reset": (0.5024, 0, 0)}
# The same for the 2^26-key table of measure_hbm_resident (profiles/slabhash_hbm_2p26_traffic.md).
HBM_TRAFFIC_BYTES = {"build": 22295350709, "search_hit": 17763213803,
                     "search_miss": 17763213803}
TRAFFIC_BYTES = {"build": 1349499276, "search_hit": 1039525491, "search_miss": 1039525491,
                 "mixed": 19521621, "reset": 56247443}


def source_sha() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_1710_11246_amd", "csrc", "slabhash.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def chain_visits(occ: np.ndarray, m: int = 31) -> float:
    """Total slabs read to reach every occupied slot once (slot p of a list sits in slab p//m)."""
    occ = occ.astype(np.int64)
    full, rem = occ // m, occ % m
    # slots in complete slabs: m * (1 + 2 + ... + full), the remainder sits in slab full + 1
    return float((m * full * (full + 1) // 2 + rem * (full + 1)).sum())


def op_bytes(kind: str, n: int, v_hit: float, v_miss: float, new_slabs: int = 0,
             mix=None) -> float:
    """Algorithmic bytes of one launch of n ops, with v_hit / v_miss the mean slabs a walk to a
    present key / to the end of a list reads (256 bytes each):
      search:  4 (key) + 256 v + 4 (value) + 1 (found);
      insert:  8 (pair) + 256 v_miss (the whole list is read to rule the key out) + 64 (the
               written sector of the swapped slot) + 1 (status), plus 8 per new slab (its
               bitmap word and the link), counted exactly when known;
      delete:  4 + 256 v_hit + 64 + 1;
      mixed:   per op 1 (op) + 4 (key) + 4 (value in) + 4 (value out) + 1 (status); slabs
               v_miss for inserts and absent searches, v_hit for deletes and present searches;
               64 per insert or delete; 8 / 31 per insert for new slabs (amortised).
    mix = (inserts, deletes, present searches, absent searches) of a mixed batch."""
    if kind == "search_hit":
        return n * (4 + 4 + 1) + 256.0 * v_hit * n
    if kind == "search_miss":
        return n * (4 + 4 + 1) + 256.0 * v_miss * n
    if kind == "insert":
        return n * (8 + 64 + 1) + 256.0 * v_miss * n + 8.0 * new_slabs
    if kind == "delete":
        return n * (4 + 64 + 1) + 256.0 * v_hit * n
    if kind == "mixed":
        ni, nd, nh, nm = mix
        assert ni + nd + nh + nm == n
        return (n * (1 + 4 + 4 + 4 + 1) + 256.0 * ((ni + nm) * v_miss + (nd + nh) * v_hit)
                + 64.0 * (ni + nd) + 8.0 * ni / 31)
    raise ValueError(kind)


def make_inputs(util: float, seed: int = 11):
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    wl = W.bulk(seed=seed, n=N_KEYS, prime=S.SH_HASH_PRIME)
    rng = W.SplitMix64(seed ^ 0xABCDEF)
    n_ins, n_del, n_hit, n_miss = W.gamma_counts(MIX_BATCH, GAMMA1)
    fresh = W.unique_keys(rng, n_ins * MIX_BATCHES, exclude=np.concatenate(
        [wl["keys"], wl["q_miss"]]))
    present = wl["keys"].copy()
    batches = []
    for bi in range(MIX_BATCHES):
        ops, bk, bv = W.mixed_batch(rng, present, fresh[bi * n_ins:(bi + 1) * n_ins],
                                    wl["q_miss"], n_ins, n_del, n_hit, n_miss)
        batches.append((ops, bk, bv))
        dels = bk[ops == 2]
        present = np.concatenate([present[~np.isin(present, dels)], bk[ops == 1]])
    return wl, batches


def repeat_for(fn, min_s: float = 10.0, max_runs: int = 30):
    """Calls fn() until at least min_s seconds have passed (at most max_runs times); returns
    (runs, seconds)."""
    runs, t0 = 0, time.perf_counter()
    while True:
        fn()
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or runs >= max_runs:
            return runs, dt


def cpu_baseline(wl, batches, B):
    """The CPU oracle (single-threaded C) over whole steps on the host: table set-up, build,
    both searches and the mixed batches, repeated on a fresh table until about 10 s of work."""
    import oracle
    from paper_1710_11246_amd import slabhash as S

    def one_step():
        o = oracle.Oracle(B, S.SH_SLAB_PAIRS, wl.hash_a, wl.hash_b)
        o.replace(wl["keys"], wl["vals"])
        o.search(wl["q_hit"])
        o.search(wl["q_miss"])
        for ops, bk, bv in batches:
            o.mixed(ops, bk, bv)

    runs, dt = repeat_for(one_step)
    n_ops = 3 * N_KEYS + MIX_BATCHES * MIX_BATCH
    return {"value": round(runs * n_ops / dt / 1e6, 3), "unit": "M ops/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d whole steps on one host core, each on a fresh table: build 2^22, 2^22 "
                      "hit + 2^22 miss searches, 16 mixed batches of 2^16 (%.1f s)" % (runs, dt),
            "host": host_info()}


def host_info() -> dict:
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "cpu": cpu}


def host_threads(cap: int = 16) -> int:
    """Threads for the host-side runs: the CPUs this process may use, at most `cap`."""
    return max(1, min(cap, len(os.sched_getaffinity(0))))


def oracle_partitioned(B, hash_a, hash_b, build, searches, batches, threads):
    """One step's ops on `threads` oracles at once. Thread i owns the buckets h(k) mod threads
    and applies its share of every phase in the original order, so each bucket sees the same
    sequence of ops as under the single-threaded oracle, and every per-op result is the same
    (ops on different buckets commute). The oracle's C calls release the interpreter lock.

    build: (keys, vals); searches: list of key arrays; batches: list of (ops, keys, vals).
    Returns (build status, [(vals, found) per search], [(vals, status) per batch], oracles)."""
    import threading
    import oracle
    from paper_1710_11246_amd import slabhash as S
    T = int(threads)
    orcs = [None] * T
    orcs[0] = oracle.Oracle(B, S.SH_SLAB_PAIRS, hash_a, hash_b)

    def part_of(keys):  # the thread each op goes to
        return (orcs[0].bucket_of(keys) % np.uint32(T)).astype(np.uint8)

    bk, bv = build
    b_part = part_of(bk)
    s_part = [part_of(q) for q in searches]
    m_part = [part_of(k) for _, k, _ in batches]
    st_build = np.empty(bk.size, np.uint8)
    s_out = [(np.empty(q.size, np.uint32), np.empty(q.size, np.uint8)) for q in searches]
    m_out = [(np.empty(k.size, np.uint32), np.empty(k.size, np.uint8)) for _, k, _ in batches]
    errors = []

    def work(i):
        try:
            if orcs[i] is None:
                orcs[i] = oracle.Oracle(B, S.SH_SLAB_PAIRS, hash_a, hash_b)
            o = orcs[i]
            # each thread finds its own share, in the original order (numpy's compare and
            # nonzero release the interpreter lock, so the routing runs in parallel too)
            ix = np.flatnonzero(b_part == i)
            st_build[ix] = o.replace(bk[ix], bv[ix])
            for q, part, (vo, fo) in zip(searches, s_part, s_out):
                ix = np.flatnonzero(part == i)
                v, f, _ = o.search(q[ix])
                vo[ix], fo[ix] = v, f
            for (ops, k, v), part, (vo, so) in zip(batches, m_part, m_out):
                ix = np.flatnonzero(part == i)
                vo[ix], so[ix] = o.mixed(ops[ix], k[ix], v[ix])
        except Exception as e:  # re-raised in the caller
            errors.append(e)

    ths = [threading.Thread(target=work, args=(i,)) for i in range(T)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    if errors:
        raise errors[0]
    return st_build, s_out, m_out, orcs


def cpu_partitioned(wl, batches, B):
    """The CPU oracle over one whole step, bucket-partitioned across the host's cores."""
    T = host_threads()
    runs, dt = repeat_for(lambda: oracle_partitioned(
        B, wl.hash_a, wl.hash_b, (wl["keys"], wl["vals"]), [wl["q_hit"], wl["q_miss"]],
        batches, T), max_runs=100)
    n_ops = 3 * N_KEYS + MIX_BATCHES * MIX_BATCH
    return {"value": round(runs * n_ops / dt / 1e6, 3), "unit": "M ops/s", "cores": T,
            "kind": "oracle, bucket-partitioned",
            "sample": "%d whole steps on %d host threads, each on fresh tables, ops routed to "
                      "thread h(k) mod %d in their original order (%.1f s, routing and table "
                      "set-up included)" % (runs, T, T, dt),
            "host": host_info()}


def run_batched(seed: int = 31, T: int = 256, rounds: int = 20, wpc_override: int = 0):
    """Batched workload: T tables with log-uniform sizes in [2^10, 2^20] (bulk-built), then
    `rounds` rounds in each of which every table gets one mixed batch of log-uniform length in
    [2^6, 2^16] (30% insert new / 10% delete existing / 60% search, half existing, half absent).
    Buckets and pools come from the autotuner's Binomial model for utilisation 0.6 at each
    table's final occupancy; the batched launch shape is picked by timing candidates on round 0.
    Three forms run the same rounds on identically built tables: one sh_mixed launch per table,
    one batched launch per round, and all rounds' batched launches captured into one graph and
    replayed once. Returns a dict of results."""
    import torch
    from paper_1710_11246_amd import autotune as A
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    t0 = time.perf_counter()
    mr = W.multi_rounds(seed=seed, T=T, n_lo=1 << 10, n_hi=1 << 20, len_lo=1 << 6,
                        len_hi=1 << 16, rounds=rounds, fractions=(0.3, 0.1, 0.3, 0.3),
                        prime=S.SH_HASH_PRIME)
    params = []
    for t in range(T):
        occ = int(mr.final_occupancy[t])
        B = A.buckets_for_utilisation(occ, 0.6)
        params.append(S.ShParams(B, A.pool_slabs_for(occ, B), int(mr.hash_a[t]),
                                 int(mr.hash_b[t])))
    log("batched inputs: %d tables, %d rounds, %d ops/round avg (%.1f s)" % (
        T, rounds, sum(k.size for k in mr.keys) // rounds, time.perf_counter() - t0))
    m = S.MultiSlabHash(params)
    init_k = [S.to_dev(k) for k in mr.init_keys]
    init_v = [S.to_dev(v) for v in mr.init_vals]
    sizes = [k.size for k in mr.keys]
    offs = np.cumsum([0] + sizes)
    all_ops = S.to_dev(np.concatenate(mr.ops))
    all_keys = S.to_dev(np.concatenate(mr.keys))
    all_vals = S.to_dev(np.concatenate(mr.vals))
    n_all = int(offs[-1])
    vout = torch.empty(n_all, dtype=torch.int32, device="cuda")
    sout = torch.empty(n_all, dtype=torch.uint8, device="cuda")
    h_descs = [S.pack_batch_descs(mr.offsets[r] + offs[r], mr.lengths[r], range(T))
               for r in range(rounds)]
    descs = [S.to_dev(d) for d in h_descs]

    def rebuild():
        for t, tb in enumerate(m.tables):
            tb.reset()
        for t, tb in enumerate(m.tables):
            S.sh_build(tb.handle, init_k[t], init_v[t], None)
        torch.cuda.synchronize()

    def timed(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3

    # launch shape for the batched form, tuned on round 0
    def run_shape(wpc, c):
        rebuild()
        S.sh_multi_set_launch(m.handle, wpc, c)
        return timed(lambda: S.sh_multi_mixed(m.handle, descs[0], T, all_ops, all_keys,
                                              all_vals, vout, sout))
    shape, timings = A.tune_launch("multi_mixed", sizes[0], run_shape,
                                   torch.cuda.get_device_name(), use_cache=False)
    if wpc_override:
        shape = (wpc_override, shape[1])
    S.sh_multi_set_launch(m.handle, *shape)

    # (i) one sh_mixed launch per table, issued from C
    rebuild()
    t_plain = timed(lambda: [S.sh_multi_mixed_each(m.handle, h_descs[r], all_ops, all_keys,
                                                   all_vals, vout, sout) for r in range(rounds)])
    st_plain = sout.clone()
    # (ii) one batched launch per round
    rebuild()
    t_batched = timed(lambda: [S.sh_multi_mixed(m.handle, descs[r], T, all_ops, all_keys,
                                                all_vals, vout, sout) for r in range(rounds)])
    mut = torch.from_numpy(np.concatenate(mr.ops) != 0).to("cuda")
    same_plain = bool(((sout == st_plain) | ~mut).all())
    # (iii) every round's batched launch captured once into one graph (sh_capture_begin/end
    # on a side stream), replayed as a single submission
    rebuild()
    cs = torch.cuda.Stream()
    S.sh_capture_begin(cs)
    try:
        for r in range(rounds):
            S.sh_multi_mixed(m.handle, descs[r], T, all_ops, all_keys, all_vals, vout, sout, cs)
    finally:
        g = S.sh_capture_end(cs)
    try:
        t_graph = timed(lambda: S.sh_graph_launch(g))
    finally:
        S.sh_graph_destroy(g)
    same_graph = bool(((sout == st_plain) | ~mut).all())
    # (iv) the plain form's per-table launches (256 a round) captured once into one graph and
    # replayed: where launches are short, the graph removes the host's cost per launch
    rebuild()
    S.sh_capture_begin(cs)
    try:
        for r in range(rounds):
            S.sh_multi_mixed_each(m.handle, h_descs[r], all_ops, all_keys, all_vals, vout, sout,
                                  cs)
    finally:
        g = S.sh_capture_end(cs)
    try:
        t_plain_graph = timed(lambda: S.sh_graph_launch(g))
    finally:
        S.sh_graph_destroy(g)
    same_graph = same_graph and bool(((sout == st_plain) | ~mut).all())
    stats = [tb.stats() for tb in m.tables[:4]]
    res = {
        "workload": "256 tables, n log-uniform [2^10, 2^20], 20 rounds of one batch per table, "
                    "length log-uniform [2^6, 2^16], 30/10/60 insert/delete/search",
        "tables": T, "rounds": rounds, "total_keys_built": int(sum(k.size for k in mr.init_keys)),
        "ops": n_all, "launch_shape": list(shape),
        "plain_ms_per_round": round(t_plain * 1e3 / rounds, 3),
        "batched_ms_per_round": round(t_batched * 1e3 / rounds, 3),
        "graph_ms_per_round": round(t_graph * 1e3 / rounds, 3),
        "plain_Mops": round(n_all / t_plain / 1e6, 1),
        "batched_Mops": round(n_all / t_batched / 1e6, 1),
        "graph_Mops": round(n_all / t_graph / 1e6, 1),
        "plain_graph_ms_per_round": round(t_plain_graph * 1e3 / rounds, 3),
        "speedup_graph_vs_plain": round(t_plain / t_graph, 2),
        "speedup_plain_graph_vs_plain": round(t_plain / t_plain_graph, 2),
        "graph_note": "a graph replay saves the host's cost per launch only: the batched form "
                      "launches one kernel a round, so its replay runs at the eager rate; the "
                      "plain form's 256 short launches a round gain from it",
        "mutation_status_equal_to_plain": same_plain and same_graph,
        "utilisation_first_tables": [round(8.0 * s["live"] / (256.0 * s["slabs_total"]), 3)
                                     for s in stats],
    }
    return res


def run_concurrent(seed: int = 51, total: int = 1 << 24, batch: int = 1 << 16,
                   B: int = 793240, per_gamma: int = 16) -> dict:
    """Concurrent workload ("Incremental insertion" and "Concurrent benchmarks"): one table with
    B buckets (final utilisation about 0.65 after 2^24 keys) grows by insert-only batches of
    `batch` fresh keys; when it holds 2^20, 2^22 and 2^24 growth keys, `per_gamma` mixed batches
    of 2^16 ops run for each of the paper's distributions Gamma0, Gamma1 and Gamma2. Every batch
    is its own sh_insert or sh_mixed launch, timed with HIP events."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    t0 = time.perf_counter()
    cps = [1 << 20, 1 << 22, 1 << 24]
    g = W.growth_checkpoints(seed, total, batch, cps, per_gamma, MIX_BATCH, S.SH_HASH_PRIME)
    log("concurrent inputs: %d growth keys, %d mixed batches (%.1f s)" % (
        total, sum(len(b) for pc in g.mixed for _, b in pc), time.perf_counter() - t0))
    pool = S.pool_slabs_bound(total + g.mixed_inserts)
    t = S.SlabHash(B, pool, g.hash_a, g.hash_b)
    kd, vd = S.to_dev(g.keys), S.to_dev(g.vals)
    st = torch.empty(batch, dtype=torch.uint8, device="cuda")
    vo = torch.empty(MIX_BATCH, dtype=torch.int32, device="cuda")
    so = torch.empty(MIX_BATCH, dtype=torch.uint8, device="cuda")
    grown = 0
    growth_ms = []
    cp_res = []
    for cp, per_cp in zip(cps, g.mixed):
        evs = []
        for s0 in range(grown, cp, batch):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            S.sh_insert(t.handle, kd[s0:s0 + batch], vd[s0:s0 + batch], st)
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        growth_ms += [a.elapsed_time(b) for a, b in evs]
        grown = cp
        stats = t.stats()
        r = {"growth_keys": cp,
             "utilisation": round(8.0 * stats["live"] / (256.0 * stats["slabs_total"]), 4),
             "insert_batch_Mops_last16": round(
                 batch * 16 / (sum(growth_ms[-16:]) * 1e-3) / 1e6, 1)}
        for name, batches in per_cp:
            dev = [(S.to_dev(o), S.to_dev(k), S.to_dev(v)) for o, k, v in batches]
            evs = []
            for o, k, v in dev:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                S.sh_mixed(t.handle, o, k, v, vo, so)
                e1.record()
                evs.append((e0, e1))
            torch.cuda.synchronize()
            ms = [a.elapsed_time(b) for a, b in evs]
            r[name + "_Mops"] = round(MIX_BATCH * len(ms) / (sum(ms) * 1e-3) / 1e6, 1)
        cp_res.append(r)
        log("  grown to %d: %s" % (cp, r))
    end = t.stats()
    return {
        "workload": "grow to 2^24 uniform keys in insert batches of 2^16 (B=793240, final "
                    "utilisation ~0.65); at 2^20, 2^22 and 2^24 keys, 16 concurrent batches of "
                    "2^16 ops for each of Gamma0 (0.5,0.5,0,0), Gamma1 (0.2,0.2,0.3,0.3), "
                    "Gamma2 (0.1,0.1,0.4,0.4)",
        "num_buckets": B, "pool_slabs": pool, "insert_batch": batch,
        "insert_batches": len(growth_ms),
        "insert_Mops_overall": round(total / (sum(growth_ms) * 1e-3) / 1e6, 1),
        "checkpoints": cp_res,
        "violations_end": end["violations"], "error_word_end": end["error_word"],
    }


def run_served(seed: int = 41, n_keys: int = 1 << 26, n_req: int = 10000,
               loads=(0.5, 0.8, 0.95)):
    """Served workload: a resident table of n_keys uint32 keys (buckets from the autotuner for
    utilisation 0.6, pool sized for the run's inserts) receiving n_req requests, each a mixed
    batch of log-uniform length in [1, 2^16] with i.i.d. ops 10% insert (fresh keys) / 5%
    delete (initial keys, each at most once) / 85% search (Zipf s = 1.1 over the initial keys).
    The plain path's capacity is measured by running every request as its own sh_mixed launch,
    back to back; the server's by submitting all requests at once. Poisson arrivals at each
    offered load (a fraction of the plain capacity, then of the server's) give p50/p99 latency
    (completion minus arrival, including time waiting for admission) and throughput. The table
    is rebuilt before each run."""
    import torch
    from paper_1710_11246_amd import autotune as A
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    t0 = time.perf_counter()
    rng = W.SplitMix64(seed)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    init = W.distinct_keys(seed, 0, n_keys)
    fresh = W.distinct_keys(seed, n_keys, n_keys // 4)  # disjoint from init by construction
    sr = W.served_requests(seed + 1, init, n_req, 1, 1 << 16, fractions=(0.10, 0.05, 0.85),
                           zipf_s=1.1, shuffle_ranking=False, fresh_keys=fresh)
    n_final = n_keys + int(sr.inserts.sum())
    B = A.buckets_for_utilisation(n_final, 0.6)
    # Admission promises each request its worst case (a new slab per insert), so beyond the
    # expected overflow the pool carries 2^20 slabs (256 MB) of headroom for those promises.
    params = [S.ShParams(B, A.pool_slabs_for(n_final, B) + (1 << 20), a, b)]
    log("served inputs: %d keys, %d requests, %d ops (%.1f s)" % (
        n_keys, n_req, sr.keys.size, time.perf_counter() - t0))
    m = S.MultiSlabHash(params)
    tb = m.tables[0]
    kd, vd = S.to_dev(init), S.to_dev(W.value_of(init))
    ops, keys, vals = S.to_dev(sr.ops), S.to_dev(sr.keys), S.to_dev(sr.vals)
    vout = torch.empty(keys.numel(), dtype=torch.int32, device="cuda")
    sout = torch.empty(keys.numel(), dtype=torch.uint8, device="cuda")
    n_ops = int(sr.keys.size)
    mean_len = n_ops / n_req

    def rebuild():
        tb.reset()
        S.sh_build(tb.handle, kd, vd, None)
        torch.cuda.synchronize()

    rebuild()
    st0 = tb.stats()
    h_desc = S.pack_batch_descs(sr.offsets, sr.lengths, np.zeros(n_req, np.int64))
    torch.cuda.synchronize()
    t = time.perf_counter()
    S.sh_multi_mixed_each(m.handle, h_desc, ops, keys, vals, vout, sout)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t
    cap_plain = n_ops / plain_s

    def serve(arrivals):
        rebuild()
        with S.Server(tb, ops, keys, vals) as srv:
            adm, done = srv.replay(sr.offsets, sr.lengths, sr.inserts, arrivals)
            srv.stop()
        ok = done != np.iinfo(np.uint64).max
        lat = (done[ok].astype(np.int64) - arrivals[ok].astype(np.int64)) / 1e3  # us
        span = (int(done[ok].max()) - int(arrivals.min())) / 1e9
        return {"p50_us": round(float(np.percentile(lat, 50)), 1),
                "p99_us": round(float(np.percentile(lat, 99)), 1),
                "mean_us": round(float(lat.mean()), 1),
                "Mops": round(float(sr.lengths[ok].sum()) / span / 1e6, 1),
                "rejected": int((~ok).sum())}

    closed = serve(np.zeros(n_req, np.uint64))
    cap_served = closed["Mops"] * 1e6
    points = []
    for ref, cap in (("plain", cap_plain), ("served", cap_served)):
        for load in loads:
            rate = load * cap / mean_len
            arr = W.poisson_arrivals(W.SplitMix64(seed + 7), n_req, rate)
            r = serve(arr)
            r.update({"offered_load": load, "of_capacity": ref,
                      "offered_Mops": round(load * cap / 1e6, 1),
                      "arrival_rate_per_s": round(rate, 1)})
            points.append(r)
    s_end = tb.stats()
    return {
        "workload": "resident 2^26-key table, %d requests of log-uniform length [1, 2^16], "
                    "10/5/85 insert/delete/search, Zipf 1.1 searches, Poisson arrivals" % n_req,
        "keys": n_keys, "num_buckets": B, "pool_slabs": params[0].pool_slabs,
        "ops": n_ops, "mean_request_ops": round(mean_len, 1),
        "utilisation_start": round(8.0 * st0["live"] / (256.0 * st0["slabs_total"]), 4),
        "plain_capacity_Mops": round(cap_plain / 1e6, 1),
        "served_closed_loop": closed,
        "served_closed_loop_vs_plain": round(closed["Mops"] * 1e6 / cap_plain, 2),
        "load_points": points,
        "violations_end": s_end["violations"], "error_word_end": s_end["error_word"],
    }


def sweep_utilisation(wl0, n_seeds: int = 5, reps: int = 3) -> dict:
    """Bulk build of 2^22 keys, then 2^22 all-hit and 2^22 all-miss searches, at every
    utilisation target's bucket count, for `n_seeds` independent workloads (the first is the
    step's). Per seed: the median of `reps` runs after one untimed run; reported: the median
    over seeds in M ops/s, the range over seeds, the achieved utilisation's range, and for the
    first workload the algorithmic bytes (op_bytes, with that table's own slabs per hit and per
    miss) over the median time as a fraction of HBM peak."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    dev = "cuda"
    st = torch.empty(N_KEYS, dtype=torch.uint8, device=dev)
    v_out = torch.empty(N_KEYS, dtype=torch.int32, device=dev)
    f_out = torch.empty(N_KEYS, dtype=torch.uint8, device=dev)
    names = ["build", "search_hit", "search_miss"]
    per = {u: {"util": [], **{nm: [] for nm in names}} for u in B_FOR_UTIL}
    for si in range(n_seeds):
        wl = wl0 if si == 0 else W.bulk(seed=1000 + si, n=N_KEYS, prime=S.SH_HASH_PRIME)
        log("utilisation sweep: seed %d of %d" % (si + 1, n_seeds))
        keys, vals = S.to_dev(wl["keys"]), S.to_dev(wl["vals"])
        q_hit, q_miss = S.to_dev(wl["q_hit"]), S.to_dev(wl["q_miss"])
        for u, Bu in sorted(B_FOR_UTIL.items()):
            tu = S.SlabHash(Bu, S.pool_slabs_bound(N_KEYS), wl.hash_a, wl.hash_b)
            res = {nm: [] for nm in names}
            for rep in range(reps + 1):
                tu.reset()
                e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                e[0].record()
                S.sh_build(tu.handle, keys, vals, st)
                e[1].record()
                S.sh_search(tu.handle, q_hit, v_out, f_out)
                e[2].record()
                S.sh_search(tu.handle, q_miss, v_out, f_out)
                e[3].record()
                torch.cuda.synchronize()
                if rep:
                    for i, nm in enumerate(names):
                        res[nm].append(e[i].elapsed_time(e[i + 1]))
            assert bool((st == 1).all()) and bool((f_out == 0).all())
            s_u = tu.stats()
            per[u]["util"].append(8.0 * s_u["live"] / (256.0 * s_u["slabs_total"]))
            for nm in names:
                per[u][nm].append(N_KEYS / (float(np.median(res[nm])) * 1e-3) / 1e6)
            if si == 0:
                _, _, _, counts, viol = tu.dump()
                assert viol == 0
                v_hit = chain_visits(counts[:, 0].astype(np.int64) + counts[:, 1]) / N_KEYS
                v_miss = float(counts[:, 2].mean())
                kinds = {"build": "insert", "search_hit": "search_hit",
                         "search_miss": "search_miss"}
                per[u]["frac_hbm"] = {
                    nm: round(op_bytes(kinds[nm], N_KEYS, v_hit, v_miss,
                                       new_slabs=s_u["pool_allocated"] if nm == "build" else 0)
                              / (float(np.median(res[nm])) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                    for nm in names}
                per[u]["slabs_per_miss"] = round(v_miss, 4)
            del tu
        del keys, vals, q_hit, q_miss
    out = {"seeds": n_seeds, "reps_per_seed": reps}
    for u, Bu in sorted(B_FOR_UTIL.items()):
        r = {"num_buckets": Bu,
             "utilisation": [round(min(per[u]["util"]), 4), round(max(per[u]["util"]), 4)]}
        for nm in names:
            xs = per[u][nm]
            r[nm] = round(float(np.median(xs)), 1)
            r[nm + "_range"] = [round(min(xs), 1), round(max(xs), 1)]
        r["frac_hbm"] = per[u]["frac_hbm"]
        r["slabs_per_miss"] = per[u]["slabs_per_miss"]
        out[str(u)] = r
    return out


def measure_config1(reps: int = 20) -> dict:
    """The small phased configuration: 2^16 unique keys (value = SplitMix64 finaliser of the
    key, seed 1) bulk-built into 2^12 buckets, 2^16 searches (half present, half absent), a
    random 25% of the keys deleted, the searches again. Median of `reps` passes after one
    untimed pass, each on a reset table; every result is checked against the first pass."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    n = 1 << 16
    wl = W.phased(seed=1, n=n, n_queries=n, hit_fraction=0.5, delete_fraction=0.25,
                  prime=S.SH_HASH_PRIME)
    t = S.SlabHash(1 << 12, S.pool_slabs_bound(n), wl.hash_a, wl.hash_b)
    kd, vd = S.to_dev(wl["keys"]), S.to_dev(wl["vals"])
    qd, dd = S.to_dev(wl["queries"]), S.to_dev(wl["deletes"])
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    ds = torch.empty(dd.numel(), dtype=torch.uint8, device="cuda")
    vo = torch.empty(n, dtype=torch.int32, device="cuda")
    fo = torch.empty(n, dtype=torch.uint8, device="cuda")
    vo2 = torch.empty(n, dtype=torch.int32, device="cuda")
    fo2 = torch.empty(n, dtype=torch.uint8, device="cuda")
    names = ("build", "search", "delete", "search_after")
    res = {k: [] for k in names}
    first = None
    for rep in range(reps + 1):
        t.reset()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record()
        S.sh_build(t.handle, kd, vd, st)
        e[1].record()
        S.sh_search(t.handle, qd, vo, fo)
        e[2].record()
        S.sh_delete(t.handle, dd, ds)
        e[3].record()
        S.sh_search(t.handle, qd, vo2, fo2)
        e[4].record()
        torch.cuda.synchronize()
        outs = (st.clone(), fo.clone(), vo.clone(), ds.clone(), fo2.clone(), vo2.clone())
        if first is None:
            first = outs
        assert all(bool((a == b).all()) for a, b in zip(outs, first))
        if rep:
            for i, k in enumerate(names):
                res[k].append(e[i].elapsed_time(e[i + 1]))
    counts = {"build": n, "search": n, "delete": int(dd.numel()), "search_after": n}
    out = {"workload": "2^16 keys into 2^12 buckets; 2^16 searches (50% present); delete 25%; "
                       "search again", "reps": reps}
    for k in names:
        ms = float(np.median(res[k]))
        out[k] = {"median_us": round(ms * 1e3, 2), "Mops": round(counts[k] / (ms * 1e-3) / 1e6, 1)}
    total = sum(float(np.median(res[k])) for k in names)
    out["pass_us"] = round(total * 1e3, 2)
    out["pass_Mops"] = round(sum(counts.values()) / (total * 1e-3) / 1e6, 1)
    del t
    return out


def sweep_sizes(log2_sizes=(16, 18, 20, 22, 24), util: float = 0.6, reps: int = 5) -> dict:
    """Bulk build, all-hit search and all-miss search against table size ("Bulk benchmarks"): n
    distinct uniform keys for each n = 2^k, buckets from the Binomial model for the target
    utilisation, median of `reps` runs (each build on a reset table). Every status, found flag
    and hit value of the last run is checked on the device."""
    import torch
    from paper_1710_11246_amd import autotune as A
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    out = {}
    for k in log2_sizes:
        n = 1 << k
        keys = W.distinct_keys(100 + k, 0, n)
        miss = W.distinct_keys(100 + k, n, n)
        perm = W.SplitMix64(200 + k).permutation(n)
        rng = W.SplitMix64(300 + k)
        a, b = W.hash_params(rng, S.SH_HASH_PRIME)
        B = A.buckets_for_utilisation(n, util)
        t = S.SlabHash(B, A.pool_slabs_for(n, B), a, b)
        vals = W.value_of(keys)
        kd, vd = S.to_dev(keys), S.to_dev(vals)
        qh, qm = S.to_dev(keys[perm]), S.to_dev(miss)
        want = S.to_dev(vals[perm])
        st = torch.empty(n, dtype=torch.uint8, device="cuda")
        vo = torch.empty(n, dtype=torch.int32, device="cuda")
        fo = torch.empty(n, dtype=torch.uint8, device="cuda")
        vm = torch.empty(n, dtype=torch.int32, device="cuda")
        fm = torch.empty(n, dtype=torch.uint8, device="cuda")
        res = {"build": [], "search_hit": [], "search_miss": []}
        for _ in range(reps + 1):
            t.reset()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record()
            S.sh_build(t.handle, kd, vd, st)
            e[1].record()
            S.sh_search(t.handle, qh, vo, fo)
            e[2].record()
            S.sh_search(t.handle, qm, vm, fm)
            e[3].record()
            torch.cuda.synchronize()
            for i, nm in enumerate(("build", "search_hit", "search_miss")):
                res[nm].append(e[i].elapsed_time(e[i + 1]))
        # every insert new, every hit found with its value, every miss absent
        assert bool((st == 1).all()) and bool((fo == 1).all()) and bool((vo == want).all())
        assert not bool(fm.any())
        su = t.stats()
        out["2^%d" % k] = {
            "num_buckets": B,
            "utilisation": round(8.0 * su["live"] / (256.0 * su["slabs_total"]), 4),
            **{nm + "_Mops": round(n / (float(np.median(v[1:])) * 1e-3) / 1e6, 1)
               for nm, v in res.items()}}
        log("  size 2^%d: %s" % (k, out["2^%d" % k]))
        del t, kd, vd, qh, qm, want, st, vo, fo, vm, fm
        torch.cuda.empty_cache()
    return out


def measure_hbm_resident(log2n: int = 26, util: float = 0.6, reps: int = 3,
                         seed: int = 61) -> dict:
    """A table far larger than the 256 MB Infinity Cache: bulk build of 2^26 distinct uniform
    keys into the bucket count whose Binomial-model utilisation is 0.6 (about 0.9 GB of base
    slabs), then 2^26 all-hit searches (a permutation of the keys) and 2^26 all-miss searches.
    Median of `reps` runs after one untimed run, each build on a reset table, HIP events around
    each call. Every status, found flag and hit value is checked on the device. Algorithmic
    bytes follow op_bytes with the built table's own slabs per hit and per miss. Afterwards the
    access patterns of measure_patterns are timed over a buffer of the table's size, and each
    kernel is reported against its own pattern's ceiling."""
    import torch
    from paper_1710_11246_amd import autotune as A
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    n = 1 << log2n
    keys = W.distinct_keys(seed, 0, n)
    miss = W.distinct_keys(seed, n, n)
    perm = W.SplitMix64(seed + 1).permutation(n)
    rng = W.SplitMix64(seed + 2)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    B = A.buckets_for_utilisation(n, util)
    t = S.SlabHash(B, A.pool_slabs_for(n, B), a, b)
    vals = W.value_of(keys)
    kd, vd = S.to_dev(keys), S.to_dev(vals)
    qh, qm = S.to_dev(keys[perm]), S.to_dev(miss)
    want = S.to_dev(vals[perm])
    del keys, miss, perm, vals
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    vo = torch.empty(n, dtype=torch.int32, device="cuda")
    fo = torch.empty(n, dtype=torch.uint8, device="cuda")
    vm = torch.empty(n, dtype=torch.int32, device="cuda")
    fm = torch.empty(n, dtype=torch.uint8, device="cuda")
    names = ("build", "search_hit", "search_miss")
    res = {k: [] for k in names}
    for rep in range(reps + 1):
        t.reset()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        S.sh_build(t.handle, kd, vd, st)
        e[1].record()
        S.sh_search(t.handle, qh, vo, fo)
        e[2].record()
        S.sh_search(t.handle, qm, vm, fm)
        e[3].record()
        torch.cuda.synchronize()
        # checked after the timed span, so that no check runs between the events
        assert bool((st == 1).all()) and bool((fo == 1).all()) and bool((vo == want).all())
        assert not bool(fm.any())
        if rep:
            for i, k in enumerate(names):
                res[k].append(e[i].elapsed_time(e[i + 1]))
    su = t.stats()
    counts = torch.empty(3 * B, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    viol = torch.zeros(1, dtype=torch.int32, device="cuda")
    S.sh_dump(t.handle, None, None, None, counts, cnt, viol)
    c = S.to_host_u32(counts).reshape(-1, 3)
    assert int(viol.item()) == 0 and int(cnt.item()) == n
    v_hit = chain_visits(c[:, 0].astype(np.int64) + c[:, 1]) / n
    v_miss = float(c[:, 2].mean())
    bytes_l = {"build": op_bytes("insert", n, v_hit, v_miss, new_slabs=su["pool_allocated"]),
               "search_hit": op_bytes("search_hit", n, v_hit, v_miss),
               "search_miss": op_bytes("search_miss", n, v_hit, v_miss)}
    traffic_ok = source_sha() == TRAFFIC_SRC_SHA
    out = {"workload": "bulk build of 2^%d uniform uint32 keys, then 2^%d all-hit and 2^%d "
                       "all-miss searches" % (log2n, log2n, log2n),
           "keys": n, "num_buckets": B, "table_bytes": int(t.storage.numel()),
           "utilisation": round(8.0 * su["live"] / (256.0 * su["slabs_total"]), 4),
           "slabs_per_hit": round(v_hit, 4), "slabs_per_miss": round(v_miss, 4)}
    for k in names:
        ms = float(np.median(res[k]))
        gbs = bytes_l[k] / (ms * 1e-3) / 1e9
        out[k] = {"avg_ms": round(ms, 4), "Mops": round(n / (ms * 1e-3) / 1e6, 1),
                  "bytes_per_launch": int(bytes_l[k]), "algorithmic_GBps": round(gbs, 1),
                  "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                  "traffic_bytes": HBM_TRAFFIC_BYTES.get(k) if traffic_ok else None}
    table_bytes = int(t.storage.numel())
    del t, kd, vd, qh, qm, want, st, vo, fo, vm, fm
    torch.cuda.empty_cache()
    # the same access patterns' ceilings over a buffer of the table's size (random 256-byte
    # slab reads and swaps from HBM, which the MALL cannot hold)
    pats = measure_patterns(table_bytes, n, reps=3)
    out["access_patterns"] = pats
    for k, pat in (("build", "insert_io"), ("search_hit", "search_io"),
                   ("search_miss", "search_io")):
        out[k]["pattern_ceiling_ms"] = round(pats[pat + "_us"] / 1e3, 4)
        out[k]["frac_of_pattern_ceiling"] = round(pats[pat + "_us"] / 1e3 / out[k]["avg_ms"], 4)
    return out


def sweep_batches(log2_batches=(15, 16, 17), total: int = 1 << 24, B: int = 793240) -> dict:
    """Incremental insertion ("Incremental insertion"): 2^24 distinct keys inserted in batches of
    each size into a table whose final utilisation is about 0.65; the rate over all batches and
    over the last eighth of them. Every insert's status is checked on the device."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    keys = W.distinct_keys(71, 0, total)
    kd, vd = S.to_dev(keys), S.to_dev(W.value_of(keys))
    rng = W.SplitMix64(72)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(B, S.pool_slabs_bound(total), a, b)
    out = {}
    for k in log2_batches:
        g = 1 << k
        t.reset()
        st = torch.empty(total, dtype=torch.uint8, device="cuda")
        evs = []
        for s0 in range(0, total, g):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            S.sh_insert(t.handle, kd[s0:s0 + g], vd[s0:s0 + g], st[s0:s0 + g])
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        assert bool((st == 1).all())  # every key new
        ms = [x.elapsed_time(y) for x, y in evs]
        tail = ms[-max(1, len(ms) // 8):]
        su = t.stats()
        out["2^%d" % k] = {"batches": len(ms),
                           "Mops_overall": round(total / (sum(ms) * 1e-3) / 1e6, 1),
                           "Mops_last_eighth": round(g * len(tail) / (sum(tail) * 1e-3) / 1e6, 1),
                           "final_utilisation": round(
                               8.0 * su["live"] / (256.0 * su["slabs_total"]), 4)}
        log("  batch 2^%d: %s" % (k, out["2^%d" % k]))
    return out


def measure_duplicates(n_keys: int = 1 << 20, copies: int = 4, B: int = 217316,
                       reps: int = 3) -> dict:
    """The multiset operations ("Supported Operations") on a table with duplicates allowed: 2^20
    keys, each inserted `copies` times (one copy per INSERT batch of 2^20), then SEARCH of 2^22
    random copies' keys, SEARCHALL of every key (a counting pass, then a pass writing the values
    into ranges sized from the counts), DELETE of each key's first copy and DELETEALL of the
    rest. Median of `reps` runs on a rebuilt table, HIP events around each call."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    keys = W.distinct_keys(81, 0, n_keys)
    kd = S.to_dev(keys)
    vd = [S.to_dev((W.value_of(keys) + np.uint32(c)).astype(np.uint32)) for c in range(copies)]
    q = S.to_dev(keys[W.SplitMix64(82).below(copies * n_keys, n_keys)])
    rng = W.SplitMix64(83)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(B, S.pool_slabs_bound(copies * n_keys), a, b, duplicates=True)
    st = torch.empty(n_keys, dtype=torch.uint8, device="cuda")
    vo = torch.empty(q.numel(), dtype=torch.int32, device="cuda")
    fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
    cnt = torch.empty(n_keys, dtype=torch.int32, device="cuda")
    off = torch.arange(0, copies * n_keys, copies, dtype=torch.int64, device="cuda")
    vals = torch.empty(copies * n_keys, dtype=torch.int32, device="cuda")
    names = ["insert", "search", "search_all_count", "search_all_values", "delete",
             "delete_all"]
    res = {k: [] for k in names}
    for _ in range(reps):
        t.reset()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        e[0].record()
        for c in range(copies):
            S.sh_insert(t.handle, kd, vd[c], st)
        e[1].record()
        S.sh_search(t.handle, q, vo, fo)
        e[2].record()
        S.sh_search_all(t.handle, kd, cnt)
        e[3].record()
        S.sh_search_all(t.handle, kd, cnt, off, vals)
        e[4].record()
        S.sh_delete(t.handle, kd, st)
        e[5].record()
        S.sh_delete_all(t.handle, kd, cnt)
        e[6].record()
        torch.cuda.synchronize()
        for i, k in enumerate(names):
            res[k].append(e[i].elapsed_time(e[i + 1]))
    assert bool((cnt == copies - 1).all()) and bool((st == 1).all())
    units = {"insert": copies * n_keys, "search": q.numel(), "search_all_count": n_keys,
             "search_all_values": n_keys, "delete": n_keys, "delete_all": n_keys}
    out = {"workload": "duplicates allowed: 2^20 keys x %d copies (one copy per insert batch), "
                       "B=%d" % (copies, B)}
    for k in names:
        ms = float(np.median(res[k]))
        out[k + "_ms"] = round(ms, 4)
        out[k + "_Mops"] = round(units[k] / (ms * 1e-3) / 1e6, 1)
    return out


def measure_keys_only(B: int = 108658, reps: int = 5) -> dict:
    """Key-only tables (the paper's 32-bit entries, 62 keys per slab): bulk build of 2^22
    distinct keys into B buckets (utilisation about 0.6), then 2^22 all-hit and 2^22 all-miss
    searches; median of `reps` runs on a reset table."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    n = 1 << 22
    keys = W.distinct_keys(91, 0, n)
    keys[keys == 0xFFFFFFFE] = W.distinct_keys(91, n, 1)[0]   # the deleted-entry marker
    miss = W.distinct_keys(91, n + 1, n)
    miss[miss == 0xFFFFFFFE] = W.distinct_keys(91, 2 * n + 1, 1)[0]
    kd, qh = S.to_dev(keys), S.to_dev(keys[W.SplitMix64(92).permutation(n)])
    qm = S.to_dev(miss)
    rng = W.SplitMix64(93)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    t = S.SlabHash(B, S.pool_slabs_bound(n), a, b, keys_only=True)
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    vo = torch.empty(n, dtype=torch.int32, device="cuda")
    fo = torch.empty(n, dtype=torch.uint8, device="cuda")
    res = {"build": [], "search_hit": [], "search_miss": []}
    for _ in range(reps):
        t.reset()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        S.sh_build(t.handle, kd, None, st)
        e[1].record()
        S.sh_search(t.handle, qh, vo, fo)
        e[2].record()
        S.sh_search(t.handle, qm, vo, fo)
        e[3].record()
        torch.cuda.synchronize()
        for i, k in enumerate(res):
            res[k].append(e[i].elapsed_time(e[i + 1]))
    assert bool((st == 1).all())
    su = t.stats()
    out = {"workload": "key-only: 2^22 distinct keys, B=%d, 62 keys per 256-byte slab" % B,
           "utilisation": round(4.0 * su["live"] / (256.0 * su["slabs_total"]), 4)}
    for k, v in res.items():
        ms = float(np.median(v))
        out[k + "_ms"] = round(ms, 4)
        out[k + "_Mops"] = round(n / (ms * 1e-3) / 1e6, 1)
    return out


def measure_flush(table, keys, vals, st, stream, reps: int = 5) -> dict:
    """FLUSH of every bucket ("Flush" subsection) of the benchmark table after half of its 2^22
    keys have been deleted: median of `reps` runs, each on a freshly built and half-deleted
    table. Algorithmic bytes: every slab read once, every kept slab written, every freed slab
    reset (256 bytes each)."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    h = table.handle
    half = keys[: keys.numel() // 2]
    dst = torch.empty(half.numel(), dtype=torch.uint8, device=keys.device)
    ts = []
    for _ in range(reps):
        S.sh_reset(h, stream)
        S.sh_build(h, keys, vals, st, stream)
        S.sh_delete(h, half, dst, stream)
        before = table.stats()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.sh_flush(h, 0, table.num_buckets, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
        after = table.stats()
    assert after["tombstones"] == 0 and after["violations"] == 0
    freed = before["pool_allocated"] - after["pool_allocated"]
    ms = float(np.median(ts))
    nbytes = 256.0 * (before["slabs_total"] + after["slabs_total"] + freed)
    return {"workload": "2^22 keys at B=%d, half deleted, flush of every bucket"
                        % table.num_buckets,
            "avg_ms": round(ms, 4), "slabs_before": before["slabs_total"],
            "slabs_after": after["slabs_total"], "slabs_freed": freed,
            "tombstones_before": before["tombstones"],
            "Mbuckets_per_s": round(table.num_buckets / (ms * 1e-3) / 1e6, 1),
            "algorithmic_GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def measure_alloc(n: int = 1 << 20, reps: int = 5) -> dict:
    """SlabAlloc on its own, as the paper measures it ("Dynamic memory allocation": a million
    slab allocations, one per thread): n allocations from a pool with 4 spare blocks, then the
    same n from a pool of exactly n slabs (the last ones must hunt for the remaining free bits),
    then freeing all n. Median of `reps` runs each, on a freshly initialised pool."""
    import torch
    from paper_1710_11246_amd import slabhash as S
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    res = {"workload": "%d slab allocations (256-byte slabs), one per lane" % n}
    for name, pool in (("alloc", n + 4 * 2048), ("alloc_full_pool", n)):
        t = S.SlabHash(1, pool, 3, 5)
        ts, tf = [], []
        for _ in range(reps):
            t.reset()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            S.sh_alloc_slabs(t.handle, n, out)
            e[1].record()
            S.sh_free_slabs(t.handle, out)
            e[2].record()
            torch.cuda.synchronize()
            ts.append(e[0].elapsed_time(e[1]))
            tf.append(e[1].elapsed_time(e[2]))
        got = S.to_host_u32(out)
        assert np.unique(got).size == n and (got < pool).all()
        # one more run with the operation counters on: claims lost to other wavefronts and
        # moves to another block
        t.reset()
        t.set_launch(0, 0, S.SH_LAUNCH_COUNTERS)
        S.sh_alloc_slabs(t.handle, n, out)
        c = t.stats()
        t.set_launch()
        res[name + "_lost_claims"] = c["alloc_lost"]
        res[name + "_block_moves"] = c["block_moves"]
        assert c["allocs"] == n
        ms = float(np.median(ts))
        res[name + "_ms"] = round(ms, 4)
        res[name + "_Mslabs_per_s"] = round(n / (ms * 1e-3) / 1e6, 1)
        if name == "alloc":
            msf = float(np.median(tf))
            res["free_ms"] = round(msf, 4)
            res["free_Mslabs_per_s"] = round(n / (msf * 1e-3) / 1e6, 1)
        del t
    return res


def measure_patterns(nbytes: int, n_ops: int, reps: int = 5) -> dict:
    """Ceilings of the operation kernels' memory access patterns, from libslabhash_roofs.so, over
    a buffer of nbytes (the benchmark table's size): n_ops random 256-byte slab reads, n_ops
    random 64-bit compare-and-swaps, n_ops slab reads each followed by a compare-and-swap into
    the slab, n_ops one-slab searches (a key loaded, the slab its mix selects read through the
    caches, value and flag written: the pattern of a search that ends in its base slab), and
    n_ops one-slab inserts (a key and value loaded, the slab read coherently, the pair swapped
    into its first empty slot, a status written: the pattern of an insert of an absent key
    into a base slab with room). Each is the median of `reps` runs at the fastest of 12 launch shapes
    (8 to 32 wavefronts per CU) and depths (1 to 16 op pairs or swaps in flight per wavefront
    iteration); the buffer is refilled with all ones before every run."""
    import torch
    from paper_1710_11246_amd import roofs as R
    buf = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    keys = torch.randint(-(1 << 31), (1 << 31) - 1, (n_ops,), dtype=torch.int32, device="cuda",
                         generator=gen)
    vals = torch.empty(n_ops, dtype=torch.int32, device="cuda")
    found = torch.empty(n_ops, dtype=torch.uint8, device="cuda")
    res = {"buffer_bytes": buf.numel() * 8, "ops": n_ops}
    runs = (("slab_load", lambda w, d, r: R.sh_roof_run(R.SH_ROOF_SLAB_LOAD, buf, n_ops, w,
                                                         seed=17 * r + 1, depth=d)),
            ("cas", lambda w, d, r: R.sh_roof_run(R.SH_ROOF_CAS, buf, n_ops, w, seed=17 * r + 1,
                                                   depth=d)),
            ("load_cas", lambda w, d, r: R.sh_roof_run(R.SH_ROOF_LOAD_CAS, buf, n_ops, w,
                                                        seed=17 * r + 1, depth=d)),
            ("search_io", lambda w, d, r: R.sh_roof_search(buf, keys, vals, found, w, d)),
            ("insert_io", lambda w, d, r: R.sh_roof_insert(buf, keys, vals, found, w, d)))
    for name, run in runs:
        best = None
        for wpc in (8, 16, 24, 32):
            for depth in (1, 4, 16):
                ts = []
                for r in range(reps + 1):
                    buf.fill_(-1)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    run(wpc, depth, r)
                    e1.record()
                    torch.cuda.synchronize()
                    if r:
                        ts.append(e0.elapsed_time(e1) * 1e3)
                t = float(np.median(ts))
                if best is None or t < best[0]:
                    best = (t, wpc, depth)
        res[name + "_us"] = round(best[0], 1)
        res[name + "_waves_per_cu"] = best[1]
        res[name + "_depth"] = best[2]
    del buf, keys, vals, found
    return res


def run_only(sections) -> dict:
    """The named sections alone (no timed step), each as the full run reports it."""
    runners = {"alloc": measure_alloc, "hbm": measure_hbm_resident, "config1": measure_config1,
               "duplicates": measure_duplicates,
               "keys_only": measure_keys_only, "batched": run_batched,
               "concurrent": run_concurrent, "served": run_served}
    out = {}
    for name in sections:
        log("section %s" % name)
        out[name] = runners[name]()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--util", type=float, default=0.6, choices=sorted(B_FOR_UTIL))
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="run the utilisation sweep over --sweep-seeds workloads (default: one)")
    ap.add_argument("--sweep-seeds", type=int, default=5,
                    help="independent workloads of the utilisation sweep with --sweep")
    ap.add_argument("--no-sweep-sizes", action="store_true",
                    help="skip build/search against table size, 2^16 .. 2^24 at utilisation 0.6 "
                         "(2^26 is the HBM-resident section)")
    ap.add_argument("--no-sweep-batches", action="store_true",
                    help="skip incremental insertion to 2^24 keys in batches of 2^15 .. 2^17")
    ap.add_argument("--step-only", action="store_true",
                    help="only the timed step and its per-kernel figures (no other section)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form section")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form section")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the incremental-growth and concurrent-batch section")
    ap.add_argument("--only", default="",
                    help="comma-separated sections to run alone, without the timed step (for "
                         "profiling runs): alloc, config1, duplicates, keys_only, hbm, batched, "
                         "concurrent, served")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, copy 1 GiB device-to-device once (a reference "
                         "for scaling hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the slab hash here is built and timed on a "
              "single MI355X (multi-GPU sharding is a design note, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1710_11246_amd import slabhash as S
    from paper_1710_11246_amd import workload as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    S.lib()
    if args.only:
        print(json.dumps(run_only(args.only.split(","))), flush=True)
        return

    B = B_FOR_UTIL[args.util]
    log("generating inputs (n=2^22, B=%d)" % B)
    wl, batches = make_inputs(args.util)
    n_ins, n_del, n_hit, n_miss = W.gamma_counts(MIX_BATCH, GAMMA1)
    pool = S.pool_slabs_bound(N_KEYS + n_ins * MIX_BATCHES)
    table = S.SlabHash(B, pool, wl.hash_a, wl.hash_b)
    if args.waves_per_cu:
        table.set_launch(args.waves_per_cu)
    h = table.handle
    dev = "cuda"
    keys, vals = S.to_dev(wl["keys"]), S.to_dev(wl["vals"])
    q_hit, q_miss = S.to_dev(wl["q_hit"]), S.to_dev(wl["q_miss"])
    st_build = torch.empty(N_KEYS, dtype=torch.uint8, device=dev)
    v_out = torch.empty(N_KEYS, dtype=torch.int32, device=dev)
    f_out = torch.empty(N_KEYS, dtype=torch.uint8, device=dev)
    mix_dev = [(S.to_dev(o), S.to_dev(k), S.to_dev(v)) for o, k, v in batches]
    mv_out = torch.empty(MIX_BATCH, dtype=torch.int32, device=dev)
    ms_out = torch.empty(MIX_BATCH, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    names = ["reset", "build", "search_hit", "search_miss", "mixed"]
    ev_warm = {k: [] for k in names}
    ev_timed = {k: [] for k in names}

    def timed(name, fn, record, ev, s):
        if name in record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            ev[name].append((e0, e1))
        else:
            fn()

    def step(record, ev, s=stream):
        timed("reset", lambda: S.sh_reset(h, s), record, ev, s)
        timed("build", lambda: S.sh_build(h, keys, vals, st_build, s), record, ev, s)
        timed("search_hit", lambda: S.sh_search(h, q_hit, v_out, f_out, s), record, ev, s)
        timed("search_miss", lambda: S.sh_search(h, q_miss, v_out, f_out, s), record, ev, s)
        for o, k, v in mix_dev:
            timed("mixed", lambda: S.sh_mixed(h, o, k, v, mv_out, ms_out, s), record, ev, s)

    def means(ev):
        return {k: (sum(a.elapsed_time(b) for a, b in v) / len(v)) for k, v in ev.items() if v}

    # Warm-up steps (untimed) carry HIP events around every launch: they give each kernel's
    # mean duration and pick the dominant kernel. The timed steps carry events only around the
    # dominant kernel's launches (events around all 20 launches of a step would add about 0.15
    # ms of gaps per step to the work being timed).
    log("warmup %d steps" % args.warmup)
    for _ in range(max(1, args.warmup)):
        step(set(names), ev_warm)
    torch.cuda.synchronize()
    avg_ms = means(ev_warm)
    per_step_ms = {k: avg_ms[k] * (MIX_BATCHES if k == "mixed" else 1) for k in avg_ms}
    dom = max((k for k in names if k != "reset"), key=lambda k: per_step_ms[k])
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step({dom}, ev_timed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("timed region done")
    ms_step = (t1 - t0) * 1e3 / args.steps
    ops_step = 3 * N_KEYS + MIX_BATCHES * MIX_BATCH
    value = ops_step / ((t1 - t0) / args.steps) / 1e6
    avg_ms[dom] = means(ev_timed)[dom]  # the dominant kernel: timed-region events
    per_step_ms[dom] = avg_ms[dom] * (MIX_BATCHES if dom == "mixed" else 1)

    # The same step captured once into a HIP graph (sh_capture_begin/end on a side stream) and
    # replayed: one submission per step instead of twenty launches. Its outputs are checked
    # after the replays.
    log("graph-replayed steps")
    gs = torch.cuda.Stream()
    S.sh_capture_begin(gs)
    try:
        step(set(), None, gs)
    finally:
        g_step = S.sh_capture_end(gs)
    try:
        for _ in range(2):
            S.sh_graph_launch(g_step, gs)
        gs.synchronize()
        ge0 = torch.cuda.Event(enable_timing=True)
        ge1 = torch.cuda.Event(enable_timing=True)
        ge0.record(gs)
        for _ in range(args.steps):
            S.sh_graph_launch(g_step, gs)
        ge1.record(gs)
        gs.synchronize()
        graph_ms_step = ge0.elapsed_time(ge1) / args.steps
    finally:
        S.sh_graph_destroy(g_step)
    assert bool((st_build == 1).all()) and not bool(f_out.any())
    graph_steps = {"ms_per_step": round(graph_ms_step, 4),
                   "Mops": round(ops_step / (graph_ms_step * 1e-3) / 1e6, 2),
                   "steps": args.steps,
                   "note": "the timed step's calls captured once with sh_capture_begin/end "
                           "and replayed as one graph per step"}

    # The table as a step leaves it (the next step's reset starts from this), then the
    # structure of the built table (before the mixed batches) for the byte accounting, with
    # the operation counters switched on for this one build.
    stats_end = table.stats()
    S.sh_set_launch(h, args.waves_per_cu, 0, S.SH_LAUNCH_COUNTERS)
    S.sh_reset(h, stream)
    S.sh_build(h, keys, vals, st_build, stream)
    assert bool((st_build == 1).all())
    stats_built = table.stats()
    _, _, _, counts, viol = table.dump()
    assert viol == 0
    occ = counts[:, 0].astype(np.int64) + counts[:, 1]
    v_hit = chain_visits(occ) / N_KEYS
    v_miss = float(counts[:, 2].mean())
    new_slabs = stats_built["pool_allocated"]
    build_counters = {k: stats_built[k] for k in
                      ("rounds", "cas_lost", "allocs", "link_lost", "block_moves")}
    build_wpc, build_opw = table.launch_shape(S.SH_OP_INSERT, N_KEYS)
    build_counters["ops_per_wave"] = build_opw
    build_counters["rounds_per_chunk"] = round(
        stats_built["rounds"] / -(-N_KEYS // build_opw), 4)
    S.sh_set_launch(h, args.waves_per_cu, 0, 0)
    util = 8.0 * stats_built["live"] / (256.0 * stats_built["slabs_total"])

    # Algorithmic bytes per launch (op_bytes): inputs and outputs once, the 256-byte slabs the
    # walks read, 64 bytes per swap and 8 per new slab; a reset writes the table's header and
    # base slabs and the pool slabs in use, and reads then zeroes the allocator bitmaps.
    bytes_l = {
        "build": op_bytes("insert", N_KEYS, v_hit, v_miss, new_slabs=new_slabs),
        "search_hit": op_bytes("search_hit", N_KEYS, v_hit, v_miss),
        "search_miss": op_bytes("search_miss", N_KEYS, v_hit, v_miss),
        "mixed": op_bytes("mixed", MIX_BATCH, v_hit, v_miss, mix=(n_ins, n_del, n_hit, n_miss)),
        "reset": float(4096 + 256 * B + 256 * stats_end["pool_allocated"] +
                       2 * 256 * (table.params.pool_slabs // 2048)),
    }
    traffic_ok = source_sha() == TRAFFIC_SRC_SHA
    kernels = {}
    for k in names:
        gbs = bytes_l[k] / (avg_ms[k] * 1e-3) / 1e9
        n_ops = {"build": N_KEYS, "search_hit": N_KEYS, "search_miss": N_KEYS,
                 "mixed": MIX_BATCH}.get(k, 0)
        kernels[k] = {"avg_ms": round(avg_ms[k], 4), "ms_per_step": round(per_step_ms[k], 4),
                      "events": "timed steps" if k == dom else "warm-up steps",
                      "algorithmic_GBps": round(gbs, 1),
                      "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
        if n_ops:
            kernels[k]["Mops"] = round(n_ops / (avg_ms[k] * 1e-3) / 1e6, 1)
        kernels[k]["traffic_bytes"] = TRAFFIC_BYTES[k] if traffic_ok else None
        # L2 hit rate and atomics per launch from the same profiled source (else null); the
        # atomic rate is those atomics over this run's mean duration
        hit, atomics, to_mem = L2_STATS.get(k, (None, None, None)) if traffic_ok else (None,) * 3
        kernels[k]["l2_hit_rate"] = hit
        kernels[k]["atomics_per_launch"] = atomics
        kernels[k]["atomics_to_memory_per_launch"] = to_mem
        kernels[k]["atomic_rate_G_per_s"] = (round(atomics / (avg_ms[k] * 1e-3) / 1e9, 2)
                                             if atomics is not None else None)
    ach = bytes_l[dom] / (avg_ms[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": TRAFFIC_BYTES[dom] if traffic_ok else None, "kernel": dom,
            "bytes_per_launch": int(bytes_l[dom])}

    if args.step_only:
        args.no_batched = args.no_served = args.no_concurrent = args.no_cpu_baseline = True
    flush = allocator = duplicates = keys_only = hbm = patterns = None
    if not args.step_only:
        log("flush")
        flush = measure_flush(table, keys, vals, st_build, stream)
        log("allocator")
        allocator = measure_alloc()
        log("duplicates")
        duplicates = measure_duplicates()
        log("keys only")
        keys_only = measure_keys_only()
        log("HBM-resident table (2^26 keys)")
        hbm = measure_hbm_resident()
        log("access-pattern ceilings")
        patterns = measure_patterns(int(table.storage.numel()), N_KEYS)
        # each kernel against the ceiling of its own access pattern, measured above
        pattern_of = {"build": "insert_io", "search_hit": "search_io", "search_miss": "search_io"}
        for k, pat in pattern_of.items():
            kernels[k]["pattern_ceiling_us"] = patterns[pat + "_us"]
            kernels[k]["frac_of_pattern_ceiling"] = round(patterns[pat + "_us"] /
                                                          (avg_ms[k] * 1e3), 4)
        # a mixed batch is one launch of 2^16 ops: its floor is the one-slab insert (read, swap,
        # input and status streams) at that size, timed the same way (HIP events around one
        # launch); the bare read-then-swap pattern is reported beside it
        floor = measure_patterns(int(table.storage.numel()), MIX_BATCH)
        patterns["mixed_batch_size"] = floor
        kernels["mixed"]["pattern_ceiling_us"] = floor["insert_io_us"]
        kernels["mixed"]["frac_of_pattern_ceiling"] = round(floor["insert_io_us"] /
                                                            (avg_ms["mixed"] * 1e3), 4)
        kernels["mixed"]["frac_of_bare_load_cas"] = round(floor["load_cas_us"] /
                                                          (avg_ms["mixed"] * 1e3), 4)
        if dom in pattern_of:
            roof["secondary"] = {
                "bound": "atomic" if dom == "build" else "hbm",
                "pattern": pattern_of[dom], "ceiling_us": patterns[pattern_of[dom] + "_us"],
                "kernel_us": round(avg_ms[dom] * 1e3, 1),
                "frac": kernels[dom]["frac_of_pattern_ceiling"]}


    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (src.numel() * 4,
                                                                 src.numel() * 4))
        del src, dst

    config1 = sweep = None
    if not args.step_only:
        log("small phased configuration (2^16 keys, 2^12 buckets)")
        config1 = measure_config1()
        log("utilisation sweep")
        sweep = sweep_utilisation(wl, args.sweep_seeds if args.sweep else 1)

    sizes = None
    if not args.step_only and not args.no_sweep_sizes:
        log("size sweep")
        sizes = sweep_sizes()
    batch_sweep = None
    if not args.step_only and not args.no_sweep_batches:
        log("batch-size sweep")
        batch_sweep = sweep_batches()

    batched = None
    if not args.no_batched:
        del table
        torch.cuda.empty_cache()
        log("batched form")
        batched = run_batched()

    concurrent = None
    if not args.no_concurrent:
        torch.cuda.empty_cache()
        log("concurrent form")
        concurrent = run_concurrent()

    served = None
    if not args.no_served:
        torch.cuda.empty_cache()
        log("served form")
        served = run_served()

    cpu = cpu_part = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(wl, batches, B)
        log("cpu baseline (oracle, bucket-partitioned)")
        cpu_part = cpu_partitioned(wl, batches, B)

    out = {
        "metric": "M ops/s build/search/mixed at 2^22 keys vs HBM peak",
        "value": round(value, 2),
        "unit": "M ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "slab hash step: reset + bulk build 2^22 uniform uint32 keys + 2^22 "
                        "all-hit + 2^22 all-miss searches + 16 concurrent Gamma1 batches of 2^16",
            "keys": N_KEYS, "num_buckets": B, "target_utilisation": args.util,
            "achieved_utilisation": round(util, 4), "pool_slabs": pool,
            "mixed_batches": MIX_BATCHES, "mixed_batch_ops": MIX_BATCH,
            "ops_per_step": ops_step, "slabs_per_hit": round(v_hit, 4),
            "slabs_per_miss": round(v_miss, 4),
        },
        "kernels": kernels,
        "graph_steps": graph_steps,
        "build_counters": build_counters,
        "roofline": roof,
        "access_patterns": patterns,
        "flush": flush,
        "allocator": allocator,
        "duplicates": duplicates,
        "keys_only": keys_only,
        "hbm_resident": hbm,
        "cpu_baseline": cpu,
        "cpu_partitioned": cpu_part,
    }
    if config1 is not None:
        out["config_small_phased"] = config1
    if sweep is not None:
        out["sweep"] = sweep
    if sizes is not None:
        out["sweep_sizes"] = sizes
    if batch_sweep is not None:
        out["sweep_batches"] = batch_sweep
    if batched is not None:
        out["batched"] = batched
    if concurrent is not None:
        out["concurrent"] = concurrent
    if served is not None:
        out["served"] = served
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
