"""Interleavings of the operation kernel's protocol on the CPU (wave_model): several wavefronts
work on one small table at once and every slot read, swap, allocation and link is a separate
step of a random schedule. After each schedule, the structure and the results must be those a
linearizable table allows:
  - duplicates mode: a bucket holds no more slabs than with every insert ahead of every delete,
    and no fewer than with every delete ahead of every insert; the live multiset is exact;
  - unique keys: the slab count is exactly max(1, ceil(occupied / M)), empty slots form a suffix
    of the tail slab, the live map is exact, and inserts of one key report new exactly once;
  - always: no slab in two lists, every allocated slab in a list, every free slab empty.
Set WAVE_MODEL_SCHEDULES to run more schedules per case (the default keeps the suite short)."""
import math
import os

import pytest

import wave_model as WM

N = int(os.environ.get("WAVE_MODEL_SCHEDULES", "400"))


class SeqTable:
    """Sequential reference with the same slot rules: an array per bucket in list order,
    slab j holding entries [jM, (j+1)M)."""

    def __init__(self, B, M, dup):
        self.B, self.M, self.dup = B, M, dup
        self.b = [[] for _ in range(B)]

    def insert(self, k, v):
        L = self.b[WM.bucket_of(k, self.B)]
        if not self.dup:
            for i, x in enumerate(L):
                if isinstance(x, tuple) and x[0] == k:
                    L[i] = (k, v)
                    return 2
        for i, x in enumerate(L):
            if x is None:
                L[i] = (k, v)
                return 1
        L.append((k, v))
        return 1

    def delete(self, k):
        L = self.b[WM.bucket_of(k, self.B)]
        for i, x in enumerate(L):
            if isinstance(x, tuple) and x[0] == k:
                L[i] = None if self.dup else WM.TOMB
                return 1
        return 0

    def slabs(self):
        return [max(1, math.ceil(len(L) / self.M)) for L in self.b]


def load(mem, seq):
    """Write the sequential table's lists into the model's memory."""
    M = mem.M
    nxt_free = 0
    for b, L in enumerate(seq.b):
        u = b
        for j in range(0, max(1, math.ceil(len(L) / M))):
            if j:
                mem.allocated[nxt_free] = True
                mem.next[u] = nxt_free
                u = mem.B + nxt_free
                nxt_free += 1
            part = L[j * M:(j + 1) * M]
            mem.slots[u][:len(part)] = part


def chunks_of(ops, sizes):
    out, i = [], 0
    for s in sizes:
        out.append(ops[i:i + s])
        i += s
    assert i == len(ops)
    return out


def slab_counts(mem):
    return [len(c) for c in WM.lists(mem)]


def dup_mixed_case(M, sd, plant=None):
    B = 1
    base = [(k, 100 + k) for k in range(2 * M + 1)]
    ins = [(0, 7), (1, 8), (0, 9), (2, 10)]
    dels = [2 * M - 1, 2 * M - 2, M]
    srch = [2 * M]
    if True:
        rng_order = __import__("random").Random(sd)
        seq = SeqTable(B, M, True)
        for k, v in base:
            seq.insert(k, v)
        mem = WM.Memory(B, 16, M)
        load(mem, seq)
        ops = [WM.Op("insert", k, v) for k, v in ins] + [WM.Op("delete", k) for k in dels] + \
              [WM.Op("search", k) for k in srch]
        rng_order.shuffle(ops)
        WM.run_schedule(mem, chunks_of(ops, [3, 2, 3]), True, sd, plant)
        assert all(op.status == 1 for op in ops)
        assert all(op.found_val == 100 + op.key for op in ops if op.kind == "search")
        lo, hi = SeqTable(B, M, True), SeqTable(B, M, True)
        for t in (lo, hi):
            for k, v in base:
                t.insert(k, v)
        for k in dels:
            lo.delete(k)
        for k, v in ins:
            lo.insert(k, v)
            hi.insert(k, v)
        for k in dels:
            hi.delete(k)
        got = slab_counts(mem)
        assert lo.slabs()[0] <= got[0] <= hi.slabs()[0], (sd, got, lo.slabs(), hi.slabs())
        want = sorted((0, x[0], x[1]) for x in lo.b[0] if isinstance(x, tuple))
        assert WM.live_multiset(mem) == want


@pytest.mark.parametrize("M", [3, 4])
def test_duplicates_mixed_batch_bounds(M):
    """The GPU duplicates-mode test in miniature: copies of some keys inserted, single-copy keys
    deleted, untouched keys searched, all in one concurrent batch over three wavefronts."""
    for sd in range(N):
        dup_mixed_case(M, sd)


@pytest.mark.parametrize("M", [2, 4])
def test_duplicates_insert_only_build(M):
    """Inserts alone from an empty table never leave a hole: slabs = ceil(n / M) exactly."""
    n = 3 * M + 1
    for sd in range(N):
        mem = WM.Memory(2, 16, M)
        ops = [WM.Op("insert", 2 * (i % 3), i) for i in range(n)]  # copies, all in bucket 0
        WM.run_schedule(mem, chunks_of(ops, [M, M, n - 2 * M]), True, sd)
        assert all(op.status == 1 for op in ops)
        assert slab_counts(mem) == [math.ceil(n / M), 1]
        assert len(WM.live_multiset(mem)) == n


def unique_mixed_case(M, sd, plant=None, traces=None):
    B = 2
    base = [(k, 1000 + k) for k in range(4 * M)]
    fresh = [100, 102, 104, 101, 100]                      # key 100 twice
    reps = [(0, 5), (3, 6)]
    dels = [4, 7, 9]
    srch = [1, 2, 6, 55]
    if True:
        rng_order = __import__("random").Random(sd)
        seq = SeqTable(B, M, False)
        for k, v in base:
            seq.insert(k, v)
        mem = WM.Memory(B, 16, M)
        load(mem, seq)
        ops = [WM.Op("insert", k, 2000 + i) for i, k in enumerate(fresh)] + \
              [WM.Op("insert", k, v) for k, v in reps] + [WM.Op("delete", k) for k in dels] + \
              [WM.Op("search", k) for k in srch]
        rng_order.shuffle(ops)
        tr = WM.run_schedule(mem, chunks_of(ops, [4, 3, 3, len(ops) - 10]), False, sd, plant)
        if traces is not None:
            traces.extend(tr)
        st100 = sorted(op.status for op in ops if op.key == 100)
        assert st100 == [1, 2]
        for op in ops:
            if op.kind == "insert" and op.key != 100:
                assert op.status == (2 if op.key < 100 else 1)
            elif op.kind == "delete":
                assert op.status == 1
            elif op.kind == "search":
                assert op.status == (op.key < 4 * M and op.key not in dels)
        # the sequential table in one linearisation (the second insert of 100 replaces)
        for op in ops:
            if op.kind == "insert":
                seq.insert(op.key, op.val)
        for k in dels:
            seq.delete(k)
        live = WM.live_multiset(mem)
        v100 = [x[2] for x in live if x[1] == 100]
        assert len(v100) == 1 and v100[0] in (2000, 2004)
        want = sorted((b, x[0], x[1]) for b, L in enumerate(seq.b) for x in L
                      if isinstance(x, tuple) and x[0] != 100)
        assert [x for x in live if x[1] != 100] == want
        assert slab_counts(mem) == seq.slabs()
        # empty slots only as a suffix of each list's tail slab
        for chain in WM.lists(mem):
            flat = [x for u in chain for x in mem.slots[u]]
            first_empty = next((i for i, x in enumerate(flat) if x is None), len(flat))
            assert all(x is None for x in flat[first_empty:])
            assert first_empty > (len(chain) - 1) * M or len(chain) == 1


@pytest.mark.parametrize("M", [3, 4])
def test_unique_mixed_batch_exact(M):
    """Unique keys: fresh inserts (one key inserted twice), replaces, deletes and searches in one
    concurrent batch over four wavefronts on two buckets; the structure is exact."""
    for sd in range(N):
        unique_mixed_case(M, sd)


@pytest.mark.parametrize("plant,case", [("half_read", "dup"), ("double_fill", "dup"),
                                        ("half_read", "unique"), ("no_takeback", "unique")])
def test_planted_mistakes_are_caught(plant, case):
    """Each planted mistake in the model fails some schedule of these checks."""
    run = dup_mixed_case if case == "dup" else unique_mixed_case
    for sd in range(2000):
        try:
            run(4, sd, plant)
        except AssertionError:
            return
    pytest.fail("planted mistake %s not caught" % plant)


def growth_race_case(M, sd, traces=None):
    """One full slab and eight fresh keys inserted by four wavefronts at once: every one of
    them meets a full tail, so the lists grow under contention."""
    seq = SeqTable(1, M, False)
    for k in range(M):
        seq.insert(k, 1000 + k)
    mem = WM.Memory(1, 16, M)
    load(mem, seq)
    ops = [WM.Op("insert", 100 + i, 2000 + i) for i in range(8)]
    tr = WM.run_schedule(mem, chunks_of(ops, [2, 2, 2, 2]), False, sd)
    if traces is not None:
        traces.extend(tr)
    assert all(op.status == 1 for op in ops)
    for op in ops:
        seq.insert(op.key, op.val)
    assert slab_counts(mem) == seq.slabs()
    assert WM.live_multiset(mem) == sorted((0, x[0], x[1]) for x in seq.b[0])


@pytest.mark.parametrize("M", [2, 4])
def test_growth_race_exact(M):
    for sd in range(N):
        growth_race_case(M, sd)


def test_schedules_reach_the_rare_paths():
    """The schedules do reach the interleavings that matter: a new slab's slot 0 filled by
    another insert before the linking op's pair lands."""
    tr = []
    for sd in range(3000):
        growth_race_case(4, sd, traces=tr)
    kinds = {t[0] for t in tr}
    assert "link" in kinds and "slot 0 taken before the pair" in kinds
