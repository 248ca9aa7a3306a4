"""CPU checks of the table-sizing model, the launch tuner's bookkeeping and the batched-workload
generator."""
import numpy as np
import pytest

from paper_1710_11246_amd import autotune as A
from paper_1710_11246_amd import workload as W


@pytest.mark.parametrize("target", [0.2, 0.4, 0.6, 0.7, 0.8])
def test_buckets_for_utilisation_is_largest(target):
    n = 1 << 20
    B = A.buckets_for_utilisation(n, target)
    assert A.utilisation(n, B) >= target
    assert A.utilisation(n, B + 1) < target or B + 1 > n


def test_pool_size_covers_oracle_use(oracle_mod):
    rng = W.SplitMix64(8)
    for n, target in [(1 << 14, 0.6), (1 << 17, 0.7), (1 << 16, 0.8), (3000, 0.9)]:
        keys = W.unique_keys(rng, n)
        B = A.buckets_for_utilisation(n, target)
        a, b = W.hash_params(rng, oracle_mod.PRIME)
        o = oracle_mod.Oracle(B, 31, a, b)
        o.replace(keys, keys)
        pool = A.pool_slabs_for(n, B)
        assert pool % 2048 == 0 and pool >= o.pool_used
        # the model's expected utilisation is close to the realised one
        assert abs(o.utilisation(8, 8) - A.utilisation(n, B)) < 0.02


def test_tune_launch_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("SLABHASH_TUNE_CACHE", str(tmp_path / "c.json"))
    cost = {(8, 16): 3.0, (16, 64): 1.0, (32, 32): 2.0}
    calls = []

    def run(w, c):
        calls.append((w, c))
        return cost[(w, c)]
    shape, t = A.tune_launch("mixed", 1 << 16, run, "dev", candidates=list(cost))
    assert shape == (16, 64) and len(calls) == 9
    shape2, _ = A.tune_launch("mixed", 1 << 16, run, "dev", candidates=list(cost))
    assert shape2 == (16, 64) and len(calls) == 9  # served from the cache


def test_sample_distinct_refuses_impossible_draws():
    with pytest.raises(ValueError):
        W.sample_distinct(W.SplitMix64(1), 5, 4)
    ok = np.array([True, False, True, False])
    assert sorted(W.sample_distinct(W.SplitMix64(1), 2, 4, ok).tolist()) == [0, 2]
    with pytest.raises(ValueError):
        W.sample_distinct(W.SplitMix64(1), 3, 4, ok)


@pytest.mark.parametrize("n_lo,len_hi", [(64, 2048), (4, 4096)])
def test_multi_rounds_generator_properties(n_lo, len_hi):
    mr = W.multi_rounds(seed=4, T=12, n_lo=n_lo, n_hi=4096, len_lo=1, len_hi=len_hi, rounds=4,
                        fractions=(0.3, 0.1, 0.3, 0.3), prime=4294967291)
    live = [dict(zip(k.tolist(), v.tolist())) for k, v in zip(mr.init_keys, mr.init_vals)]
    for t in range(12):
        assert np.unique(mr.init_keys[t]).size == mr.init_keys[t].size
    for r in range(4):
        ops, keys = mr.ops[r], mr.keys[r]
        assert mr.lengths[r].sum() == keys.size and mr.offsets[r][0] == 0
        for t in range(12):
            o = ops[mr.offsets[r][t]: mr.offsets[r][t] + mr.lengths[r][t]]
            k = keys[mr.offsets[r][t]: mr.offsets[r][t] + mr.lengths[r][t]]
            v = mr.vals[r][mr.offsets[r][t]: mr.offsets[r][t] + mr.lengths[r][t]]
            mut = k[o != 0]
            assert np.unique(mut).size == mut.size          # one mutation per key per batch
            n_live = len(live[t])
            assert int((o == W.OP_DELETE).sum()) <= n_live   # never more deletes than live keys
            for op, key, val in zip(o.tolist(), k.tolist(), v.tolist()):
                if op == W.OP_INSERT:
                    assert key not in live[t]               # inserts are fresh keys
                if op == W.OP_DELETE:
                    assert key in live[t]                   # deletes hit live keys
            for op, key, val in zip(o.tolist(), k.tolist(), v.tolist()):
                if op == W.OP_INSERT:
                    live[t][key] = val
                elif op == W.OP_DELETE:
                    del live[t][key]
    occ = [mr.init_keys[t].size + sum(int((mr.ops[r][mr.offsets[r][t]: mr.offsets[r][t] +
                                                      mr.lengths[r][t]] == 1).sum())
                                          for r in range(4)) for t in range(12)]
    assert list(mr.final_occupancy) == occ


def test_zipf_ranks_match_distribution():
    from scipy.stats import chisquare
    num, s, n = 50, 1.1, 400000
    r = W.zipf_ranks(W.SplitMix64(3), n, num, s)
    assert r.min() >= 1 and r.max() <= num
    w = np.arange(1, num + 1, dtype=float) ** -s
    expect = n * w / w.sum()
    obs = np.bincount(r, minlength=num + 1)[1:]
    assert chisquare(obs, expect).pvalue > 1e-4


def test_served_requests_properties():
    init = W.unique_keys(W.SplitMix64(1), 5000)
    sr = W.served_requests(7, init, 60, 1, 500, zipf_s=1.1)
    assert sr.lengths.sum() == sr.keys.size and (sr.lengths >= 1).all()
    mut = sr.ops != W.OP_SEARCH
    assert np.unique(sr.keys[mut]).size == int(mut.sum())   # each key mutated at most once
    ins = sr.keys[sr.ops == W.OP_INSERT]
    assert not np.isin(ins, init).any()
    assert np.isin(sr.keys[sr.ops == W.OP_DELETE], init).all()
    for i in range(60):
        a, n = sr.offsets[i], sr.lengths[i]
        assert sr.inserts[i] == int((sr.ops[a:a + n] == W.OP_INSERT).sum())
    d = W.served_requests(8, init, 40, 1, 100, zipf_s=None, disjoint=True)
    owner = {}
    for i in range(40):
        a, n = d.offsets[i], d.lengths[i]
        for k in d.keys[a:a + n][d.ops[a:a + n] != W.OP_INSERT].tolist():
            assert owner.setdefault(k, i) == i               # no initial key shared
    arr = W.poisson_arrivals(W.SplitMix64(2), 20000, 1e6)
    assert (np.diff(arr.astype(np.int64)) >= 0).all()
    assert abs(arr[-1] / 1e9 - 20000 / 1e6) < 0.05 * 20000 / 1e6


def test_distinct_keys_are_distinct_and_disjoint():
    a = W.distinct_keys(5, 0, 1 << 20)
    b = W.distinct_keys(5, 1 << 20, 1 << 18)
    assert np.unique(a).size == a.size and np.unique(b).size == b.size
    assert not np.isin(b, a).any() and (a != W.RESERVED_KEY).all()
    assert (W.distinct_keys(5, 7, 10) == a[7:17]).all()          # counter-based
    assert not (W.distinct_keys(6, 0, 1000) == a[:1000]).all()   # seeded
    # roughly uniform: the top 4 bits are balanced
    counts = np.bincount(a >> np.uint32(28), minlength=16)
    assert counts.min() > 0.9 * a.size / 16


def test_growth_checkpoints_properties():
    """Growth keys are distinct; every mixed batch inserts fresh keys, deletes distinct keys
    present at its start, searches present or never-inserted keys, in the paper's proportions."""
    g = W.growth_checkpoints(seed=5, total=6000, batch=512, checkpoints=[1000, 6000],
                             per_gamma=3, length=400, prime=4294967291)
    assert np.unique(g.keys).size == g.keys.size and (g.keys != W.RESERVED_KEY).all()
    present = set()
    grown = 0
    inserted = set(g.keys.tolist())
    for cp, per_cp in zip(g.checkpoints, g.mixed):
        present |= set(g.keys[grown:cp].tolist())
        grown = cp
        assert [name for name, _ in per_cp] == list(W.GAMMAS)
        for name, batches in per_cp:
            n_ins, n_del, n_hit, n_miss = W.gamma_counts(400, W.GAMMAS[name])
            for ops, keys, vals in batches:
                assert ops.size == keys.size == vals.size == 400
                assert (vals == W.value_of(keys)).all()
                ins, dels = keys[ops == W.OP_INSERT], keys[ops == W.OP_DELETE]
                srch = keys[ops == W.OP_SEARCH]
                assert ins.size == n_ins and dels.size == n_del and srch.size == n_hit + n_miss
                assert not (set(ins.tolist()) & inserted)          # fresh
                assert np.unique(dels).size == dels.size and set(dels.tolist()) <= present
                hit = np.array([k in present for k in srch.tolist()], dtype=bool)
                assert int(hit.sum()) == n_hit                      # the rest never inserted
                assert not (set(srch[~hit].tolist()) & inserted)
                inserted |= set(ins.tolist())
                present = (present - set(dels.tolist())) | set(ins.tolist())
    assert g.mixed_inserts == sum(W.gamma_counts(400, f)[0] for f in W.GAMMAS.values()) * 3 * 2


def test_served_mutator_lookup():
    rng = W.SplitMix64(9)
    init = W.unique_keys(rng, 5000)
    sr = W.served_requests(10, init, 60, 1, 300, zipf_s=1.1, absent_frac=0.1)
    want = dict(zip(sr.mut_keys.tolist(), sr.mut_req.tolist()))
    got = sr.mutator_of(sr.keys)
    assert got.tolist() == [want.get(k, -1) for k in sr.keys.tolist()]
    assert (sr.mutator_of(np.array([], np.uint32)).size == 0)
    # every mutating op's key maps to its own request
    req = np.searchsorted(sr.offsets, np.arange(sr.keys.size), side="right") - 1
    mut = sr.ops != W.OP_SEARCH
    assert (got[mut] == req[mut]).all()
