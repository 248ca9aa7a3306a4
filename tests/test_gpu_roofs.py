"""GPU checks of the access-pattern microbenchmarks: the compare-and-swap patterns write exactly
where their documented addressing says, the slab-read pattern leaves the buffer unchanged, and the
one-slab search and insert return and write what their documented addressing and vote give."""
import numpy as np
import pytest
import torch

from paper_1710_11246_amd import roofs as R

pytestmark = pytest.mark.gpu


def mix(x):
    x = np.asarray(x, dtype=np.uint64) & 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    R.lib()


def test_cas_pattern_addresses():
    slabs, n, seed = 4099, 20000, 12345
    buf = torch.full((slabs * 32,), -1, dtype=torch.int64, device="cuda")
    R.sh_roof_run(R.SH_ROOF_CAS, buf, n, 8, seed, depth=4)
    got = buf.cpu().numpy().view(np.uint64)
    i = np.arange(n, dtype=np.uint64)
    h = mix(i + seed)
    addr = ((h * slabs) >> 32) * 32 + (mix(h) & 31)
    written = np.flatnonzero(got != np.uint64(0xFFFFFFFFFFFFFFFF))
    assert set(written.tolist()) == set(addr.tolist())
    # each written word holds the index of an op that targets it
    first = {}
    for k, a in zip(i.tolist(), addr.tolist()):
        first.setdefault(a, set()).add(k)
    assert all(int(got[a]) in first[a] for a in written.tolist())


def test_load_cas_pattern_slabs():
    slabs, n, seed = 1031, 5001, 777
    buf = torch.full((slabs * 32,), -1, dtype=torch.int64, device="cuda")
    R.sh_roof_run(R.SH_ROOF_LOAD_CAS, buf, n, 4, seed, depth=16)
    got = buf.cpu().numpy().view(np.uint64).reshape(slabs, 32)
    ops = np.arange(n, dtype=np.uint64)
    slab_of = (mix(ops + seed) * slabs) >> 32
    full = got != np.uint64(0xFFFFFFFFFFFFFFFF)
    assert not full[:, 31].any()                       # only slots 0..30 are ever chosen
    s, w = np.nonzero(full)
    vals = got[s, w].astype(np.int64)
    assert (vals < n).all() and (slab_of[vals] == s).all()
    assert len(set(slab_of.tolist())) <= len(s) <= n
    # slots fill from the front of each slab
    for r in np.unique(s):
        row = full[r, :31]
        k = int(row.sum())
        assert row[:k].all() and not row[k:].any()


def test_slab_load_pattern_reads_only():
    slabs = 2048
    buf = torch.arange(slabs * 32, dtype=torch.int64, device="cuda")
    ref = buf.clone()
    R.sh_roof_run(R.SH_ROOF_SLAB_LOAD, buf, 1 << 16, 0, 3)
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)


@pytest.mark.parametrize("depth", [1, 16])
def test_one_slab_search_pattern(depth):
    """Keys planted in the slab their mix selects (some twice, the first copy deciding; some in
    slot 31, which is never voted on) and keys nowhere: values and flags as documented, the
    buffer unchanged, for a ragged number of ops."""
    slabs, n = 1031, 5001
    rng = np.random.default_rng(4242 + depth)
    words = rng.integers(0, 1 << 63, size=(slabs, 32), dtype=np.int64).view(np.uint64)
    keys = rng.choice(np.uint64(1) << np.uint64(32), size=n, replace=False).astype(np.uint64)
    keys = keys[keys != 0xFFFFFFFF]
    n = keys.size
    slab = (mix(keys) * slabs) >> 32
    # no stray match: clear every low word that equals one of the keys
    lo = words & np.uint64(0xFFFFFFFF)
    words[np.isin(lo, keys)] ^= np.uint64(1)
    want_v = np.full(n, 0xFFFFFFFF, np.uint64)
    want_f = np.zeros(n, np.uint8)
    for i in range(0, n, 3):                       # a third of the keys are planted
        s_, k = int(slab[i]), keys[i]
        slot = int(rng.integers(0, 32))
        hi = np.uint64(int(rng.integers(0, 1 << 32)))
        words[s_, slot] = (hi << np.uint64(32)) | k
        if slot < 31:
            want_v[i], want_f[i] = hi, 1
            if slot < 30 and i % 2 == 0:          # a later copy does not change the result
                words[s_, slot + 1] = (np.uint64(7) << np.uint64(32)) | k
    # a plant can overwrite an earlier one in the same slab: recompute from the final words
    for i in range(0, n, 3):
        row = words[int(slab[i])]
        hit = np.flatnonzero((row[:31] & np.uint64(0xFFFFFFFF)) == keys[i])
        want_v[i] = (row[hit[0]] >> np.uint64(32)) if hit.size else np.uint64(0xFFFFFFFF)
        want_f[i] = 1 if hit.size else 0
    buf = torch.from_numpy(words.view(np.int64).reshape(-1).copy()).cuda()
    ref = buf.clone()
    kd = torch.from_numpy(keys.astype(np.uint32).view(np.int32)).cuda()
    vals = torch.empty(n, dtype=torch.int32, device="cuda")
    found = torch.empty(n, dtype=torch.uint8, device="cuda")
    R.sh_roof_search(buf, kd, vals, found, 4, depth)
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)
    assert (found.cpu().numpy() == want_f).all() and int(want_f.sum()) > n // 4
    assert (vals.cpu().numpy().view(np.uint32) == want_v.astype(np.uint32)).all()


@pytest.mark.parametrize("depth", [1, 16])
def test_one_slab_insert_pattern(depth):
    """Distinct keys into a buffer of all ones: every pair lands in the slab its key's mix
    selects, slabs fill from slot 0 without gaps, and a status of 1 marks exactly the pairs that
    landed (an op whose slot another op took, or whose slab is full, loses: the pattern does
    not retry)."""
    slabs, n = 257, 9001
    rng = np.random.default_rng(77 + depth)
    keys = rng.choice(np.uint64(1) << np.uint64(32), size=n, replace=False).astype(np.uint64)
    keys = keys[keys != 0xFFFFFFFF]
    n = keys.size
    vals = rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
    buf = torch.full((slabs * 32,), -1, dtype=torch.int64, device="cuda")
    kd = torch.from_numpy(keys.astype(np.uint32).view(np.int32)).cuda()
    vd = torch.from_numpy(vals.astype(np.uint32).view(np.int32)).cuda()
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    R.sh_roof_insert(buf, kd, vd, st, 4, depth)
    torch.cuda.synchronize()
    got = buf.cpu().numpy().view(np.uint64).reshape(slabs, 32)
    status = st.cpu().numpy()
    slab_of = (mix(keys) * slabs) >> 32
    full = got != np.uint64(0xFFFFFFFFFFFFFFFF)
    assert not full[:, 31].any()
    for r in range(slabs):                          # no gaps
        k = int(full[r, :31].sum())
        assert full[r, :k].all() and not full[r, k:31].any()
    stored = got[full]
    want = (vals << np.uint64(32)) | keys
    won = status == 1
    assert set(stored.tolist()) == set(want[won].tolist()) and stored.size == int(won.sum())
    s_, _ = np.nonzero(full)
    pos = {int(x): i for i, x in enumerate(want.tolist())}
    assert all(slab_of[pos[int(x)]] == r for x, r in zip(stored.tolist(), s_.tolist()))
    per_slab = np.bincount(slab_of.astype(np.int64), minlength=slabs)
    filled = full[:, :31].sum(1)
    assert (filled <= np.minimum(per_slab, 31)).all() and ((filled > 0) == (per_slab > 0)).all()

