"""GPU checks of the access-pattern microbenchmarks: the compare-and-swap patterns write exactly
where their documented addressing says, and the slab-read pattern leaves the buffer unchanged."""
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
