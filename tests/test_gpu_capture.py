"""GPU tests of stream capture (sh_capture_begin / sh_capture_end): a captured sequence of table
calls replayed several times, with eager work and synchronisations between the replays, gives
every time what the same calls give when run eagerly."""
import sys

import numpy as np
import pytest
import torch

from paper_1710_11246_amd import slabhash as S
from paper_1710_11246_amd import workload as W

from test_gpu_parity import assert_same_table

pytestmark = pytest.mark.gpu
M = S.SH_SLAB_PAIRS


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def test_captured_pass_replays(oracle_mod):
    """reset, build, a hit and a miss search and two mixed batches, captured once and replayed
    three times; each replay's outputs and final table equal the eager run's and the oracle's."""
    say("case: captured build/search/mixed pass")
    rng = W.SplitMix64(1201)
    a, b = W.hash_params(rng, S.SH_HASH_PRIME)
    n, B = 1 << 16, 3001
    keys = W.unique_keys(rng, 3 * n)
    base, fresh, absent = keys[:n], keys[n:2 * n], keys[2 * n:]
    vals = W.value_of(base)
    batches = []
    present = base.copy()
    for i in range(2):
        ni, nd, nh, nm = W.gamma_counts(1 << 12, (0.2, 0.2, 0.3, 0.3))
        ops, bk, bv = W.mixed_batch(rng, present, fresh[i * ni:(i + 1) * ni], absent,
                                    ni, nd, nh, nm)
        batches.append((ops, bk, bv))
        present = np.concatenate([present[~np.isin(present, bk[ops == 2])], bk[ops == 1]])
    t = S.SlabHash(B, S.pool_slabs_bound(2 * n), a, b)
    dk, dv = S.to_dev(base), S.to_dev(vals)
    qh, qm = S.to_dev(base[::-1].copy()), S.to_dev(absent[:n])
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    vo = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(2)]
    fo = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in range(2)]
    mb = [(S.to_dev(o), S.to_dev(k), S.to_dev(v)) for o, k, v in batches]
    mo = [(torch.empty(k.size, dtype=torch.int32, device="cuda"),
           torch.empty(k.size, dtype=torch.uint8, device="cuda")) for _, k, _ in batches]
    s = torch.cuda.Stream()

    def one_pass():
        S.sh_reset(t.handle, s)
        S.sh_build(t.handle, dk, dv, st, s)
        S.sh_search(t.handle, qh, vo[0], fo[0], s)
        S.sh_search(t.handle, qm, vo[1], fo[1], s)
        for (o, k, v), (x, y) in zip(mb, mo):
            S.sh_mixed(t.handle, o, k, v, x, y, s)

    def outputs():
        torch.cuda.synchronize()
        return [st.clone(), vo[0].clone(), fo[0].clone(), fo[1].clone()] + \
               [x.clone() for x, _ in mo] + [y.clone() for _, y in mo]

    one_pass()
    eager = outputs()
    eager_dump = t.dump()[:4]
    S.sh_capture_begin(s)
    try:
        one_pass()
    finally:
        g = S.sh_capture_end(s)
    try:
        o = oracle_mod.Oracle(B, M, a, b)
        o.replace(base, vals)
        ovh, ofh, _ = o.search(base[::-1].copy())
        for rep in range(3):
            # eager work between replays: searches on the default stream
            S.sh_search(t.handle, qm, vo[1], fo[1])
            vo[0].fill_(0)
            torch.cuda.synchronize()
            S.sh_graph_launch(g, s)
            got = outputs()
            assert bool((got[0] == 1).all())
            assert (S.to_host_u32(got[1]) == ovh).all() and (got[2].cpu().numpy() == ofh).all()
            assert not got[3].cpu().numpy().any()
            for i, (op, k, _) in enumerate(batches):
                # mutations and searches of keys the batch does not mutate have unique results;
                # a search of a mutated key may see either state
                unique = (op != 0) | ~np.isin(k, k[op != 0])
                u = torch.from_numpy(unique).cuda()
                assert bool(((got[6 + i] == eager[6 + i]) | ~u).all())
                assert bool(((got[4 + i] == eager[4 + i]) | ~u).all())
            d = t.dump()
            for x, y in zip(d[:4], eager_dump):
                assert (x == y).all()
    finally:
        S.sh_graph_destroy(g)
    oo = oracle_mod.Oracle(B, M, a, b)
    oo.replace(base, vals)
    for op, k, v in batches:
        oo.mixed(op, k, v)
    assert_same_table(t, oo)


def test_capture_rejects_the_null_stream():
    with pytest.raises(S.SlabHashError):
        S.sh_capture_begin(0)
