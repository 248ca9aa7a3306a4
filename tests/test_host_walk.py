"""The host-side storage reader used by the GPU parity tests (CPU): on storage laid out by hand,
it follows the lists, counts live and deleted slots, and names each broken invariant."""
import numpy as np
import pytest
import torch

import host_walk as HW

E64 = 0xFFFFFFFFFFFFFFFF


class FakeParams:
    def __init__(self, B, P):
        self.num_buckets, self.pool_slabs = B, P


class FakeTable:
    """The storage of a table with B base slabs and P pool slabs, all empty and free."""

    def __init__(self, B, P):
        self.params = FakeParams(B, P)
        self.raw = np.zeros(HW.HEADER + (B + P) * HW.SLAB + (P // HW.BLOCK) * 256, np.uint8)
        self.base()[:] = E64
        self.pool()[:] = E64

    def base(self):
        B = self.params.num_buckets
        return self.raw[HW.HEADER:HW.HEADER + B * 256].view(np.uint64).reshape(B, 32)

    def pool(self):
        B, P = self.params.num_buckets, self.params.pool_slabs
        o = HW.HEADER + B * 256
        return self.raw[o:o + P * 256].view(np.uint64).reshape(P, 32)

    def bitmap(self):
        B, P = self.params.num_buckets, self.params.pool_slabs
        o = HW.HEADER + (B + P) * 256
        return self.raw[o:].view(np.uint32).reshape(-1, 64)

    def link(self, slab_row, nxt):
        slab_row[31] = np.uint64((int(nxt) << 32) | 0xFFFFFFFF)

    def alloc(self, i):
        self.bitmap()[i // 2048, (i // 32) % 64] |= np.uint32(1 << (i % 32))

    @property
    def storage(self):
        return torch.from_numpy(self.raw)


def pair(k, v):
    return np.uint64((v << 32) | k)


def sample():
    """Bucket 0: base full, then pool slab 5 with 3 pairs, one a tombstone. Bucket 1: base with
    two pairs. Bucket 2: empty."""
    t = FakeTable(3, 4096)
    for s in range(31):
        t.base()[0, s] = pair(100 + s, s)
    t.link(t.base()[0], 5)
    t.alloc(5)
    t.pool()[5, 0] = pair(7, 1)
    t.pool()[5, 1] = np.uint64(0x00000000FFFFFFFF)  # tombstone
    t.pool()[5, 2] = pair(9, 0xFFFFFFFF)           # a live pair whose value is all ones
    t.base()[1, 0] = pair(1, 2)
    t.base()[1, 1] = pair(3, 4)
    return t


def test_counts_of_a_well_formed_table():
    live, tomb, slabs = HW.check_structure(sample())
    assert live.tolist() == [33, 2, 0]
    assert tomb.tolist() == [1, 0, 0]
    assert slabs.tolist() == [2, 1, 1]


@pytest.mark.parametrize("plant,msg", [
    ("outside", "1:"), ("cycle", "1:"), ("twice", "2:"), ("unmarked", "3:"), ("leak", "4:"),
    ("dirty", "5:")])
def test_each_broken_invariant_is_named(plant, msg):
    t = sample()
    if plant == "outside":
        t.link(t.pool()[5], 4096)
    elif plant == "cycle":
        t.link(t.pool()[5], 5)
    elif plant == "twice":
        t.link(t.base()[1], 5)
    elif plant == "unmarked":
        t.bitmap()[:] = 0
    elif plant == "leak":
        t.alloc(6)
    elif plant == "dirty":
        t.pool()[100, 3] = pair(1, 1)
    with pytest.raises(AssertionError, match=msg):
        HW.check_structure(t)


def test_key_only_counts():
    t = FakeTable(1, 2048)
    t.base()[0, 0] = np.uint64((5 << 32) | 4)                  # two keys
    t.base()[0, 1] = np.uint64((0xFFFFFFFF << 32) | 0xFFFFFFFE)  # a deleted key, then empty
    live, tomb, slabs = HW.check_structure(t, keys_only=True)
    assert live.tolist() == [2] and tomb.tolist() == [1] and slabs.tolist() == [1]


def test_super_block_size_matches_the_library():
    """The reader's super-block geometry is the one the header states, and the library's byte
    count for S slabs (sh_super_block_bytes) gives back S slabs."""
    from paper_1710_11246_amd import slabhash as S
    for slabs in (2048, 4096, 3 * 2048, 1 << 20):
        nb = S.sh_super_block_bytes(slabs)
        assert nb == slabs * 256 + slabs // 2048 * 256
        assert HW.super_slabs(nb) == slabs
        assert HW.super_slabs(nb - 1) == slabs - 2048
    assert S.sh_super_block_bytes(0) == 0 and S.sh_super_block_bytes(2047) == 0
    assert S.sh_super_block_bytes((1 << 27) - 2048) > 0 and S.sh_super_block_bytes(1 << 27) == 0


def test_lists_through_super_blocks():
    """A list whose second slab is in super block 1 (address 1 << 27 | 3) and third in super
    block 2 is followed, counted and checked like any other."""
    t = sample()
    s1 = np.zeros(HW.SLAB * 2048 + 256, np.uint8)
    s2 = np.zeros(HW.SLAB * 2048 + 256, np.uint8)
    p1 = s1[:2048 * 256].view(np.uint64).reshape(2048, 32)
    p2 = s2[:2048 * 256].view(np.uint64).reshape(2048, 32)
    p1[:] = E64
    p2[:] = E64
    b1 = s1[2048 * 256:].view(np.uint32)
    b2 = s2[2048 * 256:].view(np.uint32)
    t.link(t.base()[1], (1 << 27) | 3)
    p1[3, 0] = pair(50, 5)
    t.link(p1[3], (2 << 27) | 40)
    p2[40, 0] = pair(60, 6)
    b1[0] |= np.uint32(1 << 3)
    b2[1] |= np.uint32(1 << 8)
    supers = [torch.from_numpy(s1), torch.from_numpy(s2)]
    live, tomb, slabs = HW.check_structure(t, supers=supers)
    assert live.tolist() == [33, 4, 0] and slabs.tolist() == [2, 3, 1]
    b2[1] = 0
    with pytest.raises(AssertionError, match="3:"):
        HW.check_structure(t, supers=supers)
