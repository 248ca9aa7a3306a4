"""A step-by-step CPU model of the operation kernel's protocol, for searching interleavings.

Each wavefront takes a chunk of ops and works on it in rounds, as the HIP kernel does:
  read    every unfinished op's cursor slab is read slot by slot; each slot read (and the read
          of the next index) is a separate step, so a slab is never assumed to be read at one
          instant (on the GPU it is two 128-byte lines, each possibly split further);
  decide  each op's outcome from its own snapshot: found / swap into a slot / move to the next
          slab / end of list / new slab needed ("Search", "Insertion", "Deletion" and the
          replace, delete and search parts of the pseudocode figure);
  act     every swap is a compare-and-swap step; the ops' swaps of one round run in any order.
          A unique-key insert that loses its empty slot walks on with the occupants its swaps
          return; a duplicates-mode insert tries the other empty slots its snapshot showed;
          any other lost swap re-reads the slab next round;
  grow    the first op (in lane order) that found a full tail takes a free pool slab (a step)
          and links it with a swap on the tail's next index (the others re-read next round); with unique keys a swap of the pair into slot 0 of
          the new slab is issued together with the link, the two landing in either order; a
          lost link takes the pair back out, frees the slab and follows the winner's slab.
A scheduler interleaves the steps of all wavefronts at random. The model shares nothing with
the HIP code; it restates the protocol the kernel implements.

Slots hold None (empty), TOMB (a deleted slot with unique keys) or a (key, value) pair."""
import random

TOMB = "T"


class Memory:
    def __init__(self, B, P, M):
        self.B, self.P, self.M = B, P, M
        # unified slab index: u < B is base slab u, u >= B is pool slab u - B
        self.slots = [[None] * M for _ in range(B + P)]
        self.next = [None] * (B + P)
        self.allocated = [False] * P

    def cas_slot(self, u, s, expect, desired):
        old = self.slots[u][s]
        if old == expect:
            self.slots[u][s] = desired
        return old

    def cas_next(self, u, expect, desired):
        old = self.next[u]
        if old == expect:
            self.next[u] = desired
        return old


def bucket_of(key, B):
    return key % B


class Op:
    def __init__(self, kind, key, val=None):
        self.kind, self.key, self.val = kind, key, val
        self.status = 0
        self.found_val = None
        self.cursor = None  # None: the bucket's base slab; else a pool slab index


def wavefront(mem, ops, dup, rng, trace, plant=None):
    """Generator: one wavefront working on its chunk; yields before every shared-memory step.
    `plant` names a deliberate mistake, for the tests that show each is caught:
      "half_read"    an insert decides from the first half of its slab only (the rest taken
                     as full), as if one cache line of the slab had been read;
      "double_fill"  a duplicates-mode insert that wins its slot also fills the next empty one;
      "no_takeback"  a lost link frees its slab with the prefilled pair still in it."""
    M, B = mem.M, mem.B
    todo = [op for op in ops]
    while todo:
        # ---- read: every slot of every pending op's slab, in any order ----
        snaps = {}
        reads = []
        for op in todo:
            u = bucket_of(op.key, B) if op.cursor is None else B + op.cursor
            snaps[id(op)] = (u, [None] * M, [None])
            reads += [(op, s) for s in range(M)] + [(op, "next")]
        rng.shuffle(reads)
        for op, s in reads:
            yield
            u, sl, nx = snaps[id(op)]
            if s == "next":
                nx[0] = mem.next[u]
            else:
                sl[s] = mem.slots[u][s]
        # ---- decide ----
        acts = []
        grow = []
        finished = []
        for op in todo:
            u, sl, nx = snaps[id(op)]
            k = op.key
            match = [s for s in range(M) if isinstance(sl[s], tuple) and sl[s][0] == k]
            empty = [s for s in range(M) if sl[s] is None]
            if plant == "half_read" and op.kind == "insert":
                empty = [s for s in empty if s < (M + 1) // 2]
            if op.kind == "search":
                if match:
                    op.status, op.found_val = 1, sl[match[0]][1]
                    finished.append(op)
                elif nx[0] is not None:
                    op.cursor = nx[0]
                else:
                    finished.append(op)
            elif op.kind == "delete":
                if match:
                    acts.append((op, "del", u, match[0], sl[match[0]], empty))
                elif nx[0] is not None:
                    op.cursor = nx[0]
                else:
                    finished.append(op)
            else:  # insert
                if match and not dup:
                    acts.append((op, "rep", u, match[0], sl[match[0]], empty))
                elif empty:
                    acts.append((op, "ins", u, empty[0], None, empty))
                elif nx[0] is not None:
                    op.cursor = nx[0]
                else:
                    grow.append((op, u))
        # ---- act: each op's swaps as its own sequence, the ops interleaved in any order ----
        def act(op, what, u, s, seen, empty):
            k, v = op.key, op.val
            if what == "del":
                yield
                old = mem.cas_slot(u, s, seen, None if dup else TOMB)
                if old == seen:
                    op.status = 1
                    finished.append(op)
                return
            if what == "rep":
                yield
                old = mem.cas_slot(u, s, seen, (k, v))
                if old == seen:
                    op.status = 2
                    finished.append(op)
                return
            yield
            old = mem.cas_slot(u, s, None, (k, v))
            if old is None:
                op.status = 1
                finished.append(op)
                if plant == "double_fill" and dup:
                    for s2 in [e for e in empty if e > s]:
                        yield
                        if mem.cas_slot(u, s2, None, (k, v)) is None:
                            break
                return
            if dup:
                for s2 in [e for e in empty if e > s]:
                    yield
                    if mem.cas_slot(u, s2, None, (k, v)) is None:
                        op.status = 1
                        finished.append(op)
                        return
                return
            while True:
                if isinstance(old, tuple) and old[0] == k:
                    yield
                    o2 = mem.cas_slot(u, s, old, (k, v))
                    if o2 == old:
                        op.status = 2
                        finished.append(op)
                    return
                s += 1
                if s >= M:
                    return
                yield
                old = mem.cas_slot(u, s, None, (k, v))
                if old is None:
                    op.status = 1
                    finished.append(op)
                    return

        gens = [act(*a) for a in acts]
        while gens:
            g = rng.choice(gens)
            try:
                next(g)
                yield
            except StopIteration:
                gens.remove(g)
        done_ids = {id(op) for op in finished}
        todo = [op for op in todo if id(op) not in done_ids]
        # ---- grow: every op at a full tail takes a free pool slab (claimed together with the
        # swaps above: a step of its own), then links it with a swap on its tail's next index.
        # With unique keys the pair goes into slot 0 of the new slab with a swap issued
        # together with the link, so the two land in either order: a link that lands first
        # makes the slab public, and another insert may fill slot 0 before the pair does (this
        # op then takes the next round on the new slab). A lost link leaves the slab private:
        # its pair is taken out and the slab freed, and the op follows the winner's slab. ----
        def link(op, u, idx):
            fresh = mem.B + idx
            put = None
            order = ["prefill", "link"] if not dup else ["link"]
            rng.shuffle(order)
            lold = "pending"
            for step in order:
                yield
                if step == "prefill":
                    put = mem.cas_slot(fresh, 0, None, (op.key, op.val))
                else:
                    lold = mem.cas_next(u, None, idx)
            if lold is None:
                trace.append(("link", u, idx))
                if not dup and put is None:
                    op.status = 1
                    finished.append(op)
                else:
                    if not dup:
                        trace.append(("slot 0 taken before the pair", u, idx))
                    op.cursor = idx
            else:
                if not dup and put is None and plant != "no_takeback":
                    yield
                    assert mem.cas_slot(fresh, 0, (op.key, op.val), None) == (op.key, op.val)
                yield
                mem.allocated[idx] = False
                op.cursor = lold

        finished = []
        gens = []
        # one op per round and wavefront grows a list; the others re-read their tail next round
        for op, u in grow[:1]:
            yield
            free = [i for i in range(mem.P) if not mem.allocated[i]]
            if not free:
                op.status = 0
                todo.remove(op)
                trace.append(("pool exhausted", op.key))
                continue
            idx = rng.choice(free)
            assert mem.slots[mem.B + idx] == [None] * M and mem.next[mem.B + idx] is None, \
                "an allocated slab is not empty"
            mem.allocated[idx] = True
            gens.append(link(op, u, idx))
        while gens:
            g = rng.choice(gens)
            try:
                next(g)
                yield
            except StopIteration:
                gens.remove(g)
        done_ids = {id(op) for op in finished}
        todo = [op for op in todo if id(op) not in done_ids]


def run_schedule(mem, chunks, dup, seed, plant=None):
    """Run one random interleaving of the wavefronts (one per chunk) to the end."""
    rng = random.Random(seed)
    trace = []
    waves = [wavefront(mem, ch, dup, random.Random(rng.random()), trace, plant)
             for ch in chunks]
    steps = 0
    while waves:
        w = rng.choice(waves)
        try:
            next(w)
        except StopIteration:
            waves.remove(w)
        steps += 1
        assert steps < 10 ** 6, "a schedule did not finish"
    return trace


def lists(mem):
    """Per bucket, the slab indices of its list (unified), checking the structure: every next
    index is an allocated pool slab referenced once; every allocated slab is in a list; free
    slabs are empty."""
    seen = set()
    out = []
    for b in range(mem.B):
        chain = [b]
        u = b
        while mem.next[u] is not None:
            i = mem.next[u]
            assert 0 <= i < mem.P and mem.allocated[i], "link to a free or bad slab"
            assert i not in seen, "a slab is in two lists"
            seen.add(i)
            u = mem.B + i
            chain.append(u)
        out.append(chain)
    for i in range(mem.P):
        if mem.allocated[i]:
            assert i in seen, "an allocated slab is in no list"
        else:
            assert mem.slots[mem.B + i] == [None] * mem.M and mem.next[mem.B + i] is None, \
                "a free slab is not empty"
    return out


def live_multiset(mem):
    out = []
    for b, chain in enumerate(lists(mem)):
        for u in chain:
            for x in mem.slots[u]:
                if isinstance(x, tuple):
                    out.append((b, x[0], x[1]))
    return sorted(out)
