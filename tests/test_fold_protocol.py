"""CPU model of the synchronisation inside the TSQR quad fold (tsqr.hip, q_fold).

The fold's waves share a ring of R entries of reflectors in LDS, each with a ready
and a done counter.  Group k of 16 reflectors is built by wave k.  The entries come
in m = R / 2 sets of two: tile t of the fold uses set t mod m, and its group k the
entry k mod 2 of that set, so m tiles' chains can be in flight at once, each
alternating between its two entries.  The group that used an entry before (t, k) is
(t, k - 2) if the tile has that group, else the last group of tile t - m with the
parity of k (none for the first tiles).  Group (t, k) publishes the counts
256 (t np + k) + 1 ... in its entry; these only grow from one occupant of an entry
to the next.
If an earlier group used the entry, the builder first waits until that group has
published its first reflector and then until done, which that group's builder set
to minus the number of its slot users, is back at zero (every user has arrived).
It sets done to minus its own group's slot users (itself and the sequential
appliers), writes and publishes each reflector, stores the group's panel (V, T) to
global memory, waits for those stores and publishes one count more; then it
arrives at done.
The next SEQ waves (k + 1 .. k + SEQ, the next groups' builders) wait for each
reflector, apply it from the entry as it comes and arrive at done.  The waves
further right wait once, for the group's last count (or any later group's count
in the entry, since counts only grow) and apply the whole group as one block read
from the stored panel: they never touch the entry, so the entry is free for the
next group as soon as the builder and the sequential appliers are done.  A wave
that has built its group goes on to the next tile, so the tiles' chains overlap.

Here each wave is a generator that follows exactly that control flow, and a
seeded random scheduler interleaves them.  The model fails on a deadlock, on a
reflector read from an entry that has since been refilled by another group, on an
entry refilled while some wave still reads the previous group in it, and on a
block applied before its panel was stored.  The entry map itself is checked
against a brute-force replay of the groups in fold order.
"""
import random

import pytest

PW = 16
SEQ = 2   # waves k + 1 .. k + SEQ apply group k one reflector at a time


def ring_entry(t, k, k0, np_, R):
    """(entry, previous group's index t' np + k' or None) as q_fold computes them."""
    m = max(1, R // 2)
    e = (t % m) * 2 + (k & 1)
    if k - 2 >= k0:
        prev = t * np_ + k - 2
    elif t >= m:
        prev = (t - m) * np_ + k + 2 * ((np_ - 1 - k) // 2)
    else:
        prev = None
    return e, prev


def prev_first_count(tag, k, k0, np_, R):
    """The previous group's first count from group (t, k)'s own first count
    tag = 256 (t np + k) + 1, as q_fold forms it (0 for none)."""
    if k - 2 >= k0:
        return tag - 512
    back = max(1, R // 2) * np_ * 256
    if tag <= back:
        return 0
    return tag - back + ((np_ - 1 - k) >> 1) * 512


def wave_program(w, c, tiles, st, R, block=True, naive=False):
    """Wave w's accesses over the fold's tiles (tile t starts at column tiles[t])."""
    np_ = (c + PW - 1) // PW
    for t, j0 in enumerate(tiles):
        k0 = j0 // PW
        for k in range(k0, np_):
            jb, je = PW * k, min(PW * k + PW, c)
            gid = t * np_ + k
            half, prev = ring_entry(t, k, k0, np_, R)
            slot_users = 1 + (min(SEQ, np_ - 1 - k) if block else np_ - 1 - k)
            if w >= k:
                if w == k:
                    pf = prev_first_count(gid * 256 + 1, k, k0, np_, R)
                    assert pf == (0 if prev is None else prev * 256 + 1)
                    if pf:
                        # the entry's previous group: its builder has reset done, then
                        # every one of its slot users has arrived
                        while not naive and st["ready"][half] - pf < 0:
                            yield "wait"
                        while st["done"][half] < 0:
                            yield "wait"
                    st["done"][half] = -slot_users
                    yield "step"
                    st["users"][gid] = st["users"].get(gid, 0) + 1
                    for j in range(jb, je):
                        old = st["owner"][half]
                        if old is not None and old != gid:
                            assert st["users"].get(old, 0) == 0, ("ring entry refilled while in use", w, k)
                        st["owner"][half] = gid
                        st["ready"][half] = gid * 256 + (j - jb + 1)
                        yield "step"
                    # the group's panel (V, T) to global memory, waited for, then the
                    # count the block appliers wait for
                    st["panel"][gid] = True
                    yield "step"
                    st["ready"][half] = gid * 256 + (je - jb + 1)
                    yield "step"
                    st["users"][gid] -= 1
                    st["done"][half] += 1
                elif w <= k + SEQ or not block:
                    st["users"][gid] = st["users"].get(gid, 0) + 1
                    for j in range(jb, je):
                        while st["ready"][half] - (gid * 256 + (j - jb + 1)) < 0:
                            yield "wait"
                        assert st["owner"][half] == gid, ("stale reflector", w, k)
                        yield "step"
                    st["users"][gid] -= 1
                    st["done"][half] += 1
                else:
                    while st["ready"][half] - (gid * 256 + (je - jb + 1)) < 0:
                        yield "wait"
                    assert st["panel"].get(gid), ("block applied before its panel was stored", w, k)
                    yield "step"


def run(c, tiles, seed, R=2, block=True, naive=False):
    rnd = random.Random(seed)
    np_ = (c + PW - 1) // PW
    st = {"ready": [0] * R, "done": [0] * R, "owner": [None] * R, "users": {}, "panel": {}}
    progs = {w: wave_program(w, c, tiles, st, R, block, naive) for w in range(np_)}
    alive = set(progs)
    idle = 0
    while alive:
        w = rnd.choice(sorted(alive))
        try:
            r = next(progs[w])
        except StopIteration:
            alive.discard(w)
            continue
        idle = idle + 1 if r == "wait" else 0
        if idle > 20000:
            return False
    return True


def leaf_tiles(n):
    return [0] * n


def tree_tiles(c):
    return [64 * t for t in range((c + 63) // 64)]   # one tree combine: tile t starts at 64 t


@pytest.mark.parametrize("c", [1, 15, 16, 17, 26, 32, 40, 64, 100, 184, 200, 220, 256])
@pytest.mark.parametrize("R", [2, 3, 4, 5, 6, 8, 9, 12])
def test_ring_entry_map_is_the_previous_occupant(c, R):
    """The closed form of the previous occupant equals a replay of the fold's groups."""
    np_ = (c + PW - 1) // PW
    m = max(1, R // 2)
    for tiles in (leaf_tiles(9), tree_tiles(c)):
        last = {}
        for t, j0 in enumerate(tiles):
            for k in range(j0 // PW, np_):
                e, prev = ring_entry(t, k, j0 // PW, np_, R)
                assert 0 <= e < 2 * m <= max(2, R)
                assert prev == last.get(e), (c, R, t, k)
                want = 0 if prev is None else prev * 256 + 1
                assert prev_first_count((t * np_ + k) * 256 + 1, k, j0 // PW, np_, R) == want
                last[e] = t * np_ + k


@pytest.mark.parametrize("c", [1, 15, 16, 17, 26, 32, 40, 64, 100, 184, 200, 220, 256])
@pytest.mark.parametrize("R", [2, 3, 5, 6, 7, 8, 10, 12])
@pytest.mark.parametrize("block", [False, True])
def test_fold_protocol_leaf_and_tree(c, R, block):
    for seed in range(12):
        assert run(c, leaf_tiles(7), seed, R, block), ("deadlock", c, R, "leaf", seed)
        assert run(c, tree_tiles(c), seed, R, block), ("deadlock", c, R, "tree", seed)


def test_fold_protocol_needs_the_previous_group_published():
    """Without the wait for the entry's previous group to have started, a builder can
    see done = 0 left from the group before it (whose users have all arrived) while
    the previous group has not been built yet, and refill the entry under it."""
    bad = 0
    for seed in range(40):
        try:
            ok = run(220, leaf_tiles(6), seed, 6, True, naive=True)
        except AssertionError:
            ok = False
        bad += not ok
    assert bad > 0


def test_fold_protocol_detects_a_shared_counter():
    """The model itself catches the earlier design, in which the producers of all
    groups published into one counter with plain stores: two producers of
    consecutive groups can then run at once and move the counter back."""

    def shared_counter_program(w, c, tiles, st):
        np_ = (c + PW - 1) // PW
        groups = published = 0
        owed = [0, 0]
        for j0 in tiles:
            for k in range(j0 // PW, np_):
                jb, je = PW * k, min(PW * k + PW, c)
                half = groups & 1
                if w == k:
                    while st["done"][half] - owed[half] < 0:
                        yield "wait"
                    for j in range(jb, je):
                        st["ready"] = published + (j - j0 + 1)
                        yield "step"
                elif w > k:
                    for j in range(jb, je):
                        while st["ready"] - (published + (j - j0 + 1)) < 0:
                            yield "wait"
                        yield "step"
                    st["done"][half] += 1
                owed[half] += np_ - 1 - k
                groups += 1
            published += c - j0

    found = False
    for seed in range(40):
        rnd = random.Random(seed)
        st = {"ready": 0, "done": [0, 0]}
        progs = {w: shared_counter_program(w, 26, [0, 0, 0], st) for w in range(2)}
        alive, idle = set(progs), 0
        while alive and idle <= 20000:
            w = rnd.choice(sorted(alive))
            try:
                r = next(progs[w])
            except StopIteration:
                alive.discard(w)
                continue
            idle = idle + 1 if r == "wait" else 0
        found |= bool(alive)
    assert found
