"""CPU model of the synchronisation inside the TSQR quad fold (tsqr.hip, q_fold).

The fold's waves share a ring of R group slots of reflectors in LDS, each with a
ready and a done counter.  Group k of 16 reflectors is built by wave k.  If an
earlier group G' = G - R used the slot, the builder first waits until G' has
published its first reflector (ready >= 256 G' + 1) and then until done, which
G''s builder set to minus the number of G''s slot users, is back at zero (every
user has arrived).  It sets done to minus its own group's slot users (itself and
the sequential appliers), writes and publishes each reflector (the slot's ready
counter takes 256 G + slot + 1 for the workgroup's G-th group), stores the
group's panel (V, T) to global memory, waits for those stores and publishes one
count more; then it arrives at done.
The next SEQ waves (k + 1 .. k + SEQ, the next groups' builders) wait for each
reflector, apply it from the slot as it comes and arrive at done.  The waves
further right wait once, for the group's last count (or any later group's count
in the slot, since counts only grow) and apply the whole group as one block read
from the stored panel: they never touch the slot, so the slot is free for the
next group as soon as the builder and the sequential appliers are done.  A wave
that has built its group goes on to the next tile, so the tiles' chains overlap.

Here each wave is a generator that follows exactly that control flow, and a
seeded random scheduler interleaves them.  The model fails on a deadlock, on a
reflector read from a slot that has since been refilled by another group, on a
slot refilled while some wave still reads the previous group in it, and on a
block applied before its panel was stored.
"""
import random

import pytest

PW = 16
SEQ = 2   # waves k + 1 .. k + SEQ apply group k one reflector at a time


def wave_program(w, c, tiles, st, R, block=True, naive=False):
    """Wave w's accesses over `tiles` tiles of leaf folds (starts) or tree folds."""
    np_ = (c + PW - 1) // PW
    groups = 0
    for j0 in tiles:
        for k in range(j0 // PW, np_):
            jb, je = PW * k, min(PW * k + PW, c)
            half = groups % R
            slot_users = 1 + (min(SEQ, np_ - 1 - k) if block else np_ - 1 - k)
            if w >= k:
                if w == k:
                    if groups >= R:
                        # the slot's previous group: its builder has reset done, then
                        # every one of its slot users has arrived
                        while not naive and st["ready"][half] - ((groups - R) * 256 + 1) < 0:
                            yield "wait"
                        while st["done"][half] < 0:
                            yield "wait"
                    st["done"][half] = -slot_users
                    yield "step"
                    st["users"][groups] = st["users"].get(groups, 0) + 1
                    for j in range(jb, je):
                        prev = st["owner"][half]
                        if prev is not None and prev != groups:
                            assert st["users"].get(prev, 0) == 0, ("ring half refilled while in use", w, k)
                        st["owner"][half] = groups
                        st["ready"][half] = groups * 256 + (j - jb + 1)
                        yield "step"
                    # the group's panel (V, T) to global memory, waited for, then the
                    # count the block appliers wait for
                    st["panel"][groups] = True
                    yield "step"
                    st["ready"][half] = groups * 256 + (je - jb + 1)
                    yield "step"
                    st["users"][groups] -= 1
                    st["done"][half] += 1
                elif w <= k + SEQ or not block:
                    st["users"][groups] = st["users"].get(groups, 0) + 1
                    for j in range(jb, je):
                        while st["ready"][half] - (groups * 256 + (j - jb + 1)) < 0:
                            yield "wait"
                        assert st["owner"][half] == groups, ("stale reflector", w, k)
                        yield "step"
                    st["users"][groups] -= 1
                    st["done"][half] += 1
                else:
                    while st["ready"][half] - (groups * 256 + (je - jb + 1)) < 0:
                        yield "wait"
                    assert st["panel"].get(groups), ("block applied before its panel was stored", w, k)
                    yield "step"
            groups += 1


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


@pytest.mark.parametrize("c", [1, 15, 16, 17, 26, 32, 40, 64, 100, 184, 220, 256])
@pytest.mark.parametrize("R", [1, 2, 3, 5, 7, 8, 10, 12])
@pytest.mark.parametrize("block", [False, True])
def test_fold_protocol_leaf_and_tree(c, R, block):
    leaf = [0, 0, 0, 0]                               # four leaf tiles
    tree = [64 * t for t in range((c + 63) // 64)]    # one tree combine: tile t starts at 64 t
    for seed in range(12):
        assert run(c, leaf, seed, R, block), ("deadlock", c, R, "leaf", seed)
        assert run(c, tree + tree, seed, R, block), ("deadlock", c, R, "tree", seed)


def test_fold_protocol_needs_the_previous_group_published():
    """Without the wait for the slot's previous group to have started, a builder can
    see done = 0 left from the group before it (whose users have all arrived) while
    the previous group has not been built yet, and refill the slot under it."""
    bad = 0
    for seed in range(40):
        try:
            ok = run(220, [0, 0, 0, 0], seed, 3, True, naive=True)
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
