"""Host model of the Jacobi kernels' pair schedules, written with the kernels'
index formulas.  Register-resident kernel (the slot moves of its ring phases,
splits and final circle tournament): every sweep meets every column pair
exactly once, in 2*ceil(n/2) - 1 rounds, for any column count, starting from
any arrangement.  Blocked kernel (round-robin tournament over column blocks,
a full sweep of the slot schedule on the first block round's pairs and one ring
phase on the later ones): every sweep meets every column pair exactly once."""
import itertools

import numpy as np
import pytest


def sweep(top, bot, ring_only=False):
    """One sweep on slots (top[g], bot[g]); yields the pairs of each round and
    leaves the arrangement the kernel leaves.  ring_only: the first ring phase
    alone (S rounds, S even)."""
    S = len(top)
    c, ring, s0 = S, S % 2 == 0, [0] * S
    idx = list(range(S))          # i = g - s0 per slot
    r = 0
    nrounds = S if ring_only else 2 * S - 1
    for k in range(nrounds):
        yield list(zip(top, bot))
        if k + 1 == nrounds:
            break
        if ring and r + 1 < c:
            # bottoms move one slot down the range: slot g takes slot nxt's bottom
            nb = list(bot)
            for g in range(S):
                i = idx[g]
                nxt = s0[g] + (0 if i + 1 == c else i + 1)
                nb[g] = bot[nxt]
            bot[:] = nb
            r += 1
        elif ring:
            h = c // 2
            nt, nb = list(top), list(bot)
            for g in range(S):
                if idx[g] < h:
                    nb[g] = top[g + h]       # first half takes the second half's tops as bottoms
                else:
                    nt[g] = bot[g - h]       # second half takes the first half's bottoms as tops
            top[:], bot[:] = nt, nb
            c = h
            ring = c % 2 == 0
            for g in range(S):
                s0[g] = (g // c) * c
                idx[g] = g - s0[g]
            r = 0
        else:
            # circle over each range's 2c columns through positions pos0 .. pos0 + c
            buf = {}
            for g in range(S):
                pos0 = s0[g] + s0[g] // c
                buf[pos0 + idx[g]] = top[g]
                if idx[g] == 0:
                    buf[pos0 + c] = bot[g]
            nt = list(top)
            for g in range(S):
                pos0 = s0[g] + s0[g] // c
                i = idx[g]
                if i != 0:
                    nt[g] = buf[pos0 + (c if i == 1 else i - 1)]
                    buf[pos0 + i - 1] = bot[g]
            nb = [buf[s0[g] + s0[g] // c + idx[g]] for g in range(S)]
            top[:], bot[:] = nt, nb
            r += 1


@pytest.mark.parametrize("n", list(range(2, 70)) + [96, 100, 128, 144, 150, 176, 200, 256])
def test_every_pair_once_per_sweep(n):
    S = (n + 1) // 2
    rng = np.random.default_rng(n)
    perm = rng.permutation(2 * S)
    top, bot = list(perm[:S]), list(perm[S:])
    for _ in range(3):           # consecutive sweeps start from the previous arrangement
        seen = {}
        rounds = 0
        for pairs in sweep(top, bot):
            rounds += 1
            for a, b in pairs:
                if a < n and b < n:   # ids >= n are the zero padding column
                    key = (min(a, b), max(a, b))
                    seen[key] = seen.get(key, 0) + 1
        assert rounds == 2 * S - 1
        assert len(seen) == n * (n - 1) // 2
        assert all(v == 1 for v in seen.values())
        assert sorted(top + bot) == list(range(2 * S))


def test_ring_phases_move_one_column_per_slot():
    """In a ring round only the bottoms change (the property that halves the
    LDS exchange of the circle tournament, where both columns move)."""
    top, bot = list(range(72)), list(range(72, 144))
    it = sweep(top, bot)
    prev = next(it)
    for _ in range(71):          # the first ring phase (c = 72)
        cur = next(it)
        assert [a for a, _ in cur] == [a for a, _ in prev]
        assert sorted(b for _, b in cur) == sorted(b for _, b in prev)
        prev = cur


def blk_at(pos, br, nblk):
    return 0 if pos == 0 else 1 + (pos - 1 + br) % (nblk - 1)


def blocked_sweep_pairs(n, b, nblk):
    """Pairs met in one sweep of the blocked kernel (columns >= n are padding)."""
    seen = {}
    rounds = 0
    for br in range(nblk - 1):
        for pi in range(nblk // 2):
            A, B = blk_at(pi, br, nblk), blk_at(nblk - 1 - pi, br, nblk)
            top = [A * b + g for g in range(b)]
            bot = [B * b + g for g in range(b)]
            for pairs in sweep(top, bot, ring_only=br > 0):
                rounds += 1
                for x, y in pairs:
                    if x < n and y < n:
                        key = (min(x, y), max(x, y))
                        seen[key] = seen.get(key, 0) + 1
            # columns go back to their own place: the pair's column set is unchanged
            assert sorted(top + bot) == sorted([A * b + g for g in range(b)] + [B * b + g for g in range(b)])
    return seen, rounds


# (n, b, nblk) as the blocked kernel's configuration picks them for working
# matrices of 512 x 512 and 300 x 300 (32 lanes per pair), 600 x 256 and
# 2048 x 512 (64 lanes per pair), 257 x 257, plus wider blocks and small cases
@pytest.mark.parametrize("n,b,nblk", [(512, 32, 16), (300, 30, 10), (256, 16, 16), (512, 16, 32),
                                      (257, 26, 10), (512, 64, 8), (300, 50, 6), (10, 2, 6), (9, 4, 4),
                                      (6, 2, 4), (40, 10, 4)])
def test_blocked_sweep_meets_every_pair_once(n, b, nblk):
    assert b % 2 == 0 and nblk % 2 == 0 and b * nblk >= n
    seen, rounds = blocked_sweep_pairs(n, b, nblk)
    assert len(seen) == n * (n - 1) // 2
    assert all(v == 1 for v in seen.values())
    assert rounds == (nblk // 2) * ((2 * b - 1) + (nblk - 2) * b)


def test_block_tournament_pairs_every_block_once():
    for nblk in (2, 4, 6, 8, 32):
        met = set()
        for br in range(nblk - 1):
            pos = [blk_at(p, br, nblk) for p in range(nblk)]
            assert sorted(pos) == list(range(nblk))
            for pi in range(nblk // 2):
                met.add(frozenset((pos[pi], pos[nblk - 1 - pi])))
        assert len(met) == nblk * (nblk - 1) // 2


def ring_positions(c, r, i):
    """Single exchange buffer, ring round r of a phase over c slots: the position
    slot i writes its bottom to and the one it reads its new bottom from (the
    kernels' formulas)."""
    wpos = i + r if i + r < c else i + r - c
    rpos = 0 if wpos + 1 == c else wpos + 1
    return wpos, rpos


@pytest.mark.parametrize("c", [2, 4, 6, 8, 18, 36, 72, 128])
def test_single_buffer_ring_positions(c):
    """With one buffer and one barrier per ring round: every slot reads slot
    i+1's bottom (the ring move), and the position a slot writes in round r+1
    was read in round r by that slot alone, so no other lane can still be
    reading it when it is overwritten."""
    bottoms = list(range(100, 100 + c))
    for r in range(c - 1):
        buf = {}
        for i in range(c):
            w, _ = ring_positions(c, r, i)
            assert w not in buf
            buf[w] = bottoms[i]
        new = []
        readers = {}
        for i in range(c):
            _, rd = ring_positions(c, r, i)
            new.append(buf[rd])
            readers.setdefault(rd, []).append(i)
        assert new == [bottoms[(i + 1) % c] for i in range(c)]
        if r + 1 < c - 1:
            for i in range(c):
                w_next, _ = ring_positions(c, r + 1, i)
                assert readers.get(w_next, []) in ([], [i])
        bottoms = new
