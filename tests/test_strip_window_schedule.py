"""The windowed application of a strip's picks (the GPU apply kernel of the
paper's dynamics) on the host: picks are taken in windows, every pick that
conflicts with no earlier pick of its window (it reads a word that such a
pick writes: its own word, left, right, up, down or the wrap-row patch word)
is applied at once from the state before the step, and the others are
deferred, in order, to head the next window.  Whatever the update does, this
must give the state of applying the picks one by one; here the update is an
arbitrary order-sensitive mix of the word and everything it reads."""
import random

import pytest

import oracle


def _hood(I, col, N, istar, width):
    # LDS-style addresses (column, row) of the word, left, right, up, down,
    # patch; columns 0 and width + 1 are frozen neighbours
    up = I - 1 if I > 0 else N - 1
    dn = I + 1 if I < N - 1 else 0
    patch = istar if I == 0 else (0 if I == istar else I)
    return (col, I), [(col, I), (col - 1, I), (col + 1, I), (col, up), (col, dn), (col, patch)]


def _mix(vals):
    h = 0x9E3779B97F4A7C15
    for v in vals:
        h = ((h ^ v) * 0xBF58476D1CE4E5B9 + 0x94D049BB133111EB) & (2**64 - 1)
        h ^= h >> 29
    return h


def _sequential(state, picks, N, istar, width):
    s = dict(state)
    for I, col in picks:
        w, reads = _hood(I, col, N, istar, width)
        s[w] = _mix([s[x] for x in reads])
    return s


def _windowed(state, picks, N, istar, width, G):
    s = dict(state)
    deferred, kk, steps = [], 0, 0
    while deferred or kk < len(picks):
        window = list(deferred)
        while len(window) < G and kk < len(picks):
            window.append(kk)
            kk += 1
        claim = {}
        for lane, p in enumerate(window):  # atomic minimum of the lane index
            w, _ = _hood(*picks[p], N, istar, width)
            claim[w] = min(claim.get(w, lane), lane)
        loads, commit, deferred = {}, [], []
        for lane, p in enumerate(window):
            w, reads = _hood(*picks[p], N, istar, width)
            loads[lane] = [s[x] for x in reads]  # every lane loads before any stores
            if any(claim.get(x, G) < lane for x in reads):
                deferred.append(p)
            else:
                commit.append((w, lane))
        for w, lane in commit:
            s[w] = _mix(loads[lane])
        steps += 1
    return s, steps


@pytest.mark.parametrize("L,width,G", [(84, 1, 32), (84, 3, 16), (42, 1, 64), (2016, 1, 32), (1008, 2, 32),
                                       (130, 5, 8), (4, 1, 32), (8, 2, 4)])
def test_windowed_application_equals_sequential(L, width, G):
    N = oracle.word_rows(L)
    istar = (L - 1) % N
    rng = random.Random(L * 1000 + width * 10 + G)
    state = {(c, I): rng.getrandbits(64) for c in range(width + 2) for I in range(N)}
    picks = [(rng.randrange(N), 1 + rng.randrange(width)) for _ in range(10 * N * width)]
    want = _sequential(state, picks, N, istar, width)
    got, steps = _windowed(state, picks, N, istar, width, G)
    assert got == want
    assert steps <= len(picks)


def test_every_step_applies_the_first_pick_of_its_window():
    # a window whose picks all read each other (N = 2, one column) still
    # applies one pick per step
    N, istar, width = 2, 1, 1
    state = {(c, I): 7 * c + I for c in range(3) for I in range(N)}
    picks = [(i % 2, 1) for i in range(40)]
    got, steps = _windowed(state, picks, N, istar, width, 32)
    assert got == _sequential(state, picks, N, istar, width)
    assert steps == 40
