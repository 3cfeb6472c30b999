"""Pins of the oracle's tabu search (Alg. 2 / Alg. 4) and walk schedule.

The walk is a heuristic driven by random draws, so its pins are properties
that any correct walk must satisfy, checked with energies recomputed in numpy
(never with the oracle's own scoring): every step takes an admissible minimum,
tabu moves are refused, the best is the first minimum visited, energies stay
consistent with the sequence, ties are broken uniformly, and with aspiration a
best found before the last step is a local minimum (Sec. II.A's notion).
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import npref

SCHED_64 = O.Schedule(O.STEPS_MULT_N, 4, O.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, 1)


def test_schedule_rules():
    # tenure U[floor(N/10), floor(N/5)] at N = 64 -> [6, 12]; 4N steps
    assert O.walk_schedule(64, SCHED_64, 1, 0, 0) == (256, 6, 12)
    # tenure U[1, floor(N/10)+1] at N = 20 -> [1, 3]
    memetic = O.Schedule(O.STEPS_PAPER, 0, O.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1)
    seen = set()
    for g in range(3000):
        T, lo, hi = O.walk_schedule(20, memetic, 77, 3, g)
        assert (lo, hi) == (1, 3)
        assert 10 <= T <= 30  # randomInt(0, N) + floor(N/2), Alg. 4
        seen.add(T)
    assert seen == set(range(10, 31))
    # the paper's tenure: floor(0.1 maxIter), floor(0.12 maxIter) (Sec. III.B)
    paper = O.Schedule(O.STEPS_FIXED, 50, O.TENURE_PAPER, 0, 1, 0, 0, 1, 0, 0)
    assert O.walk_schedule(64, paper, 1, 0, 0) == (50, 5, 6)
    paper = O.Schedule(O.STEPS_FIXED, 99, O.TENURE_PAPER, 0, 1, 0, 0, 1, 0, 0)
    assert O.walk_schedule(64, paper, 1, 0, 0) == (99, 9, 11)
    # a tenure range reaching N could leave no admissible move: rejected
    bad = O.Schedule(O.STEPS_FIXED, 10, O.TENURE_LINEAR, 0, 1, 1, 1, 1, 0, 1)
    with pytest.raises(ValueError):
        O.walk_schedule(8, bad, 1, 0, 0)


def test_random_start_statistics():
    # uniform +-1 starts: E[C_k^2] = N-k, so the mean energy is N(N-1)/2
    n, W = 64, 4000
    S = np.stack([O.random_start(n, 1001, w) for w in range(W)])
    e = npref.energies_rows(S)
    assert abs(e.mean() - n * (n - 1) / 2) < 4 * e.std() / np.sqrt(W)
    assert abs(S.mean()) < 0.01
    # bit i of the start is bit i%32 of word i/32 of draw (walk, 0, 0, TAG_START)
    w = O.draw(1001, 5, 0, 0, O.TAG_START)
    bits = [(int(w[i >> 5]) >> (i & 31)) & 1 for i in range(n)]
    assert list(S[5]) == [1 - 2 * b for b in bits]


def test_random_start_beyond_128():
    # bits 128.. of a start come from draw (walk, 0, 1, TAG_START), read like
    # the first; the first 128 bits do not depend on N
    n = 256
    s = O.random_start(n, 1001, 9)
    w0 = O.draw(1001, 9, 0, 0, O.TAG_START)
    w1 = O.draw(1001, 9, 0, 1, O.TAG_START)
    bits = [(int(w0[i >> 5]) >> (i & 31)) & 1 for i in range(128)]
    bits += [(int(w1[i >> 5]) >> (i & 31)) & 1 for i in range(128)]
    assert list(s) == [1 - 2 * b for b in bits]
    assert np.array_equal(O.random_start(200, 1001, 9), s[:200])
    assert np.array_equal(O.random_start(100, 1001, 9), s[:100])
    # and the mean energy of uniform starts, N(N-1)/2, at N = 200
    S = np.stack([O.random_start(200, 1001, w) for w in range(1500)])
    e = npref.energies_rows(S)
    assert abs(e.mean() - 200 * 199 / 2) < 4 * e.std() / np.sqrt(len(S))


@pytest.mark.parametrize("n,asp", [(5, 1), (16, 0), (16, 1), (33, 1), (64, 1), (64, 0), (100, 1), (128, 1),
                                   (129, 1), (200, 0), (256, 1)])
def test_walk_tables_equal_recompute(n, asp):
    lo, hi = max(n // 10, 0), max(n // 5, 1)
    steps = 3 * n if n <= 64 else (n if n <= 128 else 12)  # recompute is O(N^3) per step
    for w in range(3 if n <= 128 else 1):
        s = O.random_start(n, 42, w)
        a = O.tabu_walk(s, 42, w, 0, steps, lo, hi, asp, recompute=True, want_trace=True)
        b = O.tabu_walk(s, 42, w, 0, steps, lo, hi, asp, recompute=False, want_trace=True)
        assert np.array_equal(a[0], b[0]) and a[1:3] == b[1:3]
        assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4])


def _check_walk_properties(start, steps, lo, hi, asp, best, best_e, final_e, trace, trace_e):
    n = len(start)
    s = start.astype(np.int64).copy()
    e0 = npref.energy(s)
    bestE, best_seq = e0, s.copy()
    last_flip = {}
    best_step = 0
    for t in range(1, steps + 1):
        cand = npref.flip_energies(s)
        i = int(trace[t - 1])
        # energies are consistent with the sequence
        assert cand[i] == trace_e[t - 1]
        assert (cand[i] - npref.energy(s)) % 4 == 0
        # a move flipped within the last lo steps is tabu; it may only be
        # taken through aspiration (strictly better than the walk's best)
        if i in last_flip and t - last_flip[i] <= lo:
            assert asp and cand[i] < bestE
        # no neighbour that is surely admissible (not flipped in the last hi
        # steps) or aspirated is strictly better than the move taken
        for j in range(n):
            surely_free = j not in last_flip or t - last_flip[j] > hi
            if surely_free or (asp and cand[j] < bestE):
                assert cand[i] <= cand[j]
        s[i] = -s[i]
        last_flip[i] = t
        if cand[i] < bestE:
            bestE, best_seq, best_step = int(cand[i]), s.copy(), t
    assert best_e == bestE and np.array_equal(best, best_seq)
    assert final_e == (trace_e[-1] if steps else e0)
    assert npref.energy(best) == best_e and best_e <= e0
    if asp and best_step < steps:
        # aspiration admits every strictly improving neighbour, so a best
        # that was not improved on at the next step is a local minimum
        assert np.all(npref.flip_energies(best_seq) >= best_e)


@pytest.mark.parametrize("n,asp,lo,hi", [(7, 1, 0, 1), (12, 0, 1, 2), (20, 1, 1, 3), (20, 0, 2, 4),
                                         (31, 1, 3, 6), (64, 1, 6, 12), (64, 0, 6, 12), (96, 1, 9, 19),
                                         (160, 1, 16, 32), (256, 0, 25, 51)])
def test_walk_properties(n, asp, lo, hi):
    steps = min(3 * n, 150 if n <= 128 else 40)
    for w in range(2):
        s = O.random_start(n, 7, w)
        best, be, fe, tr, te = O.tabu_walk(s, 7, w, 3, steps, lo, hi, asp, want_trace=True)
        _check_walk_properties(s, steps, lo, hi, asp, best, be, fe, tr, te)


def test_walk_tenure_zero_and_zero_steps():
    s = O.random_start(40, 3, 0)
    best, be, fe, tr, te = O.tabu_walk(s, 3, 0, 0, 0, 0, 0, 1, want_trace=True)
    assert np.array_equal(best, s) and be == fe == npref.energy(s)
    best, be, fe, tr, te = O.tabu_walk(s, 3, 0, 0, 60, 0, 0, 1, want_trace=True)
    _check_walk_properties(s, 60, 0, 0, 1, best, be, fe, tr, te)


def test_tie_break_uniform():
    # from the all-ones sequence, flips of i and N-1-i have equal energy
    # (reversal symmetry), so step 1 always has a tie; the pick must be
    # uniform over the tied set, whose members come from numpy energies
    n = 16
    s = np.ones(n, dtype=np.int8)
    cand = npref.flip_energies(s)
    ties = np.flatnonzero(cand == cand.min())
    assert len(ties) >= 2
    counts = {int(i): 0 for i in ties}
    R = 4000
    for seed in range(R):
        _, _, _, tr, _ = O.tabu_walk(s, seed, 0, 0, 1, 1, 2, 1, want_trace=True)
        counts[int(tr[0])] += 1
    exp = R / len(ties)
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 30, counts


def test_tie_rule_exact():
    # the pick is T[(u0 * |T|) >> 32] over the ascending tied set T, with u0
    # word 0 of draw (entity, gen, t, TAG_STEP) (pure-Python Philox here)
    n = 16
    s = np.ones(n, dtype=np.int8)
    cand = npref.flip_energies(s)
    ties = np.flatnonzero(cand == cand.min())
    for seed in range(50):
        _, _, _, tr, _ = O.tabu_walk(s, seed, 9, 4, 1, 1, 2, 1, want_trace=True)
        u0 = npref.philox([9, 4, 1, O.TAG_STEP], [seed & 0xFFFFFFFF, seed >> 32])[0]
        assert tr[0] == ties[(u0 * len(ties)) >> 32]


def test_tabu_batch_matches_single_walks():
    n, W = 24, 16
    sch = O.Schedule(O.STEPS_MULT_N, 3, O.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, 1)
    best, be, fe = O.tabu_batch(W, sch, 55, n_uniform=n, stride=32, nthreads=4)
    for w in range(W):
        T, lo, hi = O.walk_schedule(n, sch, 55, w, 0)
        s = O.random_start(n, 55, w)
        b1, e1, f1, _, _ = O.tabu_walk(s, 55, w, 0, T, lo, hi, 1)
        assert np.array_equal(best[w, :n], b1) and be[w] == e1 and fe[w] == f1
        assert not best[w, n:].any()


# ---------------------------------------------------------------------------
# Tenure: the tabuList entry of each move, and the admissible set it defines.
# ---------------------------------------------------------------------------
M32 = 0xFFFFFFFF


@pytest.mark.parametrize("n,lo,hi,asp", [(9, 0, 4, 0), (20, 1, 3, 1), (33, 3, 6, 0), (64, 6, 12, 1),
                                         (130, 13, 26, 1)])
def test_tenure_expiry_exact(n, lo, hi, asp):
    # The move of step t stays tabu through step t + lo + ((u1 (hi-lo+1)) >> 32),
    # u1 word 1 of draw (entity, gen, t, STEP) (pure-Python Philox here), and
    # each step takes a minimum over exactly the moves whose entry is below t
    # (plus, with aspiration, those beating the walk's best), by numpy energies.
    seed, ent, gen = 2024, 5, 7
    steps = min(6 * n, 200)
    s = O.random_start(n, seed, ent)
    best, be, fe, tr, te, tx = O.tabu_walk(s, seed, ent, gen, steps, lo, hi, asp,
                                           want_trace=True, want_expiry=True)
    key = [seed & M32, seed >> 32]
    tabu = np.zeros(n, dtype=np.int64)
    cur = s.astype(np.int64).copy()
    bestE = npref.energy(cur)
    for t in range(1, steps + 1):
        u1 = npref.philox([ent, gen, t, O.TAG_STEP], key)[1]
        assert tx[t - 1] == t + lo + ((u1 * (hi - lo + 1)) >> 32), t
        i = int(tr[t - 1])
        cand = npref.flip_energies(cur)
        adm = (tabu < t) | (bool(asp) & (cand < bestE))
        assert adm[i] and cand[i] == cand[adm].min(), t
        cur[i] = -cur[i]
        tabu[i] = tx[t - 1]
        bestE = min(bestE, int(cand[i]))
    assert be == bestE


def test_tenure_uniform():
    # tenures tabuList - t over many steps are uniform over [lo, hi]
    n, lo, hi = 40, 2, 9
    taus = []
    for w in range(30):
        s = O.random_start(n, 11, w)
        *_, tx = O.tabu_walk(s, 11, w, 0, 120, lo, hi, 1, want_trace=True, want_expiry=True)
        taus.append(tx - np.arange(1, 121))
    taus = np.concatenate(taus)
    assert taus.min() >= lo and taus.max() <= hi
    hist = np.bincount(taus - lo, minlength=hi - lo + 1)
    exp = len(taus) / (hi - lo + 1)
    chi2 = float(np.sum((hist - exp) ** 2 / exp))
    assert chi2 < 30, hist  # 7 degrees of freedom


# ---------------------------------------------------------------------------
# Walk length drawn from a range (Sec. III.B: randInt[N/2, 3N/2]).
# ---------------------------------------------------------------------------
def test_steps_range_rule():
    # RANGE(1/2, 3/2) is Sec. III.B's statement; Alg. 4's
    # randomInt(0, N) + floor(N/2) (the PAPER rule) spans the same integers,
    # floor(3N/2) - floor(N/2) = N, and both take the same draw: they agree
    # walk for walk at every N
    paper = O.Schedule(O.STEPS_PAPER, 0, O.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1)
    rng_ = O.Schedule(O.STEPS_RANGE, 0, O.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1, 1, 2, 3, 2)
    for n in range(3, 257):
        for e in range(3):
            assert O.walk_schedule(n, rng_, 9, e, n) == O.walk_schedule(n, paper, 9, e, n)
    # RANGE(1, 2): T uniform over [N, 2N], both ends included
    two = O.Schedule(O.STEPS_RANGE, 0, O.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, 1, 1, 1, 2, 1)
    n = 10
    Ts = np.array([O.walk_schedule(n, two, 5, e, 0)[0] for e in range(11000)])
    assert Ts.min() == n and Ts.max() == 2 * n
    hist = np.bincount(Ts - n, minlength=n + 1)
    chi2 = float(np.sum((hist - 1000) ** 2 / 1000))
    assert chi2 < 35, hist  # 10 degrees of freedom
    # an empty range is invalid
    bad = O.Schedule(O.STEPS_RANGE, 0, O.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1, 2, 1, 1, 1)
    with pytest.raises(ValueError):
        O.walk_schedule(12, bad, 1, 0, 0)
