"""Pins of the oracle's memetic search (Alg. 1 / Alg. 3).

Checked against properties that hold for any correct run, with energies
recomputed in numpy: the population's energies match its sequences, the best
is never lost and never increases, the degenerate configuration (no
crossover, no mutation, empty walks) only shuffles copies of the initial
members, a run split into two calls equals the uninterrupted run, the
early-stop generation is the first one at which the target holds, and no run
beats the exhaustive optimum.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import npref

MEM = O.Schedule(O.STEPS_PAPER, 0, O.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1)


def test_init():
    st = O.MemeticState(20, 100, 1000, 0)
    assert list(st.popE) == list(npref.energies_rows(st.pop))
    a = int(np.argmin(st.popE))
    assert st.bestE == st.popE[a] and np.array_equal(st.best, st.pop[a])
    w = O.draw(1000, 0, 3, 0, O.TAG_INIT)  # member 3 of population 0
    assert list(st.pop[3]) == [1 - 2 * ((int(w[i >> 5]) >> (i & 31)) & 1) for i in range(20)]


def test_init_beyond_128():
    # bits 128.. of member m come from draw (pop, m, 1, TAG_INIT)
    st = O.MemeticState(200, 5, 1000, 4)
    assert list(st.popE) == list(npref.energies_rows(st.pop))
    w0 = O.draw(1000, 4, 2, 0, O.TAG_INIT)
    w1 = O.draw(1000, 4, 2, 1, O.TAG_INIT)
    bits = [(int(w0[i >> 5]) >> (i & 31)) & 1 for i in range(128)]
    bits += [(int(w1[(i - 128) >> 5]) >> (i & 31)) & 1 for i in range(128, 200)]
    assert list(st.pop[2]) == [1 - 2 * b for b in bits]


def test_generation_invariants_long():
    # N = 200 (four mask words on the GPU): invariants over a few generations
    n = 200
    st = O.MemeticState(n, 12, 77, 1)
    prev = st.bestE
    for g in range(3):
        assert st.advance(1, MEM, O.P_COMB_090, O.p_mut_inv_n(n)) == 1
        assert st.bestE <= prev
        prev = st.bestE
        assert npref.energy(st.best) == st.bestE
        assert list(st.popE) == list(npref.energies_rows(st.pop))


def test_generation_invariants():
    n = 20
    st = O.MemeticState(n, 100, 1000, 0)
    prev = st.bestE
    for g in range(50):
        assert st.advance(1, MEM, O.P_COMB_090, O.p_mut_inv_n(n)) == 1
        assert st.bestE <= prev
        prev = st.bestE
        assert npref.energy(st.best) == st.bestE
        assert list(st.popE) == list(npref.energies_rows(st.pop))
        assert st.bestE <= st.popE.min()
    emin, _ = O.bruteforce_min(n)
    assert st.bestE >= emin
    assert st.gen == 50


def test_degenerate_copies_only():
    # p_comb = 0, p_mutate = 0 and zero-step walks: every child is a copy of a
    # member, so best never changes and every member stays an initial one
    n = 24
    zero = O.Schedule(O.STEPS_FIXED, 0, O.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1)
    st = O.MemeticState(n, 30, 5, 2)
    init_rows = {tuple(r) for r in st.pop}
    init_best = st.bestE
    st.advance(200, zero, 0, 0)
    assert st.bestE == init_best
    assert all(tuple(r) in init_rows for r in st.pop)
    assert list(st.popE) == list(npref.energies_rows(st.pop))


def test_crossover_child_is_two_parents():
    # with mutation off and empty walks, a crossover child is a prefix of one
    # member followed by the suffix of another, cut in [1, N-1]
    n = 16
    zero = O.Schedule(O.STEPS_FIXED, 0, O.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1)
    st = O.MemeticState(n, 10, 11, 0)
    for _ in range(100):
        before = st.pop.copy()
        st.advance(1, zero, 0xFFFFFFFF, 0)
        changed = [r for r in range(10) if not np.array_equal(before[r], st.pop[r])]
        for r in changed:
            child = st.pop[r]
            ok = any(np.array_equal(child[:c], before[a, :c]) and np.array_equal(child[c:], before[b, c:])
                     for c in range(1, n) for a in range(10) for b in range(10))
            assert ok


def test_mutation_rate():
    # p_mutate = 1/N: flips per child average 1 (sample-only, empty walks)
    n = 32
    zero = O.Schedule(O.STEPS_FIXED, 0, O.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1)
    st = O.MemeticState(n, 1, 3, 0)  # K = 1: the sampled parent is member 0
    flips = []
    for _ in range(3000):
        before = st.pop[0].copy()
        st.advance(1, zero, 0, O.p_mut_inv_n(n))
        flips.append(int(np.sum(before != st.pop[0])))
    assert abs(np.mean(flips) - 1.0) < 0.08


def test_resume_equals_uninterrupted():
    n = 28
    a = O.MemeticState(n, 40, 99, 4)
    b = a.copy()
    a.advance(30, MEM, O.P_COMB_090, O.p_mut_inv_n(n))
    b.advance(13, MEM, O.P_COMB_090, O.p_mut_inv_n(n))
    b.advance(17, MEM, O.P_COMB_090, O.p_mut_inv_n(n))
    assert np.array_equal(a.pop, b.pop) and np.array_equal(a.popE, b.popE)
    assert np.array_equal(a.best, b.best) and a.bestE == b.bestE and a.gen == b.gen == 30


def test_target_stops_at_first_hit():
    n = 30
    base = O.MemeticState(n, 50, 21, 1)
    hist = [base.bestE]
    run = base.copy()
    for _ in range(40):
        run.advance(1, MEM, O.P_COMB_090, O.p_mut_inv_n(n))
        hist.append(run.bestE)
    target = hist[25]
    first = next(g for g, e in enumerate(hist) if e <= target)
    st = base.copy()
    done = st.advance(40, MEM, O.P_COMB_090, O.p_mut_inv_n(n), target=target)
    assert st.hit == first and done == first and st.bestE == hist[first]
    # a target met by the initial population is a hit at generation 0
    st = base.copy()
    assert st.advance(10, MEM, O.P_COMB_090, O.p_mut_inv_n(n), target=base.bestE) == 0
    assert st.hit == 0


# ---------------------------------------------------------------------------
# Batched-generation variant: B children per generation from one snapshot.
# ---------------------------------------------------------------------------
def test_batched_one_child_is_alg1():
    # B = 1 takes every draw and step of Alg. 1
    for n, K, target in [(20, 100, -1), (33, 17, -1), (65, 24, -1), (26, 40, 120)]:
        a = O.MemeticState(n, K, 7, 1)
        b = a.copy()
        a.advance(25, MEM, O.P_COMB_090, O.p_mut_inv_n(n), target=target)
        b.advance(25, MEM, O.P_COMB_090, O.p_mut_inv_n(n), target=target, children=1)
        assert a.bestE == b.bestE and a.gen == b.gen and a.hit == b.hit
        assert np.array_equal(a.pop, b.pop) and np.array_equal(a.popE, b.popE)
        assert np.array_equal(a.best, b.best)


def test_batched_snapshot_and_merge_order():
    # Sampling only, no mutation, empty walks: child b is the snapshot member
    # (w1 * K) >> 32 of draw (pop, g, 2b, GEN) and replaces member
    # (w2 * K) >> 32 of draw (pop, g, 2b + 1, GEN), merged in b order.
    n, K, B, seed, pid = 22, 9, 6, 31, 4
    zero = O.Schedule(O.STEPS_FIXED, 0, O.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1)
    st = O.MemeticState(n, K, seed, pid)
    for g in range(5):
        snap = st.pop.copy()
        snapE = st.popE.copy()
        want, wantE = snap.copy(), snapE.copy()
        for b in range(B):
            w1 = int(O.draw(seed, pid, g, 2 * b, O.TAG_GEN)[1])
            w2 = int(O.draw(seed, pid, g, 2 * b + 1, O.TAG_GEN)[2])
            src, dst = (w1 * K) >> 32, (w2 * K) >> 32
            want[dst], wantE[dst] = snap[src], snapE[src]
        st.advance(1, zero, 0, 0, children=B)
        assert np.array_equal(st.pop, want) and np.array_equal(st.popE, wantE)


def test_batched_mutation_words():
    # K = 1, sampling only, empty walks: every child is member 0 with bit i
    # flipped when word i%4 of draw (pop, g, 64 b + i/4, MUT) is below the
    # threshold; the last child (b = B - 1) is what member 0 holds after the
    # merge.  N = 256 uses all 64 mutation words of a child.
    n, B, seed, pid, thr = 256, 3, 17, 1, 0x20000000
    zero = O.Schedule(O.STEPS_FIXED, 0, O.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1)
    st = O.MemeticState(n, 1, seed, pid)
    for g in range(3):
        before = st.pop[0].copy()
        st.advance(1, zero, 0, thr, children=B)
        b = B - 1
        flip = [int(O.draw(seed, pid, g, 64 * b + (i >> 2), O.TAG_MUT)[i & 3]) < thr
                for i in range(n)]
        want = np.where(flip, -before, before).astype(np.int8)
        assert np.array_equal(st.pop[0], want)
        assert st.popE[0] == npref.energy(want)


def test_batched_invariants_and_resume():
    n, K, B = 40, 50, 4
    st = O.MemeticState(n, K, 11, 2)
    full = st.copy()
    prev = st.bestE
    for g in range(12):
        assert st.advance(1, MEM, O.P_COMB_090, O.p_mut_inv_n(n), children=B) == 1
        assert st.bestE <= prev
        prev = st.bestE
        assert npref.energy(st.best) == st.bestE
        assert list(st.popE) == list(npref.energies_rows(st.pop))
        assert st.bestE <= st.popE.min()
    full.advance(12, MEM, O.P_COMB_090, O.p_mut_inv_n(n), children=B)
    assert full.bestE == st.bestE and np.array_equal(full.pop, st.pop)
    # mutation words of child b come from index 64 b + i/4: with every
    # other draw fixed, a different B changes the children after the first
    other = O.MemeticState(n, K, 11, 2)
    other.advance(12, MEM, O.P_COMB_090, O.p_mut_inv_n(n), children=B - 1)
    assert not np.array_equal(other.pop, st.pop)


def test_batched_target_counts_generations():
    n, K, B = 24, 30, 3
    base = O.MemeticState(n, K, 19, 0)
    run = base.copy()
    run.advance(40, MEM, O.P_COMB_090, O.p_mut_inv_n(n), children=B)
    target = run.bestE
    # the first generation at which best <= target
    probe = base.copy()
    first = None
    for g in range(40):
        probe.advance(1, MEM, O.P_COMB_090, O.p_mut_inv_n(n), children=B)
        if probe.bestE <= target:
            first = g + 1
            break
    stop = base.copy()
    stop.advance(40, MEM, O.P_COMB_090, O.p_mut_inv_n(n), target=target, children=B)
    assert stop.hit == first and stop.gen == first and stop.bestE <= target


# ---------------------------------------------------------------------------
# The generation's draws: parents, cut, sampled member and replaced slot.
# ---------------------------------------------------------------------------
ZERO_WALK = O.Schedule(O.STEPS_FIXED, 0, O.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1)
M32 = 0xFFFFFFFF


def _gen_words(seed, pid, g):
    # words w0..w7 of generation g: draws (pid, g, 0 | 1, GEN), pure-Python Philox
    key = [seed & M32, seed >> 32]
    return (npref.philox([pid, g, 0, O.TAG_GEN], key) +
            npref.philox([pid, g, 1, O.TAG_GEN], key))


@pytest.mark.parametrize("n,K,p_comb", [(8, 30, 0xFFFFFFFF), (8, 30, O.P_COMB_090),
                                        (13, 7, 0xFFFFFFFF), (40, 100, O.P_COMB_090)])
def test_generation_rebuilt_from_draws(n, K, p_comb):
    # Mutation off and zero-step walks: each child is the crossover of two
    # tournament winners (lower energy wins, a tie goes to the first draw)
    # cut at 1 + ((w5 (N-1)) >> 32), or the member (w1 K) >> 32 when
    # w0 >= p_comb; it replaces member (w6 K) >> 32 (readings of Alg. 1's
    # selectParents, Combine and replacement).  The population is rebuilt
    # here generation by generation with numpy energies and compared exactly.
    seed, pid, G = 123457, 3, 400
    st = O.MemeticState(n, K, seed, pid)
    pop = st.pop.astype(np.int64)
    popE = npref.energies_rows(pop)
    bestE = int(popE.min())
    # how often a plausible misreading would have changed the child
    tie_matters = cut_matters = 0
    for g in range(G):
        w = _gen_words(seed, pid, g)

        def tour(u, v):
            i, j = (u * K) >> 32, (v * K) >> 32
            return i if popE[i] <= popE[j] else j

        if w[0] < p_comb:
            a, b = tour(w[1], w[2]), tour(w[3], w[4])
            cut = 1 + ((w[5] * (n - 1)) >> 32)
            child = np.concatenate([pop[a, :cut], pop[b, cut:]])
            i, j = (w[1] * K) >> 32, (w[2] * K) >> 32
            if i != j and popE[i] == popE[j] and not np.array_equal(pop[i, :cut], pop[j, :cut]):
                tie_matters += 1
            alt = (w[5] * n) >> 32  # the cut over [0, N) instead of [1, N-1]
            if alt != cut and not np.array_equal(pop[a, min(alt, cut):max(alt, cut)],
                                                 pop[b, min(alt, cut):max(alt, cut)]):
                cut_matters += 1
        else:
            child = pop[(w[1] * K) >> 32].copy()
        e = npref.energy(child)
        bestE = min(bestE, e)
        r = (w[6] * K) >> 32
        pop[r], popE[r] = child, e
        assert st.advance(1, ZERO_WALK, p_comb, 0) == 1
        assert np.array_equal(st.pop, pop), g
        assert np.array_equal(st.popE, popE) and st.bestE == bestE, g
    if p_comb == 0xFFFFFFFF and n == 8:
        assert tie_matters > 20 and cut_matters > 20


def _two_member_trials(n, m0, m1, e0, e1, trials, seed=99):
    # K = 2 with members m0, m1 restored before every generation, crossover
    # forced, mutation off, zero-step walks: the children of `trials`
    # consecutive generations.  The tournament reads only the energy array,
    # so the members get the stand-in energies e0, e1 (< floor(N/2), below
    # every real energy); the child's slot is the one whose energy changed.
    st = O.MemeticState(n, 2, seed, 0)
    base = np.stack([m0, m1]).astype(np.int8)
    out = np.zeros((trials, n), dtype=np.int8)
    for t in range(trials):
        st.pop[:] = base
        st.popE[:] = [e0, e1]
        st.best[:] = m0
        st.best_e[0] = min(e0, e1)
        st.advance(1, ZERO_WALK, 0xFFFFFFFF, 0)
        r = [k for k in range(2) if st.popE[k] != (e0, e1)[k]]
        assert len(r) == 1 and st.popE[r[0]] == npref.energy(st.pop[r[0]])
        out[t] = st.pop[r[0]]
    return out


def test_tournament_prefers_lower_energy():
    # Binary tournament with replacement between a better and a worse
    # member: the better one wins unless both draws name the worse one, so
    # each parent is the better member with probability 3/4 (a reversed
    # comparison gives 1/4, no comparison 1/2).  The members differ at every
    # position, so the child's first entry names the first parent and its
    # last entry the second (the cut lies in 1..N-1).
    n = 24
    rng = np.random.default_rng(4)
    m0 = (1 - 2 * rng.integers(0, 2, n)).astype(np.int8)
    trials = 6000
    kids = _two_member_trials(n, m0, -m0, 0, 1, trials)
    first = np.mean(kids[:, 0] == m0[0])
    second = np.mean(kids[:, n - 1] == m0[n - 1])
    sd = np.sqrt(0.75 * 0.25 / trials)
    assert abs(first - 0.75) < 5 * sd and abs(second - 0.75) < 5 * sd, (first, second)
    # the two tournaments draw independently
    both = np.mean((kids[:, 0] == m0[0]) & (kids[:, n - 1] == m0[n - 1]))
    assert abs(both - 0.5625) < 5 * np.sqrt(0.5625 * 0.4375 / trials), both


def test_crossover_cut_uniform():
    # Two members of equal energy that differ everywhere: every tournament is
    # a tie, so the parents are two independent uniform picks; half the
    # children are copies, and when the parents differ the cut -- the first
    # position taken from the second parent -- is uniform over 1..N-1 (a cut
    # drawn over 0..N-1 or 1..N would add copies: cut 0 or N).
    n = 6
    rng = np.random.default_rng(8)
    m0 = (1 - 2 * rng.integers(0, 2, n)).astype(np.int8)
    trials = 20000
    kids = _two_member_trials(n, m0, -m0, 1, 1, trials)
    copies = np.all(kids == m0, axis=1) | np.all(kids == -m0, axis=1)
    frac = copies.mean()
    assert abs(frac - 0.5) < 5 * np.sqrt(0.25 / trials), frac
    splices = kids[~copies]
    first = np.where(splices[:, :1] == m0[0], m0, -m0)  # the first parent
    cuts = np.argmax(splices != first, axis=1)  # first entry of the second parent
    assert cuts.min() >= 1
    hist = np.bincount(cuts, minlength=n)[1:n]
    exp = len(splices) / (n - 1)
    chi2 = float(np.sum((hist - exp) ** 2 / exp))
    assert chi2 < 25, hist  # 4 degrees of freedom


def test_replacement_slot_uniform():
    # Sampling only (no crossover), zero-step walks, K distinct members with
    # distinct energies: the child is a copy, and the slot it lands in is
    # uniform over the K members.  The slot is seen as the member whose row
    # changed (or none, when a member was copied onto itself).
    n, K, trials = 30, 8, 8000
    st = O.MemeticState(n, K, 5, 1)
    assert len({tuple(r) for r in st.pop}) == K
    base, baseE = st.pop.copy(), st.popE.copy()
    hits = np.zeros(K, dtype=np.int64)
    same = 0
    for _ in range(trials):
        st.pop[:] = base
        st.popE[:] = baseE
        st.advance(1, ZERO_WALK, 0, 0)
        changed = [k for k in range(K) if not np.array_equal(st.pop[k], base[k])]
        assert len(changed) <= 1
        if changed:
            hits[changed[0]] += 1
        else:
            same += 1
    # sampled member and slot are independent uniform picks: a copy onto
    # itself has probability 1/K, every other slot (K-1)/K^2
    assert abs(same / trials - 1 / K) < 5 * np.sqrt((1 / K) * (1 - 1 / K) / trials)
    exp = trials * (K - 1) / K / K
    chi2 = float(np.sum((hits - exp) ** 2 / exp))
    assert chi2 < 30, hits  # 7 degrees of freedom
