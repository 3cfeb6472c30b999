"""Pins of the oracle's objective (Eq. 1-2), neighbourhood scoring and RNG.

Each check compares the oracle with something other than itself: values the
paper prints (Table "labs_results"), published known-answer vectors, closed
forms, textbook Barker sequences, exact symmetries (Sec. II.B-C) and
exhaustive enumeration written independently in numpy.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests import npref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table():
    rows = []
    with open(os.path.join(GOLDEN, "labs_results_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, oe, ne, omf, nmf, hexs, d = line.split()
            rows.append((int(n), int(oe), int(ne), float(omf), float(nmf), hexs, int(d)))
    return rows


def decode_hex(hexs, n):
    """Most-significant bit first; the first n bits are the sequence, bit 1 -> -1."""
    bits = []
    for ch in hexs:
        v = int(ch, 16)
        bits += [(v >> (3 - b)) & 1 for b in range(4)]
    assert len(bits) >= n and not any(bits[n:]), "padding bits must be zero"
    return np.array([1 - 2 * b for b in bits[:n]], dtype=np.int8)


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr, key, want = v[0:4], v[4:6], v[6:10]
        assert list(O.philox4x32_10(ctr, key)) == want
        assert npref.philox(ctr, key) == want


def test_draw_counter_layout():
    # key = (seed low, seed high), counter = (entity, gen, index, tag)
    seed = 0x0123456789ABCDEF
    got = O.draw(seed, 7, 11, 13, 2)
    want = npref.philox([7, 11, 13, 2], [seed & 0xFFFFFFFF, seed >> 32])
    assert list(got) == want


@pytest.mark.parametrize("row", _table(), ids=lambda r: f"N{r[0]}-{r[5][:6]}")
def test_paper_table_energies(row):
    n, old_e, new_e, old_mf, new_mf, hexs, _ = row
    s = decode_hex(hexs, n)
    assert O.energy(s) == new_e
    assert npref.energy(s) == new_e
    # Eq. 3: F = N^2 / (2E), printed to two decimals
    assert round(n * n / (2 * new_e), 2) == pytest.approx(new_mf, abs=1e-9)
    assert round(n * n / (2 * old_e), 2) == pytest.approx(old_mf, abs=1e-9)
    # both printed energies obey E = floor(N/2) (mod 4): C_k = N-k (mod 2)
    assert new_e % 4 == (n // 2) % 4 and old_e % 4 == (n // 2) % 4


def test_paper_n92_pair_is_alternation_image():
    # the two N = 92 sequences (printed as non-equivalent under the two
    # symmetries of Sec. II.B) map to each other under s_i -> (-1)^i s_i up to
    # reversal/complement, a third exact symmetry of Eq. 2
    rows = [r for r in _table() if r[0] == 92]
    a, b = (decode_hex(r[5], 92) for r in rows)
    alt = np.array([(-1) ** i for i in range(92)], dtype=np.int8)
    images = []
    for x in (a * alt,):
        for y in (x, x[::-1]):
            images += [y, -y]
    assert any(np.array_equal(b, y) for y in images)
    assert O.energy(a) == O.energy(b) == 490


@pytest.mark.parametrize("n", [3, 4, 5, 17, 64, 120, 128, 129, 200, 256])
def test_closed_forms(n):
    ones = np.ones(n, dtype=np.int8)
    alt = np.array([(-1) ** i for i in range(n)], dtype=np.int8)
    k = np.arange(n)
    assert list(O.autocorrelation(ones)) == list(n - k)
    assert list(O.autocorrelation(alt)[1:]) == list(((-1) ** k[1:]) * (n - k[1:]))
    e = (n - 1) * n * (2 * n - 1) // 6
    assert O.energy(ones) == e and O.energy(alt) == e


BARKER = {
    2: "++", 3: "++-", 4: "++-+", 5: "+++-+", 7: "+++--+-",
    11: "+++---+--+-", 13: "+++++--++-+-+",
}


@pytest.mark.parametrize("n", sorted(BARKER))
def test_barker_sequences(n):
    s = np.array([1 if c == "+" else -1 for c in BARKER[n]], dtype=np.int8)
    c = O.autocorrelation(s)[1:]
    assert np.all(np.abs(c) <= 1)
    assert O.energy(s) == n // 2


def _numpy_bruteforce(n):
    codes = np.arange(1 << n, dtype=np.int64)
    S = (1 - 2 * ((codes[:, None] >> np.arange(n)) & 1)).astype(np.int8)
    e = npref.energies_rows(S)
    m = int(e.min())
    return m, int(np.sum(e == m))


@pytest.mark.parametrize("n", list(range(3, 17)) + [20])
def test_bruteforce(n):
    emin, cnt = O.bruteforce_min(n)
    assert (emin, cnt) == _numpy_bruteforce(n)
    # lower bound floor(N/2), attained exactly at the Barker lengths
    assert emin >= n // 2
    assert (emin == n // 2) == (n in BARKER)
    # complementation has no fixed point, so optima come in pairs
    assert cnt % 2 == 0


def test_autocorrelation_matches_numpy():
    rng = np.random.default_rng(5)
    for n in [3, 8, 31, 64, 65, 97, 128]:
        s = (1 - 2 * rng.integers(0, 2, n)).astype(np.int8)
        assert list(O.autocorrelation(s)[1:]) == list(npref.corr(s))
        assert O.autocorrelation(s)[0] == n


def test_energy_batch_ragged():
    rng = np.random.default_rng(6)
    ns = rng.integers(3, 129, size=40).astype(np.int32)
    S = np.zeros((40, 128), dtype=np.int8)
    for b, n in enumerate(ns):
        S[b, :n] = 1 - 2 * rng.integers(0, 2, n)
    got = O.energy_batch(S, ns=ns)
    assert list(got) == [npref.energy(S[b, :n]) for b, n in enumerate(ns)]


def test_symmetries():
    rng = np.random.default_rng(7)
    for n in [5, 20, 64, 99, 128]:
        s = (1 - 2 * rng.integers(0, 2, n)).astype(np.int8)
        alt = np.array([(-1) ** i for i in range(n)], dtype=np.int8)
        C = O.autocorrelation(s)
        assert list(O.autocorrelation(-s)) == list(C)          # complementation
        assert list(O.autocorrelation(s[::-1].copy())) == list(C)  # reversal
        Ca = O.autocorrelation(s * alt)                         # alternation
        k = np.arange(n)
        assert list(Ca) == list(((-1) ** k) * C)
        assert O.energy(s * alt) == O.energy(s) == O.energy(-s[::-1].copy())


def test_skew_symmetric_odd_lags_vanish():
    # Eq. 4: N = 2n-1, s_{n+i} = (-1)^i s_{n-i} (1-based) => C_k = 0 for odd k
    rng = np.random.default_rng(8)
    for N in [5, 13, 63, 99, 127]:
        n = (N + 1) // 2
        s = np.zeros(N + 1, dtype=np.int8)  # 1-based
        s[1 : n + 1] = 1 - 2 * rng.integers(0, 2, n)
        for i in range(1, n):
            s[n + i] = (-1) ** i * s[n - i]
        C = O.autocorrelation(s[1:])
        assert all(C[k] == 0 for k in range(1, N, 2))


# ---------------------------------------------------------------------------
# The search restricted to skew-symmetric sequences (Sec. II.C)
# ---------------------------------------------------------------------------
def _numpy_skew_bruteforce(n):
    """Every sequence of odd length n enumerated by numpy, kept when Eq. 4's
    condition s_{c+i} = (-1)^i s_{c-i} holds; energies by numpy."""
    c = (n - 1) // 2
    codes = np.arange(1 << n, dtype=np.int64)
    S = (1 - 2 * ((codes[:, None] >> np.arange(n)) & 1)).astype(np.int8)
    keep = np.ones(len(S), dtype=bool)
    for i in range(1, c + 1):
        keep &= S[:, c + i] == (-1) ** i * S[:, c - i]
    K, kc = S[keep], codes[keep]
    e = npref.energies_rows(K)
    m = int(e.min())
    # of the minima with s_0 = +1, the one whose free spins s_0..s_c read as
    # the smallest integer (bit i set <=> s_i = -1)
    free = kc & ((1 << (c + 1)) - 1)
    at = (e == m) & (K[:, 0] == 1)
    arg = K[at][np.argmin(free[at])]
    return m, int(np.sum(e == m)), arg, len(K)


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13, 15, 17])
def test_skew_bruteforce_against_numpy(n):
    m, cnt, arg, size = _numpy_skew_bruteforce(n)
    assert size == 2 ** ((n + 1) // 2)  # the subspace's size (Sec. II.C)
    em, c, a = O.skew_bruteforce_min(n)
    assert (em, c) == (m, cnt)
    assert np.array_equal(a, arg)


def test_skew_sequence_is_the_subspace():
    # the code -> sequence map hits every skew-symmetric sequence once, and
    # each has C_k = 0 at odd k
    for n in (1, 3, 9, 15, 21):
        c = (n - 1) // 2
        seen = set()
        for code in range(1 << (c + 1)):
            s = O.skew_sequence(n, code)
            assert all(s[c + i] == (-1) ** i * s[c - i] for i in range(1, c + 1))
            assert all(s[i] == (-1 if (code >> i) & 1 else 1) for i in range(c + 1))
            C = O.autocorrelation(s)
            assert all(C[k] == 0 for k in range(1, n, 2))
            seen.add(s.tobytes())
        assert len(seen) == 1 << (c + 1)


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13, 15, 17, 19, 21])
def test_skew_minimum_against_unrestricted(n):
    # restricting the space never helps; at the odd Barker lengths the
    # optimum (E = floor(N/2)) is skew-symmetric, and at N = 19 no optimum is
    # (the paper's point that odd N need not have skew-symmetric optima)
    em, c, a = O.skew_bruteforce_min(n)
    gm, gc = O.bruteforce_min(n)
    assert em >= gm and O.energy(a) == em
    if n in BARKER:
        assert em == gm == n // 2
    if n == 19:
        assert em > gm
    assert c % 2 == 0 and c <= gc or em > gm


def test_congruences():
    rng = np.random.default_rng(9)
    for n in [3, 10, 33, 64, 101, 128]:
        for _ in range(5):
            s = (1 - 2 * rng.integers(0, 2, n)).astype(np.int8)
            e = O.energy(s)
            assert e % 4 == (n // 2) % 4
            nb = O.neighbour_energies(s, recompute=False)
            assert np.all((nb - e) % 4 == 0)


def test_neighbour_energies_three_ways():
    rng = np.random.default_rng(10)
    for n in [3, 4, 7, 20, 64, 65, 120, 128]:
        s = (1 - 2 * rng.integers(0, 2, n)).astype(np.int8)
        rec = O.neighbour_energies(s, recompute=True)
        tab = O.neighbour_energies(s, recompute=False)
        ref = npref.flip_energies(s)
        assert list(rec) == list(ref)
        assert list(tab) == list(ref)
        # closed form of the change: flipping s_j changes C_k by -2 s_j t_jk
        # with t_jk = s_{j+k} + s_{j-k} (missing terms 0), hence
        # dE_j = 4 (sum_k t_jk^2 - s_j sum_k t_jk C_k)
        C = npref.corr(s)
        sl = s.astype(np.int64)
        for j in range(n):
            t = np.array([(sl[j + k] if j + k < n else 0) + (sl[j - k] if j - k >= 0 else 0)
                          for k in range(1, n)], dtype=np.int64)
            de = 4 * (int(t @ t) - int(sl[j]) * int(t @ C))
            assert tab[j] == npref.energy(s) + de


def test_neighbour_energies_exhaustive_small():
    for n in range(3, 11):
        for code in range(1 << n):
            s = np.array([1 - 2 * ((code >> i) & 1) for i in range(n)], dtype=np.int8)
            assert list(O.neighbour_energies(s, recompute=False)) == list(npref.flip_energies(s))


# ---------------------------------------------------------------------------
# Deviation from skew-symmetry, d(S) (App. A)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("row", _table(), ids=lambda r: f"N{r[0]}-{r[5][:6]}")
def test_skew_deviation_paper_column(row):
    # the d(S) column of Table "labs_results": odd N over rotations, even N
    # over rotation + one deletion
    n, _, _, _, _, hexs, d = row
    s = decode_hex(hexs, n)
    assert O.skew_deviation(s) == d
    # allowing an insertion as well can only lower it (odd N: no change)
    di = O.skew_deviation(s, with_insertion=True)
    assert di <= d and (n % 2 == 0 or di == d)


def _skew_symmetric(c, rng):
    # odd length 2c + 1: free centre half, s_{c+i} = (-1)^i s_{c-i} (Sec. II.C)
    left = rng.choice(np.array([-1, 1], dtype=np.int8), size=c + 1)
    s = np.zeros(2 * c + 1, dtype=np.int8)
    s[: c + 1] = left
    for i in range(1, c + 1):
        s[c + i] = (-1) ** i * s[c - i]
    return s


def test_skew_deviation_constructions():
    rng = np.random.default_rng(8)
    for c in (1, 5, 30, 59, 100):
        s = _skew_symmetric(c, rng)
        n = len(s)
        assert O.non_skew(s) == 0 and O.skew_deviation(s) == 0
        # skew-symmetric sequences have C_k = 0 at every odd k
        C = O.autocorrelation(s)
        assert not np.any(C[1::2])
        # breaking k pairs (flipping right-half elements) gives n_non-skew k
        k = min(c, 7)
        t = s.copy()
        t[c + 1 + rng.choice(c, size=k, replace=False)] *= -1
        assert O.non_skew(t) == k and O.skew_deviation(t) <= k
        # rotations do not change d
        for r in (1, n // 2, n - 1):
            assert O.skew_deviation(np.roll(t, -r)) == O.skew_deviation(t)
        # an even sequence one insertion away from a skew-symmetric one
        # (some deletion undoes it): d = 0
        for i in (0, c, n):
            e = np.insert(s, i, np.int8(1 if i % 2 else -1))
            assert O.skew_deviation(e) == 0
    assert O.non_skew(np.ones(4, dtype=np.int8)) == -1


def test_skew_deviation_bounds():
    # d <= the unrotated value; d(S) = d(-S) = d(reversed S) (the condition
    # is invariant under negation; reversal maps i -> -i pairs onto themselves)
    rng = np.random.default_rng(9)
    for n in (9, 10, 31, 64, 65, 120):
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=n)
        d = O.skew_deviation(s)
        if n % 2:
            assert d <= O.non_skew(s)
        else:
            assert d <= O.non_skew(s[:-1]) and d <= O.non_skew(s[1:])
        assert O.skew_deviation(-s) == d
        assert O.skew_deviation(s[::-1].copy()) == d
        assert 0 <= d <= (n - 1) // 2
