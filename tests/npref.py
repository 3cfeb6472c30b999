"""Independent numpy statements of the objective, used to pin the oracle.

Test infrastructure.  Written from the definitions (Eq. 1 and Eq. 2) with
numpy.correlate rather than the oracle's loops, plus a pure-Python Philox
written from its published definition.
"""
import numpy as np


def corr(s):
    """C_k for k = 1..n-1 (Eq. 1) via numpy.correlate."""
    s = np.asarray(s, dtype=np.int64)
    n = len(s)
    full = np.correlate(s, s, mode="full")  # lags -(n-1)..(n-1)
    return full[n:]


def energy(s):
    """E = sum_k C_k^2 (Eq. 2)."""
    c = corr(s)
    return int(np.dot(c, c))


def energies_rows(S):
    """Energies of every row of the +-1 matrix S (vectorised over rows)."""
    S = np.asarray(S, dtype=np.int64)
    n = S.shape[1]
    e = np.zeros(S.shape[0], dtype=np.int64)
    for k in range(1, n):
        c = np.sum(S[:, : n - k] * S[:, k:], axis=1)
        e += c * c
    return e


def flip_energies(s):
    """E(flip(s, i)) for every i, by rebuilding each neighbour."""
    s = np.asarray(s, dtype=np.int64)
    n = len(s)
    S = np.tile(s, (n, 1))
    S[np.arange(n), np.arange(n)] *= -1
    return energies_rows(S)


M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox(ctr, key):
    """Philox4x32-10 in pure Python (SC'11 definition)."""
    x0, x1, x2, x3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
        p0, p1 = M0 * x0, M1 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ x3 ^ k1) & MASK, p0 & MASK
    return [x0, x1, x2, x3]
