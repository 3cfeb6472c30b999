"""Seeded synthetic inputs and workload recipes.

This module is shared by the tests, the benchmark, the GPU binding and the
CPU oracle's callers.  It holds sizes, seeds and numpy generators only -- none
of the method's arithmetic.  LABS has no dataset: an instance is a length N,
and every input below is drawn from a fixed numpy seed or, inside the method,
from the counter-based generator keyed by the workload seed.

Workloads (sizes follow the paper's setting, Sec. III and Sec. V):
  memetic_n20   N=20, one population of K=100, 50 generations, p_comb=0.9,
                p_mutate=1/N, walk length floor(N/2)+U[0,N], tenure
                U[1, floor(N/10)+1]; brute force of all 2^20 sequences.
  tabu_n64      4096 independent walks at N=64 from random starts, 4N steps,
                tenure U[floor(N/10), floor(N/5)].
  tabu_uneven   8192 walks with N uniform in {48..120}, 3N steps, same tenure.
  tabu_n120     4096 walks at N=120, 4N steps, same tenure.
  memetic_n120  256 populations of K=100 at N=120, memetic_n20's rules.
  serving       Poisson stream of solve requests, N uniform in {32..128},
                16 populations x 200 generations each.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Rule identifiers (the numbering used by both the library ABI and the
# oracle's entry points).
STEPS_FIXED, STEPS_MULT_N, STEPS_PAPER, STEPS_RANGE = 0, 1, 2, 3
TENURE_LINEAR, TENURE_PAPER = 0, 1

P_COMB_090 = 3865470566  # floor(0.9 * 2^32)


@dataclass(frozen=True)
class Rules:
    """Walk length / tenure rule as plain integers."""
    steps_rule: int
    steps_a: int
    tenure_rule: int
    lo_num: int
    lo_den: int
    lo_add: int
    hi_num: int
    hi_den: int
    hi_add: int
    aspiration: int = 1
    # bounds of STEPS_RANGE: walk length uniform in
    # [floor(slo_num N / slo_den), floor(shi_num N / shi_den)]
    slo_num: int = 0
    slo_den: int = 1
    shi_num: int = 0
    shi_den: int = 1

    def as_dict(self):
        return dict(steps_rule=self.steps_rule, steps_a=self.steps_a,
                    tenure_rule=self.tenure_rule, lo_num=self.lo_num,
                    lo_den=self.lo_den, lo_add=self.lo_add, hi_num=self.hi_num,
                    hi_den=self.hi_den, hi_add=self.hi_add,
                    aspiration=self.aspiration, slo_num=self.slo_num, slo_den=self.slo_den,
                    shi_num=self.shi_num, shi_den=self.shi_den)


# Walk length 4N (or 3N), tenure U[floor(N/10), floor(N/5)].
def rules_tabu(mult: int) -> Rules:
    return Rules(STEPS_MULT_N, mult, TENURE_LINEAR, 1, 10, 0, 1, 5, 0, 1)


# Walk length floor(N/2) + U[0, N], tenure U[1, floor(N/10) + 1].
RULES_MEMETIC = Rules(STEPS_PAPER, 0, TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1)

# The paper's own rule: tenure [floor(0.1 T), floor(0.12 T)], no aspiration.
RULES_PAPER_LITERAL = Rules(STEPS_PAPER, 0, TENURE_PAPER, 0, 1, 0, 0, 1, 0, 0)


@dataclass(frozen=True)
class TabuWorkload:
    name: str
    walks: int
    n: int | None          # uniform length, or None for per-walk lengths
    n_lo: int = 0
    n_hi: int = 0
    rules: Rules = field(default_factory=lambda: rules_tabu(4))
    seed: int = 0

    def lengths(self) -> np.ndarray:
        if self.n is not None:
            return np.full(self.walks, self.n, dtype=np.int32)
        return uneven_lengths(self.walks, self.n_lo, self.n_hi, self.seed)


@dataclass(frozen=True)
class MemeticWorkload:
    name: str
    n: int
    K: int
    pops: int
    generations: int
    rules: Rules = RULES_MEMETIC
    p_comb: int = P_COMB_090
    seed: int = 0


TABU_N64 = TabuWorkload("tabu_n64", 4096, 64, rules=rules_tabu(4), seed=1001)
TABU_UNEVEN = TabuWorkload("tabu_uneven", 8192, None, 48, 120, rules=rules_tabu(3), seed=1002)
# The longest class (four neighbours per lane), same rules as tabu_n64.
TABU_N256 = TabuWorkload("tabu_n256", 4096, 256, rules=rules_tabu(4), seed=1005)
# Both classes of N > 128 (four neighbours per lane), mixed.
TABU_LONG_UNEVEN = TabuWorkload("tabu_long_uneven", 4096, None, 129, 256, rules=rules_tabu(4),
                                seed=1007)
# The top of the N = 64..120 range in one length (two neighbours per lane).
TABU_N120 = TabuWorkload("tabu_n120", 4096, 120, rules=rules_tabu(4), seed=1008)
# Short walks, as many as fill the device two walks per wavefront.
TABU_N32 = TabuWorkload("tabu_n32", 16384, 32, rules=rules_tabu(4), seed=1009)
TABU_WORKLOADS = {w.name: w for w in (TABU_N64, TABU_UNEVEN, TABU_N120, TABU_N256,
                                      TABU_LONG_UNEVEN, TABU_N32)}
MEMETIC_N20 = MemeticWorkload("memetic_n20", 20, 100, 1, 50, seed=1000)
MEMETIC_N120 = MemeticWorkload("memetic_n120", 120, 100, 256, 100000, seed=1003)
SERVING_SEED = 1004
SERVING_N_RANGE = (32, 128)
SERVING_POPS, SERVING_GENS = 16, 200


def uneven_lengths(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Lengths drawn uniformly from {lo..hi} (inclusive)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count, dtype=np.int64).astype(np.int32)


def random_pm1(count: int, n: int, stride: int, seed: int) -> np.ndarray:
    """count x stride int8 rows, the first n entries uniform +-1, the rest 0."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, stride), dtype=np.int8)
    out[:, :n] = (1 - 2 * rng.integers(0, 2, size=(count, n))).astype(np.int8)
    return out


def random_pm1_ragged(ns: np.ndarray, stride: int, seed: int) -> np.ndarray:
    """One +-1 row per entry of ns (row b has ns[b] entries, zero padded)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((len(ns), stride), dtype=np.int8)
    bits = rng.integers(0, 2, size=(len(ns), stride))
    for b, n in enumerate(ns):
        out[b, :n] = (1 - 2 * bits[b, :n]).astype(np.int8)
    return out


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def serving_requests(count: int, seed: int = SERVING_SEED):
    """(N, request seed) pairs of the serving workload."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(SERVING_N_RANGE[0], SERVING_N_RANGE[1] + 1, size=count)
    seeds = rng.integers(1, 2**62, size=count, dtype=np.int64)
    return [(int(n), int(s)) for n, s in zip(ns, seeds)]
