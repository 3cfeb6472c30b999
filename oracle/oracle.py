"""ctypes binding of the plain CPU oracle in ``labs_oracle.c``.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously-correct
statement of what the GPU library computes.  Only ``tests/``, the smoke check
in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import
this module; the product package never does, and the two share no code.

Energies come back as int64 numpy arrays; sequences are int8 arrays of +-1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "labs_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
MAX_N = 256  # longest sequence of the walk and memetic routines

STEPS_FIXED, STEPS_MULT_N, STEPS_PAPER, STEPS_RANGE = 0, 1, 2, 3
TENURE_LINEAR, TENURE_PAPER = 0, 1
TAG_START, TAG_STEP, TAG_LEN, TAG_INIT, TAG_GEN, TAG_MUT = 1, 2, 3, 4, 5, 6


def build() -> str:
    """Compile the oracle with gcc -O2 (plain C99, no intrinsics)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lpthread"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_draw.argtypes = [u64, u32, u32, u32, u32, P]
        L.orc_autocorrelation.argtypes = [P, ctypes.c_int, P]
        L.orc_energy.argtypes = [P, ctypes.c_int]
        L.orc_energy.restype = i64
        L.orc_energy_batch.argtypes = [P, P, i32, i32, i64, P]
        L.orc_bruteforce_min.argtypes = [ctypes.c_int, P, P]
        L.orc_skew_sequence.argtypes = [ctypes.c_int, ctypes.c_uint64, P]
        L.orc_skew_bruteforce_min.argtypes = [ctypes.c_int, P, P, P]
        L.orc_non_skew.argtypes = [P, ctypes.c_int]
        L.orc_skew_deviation.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.orc_neighbour_energies_recompute.argtypes = [P, ctypes.c_int, P]
        L.orc_neighbour_energies_tables.argtypes = [P, ctypes.c_int, P]
        R = ctypes.POINTER(_Rule)
        L.orc_walk_schedule.argtypes = [ctypes.c_int, R, u64, u32, u32, P, P, P]
        L.orc_random_start.argtypes = [ctypes.c_int, u64, u32, P]
        L.orc_tabu_walk.argtypes = [ctypes.c_int, P, u64, u32, u32, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, P, P, P, P, P, P]
        L.orc_tabu_batch.argtypes = [i64, P, i32, P, i32, u64, R, P, P, P, ctypes.c_int]
        L.orc_memetic_init.argtypes = [ctypes.c_int, ctypes.c_int, u64, u32, P, P, P, P]
        L.orc_memetic_advance.argtypes = [ctypes.c_int, ctypes.c_int, u32, u32, R,
                                          u64, u32, i64, i64, i64, P, P, P, P, P]
        L.orc_memetic_advance.restype = i64
        L.orc_memetic_advance_batched.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32,
                                                  u32, R, u64, u32, i64, i64, i64, P, P, P, P, P]
        L.orc_memetic_advance_batched.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


_RULE_FIELDS = ("steps_rule", "steps_a", "tenure_rule", "lo_num", "lo_den", "lo_add",
                "hi_num", "hi_den", "hi_add", "aspiration", "slo_num", "slo_den", "shi_num",
                "shi_den")


class _Rule(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int) for f in _RULE_FIELDS]


@dataclass(frozen=True)
class Schedule:
    """Walk length and tenure rule (see ``orc_walk_schedule``); the last four
    fields bound the walk length of STEPS_RANGE."""
    steps_rule: int = STEPS_MULT_N
    steps_a: int = 4
    tenure_rule: int = TENURE_LINEAR
    lo_num: int = 1
    lo_den: int = 10
    lo_add: int = 0
    hi_num: int = 1
    hi_den: int = 5
    hi_add: int = 0
    aspiration: int = 1
    slo_num: int = 0
    slo_den: int = 1
    shi_num: int = 0
    shi_den: int = 1

    def rule(self) -> "_Rule":
        return _Rule(*(getattr(self, f) for f in _RULE_FIELDS))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed: int, entity: int, gen: int, index: int, tag: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_draw(seed, entity, gen, index, tag, _p(out))
    return out


def _seq(s) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(s, dtype=np.int8))


def autocorrelation(s) -> np.ndarray:
    s = _seq(s)
    C = np.zeros(len(s), dtype=np.int64)
    lib().orc_autocorrelation(_p(s), len(s), _p(C))
    return C


def energy(s) -> int:
    s = _seq(s)
    return int(lib().orc_energy(_p(s), len(s)))


def energy_batch(seqs: np.ndarray, ns=None, n_uniform: int = 0) -> np.ndarray:
    seqs = np.ascontiguousarray(seqs, dtype=np.int8)
    B, stride = seqs.shape
    out = np.zeros(B, dtype=np.int64)
    nsa = None if ns is None else np.ascontiguousarray(ns, dtype=np.int32)
    lib().orc_energy_batch(_p(seqs), None if nsa is None else _p(nsa), n_uniform,
                           stride, B, _p(out))
    return out


def bruteforce_min(n: int):
    emin = np.zeros(1, dtype=np.int64)
    cnt = np.zeros(1, dtype=np.int64)
    if lib().orc_bruteforce_min(n, _p(emin), _p(cnt)) != 0:
        raise ValueError("n out of range")
    return int(emin[0]), int(cnt[0])


def skew_sequence(n: int, code: int) -> np.ndarray:
    """The skew-symmetric sequence of odd length n with free spins s_0..s_c
    from code (Sec. II.C)."""
    s = np.zeros(n, dtype=np.int8)
    if lib().orc_skew_sequence(n, code, _p(s)) != 0:
        raise ValueError("n must be odd and in [1, 63]")
    return s


def skew_bruteforce_min(n: int):
    """(E_min, count, argmin) over the skew-symmetric sequences of odd n."""
    emin = np.zeros(1, dtype=np.int64)
    cnt = np.zeros(1, dtype=np.int64)
    arg = np.zeros(n, dtype=np.int8)
    if lib().orc_skew_bruteforce_min(n, _p(emin), _p(cnt), _p(arg)) != 0:
        raise ValueError("n must be odd and in [1, 45]")
    return int(emin[0]), int(cnt[0]), arg


def non_skew(t) -> int:
    """n_non-skew of an odd-length sequence (App. A); -1 for even lengths."""
    t = _seq(t)
    return int(lib().orc_non_skew(_p(t), len(t)))


def skew_deviation(s, with_insertion: bool = False) -> int:
    """d(S) of App. A (odd N: rotations; even N: rotation + one deletion,
    and one insertion too when with_insertion)."""
    s = _seq(s)
    if not 1 <= len(s) <= MAX_N:
        raise ValueError(f"sequence length must be in [1, {MAX_N}]")
    return int(lib().orc_skew_deviation(_p(s), len(s), 1 if with_insertion else 0))


def neighbour_energies(s, recompute: bool = True) -> np.ndarray:
    s = _seq(s)
    if not 1 <= len(s) <= MAX_N:
        raise ValueError(f"sequence length must be in [1, {MAX_N}]")
    out = np.zeros(len(s), dtype=np.int64)
    f = lib().orc_neighbour_energies_recompute if recompute else lib().orc_neighbour_energies_tables
    f(_p(s), len(s), _p(out))
    return out


def walk_schedule(n: int, sched: Schedule, seed: int, entity: int, gen: int):
    T = np.zeros(1, dtype=np.int32)
    lo = np.zeros(1, dtype=np.int32)
    hi = np.zeros(1, dtype=np.int32)
    r = sched.rule()
    rc = lib().orc_walk_schedule(n, ctypes.byref(r), seed, entity, gen, _p(T), _p(lo), _p(hi))
    if rc != 0:
        raise ValueError("invalid walk schedule")
    return int(T[0]), int(lo[0]), int(hi[0])


def random_start(n: int, seed: int, walk: int) -> np.ndarray:
    s = np.zeros(n, dtype=np.int8)
    lib().orc_random_start(n, seed, walk, _p(s))
    return s


def tabu_walk(start, seed: int, entity: int, gen: int, steps: int, lo: int, hi: int,
              aspiration: int = 1, recompute: bool = False, want_trace: bool = False,
              want_expiry: bool = False):
    """One walk; returns (best, best_e, final_e, trace, trace_e), and with
    want_expiry a sixth entry: the tabuList value the move of step t receives
    (the last step at which it is tabu), one per step."""
    s = _seq(start)
    n = len(s)
    best = np.zeros(n, dtype=np.int8)
    be = np.zeros(1, dtype=np.int64)
    fe = np.zeros(1, dtype=np.int64)
    tr = np.zeros(max(steps, 1), dtype=np.int16) if want_trace else None
    te = np.zeros(max(steps, 1), dtype=np.int64) if want_trace else None
    tx = np.zeros(max(steps, 1), dtype=np.int64) if want_expiry else None
    rc = lib().orc_tabu_walk(n, _p(s), seed, entity, gen, steps, lo, hi, aspiration,
                             1 if recompute else 0, _p(best), _p(be), _p(fe),
                             None if tr is None else _p(tr), None if te is None else _p(te),
                             None if tx is None else _p(tx))
    if rc != 0:
        raise ValueError("walk failed (invalid arguments or no admissible move)")
    if want_trace:
        tr, te = tr[:steps], te[:steps]
    if want_expiry:
        return best, int(be[0]), int(fe[0]), tr, te, tx[:steps]
    return best, int(be[0]), int(fe[0]), tr, te


def tabu_batch(W: int, sched: Schedule, seed: int, ns=None, n_uniform: int = 0,
               starts=None, stride: int = 128, nthreads: int = 1):
    """Stand-alone walks 0..W-1 (walk id = index); returns (best_seq, best_e, final_e)."""
    nsa = None if ns is None else np.ascontiguousarray(ns, dtype=np.int32)
    st = None if starts is None else np.ascontiguousarray(starts, dtype=np.int8)
    if st is not None:
        stride = st.shape[1]
    best = np.zeros((W, stride), dtype=np.int8)
    be = np.zeros(W, dtype=np.int64)
    fe = np.zeros(W, dtype=np.int64)
    r = sched.rule()
    rc = lib().orc_tabu_batch(W, None if nsa is None else _p(nsa), n_uniform,
                              None if st is None else _p(st), stride, seed, ctypes.byref(r),
                              _p(best), _p(be), _p(fe), nthreads)
    if rc != 0:
        raise ValueError("tabu batch failed")
    return best, be, fe


class MemeticState:
    """One replica of Alg. 1: population, energies, best, generation, hit."""

    def __init__(self, n: int, K: int, seed: int, pop_id: int):
        self.n, self.K, self.seed, self.pop_id = n, K, seed, pop_id
        self.pop = np.zeros((K, n), dtype=np.int8)
        self.popE = np.zeros(K, dtype=np.int64)
        self.best = np.zeros(n, dtype=np.int8)
        self.best_e = np.zeros(1, dtype=np.int64)
        self.hit_gen = np.full(1, -1, dtype=np.int64)
        self.gen = 0
        lib().orc_memetic_init(n, K, seed, pop_id, _p(self.pop), _p(self.popE),
                               _p(self.best), _p(self.best_e))

    def advance(self, n_gens: int, sched: Schedule, p_comb: int, p_mut: int,
                target: int = -1, children: int = 0) -> int:
        """Alg. 1 generations (children == 0), or the batched-generation
        variant with `children` children per generation (1 reproduces Alg. 1
        through the batched code)."""
        r = sched.rule()
        if children == 0:
            done = lib().orc_memetic_advance(
                self.n, self.K, p_comb, p_mut, ctypes.byref(r),
                self.seed, self.pop_id, self.gen, n_gens, target, _p(self.pop),
                _p(self.popE), _p(self.best), _p(self.best_e), _p(self.hit_gen))
        else:
            done = lib().orc_memetic_advance_batched(
                self.n, self.K, children, p_comb, p_mut, ctypes.byref(r),
                self.seed, self.pop_id, self.gen, n_gens, target, _p(self.pop),
                _p(self.popE), _p(self.best), _p(self.best_e), _p(self.hit_gen))
        if done < 0:
            raise ValueError("memetic advance failed")
        self.gen += int(done)
        return int(done)

    @property
    def bestE(self) -> int:
        return int(self.best_e[0])

    @property
    def hit(self) -> int:
        return int(self.hit_gen[0])

    def copy(self) -> "MemeticState":
        c = MemeticState.__new__(MemeticState)
        c.n, c.K, c.seed, c.pop_id, c.gen = self.n, self.K, self.seed, self.pop_id, self.gen
        c.pop, c.popE, c.best = self.pop.copy(), self.popE.copy(), self.best.copy()
        c.best_e, c.hit_gen = self.best_e.copy(), self.hit_gen.copy()
        return c


def p_mut_inv_n(n: int) -> int:
    """Mutation threshold for p_mutate = 1/N (Sec. III.A): floor(2^32 / N)."""
    return (1 << 32) // n


P_COMB_090 = int(0.9 * (1 << 32))  # 3865470566: randReal < 0.9
