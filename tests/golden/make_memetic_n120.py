"""Write memetic_n120_deep.txt: the oracle's results for the N = 120 memetic
workload (Alg. 1, replicas of K = 100, seed 1003, walk floor(N/2) + U[0, N]
steps, tenure U[1, floor(N/10) + 1], aspiration), deeper than a GPU test can
afford to recompute:

  full   all 256 replicas after 1000 generations
  long   replicas 0..3 after 25000, 50000, 75000 and 100000 generations
  hist   every improvement of the best of replicas 0..3 over the 100000
         generations: the generation count at which it happened and the
         new best energy

Only the oracle computes these values.

    python tests/golden/make_memetic_n120.py [--threads 8]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2504_00987_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "memetic_n120_deep.txt")
FULL_GENS = 1000
LONG_REPLICAS = 4
LONG_CHECKPOINTS = (25000, 50000, 75000, 100000)


def seq_hex(seq) -> str:
    """Bit i set <=> s_i = -1, as a hexadecimal integer."""
    v = 0
    for i, s in enumerate(seq):
        if s < 0:
            v |= 1 << i
    return format(v, "x")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    args = ap.parse_args()
    wl = I.MEMETIC_N120
    r = wl.rules
    sched = O.Schedule(r.steps_rule, r.steps_a, r.tenure_rule, r.lo_num, r.lo_den, r.lo_add,
                       r.hi_num, r.hi_den, r.hi_add, r.aspiration)
    thr = O.p_mut_inv_n(wl.n)

    def full(p):
        st = O.MemeticState(wl.n, wl.K, wl.seed, p)
        st.advance(FULL_GENS, sched, wl.p_comb, thr)
        return p, st.gen, st.bestE, seq_hex(st.best)

    def long(p):
        st = O.MemeticState(wl.n, wl.K, wl.seed, p)
        rows, hist = [], []
        while st.gen < LONG_CHECKPOINTS[-1]:
            e = st.bestE
            st.advance(1, sched, wl.p_comb, thr)
            if st.bestE < e:
                hist.append((p, st.gen, st.bestE))
            if st.gen in LONG_CHECKPOINTS:
                rows.append((p, st.gen, st.bestE, seq_hex(st.best)))
        return rows, hist

    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=args.threads) as ex:
        fut_long = [ex.submit(long, p) for p in range(LONG_REPLICAS)]
        full_rows = list(ex.map(full, range(wl.pops)))
        print(f"full: {time.time() - t0:.0f} s", file=sys.stderr, flush=True)
        long_rows = [row for f in fut_long for row in f.result()[0]]
        hist_rows = [row for f in fut_long for row in f.result()[1]]
    print(f"long: {time.time() - t0:.0f} s", file=sys.stderr, flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle results of the N = 120 memetic workload (Alg. 1; 256 replicas of\n"
                f"# K = {wl.K}, seed {wl.seed}, walk floor(N/2) + U[0, N] steps, tenure\n"
                "# U[1, floor(N/10) + 1], aspiration, p_comb 0.9, mutation 1/N), written by\n"
                "# make_memetic_n120.py from the oracle alone.\n"
                "# columns: section replica generations best_e best_seq (hex: bit i set <=> s_i = -1)\n"
                "# (hist rows: hist replica generations new_best_e)\n")
        for p, g, e, h in full_rows:
            f.write(f"full {p} {g} {e} {h}\n")
        for p, g, e, h in long_rows:
            f.write(f"long {p} {g} {e} {h}\n")
        for p, g, e in hist_rows:
            f.write(f"hist {p} {g} {e}\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
