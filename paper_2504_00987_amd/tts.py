"""Time to solution at small N, the paper-literal configuration (Sec. V.B).

    python -m paper_2504_00987_amd.tts [--n-min 20] [--n-max 36] [--seeds 8]

For every length N the target is the exhaustive minimum (labs_bruteforce_min),
and a run is one labs_memetic_run of R replicas with the paper's own rules
(no aspiration, walk length floor(N/2) + U[0, N], tenure
U[floor(T/10), floor(3T/25)], p_comb = 0.9, mutation 1/N, K = 100) and the
global termination flag: the run ends at the first generation chunk in which
some replica reaches the target.  The time to solution is the wall time of
that call (initial populations included).  The median over seeds is fitted
by a * b^N with ordinary least squares on log(time), as the paper does for
Table `fit`, reporting b with its 95 % confidence interval.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs as I
from .labs import Labs, PERSISTENT


def time_to_solution(lb: Labs, n: int, target: int, replicas: int, seed: int,
                     rules=I.RULES_PAPER_LITERAL, K: int = 100, max_generations: int = 10**7,
                     chunk: int = 16):
    """(seconds, generation of the first hit or None, best energy) of one run."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = lb.memetic_run(K, rules, max_generations, replicas, seed, n_uniform=n, mode=PERSISTENT,
                       chunk=chunk, target=target, stop_all=1)
    dt = time.perf_counter() - t0
    hit = r.hit_gen.cpu().numpy()
    first = int(hit[hit >= 0].min()) if (hit >= 0).any() else None
    return dt, first, int(r.best_e.min().item())


def fit_exponential(ns, times, conf: float = 0.95):
    """OLS of log(time) on N: returns a, b and the confidence intervals."""
    x = np.asarray(ns, dtype=np.float64)
    y = np.log(np.asarray(times, dtype=np.float64))
    A = np.stack([np.ones_like(x), x], axis=1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    resid = y - A @ coef
    dof = max(len(x) - 2, 1)
    s2 = float(resid @ resid) / dof
    cov = s2 * np.linalg.inv(A.T @ A)
    try:
        from scipy.stats import t as student
        q = float(student.ppf(0.5 + conf / 2, dof))
    except ImportError:  # normal approximation
        q = 1.959963984540054
    se = np.sqrt(np.diag(cov))
    lo, hi = coef - q * se, coef + q * se
    return {"a": math.exp(coef[0]), "b": math.exp(coef[1]),
            "a_ci": [math.exp(lo[0]), math.exp(hi[0])], "b_ci": [math.exp(lo[1]), math.exp(hi[1])],
            "points": len(x)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-min", type=int, default=20)
    ap.add_argument("--n-max", type=int, default=36)
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--replicas", type=int, default=1024)
    ap.add_argument("--chunk", type=int, default=16)
    ap.add_argument("--fit-min", default="20,25,30", help="N_min values of the fits")
    args = ap.parse_args()

    lb = Labs(0)
    rows = []
    for n in range(args.n_min, args.n_max + 1):
        t0 = time.perf_counter()
        emin, count, _ = lb.bruteforce_min(n)
        t_brute = time.perf_counter() - t0
        lb.memetic_run(100, I.RULES_PAPER_LITERAL, 4, 64, 1, n_uniform=n)  # warm-up
        runs = [time_to_solution(lb, n, emin, args.replicas, 1000003 * n + s, chunk=args.chunk)
                for s in range(args.seeds)]
        times = [r[0] for r in runs]
        gens = [r[1] for r in runs]
        rows.append({"n": n, "e_min": emin, "minima": count, "exhaustive_s": t_brute,
                     "median_s": float(np.median(times)), "times_s": times,
                     "hit_generations": gens,
                     "reached": all(r[1] is not None for r in runs)})
        print(f"# N={n} E_min={emin} ({count} minima, {t_brute:.2f} s) median TTS "
              f"{rows[-1]['median_s']:.4f} s, hit generations {gens}", file=sys.stderr, flush=True)
    fits = {}
    for nmin in [int(x) for x in args.fit_min.split(",") if x]:
        pts = [r for r in rows if r["n"] >= nmin and r["reached"]]
        if len(pts) >= 3:
            fits[str(nmin)] = fit_exponential([r["n"] for r in pts], [r["median_s"] for r in pts])
    print(json.dumps({"replicas": args.replicas, "K": 100, "seeds": args.seeds,
                      "rules": "paper-literal: no aspiration, T = floor(N/2) + U[0,N], tenure "
                               "U[floor(T/10), floor(3T/25)], p_comb 0.9, mutation 1/N",
                      "rows": rows, "fits": fits}), flush=True)
    lb.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
