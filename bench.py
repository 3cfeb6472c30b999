"""Benchmark of the batched tabu-search hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload tabu_n64|tabu_uneven]

A step is one labs_tabu_batch call over the whole batch (every walk scores
all N single-flip neighbours at each of its steps).  The default workload is
4096 independent walks at N=64 from random starts, 4N = 256 steps each,
tenure U[6, 12] with aspiration.  Inputs are synthetic and seeded (LABS has
no dataset: an instance is its length N).

Prints one JSON line: whole-job flip-neighbour evaluations per second, the
roofline of the walk kernel (integer VALU bound) timed with HIP events on the
stream it runs on, and the CPU oracle timed on a bounded sample of the same
workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X (gfx950): 256 CUs x 64 int32 lanes x 2.4 GHz
PEAK_INT32_OPS = 256 * 64 * 2.4e9
METRIC = "flip-neighbour evals/sec (N=64..120) + time-to-target energy; batched vs plain"


def lag_terms_per_step(n: int) -> int:
    """Sum over neighbours j of L_j = max(N-j, j-1) (1-based): floor((3N^2-2N)/4)."""
    return sum(max(n - j, j - 1) for j in range(1, n + 1))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tabu_n64", choices=["tabu_n64", "tabu_uneven"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-walks", type=int, default=0, help="oracle sample size (0: all walks)")
    ap.add_argument("--cpu-min-s", type=float, default=10.0, help="minimum oracle timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (the reference kernel "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}), flush=True)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "the walks are independent, so several GPUs would each run their own share",
              file=sys.stderr)
        return 2

    import torch
    from paper_2504_00987_amd import inputs as I
    from paper_2504_00987_amd.labs import Labs

    wl = I.TABU_N64 if args.workload == "tabu_n64" else I.TABU_UNEVEN
    ns = wl.lengths()
    W = wl.walks
    steps_per_walk = ns.astype(np.int64) * wl.rules.steps_a
    evals_per_step = int(np.sum(steps_per_walk * ns))
    ops_per_launch = 3 * int(sum(int(s) * lag_terms_per_step(int(n)) for s, n in zip(steps_per_walk, ns)))

    torch.cuda.set_device(0)
    lb = Labs(0)
    dev = torch.device("cuda", 0)
    out = (torch.empty((W, 128), dtype=torch.int8, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev), None)
    uniform = wl.n is not None
    kw = dict(n_uniform=wl.n) if uniform else dict(ns=ns)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        lb.tabu_batch(wl.rules, W, wl.seed, out=out, stream=stream, **kw)
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        lb.tabu_batch(wl.rules, W, wl.seed, out=out, stream=stream, **kw)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    ms_per_step = wall * 1e3 / args.steps
    value = evals_per_step * args.steps / wall
    achieved = ops_per_launch / (kernel_ms * 1e-3)
    launch = lb.get_launch(int(ns.max()))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded random +-1 starts; LABS instances are defined by N alone)",
        "config": {
            "workload": wl.name,
            "walks": W,
            "n": wl.n if uniform else f"uniform {{{wl.n_lo}..{wl.n_hi}}}",
            "steps_per_walk": f"{wl.rules.steps_a}N",
            "tenure": "U[floor(N/10), floor(N/5)]",
            "aspiration": bool(wl.rules.aspiration),
            "launch": {"waves_per_group": launch[0], "persistent": launch[1],
                       "groups_per_cu": launch[2]},
            "evals_per_step": evals_per_step,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_INT32_OPS / 1e12,
            "unit": "Top/s (int32, 3 ops per lag term)",
            "frac": achieved / PEAK_INT32_OPS,
            "traffic": None,
            "kernel": "tabu_kernel",
            "kernel_ms": kernel_ms,
            "algorithmic_ops_per_launch": ops_per_launch,
        },
    }

    if not args.no_cpu:
        # The oracle on this host's cores over the same workload, repeated
        # until at least min_s seconds have elapsed (one pass is well under a
        # second with 16 threads).  Walks are independent, so the oracle's
        # batch call spreads them over threads; nothing else is tuned.
        from oracle import oracle as O
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        sample = args.cpu_walks or W
        sched = O.Schedule(wl.rules.steps_rule, wl.rules.steps_a, wl.rules.tenure_rule,
                           wl.rules.lo_num, wl.rules.lo_den, wl.rules.lo_add, wl.rules.hi_num,
                           wl.rules.hi_den, wl.rules.hi_add, wl.rules.aspiration)
        sub_ns = ns[:sample]
        passes, c0 = 0, time.perf_counter()
        while True:
            O.tabu_batch(sample, sched, wl.seed, ns=sub_ns, stride=128, nthreads=threads)
            passes += 1
            if time.perf_counter() - c0 >= args.cpu_min_s or passes >= 100:
                break
        cpu_s = time.perf_counter() - c0
        cpu_evals = passes * int(np.sum(sub_ns.astype(np.int64) * wl.rules.steps_a * sub_ns))
        line["cpu_baseline"] = {
            "value": cpu_evals / cpu_s,
            "unit": "evals/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"{passes} passes over walks 0..{sample - 1} of {wl.name} in {cpu_s:.1f} s "
                      f"(plain C, gcc -O2, {threads} threads)",
        }
    print(json.dumps(line), flush=True)
    lb.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
