"""Benchmark of the batched tabu-search hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload tabu_n64|tabu_uneven|tabu_n120|tabu_n32|tabu_n256|tabu_long_uneven]
                    [--no-cpu] [--no-ttt] [--no-serving] [--no-skew]

A step is one labs_tabu_batch call over the whole batch (every walk scores
all N single-flip neighbours at each of its steps).  The default workload is
4096 independent walks at N=64 from random starts, 4N = 256 steps each,
tenure U[6, 12] with aspiration.  Inputs are synthetic and seeded (LABS has
no dataset: an instance is its length N).

Prints one JSON line: whole-job flip-neighbour evaluations per second, the
roofline of the walk kernel (integer VALU bound) timed with HIP events on the
stream it runs on, the CPU oracle timed on a bounded sample of the same
workload on this host, time-to-target energy of the memetic search at N=120
(256 replicas of K=100; one launch per generation, a replayed graph of
one-generation launches, the persistent form, and the batched-generation
variant), the deviation from skew-symmetry d(S) of App. A over a batch of
N=120 rows, and the serving loop's throughput and latency percentiles under
Poisson arrivals.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X (gfx950) figures at its 2.4 GHz peak clock, 256 CUs: v_dot4_i32_i8
# sums four int8 products into an int32 per lane, 64 lanes per CU-cycle (a
# wave64 dot instruction every 4 cycles per SIMD) -- the contraction of the
# neighbour scoring; one int32 operation per lane at that issue rate; the
# CDNA4 LDS serves 256 bytes per CU-cycle (twice CDNA3's 128).  Under the
# dot-product load of labs_device_peaks the clock measures about 2.06 GHz,
# which is reported beside these.
CLOCK_HZ, CUS = 2.4e9, 256
PEAK_DOT4_OPS = CUS * 64 * 4 * CLOCK_HZ    # 157.3e12 int8 products/s
PEAK_INT32_OPS = CUS * 64 * CLOCK_HZ       # 39.3e12 int32 lane-ops/s
PEAK_LDS_BYTES = CUS * 256 * CLOCK_HZ      # 157.3e12 B/s
METRIC = "flip-neighbour evals/sec (N=64..120) + time-to-target energy; batched vs plain"
# What decides which walk kernels a call runs and how they are compiled: the
# kernels, the length classes, the launch selection and the build flags.
KERNEL_SOURCES = ("paper_2504_00987_amd/csrc/labs_device.hpp",
                  "paper_2504_00987_amd/csrc/labs_walk.hip",
                  "paper_2504_00987_amd/csrc/labs_internal.h",
                  "paper_2504_00987_amd/csrc/labs_api.cpp")

# Counter readings per call of labs_tabu_batch (rocprofv3 --pmc, one pass per
# counter group, the same bench command with --launch), per workload and the
# launch it was profiled under, valid only for the walk kernel digest they
# were taken with; otherwise nothing is attached (they are never carried over
# to other code or another launch).  FETCH_SIZE / WRITE_SIZE are in KiB and
# scaled by what the same counters read for a 256 MiB device copy (FETCH 0.5x,
# WRITE 1.0x of the bytes moved).  GRBM_GUI_ACTIVE is the sum over the 8
# XCDs; the LDS busy fraction is SQ_LDS_IDX_ACTIVE over one XCD's busy cycles
# times the CUs.  SQ_WAVE_CYCLES and the SQ_*_ANY counters are wave-time in
# units of four cycles.  The summaries live in profiles/.
COPY_SCALE = {"FETCH_SIZE": 262144 / 131087, "WRITE_SIZE": 262144 / 262144}
XCDS = 8
COUNTERS_SOURCE = "profiles/tabu_kernel_counters.md"
COUNTERS_DIGEST = "65597ff269d66762"
COUNTERS = {
    ("tabu_n64", (64, 1, 0, 0, 0)): {
        "SQ_WAVES": 4096, "SQ_INSTS_VALU": 45513148, "SQ_INSTS_SALU": 33101021,
        "SQ_INSTS_LDS": 13721600, "SQ_LDS_BANK_CONFLICT": 2847176,
        "SQ_LDS_IDX_ACTIVE": 47100360, "GRBM_GUI_ACTIVE": 2602963, "SQ_WAVE_CYCLES": 249625723,
        "SQ_ACTIVE_INST_ANY": 100487299, "SQ_WAIT_ANY": 90887124, "SQ_WAIT_INST_ANY": 58246496,
        "FETCH_SIZE": 86.3, "WRITE_SIZE": 768.0},
    ("tabu_n64", (128, 2, 0, 0, 0)): {
        "SQ_WAVES": 4096, "SQ_INSTS_VALU": 45537724, "SQ_INSTS_SALU": 33121501,
        "SQ_INSTS_LDS": 13721600, "SQ_LDS_BANK_CONFLICT": 2847176,
        "SQ_LDS_IDX_ACTIVE": 47100360, "GRBM_GUI_ACTIVE": 2641890, "SQ_WAVE_CYCLES": 244954014,
        "SQ_ACTIVE_INST_ANY": 100529590, "SQ_WAIT_ANY": 84688251, "SQ_WAIT_INST_ANY": 59949379,
        "FETCH_SIZE": 82.9, "WRITE_SIZE": 640.0},
    ("tabu_n64", (256, 4, 0, 0, 0)): {
        "SQ_WAVES": 4096, "SQ_INSTS_VALU": 45537724, "SQ_INSTS_SALU": 33121501,
        "SQ_INSTS_LDS": 13721600, "SQ_LDS_BANK_CONFLICT": 2847176,
        "SQ_LDS_IDX_ACTIVE": 47100360, "GRBM_GUI_ACTIVE": 2565526, "SQ_WAVE_CYCLES": 245254690,
        "SQ_ACTIVE_INST_ANY": 100531017, "SQ_WAIT_ANY": 85030196, "SQ_WAIT_INST_ANY": 59846120,
        "FETCH_SIZE": 84.3, "WRITE_SIZE": 576.0},
    ("tabu_uneven", (64, 1, 0, 0, 0)): {
        "SQ_WAVES": 8192, "SQ_INSTS_VALU": 238153444, "SQ_INSTS_SALU": 107004426,
        "SQ_INSTS_LDS": 65717792, "SQ_LDS_BANK_CONFLICT": 35697887,
        "SQ_LDS_IDX_ACTIVE": 263385095, "GRBM_GUI_ACTIVE": 10981097,
        "SQ_WAVE_CYCLES": 1235198368, "SQ_ACTIVE_INST_ANY": 427094313, "SQ_WAIT_ANY": 286088155,
        "SQ_WAIT_INST_ANY": 522007640, "FETCH_SIZE": 649.8, "WRITE_SIZE": 1361.1},
    ("tabu_uneven", (128, 2, 0, 0, 0)): {
        "SQ_WAVES": 8192, "SQ_INSTS_VALU": 238981029, "SQ_INSTS_SALU": 107045386,
        "SQ_INSTS_LDS": 65717792, "SQ_LDS_BANK_CONFLICT": 35697887,
        "SQ_LDS_IDX_ACTIVE": 263385095, "GRBM_GUI_ACTIVE": 12292234,
        "SQ_WAVE_CYCLES": 1042541253, "SQ_ACTIVE_INST_ANY": 427827244, "SQ_WAIT_ANY": 249638089,
        "SQ_WAIT_INST_ANY": 365200678, "FETCH_SIZE": 652.3, "WRITE_SIZE": 1357.5},
    ("tabu_n120", (64, 1, 0, 0, 1)): {
        "SQ_WAVES": 4096, "SQ_INSTS_VALU": 215952677, "SQ_INSTS_SALU": 116891741,
        "SQ_INSTS_LDS": 67190784, "SQ_LDS_BANK_CONFLICT": 12524579,
        "SQ_LDS_IDX_ACTIVE": 241409059, "GRBM_GUI_ACTIVE": 14282818,
        "SQ_WAVE_CYCLES": 800668253, "SQ_ACTIVE_INST_ANY": 421353424, "SQ_WAIT_ANY": 213610749,
        "SQ_WAIT_INST_ANY": 165679612, "FETCH_SIZE": 221.8, "WRITE_SIZE": 768.0},
    ("tabu_n120", (64, 1, 0, 0, 0)): {
        "SQ_WAVES": 4096, "SQ_INSTS_VALU": 283060663, "SQ_INSTS_SALU": 107530772,
        "SQ_INSTS_LDS": 80859136, "SQ_LDS_BANK_CONFLICT": 17711104,
        "SQ_LDS_IDX_ACTIVE": 305389568, "GRBM_GUI_ACTIVE": 13829119,
        "SQ_WAVE_CYCLES": 1335726845, "SQ_ACTIVE_INST_ANY": 486242331, "SQ_WAIT_ANY": 371388113,
        "SQ_WAIT_INST_ANY": 478146242, "FETCH_SIZE": 72.8, "WRITE_SIZE": 768.0},
    ("tabu_n32", (64, 2, 0, 0, 0)): {
        "SQ_WAVES": 8192, "SQ_INSTS_VALU": 65617920, "SQ_INSTS_SALU": 11116544,
        "SQ_INSTS_LDS": 11632640, "SQ_LDS_BANK_CONFLICT": 3187117,
        "SQ_LDS_IDX_ACTIVE": 39068077, "GRBM_GUI_ACTIVE": 2257454, "SQ_WAVE_CYCLES": 347045904,
        "SQ_ACTIVE_INST_ANY": 99851470, "SQ_WAIT_ANY": 79889195, "SQ_WAIT_INST_ANY": 167204589,
        "FETCH_SIZE": 66.1, "WRITE_SIZE": 2560.0},
    ("tabu_n32", (128, 4, 0, 0, 0)): {
        "SQ_WAVES": 8192, "SQ_INSTS_VALU": 65658880, "SQ_INSTS_SALU": 11124736,
        "SQ_INSTS_LDS": 11632640, "SQ_LDS_BANK_CONFLICT": 3187117,
        "SQ_LDS_IDX_ACTIVE": 39068077, "GRBM_GUI_ACTIVE": 2248578, "SQ_WAVE_CYCLES": 351115208,
        "SQ_ACTIVE_INST_ANY": 99899866, "SQ_WAIT_ANY": 84375146, "SQ_WAIT_INST_ANY": 166874530,
        "FETCH_SIZE": 66.4, "WRITE_SIZE": 2304.0},
    ("tabu_n32", (64, 4, 0, 0, 0)): {
        "SQ_WAVES": 8192, "SQ_INSTS_VALU": 65617920, "SQ_INSTS_SALU": 11116544,
        "SQ_INSTS_LDS": 11632640, "SQ_LDS_BANK_CONFLICT": 3187117,
        "SQ_LDS_IDX_ACTIVE": 39068077, "GRBM_GUI_ACTIVE": 2251066, "SQ_WAVE_CYCLES": 347053631,
        "SQ_ACTIVE_INST_ANY": 99853791, "SQ_WAIT_ANY": 80004182, "SQ_WAIT_INST_ANY": 167201910,
        "FETCH_SIZE": 66.4, "WRITE_SIZE": 2560.0},
    ("tabu_n256", (256, 4, 0, 0, 0)): {
        "SQ_WAVES": 4096, "SQ_INSTS_VALU": 2027584427, "SQ_INSTS_SALU": 381779144,
        "SQ_INSTS_LDS": 541691904, "SQ_LDS_BANK_CONFLICT": 4194304,
        "SQ_LDS_IDX_ACTIVE": 2027626496, "GRBM_GUI_ACTIVE": 105383441,
        "SQ_WAVE_CYCLES": 5970235536, "SQ_ACTIVE_INST_ANY": 3033241847,
        "SQ_WAIT_ANY": 1285363394, "SQ_WAIT_INST_ANY": 1651510685, "FETCH_SIZE": 178.8,
        "WRITE_SIZE": 1088.0},
    ("tabu_long_uneven", (256, 4, 0, 0, 0)): {
        "SQ_WAVES": 4096, "SQ_INSTS_VALU": 1391622528, "SQ_INSTS_SALU": 281735379,
        "SQ_INSTS_LDS": 368409501, "SQ_LDS_BANK_CONFLICT": 114441374,
        "SQ_LDS_IDX_ACTIVE": 1480472504, "GRBM_GUI_ACTIVE": 73559732,
        "SQ_WAVE_CYCLES": 4305539543, "SQ_ACTIVE_INST_ANY": 2100988348,
        "SQ_WAIT_ANY": 989369525, "SQ_WAIT_INST_ANY": 1215187811, "FETCH_SIZE": 451.0,
        "WRITE_SIZE": 1184.9},
}


def kernel_digest() -> str:
    # hash of the walk kernels' code with comments and whitespace removed,
    # and of the compiler flags, so that the counter readings outlive edits
    # that change no code and nothing else
    import re
    from paper_2504_00987_amd import build as B
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    h.update(" ".join(f for f in B._flags() if not f.startswith("/")).encode())
    return h.hexdigest()[:16]


def host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def lag_terms_per_step(n: int) -> int:
    """Sum over neighbours j of L_j = max(N-j, j-1) (1-based): floor((3N^2-2N)/4)."""
    return sum(max(n - j, j - 1) for j in range(1, n + 1))


# ---------------------------------------------------------------------------
# Batched walks (the headline number)
# ---------------------------------------------------------------------------
def tabu_section(args, lb, wl, peaks=None):
    import torch
    ns = wl.lengths()
    W = wl.walks
    steps_per_walk = ns.astype(np.int64) * wl.rules.steps_a
    evals_per_step = int(np.sum(steps_per_walk * ns))
    ops_per_launch = 3 * int(sum(int(s) * lag_terms_per_step(int(n)) for s, n in zip(steps_per_walk, ns)))

    dev = torch.device("cuda", 0)
    out = (torch.empty((W, max(128, int(ns.max()))), dtype=torch.int8, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev), None)
    uniform = wl.n is not None
    kw = dict(n_uniform=wl.n) if uniform else dict(ns=ns)
    stream = torch.cuda.current_stream()

    def launch_ms(reps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            lb.tabu_batch(wl.rules, W, wl.seed, out=out, stream=stream, **kw)
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    if args.launch:
        # a fixed launch (the one a counter set was profiled under)
        lb.set_launch(*[int(x) for x in args.launch.split(",")])
    for _ in range(args.warmup):
        lb.tabu_batch(wl.rules, W, wl.seed, out=out, stream=stream, **kw)
    torch.cuda.synchronize()

    tune = None
    if not args.launch and not args.no_autotune:
        # the library's autotuner over the workload's length range; the
        # untuned default is timed first for comparison, once the GPU runs
        # at its steady clock (untimed calls for at least 50 ms)
        n_lo, n_hi = int(ns.min()), int(ns.max())
        default_launch = lb.get_launch(n_lo, n_hi)
        t_end = time.perf_counter() + 0.05
        while time.perf_counter() < t_end:
            lb.tabu_batch(wl.rules, W, wl.seed, out=out, stream=stream, **kw)
            torch.cuda.synchronize()
        default_ms = launch_ms(10)
        t0 = time.perf_counter()
        tried = lb.autotune(wl.rules, n_lo, n_hi, W, seed=wl.seed + 17)
        tune = {"range": [n_lo, n_hi], "configurations_timed": tried,
                "seconds": time.perf_counter() - t0,
                "default_launch": list(default_launch), "default_kernel_ms": default_ms}
        launch_ms(2)

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
    launch = lb.get_launch(int(ns.min()), int(ns.max()))

    lag_terms = ops_per_launch // 3
    roof = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_DOT4_OPS / 1e12,
        "unit": "Top/s (3 integer ops per lag term; peak: v_dot4_i32_i8, 4 int8 products "
                "per lane per clock)",
        "frac": achieved / PEAK_DOT4_OPS,
        "traffic": None,
        "kernel": "tabu_kernel",
        "kernel_ms": kernel_ms,
        "algorithmic_ops_per_launch": ops_per_launch,
        # the same work against one int32 operation per lane per clock: above
        # 1 it shows the reduction of work by the packed int8 products, it is
        # not a fraction of any peak
        "work_vs_int32_issue": achieved / PEAK_INT32_OPS,
        "lds": {
            # algorithmic LDS bytes: two spins and C_k as int8 per lag term;
            # the lag form reads one byte of its row per lag term and C_k as
            # a broadcast, so the hardware figure (hardware.lds_busy_frac, from
            # counters) is the measured one
            "algorithmic_bytes_per_launch": 3 * lag_terms,
            "achieved": 3 * lag_terms / (kernel_ms * 1e-3) / 1e12,
            "peak": PEAK_LDS_BYTES / 1e12,
            "unit": "TB/s",
            "frac": 3 * lag_terms / (kernel_ms * 1e-3) / PEAK_LDS_BYTES,
        },
    }
    if peaks is not None:
        roof["measured_peak"] = peaks["dot4_ops_per_s"] / 1e12
        roof["frac_of_measured_peak"] = achieved / peaks["dot4_ops_per_s"]
        roof["clock_hz_under_load"] = peaks["clock_hz"]
        roof["lds"]["measured_peak"] = peaks["lds_bytes_per_s"] / 1e12
        roof["lds"]["frac_of_measured_peak"] = 3 * lag_terms / (kernel_ms * 1e-3) / peaks["lds_bytes_per_s"]
    digest = kernel_digest()
    c = COUNTERS.get((wl.name, tuple(launch)))
    if c is not None and COUNTERS_DIGEST == digest:
        roof["traffic"] = (c["FETCH_SIZE"] * COPY_SCALE["FETCH_SIZE"]
                           + c["WRITE_SIZE"] * COPY_SCALE["WRITE_SIZE"]) * 1024
        lane_ops = c["SQ_INSTS_VALU"] * 64
        wave = c["SQ_WAVE_CYCLES"]
        roof["hardware"] = {
            "valu_lane_ops_per_launch": lane_ops,
            "valu_issue_frac": lane_ops / (kernel_ms * 1e-3) / PEAK_INT32_OPS,
            "salu_instructions_per_launch": c["SQ_INSTS_SALU"],
            "lds_instructions_per_launch": c["SQ_INSTS_LDS"],
            "lds_bank_conflict_cycles_per_launch": c["SQ_LDS_BANK_CONFLICT"],
            "lds_busy_frac": c["SQ_LDS_IDX_ACTIVE"] / (c["GRBM_GUI_ACTIVE"] / XCDS * CUS),
            "wave_time": {"issuing": c["SQ_ACTIVE_INST_ANY"] / wave,
                          "waiting_any": c["SQ_WAIT_ANY"] / wave,
                          "waiting_for_issue": c["SQ_WAIT_INST_ANY"] / wave},
            "launch": list(launch),
            "source": COUNTERS_SOURCE,
        }
    roof["kernel_digest"] = digest

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
            "seed": wl.seed,
            "tenure": "U[floor(N/10), floor(N/5)]",
            "aspiration": bool(wl.rules.aspiration),
            "launch": {"group_lanes": launch[0], "walks_per_group": launch[1],
                       "persistent": launch[2], "groups_per_cu": launch[3], "layout": launch[4]},
            "evals_per_step": evals_per_step,
        },
        "roofline": roof,
    }
    if tune is not None:
        tune["chosen_launch"] = list(launch)
        line["config"]["autotune"] = tune
    return line, ns


def cpu_tabu(args, wl, ns):
    # The oracle on this host's cores over the same workload, repeated until
    # at least min_s seconds have elapsed (one pass is well under a second
    # with 16 threads).  Walks are independent, so the oracle's batch call
    # spreads them over threads; nothing else is tuned.
    from oracle import oracle as O
    # the machine's CPU share for one GPU is 16 threads
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    # all walks up to N = 128; a bounded prefix of the N = 256 workload
    sample = args.cpu_walks or (wl.walks if int(ns.max()) <= 128 else 128)
    r = wl.rules
    sched = O.Schedule(r.steps_rule, r.steps_a, r.tenure_rule, r.lo_num, r.lo_den, r.lo_add,
                       r.hi_num, r.hi_den, r.hi_add, r.aspiration)
    sub_ns = ns[:sample]
    passes, c0 = 0, time.perf_counter()
    while True:
        O.tabu_batch(sample, sched, wl.seed, ns=sub_ns, stride=max(128, int(sub_ns.max())), nthreads=threads)
        passes += 1
        if time.perf_counter() - c0 >= args.cpu_min_s or passes >= 100:
            break
    cpu_s = time.perf_counter() - c0
    cpu_evals = passes * int(np.sum(sub_ns.astype(np.int64) * r.steps_a * sub_ns))
    return {
        "value": cpu_evals / cpu_s,
        "unit": "evals/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{passes} passes over walks 0..{sample - 1} of {wl.name} in {cpu_s:.1f} s "
                  f"(plain C, gcc -O2, {threads} threads)",
        "host": host_cpu(),
    }


# ---------------------------------------------------------------------------
# Deviation from skew-symmetry d(S) (App. A), an analysis of results
# ---------------------------------------------------------------------------
def skew_section(args, lb):
    import torch
    from paper_2504_00987_amd import inputs as I
    count, n, seed = 4096, 120, 1006
    S = torch.from_numpy(I.random_pm1(count, n, n, seed=seed)).cuda()
    stream = torch.cuda.current_stream()
    for _ in range(3):
        lb.skew_deviation(S, n_uniform=n, stream=stream)
    reps = 10
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        d = lb.skew_deviation(S, n_uniform=n, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    # even N: N rotations x N deletions, (N - 2) / 2 pair tests each
    tests = count * n * n * ((n - 2) // 2)
    res = {"rows": count, "n": n, "data": f"uniform random +-1 rows, numpy seed {seed}",
           "kernel_ms": ms, "rows_per_s": count / (ms * 1e-3),
           "pair_tests_per_s": tests / (ms * 1e-3),
           "d_histogram": np.bincount(d.cpu().numpy()).tolist()}
    if not args.no_cpu:
        from oracle import oracle as O
        rows = S[:32].cpu().numpy()
        t0 = time.perf_counter()
        want = [O.skew_deviation(r) for r in rows]
        dt = time.perf_counter() - t0
        if want != d[:32].cpu().numpy().tolist():
            raise RuntimeError("skew deviation differs from the oracle")
        res["cpu_baseline"] = {"value": len(rows) / dt, "unit": "rows/s", "cores": 1,
                               "kind": "oracle", "sample": f"rows 0..31 in {dt:.2f} s"}
    return res


# ---------------------------------------------------------------------------
# Time to target: memetic search at N=120
# ---------------------------------------------------------------------------
MODES = {"plain": 0, "graph": 1, "persistent": 2}


def ttt_section(args, lb):
    import torch
    from paper_2504_00987_amd import inputs as I
    wl = I.MEMETIC_N120
    n = wl.n
    G = args.ttt_gens
    targets = [int(t) for t in args.ttt_targets.split(",") if t]
    res = {"workload": wl.name, "n": n, "replicas": wl.pops, "K": wl.K,
           "generation_budget": G, "chunk": args.ttt_chunk,
           "rules": "crossover p=0.9, tournament parents, one cut; mutation 1/N; walk "
                    "floor(N/2)+U[0,N] steps, tenure U[1, floor(N/10)+1], aspiration",
           "stop": "all replicas stop at the end of the chunk in which the first reaches "
                   "the target", "targets": []}
    for tgt in targets:
        row = {"target_e": tgt, "target_mf": n * n / (2 * tgt)}
        hit = None
        for name in args.ttt_modes.split(","):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = lb.memetic_run(wl.K, wl.rules, G, wl.pops, wl.seed, n_uniform=n,
                               mode=MODES[name], chunk=args.ttt_chunk, target=tgt, stop_all=1)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h = r.hit_gen.cpu().numpy()
            first = int(h[h >= 0].min()) if (h >= 0).any() else None
            gens = int(r.gens_done.max().item())
            be = int(r.best_e.min().item())
            if hit is None:
                hit = (first, be, gens)
            elif hit != (first, be, gens):
                raise RuntimeError(f"execution modes disagree at target {tgt}: {hit} vs "
                                   f"{(first, be, gens)}")
            row[f"seconds_{name}"] = dt
            row[f"us_per_generation_{name}"] = dt / max(gens, 1) * 1e6
        row["hit_generation"], row["best_e"], row["generations_run"] = hit
        row["reached"] = hit[0] is not None
        if "seconds_plain" in row and "seconds_persistent" in row:
            row["persistent_speedup_vs_plain"] = row["seconds_plain"] / row["seconds_persistent"]
        # batched generations: B children per generation from one snapshot
        # (another trajectory than one child per generation), persistent
        # form, the same budget of children
        for B in [int(b) for b in args.ttt_children.split(",") if b]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = lb.memetic_run(wl.K, wl.rules, max(G // B, 1), wl.pops, wl.seed, n_uniform=n,
                               mode=MODES["persistent"], chunk=args.ttt_chunk, target=tgt,
                               stop_all=1, children=B)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h = r.hit_gen.cpu().numpy()
            gens = int(r.gens_done.max().item())
            row[f"children_{B}"] = {
                "seconds": dt, "hit_generation": int(h[h >= 0].min()) if (h >= 0).any() else None,
                "best_e": int(r.best_e.min().item()), "generations_run": gens,
                "us_per_generation": dt / max(gens, 1) * 1e6,
                "us_per_child": dt / max(gens * B, 1) * 1e6}
        res["targets"].append(row)
    return res


def cpu_memetic(args, n_gens_sample: int = 256):
    # The oracle's memetic replicas at the same size, one thread per replica
    # group (each replica is independent), timed on a bounded number of
    # generations; its time to a target reached at generation g is g times
    # the per-generation time (the trajectories are identical).
    import concurrent.futures as cf
    from oracle import oracle as O
    from paper_2504_00987_amd import inputs as I
    wl = I.MEMETIC_N120
    r = wl.rules
    sched = O.Schedule(r.steps_rule, r.steps_a, r.tenure_rule, r.lo_num, r.lo_den, r.lo_add,
                       r.hi_num, r.hi_den, r.hi_add, r.aspiration)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    reps = [O.MemeticState(wl.n, wl.K, wl.seed, p) for p in range(wl.pops)]
    pm = O.p_mut_inv_n(wl.n)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda st: st.advance(n_gens_sample, sched, wl.p_comb, pm), reps))
    dt = time.perf_counter() - t0
    return {"us_per_generation": dt / n_gens_sample * 1e6, "cores": threads, "kind": "oracle",
            "sample": f"{wl.pops} replicas x {n_gens_sample} generations at N={wl.n} in {dt:.1f} s"}


# ---------------------------------------------------------------------------
# Serving: Poisson arrivals, continuous batching
# ---------------------------------------------------------------------------
def serve(lb, reqs, arrivals, max_slots, chunk, K, rules, pops, gens):
    from paper_2504_00987_amd.labs import Server
    srv = Server(lb, K, rules, max_slots=max_slots, chunk=chunk)
    pending, lats = {}, []
    try:
        t0 = time.perf_counter()
        i = 0
        while i < len(reqs) or pending:
            now = time.perf_counter() - t0
            while i < len(reqs) and arrivals[i] <= now:
                n, s = reqs[i]
                pending[srv.submit(n, s, pops, gens)] = n
                i += 1
            for rid in list(pending):
                r = srv.poll(rid, pending[rid])
                if r is not None:
                    lats.append(r[2])
                    del pending[rid]
            time.sleep(0.0002)
        wall = time.perf_counter() - t0
    finally:
        srv.close()
    lats = np.array(lats)
    return {"solves_per_s": len(reqs) / wall, "p50_ms": float(np.percentile(lats, 50)) * 1e3,
            "p99_ms": float(np.percentile(lats, 99)) * 1e3, "seconds": wall}


def serving_section(args, lb):
    from paper_2504_00987_amd import inputs as I
    K, rules = 100, I.RULES_MEMETIC
    pops, gens = I.SERVING_POPS, I.SERVING_GENS
    reqs = I.serving_requests(args.serve_requests)
    cfg = dict(max_slots=args.serve_slots, chunk=args.serve_chunk, K=K, rules=rules, pops=pops,
               gens=gens)
    burst = serve(lb, reqs, np.zeros(len(reqs)), **cfg)
    cap = burst["solves_per_s"]
    out = {"requests_per_rate": len(reqs), "n": "uniform {32..128}", "replicas_per_request": pops,
           "generations": gens, "K": K, "resident_slots": args.serve_slots,
           "chunk": args.serve_chunk, "capacity_solves_per_s": cap, "burst": burst, "rates": []}
    for frac in [float(x) for x in args.serve_rates.split(",") if x]:
        arr = I.poisson_arrivals(frac * cap, len(reqs), seed=I.SERVING_SEED + 1)
        r = serve(lb, reqs, arr, **cfg)
        r["offered_per_s"] = frac * cap
        r["load"] = frac
        out["rates"].append(r)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="tabu_n64",
                    choices=["tabu_n64", "tabu_uneven", "tabu_n120", "tabu_n256", "tabu_long_uneven",
                             "tabu_n32"])
    ap.add_argument("--more-workloads", default="tabu_uneven,tabu_n120,tabu_n32",
                    help="walk workloads timed after the headline one, each with its own "
                         "roofline and CPU baseline (comma list, empty for none)")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the measured dot4 / int32 / LDS peaks")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch configuration instead of the tuned one")
    ap.add_argument("--launch", default="",
                    help="time this launch instead of the tuned one: group_lanes,walks_per_group,"
                         "persistent,groups_per_cu,layout (labs_set_launch)")
    ap.add_argument("--cpu-walks", type=int, default=0, help="oracle sample size (0: all walks)")
    ap.add_argument("--cpu-min-s", type=float, default=10.0, help="minimum oracle timing")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-target section")
    ap.add_argument("--ttt-gens", type=int, default=100000)
    ap.add_argument("--ttt-targets", default="1200,1107,1028")
    ap.add_argument("--ttt-modes", default="persistent,graph,plain")
    ap.add_argument("--ttt-chunk", type=int, default=64)
    ap.add_argument("--ttt-children", default="8",
                    help="children per generation of the batched-generation rows (comma list)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--no-skew", action="store_true", help="skip the skew-deviation section")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=8192)
    ap.add_argument("--serve-chunk", type=int, default=25)
    ap.add_argument("--serve-rates", default="0.1,0.25,0.5,0.75,0.9,1.1")
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

    wl = I.TABU_WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    lb = Labs(0)
    peaks = None
    if not args.no_peaks:
        peaks = lb.device_peaks()
        print(f"# measured peaks: dot4 {peaks['dot4_ops_per_s'] / 1e12:.1f} T products/s, "
              f"int32 {peaks['int32_ops_per_s'] / 1e12:.1f} T ops/s, "
              f"LDS {peaks['lds_bytes_per_s'] / 1e12:.1f} TB/s, clock {peaks['clock_hz'] / 1e9:.2f} GHz",
              file=sys.stderr, flush=True)
    line, ns = tabu_section(args, lb, wl, peaks)
    print(f"# tabu: {line['value']:.4g} evals/s, kernel {line['roofline']['kernel_ms']:.4f} ms",
          file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_tabu(args, wl, ns)
    if peaks is not None:
        line["peaks"] = {
            "measured": {"dot4_products_per_s": peaks["dot4_ops_per_s"],
                         "int32_ops_per_s": peaks["int32_ops_per_s"],
                         "lds_bytes_per_s": peaks["lds_bytes_per_s"],
                         "clock_hz_under_dot4_load": peaks["clock_hz"]},
            "published": {"dot4_products_per_s": PEAK_DOT4_OPS, "int32_ops_per_s": PEAK_INT32_OPS,
                          "lds_bytes_per_s": PEAK_LDS_BYTES},
            "how": "labs_device_peaks: independent chains of v_dot4_i32_i8 / v_add_u32 per lane, "
                   "and conflict-free 16-byte LDS reads, on 16 (8 for LDS) workgroups of 256 "
                   "lanes per CU, one launch timed with HIP events after a warm-up"}
    more = []
    for name in [x for x in args.more_workloads.split(",") if x and x != wl.name]:
        w2 = I.TABU_WORKLOADS[name]
        row, ns2 = tabu_section(args, lb, w2, peaks)
        entry = {"workload": name, "value": row["value"], "unit": "evals/s",
                 "ms_per_step": row["ms_per_step"], "config": row["config"],
                 "roofline": row["roofline"]}
        if not args.no_cpu:
            entry["cpu_baseline"] = cpu_tabu(args, w2, ns2)
        more.append(entry)
        print(f"# {name}: {row['value']:.4g} evals/s, kernel {row['roofline']['kernel_ms']:.4f} ms",
              file=sys.stderr, flush=True)
    if more:
        line["more_workloads"] = more
    if not args.no_ttt:
        line["time_to_target"] = ttt_section(args, lb)
        print("# time to target done", file=sys.stderr, flush=True)
        if not args.no_cpu:
            line["time_to_target"]["cpu_baseline"] = cpu_memetic(args)
    if not args.no_skew:
        line["skew_deviation"] = skew_section(args, lb)
        print("# skew deviation done", file=sys.stderr, flush=True)
    if not args.no_serving:
        line["serving"] = serving_section(args, lb)
        print("# serving done", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)
    lb.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
