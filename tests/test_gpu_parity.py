"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

All results are integers decided by integer arithmetic and the shared RNG
contract, so the bar is bit-exact equality of energies, best sequences,
final energies and per-step flip traces.
"""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_00987_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lb():
    from paper_2504_00987_amd.labs import Labs
    h = Labs(0)
    yield h
    h.close()


def osched(r: I.Rules) -> O.Schedule:
    return O.Schedule(r.steps_rule, r.steps_a, r.tenure_rule, r.lo_num, r.lo_den, r.lo_add,
                      r.hi_num, r.hi_den, r.hi_add, r.aspiration, r.slo_num, r.slo_den,
                      r.shi_num, r.shi_den)


# ---------------------------------------------------------------------------
# Eq. (2)
# ---------------------------------------------------------------------------
def test_energy_uniform_and_ragged(lb):
    say("energy: uniform N=64 x 1000, ragged 3..128 x 777")
    S = I.random_pm1(1000, 64, 64, seed=1)
    got = lb.energy_batch(torch.from_numpy(S).cuda(), n_uniform=64).cpu().numpy()
    assert np.array_equal(got, O.energy_batch(S, n_uniform=64))
    ns = I.uneven_lengths(777, 3, 128, seed=2)
    R = I.random_pm1_ragged(ns, 136, seed=3)
    got = lb.energy_batch(torch.from_numpy(R).cuda(), ns=torch.from_numpy(ns).cuda()).cpu().numpy()
    assert np.array_equal(got, O.energy_batch(R, ns=ns))


def test_energy_closed_forms_and_edges(lb):
    say("energy: all-ones/alternating, N = 3..128")
    rows = []
    ns = []
    for n in range(3, 129):
        for s in (np.ones(n), np.array([(-1) ** i for i in range(n)])):
            r = np.zeros(128, dtype=np.int8)
            r[:n] = s
            rows.append(r)
            ns.append(n)
    R = np.stack(rows)
    ns = np.array(ns, dtype=np.int32)
    got = lb.energy_batch(torch.from_numpy(R).cuda(), ns=torch.from_numpy(ns).cuda()).cpu().numpy()
    want = np.array([(n - 1) * n * (2 * n - 1) // 6 for n in ns])
    assert np.array_equal(got, want)
    empty = lb.energy_batch(torch.zeros((0, 64), dtype=torch.int8, device="cuda"), n_uniform=64)
    assert empty.numel() == 0


def test_skew_deviation(lb):
    # App. A's d(S): the printed column of Table labs_results, then random
    # rows of every length class against the oracle
    from tests.test_oracle_objective import _table, decode_hex
    say("skew deviation: paper rows and random ragged rows N = 3..256")
    rows, ns, want = [], [], []
    for n, _, _, _, _, hexs, d in _table():
        r = np.zeros(256, dtype=np.int8)
        r[:n] = decode_hex(hexs, n)
        rows.append(r)
        ns.append(n)
        want.append(d)
    rng = np.random.default_rng(17)
    extra = [3, 4, 5, 6, 63, 64, 65, 128, 129, 255, 256] + list(rng.integers(3, 257, 120))
    R = I.random_pm1_ragged(np.array(extra, dtype=np.int32), 256, seed=18)
    for n, r in zip(extra, R):
        rows.append(r)
        ns.append(int(n))
        want.append(O.skew_deviation(r[:n]))
    got = lb.skew_deviation(torch.from_numpy(np.stack(rows)).cuda(),
                            ns=torch.from_numpy(np.array(ns, dtype=np.int32)).cuda())
    assert np.array_equal(got.cpu().numpy(), want)
    # uniform length and the empty batch
    U = I.random_pm1(50, 120, 120, seed=19)
    got = lb.skew_deviation(torch.from_numpy(U).cuda(), n_uniform=120).cpu().numpy()
    assert np.array_equal(got, [O.skew_deviation(u) for u in U])
    assert lb.skew_deviation(torch.zeros((0, 64), dtype=torch.int8, device="cuda"),
                             n_uniform=64).numel() == 0


def test_bruteforce_min(lb):
    say("exhaustive minimum: oracle enumeration for n <= 22, properties beyond")
    for n in [3, 4, 5, 7, 8, 11, 13, 16, 20, 22]:
        e, cnt, seq = lb.bruteforce_min(n)
        oe, oc = O.bruteforce_min(n)
        assert (e, cnt) == (oe, oc), n
        assert seq[0] == 1 and O.energy(seq) == e
        if n <= 14:  # the smallest attaining bit pattern with s_0 = +1
            codes = np.arange(0, 1 << n, 2, dtype=np.int64)
            bits = ((codes[:, None] >> np.arange(n)) & 1).astype(np.int8)
            seqs = 1 - 2 * bits
            E = np.array([O.energy(r) for r in seqs])
            first = int(codes[np.argmax(E == e)])
            assert np.array_equal(seq, 1 - 2 * ((first >> np.arange(n)) & 1)), n
    # 32-bit and 64-bit enumeration paths at their boundary
    for n in (31, 32, 33, 34):
        e, cnt, seq = lb.bruteforce_min(n)
        assert seq[0] == 1 and O.energy(seq) == e
        assert e % 4 == (n // 2) % 4 and cnt >= 2 and cnt % 2 == 0
    from paper_2504_00987_amd._lib import LabsError
    with pytest.raises(LabsError):
        lb.bruteforce_min(41)


def test_skew_bruteforce_min(lb):
    # the search restricted to skew-symmetric sequences (Sec. II.C) against
    # the oracle's enumeration, then against the unrestricted exhaustive
    # minimum on the GPU (never better; equal at the Barker lengths)
    say("skew-symmetric exhaustive minima, odd N = 3..33")
    for n in range(3, 34, 2):
        e, c, a = lb.skew_bruteforce_min(n)
        if n <= 33:
            oe, oc, oa = O.skew_bruteforce_min(n)
            assert (e, c) == (oe, oc) and np.array_equal(a, oa), n
        assert e == O.energy(a)
        cc = (n - 1) // 2
        assert all(a[cc + i] == (-1) ** i * a[cc - i] for i in range(1, cc + 1))
        if n <= 31:
            ge, gc, _ = lb.bruteforce_min(n)
            assert e >= ge
            if n in (3, 5, 7, 11, 13):
                assert e == ge == n // 2
    from paper_2504_00987_amd._lib import LabsError
    for bad in (4, 1, 77):
        with pytest.raises(LabsError):
            lb.skew_bruteforce_min(bad)


def test_skew_bruteforce_long(lb):
    # lengths past 64 take the 128-bit masks: the returned sequence is
    # skew-symmetric and has the reported energy (Eq. 2 on the GPU and in
    # the oracle), and odd lags vanish
    for n in (63, 65, 71):
        say(f"skew-symmetric exhaustive minimum, N={n}")
        e, c, a = lb.skew_bruteforce_min(n)
        cc = (n - 1) // 2
        assert all(a[cc + i] == (-1) ** i * a[cc - i] for i in range(1, cc + 1))
        assert a[0] == 1 and c >= 2 and c % 2 == 0
        assert e == O.energy(a)
        row = torch.from_numpy(a.reshape(1, n).copy()).cuda()
        assert lb.energy_batch(row, n_uniform=n).item() == e
        C = O.autocorrelation(a)
        assert all(C[k] == 0 for k in range(1, n, 2))


# ---------------------------------------------------------------------------
# Alg. 2 / Alg. 4: batched walks
# ---------------------------------------------------------------------------
def _oracle_walks(W, n, rules, seed, starts=None, with_trace=True):
    best = np.zeros((W, max(128, int(np.max(n)))), dtype=np.int8)
    be = np.zeros(W, dtype=np.int64)
    fe = np.zeros(W, dtype=np.int64)
    trs = []
    sch = osched(rules)
    for w in range(W):
        nn = n[w] if hasattr(n, "__len__") else n
        T, lo, hi = O.walk_schedule(nn, sch, seed, w, 0)
        s = starts[w, :nn] if starts is not None else O.random_start(nn, seed, w)
        b, e1, f1, tr, _ = O.tabu_walk(s, seed, w, 0, T, lo, hi, rules.aspiration, want_trace=with_trace)
        best[w, :nn] = b
        be[w], fe[w] = e1, f1
        trs.append(tr)
    return best, be, fe, trs


@pytest.mark.parametrize("n", [3, 4, 5, 20, 31, 33, 63, 64, 65, 100, 127, 128])
@pytest.mark.parametrize("asp", [1, 0])
def test_tabu_small_trace(lb, n, asp):
    say(f"tabu trace parity N={n} aspiration={asp}")
    rules = I.Rules(I.STEPS_MULT_N, 2, I.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, asp)
    if rules.hi_num * n // rules.hi_den >= n:
        rules = I.Rules(I.STEPS_MULT_N, 2, I.TENURE_LINEAR, 0, 1, 0, 0, 1, 1, asp)
    W, seed = 24, 4242 + n
    res = lb.tabu_batch(rules, W, seed, n_uniform=n, trace_stride=2 * n)
    best, be, fe, trs = _oracle_walks(W, n, rules, seed)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(W):
        assert np.array_equal(tr[w, : 2 * n], trs[w])


def test_tabu_explicit_starts_paper_rules(lb):
    say("tabu: explicit starts, paper walk length and tenure, ragged N")
    ns = I.uneven_lengths(96, 3, 128, seed=11)
    starts = I.random_pm1_ragged(ns, 128, seed=12)
    rules = I.RULES_PAPER_LITERAL
    res = lb.tabu_batch(rules, len(ns), 99, ns=ns, starts=torch.from_numpy(starts).cuda(),
                        trace_stride=200)
    best, be, fe, trs = _oracle_walks(len(ns), ns, rules, 99, starts=starts)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(len(ns)):
        assert np.array_equal(tr[w, : len(trs[w])], trs[w])


# Every launch configuration: (group lanes, walks per group) of one
# wavefront per walk or two (128, 1), both layouts of 64 < N <= 128, one walk
# per wavefront (pair) or a persistent queue at the automatic and a fixed
# grid.
LAUNCH_GRID = [(gl, wpg, p, g, lay) for gl, wpg in ((64, 1), (128, 2), (256, 4), (128, 1))
               for lay in (1, 2) for p, g in ((0, 0), (1, 0), (1, 2))]


@pytest.mark.parametrize("launch", LAUNCH_GRID)
def test_tabu_launch_invariance(lb, launch):
    say(f"tabu: launch configuration {launch} gives identical walks")
    ns = I.uneven_lengths(300, 48, 120, seed=21)
    rules = I.rules_tabu(3)
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, len(ns), 1002, ns=ns)
    finally:
        lb.set_launch(None)
    best, be, fe = O.tabu_batch(len(ns), osched(rules), 1002, ns=ns, stride=128, nthreads=8)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)


# Several walks per wavefront: 32 lanes per walk ({64, 2}, {128, 4}) or 16
# ({64, 4}: N <= 16 four per wavefront, 16 < N <= 32 two), as a grid of one
# wavefront per two or four walks or a persistent queue at the automatic and
# a fixed grid; the batch's longer walks keep their one-wavefront kernels.
SUBWAVE_GRID = [(gl, wpg, p, g, 0) for gl, wpg in ((64, 2), (128, 4), (64, 4))
                for p, g in ((0, 0), (1, 0), (1, 2))]


@pytest.mark.parametrize("launch", SUBWAVE_GRID)
def test_tabu_subwave_launch(lb, launch):
    # N in 3..40 (both short classes and part of 32 < N <= 49), 301 walks:
    # the last wavefront of each class has empty groups
    ns = I.uneven_lengths(301, 3, 40, seed=51)
    say(f"tabu: N in 3..40, launch configuration {launch} gives identical walks")
    rules = I.rules_tabu(3)
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, len(ns), 5151, ns=ns)
    finally:
        lb.set_launch(None)
    best, be, fe = O.tabu_batch(len(ns), osched(rules), 5151, ns=ns, stride=128, nthreads=8)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)


@pytest.mark.parametrize("launch", [(64, 2, 0, 0, 0), (64, 4, 1, 0, 0), (128, 4, 1, 1, 0)])
@pytest.mark.parametrize("asp", [1, 0])
def test_tabu_subwave_traces_and_starts(lb, launch, asp):
    # every N in 3..33 three times, the caller's starts (all +1, alternating,
    # random), paper walk lengths (differing within a wavefront) and traces
    ns = np.repeat(np.arange(3, 34, dtype=np.int32), 3)
    say(f"tabu: every N in 3..33, starts and traces, aspiration={asp}, launch {launch}")
    starts = I.random_pm1_ragged(ns, 64, seed=52)
    for i, n in enumerate(ns):
        if i % 3 == 0:
            starts[i, :n] = 1
        elif i % 3 == 1:
            starts[i, :n] = [(-1) ** j for j in range(n)]
    rules = dataclasses.replace(I.RULES_PAPER_LITERAL, aspiration=asp)
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, len(ns), 53, ns=ns, starts=torch.from_numpy(starts).cuda(),
                            trace_stride=64)
    finally:
        lb.set_launch(None)
    best, be, fe, trs = _oracle_walks(len(ns), ns, rules, 53, starts=starts)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(len(ns)):
        assert np.array_equal(tr[w, : len(trs[w])], trs[w]), f"N={ns[w]}"


@pytest.mark.parametrize("n,W", [(32, 37), (17, 3), (16, 13), (5, 66), (3, 1)])
@pytest.mark.parametrize("launch", [(64, 2, 0, 0, 0), (64, 4, 0, 0, 0), (128, 4, 1, 2, 0)])
def test_tabu_subwave_uniform(lb, n, W, launch):
    # one length for the whole batch (no per-walk lengths), walk counts that
    # leave the last wavefront partly empty
    say(f"tabu: {W} walks of N={n}, launch {launch}")
    rules = I.rules_tabu(4)
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, W, 600 + n, n_uniform=n, trace_stride=4 * n)
    finally:
        lb.set_launch(None)
    best, be, fe, trs = _oracle_walks(W, n, rules, 600 + n)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(W):
        assert np.array_equal(tr[w, : len(trs[w])], trs[w])


def test_autotune_short_range():
    # N <= 32 adds the several-walks-per-wavefront points to the tuned grid
    from paper_2504_00987_amd.labs import Labs
    say("autotune over N in [3, 32], then parity under the tuned launch")
    h = Labs(0)
    try:
        rules = I.rules_tabu(3)
        tried = h.autotune(rules, 3, 32, 2048, seed=5)
        assert tried >= 25
        gl, wpg, pers, gpc, lay = h.get_launch(3, 32)
        assert (gl, wpg) in ((64, 1), (128, 2), (256, 4), (64, 2), (128, 4), (64, 4))
        say(f"autotune chose {(gl, wpg, pers, gpc, lay)} after {tried} configurations")
        ns = I.uneven_lengths(500, 3, 32, seed=54)
        res = h.tabu_batch(rules, len(ns), 55, ns=ns)
        best, be, fe = O.tabu_batch(len(ns), osched(rules), 55, ns=ns, stride=128, nthreads=8)
        assert np.array_equal(res.best_e.cpu().numpy(), be)
        assert np.array_equal(res.final_e.cpu().numpy(), fe)
        assert np.array_equal(res.best_seq.cpu().numpy(), best)
    finally:
        h.close()


def test_autotune_then_parity():
    # the autotuner times every launch configuration and keeps the fastest
    # for the length bucket of the range's longest walk; results stay
    # bit-identical under the chosen configuration
    from paper_2504_00987_amd.labs import Labs
    say("autotune over N in [48, 120], then parity under the tuned launch")
    h = Labs(0)
    try:
        rules = I.rules_tabu(3)
        before = h.get_launch(48, 120)
        other = h.get_launch(64)
        tried = h.autotune(rules, 48, 120, 512, seed=3)
        assert tried >= 30  # the grid of one- and two-wavefront walks, both layouts
        gl, wpg, pers, gpc, lay = h.get_launch(48, 120)
        assert (gl, wpg) in ((64, 1), (128, 2), (256, 4), (128, 1)) and pers in (0, 1)
        assert lay in (0, 1, 2) and ((not pers and gpc == 0) or (pers and gpc > 0))
        assert before == (64, 1, 0, 0, 0)  # the default up to N = 128
        assert h.get_launch(64) == other  # another length range keeps its launch
        ns = I.uneven_lengths(200, 48, 120, seed=23)
        res = h.tabu_batch(rules, len(ns), 1002, ns=ns)
        best, be, fe = O.tabu_batch(len(ns), osched(rules), 1002, ns=ns, stride=128, nthreads=8)
        assert np.array_equal(res.best_e.cpu().numpy(), be)
        assert np.array_equal(res.final_e.cpu().numpy(), fe)
        assert np.array_equal(res.best_seq.cpu().numpy(), best)
    finally:
        h.close()


def test_tabu_n64_full_size(lb):
    wl = I.TABU_N64
    say(f"tabu: {wl.name} full size W={wl.walks} N={wl.n}, all walks against the oracle")
    res = lb.tabu_batch(wl.rules, wl.walks, wl.seed, n_uniform=wl.n)
    best, be, fe = O.tabu_batch(wl.walks, osched(wl.rules), wl.seed, n_uniform=wl.n, stride=128,
                                nthreads=16)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)


@pytest.fixture(scope="module")
def n120_oracle():
    wl = I.TABU_N120
    return O.tabu_batch(wl.walks, osched(wl.rules), wl.seed, n_uniform=wl.n, stride=128, nthreads=16)


@pytest.mark.parametrize("launch", [(64, 1, 0, 0, 0), (64, 1, 0, 0, 1), (128, 1, 0, 0, 0)])
def test_tabu_n120_full_size(lb, n120_oracle, launch):
    # the N = 120 bench row at full size, all walks, in the record and the lag
    # layout (the two the autotuner chooses between) and on two wavefronts
    wl = I.TABU_N120
    say(f"tabu: {wl.name} full size W={wl.walks} N={wl.n}, launch {launch}, all walks against the oracle")
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(wl.rules, wl.walks, wl.seed, n_uniform=wl.n)
    finally:
        lb.set_launch(None)
    best, be, fe = n120_oracle
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)


@pytest.fixture(scope="module")
def n32_oracle():
    wl = I.TABU_N32
    return O.tabu_batch(wl.walks, osched(wl.rules), wl.seed, n_uniform=wl.n, stride=128, nthreads=16)


@pytest.mark.parametrize("launch", [None, (64, 2, 0, 0, 0), (128, 4, 0, 0, 0), (64, 4, 0, 0, 0)])
def test_tabu_n32_full_size(lb, n32_oracle, launch):
    # the short-walk bench row at full size, all walks, in the default launch
    # and in each several-walks-per-wavefront launch the autotuner picks from
    wl = I.TABU_N32
    say(f"tabu: {wl.name} full size W={wl.walks} N={wl.n}, launch {launch}, all walks against the oracle")
    if launch is not None:
        lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(wl.rules, wl.walks, wl.seed, n_uniform=wl.n)
    finally:
        lb.set_launch(None)
    best, be, fe = n32_oracle
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)


@pytest.mark.parametrize("name,n_sample", [("tabu_uneven", 256), ("tabu_long_uneven", 48)])
def test_tabu_uneven_full_size_sampled(lb, name, n_sample):
    # tabu_long_uneven: both N > 128 classes, mixed in one launch
    wl = I.TABU_WORKLOADS[name]
    ns = wl.lengths()
    say(f"tabu: {wl.name} full size W={wl.walks}, sampled walks against the oracle")
    res = lb.tabu_batch(wl.rules, wl.walks, wl.seed, ns=ns)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(wl.walks, size=n_sample, replace=False))
    sample = np.unique(np.concatenate([sample, [0, wl.walks - 1], np.argsort(-ns)[:4]]))
    sch = osched(wl.rules)
    be_g = res.best_e.cpu().numpy()
    fe_g = res.final_e.cpu().numpy()
    bs_g = res.best_seq.cpu().numpy()
    for w in sample:
        n = int(ns[w])
        T, lo, hi = O.walk_schedule(n, sch, wl.seed, int(w), 0)
        b, e1, f1, _, _ = O.tabu_walk(O.random_start(n, wl.seed, int(w)), wl.seed, int(w), 0, T, lo, hi, 1)
        assert be_g[w] == e1 and fe_g[w] == f1
        assert np.array_equal(bs_g[w, :n], b) and not bs_g[w, n:].any()
    # properties at every walk: energies agree with the returned sequences
    E = lb.energy_batch(res.best_seq, ns=torch.from_numpy(ns).cuda()).cpu().numpy()
    assert np.array_equal(E, be_g)
    assert np.all(be_g <= fe_g)
    assert np.all(be_g % 4 == (ns // 2) % 4)


@pytest.mark.parametrize("launch,n", [((64, 1, 0, 0, 0), 8), (None, 8), ((128, 1, 0, 0, 1), 70)])
def test_tabu_largest_grids(lb, launch, n):
    # 2^24 + 37 walks: one walk per 64-lane workgroup (and one per two
    # wavefronts) passes 2^30 work-items, so the batch runs as several
    # launches; 128-byte rows put the last walks past 2^31 bytes of output.
    # Sampled walks (both sides of every launch boundary) against the
    # oracle, and the energy of every returned sequence (that launch splits
    # too) against its best energy.
    from paper_2504_00987_amd import _lib
    W = (1 << 24) + 37
    rules = I.rules_tabu(1)
    say(f"tabu: {W} walks of N={n}, launch {launch}")
    if launch is not None:
        lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, W, 2024, n_uniform=n)
    finally:
        lb.set_launch(None)
    torch.cuda.synchronize()
    be = res.best_e.cpu().numpy()
    fe = res.final_e.cpu().numpy()
    rng = np.random.default_rng(64)
    edges = [0, 1, (1 << 23) - 1, 1 << 23, (1 << 24) - 1, 1 << 24, (1 << 24) + 1, W - 1]
    sample = np.unique(np.concatenate([edges, rng.choice(W, size=24, replace=False)]))
    sch = osched(rules)
    for w in sample:
        w = int(w)
        T, lo, hi = O.walk_schedule(n, sch, 2024, w, 0)
        b, e1, f1, _, _ = O.tabu_walk(O.random_start(n, 2024, w), 2024, w, 0, T, lo, hi, 1)
        assert be[w] == e1 and fe[w] == f1, w
        assert np.array_equal(res.best_seq[w, :n].cpu().numpy(), b), w
        assert not res.best_seq[w, n:].any()
    E = lb.energy_batch(res.best_seq, n_uniform=n).cpu().numpy()
    assert np.array_equal(E, be)
    assert np.all(be <= fe)
    del res, E
    torch.cuda.empty_cache()


def test_memetic_replica_limit(lb):
    from paper_2504_00987_amd import _lib
    with pytest.raises(_lib.LabsError) as ex:
        lb.memetic_run(16, I.RULES_MEMETIC, 1, (1 << 22) + 1, 1, n_uniform=20)
    assert ex.value.code == _lib.LABS_E_INVAL


def test_tabu_zero_walks_and_zero_steps(lb):
    say("tabu: W=0 and zero-step walks")
    r = lb.tabu_batch(I.rules_tabu(4), 0, 1, n_uniform=64)
    assert r.best_e.numel() == 0
    zero = I.Rules(I.STEPS_FIXED, 0, I.TENURE_LINEAR, 0, 1, 0, 0, 1, 0, 1)
    res = lb.tabu_batch(zero, 10, 5, n_uniform=50)
    starts = np.stack([O.random_start(50, 5, w) for w in range(10)])
    assert np.array_equal(res.best_seq.cpu().numpy()[:, :50], starts)
    assert np.array_equal(res.best_e.cpu().numpy(), [O.energy(s) for s in starts])


def test_invalid_arguments(lb):
    say("invalid arguments are rejected")
    from paper_2504_00987_amd._lib import LabsError
    with pytest.raises(LabsError):
        lb.tabu_batch(I.rules_tabu(4), 4, 1, n_uniform=2)
    with pytest.raises(LabsError):
        lb.tabu_batch(I.rules_tabu(4), 4, 1, n_uniform=257)
    bad = I.Rules(I.STEPS_FIXED, 10, I.TENURE_LINEAR, 0, 1, 0, 1, 1, 0, 1)  # maxTabu = N
    with pytest.raises(LabsError):
        lb.tabu_batch(bad, 4, 1, n_uniform=20)
    with pytest.raises(LabsError):
        lb.tabu_batch(I.rules_tabu(4), 4, 1, n_uniform=64, out_stride=32)


# ---------------------------------------------------------------------------
# Alg. 1 / Alg. 3: memetic replicas
# ---------------------------------------------------------------------------
def _oracle_memetic(n_list, K, rules, gens, seed, target=-1, p_comb=I.P_COMB_090, p_mut=None,
                    children=0):
    # replicas are independent: one oracle replica per worker thread (the
    # oracle's C code releases the interpreter lock); p_mut None: 1/N
    import concurrent.futures as cf

    def one(p):
        n = int(n_list[p])
        st = O.MemeticState(n, K, seed, p)
        thr = O.p_mut_inv_n(n) if p_mut is None else p_mut
        st.advance(gens, osched(rules), p_comb, thr, target=target, children=children)
        return st

    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(one, range(len(n_list))))


@pytest.mark.parametrize("launch", [(64, 2, 0, 0, 0), (64, 4, 1, 0, 0)])
def test_tabu_range_rule_subwave(lb, launch):
    # the RANGE walk length (different lengths per walk within a wavefront's
    # groups) with several walks per wavefront, traced
    ns = np.repeat(np.array([3, 9, 16, 17, 25, 32], dtype=np.int32), 5)
    rules = I.Rules(I.STEPS_RANGE, 0, I.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1, 1, 2, 3, 2)
    say(f"tabu RANGE rule, N <= 32, launch {launch}")
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, len(ns), 4343, ns=ns, trace_stride=64)
    finally:
        lb.set_launch(None)
    best, be, fe, trs = _oracle_walks(len(ns), ns, rules, 4343)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(len(ns)):
        assert np.array_equal(tr[w, : len(trs[w])], trs[w])


def test_autotune_across_all_short_forms():
    # a range from the several-walks-per-wavefront classes to 64 < N <= 128:
    # every launch form is a candidate; parity under the kept one
    from paper_2504_00987_amd.labs import Labs
    say("autotune over N in [3, 130], then parity under the tuned launch")
    h = Labs(0)
    try:
        rules = I.rules_tabu(2)
        tried = h.autotune(rules, 3, 130, 1024, seed=9)
        assert tried >= 40
        launch = h.get_launch(3, 130)
        say(f"autotune kept {launch} after {tried} configurations")
        ns = I.uneven_lengths(400, 3, 130, seed=57)
        res = h.tabu_batch(rules, len(ns), 58, ns=ns, out_stride=256)
        best, be, fe = O.tabu_batch(len(ns), osched(rules), 58, ns=ns, stride=256, nthreads=8)
        assert np.array_equal(res.best_e.cpu().numpy(), be)
        assert np.array_equal(res.final_e.cpu().numpy(), fe)
        assert np.array_equal(res.best_seq.cpu().numpy(), best)
    finally:
        h.close()


def test_tabu_range_rule(lb):
    # Sec. III.B's walk length randInt[N/2, 3N/2] as the RANGE rule, and an
    # asymmetric range, traced, against the oracle; lengths over two classes
    ns = np.array([3, 10, 31, 64, 65, 100, 128, 129, 200], dtype=np.int32)
    for bounds in ((1, 2, 3, 2), (1, 3, 7, 4)):
        rules = I.Rules(I.STEPS_RANGE, 0, I.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1, *bounds)
        say(f"tabu RANGE rule {bounds}, N={list(ns)}")
        res = lb.tabu_batch(rules, len(ns), 4242, ns=ns, trace_stride=512)
        sch = osched(rules)
        for w, n in enumerate(ns):
            n = int(n)
            T, lo, hi = O.walk_schedule(n, sch, 4242, w, 0)
            s = O.random_start(n, 4242, w)
            b, e1, f1, tr, _ = O.tabu_walk(s, 4242, w, 0, T, lo, hi, rules.aspiration,
                                           want_trace=True)
            assert res.best_e[w].item() == e1 and res.final_e[w].item() == f1
            assert np.array_equal(res.best_seq[w, :n].cpu().numpy(), b)
            assert np.array_equal(res.trace[w, :T].cpu().numpy(), tr)
    from paper_2504_00987_amd._lib import LabsError
    with pytest.raises(LabsError):  # an empty range is rejected
        lb.tabu_batch(I.Rules(I.STEPS_RANGE, 0, I.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1, 2, 1, 1, 1),
                      4, 1, n_uniform=40)


def test_memetic_range_rule_modes(lb):
    # memetic replicas whose walks take the RANGE rule (Sec. III.B's
    # randInt[N/2, 3N/2]) equal those of Alg. 4's rule draw for draw
    ns = np.array([17, 64, 90], dtype=np.int32)
    r_range = I.Rules(I.STEPS_RANGE, 0, I.TENURE_LINEAR, 0, 1, 1, 1, 10, 1, 1, 1, 2, 3, 2)
    ref = _oracle_memetic(ns, 24, I.RULES_MEMETIC, 9, 314)
    for mode in (0, 2):
        say(f"memetic RANGE rule, mode {mode}")
        res = lb.memetic_run(24, r_range, 9, len(ns), 314, ns=ns, mode=mode, chunk=4)
        for p, st in enumerate(ref):
            assert res.best_e[p].item() == st.bestE
            assert np.array_equal(res.best_seq[p, :int(ns[p])].cpu().numpy(), st.best)


def test_memetic_stream_ordered(lb):
    # runs are enqueued on the caller's stream without synchronising it: two
    # runs back to back on two streams (the second waits for the first's use
    # of the state memory on the GPU), then checked against the oracle
    n, K, G = 40, 30, 12
    rules = I.RULES_MEMETIC
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    say("memetic stream-ordered: two runs on two streams")
    a = lb.memetic_run(K, rules, G, 5, 21, n_uniform=n, mode=1, chunk=5, stream=s1)
    b = lb.memetic_run(K, rules, G, 5, 22, n_uniform=n, mode=2, chunk=5, stream=s2)
    s1.synchronize()
    s2.synchronize()
    for res, seed in ((a, 21), (b, 22)):
        ref = _oracle_memetic([n] * 5, K, rules, G, seed)
        for p, st in enumerate(ref):
            assert res.best_e[p].item() == st.bestE
            assert np.array_equal(res.best_seq[p, :n].cpu().numpy(), st.best)
            assert res.gens_done[p].item() == G


@pytest.mark.parametrize("mode", [0, 2])
def test_memetic_cancel(lb, mode):
    # labs_cancel from another thread: the run stops at a chunk boundary, a
    # call still enqueueing returns LABS_E_CANCELLED, and what it leaves is
    # the oracle's state after the generations it ran
    import threading
    from paper_2504_00987_amd import _lib
    n, K, pops, G, chunk = 24, 16, 6, 10**6, 16
    rules = I.RULES_MEMETIC
    say(f"memetic cancel, mode {mode}")
    t = threading.Timer(0.3, lb.cancel)
    t.start()
    try:
        res = lb.memetic_run(K, rules, G, pops, 777, n_uniform=n, mode=mode, chunk=chunk)
        code = _lib.LABS_OK
    except _lib.LabsError as ex:
        code = ex.code
        res = lb._last_memetic
    t.join()
    torch.cuda.synchronize()
    done = res.gens_done.cpu().numpy()
    assert (done == done[0]).all() and 0 < done[0] < G and done[0] % chunk == 0
    if mode == 0:
        assert code == _lib.LABS_E_CANCELLED  # one launch per generation: still enqueueing
    g = int(min(done[0], 100000))
    ref = _oracle_memetic([n] * pops, K, rules, g, 777)
    if g == done[0]:
        for p, st in enumerate(ref):
            assert res.best_e[p].item() == st.bestE
            assert np.array_equal(res.best_seq[p, :n].cpu().numpy(), st.best)
    # a run started after the cancel is not affected
    res2 = lb.memetic_run(K, rules, 8, pops, 777, n_uniform=n, mode=mode, chunk=chunk)
    assert (res2.gens_done.cpu().numpy() == 8).all()


def _same_memetic(a, b):
    torch.cuda.synchronize()
    for x, y in ((a.best_seq, b.best_seq), (a.best_e, b.best_e), (a.hit_gen, b.hit_gen),
                 (a.gens_done, b.gens_done)):
        assert torch.equal(x, y)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("stop", [False, True])
def test_memetic_checkpoint_resume(lb, mode, stop):
    # a run to G equals a run to G1 continued to G on its own handle, and
    # equals the same run saved, loaded into another handle and continued
    # there; with a target and the global stop flag as well (G1 a multiple
    # of the chunk). Lengths over all three replica classes.
    from paper_2504_00987_amd.labs import Labs
    ns = I.uneven_lengths(40, 20, 140, seed=61)
    K, G, G1, chunk, seed = 24, 96, 40, 8, 6161
    rules = I.RULES_MEMETIC
    kw = dict(ns=ns, mode=mode, chunk=chunk)
    if stop:
        probe = lb.memetic_run(K, rules, G, len(ns), seed, ns=ns, mode=2, chunk=chunk)
        kw.update(target=int(np.median(probe.best_e.cpu().numpy())), stop_all=1)
    say(f"memetic checkpoint and resume, mode {mode}, stop {stop}")
    full = lb.memetic_run(K, rules, G, len(ns), seed, **kw)
    torch.cuda.synchronize()
    if stop:
        assert (full.hit_gen.cpu().numpy() >= 0).any()
    lb.memetic_run(K, rules, G1, len(ns), seed, **kw)
    blob = lb.memetic_save()
    cont = lb.memetic_run(K, rules, G, len(ns), seed, resume=1, **kw)
    _same_memetic(full, cont)
    # a resumed run past the limit changes nothing
    again = lb.memetic_run(K, rules, G, len(ns), seed, resume=1, **kw)
    _same_memetic(full, again)
    h2 = Labs(0)
    try:
        h2.memetic_load(blob)
        assert h2.memetic_save() == blob  # the loaded state is the saved one
        res = h2.memetic_run(K, rules, G, len(ns), seed, resume=1, **kw)
        _same_memetic(full, res)
    finally:
        h2.close()


def test_memetic_checkpoint_resume_batched_children(lb):
    # the batched-generation variant (4 children per generation) resumes too
    from paper_2504_00987_amd.labs import Labs
    ns = I.uneven_lengths(24, 30, 120, seed=63)
    K, G, G1, chunk, seed = 24, 48, 16, 8, 6363
    rules = I.RULES_MEMETIC
    kw = dict(ns=ns, mode=2, chunk=chunk, children=4)
    say("memetic checkpoint and resume, 4 children per generation")
    full = lb.memetic_run(K, rules, G, len(ns), seed, **kw)
    lb.memetic_run(K, rules, G1, len(ns), seed, **kw)
    blob = lb.memetic_save()
    h2 = Labs(0)
    try:
        h2.memetic_load(blob)
        res = h2.memetic_run(K, rules, G, len(ns), seed, resume=1, **kw)
        _same_memetic(full, res)
    finally:
        h2.close()


def test_memetic_cancel_then_resume(lb):
    # a cancelled run, continued, equals the uninterrupted run
    import threading
    from paper_2504_00987_amd import _lib
    n, K, pops, chunk, seed = 24, 16, 6, 16, 778
    rules = I.RULES_MEMETIC
    say("memetic cancel, then resume")
    t = threading.Timer(0.3, lb.cancel)
    t.start()
    try:
        lb.memetic_run(K, rules, 10**6, pops, seed, n_uniform=n, mode=2, chunk=chunk)
    except _lib.LabsError as ex:
        assert ex.code == _lib.LABS_E_CANCELLED
    t.join()
    torch.cuda.synchronize()
    done = int(lb._last_memetic.gens_done[0].item())
    assert 0 < done < 10**6 and done % chunk == 0
    Gf = done + 3 * chunk
    cont = lb.memetic_run(K, rules, Gf, pops, seed, n_uniform=n, mode=2, chunk=chunk, resume=1)
    torch.cuda.synchronize()
    full = lb.memetic_run(K, rules, Gf, pops, seed, n_uniform=n, mode=2, chunk=chunk)
    _same_memetic(full, cont)


def test_memetic_resume_errors(lb):
    from paper_2504_00987_amd import _lib
    from paper_2504_00987_amd.labs import Labs
    rules = I.RULES_MEMETIC
    say("memetic resume and checkpoint: invalid uses")
    h2 = Labs(0)
    try:
        with pytest.raises(_lib.LabsError) as ex:
            h2.memetic_run(16, rules, 8, 4, 1, n_uniform=20, resume=1)  # nothing held
        assert ex.value.code == _lib.LABS_E_INVAL
        with pytest.raises(_lib.LabsError):
            h2.memetic_save()
        h2.memetic_run(16, rules, 8, 4, 1, n_uniform=20)
        blob = h2.memetic_save()
        for bad in (dict(seed=2), dict(pops=5), dict(K=17), dict(n=21)):
            a = dict(seed=1, pops=4, K=16, n=20)
            a.update(bad)
            with pytest.raises(_lib.LabsError) as ex:
                h2.memetic_run(a["K"], rules, 16, a["pops"], a["seed"], n_uniform=a["n"], resume=1)
            assert ex.value.code == _lib.LABS_E_INVAL
        for junk in (blob[:100], b"X" + blob[1:], blob[:-1]):
            with pytest.raises(_lib.LabsError) as ex:
                h2.memetic_load(junk)
            assert ex.value.code == _lib.LABS_E_INVAL
        # a failed load leaves the held replicas usable
        res = h2.memetic_run(16, rules, 16, 4, 1, n_uniform=20, resume=1)
        torch.cuda.synchronize()
        assert (res.gens_done.cpu().numpy() == 16).all()
        # the server starts every request afresh
        import ctypes
        p = Labs.memetic_params(16, rules, 0, resume=1)
        out = ctypes.c_void_p()
        assert h2.L.labs_server_create(h2.h, ctypes.byref(p), 8, ctypes.byref(out)) == _lib.LABS_E_INVAL
    finally:
        h2.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_memetic_n20_modes(lb, mode):
    wl = I.MEMETIC_N20
    pops = 6
    say(f"memetic N=20 K=100 {wl.generations} generations x {pops} replicas, mode {mode}")
    res = lb.memetic_run(wl.K, wl.rules, wl.generations, pops, wl.seed, n_uniform=wl.n,
                         mode=mode, chunk=7)
    ref = _oracle_memetic([wl.n] * pops, wl.K, wl.rules, wl.generations, wl.seed)
    emin, _ = O.bruteforce_min(20)
    for p, st in enumerate(ref):
        assert res.best_e[p].item() == st.bestE >= emin
        assert np.array_equal(res.best_seq[p, :20].cpu().numpy(), st.best)
        assert res.gens_done[p].item() == wl.generations and res.hit_gen[p].item() == -1


@pytest.mark.parametrize("mode,waves", [(0, 1), (1, 1), (2, 1), (0, 2), (1, 2), (2, 2)])
def test_memetic_uneven_lengths(lb, mode, waves):
    # both length classes: their kernels run on two forked streams (captured
    # into the graph in mode 1); replicas with N > 64 on one or two
    # wavefronts each
    ns = np.array([3, 7, 31, 64, 65, 96, 120, 128], dtype=np.int32)
    say(f"memetic ragged N={list(ns)}, K=24, 12 generations, mode {mode}, {waves} waves")
    rules = I.RULES_MEMETIC
    res = lb.memetic_run(24, rules, 12, len(ns), 77, ns=ns, mode=mode, chunk=5,
                         waves_per_replica=waves)
    ref = _oracle_memetic(ns, 24, rules, 12, 77)
    for p, st in enumerate(ref):
        n = int(ns[p])
        assert res.best_e[p].item() == st.bestE
        assert np.array_equal(res.best_seq[p, :n].cpu().numpy(), st.best)


@pytest.mark.parametrize("K,p_comb,p_mut", [(2, I.P_COMB_090, None), (128, 0, None),
                                             (37, 1 << 31, 0x30000000)])
def test_memetic_edge_parameters(lb, K, p_comb, p_mut):
    # smallest and largest population, sampling only (no crossover), a fixed
    # mutation threshold; lengths at the class edges, both wavefront forms
    from paper_2504_00987_amd.labs import MUT_FIXED, MUT_INV_N
    ns = np.array([3, 4, 64, 65, 127, 128], dtype=np.int32)
    rules = I.RULES_MEMETIC
    say(f"memetic edges K={K} p_comb={p_comb} p_mut={p_mut} N={list(ns)}")
    ref = _oracle_memetic(ns, K, rules, 7, 555, p_comb=p_comb, p_mut=p_mut)
    for waves in (1, 2):
        kw = dict(mut_rule=MUT_INV_N) if p_mut is None else dict(mut_rule=MUT_FIXED, p_mut=p_mut)
        res = lb.memetic_run(K, rules, 7, len(ns), 555, ns=ns, mode=2, chunk=3, p_comb=p_comb,
                             waves_per_replica=waves, **kw)
        for p, st in enumerate(ref):
            n = int(ns[p])
            assert res.best_e[p].item() == st.bestE
            assert np.array_equal(res.best_seq[p, :n].cpu().numpy(), st.best)
            assert res.gens_done[p].item() == 7


def test_memetic_target_and_stop_all(lb):
    n, K, G = 26, 40, 60
    rules = I.RULES_MEMETIC
    base = _oracle_memetic([n] * 4, K, rules, G, 31)
    target = sorted(st.bestE for st in base)[1]
    say(f"memetic target {target}: per-replica hit generations")
    ref = _oracle_memetic([n] * 4, K, rules, G, 31, target=target)
    res = lb.memetic_run(K, rules, G, 4, 31, n_uniform=n, target=target, mode=2, chunk=4)
    for p, st in enumerate(ref):
        assert res.hit_gen[p].item() == st.hit
        assert res.best_e[p].item() == st.bestE
        assert res.gens_done[p].item() == st.gen
    # global flag: everyone stops at the end of the chunk in which the first hit happened
    res2 = lb.memetic_run(K, rules, G, 4, 31, n_uniform=n, target=target, mode=0, chunk=4, stop_all=1)
    first = min(st.hit for st in ref if st.hit >= 0)
    stop = max(4, ((first + 3) // 4) * 4)
    for p, st in enumerate(ref):
        g = int(res2.gens_done[p].item())
        assert g == (st.gen if st.hit >= 0 and st.hit <= stop else stop)


def _oracle_stop_all(n_list, K, rules, G, seed, target, chunk, children=0):
    """The oracle's replicas under the global termination flag (Alg. 3): every
    replica stops at the end of the generation chunk in which the first one
    reached the target (the first chunk runs even when an initial population
    already does); a replica that hit earlier stopped at its own hit."""
    ref = _oracle_memetic(n_list, K, rules, G, seed, target=target, children=children)
    hits = [st.hit for st in ref if st.hit >= 0]
    if not hits:
        return ref, G
    stop = min(G, max(chunk, -(-min(hits) // chunk) * chunk))
    return _oracle_memetic(n_list, K, rules, stop, seed, target=target, children=children), stop


@pytest.mark.parametrize("n", [20, 33, 64, 65, 120])
def test_memetic_paper_literal_stop_all(lb, n):
    # the configuration the small-N time-to-solution experiment times: the
    # paper's own walk rules (Alg. 4's walk length, Sec. III.B's tenure
    # floor(T/10)..floor(3T/25), no aspiration), a target and the global
    # termination flag, in every execution mode
    rules = I.RULES_PAPER_LITERAL
    pops, K, G = 8, 100, 160
    seed = 7000 + n
    # a target two replicas reach within the first half of the budget
    base = _oracle_memetic([n] * pops, K, rules, G // 2, seed)
    target = sorted(st.bestE for st in base)[1]
    for mode, chunk, waves in ((0, 16, 0), (1, 7, 1), (2, 16, 0), (2, 5, 1)):
        ref, stop = _oracle_stop_all([n] * pops, K, rules, G, seed, target, chunk)
        say(f"memetic paper-literal N={n} target {target} mode {mode} chunk {chunk} "
            f"waves {waves}: stop at {stop}")
        res = lb.memetic_run(K, rules, G, pops, seed, n_uniform=n, target=target, mode=mode,
                             chunk=chunk, stop_all=1, waves_per_replica=waves)
        assert stop < G  # some replica hits, and the flag cuts the others short
        for p, st in enumerate(ref):
            assert res.hit_gen[p].item() == st.hit
            assert res.gens_done[p].item() == st.gen
            assert res.best_e[p].item() == st.bestE
            assert np.array_equal(res.best_seq[p, :n].cpu().numpy(), st.best)


def _deep_n120():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "memetic_n120_deep.txt")
    rows = {"full": {}, "long": {}, "hist": {}}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        if line.startswith("hist "):
            _, p, g, e = line.split()
            rows["hist"].setdefault(int(p), []).append((int(g), int(e)))
            continue
        sec, p, g, e, h = line.split()
        v = int(h, 16)
        seq = np.array([-1 if (v >> i) & 1 else 1 for i in range(120)], dtype=np.int8)
        rows[sec][(int(p), int(g))] = (int(e), seq)
    return rows


@pytest.mark.parametrize("mode,chunk,waves", [(2, 64, 0), (2, 64, 1), (0, 64, 0)])
def test_memetic_n120_deep_full_width(lb, mode, chunk, waves):
    # all 256 replicas of the N=120 configuration for 1000 generations against
    # the oracle's stored results (written by tests/golden/make_memetic_n120.py)
    wl = I.MEMETIC_N120
    want = _deep_n120()["full"]
    say(f"memetic N=120: 256 replicas x 1000 generations, mode {mode}, waves {waves}")
    res = lb.memetic_run(wl.K, wl.rules, 1000, wl.pops, wl.seed, n_uniform=wl.n, mode=mode,
                         chunk=chunk, waves_per_replica=waves)
    be, bs = res.best_e.cpu().numpy(), res.best_seq.cpu().numpy()
    assert len(want) == wl.pops
    for p in range(wl.pops):
        e, seq = want[(p, 1000)]
        assert be[p] == e and np.array_equal(bs[p, :120], seq)
    assert (res.gens_done.cpu().numpy() == 1000).all()


@pytest.mark.parametrize("gens", [25000, 50000, 100000])
def test_memetic_n120_deep_long(lb, gens):
    # replicas 0..3 of the N=120 configuration through its whole budget of
    # 10^5 generations, checked against the oracle's stored results at a
    # quarter and at the end; the persistent form the benchmark times, two
    # wavefronts each
    wl = I.MEMETIC_N120
    want = _deep_n120()["long"]
    say(f"memetic N=120: 4 replicas x {gens} generations, persistent")
    res = lb.memetic_run(wl.K, wl.rules, gens, 4, wl.seed, n_uniform=wl.n, mode=2, chunk=64)
    for p in range(4):
        e, seq = want[(p, gens)]
        assert res.best_e[p].item() == e
        assert np.array_equal(res.best_seq[p, :120].cpu().numpy(), seq)
        assert res.gens_done[p].item() == gens


def test_memetic_n120_deep_hit_generations(lb):
    # with a target the four replicas all reach, each stops at the generation
    # at which the oracle's best first fell to it (one of its improvements)
    wl = I.MEMETIC_N120
    hist = _deep_n120()["hist"]
    target = max(h[-1][1] for h in hist.values())
    say(f"memetic N=120: 4 replicas, target {target}")
    res = lb.memetic_run(wl.K, wl.rules, 100000, 4, wl.seed, n_uniform=wl.n, mode=2, chunk=64,
                         target=target)
    for p in range(4):
        g, e = next((g, e) for g, e in hist[p] if e <= target)
        assert res.hit_gen[p].item() == g and res.gens_done[p].item() == g
        assert res.best_e[p].item() == e


def test_memetic_n120_deep_long_other_forms(lb):
    # the full budget in the graph form and with one wavefront per replica
    wl = I.MEMETIC_N120
    want = _deep_n120()["long"]
    for mode, chunk, waves in ((1, 64, 0), (2, 256, 1)):
        say(f"memetic N=120: 4 replicas x 100000 generations, mode {mode}, waves {waves}")
        res = lb.memetic_run(wl.K, wl.rules, 100000, 4, wl.seed, n_uniform=wl.n, mode=mode,
                             chunk=chunk, waves_per_replica=waves)
        for p in range(4):
            e, seq = want[(p, 100000)]
            assert res.best_e[p].item() == e
            assert np.array_equal(res.best_seq[p, :120].cpu().numpy(), seq)


@pytest.mark.parametrize("mode,chunk,waves", [(1, 3, 1), (2, 64, 0)])
def test_memetic_n120_prefix(lb, mode, chunk, waves):
    # the N=120 configuration at full width (256 replicas of K=100) for its
    # first generations; (2, 64, 0) is the launch form the benchmark times
    wl = I.MEMETIC_N120
    pops, gens = wl.pops, 24
    say(f"memetic N=120 K=100: {pops} replicas x {gens} generations, mode {mode}, waves {waves}")
    res = lb.memetic_run(wl.K, wl.rules, gens, pops, wl.seed, n_uniform=wl.n, mode=mode,
                         chunk=chunk, waves_per_replica=waves)
    ref = _oracle_memetic([wl.n] * pops, wl.K, wl.rules, gens, wl.seed)
    be = res.best_e.cpu().numpy()
    bs = res.best_seq.cpu().numpy()
    for p, st in enumerate(ref):
        assert be[p] == st.bestE
        assert np.array_equal(bs[p, :120], st.best)


@pytest.mark.parametrize("B,mode,chunk", [(2, 0, 4), (3, 1, 5), (4, 2, 3), (8, 2, 9), (8, 0, 2)])
def test_memetic_batched_children(lb, B, mode, chunk):
    # B children per generation from one snapshot, merged in child order;
    # B = 8 with N > 64 needs more than 64 KiB of LDS per workgroup
    ns = np.array([3, 20, 49, 64, 65, 100, 127, 128], dtype=np.int32)
    rules = I.RULES_MEMETIC
    G = 9
    say(f"memetic batched B={B} mode {mode} chunk {chunk} N={list(ns)}")
    ref = _oracle_memetic(ns, 24, rules, G, 808, children=B)
    res = lb.memetic_run(24, rules, G, len(ns), 808, ns=ns, mode=mode, chunk=chunk, children=B)
    for p, st in enumerate(ref):
        n = int(ns[p])
        assert res.best_e[p].item() == st.bestE
        assert np.array_equal(res.best_seq[p, :n].cpu().numpy(), st.best)
        assert res.gens_done[p].item() == G and res.hit_gen[p].item() == -1


def test_memetic_batched_target(lb):
    # the target test runs after every child; the hit generation counts
    # generations (B children each), as in the oracle
    n, K, G, B = 30, 40, 40, 4
    rules = I.RULES_MEMETIC
    base = _oracle_memetic([n] * 6, K, rules, G, 91, children=B)
    target = sorted(st.bestE for st in base)[2]
    say(f"memetic batched B={B}, target {target}")
    ref = _oracle_memetic([n] * 6, K, rules, G, 91, target=target, children=B)
    for mode in (0, 2):
        res = lb.memetic_run(K, rules, G, 6, 91, n_uniform=n, target=target, mode=mode, chunk=4,
                             children=B)
        for p, st in enumerate(ref):
            assert res.hit_gen[p].item() == st.hit
            assert res.best_e[p].item() == st.bestE
            assert res.gens_done[p].item() == st.gen


def test_memetic_batched_one_child_is_default(lb):
    # children = 1 is the one-child-per-generation kernel itself
    ns = np.array([20, 64, 90], dtype=np.int32)
    rules = I.RULES_MEMETIC
    a = lb.memetic_run(16, rules, 6, 3, 5, ns=ns, mode=2, chunk=3, children=1)
    b = lb.memetic_run(16, rules, 6, 3, 5, ns=ns, mode=2, chunk=3)
    assert torch.equal(a.best_e, b.best_e) and torch.equal(a.best_seq, b.best_seq)


# ---------------------------------------------------------------------------
# N up to 256: four neighbours per lane, C_k >> 1 in the int8 mirror
# ---------------------------------------------------------------------------
def test_energy_long(lb):
    say("energy: N = 129..256 closed forms and random ragged rows")
    rows, ns = [], []
    for n in range(129, 257):
        for s in (np.ones(n), np.array([(-1) ** i for i in range(n)])):
            r = np.zeros(256, dtype=np.int8)
            r[:n] = s
            rows.append(r)
            ns.append(n)
    R = np.stack(rows)
    ns = np.array(ns, dtype=np.int32)
    got = lb.energy_batch(torch.from_numpy(R).cuda(), ns=torch.from_numpy(ns).cuda()).cpu().numpy()
    assert np.array_equal(got, [(n - 1) * n * (2 * n - 1) // 6 for n in ns])
    ns = I.uneven_lengths(300, 3, 256, seed=31)
    R = I.random_pm1_ragged(ns, 256, seed=32)
    got = lb.energy_batch(torch.from_numpy(R).cuda(), ns=torch.from_numpy(ns).cuda()).cpu().numpy()
    assert np.array_equal(got, O.energy_batch(R, ns=ns))


@pytest.mark.parametrize("n", [129, 160, 193, 194, 255, 256])
@pytest.mark.parametrize("asp", [1, 0])
def test_tabu_long_trace(lb, n, asp):
    say(f"tabu trace parity N={n} aspiration={asp}")
    rules = I.Rules(I.STEPS_MULT_N, 1, I.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, asp)
    W, seed = 8, 5151 + n
    res = lb.tabu_batch(rules, W, seed, n_uniform=n, trace_stride=n)
    best, be, fe, trs = _oracle_walks(W, n, rules, seed)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(W):
        assert np.array_equal(tr[w, :n], trs[w])


@pytest.mark.parametrize("launch", [(256, 4, 0, 0, 0), (64, 1, 1, 0, 0), (128, 2, 1, 1, 0),
                                    (128, 1, 1, 2, 1)])
def test_tabu_long_extreme_starts(lb, launch):
    # all-ones and alternating starts have |C_k| = N - k up to 255, the
    # values that need the halved mirror
    ns = np.array([256, 255, 200, 193, 160, 129, 256, 201, 128, 64], dtype=np.int32)
    say(f"tabu: extreme starts N={list(ns)}, launch {launch}")
    starts = np.zeros((len(ns), 256), dtype=np.int8)
    for i, n in enumerate(ns):
        starts[i, :n] = (np.ones(n) if i % 3 == 0 else
                         np.array([(-1) ** j for j in range(n)]) if i % 3 == 1 else -np.ones(n))
    rules = I.Rules(I.STEPS_MULT_N, 1, I.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, 1)
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, len(ns), 5, ns=ns, starts=torch.from_numpy(starts).cuda(),
                            trace_stride=256)
    finally:
        lb.set_launch(None)
    best, be, fe, trs = _oracle_walks(len(ns), ns, rules, 5, starts=starts)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(len(ns)):
        assert np.array_equal(tr[w, : len(trs[w])], trs[w])


@pytest.mark.parametrize("launch", [(64, 1, 0, 0, 0), (128, 2, 0, 0, 0), (256, 4, 0, 0, 0),
                                    (64, 1, 1, 0, 0), (128, 2, 1, 1, 0), (256, 4, 1, 2, 0)])
def test_tabu_long_launch_invariance(lb, launch):
    # both N > 128 classes in one batch: their single launch, every form
    say(f"tabu: N in 129..256, launch configuration {launch} gives identical walks")
    ns = I.uneven_lengths(120, 129, 256, seed=43)
    assert ns.min() <= 193 < ns.max()
    rules = I.rules_tabu(2)
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, len(ns), 77, ns=ns, out_stride=256)
    finally:
        lb.set_launch(None)
    best, be, fe = O.tabu_batch(len(ns), osched(rules), 77, ns=ns, stride=256, nthreads=16)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)


def test_tabu_all_classes_ragged(lb):
    ns = I.uneven_lengths(240, 3, 256, seed=41)
    say("tabu: ragged N in 3..256 (all six length classes), Philox starts")
    rules = I.rules_tabu(2)
    res = lb.tabu_batch(rules, len(ns), 1234, ns=ns, out_stride=256)
    best, be, fe = O.tabu_batch(len(ns), osched(rules), 1234, ns=ns, stride=256, nthreads=16)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)


@pytest.mark.parametrize("launch", [(256, 4, 0, 0, 0), (128, 2, 1, 1, 0), (128, 1, 0, 0, 1),
                                    (128, 1, 1, 2, 2), (64, 1, 0, 0, 1), (64, 4, 0, 0, 0),
                                    (128, 4, 1, 2, 1)])
def test_tabu_every_length(lb, launch):
    """One walk at every N in 3..256, move traces compared: each N has its own
    placement of the reversed records (a shift of 0..15 records that keeps the
    window reads conflict-free) and its own start of the zero window for lanes
    past N, and the lengths span every class boundary."""
    say(f"tabu: every N in 3..256, traces, launch {launch}")
    ns = np.arange(3, 257, dtype=np.int32)
    rules = I.Rules(I.STEPS_MULT_N, 1, I.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, 1)
    lb.set_launch(*launch)
    try:
        res = lb.tabu_batch(rules, len(ns), 7007, ns=ns, out_stride=256, trace_stride=256)
    finally:
        lb.set_launch(None)
    best, be, fe, trs = _oracle_walks(len(ns), ns, rules, 7007)
    assert np.array_equal(res.best_e.cpu().numpy(), be)
    assert np.array_equal(res.final_e.cpu().numpy(), fe)
    assert np.array_equal(res.best_seq.cpu().numpy(), best)
    tr = res.trace.cpu().numpy()
    for w in range(len(ns)):
        assert np.array_equal(tr[w, : len(trs[w])], trs[w]), f"N={ns[w]}"


def test_tabu_n256_full_size_sampled(lb):
    # 4096 walks of N = 256 (four per workgroup, the default launch);
    # sampled walks against the oracle, properties at every walk
    W, n, seed = 4096, 256, 2561
    rules = I.Rules(I.STEPS_MULT_N, 1, I.TENURE_LINEAR, 1, 10, 0, 1, 5, 0, 1)
    say(f"tabu: W={W} N={n}, sampled walks against the oracle")
    res = lb.tabu_batch(rules, W, seed, n_uniform=n)
    be_g = res.best_e.cpu().numpy()
    fe_g = res.final_e.cpu().numpy()
    bs_g = res.best_seq.cpu().numpy()
    sample = [0, 1, 63, 64, 1000, 2047, 2048, 4094, 4095]
    sch = osched(rules)
    for w in sample:
        T, lo, hi = O.walk_schedule(n, sch, seed, w, 0)
        b, e1, f1, _, _ = O.tabu_walk(O.random_start(n, seed, w), seed, w, 0, T, lo, hi, 1)
        assert be_g[w] == e1 and fe_g[w] == f1
        assert np.array_equal(bs_g[w, :n], b)
    E = lb.energy_batch(res.best_seq, n_uniform=n).cpu().numpy()
    assert np.array_equal(E, be_g)
    assert np.all(be_g <= fe_g) and np.all(be_g % 4 == (n // 2) % 4)


@pytest.mark.parametrize("mode,children", [(0, 1), (1, 1), (2, 1), (2, 4), (0, 8)])
def test_memetic_long(lb, mode, children):
    ns = np.array([3, 64, 65, 128, 129, 200, 256], dtype=np.int32)
    rules = I.RULES_MEMETIC
    say(f"memetic N={list(ns)} K=20, mode {mode}, children {children}")
    ref = _oracle_memetic(ns, 20, rules, 5, 4321, children=0 if children == 1 else children)
    res = lb.memetic_run(20, rules, 5, len(ns), 4321, ns=ns, mode=mode, chunk=2,
                         children=children)
    for p, st in enumerate(ref):
        n = int(ns[p])
        assert res.best_e[p].item() == st.bestE
        assert np.array_equal(res.best_seq[p, :n].cpu().numpy(), st.best)
        assert res.gens_done[p].item() == 5


def test_server_long(lb):
    import time
    from paper_2504_00987_amd.labs import Server
    reqs = [(256, 11), (150, 12), (40, 13), (200, 14)]
    pops, gens, K = 2, 3, 12
    rules = I.RULES_MEMETIC
    say(f"server: requests N={[n for n, _ in reqs]}")
    srv = Server(lb, K, rules, max_slots=8, chunk=2)
    try:
        ids = [(srv.submit(n, s, pops, gens), n, s) for n, s in reqs]
        results = {}
        t0 = time.time()
        while len(results) < len(ids) and time.time() - t0 < 60:
            for rid, n, s in ids:
                if rid not in results:
                    r = srv.poll(rid, n)
                    if r is not None:
                        results[rid] = r
            time.sleep(0.005)
        assert len(results) == len(ids)
    finally:
        srv.close()
    for rid, n, s in ids:
        seq, e, _ = results[rid]
        alone = lb.memetic_run(K, rules, gens, pops, s, n_uniform=n, mode=2, chunk=gens)
        be = alone.best_e.cpu().numpy()
        p = int(np.argmin(be))
        assert e == be[p]
        assert np.array_equal(seq, alone.best_seq[p, :n].cpu().numpy())


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("children", [1, 4])
def test_server_alone_equals_mix(lb, children):
    import time
    from paper_2504_00987_amd.labs import Server
    reqs = I.serving_requests(10, seed=77)
    pops, gens, K = 3, 6, 16
    rules = I.RULES_MEMETIC
    say(f"server: {len(reqs)} requests, N={[n for n, _ in reqs]}")
    srv = Server(lb, K, rules, max_slots=8, chunk=2, children=children)
    try:
        ids = [(srv.submit(n, s, pops, gens), n, s) for n, s in reqs]
        results = {}
        t0 = time.time()
        while len(results) < len(ids) and time.time() - t0 < 60:
            for rid, n, s in ids:
                if rid not in results:
                    r = srv.poll(rid, n)
                    if r is not None:
                        results[rid] = r
            time.sleep(0.005)
        assert len(results) == len(ids)
    finally:
        srv.close()
    for rid, n, s in ids:
        seq, e, lat = results[rid]
        alone = lb.memetic_run(K, rules, gens, pops, s, n_uniform=n, mode=2, chunk=gens,
                               children=children)
        be = alone.best_e.cpu().numpy()
        p = int(np.argmin(be))
        assert e == be[p]
        assert np.array_equal(seq, alone.best_seq[p, :n].cpu().numpy())
        assert lat > 0
    # and the smallest request against the oracle
    n, s = min(reqs)
    ref = _oracle_memetic([n] * pops, K, rules, gens, s, children=children)
    rid = [r for r, nn, ss in ids if (nn, ss) == (n, s)][0]
    assert results[rid][1] == min(st.bestE for st in ref)


def test_server_cancel_and_errors(lb):
    import time
    from paper_2504_00987_amd import _lib
    from paper_2504_00987_amd.labs import Server
    say("server: cancel, unknown ids, invalid requests, counters")
    srv = Server(lb, 16, I.RULES_MEMETIC, max_slots=4, chunk=2)
    try:
        with pytest.raises(_lib.LabsError):
            srv.submit(2, 1, 2, 4)           # N below 3
        with pytest.raises(_lib.LabsError):
            srv.submit(40, 1, 5, 4)          # more replicas than slots
        keep = srv.submit(40, 11, 2, 30)
        drop = srv.submit(41, 12, 4, 10**6)  # queued behind `keep`, then cancelled
        srv.cancel(drop)
        with pytest.raises(_lib.LabsError) as err:
            srv.poll(999999, 40)
        assert err.value.code == _lib.LABS_E_NOTFOUND
        t0 = time.time()
        got = None
        while got is None and time.time() - t0 < 60:
            got = srv.poll(keep, 40)
            time.sleep(0.005)
        assert got is not None
        with pytest.raises(_lib.LabsError) as err:
            srv.poll(drop, 41)
        assert err.value.code == _lib.LABS_E_CANCELLED
        t0 = time.time()
        while srv.stats()[3] != 0 and time.time() - t0 < 30:  # cancelled slots are freed
            time.sleep(0.005)
        waiting, running, done, resident = srv.stats()
        assert done >= 1 and waiting == 0 and running == 0 and resident == 0
    finally:
        srv.close()
    alone = lb.memetic_run(16, I.RULES_MEMETIC, 30, 2, 11, n_uniform=40, mode=2, chunk=30)
    assert got[1] == int(alone.best_e.min().item())
