"""The allocation-free tabu batch (labs_tabu_batch_noalloc) against
labs_tabu_batch, through the C ABI: bit-exact best sequences, best and final
energies and per-step traces on two calls in a row, the second smaller, over
every length class and launch form; and its size limit."""
import sys

import numpy as np
import pytest

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


def _same(a, b):
    for x, y in ((a.best_seq, b.best_seq), (a.best_e, b.best_e), (a.final_e, b.final_e)):
        assert torch.equal(x, y)
    if a.trace is not None:
        assert torch.equal(a.trace, b.trace)


@pytest.mark.parametrize("launch", [None, (64, 1, 1, 0, 0), (256, 4, 1, 2, 0), (128, 2, 0, 0, 0),
                                    (128, 1, 1, 0, 1), (64, 4, 1, 0, 0), (128, 4, 0, 0, 0)])
def test_noalloc_equals_allocating_entry_point(lb, launch):
    rules = I.rules_tabu(3)
    if launch is None:
        lb.set_launch(None)
    else:
        lb.set_launch(*launch)
    try:
        # first call: every length class, ragged, traced
        ns1 = I.uneven_lengths(3000, 3, 256, seed=51)
        say(f"noalloc: launch {launch}, 3000 walks of N 3..256 traced")
        ref = lb.tabu_batch(rules, 3000, 2101, ns=ns1, trace_stride=768)
        got = lb.tabu_batch(rules, 3000, 2101, ns=ns1, trace_stride=768, noalloc=True)
        torch.cuda.synchronize()
        _same(ref, got)
        # second call, smaller: the short classes only, untraced
        ns2 = I.uneven_lengths(777, 48, 120, seed=52)
        say(f"noalloc: launch {launch}, 777 walks of N 48..120")
        ref = lb.tabu_batch(rules, 777, 2102, ns=ns2)
        got = lb.tabu_batch(rules, 777, 2102, ns=ns2, noalloc=True)
        torch.cuda.synchronize()
        _same(ref, got)
        # one length (no per-walk lengths), then a handful of walks
        say(f"noalloc: launch {launch}, 4096 walks of N=64, then 5 of N=17")
        ref = lb.tabu_batch(rules, 4096, 2103, n_uniform=64)
        got = lb.tabu_batch(rules, 4096, 2103, n_uniform=64, noalloc=True)
        torch.cuda.synchronize()
        _same(ref, got)
        ref = lb.tabu_batch(rules, 5, 2104, n_uniform=17, trace_stride=51)
        got = lb.tabu_batch(rules, 5, 2104, n_uniform=17, trace_stride=51, noalloc=True)
        torch.cuda.synchronize()
        _same(ref, got)
    finally:
        lb.set_launch(None)


def test_noalloc_caller_starts_and_limits(lb):
    from paper_2504_00987_amd import _lib
    rules = I.rules_tabu(2)
    ns = I.uneven_lengths(500, 60, 140, seed=53)
    S = torch.from_numpy(I.random_pm1_ragged(ns, 160, seed=54)).cuda()
    say("noalloc: caller starts, 500 walks of N 60..140")
    ref = lb.tabu_batch(rules, 500, 9, ns=ns, starts=S)
    got = lb.tabu_batch(rules, 500, 9, ns=ns, starts=S, noalloc=True)
    torch.cuda.synchronize()
    _same(ref, got)
    # per-walk lengths beyond the fixed scratch are rejected before any work
    big = np.full(_lib.NOALLOC_MAX_WALKS + 1, 40, dtype=np.int32)
    with pytest.raises(_lib.LabsError) as ei:
        lb.tabu_batch(rules, big.size, 1, ns=big, noalloc=True)
    assert ei.value.code == _lib.LABS_E_INVAL
    # ... while a batch of one length that size needs the queue heads only
    say("noalloc: 65537 walks of N=20")
    ref = lb.tabu_batch(rules, big.size, 1, n_uniform=20)
    got = lb.tabu_batch(rules, big.size, 1, n_uniform=20, noalloc=True)
    torch.cuda.synchronize()
    _same(ref, got)
    # W = 0 is a no-op
    lb.tabu_batch(rules, 0, 1, n_uniform=20, noalloc=True)


@pytest.mark.parametrize("launch", [None, (64, 1, 1, 0, 0), (64, 2, 0, 0, 0)])
def test_noalloc_replayed_in_a_graph(lb, launch):
    # what the allocation-free entry point is for: a call captured into a HIP
    # graph (one length, so the call copies nothing from the host), replayed
    # several times with eager work between the replays; every replay equals
    # the eager call (the persistent launch resets its queue head with a fill
    # kernel inside the graph)
    rules = I.rules_tabu(2)
    W, seed = 2048, 4321
    n = 24 if launch == (64, 2, 0, 0, 0) else 64
    say(f"noalloc in a graph: launch {launch}, {W} walks of N={n}")
    if launch is not None:
        lb.set_launch(*launch)
    try:
        ref = lb.tabu_batch(rules, W, seed, n_uniform=n)
        torch.cuda.synchronize()
        dev = torch.device("cuda", 0)
        out = (torch.empty((W, 128), dtype=torch.int8, device=dev),
               torch.empty(W, dtype=torch.int32, device=dev),
               torch.empty(W, dtype=torch.int32, device=dev), None)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # a first call on the capture stream
            lb.tabu_batch(rules, W, seed, n_uniform=n, out=out, stream=s, noalloc=True)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            lb.tabu_batch(rules, W, seed, n_uniform=n, out=out, stream=s, noalloc=True)
        torch.cuda.synchronize()
        for rep in range(4):
            out[0].fill_(7)
            out[1].fill_(-1)
            out[2].fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out[0], ref.best_seq), f"replay {rep}"
            assert torch.equal(out[1], ref.best_e) and torch.equal(out[2], ref.final_e)
            # eager work on the same scratch between replays
            lb.tabu_batch(rules, 64, rep, n_uniform=20, noalloc=True)
            torch.cuda.synchronize()
        del g
    finally:
        lb.set_launch(None)
