"""Python front end of liblabs: torch tensors in, torch tensors out.

PyTorch only provides device memory and the current stream; every step of
the search runs in the HIP library through the C ABI (``_lib``).  Names follow
``include/liblabs.h``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from .inputs import Rules, P_COMB_090

PLAIN, GRAPH, PERSISTENT = 0, 1, 2
MUT_INV_N, MUT_FIXED = 0, 1


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def tabu_params(rules: Rules) -> _lib.TabuParams:
    return _lib.TabuParams(rules.steps_rule, rules.steps_a, rules.tenure_rule, rules.lo_num,
                           rules.lo_den, rules.lo_add, rules.hi_num, rules.hi_den, rules.hi_add,
                           rules.aspiration, rules.slo_num, rules.slo_den, rules.shi_num,
                           rules.shi_den)


@dataclass
class TabuResult:
    best_seq: torch.Tensor   # int8 [W, out_stride]
    best_e: torch.Tensor     # int32 [W]
    final_e: torch.Tensor    # int32 [W]
    trace: torch.Tensor | None  # int16 [W, trace_stride]


@dataclass
class MemeticResult:
    best_seq: torch.Tensor   # int8 [P, out_stride]
    best_e: torch.Tensor     # int32 [P]
    hit_gen: torch.Tensor    # int64 [P]
    gens_done: torch.Tensor  # int64 [P]


def _default_stride(ns_arr, n_uniform: int) -> int:
    """Output row stride: 128, or the longest sequence when that is longer."""
    n_max = int(ns_arr.max()) if ns_arr is not None and ns_arr.size else n_uniform
    return max(128, n_max)


class Labs:
    """A liblabs handle bound to one GPU."""

    def __init__(self, device: int = 0):
        self.L = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.L.labs_create(ctypes.byref(h), device)
        if rc != _lib.LABS_OK:
            raise _lib.LabsError(rc, f"labs_create(device={device}) failed")
        self.h = h

    def close(self):
        if self.h:
            self.L.labs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        _lib.check(rc, self.h)

    # -- Eq. (2) -----------------------------------------------------------
    def energy_batch(self, seqs: torch.Tensor, ns: torch.Tensor | None = None,
                     n_uniform: int = 0, stream=None) -> torch.Tensor:
        assert seqs.is_cuda and seqs.dtype == torch.int8 and seqs.dim() == 2 and seqs.is_contiguous()
        if ns is not None:
            assert ns.is_cuda and ns.dtype == torch.int32 and ns.numel() == seqs.shape[0]
        out = torch.empty(seqs.shape[0], dtype=torch.int32, device=seqs.device)
        self._check(self.L.labs_energy_batch(self.h, _ptr(seqs), _ptr(ns), n_uniform,
                                             seqs.shape[1], seqs.shape[0], _ptr(out),
                                             _stream(stream)))
        return out

    def skew_deviation(self, seqs: torch.Tensor, ns: torch.Tensor | None = None,
                       n_uniform: int = 0, stream=None) -> torch.Tensor:
        """d(S) of App. A for every row (odd N: rotations; even N: rotation
        and one deletion)."""
        assert seqs.is_cuda and seqs.dtype == torch.int8 and seqs.dim() == 2 and seqs.is_contiguous()
        if ns is not None:
            assert ns.is_cuda and ns.dtype == torch.int32 and ns.numel() == seqs.shape[0]
        out = torch.empty(seqs.shape[0], dtype=torch.int32, device=seqs.device)
        self._check(self.L.labs_skew_deviation_batch(self.h, _ptr(seqs), _ptr(ns), n_uniform,
                                                     seqs.shape[1], seqs.shape[0], _ptr(out),
                                                     _stream(stream)))
        return out

    # -- Alg. 2 / Alg. 4 -----------------------------------------------------
    def bruteforce_min(self, n: int):
        """Exhaustive minimum energy at length n: (E_min, how many of the 2^n
        sequences attain it, the attaining int8 sequence with s_0 = +1 whose
        bit pattern is smallest)."""
        e = ctypes.c_int32(0)
        cnt = ctypes.c_int64(0)
        seq = np.zeros(n, dtype=np.int8)
        self._check(self.L.labs_bruteforce_min(self.h, n, ctypes.byref(e), ctypes.byref(cnt),
                                               seq.ctypes.data_as(ctypes.c_void_p)))
        return e.value, cnt.value, seq

    def skew_bruteforce_min(self, n: int):
        """Exhaustive minimum over the skew-symmetric sequences of odd length
        n (Sec. II.C): (E_min, how many of the 2^((n+1)/2) attain it, the
        attaining sequence with s_0 = +1 whose free spins form the smallest
        integer)."""
        e = ctypes.c_int32(0)
        cnt = ctypes.c_int64(0)
        seq = np.zeros(n, dtype=np.int8)
        self._check(self.L.labs_skew_bruteforce_min(self.h, n, ctypes.byref(e), ctypes.byref(cnt),
                                                    seq.ctypes.data_as(ctypes.c_void_p)))
        return e.value, cnt.value, seq

    def tabu_batch(self, rules: Rules, walks: int, seed: int, ns=None, n_uniform: int = 0,
                   starts: torch.Tensor | None = None, out_stride: int | None = None,
                   trace_stride: int = 0, out=None, stream=None,
                   noalloc: bool = False) -> TabuResult:
        """Independent tabu walks (labs_tabu_batch; with ``noalloc`` the
        allocation-free labs_tabu_batch_noalloc, whose per-walk lengths are
        read by a copy on the stream: the array is kept alive on the result)."""
        dev = torch.device("cuda", self.device)
        ns_arr = None
        if ns is not None:
            ns_arr = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
            assert ns_arr.shape == (walks,)
        if out_stride is None:
            out_stride = _default_stride(ns_arr, n_uniform)
        if starts is not None:
            assert starts.is_cuda and starts.dtype == torch.int8 and starts.is_contiguous()
            assert starts.shape[0] == walks
        if out is None:
            best = torch.empty((walks, out_stride), dtype=torch.int8, device=dev)
            be = torch.empty(walks, dtype=torch.int32, device=dev)
            fe = torch.empty(walks, dtype=torch.int32, device=dev)
            tr = torch.zeros((walks, trace_stride), dtype=torch.int16, device=dev) if trace_stride else None
        else:
            best, be, fe, tr = out
            out_stride = best.shape[1]
            trace_stride = 0 if tr is None else tr.shape[1]
        p = tabu_params(rules)
        fn = self.L.labs_tabu_batch_noalloc if noalloc else self.L.labs_tabu_batch
        self._check(fn(
            self.h, ctypes.byref(p), _ptr(starts), 0 if starts is None else starts.shape[1],
            None if ns_arr is None else ns_arr.ctypes.data_as(ctypes.c_void_p), n_uniform,
            walks, ctypes.c_uint64(seed & (2**64 - 1)), _ptr(best), out_stride, _ptr(be),
            _ptr(fe), _ptr(tr), trace_stride, _stream(stream)))
        res = TabuResult(best, be, fe, tr)
        res._lengths = ns_arr  # read by a copy on the stream in the allocation-free form
        return res

    def device_peaks(self) -> dict:
        """Measured dot4 / int32 / LDS throughput of this GPU (labs_device_peaks)."""
        v = [ctypes.c_double(0.0) for _ in range(4)]
        self._check(self.L.labs_device_peaks(self.h, *[ctypes.byref(x) for x in v]))
        return {"dot4_ops_per_s": v[0].value, "int32_ops_per_s": v[1].value,
                "lds_bytes_per_s": v[2].value, "clock_hz": v[3].value}

    def set_launch(self, group_lanes: int | None = None, walks_per_group: int = 1,
                   persistent: int = 0, groups_per_cu: int = 0, layout: int = 0):
        """labs_set_launch; no arguments clears the override."""
        if group_lanes is None:
            self._check(self.L.labs_set_launch(self.h, None))
            return
        l = _lib.Launch(group_lanes, walks_per_group, persistent, groups_per_cu, layout)
        self._check(self.L.labs_set_launch(self.h, ctypes.byref(l)))

    def get_launch(self, n_min: int, n_max: int | None = None):
        """(group_lanes, walks_per_group, persistent, groups_per_cu, layout) for a
        batch of lengths in [n_min, n_max]."""
        l = _lib.Launch()
        self._check(self.L.labs_get_launch(self.h, n_min, n_min if n_max is None else n_max,
                                           ctypes.byref(l)))
        return (l.group_lanes, l.walks_per_group, l.persistent, l.groups_per_cu, l.layout)

    def autotune(self, rules: Rules, n_min: int, n_max: int, walks: int, seed: int = 7) -> int:
        tried = ctypes.c_int32(0)
        p = tabu_params(rules)
        self._check(self.L.labs_autotune(self.h, ctypes.byref(p), n_min, n_max, walks,
                                         ctypes.c_uint64(seed), ctypes.byref(tried)))
        return tried.value

    # -- Alg. 1 / Alg. 3 -----------------------------------------------------
    @staticmethod
    def memetic_params(K: int, rules: Rules, generations: int, p_comb: int = P_COMB_090,
                       mut_rule: int = MUT_INV_N, p_mut: int = 0, target: int = -1,
                       mode: int = PERSISTENT, chunk: int = 64,
                       stop_all: int = 0, waves_per_replica: int = 0,
                       children: int = 1, resume: int = 0) -> _lib.MemeticParams:
        return _lib.MemeticParams(K, p_comb, mut_rule, p_mut, tabu_params(rules), generations,
                                  target, mode, chunk, stop_all, waves_per_replica, children,
                                  resume)

    def memetic_run(self, K: int, rules: Rules, generations: int, pops: int, seed: int,
                    ns=None, n_uniform: int = 0, out_stride: int | None = None, stream=None,
                    **kw) -> MemeticResult:
        dev = torch.device("cuda", self.device)
        ns_arr = None
        if ns is not None:
            ns_arr = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
            assert ns_arr.shape == (pops,)
        if out_stride is None:
            out_stride = _default_stride(ns_arr, n_uniform)
        best = torch.empty((pops, out_stride), dtype=torch.int8, device=dev)
        be = torch.empty(pops, dtype=torch.int32, device=dev)
        hit = torch.empty(pops, dtype=torch.int64, device=dev)
        done = torch.empty(pops, dtype=torch.int64, device=dev)
        p = self.memetic_params(K, rules, generations, **kw)
        # kept for a caller that catches LABS_E_CANCELLED: the outputs hold
        # the state where the run stopped
        self._last_memetic = MemeticResult(best, be, hit, done)
        self._check(self.L.labs_memetic_run(
            self.h, ctypes.byref(p), None if ns_arr is None else ns_arr.ctypes.data_as(ctypes.c_void_p),
            n_uniform, pops, ctypes.c_uint64(seed & (2**64 - 1)), _ptr(best), out_stride,
            _ptr(be), _ptr(hit), _ptr(done), _stream(stream)))
        return MemeticResult(best, be, hit, done)


    def cancel(self):
        """labs_cancel: stop this handle's memetic runs at their next chunk boundary."""
        self._check(self.L.labs_cancel(self.h))

    def memetic_save(self, stream=None) -> bytes:
        """labs_memetic_save: a checkpoint of the replicas this handle holds."""
        n = ctypes.c_int64(0)
        self._check(self.L.labs_memetic_checkpoint_bytes(self.h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.L.labs_memetic_save(self.h, buf, n.value, _stream(stream)))
        return buf.raw

    def memetic_load(self, blob: bytes, stream=None):
        """labs_memetic_load: hold the replicas of a checkpoint (resume=1 continues them)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(self.L.labs_memetic_load(self.h, buf, len(blob), _stream(stream)))


class Server:
    """Continuous-batching request loop over resident memetic replicas."""

    def __init__(self, labs: Labs, K: int, rules: Rules, max_slots: int, chunk: int = 8,
                 target: int = -1, p_comb: int = P_COMB_090, mut_rule: int = MUT_INV_N,
                 p_mut: int = 0, children: int = 1):
        self.labs = labs
        self.L = labs.L
        p = Labs.memetic_params(K, rules, 0, p_comb=p_comb, mut_rule=mut_rule, p_mut=p_mut,
                                target=target, chunk=chunk, children=children)
        s = ctypes.c_void_p()
        _lib.check(self.L.labs_server_create(labs.h, ctypes.byref(p), max_slots, ctypes.byref(s)),
                   labs.h)
        self.s = s

    def submit(self, n: int, seed: int, pops: int, generations: int) -> int:
        rid = ctypes.c_int64(0)
        rc = self.L.labs_server_submit(self.s, n, ctypes.c_uint64(seed & (2**64 - 1)), pops,
                                       generations, ctypes.byref(rid))
        _lib.check(rc)
        return rid.value

    def poll(self, rid: int, n: int):
        """None while pending; (best_seq int8 numpy [n], best_e, latency_s) when done."""
        buf = np.zeros(n, dtype=np.int8)
        e = ctypes.c_int32(0)
        lat = ctypes.c_double(0.0)
        rc = self.L.labs_server_poll(self.s, rid, buf.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.byref(e), ctypes.byref(lat))
        if rc == _lib.LABS_E_AGAIN:
            return None
        _lib.check(rc)
        return buf, e.value, lat.value

    def cancel(self, rid: int):
        _lib.check(self.L.labs_server_cancel(self.s, rid))

    def stats(self):
        v = [ctypes.c_int64(0) for _ in range(4)]
        _lib.check(self.L.labs_server_stats(self.s, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def close(self):
        if self.s:
            self.L.labs_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
