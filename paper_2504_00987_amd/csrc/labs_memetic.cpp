// labs_memetic_run: memetic replicas (Alg. 1 / Alg. 3) driven one generation
// per launch (PLAIN), as a replayed graph of one-generation launches (GRAPH),
// or `chunk` generations per launch with the population resident in LDS
// (PERSISTENT).  All three give identical results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "labs_handle.h"

namespace liblabs {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

MemeticStateDev carve_state(void *base, int S, int K, size_t *bytes_out) {
    MemeticStateDev st;
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = p ? p + off : nullptr;
        off += align256(bytes);
        return q;
    };
    st.pop = (uint64_t *)take((size_t)S * K * kStateWords * sizeof(uint64_t));
    st.popE = (int32_t *)take((size_t)S * K * sizeof(int32_t));
    st.best = (uint64_t *)take((size_t)S * kStateWords * sizeof(uint64_t));
    st.bestE = (int32_t *)take((size_t)S * sizeof(int32_t));
    st.gen = (int64_t *)take((size_t)S * sizeof(int64_t));
    st.hit = (int64_t *)take((size_t)S * sizeof(int64_t));
    if (bytes_out) *bytes_out = off;
    return st;
}

// Device layout of a run in `mem`: [slots][ns][flags: any_hit, stop][state].
struct MemLayout {
    size_t off_ns, off_flag, off_state, state_bytes;
    size_t total() const { return off_state + state_bytes; }
};
static MemLayout mem_layout(int pops, int K) {
    MemLayout l;
    carve_state(nullptr, pops, K, &l.state_bytes);
    const size_t slots_bytes = (size_t)pops * sizeof(MemeticSlot);
    l.off_ns = align256(slots_bytes);
    l.off_flag = l.off_ns + align256((size_t)pops * 4);
    l.off_state = l.off_flag + 256;
    return l;
}

static_assert(kMaxChildren == LABS_MAX_CHILDREN, "kernel and ABI limits agree");

int split_wide(const labs_handle *h, int waves_per_replica, int64_t n_wide) {
    if (waves_per_replica != 0) return waves_per_replica == 2;
    return n_wide <= 2 * (int64_t)std::max(h->num_cus, 1);
}

int check_children(labs_handle *h, int children, int classes) {
    if (children > 1 && (classes & 4) && children > h->max_children_wide)
        return fail(h, LABS_E_INVAL, "children=%d: this device fits at most %d per generation "
                    "for N > 128", children, h->max_children_wide);
    return LABS_OK;
}

int check_memetic(labs_handle *h, const labs_memetic_params *p) {
    if (!p) return fail(h, LABS_E_INVAL, "null memetic params");
    if (p->K < 2 || p->K > LABS_MAX_K) return fail(h, LABS_E_INVAL, "K=%d out of [2, %d]", p->K, LABS_MAX_K);
    if (p->mut_rule != LABS_MUT_INV_N && p->mut_rule != LABS_MUT_FIXED)
        return fail(h, LABS_E_INVAL, "unknown mut_rule %d", p->mut_rule);
    if (p->generations < 0) return fail(h, LABS_E_INVAL, "generations < 0");
    if (p->generations > 0xffffffffLL) return fail(h, LABS_E_INVAL, "generations >= 2^32");
    if (p->mode < LABS_MODE_PLAIN || p->mode > LABS_MODE_PERSISTENT)
        return fail(h, LABS_E_INVAL, "unknown mode %d", p->mode);
    if (p->chunk < 1 || p->chunk > (1 << 20)) return fail(h, LABS_E_INVAL, "chunk out of [1, 2^20]");
    if (p->stop_all != 0 && p->stop_all != 1) return fail(h, LABS_E_INVAL, "stop_all must be 0 or 1");
    if (p->resume != 0 && p->resume != 1) return fail(h, LABS_E_INVAL, "resume must be 0 or 1");
    if (p->waves_per_replica < 0 || p->waves_per_replica > 2)
        return fail(h, LABS_E_INVAL, "waves_per_replica must be 0, 1 or 2");
    if (p->children < 0 || p->children > LABS_MAX_CHILDREN)
        return fail(h, LABS_E_INVAL, "children must be in [0, %d]", LABS_MAX_CHILDREN);
    return LABS_OK;
}

}  // namespace liblabs

using namespace liblabs;

namespace {

// Graphs of earlier runs whose last launch has completed are destroyed.
void reap_graphs(labs_handle *h, bool wait) {
    for (size_t i = 0; i < h->retired.size();) {
        labs_handle::Retired &r = h->retired[i];
        if (wait) hipEventSynchronize(r.done);
        if (hipEventQuery(r.done) == hipSuccess) {
            hipGraphExecDestroy(r.exec);
            hipGraphDestroy(r.graph);
            hipEventDestroy(r.done);
            r = h->retired.back();
            h->retired.pop_back();
        } else {
            (void)hipGetLastError();  // hipErrorNotReady
            ++i;
        }
    }
}

// The memetic state buffer `mem` is shared by the handle's runs on any
// stream: a new run waits (on the GPU) for the previous one, and the host
// waits only when the buffer must grow.
int mem_acquire(labs_handle *h, hipStream_t s, size_t bytes) {
    if (h->mem_event_valid) {
        hipError_t e = bytes > h->mem.size ? hipEventSynchronize(h->mem_event)
                                           : hipStreamWaitEvent(s, h->mem_event, 0);
        if (e != hipSuccess) return hip_fail(h, e, "memetic state wait");
    }
    return h->mem.reserve(h, bytes);
}

}  // namespace

extern "C" int labs_cancel(labs_handle *h) {
    if (!h) return LABS_E_INVAL;
    const uint32_t next = h->cancel_epoch.fetch_add(1u) + 1u;
    if (h->cancel_host) __atomic_store_n(&h->cancel_host[0], next, __ATOMIC_SEQ_CST);
    return LABS_OK;
}

extern "C" int labs_memetic_run(labs_handle *h, const labs_memetic_params *p,
                                const int32_t *ns_host, int32_t n_uniform, int32_t pops,
                                uint64_t seed, int8_t *best_seq, int32_t out_stride,
                                int32_t *best_e, int64_t *hit_gen, int64_t *gens_done,
                                void *stream) {
    if (!h) return LABS_E_INVAL;
    h->last_error.clear();
    int rc = check_memetic(h, p);
    if (rc) return rc;
    if (pops < 0) return fail(h, LABS_E_INVAL, "pops < 0");
    // one workgroup of up to 8 wavefronts per replica in one grid
    if (pops > LABS_MAX_REPLICAS) return fail(h, LABS_E_INVAL, "pops > %d", LABS_MAX_REPLICAS);
    if (pops == 0) return LABS_OK;
    if (!best_seq || !best_e) return fail(h, LABS_E_INVAL, "null output");
    const RuleParams rule = to_rule(p->tabu);
    int n_max = 0;
    char seen[LABS_MAX_N + 1] = {};
    for (int i = 0; i < pops; ++i) {
        const int n = ns_host ? ns_host[i] : n_uniform;
        if (n < LABS_MIN_N || n > LABS_MAX_N)
            return fail(h, LABS_E_INVAL, "N=%d out of [%d, %d]", n, LABS_MIN_N, LABS_MAX_N);
        if (!seen[n]) {
            seen[n] = 1;
            if ((rc = check_rule(h, rule, n))) return rc;
        }
        n_max = std::max(n_max, n);
    }
    if (out_stride < n_max) return fail(h, LABS_E_INVAL, "out_stride=%d < N=%d", out_stride, n_max);
    int classes = 0;
    int64_t n_wide = 0;
    for (int i = 0; i < pops; ++i) {
        const int c = memetic_class(ns_host ? ns_host[i] : n_uniform);
        classes |= 1 << c;
        n_wide += c == 1;
    }
    const int children = std::max(1, (int)p->children);
    if ((rc = check_children(h, children, classes))) return rc;
    const bool resume = p->resume == 1;
    if (resume) {
        const auto &hd = h->held;
        if (!hd.valid) return fail(h, LABS_E_INVAL, "resume: this handle holds no memetic replicas");
        if (hd.pops != pops || hd.K != p->K || hd.seed != seed)
            return fail(h, LABS_E_INVAL, "resume: pops, K or seed differ from the held replicas "
                        "(%d, %d, %llu)", hd.pops, hd.K, (unsigned long long)hd.seed);
        for (int i = 0; i < pops; ++i)
            if ((ns_host ? ns_host[i] : n_uniform) != hd.ns[(size_t)i])
                return fail(h, LABS_E_INVAL, "resume: the length of replica %d differs", i);
    }

    // Everything below is enqueued on the caller's stream.
    DeviceGuard g(h->device);
    hipStream_t s = (hipStream_t)stream;
    reap_graphs(h, false);
    const uint32_t epoch = h->cancel_epoch.load();

    // Device memory: [slots][ns][flags: any_hit, stop][state]
    const MemLayout lay = mem_layout(pops, p->K);
    const size_t off_ns = lay.off_ns, off_flag = lay.off_flag;
    // A fresh run replaces the held replicas (valid again once enqueued;
    // growing the buffer frees the old one); a resumed run keeps the size.
    if (!resume) h->held.valid = false;
    if ((rc = mem_acquire(h, s, lay.total()))) return rc;
    char *base = (char *)h->mem.ptr;
    MemeticSlot *d_slots = (MemeticSlot *)base;
    int32_t *d_ns = (int32_t *)(base + off_ns);
    uint32_t *d_flag = (uint32_t *)(base + off_flag);  // [0] any_hit, [1] stop
    MemeticStateDev st = carve_state(base + lay.off_state, pops, p->K, nullptr);

    // A resumed run starts from the smallest generation count among the
    // replicas still going (read back once); launches past a replica's
    // limit do nothing, so a lower start only costs launches.
    int64_t gen_start = 0;
    if (resume) {
        std::vector<int64_t> gen((size_t)pops);
        std::vector<int32_t> be((size_t)pops);
        hipError_t e = hipMemcpyAsync(gen.data(), st.gen, (size_t)pops * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(be.data(), st.bestE, (size_t)pops * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "resume: generation counts");
        gen_start = p->generations;
        for (int i = 0; i < pops; ++i)
            if (gen[(size_t)i] < p->generations && (p->target_e < 0 || be[(size_t)i] > p->target_e))
                gen_start = std::min(gen_start, gen[(size_t)i]);
    }

    const size_t stage = off_flag;  // slots + ns
    if ((rc = stage_acquire(h, stage))) return rc;
    std::memset(h->pin.ptr, 0, stage);
    MemeticSlot *hs = (MemeticSlot *)h->pin.ptr;
    int32_t *hn = (int32_t *)((char *)h->pin.ptr + off_ns);
    const int target = p->target_e;
    for (int i = 0; i < pops; ++i) {
        const int n = ns_host ? ns_host[i] : n_uniform;
        hs[i].n = n;
        hs[i].pop_id = (uint32_t)i;
        hs[i].k0 = (uint32_t)(seed & 0xffffffffu);
        hs[i].k1 = (uint32_t)(seed >> 32);
        hs[i].gen_limit = p->generations;
        hs[i].target = target < 0 ? -1 : target;
        hs[i].state = i;
        hn[i] = n;
    }
    hipError_t e = hipMemcpyAsync(base, h->pin.ptr, stage, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync(slots)");
    if ((rc = stage_release(h, s))) return rc;  // the staging copy is in flight

    MemeticLaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.slots = d_slots;
    a.n_slots = pops;
    a.K = p->K;
    a.p_comb = p->p_comb;
    a.mut_rule = p->mut_rule;
    a.p_mut = p->p_mut;
    a.rule = rule;
    a.st = st;
    a.any_hit = d_flag;
    a.stop = d_flag + 1;
    a.classes = classes;
    a.split_wide = split_wide(h, p->waves_per_replica, n_wide);
    a.children = children;
    if (resume) {
        // any_hit carries over (the global flag of the run being continued);
        // the stop flag is this run's
        if ((e = launch_fill_u32(d_flag + 1, 0u, 1, s)) != hipSuccess) return hip_fail(h, e, "fill");
    } else {
        if ((e = launch_fill_u32(d_flag, 0u, 2, s)) != hipSuccess) return hip_fail(h, e, "fill");
        if ((e = launch_memetic_init(a, s)) != hipSuccess) return hip_fail(h, e, "memetic init");
    }

    // Chunk boundaries: the latch turns a reached target (stop_all) or a
    // cancel into the stop flag every later launch of the run reads first,
    // so the outcome is fixed by the chunk in which the first replica hit,
    // whenever the host notices.  With stop_all the host reads the flag back
    // two chunks behind and stops enqueueing once it is set.
    const bool stop_all = p->stop_all && target >= 0;
    const int64_t G = p->generations;
    const int64_t chunk = p->chunk;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    if (p->mode == LABS_MODE_GRAPH && G > 0) {
        // Capture the latch and `chunk` one-generation launches once (on the
        // handle's stream, which may be captured; the caller's may be the
        // null stream); replay them on the caller's stream.
        MemeticLaunchArgs one = a;
        one.gens = 1;
        const int64_t n_launch = std::min<int64_t>(chunk, G);
        e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
        e = launch_memetic_latch(d_flag, d_flag + 1, h->cancel_dev, epoch, stop_all, h->stream);
        for (int64_t i = 0; i < n_launch && e == hipSuccess; ++i)
            e = launch_memetic_advance(one, h->stream, &h->sides);
        hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return hip_fail(h, e != hipSuccess ? e : e2, "graph capture");
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(graph);
            return hip_fail(h, e, "hipGraphInstantiate");
        }
    }

    rc = LABS_OK;
    bool cancelled = false;
    constexpr int kLag = 2;
    int64_t n_chunks = 0;
    for (int64_t done = gen_start; done < G;) {
        const int64_t step = std::min(chunk, G - done);
        if (p->mode == LABS_MODE_GRAPH) {
            // launches past a replica's generation limit return at once, so
            // the final replay may safely run past G
            e = hipGraphLaunch(exec, s);
        } else {
            e = launch_memetic_latch(d_flag, d_flag + 1, h->cancel_dev, epoch, stop_all, s);
            if (p->mode == LABS_MODE_PLAIN) {
                MemeticLaunchArgs one = a;
                one.gens = 1;
                for (int64_t i = 0; i < step && e == hipSuccess; ++i)
                    e = launch_memetic_advance(one, s, &h->sides);
            } else if (e == hipSuccess) {
                MemeticLaunchArgs many = a;
                many.gens = (int32_t)step;
                e = launch_memetic_advance(many, s, &h->sides);
            }
        }
        if (e != hipSuccess) {
            rc = hip_fail(h, e, "memetic advance");
            break;
        }
        done += p->mode == LABS_MODE_GRAPH ? std::min<int64_t>(chunk, G) : step;
        if (h->cancel_epoch.load() != epoch) {
            cancelled = true;  // the device stops at its next latch
            break;
        }
        if (stop_all && done < G) {
            // snapshot of any_hit after this chunk, read kLag chunks later
            const int slot = (int)(n_chunks % 4);
            e = hipMemcpyAsync(h->cancel_host + 1 + slot, d_flag, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipEventRecord(h->poll_event[slot], s);
            if (e == hipSuccess && n_chunks >= kLag) {
                const int old = (int)((n_chunks - kLag) % 4);
                e = hipEventSynchronize(h->poll_event[old]);
                if (e == hipSuccess && __atomic_load_n(&h->cancel_host[1 + old], __ATOMIC_ACQUIRE)) {
                    ++n_chunks;
                    break;
                }
            }
            if (e != hipSuccess) {
                rc = hip_fail(h, e, "flag poll");
                break;
            }
            ++n_chunks;
        }
    }
    if (rc == LABS_OK) {
        e = launch_gather_best(st, nullptr, d_ns, 0, pops, best_seq, out_stride, best_e, hit_gen,
                               gens_done, s);
        if (e != hipSuccess) rc = hip_fail(h, e, "gather");
    }
    hipError_t er = hipEventRecord(h->mem_event, s);
    if (er == hipSuccess) h->mem_event_valid = true;
    if (exec) {
        hipEvent_t done_ev = nullptr;
        if (er == hipSuccess && hipEventCreateWithFlags(&done_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventRecord(done_ev, s) == hipSuccess) {
            h->retired.push_back({exec, graph, done_ev});
        } else {
            // cannot tell when its launches end: wait for them here
            hipStreamSynchronize(s);
            if (done_ev) hipEventDestroy(done_ev);
            hipGraphExecDestroy(exec);
            hipGraphDestroy(graph);
        }
    }
    if (rc) return rc;
    if (er != hipSuccess) return hip_fail(h, er, "hipEventRecord");
    if (!resume) {
        h->held.valid = true;
        h->held.pops = pops;
        h->held.K = p->K;
        h->held.seed = seed;
        h->held.ns.assign((size_t)pops, n_uniform);
        if (ns_host) h->held.ns.assign(ns_host, ns_host + pops);
    }
    if (cancelled) return fail(h, LABS_E_CANCELLED, "cancelled by labs_cancel");
    return LABS_OK;
}

// ---------------------------------------------------------------------------
// Checkpoints of the held replicas.
// ---------------------------------------------------------------------------
namespace {

constexpr char kCkptMagic[8] = {'L', 'A', 'B', 'S', 'M', 'E', 'M', '\0'};
constexpr uint32_t kCkptVersion = 1;
constexpr size_t kCkptHeaderBytes = 256;

struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t pops, K;
    uint32_t any_hit;   // a replica has reached the target (the global flag)
    uint64_t seed;
    int64_t gen_min;    // smallest generation count (informative)
    int64_t state_bytes;
};
static_assert(sizeof(CkptHeader) <= kCkptHeaderBytes, "header fits its slot");

size_t ckpt_bytes(int pops, int K) {
    return kCkptHeaderBytes + align256((size_t)pops * 4) + mem_layout(pops, K).state_bytes;
}

}  // namespace

extern "C" int labs_memetic_checkpoint_bytes(labs_handle *h, int64_t *bytes) {
    if (!h || !bytes) return LABS_E_INVAL;
    h->last_error.clear();
    if (!h->held.valid) return fail(h, LABS_E_INVAL, "this handle holds no memetic replicas");
    *bytes = (int64_t)ckpt_bytes(h->held.pops, h->held.K);
    return LABS_OK;
}

extern "C" int labs_memetic_save(labs_handle *h, void *dst, int64_t bytes, void *stream) {
    if (!h) return LABS_E_INVAL;
    h->last_error.clear();
    if (!dst) return fail(h, LABS_E_INVAL, "null destination");
    if (!h->held.valid) return fail(h, LABS_E_INVAL, "this handle holds no memetic replicas");
    const int pops = h->held.pops, K = h->held.K;
    const size_t need = ckpt_bytes(pops, K);
    if (bytes < (int64_t)need) return fail(h, LABS_E_INVAL, "bytes=%lld < %zu", (long long)bytes, need);
    DeviceGuard g(h->device);
    hipStream_t s = (hipStream_t)stream;
    const MemLayout lay = mem_layout(pops, K);
    char *out = (char *)dst;
    char *state = out + kCkptHeaderBytes + align256((size_t)pops * 4);
    uint32_t any_hit = 0;
    hipError_t e = hipSuccess;
    if (h->mem_event_valid) e = hipStreamWaitEvent(s, h->mem_event, 0);
    const char *base = (const char *)h->mem.ptr;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&any_hit, base + lay.off_flag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(state, base + lay.off_state, lay.state_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "checkpoint copy");
    CkptHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.magic, kCkptMagic, sizeof(kCkptMagic));
    hd.version = kCkptVersion;
    hd.pops = pops;
    hd.K = K;
    hd.any_hit = any_hit;
    hd.seed = h->held.seed;
    hd.state_bytes = (int64_t)lay.state_bytes;
    const MemeticStateDev st = carve_state(state, pops, K, nullptr);
    hd.gen_min = INT64_MAX;
    for (int i = 0; i < pops; ++i) hd.gen_min = std::min<int64_t>(hd.gen_min, st.gen[i]);
    std::memset(out, 0, kCkptHeaderBytes + align256((size_t)pops * 4));
    std::memcpy(out, &hd, sizeof(hd));
    std::memcpy(out + kCkptHeaderBytes, h->held.ns.data(), (size_t)pops * 4);
    return LABS_OK;
}

extern "C" int labs_memetic_load(labs_handle *h, const void *src, int64_t bytes, void *stream) {
    if (!h) return LABS_E_INVAL;
    h->last_error.clear();
    if (!src) return fail(h, LABS_E_INVAL, "null source");
    if (bytes < (int64_t)kCkptHeaderBytes) return fail(h, LABS_E_INVAL, "not a checkpoint (too short)");
    CkptHeader hd;
    std::memcpy(&hd, src, sizeof(hd));
    if (std::memcmp(hd.magic, kCkptMagic, sizeof(kCkptMagic)) != 0)
        return fail(h, LABS_E_INVAL, "not a checkpoint (magic)");
    if (hd.version != kCkptVersion) return fail(h, LABS_E_INVAL, "checkpoint version %u", hd.version);
    if (hd.pops < 1 || hd.pops > LABS_MAX_REPLICAS || hd.K < 2 || hd.K > LABS_MAX_K)
        return fail(h, LABS_E_INVAL, "checkpoint pops=%d K=%d out of range", hd.pops, hd.K);
    const MemLayout lay = mem_layout(hd.pops, hd.K);
    if (hd.state_bytes != (int64_t)lay.state_bytes || bytes < (int64_t)ckpt_bytes(hd.pops, hd.K))
        return fail(h, LABS_E_INVAL, "checkpoint sizes do not match pops=%d K=%d", hd.pops, hd.K);
    const char *in = (const char *)src;
    std::vector<int32_t> ns((size_t)hd.pops);
    std::memcpy(ns.data(), in + kCkptHeaderBytes, (size_t)hd.pops * 4);
    for (int32_t n : ns)
        if (n < LABS_MIN_N || n > LABS_MAX_N)
            return fail(h, LABS_E_INVAL, "checkpoint length N=%d out of [%d, %d]", n, LABS_MIN_N,
                        LABS_MAX_N);
    DeviceGuard g(h->device);
    hipStream_t s = (hipStream_t)stream;
    h->held.valid = false;  // growing the buffer frees the held replicas
    int rc = mem_acquire(h, s, lay.total());
    if (rc) return rc;
    char *base = (char *)h->mem.ptr;
    const uint32_t flags[2] = {hd.any_hit ? 1u : 0u, 0u};
    hipError_t e = hipMemcpyAsync(base + lay.off_flag, flags, sizeof(flags), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + lay.off_state, in + kCkptHeaderBytes + align256((size_t)hd.pops * 4),
                           lay.state_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // `src` may be reused on return
    if (e == hipSuccess) e = hipEventRecord(h->mem_event, s);
    if (e != hipSuccess) return hip_fail(h, e, "checkpoint load");
    h->mem_event_valid = true;
    h->held.valid = true;
    h->held.pops = hd.pops;
    h->held.K = hd.K;
    h->held.seed = hd.seed;
    h->held.ns = std::move(ns);
    return LABS_OK;
}
