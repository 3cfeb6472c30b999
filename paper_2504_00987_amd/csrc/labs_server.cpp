// Serving loop: continuous batching of memetic solve requests of different N.
//
// A host thread owns a table of resident replica slots on the device.  Each
// iteration it (1) admits waiting requests in FIFO order while enough slots
// are free, initialising their populations, (2) advances every resident
// replica by `chunk` generations in one kernel launch, (3) reads back each
// slot's progress and retires requests whose replicas are all finished,
// freeing their slots.  A replica's trajectory depends only on (request
// seed, replica id, generation), never on its slot or on the other requests,
// so a request's result is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "labs_handle.h"

using namespace liblabs;

namespace {

enum ReqState { kWaiting, kRunning, kDone, kCancelled };

struct Request {
    int64_t id = 0;
    int n = 0;
    uint64_t seed = 0;
    int pops = 0;
    int64_t gens = 0;
    ReqState state = kWaiting;
    std::vector<int> slots;
    std::vector<int8_t> best;
    int32_t best_e = 0;
    std::chrono::steady_clock::time_point t_submit, t_done;
};

double seconds(std::chrono::steady_clock::duration d) {
    return std::chrono::duration<double>(d).count();
}

}  // namespace

struct labs_server {
    labs_handle *h = nullptr;
    labs_memetic_params params{};
    int max_slots = 0;
    hipStream_t stream = nullptr;
    SideStreams sides{};  // further length classes, concurrent with the widest
    // device: [slots table][init table][state]
    void *dmem = nullptr;
    MemeticSlot *d_slots = nullptr;
    MemeticSlot *d_init = nullptr;
    MemeticStateDev st{};
    // pinned host mirrors
    MemeticSlot *h_slots = nullptr;
    MemeticSlot *h_init = nullptr;
    int32_t *h_bestE = nullptr;
    int64_t *h_gen = nullptr;
    int64_t *h_hit = nullptr;
    uint64_t *h_best = nullptr;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<int64_t> waiting;
    std::map<int64_t, Request> reqs;
    std::vector<int64_t> owner;  // slot -> request id or -1
    int64_t next_id = 1;
    int64_t n_done = 0;
    bool stop = false;
    std::string error;
    std::thread worker;

    void loop();
    int iterate(std::unique_lock<std::mutex> &lk);
};

int labs_server::iterate(std::unique_lock<std::mutex> &lk) {
    // (1) admission: FIFO while the head fits in the free slots
    std::vector<int> fresh;
    for (;;) {
        while (!waiting.empty() && reqs[waiting.front()].state == kCancelled) waiting.pop_front();
        if (waiting.empty()) break;
        Request &r = reqs[waiting.front()];
        int free_slots = 0;
        for (int s = 0; s < max_slots; ++s) free_slots += owner[s] < 0;
        if (free_slots < r.pops) break;
        for (int s = 0, k = 0; s < max_slots && k < r.pops; ++s) {
            if (owner[s] >= 0) continue;
            owner[s] = r.id;
            MemeticSlot &d = h_slots[s];
            d.n = r.n;
            d.pop_id = (uint32_t)k;
            d.k0 = (uint32_t)(r.seed & 0xffffffffu);
            d.k1 = (uint32_t)(r.seed >> 32);
            d.gen_limit = r.gens;
            d.target = params.target_e < 0 ? -1 : params.target_e;
            d.state = s;
            r.slots.push_back(s);
            fresh.push_back(s);
            ++k;
        }
        r.state = kRunning;
        waiting.pop_front();
    }
    // free cancelled running requests
    for (auto &kv : reqs) {
        Request &r = kv.second;
        if (r.state == kCancelled && !r.slots.empty()) {
            for (int s : r.slots) {
                owner[s] = -1;
                h_slots[s].state = -1;
            }
            r.slots.clear();
        }
    }
    bool any = false;
    for (int s = 0; s < max_slots; ++s) any |= owner[s] >= 0;
    if (!any) return 0;  // idle
    int classes = 0;
    int64_t n_wide = 0;
    for (int s = 0; s < max_slots; ++s)
        if (owner[s] >= 0) {
            const int c = memetic_class(h_slots[s].n);
            classes |= 1 << c;
            n_wide += c == 1;
        }
    const int n_init = (int)fresh.size();
    for (int i = 0; i < n_init; ++i) h_init[i] = h_slots[fresh[i]];
    lk.unlock();

    // (2) device work
    DeviceGuard g(h->device);
    MemeticLaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.K = params.K;
    a.p_comb = params.p_comb;
    a.mut_rule = params.mut_rule;
    a.p_mut = params.p_mut;
    a.rule = to_rule(params.tabu);
    a.st = st;
    a.any_hit = nullptr;
    hipError_t e = hipSuccess;
    if (n_init > 0) {
        e = hipMemcpyAsync(d_init, h_init, n_init * sizeof(MemeticSlot), hipMemcpyHostToDevice, stream);
        a.slots = d_init;
        a.n_slots = n_init;
        if (e == hipSuccess) e = launch_memetic_init(a, stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_slots, h_slots, max_slots * sizeof(MemeticSlot), hipMemcpyHostToDevice, stream);
    a.slots = d_slots;
    a.n_slots = max_slots;
    a.gens = params.chunk;
    a.classes = classes;
    a.split_wide = split_wide(h, params.waves_per_replica, n_wide);
    a.children = std::max(1, (int)params.children);
    if (e == hipSuccess) e = launch_memetic_advance(a, stream, &sides);
    if (e == hipSuccess) e = hipMemcpyAsync(h_bestE, st.bestE, max_slots * 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h_gen, st.gen, max_slots * 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h_hit, st.hit, max_slots * 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h_best, st.best, max_slots * kStateWords * 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    lk.lock();
    if (e != hipSuccess) {
        error = hipGetErrorString(e);
        return -1;
    }

    // (3) retire finished requests
    const auto now = std::chrono::steady_clock::now();
    for (auto &kv : reqs) {
        Request &r = kv.second;
        if (r.state != kRunning) continue;
        bool finished = true;
        for (int s : r.slots) {
            const bool hit = params.target_e >= 0 && h_hit[s] >= 0;
            finished &= hit || h_gen[s] >= r.gens;
        }
        if (!finished) continue;
        int bs = r.slots[0];
        for (int s : r.slots)
            if (h_bestE[s] < h_bestE[bs] || (h_bestE[s] == h_bestE[bs] && h_slots[s].pop_id < h_slots[bs].pop_id))
                bs = s;
        r.best_e = h_bestE[bs];
        r.best.assign(r.n, 0);
        for (int i = 0; i < r.n; ++i) {
            const uint64_t w = h_best[bs * kStateWords + (i >> 6)];
            r.best[i] = ((w >> (i & 63)) & 1ull) ? -1 : 1;
        }
        for (int s : r.slots) {
            owner[s] = -1;
            h_slots[s].state = -1;
        }
        r.slots.clear();
        r.state = kDone;
        r.t_done = now;
        ++n_done;
    }
    return 1;
}

void labs_server::loop() {
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        const int rc = iterate(lk);
        if (rc < 0) {
            // a device error: fail every pending request
            for (auto &kv : reqs)
                if (kv.second.state == kWaiting || kv.second.state == kRunning) kv.second.state = kCancelled;
            waiting.clear();
            break;
        }
        if (rc == 0) cv.wait_for(lk, std::chrono::milliseconds(2));
    }
}

extern "C" int labs_server_create(labs_handle *h, const labs_memetic_params *params,
                                  int32_t max_slots, labs_server **out) {
    if (!h || !out) return LABS_E_INVAL;
    *out = nullptr;
    h->last_error.clear();
    int rc = check_memetic(h, params);
    if (rc) return rc;
    if (params->resume) return fail(h, LABS_E_INVAL, "the server starts every request afresh (resume=0)");
    if (max_slots < 1 || max_slots > (1 << 20)) return fail(h, LABS_E_INVAL, "max_slots out of [1, 2^20]");
    DeviceGuard g(h->device);
    labs_server *s = new labs_server();
    s->h = h;
    s->params = *params;
    s->max_slots = max_slots;
    s->owner.assign(max_slots, -1);
    size_t state_bytes = 0;
    carve_state(nullptr, max_slots, params->K, &state_bytes);
    const size_t tbl = ((size_t)max_slots * sizeof(MemeticSlot) + 255) & ~(size_t)255;
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->sides.fork, hipEventDisableTiming);
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&s->sides.s[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->sides.join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipMalloc(&s->dmem, 2 * tbl + state_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_slots, tbl, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_init, tbl, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_bestE, (size_t)max_slots * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_gen, (size_t)max_slots * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_hit, (size_t)max_slots * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_best, (size_t)max_slots * kStateWords * 8,
                                             hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        labs_server_destroy(s);
        return fail(h, LABS_E_NOMEM, "server allocation failed: %s", hipGetErrorString(e));
    }
    s->d_slots = (MemeticSlot *)s->dmem;
    s->d_init = (MemeticSlot *)((char *)s->dmem + tbl);
    s->st = carve_state((char *)s->dmem + 2 * tbl, max_slots, params->K, nullptr);
    for (int i = 0; i < max_slots; ++i) {
        std::memset(&s->h_slots[i], 0, sizeof(MemeticSlot));
        s->h_slots[i].state = -1;
    }
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return LABS_OK;
}

extern "C" int labs_server_submit(labs_server *s, int32_t n, uint64_t seed, int32_t pops,
                                  int64_t generations, int64_t *request_id) {
    if (!s || !request_id) return LABS_E_INVAL;
    if (n < LABS_MIN_N || n > LABS_MAX_N || pops < 1 || pops > s->max_slots || generations < 0 ||
        generations > 0xffffffffLL)
        return LABS_E_INVAL;
    {
        // the tabu rule must be valid at this length
        labs_handle tmp;
        tmp.max_children_wide = s->h->max_children_wide;
        if (check_rule(&tmp, to_rule(s->params.tabu), n) ||
            check_children(&tmp, std::max(1, (int)s->params.children), 1 << memetic_class(n)))
            return LABS_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return LABS_E_CANCELLED;
    Request r;
    r.id = s->next_id++;
    r.n = n;
    r.seed = seed;
    r.pops = pops;
    r.gens = generations;
    r.t_submit = std::chrono::steady_clock::now();
    s->reqs[r.id] = r;
    s->waiting.push_back(r.id);
    *request_id = r.id;
    s->cv.notify_all();
    return LABS_OK;
}

extern "C" int labs_server_poll(labs_server *s, int64_t request_id, int8_t *best_seq,
                                int32_t *best_e, double *latency_s) {
    if (!s) return LABS_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return LABS_E_NOTFOUND;
    Request &r = it->second;
    if (r.state == kCancelled) {
        if (r.slots.empty()) s->reqs.erase(it);
        return LABS_E_CANCELLED;
    }
    if (r.state != kDone) return LABS_E_AGAIN;
    if (best_seq) std::memcpy(best_seq, r.best.data(), r.best.size());
    if (best_e) *best_e = r.best_e;
    if (latency_s) *latency_s = seconds(r.t_done - r.t_submit);
    s->reqs.erase(it);
    return LABS_OK;
}

extern "C" int labs_server_cancel(labs_server *s, int64_t request_id) {
    if (!s) return LABS_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return LABS_E_NOTFOUND;
    if (it->second.state == kWaiting || it->second.state == kRunning) it->second.state = kCancelled;
    s->cv.notify_all();
    return LABS_OK;
}

extern "C" int labs_server_stats(labs_server *s, int64_t *waiting, int64_t *running,
                                 int64_t *done, int64_t *resident) {
    if (!s) return LABS_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t w = 0, r = 0, res = 0;
    for (auto &kv : s->reqs) {
        w += kv.second.state == kWaiting;
        r += kv.second.state == kRunning;
    }
    for (int64_t o : s->owner) res += o >= 0;
    if (waiting) *waiting = w;
    if (running) *running = r;
    if (done) *done = s->n_done;
    if (resident) *resident = res;
    return s->error.empty() ? LABS_OK : LABS_E_HIP;
}

extern "C" int labs_server_destroy(labs_server *s) {
    if (!s) return LABS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    DeviceGuard g(s->h->device);
    if (s->stream) hipStreamSynchronize(s->stream);
    if (s->dmem) hipFree(s->dmem);
    if (s->h_slots) hipHostFree(s->h_slots);
    if (s->h_init) hipHostFree(s->h_init);
    if (s->h_bestE) hipHostFree(s->h_bestE);
    if (s->h_gen) hipHostFree(s->h_gen);
    if (s->h_hit) hipHostFree(s->h_hit);
    if (s->h_best) hipHostFree(s->h_best);
    if (s->sides.fork) hipEventDestroy(s->sides.fork);
    for (int i = 0; i < kSideStreams; ++i) {
        if (s->sides.join[i]) hipEventDestroy(s->sides.join[i]);
        if (s->sides.s[i]) hipStreamDestroy(s->sides.s[i]);
    }
    if (s->stream) hipStreamDestroy(s->stream);
    delete s;
    return LABS_OK;
}
