// Host-side state of a liblabs handle and helpers shared by the C ABI
// translation units.  Internal; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/liblabs.h"
#include "labs_internal.h"

namespace liblabs {

struct DevBuf {
    void *ptr = nullptr;
    size_t size = 0;
    int reserve(labs_handle *h, size_t bytes);
    void release();
};

struct PinBuf {
    void *ptr = nullptr;
    size_t size = 0;
    int reserve(labs_handle *h, size_t bytes);
    void release();
};

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
  private:
    int prev_ = -1;
};

}  // namespace liblabs

struct labs_handle {
    int device = 0;
    int num_cus = 0;
    std::string arch;
    std::string last_error;
    hipStream_t stream = nullptr;      // internal stream (default priority)
    liblabs::SideStreams sides{};      // further length classes of a mixed batch
    hipEvent_t ws_event = nullptr;     // completion of the last device-workspace user
    hipEvent_t stage_event = nullptr;  // completion of the last copy out of `pin`
    int max_children_wide = 0;         // batched children per generation at N > 128
    void *scratch = nullptr;           // this device's allocation-free scratch
    bool ws_event_valid = false;
    bool stage_event_valid = false;
    liblabs::DevBuf ws;                   // tabu workspace: queue head, ns, order
    liblabs::DevBuf mem;                  // memetic state and slot table
    liblabs::PinBuf pin;                  // pinned staging
    // Memetic runs are stream-ordered: the next user of `mem` waits for
    // mem_event; graphs of earlier runs are destroyed once their last
    // launch has completed.
    hipEvent_t mem_event = nullptr;
    bool mem_event_valid = false;
    struct Retired {
        hipGraphExec_t exec;
        hipGraph_t graph;
        hipEvent_t done;
    };
    std::vector<Retired> retired;
    // labs_cancel: word 0 of `cancel_host` (pinned, mapped for the device)
    // holds the cancel epoch; a run keeps the epoch it started under and
    // stops at its next chunk boundary once the word differs.  Words 1..4:
    // stop-flag snapshots copied back for the host's polling.
    uint32_t *cancel_host = nullptr;
    uint32_t *cancel_dev = nullptr;
    std::atomic<uint32_t> cancel_epoch{0};
    hipEvent_t poll_event[4] = {};
    // The memetic replicas held in `mem` (after a run or a load): what a
    // resumed run or a checkpoint must match.
    struct MemState {
        bool valid = false;
        int32_t pops = 0, K = 0;
        uint64_t seed = 0;
        std::vector<int32_t> ns;
    } held;
    bool has_override = false;
    labs_launch override_launch{64, 1, 0, 0, 0};
    // tuned launches by (length bucket of n_min, of n_max), buckets of 16
    std::map<std::pair<int, int>, labs_launch> tuned;
};

namespace liblabs {

int fail(labs_handle *h, int code, const char *fmt, ...);
int hip_fail(labs_handle *h, hipError_t e, const char *where);
// Device workspace `ws` of at least `bytes`, its reuse ordered after the
// previous user on the GPU (the host waits only when it must grow).
int ws_acquire(labs_handle *h, hipStream_t s, size_t bytes);
int ws_release(labs_handle *h, hipStream_t s);
// Pinned staging `pin` of at least `bytes`, once the previous copy out of it
// has completed; stage_release marks a copy out of it on stream s.
int stage_acquire(labs_handle *h, size_t bytes);
int stage_release(labs_handle *h, hipStream_t s);
int check_rule(labs_handle *h, const RuleParams &r, int n);
long long max_steps(const RuleParams &r, int n);
RuleParams to_rule(const labs_tabu_params &p);
labs_launch choose_launch(labs_handle *h, int n_min, int n_max);
// The kernels' view of a launch configuration.
WalkLaunch walk_launch(const labs_handle *h, const labs_launch &l);
int tabu_batch_impl(labs_handle *h, const labs_tabu_params *p, const int8_t *starts,
                    int32_t start_stride, const int32_t *ns_host, int32_t n_uniform, int64_t W,
                    uint64_t seed, int8_t *best_seq, int32_t out_stride, int32_t *best_e,
                    int32_t *final_e, int16_t *trace, int32_t trace_stride, hipStream_t s,
                    const labs_launch *force, void *scratch = nullptr);
int check_memetic(labs_handle *h, const labs_memetic_params *p);
// Children per generation against what the device fits (classes: bit c set
// when a replica of memetic_class c is present).
int check_children(labs_handle *h, int children, int classes);
// 1 when replicas with 64 < N <= 128 should run on two wavefronts each.
int split_wide(const labs_handle *h, int waves_per_replica, int64_t n_wide);

// Bytes of device state per memetic replica with population size K.
inline size_t memetic_state_bytes(int K) {
    return (size_t)K * (kStateWords * sizeof(uint64_t) + sizeof(int32_t)) +
           kStateWords * sizeof(uint64_t) + sizeof(int32_t) + 2 * sizeof(int64_t);
}

// Carve a MemeticStateDev for S replicas out of `base` (256-byte aligned parts).
MemeticStateDev carve_state(void *base, int S, int K, size_t *bytes_out);

}  // namespace liblabs
