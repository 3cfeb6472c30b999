// Internal interface between the C ABI (labs_api.cpp, labs_memetic.cpp,
// labs_server.cpp) and the kernels (labs_walk.hip, labs_memetic_kernels.hip,
// labs_brute.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/liblabs.h"

namespace liblabs {

struct RuleParams {
    int32_t steps_rule, steps_a, tenure_rule;
    int32_t lo_num, lo_den, lo_add, hi_num, hi_den, hi_add;
    int32_t aspiration;
    int32_t slo_num, slo_den, shi_num, shi_den;  // LABS_STEPS_RANGE bounds
};

// Length classes of stand-alone walks, longest first: a class fixes the
// neighbours per lane (NW) and how many 16-lag chunks a window spans (NB).
// The last two (N <= 32, N <= 16) are also the walks that fit a 32- or
// 16-lane group of a wavefront that runs several walks.
constexpr int kWalkClasses = 8;
constexpr int kClassMaxN[kWalkClasses] = {256, 193, 128, 97, 64, 49, 32, 16};
inline int walk_class(int n) {
    int c = 0;
    while (c + 1 < kWalkClasses && n <= kClassMaxN[c + 1]) ++c;
    return c;
}

struct TabuLaunchArgs {
    const int8_t *starts;     // [W][start_stride] or null
    int32_t start_stride;
    const int32_t *ns;        // device [W] or null
    int32_t n_uniform;
    int32_t n_max;            // longest walk in the batch
    const int32_t *order;     // device [W] walk ids in processing order, or null
    int64_t W;
    int64_t class_end[kWalkClasses];  // processing-order positions [class_end[c-1],
                                      // class_end[c]) hold the walks of class c
    uint32_t k0, k1;
    RuleParams rule;
    int8_t *best_seq;
    int32_t out_stride;
    int32_t *best_e;
    int32_t *final_e;
    int16_t *trace;
    int32_t trace_stride;
    uint32_t *counter;        // device, 32 words per class: persistent queue heads
};

// Streams besides the caller's one that a batch may fork onto.
constexpr int kSideStreams = kWalkClasses - 1;

// Kernel forms of a launch group.
enum WalkKind : int {
    kKindWave = 0,    // one walk per wavefront
    kKindSplit = 1,   // one walk of 64 < N <= 128 per two wavefronts
    kKindGroup2 = 2,  // two walks of N <= 32 per wavefront (32 lanes each)
    kKindGroup4 = 4,  // four walks of N <= 16 per wavefront (16 lanes each)
};

// Launch groups of a batch: runs of consecutive length classes (hence of
// consecutive positions of the processing order) that one kernel launch
// covers, each on a stream of its own.  Both classes of N > 128, when
// present, share one launch (the four-neighbour layout serves both); so do
// the classes of N <= 128 when more than one is present -- or, with
// two-wavefront walks (split), classes 2..3 (64 < N <= 128) form one group
// and the shorter classes another.  With several walks per wavefront
// (`lanes` = 32 or 16 lanes per walk) the walks of N <= 32 leave the
// one-walk-per-wavefront group: with 32 lanes both short classes form one
// group of two walks per wavefront; with 16, N <= 16 runs four per
// wavefront and 16 < N <= 32 two.
struct WalkGroups {
    int n;
    int first[kWalkClasses], last[kWalkClasses], kind[kWalkClasses];
};
inline WalkGroups walk_launch_groups(const int64_t *class_end, bool split, int lanes = 64) {
    WalkGroups g;
    g.n = 0;
    auto present = [&](int c) { return class_end[c] > (c ? class_end[c - 1] : 0); };
    auto add = [&](int f, int z, int kind) {
        g.first[g.n] = f;
        g.last[g.n] = z;
        g.kind[g.n] = kind;
        ++g.n;
    };
    auto range = [&](int lo, int hi, int kind) {
        int f = -1, z = -1;
        for (int c = lo; c <= hi; ++c)
            if (present(c)) {
                if (f < 0) f = c;
                z = c;
            }
        if (f >= 0) add(f, z, kind);
    };
    const int short_end = lanes < 64 ? 5 : kWalkClasses - 1;
    range(0, 1, kKindWave);
    if (split) {
        if (present(2) || present(3)) add(2, 3, kKindSplit);  // the two-wavefront kernel takes both
        range(4, short_end, kKindWave);
    } else {
        range(2, short_end, kKindWave);
    }
    if (lanes == 32) {
        range(6, 7, kKindGroup2);
    } else if (lanes == 16) {
        range(6, 6, kKindGroup2);
        range(7, 7, kKindGroup4);
    }
    return g;
}

// How labs_tabu_batch launches its walks.
struct WalkLaunch {
    int waves_per_group;  // wavefronts per workgroup (one-wavefront walks: that many per group)
    bool split;           // walks of 64 < N <= 128 on two wavefronts each
    bool lag;             // walks of 64 < N <= 128 in the lag form
    int lanes;            // lanes per walk of N <= 32: 64 (one walk per wavefront), 32 or 16
    int groups;           // persistent grid of the one-wavefront and group kernels (0: none)
    int split_groups;     // persistent grid of the two-wavefront kernel (0: none)
};

// Words of a sequence mask in the memetic state (N <= 256).
constexpr int kStateWords = 4;

// Device layout of a memetic replica's state (structure of arrays).
struct MemeticStateDev {
    uint64_t *pop;    // [S][K][kStateWords] member masks (bit i: s_i = -1)
    int32_t *popE;    // [S][K]
    uint64_t *best;   // [S][kStateWords]
    int32_t *bestE;   // [S]
    int64_t *gen;     // [S] generations done
    int64_t *hit;     // [S] hit generation or -1
};

struct MemeticSlot {
    int32_t n;
    uint32_t pop_id;
    uint32_t k0, k1;
    int64_t gen_limit;
    int32_t target;
    int32_t state;    // index into MemeticStateDev arrays; < 0 means idle
};

constexpr int kMaxChildren = 8;  // children per generation (batched variant)

// Length classes of memetic replicas: mask words 1, 2 or 4.
__host__ __device__ inline int memetic_class(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : 2; }

// Side streams a launch may fork onto (fork recorded on the caller's stream,
// side i joined back through join[i]).
struct SideStreams {
    hipStream_t s[kSideStreams];
    hipEvent_t join[kSideStreams];
    hipEvent_t fork;
};

struct MemeticLaunchArgs {
    const MemeticSlot *slots;
    int32_t n_slots;
    int32_t K;
    uint32_t p_comb;
    int32_t mut_rule;
    uint32_t p_mut;
    RuleParams rule;
    int32_t gens;            // generations per launch
    int32_t classes;         // bit c set: some slot is of memetic_class c
    int32_t split_wide;      // 1: a replica with N > 64 runs on two wavefronts
    int32_t children;        // children per generation (1: Alg. 1)
    MemeticStateDev st;
    uint32_t *any_hit;       // set to 1 when a replica reaches its target
    const uint32_t *stop;    // nonzero: the launch does nothing (null: never)
};

// Fixed device scratch of the allocation-free tabu batch: queue heads, then
// per-walk lengths and the processing order for at most kNoAllocMaxWalks
// walks of per-walk lengths (a batch of one length needs the heads only).
constexpr int64_t kNoAllocMaxWalks = LABS_NOALLOC_MAX_WALKS;
constexpr size_t kNoAllocHeadBytes = 1024;
constexpr size_t kNoAllocScratchBytes =
    kNoAllocHeadBytes + 2 * (size_t)kNoAllocMaxWalks * sizeof(int32_t);
static_assert(kNoAllocScratchBytes == LABS_NOALLOC_SCRATCH_BYTES, "scratch size as declared");
constexpr int kMaxDevices = 64;
// Device address of that scratch on `device`, which the caller has made
// current; looked up once per device (hipGetSymbolAddress) and kept.
hipError_t noalloc_scratch_address(int device, void **ptr);
// Longest-first processing order of W walks from their device lengths.
hipError_t launch_order_by_length(const int32_t *ns, int64_t W, int32_t *order, hipStream_t s);

hipError_t launch_energy(const int8_t *seqs, const int32_t *ns, int32_t n_uniform,
                         int32_t stride, int64_t count, int32_t *out, hipStream_t s);

// Exhaustive minimum over the 2^(n-1) codes with s_0 = +1.  `waves`
// wavefronts each write (min E, count, smallest code attaining it) to
// part_e/part_count/part_code; a second kernel reduces them into out_e,
// out_count (over all 2^n sequences) and out_code.
struct BruteParts {
    int32_t *part_e;
    int64_t *part_count;
    uint64_t *part_code;
    int32_t *out_e;
    int64_t *out_count;
    uint64_t *out_code;
};
int64_t brute_waves(int n);
hipError_t launch_bruteforce(int n, const BruteParts &p, hipStream_t s);
// The same over the skew-symmetric sequences of odd length n (Sec. II.C):
// out_code receives the free-spin pattern (bit i set <=> s_i = -1, i <= c).
int64_t skew_brute_waves(int n);
hipError_t launch_skew_bruteforce(int n, const BruteParts &p, hipStream_t s);

// Launch group g (walk_launch_groups(a.class_end, l.split, l.lanes)) runs on
// streams[g]; a.counter must point at 32 * kWalkClasses writable uint32 (the
// queue head of a group at 32 * its first class).
hipError_t launch_tabu(const TabuLaunchArgs &a, const WalkLaunch &l, const hipStream_t *streams);

hipError_t launch_memetic_init(const MemeticLaunchArgs &a, hipStream_t s);
// At a chunk boundary: *stop becomes (and stays) 1 when stop_all is set and
// *any_hit is, or when *cancel (host memory mapped for the device) no
// longer holds `epoch`.  One thread; capturable.
hipError_t launch_memetic_latch(const uint32_t *any_hit, uint32_t *stop,
                                const volatile uint32_t *cancel, uint32_t epoch, int stop_all,
                                hipStream_t s);
// Once per device before the first launch: raises the dynamic LDS limit of
// the batched-generation kernels to what kMaxChildren children need (N > 128:
// as far as the device allows).  Returns the most children per generation
// the N > 128 kernel can take, or -1 on failure.
int prepare_memetic_kernels();
// Advances every slot by a.gens generations.  With several length classes
// present and `sides` given, the widest class runs on s and the others on
// side streams forked from and joined back into s, concurrently; the
// sequence of calls is capturable into a graph.
hipError_t launch_memetic_advance(const MemeticLaunchArgs &a, hipStream_t s,
                                  const SideStreams *sides = nullptr);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s);
hipError_t launch_skew_deviation(const int8_t *seqs, const int32_t *ns, int32_t n_uniform,
                                 int32_t stride, int64_t count, int32_t *out, hipStream_t s);
hipError_t launch_gather_best(const MemeticStateDev &st, const int32_t *state_idx,
                              const int32_t *ns, int32_t n_uniform, int32_t count,
                              int8_t *best_seq, int32_t out_stride, int32_t *best_e,
                              int64_t *hit_gen, int64_t *gens_done, hipStream_t s);

}  // namespace liblabs
