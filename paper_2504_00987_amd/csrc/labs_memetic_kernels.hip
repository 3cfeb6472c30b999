// Memetic kernels of liblabs for gfx950 and their launchers.
//
//   memetic_init_kernel    random populations (Alg. 1, first two lines)
//   memetic_advance_kernel memetic generations (Alg. 1 / Alg. 3), one replica
//                          per workgroup of one or two wavefronts, population
//                          resident in LDS
//   memetic_batched_kernel B children per generation, one wavefront each,
//                          from one snapshot of the population
//   gather_best_kernel     best sequences and energies to caller buffers
#include <algorithm>

#include "labs_device.hpp"
#include "labs_internal.h"

namespace liblabs {

namespace {

constexpr int kMaxK = 128;

// Walk form of the one-child kernels: the lag form for N <= 64, and for
// 64 < N <= 128 when two wavefronts run a replica (few replicas per CU).
template <int NW, int SPLIT>
constexpr bool kAdvanceLag = NW == 1 || (NW == 2 && SPLIT == 2);


// ---------------------------------------------------------------------------
// Memetic replicas.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t word_of(const Draw4 &d, int i) {
    return i == 0 ? d.w0 : (i == 1 ? d.w1 : (i == 2 ? d.w2 : d.w3));
}

// Member m = lane + 64 h of the replica (K <= 128): bits 128 q .. 128 q + 127
// are the draw (pop, m, q, INIT); its energy is computed lane-serially.
template <typename Mask>
__device__ __forceinline__ int init_member(const MemeticLaunchArgs &a, const MemeticSlot &sl,
                                           int m, uint64_t wd[kStateWords]) {
    const int N = sl.n;
#pragma unroll
    for (int q = 0; q < kStateWords / 2; ++q) {
        const Draw4 d = philox10(sl.pop_id, (uint32_t)m, (uint32_t)q, kTagInit, sl.k0, sl.k1);
        wd[2 * q] = (uint64_t)d.w0 | ((uint64_t)d.w1 << 32);
        wd[2 * q + 1] = (uint64_t)d.w2 | ((uint64_t)d.w3 << 32);
    }
#pragma unroll
    for (int h = 0; h < kStateWords; ++h) {
        const int b = N - 64 * h;  // bits of word h inside the sequence
        wd[h] &= b >= 64 ? ~0ull : b <= 0 ? 0ull : ((1ull << b) - 1ull);
    }
    return lane_energy<Mask>(make_mask<sizeof(Mask) / 8>(wd[0], wd[1], wd[2], wd[3]), N);
}

__global__ __launch_bounds__(64) void memetic_init_kernel(MemeticLaunchArgs a) {
    const int s = blockIdx.x;
    if (s >= a.n_slots) return;
    const MemeticSlot sl = a.slots[s];
    if (sl.state < 0) return;
    const int lane = lane_id();
    const int N = sl.n, K = a.K;
    const int64_t base = (int64_t)sl.state * K;
    uint64_t wd[2][kStateWords] = {};
    int e[2] = {INT_MAX, INT_MAX};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int m = lane + 64 * h;
        if (m < K) {
            const int c = memetic_class(N);
            e[h] = c == 0 ? init_member<uint64_t>(a, sl, m, wd[h])
                 : c == 1 ? init_member<M128>(a, sl, m, wd[h])
                          : init_member<M256>(a, sl, m, wd[h]);
#pragma unroll
            for (int w = 0; w < kStateWords; ++w)
                a.st.pop[(base + m) * kStateWords + w] = wd[h][w];
            a.st.popE[base + m] = e[h];
        }
    }
    // bestSeq: the lowest-index member of minimum energy.
    const int mn = wave_min(min(e[0], e[1]));
    const uint64_t t0 = ballot(e[0] == mn), t1 = ballot(e[1] == mn);
    const int h = t0 ? 0 : 1;
    const int src = t0 ? __builtin_ctzll(t0) : __builtin_ctzll(t1);
#pragma unroll
    for (int w = 0; w < kStateWords; ++w) {
        const uint64_t sel = h == 0 ? wd[0][w] : wd[1][w];
        const uint64_t v = ((uint64_t)readlane_u((uint32_t)(sel >> 32), src) << 32) |
                           readlane_u((uint32_t)sel, src);
        a.st.best[(int64_t)sl.state * kStateWords + w] = v;  // uniform values, every lane
    }
    a.st.bestE[sl.state] = mn;
    a.st.gen[sl.state] = 0;
    a.st.hit[sl.state] = -1;
}

// Mutation mask of a child: bit i flips when word i%4 of draw
// (pop, g, base + i/4, MUT) is below thr.
template <int NW>
__device__ __forceinline__ typename MaskOf<NW>::type mutation_mask(const MemeticSlot &sl,
                                                                   uint32_t gg, uint32_t base,
                                                                   uint32_t thr) {
    const int lane = lane_id();
    uint64_t f[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
    for (int h = 0; h < NW; ++h) {
        const int i = lane + 64 * h;
        const Draw4 d = philox10(sl.pop_id, gg, base + (uint32_t)(i >> 2), kTagMut, sl.k0, sl.k1);
        f[h] = ballot(i < sl.n && word_of(d, i & 3) < thr);
    }
    return make_mask<NW>(f[0], f[1], f[2], f[3]);
}

// One replica on SPLIT wavefronts (wavefront `part` of them); every
// wavefront runs the generation logic redundantly on wave-uniform values and
// the walk is split between them.
template <int NW, int SPLIT>
__device__ void memetic_replica(const MemeticLaunchArgs &a, const MemeticSlot &sl,
                                uint64_t (*pop)[NW], int *popE, uint8_t *lds, int part) {
    using Mask = typename MaskOf<NW>::type;
    const int lane = lane_id();
    const int N = sl.n, K = a.K, st = sl.state;
    const int64_t base = (int64_t)st * K;
    for (int i = lane + 64 * part; i < K; i += 64 * SPLIT) {
#pragma unroll
        for (int w = 0; w < NW; ++w) pop[i][w] = a.st.pop[(base + i) * kStateWords + w];
        popE[i] = a.st.popE[base + i];
    }
    walk_sync<SPLIT>();
    Mask best = load_mask<NW>(a.st.best + (int64_t)st * kStateWords);
    int bestE = a.st.bestE[st];
    int64_t g = a.st.gen[st];
    int64_t hit = a.st.hit[st];
    const uint32_t thr = a.mut_rule == 0 ? (uint32_t)(0x100000000ull / (uint64_t)N) : a.p_mut;
    const bool targeted = sl.target >= 0;

    for (int it = 0; it < a.gens; ++it) {
        if (g >= sl.gen_limit) break;
        if (targeted && bestE <= sl.target) {
            if (hit < 0) hit = g;
            break;
        }
        const uint32_t gg = (uint32_t)g;
        const Draw4 da = philox10(sl.pop_id, gg, 0u, kTagGen, sl.k0, sl.k1);
        const Draw4 db = philox10(sl.pop_id, gg, 1u, kTagGen, sl.k0, sl.k1);
        Mask child;
        if (da.w0 < a.p_comb) {
            // selectParents: two binary tournaments; Combine: one-point crossover
            int i = (int)below(da.w1, (uint32_t)K), j = (int)below(da.w2, (uint32_t)K);
            const int pa = popE[i] <= popE[j] ? i : j;
            i = (int)below(da.w3, (uint32_t)K);
            j = (int)below(db.w0, (uint32_t)K);
            const int pb = popE[i] <= popE[j] ? i : j;
            const int cut = 1 + (int)below(db.w1, (uint32_t)(N - 1));
            const Mask A = load_mask<NW>(pop[pa]);
            const Mask B = load_mask<NW>(pop[pb]);
            const Mask lowm = m_low(A, cut);
            child = m_or(m_and(A, lowm), m_and(B, m_not(lowm)));
        } else {
            const int c = (int)below(da.w1, (uint32_t)K);
            child = load_mask<NW>(pop[c]);
        }
        // Mutate: bit i flips when word i%4 of draw (pop, g, i/4, MUT) < thr.
        child = m_xor(child, mutation_mask<NW>(sl, gg, 0u, thr));
        const Schedule sch = make_schedule(a.rule, N, sl.k0, sl.k1, sl.pop_id, gg);
        const WalkResult<NW> r = tabu_walk<NW, false, SPLIT, WalkLds<NW>::NBIG, kAdvanceLag<NW, SPLIT>>(
            N, child, sch, a.rule.aspiration, sl.k0, sl.k1, sl.pop_id, gg, lds, nullptr, part);
        if (r.best_e < bestE) {
            bestE = r.best_e;
            best = r.best;
        }
        const int rep = (int)below(db.w2, (uint32_t)K);
        walk_sync<SPLIT>();
        store_mask<NW>(pop[rep], r.best);  // uniform values, every lane
        popE[rep] = r.best_e;
        walk_sync<SPLIT>();
        ++g;
        if (targeted && bestE <= sl.target) {
            if (hit < 0) hit = g;
            break;
        }
    }

    for (int i = lane + 64 * part; i < K; i += 64 * SPLIT) {
#pragma unroll
        for (int w = 0; w < NW; ++w) a.st.pop[(base + i) * kStateWords + w] = pop[i][w];
        a.st.popE[base + i] = popE[i];
    }
    if (part != 0) return;
    store_mask<NW>(a.st.best + (int64_t)st * kStateWords, best);  // uniform values, every lane
    a.st.bestE[st] = bestE;
    a.st.gen[st] = g;
    a.st.hit[st] = hit;
    if (hit >= 0 && a.any_hit != nullptr) atomicOr(a.any_hit, 1u);
}

// Replicas of one length class: N <= 64 (NW = 1), 64 < N <= 128 (NW = 2) or
// 128 < N <= 256 (NW = 4), one workgroup of SPLIT wavefronts per replica;
// slots of the other classes and idle slots return at once.  The
// two-wavefront form only runs when there are at most two replicas per
// compute unit, so it is compiled for latency (all of a step's LDS reads in
// flight at once) rather than for occupancy, and its walks take the lag form
// (18 KB of LDS, which costs nothing at that occupancy).
template <int NW, int SPLIT>
__global__ __launch_bounds__(64 * SPLIT)
__attribute__((amdgpu_waves_per_eu(1, SPLIT == 2 ? 2 : 8))) void memetic_advance_kernel(
    MemeticLaunchArgs a) {
    __shared__ uint64_t pop[kMaxK][NW];
    __shared__ int popE[kMaxK];
    __shared__ __attribute__((aligned(16))) uint8_t lds[walk_lds_bytes<NW, kAdvanceLag<NW, SPLIT>>()];
    const int s = blockIdx.x;
    if (s >= a.n_slots) return;
    if (a.stop != nullptr && *a.stop != 0u) return;  // one value for the whole grid
    const MemeticSlot sl = a.slots[s];
    if (sl.state < 0 || (1 << memetic_class(sl.n)) != NW) return;
    memetic_replica<NW, SPLIT>(a, sl, pop, popE, lds, SPLIT == 1 ? 0 : (int)(threadIdx.x >> 6));
}

// Batched-generation variant: one workgroup of B = a.children wavefronts per
// replica.  Wavefront b makes child b of generation g from the population as
// it stands at the start of g (LDS, read-only while the children walk) and
// walks it in its own LDS scratch; after a barrier every wavefront merges the
// B results in order b = 0..B-1 into its copy of best, and wavefront 0
// alone writes the replacements (so they land in order); a second barrier
// publishes them.  All control flow depends only on values every wavefront
// holds identically, so every wavefront reaches every barrier.
// Dynamic LDS: population [kMaxK][NW] words, energies [kMaxK], per child
// kResWords words (mask, energy, replaced slot), then the B walk scratches.
// Children walk in the lag form up to N = 128: a replica's workgroup of B
// wavefronts occupies its CU whatever the LDS per walk.
constexpr int kResWords = 8;
template <int NW>
constexpr bool kBatchedLag = NW <= 2;
template <int NW>
constexpr int batched_header() {
    return kMaxK * 8 * NW + kMaxK * 4 + kMaxChildren * kResWords * 8;
}

template <int NW>
__global__ __launch_bounds__(64 * kMaxChildren) void memetic_batched_kernel(
    MemeticLaunchArgs a) {
    using Mask = typename MaskOf<NW>::type;
    extern __shared__ __attribute__((aligned(16))) uint8_t dyn_lds[];
    uint64_t(*pop)[NW] = (uint64_t(*)[NW])dyn_lds;
    int *popE = (int *)(dyn_lds + kMaxK * 8 * NW);
    uint64_t *res = (uint64_t *)(dyn_lds + kMaxK * (8 * NW + 4));  // [B][kResWords]
    const int s = blockIdx.x;
    if (s >= a.n_slots) return;
    if (a.stop != nullptr && *a.stop != 0u) return;  // one value for the whole grid
    const MemeticSlot sl = a.slots[s];
    if (sl.state < 0 || (1 << memetic_class(sl.n)) != NW) return;
    const int B = a.children;
    const int b = (int)(threadIdx.x >> 6);
    uint8_t *lds = dyn_lds + batched_header<NW>() + b * walk_lds_bytes<NW, kBatchedLag<NW>>();
    const int N = sl.n, K = a.K, st = sl.state;
    const int64_t base = (int64_t)st * K;
    for (int i = (int)threadIdx.x; i < K; i += 64 * B) {
#pragma unroll
        for (int w = 0; w < NW; ++w) pop[i][w] = a.st.pop[(base + i) * kStateWords + w];
        popE[i] = a.st.popE[base + i];
    }
    __syncthreads();
    Mask best = load_mask<NW>(a.st.best + (int64_t)st * kStateWords);
    int bestE = a.st.bestE[st];
    int64_t g = a.st.gen[st];
    int64_t hit = a.st.hit[st];
    const uint32_t thr = a.mut_rule == 0 ? (uint32_t)(0x100000000ull / (uint64_t)N) : a.p_mut;
    const bool targeted = sl.target >= 0;

    for (int it = 0; it < a.gens; ++it) {
        if (g >= sl.gen_limit) break;
        if (targeted && bestE <= sl.target) {
            if (hit < 0) hit = g;
            break;
        }
        const uint32_t gg = (uint32_t)g;
        const Draw4 da = philox10(sl.pop_id, gg, (uint32_t)(2 * b), kTagGen, sl.k0, sl.k1);
        const Draw4 db = philox10(sl.pop_id, gg, (uint32_t)(2 * b + 1), kTagGen, sl.k0, sl.k1);
        Mask child;
        if (da.w0 < a.p_comb) {
            int i = (int)below(da.w1, (uint32_t)K), j = (int)below(da.w2, (uint32_t)K);
            const int pa = popE[i] <= popE[j] ? i : j;
            i = (int)below(da.w3, (uint32_t)K);
            j = (int)below(db.w0, (uint32_t)K);
            const int pb = popE[i] <= popE[j] ? i : j;
            const int cut = 1 + (int)below(db.w1, (uint32_t)(N - 1));
            const Mask A = load_mask<NW>(pop[pa]);
            const Mask Bm = load_mask<NW>(pop[pb]);
            const Mask lowm = m_low(A, cut);
            child = m_or(m_and(A, lowm), m_and(Bm, m_not(lowm)));
        } else {
            const int c = (int)below(da.w1, (uint32_t)K);
            child = load_mask<NW>(pop[c]);
        }
        // child b's mutation words: (pop, g, 64 b + i/4, MUT)
        child = m_xor(child, mutation_mask<NW>(sl, gg, (uint32_t)(64 * b), thr));
        const uint32_t wgen = (uint32_t)(g * B + b);
        const Schedule sch = make_schedule(a.rule, N, sl.k0, sl.k1, sl.pop_id, wgen);
        const WalkResult<NW> r = tabu_walk<NW, false, 1, WalkLds<NW>::NBIG, kBatchedLag<NW>>(
            N, child, sch, a.rule.aspiration, sl.k0, sl.k1, sl.pop_id, wgen, lds, nullptr);
        uint64_t *mine = res + kResWords * b;
        store_mask<NW>(mine, r.best);  // uniform values, every lane of wavefront b
        mine[4] = (uint64_t)(uint32_t)r.best_e;
        mine[5] = (uint64_t)below(db.w2, (uint32_t)K);
        __syncthreads();
        for (int c = 0; c < B; ++c) {
            const uint64_t *rc = res + kResWords * c;
            uint64_t wd[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
            for (int w = 0; w < NW; ++w) wd[w] = uniform64(rc[w]);
            const int e = __builtin_amdgcn_readfirstlane((int)(uint32_t)rc[4]);
            const int slot = __builtin_amdgcn_readfirstlane((int)(uint32_t)rc[5]);
            const Mask m = make_mask<NW>(wd[0], wd[1], wd[2], wd[3]);
            if (e < bestE) {
                bestE = e;
                best = m;
            }
            if (b == 0) {
                store_mask<NW>(pop[slot], m);  // uniform values, every lane of wavefront 0
                popE[slot] = e;
            }
        }
        __syncthreads();
        ++g;
        if (targeted && bestE <= sl.target) {
            if (hit < 0) hit = g;
            break;
        }
    }

    for (int i = (int)threadIdx.x; i < K; i += 64 * B) {
#pragma unroll
        for (int w = 0; w < NW; ++w) a.st.pop[(base + i) * kStateWords + w] = pop[i][w];
        a.st.popE[base + i] = popE[i];
    }
    if (b != 0) return;
    store_mask<NW>(a.st.best + (int64_t)st * kStateWords, best);  // uniform values, every lane
    a.st.bestE[st] = bestE;
    a.st.gen[st] = g;
    a.st.hit[st] = hit;
    if (hit >= 0 && a.any_hit != nullptr) atomicOr(a.any_hit, 1u);
}

// The stop latch of a chunk boundary (see launch_memetic_latch).
__global__ void memetic_latch_kernel(const uint32_t *any_hit, uint32_t *stop,
                                     const volatile uint32_t *cancel, uint32_t epoch,
                                     int stop_all) {
    const bool hit = stop_all != 0 && *any_hit != 0u;
    const bool cancelled = cancel != nullptr && *cancel != epoch;
    if (hit || cancelled) *stop = 1u;
}

__global__ void gather_best_kernel(MemeticStateDev st, const int32_t *__restrict__ state_idx,
                                   const int32_t *__restrict__ ns, int32_t n_uniform,
                                   int32_t count, int8_t *__restrict__ best_seq,
                                   int32_t out_stride, int32_t *__restrict__ best_e,
                                   int64_t *__restrict__ hit_gen,
                                   int64_t *__restrict__ gens_done) {
    const int i = blockIdx.x;
    if (i >= count) return;
    const int lane = lane_id();
    const int s = state_idx ? state_idx[i] : i;
    const int N = ns ? ns[i] : n_uniform;
    const M256 b = load_mask<4>(st.best + (int64_t)s * kStateWords);
    int8_t *out = best_seq + (int64_t)i * out_stride;
    for (int k = lane; k < out_stride; k += 64)
        out[k] = k < N ? (m_bit(b, k) ? (int8_t)-1 : (int8_t)1) : (int8_t)0;
    best_e[i] = st.bestE[s];  // uniform values, every lane
    if (hit_gen) hit_gen[i] = st.hit[s];
    if (gens_done) gens_done[i] = st.gen[s];
}

}  // namespace

hipError_t launch_memetic_init(const MemeticLaunchArgs &a, hipStream_t s) {
    if (a.n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(memetic_init_kernel, dim3((unsigned)a.n_slots), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_memetic_latch(const uint32_t *any_hit, uint32_t *stop,
                                const volatile uint32_t *cancel, uint32_t epoch, int stop_all,
                                hipStream_t s) {
    hipLaunchKernelGGL(memetic_latch_kernel, dim3(1), dim3(1), 0, s, any_hit, stop, cancel, epoch,
                       stop_all);
    return hipGetLastError();
}

namespace {

// Batched generations: B wavefronts per replica and dynamic LDS for the
// population plus B walk scratches.
template <int NW>
constexpr size_t batched_lds_bytes(int children) {
    return batched_header<NW>() + (size_t)children * walk_lds_bytes<NW, kBatchedLag<NW>>();
}

template <int NW>
hipError_t launch_batched(const MemeticLaunchArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((memetic_batched_kernel<NW>), dim3((unsigned)a.n_slots), dim3(64 * a.children),
                       batched_lds_bytes<NW>(a.children), s, a);
    return hipGetLastError();
}

}  // namespace

int prepare_memetic_kernels() {
    // more than 64 KB of dynamic LDS (eight children of N > 64) needs the
    // attribute; the CU has 160 KB.  N > 128 takes 17.7 KB per child: the
    // largest child count the device accepts is returned.
    hipError_t e = hipFuncSetAttribute((const void *)memetic_batched_kernel<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)batched_lds_bytes<1>(kMaxChildren));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)memetic_batched_kernel<2>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)batched_lds_bytes<2>(kMaxChildren));
    if (e != hipSuccess) return -1;
    for (int b = kMaxChildren; b >= 1; --b) {
        if (hipFuncSetAttribute((const void *)memetic_batched_kernel<4>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)batched_lds_bytes<4>(b)) == hipSuccess)
            return b;
        (void)hipGetLastError();  // clear the refusal
    }
    return 0;
}

namespace {

// Kernels of one memetic length class c (mask words 1 << c) on stream s.
hipError_t launch_memetic_class(const MemeticLaunchArgs &a, int c, hipStream_t s) {
    const dim3 grid((unsigned)a.n_slots);
    if (a.children > 1) {
        if (c == 0) return launch_batched<1>(a, s);
        if (c == 1) return launch_batched<2>(a, s);
        return launch_batched<4>(a, s);
    }
    if (c == 0)
        hipLaunchKernelGGL((memetic_advance_kernel<1, 1>), grid, dim3(64), 0, s, a);
    else if (c == 1 && a.split_wide)
        hipLaunchKernelGGL((memetic_advance_kernel<2, 2>), grid, dim3(128), 0, s, a);
    else if (c == 1)
        hipLaunchKernelGGL((memetic_advance_kernel<2, 1>), grid, dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((memetic_advance_kernel<4, 1>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_memetic_advance(const MemeticLaunchArgs &a, hipStream_t s,
                                  const SideStreams *sides) {
    if (a.n_slots <= 0) return hipSuccess;
    // the widest class present runs on s, each further one on a side stream
    int present[3], n = 0;
    for (int c = 2; c >= 0; --c)
        if (a.classes & (1 << c)) present[n++] = c;
    const int n_sides = sides != nullptr ? std::min(n - 1, kSideStreams) : 0;
    hipError_t e = hipSuccess;
    if (n_sides > 0) {
        e = hipEventRecord(sides->fork, s);
        for (int i = 0; i < n_sides && e == hipSuccess; ++i)
            e = hipStreamWaitEvent(sides->s[i], sides->fork, 0);
        if (e != hipSuccess) return e;
    }
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = launch_memetic_class(a, present[i], i > 0 && i <= n_sides ? sides->s[i - 1] : s);
    for (int i = 0; i < n_sides && e == hipSuccess; ++i) {
        e = hipEventRecord(sides->join[i], sides->s[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, sides->join[i], 0);
    }
    return e;
}

hipError_t launch_gather_best(const MemeticStateDev &st, const int32_t *state_idx,
                              const int32_t *ns, int32_t n_uniform, int32_t count,
                              int8_t *best_seq, int32_t out_stride, int32_t *best_e,
                              int64_t *hit_gen, int64_t *gens_done, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_best_kernel, dim3((unsigned)count), dim3(64), 0, s, st, state_idx,
                       ns, n_uniform, count, best_seq, out_stride, best_e, hit_gen, gens_done);
    return hipGetLastError();
}

}  // namespace liblabs
