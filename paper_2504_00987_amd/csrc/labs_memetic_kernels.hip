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


// ---------------------------------------------------------------------------
// Memetic replicas.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t word_of(const Draw4 &d, int i) {
    return i == 0 ? d.w0 : (i == 1 ? d.w1 : (i == 2 ? d.w2 : d.w3));
}

__global__ __launch_bounds__(64) void memetic_init_kernel(MemeticLaunchArgs a) {
    const int s = blockIdx.x;
    if (s >= a.n_slots) return;
    const MemeticSlot sl = a.slots[s];
    if (sl.state < 0) return;
    const int lane = lane_id();
    const int N = sl.n, K = a.K;
    const int64_t base = (int64_t)sl.state * K;
    uint64_t lo[2] = {0ull, 0ull}, hi[2] = {0ull, 0ull};
    int e[2] = {INT_MAX, INT_MAX};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int m = lane + 64 * h;
        if (m < K) {
            const Draw4 d = philox10(sl.pop_id, (uint32_t)m, 0u, kTagInit, sl.k0, sl.k1);
            uint64_t l = (uint64_t)d.w0 | ((uint64_t)d.w1 << 32);
            uint64_t u = (uint64_t)d.w2 | ((uint64_t)d.w3 << 32);
            if (N < 64) {
                l &= (1ull << N) - 1ull;
                u = 0ull;
            } else {
                u &= (N >= 128) ? ~0ull : ((1ull << (N - 64)) - 1ull);
            }
            lo[h] = l;
            hi[h] = u;
            e[h] = N <= 64 ? lane_energy<uint64_t>(l, N) : lane_energy<M128>(M128{l, u}, N);
            a.st.pop[(base + m) * 2 + 0] = l;
            a.st.pop[(base + m) * 2 + 1] = u;
            a.st.popE[base + m] = e[h];
        }
    }
    // bestSeq: the lowest-index member of minimum energy.
    const int mn = wave_min(min(e[0], e[1]));
    const uint64_t t0 = ballot(e[0] == mn), t1 = ballot(e[1] == mn);
    const int h = t0 ? 0 : 1;
    const int src = t0 ? __builtin_ctzll(t0) : __builtin_ctzll(t1);
    const uint64_t sel_lo = h == 0 ? lo[0] : lo[1];
    const uint64_t sel_hi = h == 0 ? hi[0] : hi[1];
    const uint64_t blo = ((uint64_t)readlane_u((uint32_t)(sel_lo >> 32), src) << 32) |
                         readlane_u((uint32_t)sel_lo, src);
    const uint64_t bhi = ((uint64_t)readlane_u((uint32_t)(sel_hi >> 32), src) << 32) |
                         readlane_u((uint32_t)sel_hi, src);
    a.st.best[(int64_t)sl.state * 2 + 0] = blo;  // uniform values, every lane
    a.st.best[(int64_t)sl.state * 2 + 1] = bhi;
    a.st.bestE[sl.state] = mn;
    a.st.gen[sl.state] = 0;
    a.st.hit[sl.state] = -1;
}

// One replica on SPLIT wavefronts (wavefront `part` of them); every
// wavefront runs the generation logic redundantly on wave-uniform values and
// the walk is split between them.
template <int NW, int SPLIT>
__device__ void memetic_replica(const MemeticLaunchArgs &a, const MemeticSlot &sl,
                                uint64_t (*pop)[2], int *popE, uint8_t *lds, int part) {
    using Mask = typename MaskOf<NW>::type;
    const int lane = lane_id();
    const int N = sl.n, K = a.K, st = sl.state;
    const int64_t base = (int64_t)st * K;
    for (int i = lane + 64 * part; i < K; i += 64 * SPLIT) {
        pop[i][0] = a.st.pop[(base + i) * 2 + 0];
        pop[i][1] = a.st.pop[(base + i) * 2 + 1];
        popE[i] = a.st.popE[base + i];
    }
    walk_sync<SPLIT>();
    Mask best = make_mask<NW>(a.st.best[(int64_t)st * 2 + 0], a.st.best[(int64_t)st * 2 + 1]);
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
            const Mask A = make_mask<NW>(pop[pa][0], pop[pa][1]);
            const Mask B = make_mask<NW>(pop[pb][0], pop[pb][1]);
            const Mask lowm = m_low(A, cut);
            child = m_or(m_and(A, lowm), m_and(B, m_not(lowm)));
        } else {
            const int c = (int)below(da.w1, (uint32_t)K);
            child = make_mask<NW>(pop[c][0], pop[c][1]);
        }
        // Mutate: bit i flips when word i%4 of draw (pop, g, i/4, MUT) < thr.
        uint64_t flo, fhi = 0ull;
        {
            const int i0 = lane;
            const Draw4 d = philox10(sl.pop_id, gg, (uint32_t)(i0 >> 2), kTagMut, sl.k0, sl.k1);
            flo = ballot(i0 < N && word_of(d, i0 & 3) < thr);
            if constexpr (NW == 2) {
                const int i1 = lane + 64;
                const Draw4 d1 = philox10(sl.pop_id, gg, (uint32_t)(i1 >> 2), kTagMut, sl.k0, sl.k1);
                fhi = ballot(i1 < N && word_of(d1, i1 & 3) < thr);
            }
        }
        child = m_xor(child, make_mask<NW>(flo, fhi));
        const Schedule sch = make_schedule(a.rule, N, sl.k0, sl.k1, sl.pop_id, gg);
        const WalkResult<NW> r = tabu_walk<NW, false, SPLIT>(N, child, sch, a.rule.aspiration,
                                                             sl.k0, sl.k1, sl.pop_id, gg, lds,
                                                             nullptr, part);
        if (r.best_e < bestE) {
            bestE = r.best_e;
            best = r.best;
        }
        const int rep = (int)below(db.w2, (uint32_t)K);
        walk_sync<SPLIT>();
        pop[rep][0] = mask_lo(r.best);  // uniform values, every lane
        pop[rep][1] = mask_hi(r.best);
        popE[rep] = r.best_e;
        walk_sync<SPLIT>();
        ++g;
        if (targeted && bestE <= sl.target) {
            if (hit < 0) hit = g;
            break;
        }
    }

    for (int i = lane + 64 * part; i < K; i += 64 * SPLIT) {
        a.st.pop[(base + i) * 2 + 0] = pop[i][0];
        a.st.pop[(base + i) * 2 + 1] = pop[i][1];
        a.st.popE[base + i] = popE[i];
    }
    if (part != 0) return;
    a.st.best[(int64_t)st * 2 + 0] = mask_lo(best);  // uniform values, every lane
    a.st.best[(int64_t)st * 2 + 1] = mask_hi(best);
    a.st.bestE[st] = bestE;
    a.st.gen[st] = g;
    a.st.hit[st] = hit;
    if (hit >= 0 && a.any_hit != nullptr) atomicOr(a.any_hit, 1u);
}

// Replicas of one length class: N <= 64 (NW = 1) or 64 < N <= 128 (NW = 2),
// one workgroup of SPLIT wavefronts per replica; slots of the other class
// and idle slots return at once.  The two-wavefront form only runs when
// there are at most two replicas per compute unit, so it is compiled for
// latency (all of a step's LDS reads in flight at once) rather than for
// occupancy.
template <int NW, int SPLIT>
__global__ __launch_bounds__(64 * SPLIT)
__attribute__((amdgpu_waves_per_eu(1, SPLIT == 2 ? 2 : 8))) void memetic_advance_kernel(
    MemeticLaunchArgs a) {
    __shared__ uint64_t pop[kMaxK][2];
    __shared__ int popE[kMaxK];
    __shared__ __attribute__((aligned(16))) uint8_t lds[walk_lds_bytes<NW>()];
    const int s = blockIdx.x;
    if (s >= a.n_slots) return;
    const MemeticSlot sl = a.slots[s];
    if (sl.state < 0 || (sl.n > 64) != (NW == 2)) return;
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
constexpr int kBatchedHeader = kMaxK * 16 + kMaxK * 4 + kMaxChildren * 32;

template <int NW>
__global__ __launch_bounds__(64 * kMaxChildren) void memetic_batched_kernel(
    MemeticLaunchArgs a) {
    using Mask = typename MaskOf<NW>::type;
    extern __shared__ __attribute__((aligned(16))) uint8_t dyn_lds[];
    uint64_t(*pop)[2] = (uint64_t(*)[2])dyn_lds;
    int *popE = (int *)(dyn_lds + kMaxK * 16);
    uint64_t *res = (uint64_t *)(dyn_lds + kMaxK * 20);  // [B][lo, hi, e, slot]
    const int s = blockIdx.x;
    if (s >= a.n_slots) return;
    const MemeticSlot sl = a.slots[s];
    if (sl.state < 0 || (sl.n > 64) != (NW == 2)) return;
    const int B = a.children;
    const int b = (int)(threadIdx.x >> 6);
    uint8_t *lds = dyn_lds + kBatchedHeader + b * walk_lds_bytes<NW>();
    const int lane = lane_id();
    const int N = sl.n, K = a.K, st = sl.state;
    const int64_t base = (int64_t)st * K;
    for (int i = (int)threadIdx.x; i < K; i += 64 * B) {
        pop[i][0] = a.st.pop[(base + i) * 2 + 0];
        pop[i][1] = a.st.pop[(base + i) * 2 + 1];
        popE[i] = a.st.popE[base + i];
    }
    __syncthreads();
    Mask best = make_mask<NW>(a.st.best[(int64_t)st * 2 + 0], a.st.best[(int64_t)st * 2 + 1]);
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
            const Mask A = make_mask<NW>(pop[pa][0], pop[pa][1]);
            const Mask Bm = make_mask<NW>(pop[pb][0], pop[pb][1]);
            const Mask lowm = m_low(A, cut);
            child = m_or(m_and(A, lowm), m_and(Bm, m_not(lowm)));
        } else {
            const int c = (int)below(da.w1, (uint32_t)K);
            child = make_mask<NW>(pop[c][0], pop[c][1]);
        }
        uint64_t flo, fhi = 0ull;
        {
            const int i0 = lane;
            const Draw4 d = philox10(sl.pop_id, gg, (uint32_t)(32 * b + (i0 >> 2)), kTagMut,
                                     sl.k0, sl.k1);
            flo = ballot(i0 < N && word_of(d, i0 & 3) < thr);
            if constexpr (NW == 2) {
                const int i1 = lane + 64;
                const Draw4 d1 = philox10(sl.pop_id, gg, (uint32_t)(32 * b + (i1 >> 2)), kTagMut,
                                          sl.k0, sl.k1);
                fhi = ballot(i1 < N && word_of(d1, i1 & 3) < thr);
            }
        }
        child = m_xor(child, make_mask<NW>(flo, fhi));
        const uint32_t wgen = (uint32_t)(g * B + b);
        const Schedule sch = make_schedule(a.rule, N, sl.k0, sl.k1, sl.pop_id, wgen);
        const WalkResult<NW> r = tabu_walk<NW>(N, child, sch, a.rule.aspiration, sl.k0, sl.k1,
                                               sl.pop_id, wgen, lds, nullptr);
        res[4 * b + 0] = mask_lo(r.best);  // uniform values, every lane of wavefront b
        res[4 * b + 1] = mask_hi(r.best);
        res[4 * b + 2] = (uint64_t)(uint32_t)r.best_e;
        res[4 * b + 3] = (uint64_t)below(db.w2, (uint32_t)K);
        __syncthreads();
        for (int c = 0; c < B; ++c) {
            const uint64_t lo = uniform64(res[4 * c + 0]);
            const uint64_t hi = uniform64(res[4 * c + 1]);
            const int e = __builtin_amdgcn_readfirstlane((int)(uint32_t)res[4 * c + 2]);
            const int slot = __builtin_amdgcn_readfirstlane((int)(uint32_t)res[4 * c + 3]);
            if (e < bestE) {
                bestE = e;
                best = make_mask<NW>(lo, hi);
            }
            if (b == 0) {
                pop[slot][0] = lo;  // uniform values, every lane of wavefront 0
                pop[slot][1] = hi;
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
        a.st.pop[(base + i) * 2 + 0] = pop[i][0];
        a.st.pop[(base + i) * 2 + 1] = pop[i][1];
        a.st.popE[base + i] = popE[i];
    }
    if (b != 0) return;
    a.st.best[(int64_t)st * 2 + 0] = mask_lo(best);  // uniform values, every lane
    a.st.best[(int64_t)st * 2 + 1] = mask_hi(best);
    a.st.bestE[st] = bestE;
    a.st.gen[st] = g;
    a.st.hit[st] = hit;
    if (hit >= 0 && a.any_hit != nullptr) atomicOr(a.any_hit, 1u);
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
    const M128 b{st.best[(int64_t)s * 2 + 0], st.best[(int64_t)s * 2 + 1]};
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

namespace {

// Batched generations: B wavefronts per replica and dynamic LDS for the
// population plus B walk scratches.
template <int NW>
constexpr size_t batched_lds_bytes(int children) {
    return kBatchedHeader + (size_t)children * walk_lds_bytes<NW>();
}

template <int NW>
hipError_t launch_batched(const MemeticLaunchArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((memetic_batched_kernel<NW>), dim3((unsigned)a.n_slots), dim3(64 * a.children),
                       batched_lds_bytes<NW>(a.children), s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t prepare_memetic_kernels() {
    // eight children of N > 64 take more than the 64 KB of dynamic LDS a
    // launch gets without the attribute (the CU has 160 KB)
    hipError_t e = hipFuncSetAttribute((const void *)memetic_batched_kernel<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)batched_lds_bytes<1>(kMaxChildren));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)memetic_batched_kernel<2>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)batched_lds_bytes<2>(kMaxChildren));
    return e;
}

hipError_t launch_memetic_advance(const MemeticLaunchArgs &a, hipStream_t s, hipStream_t side,
                                  hipEvent_t fork, hipEvent_t join) {
    if (a.n_slots <= 0) return hipSuccess;
    const bool split = a.classes == 3 && side != nullptr && fork != nullptr && join != nullptr;
    hipStream_t s1 = s;
    if (split) {
        hipError_t e = hipEventRecord(fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
        if (e != hipSuccess) return e;
        s1 = side;
    }
    hipError_t e = hipSuccess;
    if (a.children > 1) {
        if (a.classes & 1) e = launch_batched<1>(a, s1);
        if (e == hipSuccess && (a.classes & 2)) e = launch_batched<2>(a, s);
    } else {
        if (a.classes & 1)
            hipLaunchKernelGGL((memetic_advance_kernel<1, 1>), dim3((unsigned)a.n_slots), dim3(64),
                               0, s1, a);
        if ((a.classes & 2) && a.split_wide)
            hipLaunchKernelGGL((memetic_advance_kernel<2, 2>), dim3((unsigned)a.n_slots),
                               dim3(128), 0, s, a);
        else if (a.classes & 2)
            hipLaunchKernelGGL((memetic_advance_kernel<2, 1>), dim3((unsigned)a.n_slots), dim3(64),
                               0, s, a);
        e = hipGetLastError();
    }
    if (split && e == hipSuccess) {
        e = hipEventRecord(join, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
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
