// Kernels of liblabs for gfx950 and their launchers.
//
//   energy_kernel          Eq. (2) for a batch of +-1 rows, one row per wave
//   tabu_kernel            independent tabu walks (Alg. 2 / Alg. 4), one walk
//                          per wave, either one wave per walk or a persistent
//                          grid draining a longest-first work queue
//   memetic_init_kernel    random populations (Alg. 1, first two lines)
//   memetic_advance_kernel memetic generations (Alg. 1 / Alg. 3), one replica
//                          per wave, population resident in LDS
#include <algorithm>

#include "labs_device.hpp"
#include "labs_internal.h"

namespace liblabs {

namespace {

constexpr int kMaxK = 128;

// ---------------------------------------------------------------------------
// Energies.
// ---------------------------------------------------------------------------
template <int WPG>
__global__ __launch_bounds__(64 * WPG) void energy_kernel(const int8_t *__restrict__ seqs,
                                                          const int32_t *__restrict__ ns,
                                                          int32_t n_uniform, int32_t stride,
                                                          int64_t count,
                                                          int32_t *__restrict__ out) {
    const int lane = lane_id();
    const int64_t b = (int64_t)blockIdx.x * WPG + (threadIdx.x >> 6);
    if (b >= count) return;
    const int N = ns ? ns[b] : n_uniform;
    const int8_t *row = seqs + b * (int64_t)stride;
    bool b0 = false, b1 = false;
    if (lane < N) b0 = row[lane] < 0;
    if (lane + 64 < N) b1 = row[lane + 64] < 0;
    const M128 M{ballot(b0), ballot(b1)};
    int acc = 0;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const int k = lane + 1 + 64 * w;
        if (k < N) {
            const int c = lag_corr(M, N, k);
            acc += c * c;
        }
    }
    const int E = wave_sum(acc);
    out[b] = E;  // every lane stores the same value: no lane-0 branch
}

// ---------------------------------------------------------------------------
// Exhaustive minimum.  Lane g of the grid evaluates the codes
// [g * per, (g + 1) * per) (code c <=> sequence mask c << 1, so s_0 = +1) by
// Eq. (1)-(2) through popcounts: C_k = (N - k) - 2 popc((M ^ M >> k) & low).
// Masks fit 32 bits up to N = 32, 64 bits up to N = 40.
// ---------------------------------------------------------------------------
template <typename U>
__device__ __forceinline__ int code_energy(U M, int N) {
    int e = 0;
    for (int k = 1; k < N; ++k) {
        const U low = (U)((U)~(U)0 >> (8 * sizeof(U) - (N - k)));
        int p;
        if constexpr (sizeof(U) == 8)
            p = __popcll((M ^ (M >> k)) & low);
        else
            p = __popc((M ^ (M >> k)) & low);
        const int c = (N - k) - 2 * p;
        e += c * c;
    }
    return e;
}

template <typename U>
__global__ __launch_bounds__(256) void bruteforce_kernel(int N, uint64_t per, uint64_t total,
                                                         int32_t *part_e, int64_t *part_count,
                                                         uint64_t *part_code) {
    const int lane = lane_id();
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t wave = g >> 6;
    uint64_t c0 = g * per, c1 = c0 + per;
    if (c0 > total) c0 = total;
    if (c1 > total) c1 = total;
    int best = INT_MAX;
    int64_t cnt = 0;
    uint64_t best_code = ~0ull;
    for (uint64_t c = c0; c < c1; ++c) {
        const int e = code_energy<U>((U)(c << 1), N);
        if (e < best) {
            best = e;
            cnt = 1;
            best_code = c;
        } else if (e == best) {
            ++cnt;
        }
    }
    // Wavefront: minimum, its count, and the smallest code (lanes hold
    // ascending code ranges, so the lowest attaining lane has it).
    const int m = wave_min(best);
    const uint64_t at = ballot(best == m);
    const int src = __builtin_ctzll(at);
    const uint64_t code = ((uint64_t)readlane_u((uint32_t)(best_code >> 32), src) << 32) |
                          readlane_u((uint32_t)best_code, src);
    const int32_t n_at = best == m ? (int32_t)cnt : 0;
    int64_t tot = 0;
    for (int l = 0; l < 64; ++l) tot += (int64_t)readlane(n_at, l);
    part_e[wave] = m;  // uniform values, stored by every lane
    part_count[wave] = tot;
    part_code[wave] = code;
    (void)lane;
}

__global__ __launch_bounds__(64) void bruteforce_reduce_kernel(int64_t waves, BruteParts p) {
    const int lane = lane_id();
    int best = INT_MAX;
    for (int64_t w = lane; w < waves; w += 64) best = min(best, p.part_e[w]);
    const int m = wave_min(best);
    int64_t cnt = 0;
    uint64_t code = ~0ull;
    for (int64_t w = lane; w < waves; w += 64) {
        if (p.part_e[w] == m) {
            cnt += p.part_count[w];
            code = p.part_code[w] < code ? p.part_code[w] : code;
        }
    }
    int64_t tot = 0;
    uint64_t cmin = ~0ull;
    for (int l = 0; l < 64; ++l) {
        tot += ((int64_t)readlane_u((uint32_t)(cnt >> 32), l) << 32) |
               readlane_u((uint32_t)cnt, l);
        const uint64_t cl = ((uint64_t)readlane_u((uint32_t)(code >> 32), l) << 32) |
                            readlane_u((uint32_t)code, l);
        cmin = cl < cmin ? cl : cmin;
    }
    p.out_e[0] = m;  // uniform values, stored by every lane
    p.out_count[0] = 2 * tot;  // and the negations (s_0 = -1)
    p.out_code[0] = cmin << 1;
}

// ---------------------------------------------------------------------------
// Batched tabu walks.
// ---------------------------------------------------------------------------
template <int NW, int NB, bool TRACE>
__device__ void run_tabu_item(const TabuLaunchArgs &a, int64_t w, int N, uint8_t *lds) {
    using Mask = typename MaskOf<NW>::type;
    const int lane = lane_id();
    uint64_t lo, hi;
    if (a.starts != nullptr) {
        const int8_t *row = a.starts + w * (int64_t)a.start_stride;
        bool b0 = false, b1 = false;
        if (lane < N) b0 = row[lane] < 0;
        if (lane + 64 < N) b1 = row[lane + 64] < 0;
        lo = ballot(b0);
        hi = ballot(b1);
    } else {
        const Draw4 d = philox10((uint32_t)w, 0u, 0u, kTagStart, a.k0, a.k1);
        lo = (uint64_t)d.w0 | ((uint64_t)d.w1 << 32);
        hi = (uint64_t)d.w2 | ((uint64_t)d.w3 << 32);
        if (N < 64) {
            lo &= (1ull << N) - 1ull;
            hi = 0ull;
        } else {
            hi &= (N >= 128) ? ~0ull : ((1ull << (N - 64)) - 1ull);
        }
    }
    const Mask M = make_mask<NW>(lo, hi);
    const Schedule sch = make_schedule(a.rule, N, a.k0, a.k1, (uint32_t)w, 0u);
    const WalkResult<NW> r =
        tabu_walk<NW, TRACE, 1, NB>(N, M, sch, a.rule.aspiration, a.k0, a.k1, (uint32_t)w, 0u, lds,
                                    TRACE ? a.trace + w * (int64_t)a.trace_stride : nullptr);
    int8_t *out = a.best_seq + w * (int64_t)a.out_stride;
    for (int i = lane; i < a.out_stride; i += 64)
        out[i] = i < N ? (m_bit(r.best, i) ? (int8_t)-1 : (int8_t)1) : (int8_t)0;
    a.best_e[w] = r.best_e;  // uniform values, stored by every lane
    a.final_e[w] = r.final_e;
}

// Next index of the persistent work queue, wave-uniform.  Every lane executes
// the atomic (lane 0 adds 1, the others add 0) so that the value read back
// with readlane is never produced under a lane-dependent branch: a
// lane-0-only fetch lets the optimiser thread that branch into the loop's
// other lane-0 branches, and lanes then reach the readlane before lane 0 has
// fetched, disagreeing on the index.
__device__ __forceinline__ uint32_t next_work(uint32_t *counter) {
    const uint32_t v = atomicAdd(counter, lane_id() == 0 ? 1u : 0u);
    return readlane_u(v, 0);
}

// Walks at positions [begin, end) of the processing order, all of one length
// class: NW neighbours per lane (N <= 64 NW) and windows of NB chunks
// (N - 1 <= 16 NB).  PERSIST: a grid sized to the device drains the range
// through the queue head `counter`; otherwise one wave per position.
// TRACE: record every walk's moves (a separate instantiation, so that the
// untraced kernel does not carry the registers of the traced one).
template <int NW, int NB, int WPG, bool PERSIST, bool TRACE>
__global__ __launch_bounds__(64 * WPG) void tabu_kernel(TabuLaunchArgs a, int64_t begin,
                                                        int64_t end, uint32_t *counter) {
    __shared__ __attribute__((aligned(16))) uint8_t lds_all[WPG][walk_lds_bytes<NW>()];
    const int wave = threadIdx.x >> 6;
    uint8_t *lds = lds_all[wave];
    if constexpr (PERSIST) {
        for (int64_t pos = begin + next_work(counter); pos < end;
             pos = begin + next_work(counter)) {
            const int64_t w = a.order ? (int64_t)a.order[pos] : pos;
            run_tabu_item<NW, NB, TRACE>(a, w, a.ns ? a.ns[w] : a.n_uniform, lds);
        }
    } else {
        const int64_t pos = begin + (int64_t)blockIdx.x * WPG + wave;
        if (pos < end) {
            const int64_t w = a.order ? (int64_t)a.order[pos] : pos;
            run_tabu_item<NW, NB, TRACE>(a, w, a.ns ? a.ns[w] : a.n_uniform, lds);
        }
    }
}

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

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

}  // namespace

// Lanes of the exhaustive search: every lane gets at least 64 codes, at
// most 2^18 lanes (4096 wavefronts) share the space.
static uint64_t brute_lanes(int n) {
    const uint64_t total = 1ull << (n - 1);
    uint64_t lanes = total >> 6;
    if (lanes < 64) lanes = 64;
    if (lanes > (1ull << 18)) lanes = 1ull << 18;
    return lanes;
}

int64_t brute_waves(int n) { return (int64_t)(brute_lanes(n) >> 6); }

hipError_t launch_bruteforce(int n, const BruteParts &p, hipStream_t s) {
    const uint64_t total = 1ull << (n - 1);
    const uint64_t lanes = brute_lanes(n);
    const uint64_t per = (total + lanes - 1) / lanes;
    const unsigned blocks = (unsigned)(lanes / 256 > 0 ? lanes / 256 : 1);
    const unsigned threads = (unsigned)(lanes < 256 ? lanes : 256);
    if (n <= 32)
        hipLaunchKernelGGL(bruteforce_kernel<uint32_t>, dim3(blocks), dim3(threads), 0, s, n, per,
                           total, p.part_e, p.part_count, p.part_code);
    else
        hipLaunchKernelGGL(bruteforce_kernel<uint64_t>, dim3(blocks), dim3(threads), 0, s, n, per,
                           total, p.part_e, p.part_count, p.part_code);
    hipLaunchKernelGGL(bruteforce_reduce_kernel, dim3(1), dim3(64), 0, s, (int64_t)(lanes >> 6), p);
    return hipGetLastError();
}

hipError_t launch_energy(const int8_t *seqs, const int32_t *ns, int32_t n_uniform,
                         int32_t stride, int64_t count, int32_t *out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    constexpr int WPG = 4;
    const int64_t grid = (count + WPG - 1) / WPG;
    hipLaunchKernelGGL(energy_kernel<WPG>, dim3((unsigned)grid), dim3(64 * WPG), 0, s, seqs, ns,
                       n_uniform, stride, count, out);
    return hipGetLastError();
}

namespace {

template <int NW, int NB, int WPG, bool TRACE>
hipError_t launch_tabu_part_t(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                              uint32_t *counter, hipStream_t s) {
    if (groups > 0) {
        hipError_t e = launch_fill_u32(counter, 0u, 1, s);
        if (e != hipSuccess) return e;
        const int64_t need = (end - begin + WPG - 1) / WPG;
        hipLaunchKernelGGL((tabu_kernel<NW, NB, WPG, true, TRACE>),
                           dim3((unsigned)std::min<int64_t>(groups, need)), dim3(64 * WPG), 0, s, a,
                           begin, end, counter);
    } else {
        const int64_t grid = (end - begin + WPG - 1) / WPG;
        hipLaunchKernelGGL((tabu_kernel<NW, NB, WPG, false, TRACE>), dim3((unsigned)grid),
                           dim3(64 * WPG), 0, s, a, begin, end, counter);
    }
    return hipGetLastError();
}

template <int NW, int NB, int WPG>
hipError_t launch_tabu_part(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                            uint32_t *counter, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    return a.trace != nullptr
               ? launch_tabu_part_t<NW, NB, WPG, true>(a, begin, end, groups, counter, s)
               : launch_tabu_part_t<NW, NB, WPG, false>(a, begin, end, groups, counter, s);
}

// One launch per non-empty length class, each on its own stream with its
// own queue head (32 words apart).
template <int WPG>
hipError_t launch_tabu_wpg(const TabuLaunchArgs &a, int groups, const hipStream_t *st) {
    static_assert(kWalkClasses == 4, "one launcher per class below");
    const int64_t *ce = a.class_end;
    hipError_t e = launch_tabu_part<2, 8, WPG>(a, 0, ce[0], groups, a.counter, st[0]);
    if (e == hipSuccess) e = launch_tabu_part<2, 6, WPG>(a, ce[0], ce[1], groups, a.counter + 32, st[1]);
    if (e == hipSuccess) e = launch_tabu_part<1, 4, WPG>(a, ce[1], ce[2], groups, a.counter + 64, st[2]);
    if (e == hipSuccess) e = launch_tabu_part<1, 3, WPG>(a, ce[2], ce[3], groups, a.counter + 96, st[3]);
    return e;
}

}  // namespace

hipError_t launch_tabu(const TabuLaunchArgs &a, int waves_per_group, int groups,
                       const hipStream_t *streams) {
    if (a.W <= 0) return hipSuccess;
    switch (waves_per_group) {
    case 1: return launch_tabu_wpg<1>(a, groups, streams);
    case 2: return launch_tabu_wpg<2>(a, groups, streams);
    case 4: return launch_tabu_wpg<4>(a, groups, streams);
    default: return hipErrorInvalidValue;
    }
}

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

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t grid = (count + 255) / 256;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)grid), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
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
