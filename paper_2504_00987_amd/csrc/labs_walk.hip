// Walk kernels of liblabs for gfx950 and their launchers.
//
//   energy_kernel   Eq. (2) for a batch of +-1 rows, one row per wave
//   tabu_kernel     independent tabu walks (Alg. 2 / Alg. 4), one walk per
//                   wave, either one wave per walk or a persistent grid
//                   draining a longest-first work queue; one instantiation
//                   per length class (tabu_kernel_mixed: several classes in
//                   one launch; tabu_kernel_split: a walk on two waves;
//                   tabu_kernel_group: two or four walks of N <= 32 per wave)
//   fill_u32_kernel device-side fill (queue heads, flags), capturable
//   order_by_length_kernel  longest-first processing order built on the
//                   device (the allocation-free entry point's lengths)
#include <algorithm>
#include <mutex>

#include "../../include/liblabs.h"
#include "labs_device.hpp"
#include "labs_internal.h"

namespace liblabs {

namespace {


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
    uint64_t wd[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int i = lane + 64 * h;
        wd[h] = ballot(i < N && row[i] < 0);
    }
    const M256 M{wd[0], wd[1], wd[2], wd[3]};
    int acc = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
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
// Batched tabu walks.
// ---------------------------------------------------------------------------
// Start mask of walk w: row w of the caller's starts, or the draws
// (w, 0, q, START) (bits 128 q .. 128 q + 127).
template <int NW>
__device__ __forceinline__ typename MaskOf<NW>::type walk_start(const TabuLaunchArgs &a,
                                                                int64_t w, int N) {
    const int lane = lane_id();
    uint64_t wd[4] = {0ull, 0ull, 0ull, 0ull};
    if (a.starts != nullptr) {
        const int8_t *row = a.starts + w * (int64_t)a.start_stride;
#pragma unroll
        for (int h = 0; h < NW; ++h) {
            const int i = lane + 64 * h;
            wd[h] = ballot(i < N && row[i] < 0);
        }
    } else {
#pragma unroll
        for (int q = 0; q < (NW + 1) / 2; ++q) {
            const Draw4 d = philox10((uint32_t)w, 0u, (uint32_t)q, kTagStart, a.k0, a.k1);
            wd[2 * q] = (uint64_t)d.w0 | ((uint64_t)d.w1 << 32);
            if (2 * q + 1 < NW) wd[2 * q + 1] = (uint64_t)d.w2 | ((uint64_t)d.w3 << 32);
        }
#pragma unroll
        for (int h = 0; h < NW; ++h) {
            const int b = N - 64 * h;  // bits of word h inside the sequence
            wd[h] &= b >= 64 ? ~0ull : b <= 0 ? 0ull : ((1ull << b) - 1ull);
        }
    }
    return make_mask<NW>(wd[0], wd[1], wd[2], wd[3]);
}

// One walk on one wavefront: NW neighbours per lane, windows of NB chunks,
// the lag form when LAG (N <= 128), else the record form.
template <int NW, int NB, bool TRACE, bool LAG = (NW == 1)>
__device__ void run_tabu_item(const TabuLaunchArgs &a, int64_t w, int N, uint8_t *lds) {
    const int lane = lane_id();
    const auto M = walk_start<NW>(a, w, N);
    const Schedule sch = make_schedule(a.rule, N, a.k0, a.k1, (uint32_t)w, 0u);
    const WalkResult<NW> r =
        tabu_walk<NW, TRACE, 1, NB, LAG>(N, M, sch, a.rule.aspiration, a.k0, a.k1, (uint32_t)w, 0u,
                                         lds, TRACE ? a.trace + w * (int64_t)a.trace_stride : nullptr);
    int8_t *out = a.best_seq + w * (int64_t)a.out_stride;
    for (int i = lane; i < a.out_stride; i += 64)
        out[i] = i < N ? (m_bit(r.best, i) ? (int8_t)-1 : (int8_t)1) : (int8_t)0;
    a.best_e[w] = r.best_e;  // uniform values, stored by every lane
    a.final_e[w] = r.final_e;
}

// One walk of 64 < N <= 128 on the two wavefronts of a 128-lane workgroup,
// wavefront `part` owning neighbours and lags 64 part .. 64 part + 63; each
// writes half of the output row.
template <int NB, bool TRACE, bool LAG>
__device__ void run_split_item(const TabuLaunchArgs &a, int64_t w, int N, uint8_t *lds,
                               int part) {
    const int lane = lane_id();
    const auto M = walk_start<2>(a, w, N);
    const Schedule sch = make_schedule(a.rule, N, a.k0, a.k1, (uint32_t)w, 0u);
    const WalkResult<2> r =
        tabu_walk<2, TRACE, 2, NB, LAG>(N, M, sch, a.rule.aspiration, a.k0, a.k1, (uint32_t)w, 0u,
                                        lds, TRACE ? a.trace + w * (int64_t)a.trace_stride : nullptr,
                                        part);
    int8_t *out = a.best_seq + w * (int64_t)a.out_stride;
    for (int i = lane + 64 * part; i < a.out_stride; i += 128)
        out[i] = i < N ? (m_bit(r.best, i) ? (int8_t)-1 : (int8_t)1) : (int8_t)0;
    if (part == 0) {
        a.best_e[w] = r.best_e;  // uniform values, stored by every lane of wavefront 0
        a.final_e[w] = r.final_e;
    }
}

// Next index of the persistent work queue, wave-uniform.  Every lane executes
// the atomic (lane 0 adds 1, the others add 0) so that the value read back
// with readlane is never produced under a lane-dependent branch: a
// lane-0-only fetch lets the optimiser thread that branch into the loop's
// other lane-0 branches, and lanes then reach the readlane before lane 0 has
// fetched, disagreeing on the index.
__device__ __forceinline__ uint32_t next_work(uint32_t *counter, uint32_t take = 1u) {
    const uint32_t v = atomicAdd(counter, lane_id() == 0 ? take : 0u);
    return readlane_u(v, 0);
}

// ---------------------------------------------------------------------------
// Several walks per wavefront (N <= 32).
// ---------------------------------------------------------------------------
// A wavefront runs G walks of N <= GL = 64 / G at once, lane l of group
// g = l / GL owning neighbour j = l % GL and lag k = j + 1 of walk g.  The
// step is the lag form's (rows of t_jk; v_j as dot products of row j with
// C; u_j kept per neighbour; one byte of each row rewritten per move), with
// every per-walk quantity (the sequence mask, E, the best, the chosen move,
// the schedule) held per lane for the lane's own walk instead of in scalar
// registers, the minimum and the energy taken within each group of lanes,
// and a tied move picked by its rank within the group.  Walks of different
// lengths share the step loop; a walk past its last step, or a group past
// the end of the range, takes no move.
//
// LDS of one walk: 16 spare bytes, rows j = 0..GL-1 of kGroupRow bytes
// (t_jk for k = 1..GL in bytes 0..GL-1, zero past the sequence; 48 bytes
// apart, an odd number of 16-byte slots, so that 16-byte reads of
// consecutive rows are conflict-free), C_k as int8 (GL bytes), then the
// sequence as int8 with zeros around it, SP[q] for q = -GL .. 2 GL - 1.
constexpr int kGroupRow = 48;
template <int GL>
struct GroupLds {
    static constexpr int BASE = 16;
    static constexpr int CB = BASE + GL * kGroupRow;
    static constexpr int SPLO = CB + GL, SP = SPLO + GL;
    static constexpr int BYTES = SPLO + 3 * GL;
    static_assert(BYTES % 16 == 0, "16-byte aligned walks");
};

// The two 16-lane rows of each 32-lane half, every lane receiving both:
// v_permlane16_swap with the value as both operands swaps the odd rows of
// one copy with the even rows of the other, so one copy holds rows 0, 0,
// 2, 2 and the other 1, 1, 3, 3 (a register exchange, no LDS trip).
__device__ __forceinline__ void row_pair(int v, int &a, int &b) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    a = (int)r[0];
    b = (int)r[1];
}

// Minimum and sum over each group of GL = 16 or 32 consecutive lanes, every
// lane receiving its group's value: row (16-lane) reductions by DPP, then,
// for GL = 32, the two rows of a group combined.
template <int GL>
__device__ __forceinline__ int group_min(int v) {
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_QUAD_1032, 0xf, 0xf, true));
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_QUAD_2301, 0xf, 0xf, true));
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_ROW_HALF_MIRROR, 0xf, 0xf, true));
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_ROW_MIRROR, 0xf, 0xf, true));
    if constexpr (GL == 32) {
        int a, b;
        row_pair(v, a, b);
        v = min(a, b);
    }
    return v;
}

template <int GL>
__device__ __forceinline__ int group_sum(int v) {
    v += __builtin_amdgcn_mov_dpp(v, LABS_DPP_QUAD_1032, 0xf, 0xf, true);
    v += __builtin_amdgcn_mov_dpp(v, LABS_DPP_QUAD_2301, 0xf, 0xf, true);
    v += __builtin_amdgcn_mov_dpp(v, LABS_DPP_ROW_HALF_MIRROR, 0xf, 0xf, true);
    v += __builtin_amdgcn_mov_dpp(v, LABS_DPP_ROW_MIRROR, 0xf, 0xf, true);
    if constexpr (GL == 32) {
        int a, b;
        row_pair(v, a, b);
        v = a + b;
    }
    return v;
}

// Group g's GL bits of a wave-wide ballot.
template <int GL>
__device__ __forceinline__ uint32_t group_bits(uint64_t m, int g) {
    return (uint32_t)(m >> (GL * g)) & (GL == 32 ? 0xffffffffu : 0xffffu);
}

// |a - b| + c in one instruction, every operand per lane.
__device__ __forceinline__ uint32_t absdiff_add_v(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// The value v of lane `src` (any lane of the wavefront), per lane.
__device__ __forceinline__ int lane_value(int v, int src) {
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

// Walks at processing-order positions pos0 .. pos0 + G - 1 (those below
// `end`), all of N <= 64 / G, on one wavefront; `lds` holds G walks'
// GroupLds.  Results as the one-walk-per-wavefront form writes them.
template <int G, bool TRACE>
__device__ void run_group_walks(const TabuLaunchArgs &a, int64_t pos0, int64_t end,
                                uint8_t *lds_wave) {
    constexpr int GL = 64 / G;
    constexpr int NB = GL / 16;  // 16-lag chunks of a row
    using L = GroupLds<GL>;
    const int lane = lane_id();
    const int g = lane / GL, j = lane % GL;
    const int64_t pos = pos0 + g;
    const bool live = pos < end;
    const int64_t w = live ? (a.order ? (int64_t)a.order[pos] : pos) : 0;
    const int N = live ? (a.ns ? a.ns[w] : a.n_uniform) : 0;
    uint8_t *const lds = lds_wave + g * L::BYTES;
    uint8_t *const rows = lds + L::BASE;
    int8_t *const CB = (int8_t *)(lds + L::CB);

    // start (bit i set <=> s_i = -1): the caller's row, or the low N bits
    // of the draw (w, 0, 0, START)
    uint32_t M;
    if (a.starts != nullptr) {
        const int8_t *row = a.starts + w * (int64_t)a.start_stride;
        M = group_bits<GL>(ballot(j < N && row[j] < 0), g);
    } else {
        const Draw4 d = philox10((uint32_t)w, 0u, 0u, kTagStart, a.k0, a.k1);
        M = N > 0 ? d.w0 & (0xffffffffu >> (32 - N)) : 0u;
    }
    Schedule sch = make_schedule(a.rule, N, a.k0, a.k1, (uint32_t)w, 0u);
    if (!live) sch.T = 0;
    const uint32_t Mr = N > 0 ? __builtin_bitreverse32(M) >> (32 - N) : 0u;  // bit i: s_{N-1-i}

    // row j: s_{j+k} is bit k-1 of R, s_{j-k} bit k-1 of Lb
    const int nr = max(N - 1 - j, 0), nl = j < N ? j : 0;
    const uint64_t R = (uint64_t)M >> (j + 1);
    const uint64_t Lb = j < N ? (uint64_t)Mr >> (N - j) : 0ull;
    uint32_t *const row = (uint32_t *)(rows + kGroupRow * j);
#pragma unroll
    for (int d = 0; d < GL / 4; ++d)
        row[d] = add_bytes(pack_bits4(R, 4 * d, nr), pack_bits4(Lb, 4 * d, nl));
    for (int idx = j; idx < 3 * GL / 4; idx += GL) {
        const int x = 4 * idx - GL;  // SP[x .. x+3]
        ((uint32_t *)(lds + L::SPLO))[idx] = x < 0 ? 0u : pack_bits4(M, x, N);
    }
    const int nu = min(nr, nl);
    int u2 = 2 * (nu - 2 * __popcll((R ^ Lb) & ((1ull << nu) - 1ull)));
    const int k = j + 1;
    int C = k < N ? (N - k) - 2 * __popcll(((uint64_t)M ^ ((uint64_t)M >> k)) &
                                           ((1ull << (N - k)) - 1ull))
                  : 0;
    CB[j] = (int8_t)C;
    int E = group_sum<GL>(C * C);
    int tabu = j < N ? 0 : INT_MAX;  // lanes past the sequence are never admissible
    const bool asp = a.rule.aspiration && j < N;
    const uint32_t rowm1 = lds_offset(lds) + (uint32_t)(L::BASE + kGroupRow * j - 1);
    const uint32_t spj = lds_offset(lds) + (uint32_t)(L::SP + 2 * j);
    uint32_t best = M;
    int bestE = E;
    int thr = -(N - 1);                   // ((bestE - E) >> 2) - (N - 1), kept per move
    int ns = (M >> j) & 1u ? 1 : -1;      // -s_j (lanes past the sequence: unused)
    const int T_all = -wave_min(-sch.T);  // the longest walk of the wavefront

    wave_sync();
    uint4 tc[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) tc[r] = ((const uint4 *)(rows + kGroupRow * j))[r];

    for (int t0 = 1; t0 <= T_all; t0 += GL) {
        // lane j of a group: the draws of its walk's step t0 + j
        uint32_t dr0;
        int expire;
        {
            const Draw4 d = philox10((uint32_t)w, 0u, (uint32_t)(t0 + j), kTagStep, a.k0, a.k1);
            dr0 = d.w0;
            expire = t0 + j + sch.lo + (int)below(d.w1, (uint32_t)(sch.hi - sch.lo + 1));
        }
        const int t_end = min(T_all, t0 + GL - 1);
        for (int t = t0; t <= t_end; ++t) {
            const int src = g * GL + (t - t0);  // the lane holding this step's draws
            wave_sync();                        // the previous move's C and row bytes
            uint4 cc[NB];
#pragma unroll
            for (int r = 0; r < NB; ++r) cc[r] = ((const uint4 *)CB)[r];
            const uint32_t dr = (uint32_t)lane_value((int)dr0, src);
            const int tabu_new = lane_value(expire, src);
            // key d_j = 2 u_j - s_j v_j: candE_j = E + 4 (N - 1) + 4 d_j, an
            // aspiration candidate when d_j < thr
            int v = 0;
#pragma unroll
            for (int r = 0; r < NB; ++r) v = dot16(tc[r], cc[r], v);
            const int d = mad_i24_after_dot(ns, v, u2);
            const int key = tabu < t || (asp && d < thr) ? d : INT_MAX;
            const int m = group_min<GL>(key);
            // ties: the r-th lowest tied neighbour of the group, r from the
            // step's first draw
            const uint64_t tied_all = ballot(key == m);
            const uint32_t tied = group_bits<GL>(tied_all, g);
            const int r = (int)below(dr, (uint32_t)__popc(tied));
            const uint64_t mine = tied_all & ballot(__popc(tied & ((1u << j) - 1u)) == r);
            int pick = __builtin_ctz(group_bits<GL>(mine, g));
            asm("" : "+v"(pick));  // taken here, before the branch below
            if (t <= sch.T) {
                const bool neg = (M >> pick) & 1u;
                const int sm = neg ? -1 : 1;  // old s_pick
                const int k2 = neg ? 2 : -2;  // -2 s_pick(old)
                const int k4 = neg ? 4 : -4;
                M ^= 1u << pick;
                // E changes by 4 (N - 1 + m); every energy of a walk is the
                // same modulo 4, so the threshold moves by N - 1 + m exactly
                E += 4 * (N - 1 + m);
                thr -= N - 1 + m;
                if (E < bestE) {
                    bestE = E;
                    best = M;
                    thr = -(N - 1);
                }
                if constexpr (TRACE) {
                    if (j == 0) a.trace[w * (int64_t)a.trace_stride + t - 1] = (int16_t)pick;
                }
                // as in the lag form: q = 2j - pick is the other end of lag
                // |pick - j| of row j; C_k -= 2 s_pick(old) t_pick,k from row
                // pick, which the move leaves unchanged; lane pick stores the
                // new s_pick into SP[pick] after every read of it
                const uint32_t qa = spj - (uint32_t)pick;
                int sq = lds_load_i8(qa);
                asm("" : "+v"(sq));  // one sign-extending load
                const int tpk = ((const int8_t *)rows)[__umul24(kGroupRow, pick) + j];
                C += __mul24(k2, tpk);  // 24-bit products: full-rate multiply-adds
                CB[j] = (int8_t)C;
                u2 += __mul24(k4, sq);
                lds_store_i8(absdiff_add_v((uint32_t)pick, (uint32_t)j, rowm1), sq - sm);
                if (j == pick) {
                    lds_store_i8(qa, ns);
                    ns = -ns;
                    u2 += 4;
                    tabu = tabu_new;
                }
            }
            wave_sync();
#pragma unroll
            for (int r = 0; r < NB; ++r) tc[r] = ((const uint4 *)(rows + kGroupRow * j))[r];
        }
    }
    if (live) {
        int8_t *out = a.best_seq + w * (int64_t)a.out_stride;
        for (int i = j; i < a.out_stride; i += GL)
            out[i] = i < N ? (((best >> i) & 1u) ? (int8_t)-1 : (int8_t)1) : (int8_t)0;
        if (j == 0) {
            a.best_e[w] = bestE;
            a.final_e[w] = E;
        }
    }
}

// Walks of N <= 64 / G at positions [begin, end), G per wavefront and WAVES
// wavefronts per workgroup.  PERSIST: a grid sized to the device takes G
// positions at a time from the queue head `counter`; otherwise one
// wavefront per G positions.
template <int G, int WAVES, bool PERSIST, bool TRACE>
__global__ __launch_bounds__(64 * WAVES) void tabu_kernel_group(TabuLaunchArgs a, int64_t begin,
                                                                int64_t end, uint32_t *counter) {
    __shared__ __attribute__((aligned(16))) uint8_t lds_all[WAVES][G * GroupLds<64 / G>::BYTES];
    uint8_t *lds = lds_all[threadIdx.x >> 6];
    if constexpr (PERSIST) {
        for (int64_t pos = begin + next_work(counter, G); pos < end;
             pos = begin + next_work(counter, G))
            run_group_walks<G, TRACE>(a, pos, end, lds);
    } else {
        const int64_t pos = begin + ((int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6)) * G;
        if (pos < end) run_group_walks<G, TRACE>(a, pos, end, lds);
    }
}

// Walks at positions [begin, end) of the processing order, all of one length
// class: NW neighbours per lane (N <= 64 NW) and windows of NB chunks
// (N - 1 <= 16 NB).  PERSIST: a grid sized to the device drains the range
// through the queue head `counter`; otherwise one wave per position.
// TRACE: record every walk's moves (a separate instantiation, so that the
// untraced kernel does not carry the registers of the traced one).
template <int NW, int NB, int WPG, bool PERSIST, bool TRACE, bool LAG = (NW == 1)>
__global__ __launch_bounds__(64 * WPG) void tabu_kernel(TabuLaunchArgs a, int64_t begin,
                                                        int64_t end, uint32_t *counter) {
    __shared__ __attribute__((aligned(16))) uint8_t lds_all[WPG][walk_lds_bytes<NW, LAG>()];
    const int wave = threadIdx.x >> 6;
    uint8_t *lds = lds_all[wave];
    if constexpr (PERSIST) {
        for (int64_t pos = begin + next_work(counter); pos < end;
             pos = begin + next_work(counter)) {
            const int64_t w = a.order ? (int64_t)a.order[pos] : pos;
            run_tabu_item<NW, NB, TRACE, LAG>(a, w, a.ns ? a.ns[w] : a.n_uniform, lds);
        }
    } else {
        const int64_t pos = begin + (int64_t)blockIdx.x * WPG + wave;
        if (pos < end) {
            const int64_t w = a.order ? (int64_t)a.order[pos] : pos;
            run_tabu_item<NW, NB, TRACE, LAG>(a, w, a.ns ? a.ns[w] : a.n_uniform, lds);
        }
    }
}

// Walks of 64 < N <= 128 at positions [begin, end), one per 128-lane
// workgroup of two wavefronts (the walk's barriers are the workgroup's).
// Each walk spans the fewest 16-lag chunks that hold its N - 1 lags.  The
// persistent form: wavefront 0 takes the next position from the queue and
// hands it to wavefront 1 through LDS, so both run the same walk and reach
// the same barriers, and both leave when the queue is drained.
template <bool TRACE, bool LAG>
__device__ __forceinline__ void run_split_range_item(const TabuLaunchArgs &a, int64_t pos,
                                                     uint8_t *lds, int part) {
    const int64_t w = a.order ? (int64_t)a.order[pos] : pos;
    const int N = __builtin_amdgcn_readfirstlane(a.ns ? a.ns[w] : a.n_uniform);
    if (N > 113)
        run_split_item<8, TRACE, LAG>(a, w, N, lds, part);
    else if (N > kClassMaxN[3])
        run_split_item<7, TRACE, LAG>(a, w, N, lds, part);
    else if (N > 81)
        run_split_item<6, TRACE, LAG>(a, w, N, lds, part);
    else
        run_split_item<5, TRACE, LAG>(a, w, N, lds, part);
}

template <bool PERSIST, bool TRACE, bool LAG>
__global__ __launch_bounds__(128) void tabu_kernel_split(TabuLaunchArgs a, int64_t begin,
                                                         int64_t end, uint32_t *counter) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[walk_lds_bytes<2, LAG>()];
    __shared__ int64_t shared_pos;
    const int part = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if constexpr (PERSIST) {
        for (;;) {
            if (part == 0) {
                const int64_t p = begin + next_work(counter);
                shared_pos = p;  // uniform value, every lane of wavefront 0
            }
            __syncthreads();
            const int64_t pos = (int64_t)__builtin_amdgcn_readfirstlane((int)(shared_pos - begin)) + begin;
            __syncthreads();  // both have read before wavefront 0 writes again
            if (pos >= end) break;
            run_split_range_item<TRACE, LAG>(a, pos, lds, part);
        }
    } else {
        const int64_t pos = begin + (int64_t)blockIdx.x;
        if (pos < end) run_split_range_item<TRACE, LAG>(a, pos, lds, part);
    }
}

// Walks of the classes with N <= 128 (processing-order positions from
// class_end[1] on) in one launch: each wavefront runs the
// instantiation of its own walk's class, in LDS scratch sized for the
// largest of them.  One launch on the caller's stream spares a batch of
// several such classes the fork to side streams and the join back, whose
// event waits cost tens of microseconds per call, and drains the whole
// longest-first order at once.
constexpr int kMixedLds = walk_lds_bytes<2>() > walk_lds_bytes<1>() ? walk_lds_bytes<2>()
                                                                    : walk_lds_bytes<1>();

template <bool TRACE, bool LAG>
__device__ __forceinline__ void run_mixed_item(const TabuLaunchArgs &a, int64_t w, uint8_t *lds) {
    // windows of the fewest 16-lag chunks that hold N - 1 lags (within the
    // launch, finer steps than the classes cost only code)
    const int N = __builtin_amdgcn_readfirstlane(a.ns ? a.ns[w] : a.n_uniform);
    if (N > 113)
        run_tabu_item<2, 8, TRACE, LAG>(a, w, N, lds);
    else if (N > kClassMaxN[3])
        run_tabu_item<2, 7, TRACE, LAG>(a, w, N, lds);
    else if (N > 81)
        run_tabu_item<2, 6, TRACE, LAG>(a, w, N, lds);
    else if (N > kClassMaxN[4])
        run_tabu_item<2, 5, TRACE, LAG>(a, w, N, lds);
    else if (N > kClassMaxN[5])
        run_tabu_item<1, 4, TRACE>(a, w, N, lds);
    else if (N > kClassMaxN[6])
        run_tabu_item<1, 3, TRACE>(a, w, N, lds);
    else if (N > kClassMaxN[7])
        run_tabu_item<1, 2, TRACE>(a, w, N, lds);
    else
        run_tabu_item<1, 1, TRACE>(a, w, N, lds);
}

// Walks of N > 128 (classes 0 and 1, positions [0, class_end[1])) in one
// launch, for the same reason; all take four neighbours per lane, so they
// share one LDS layout, and each walk again spans the fewest chunks that
// hold its N - 1 lags.
template <bool TRACE>
__device__ __forceinline__ void run_mixed_long_item(const TabuLaunchArgs &a, int64_t w,
                                                    uint8_t *lds) {
    const int N = __builtin_amdgcn_readfirstlane(a.ns ? a.ns[w] : a.n_uniform);
    if (N > kClassMaxN[1])
        run_tabu_item<4, 16, TRACE>(a, w, N, lds);
    else
        run_tabu_item<4, 12, TRACE>(a, w, N, lds);
}

template <bool TRACE, bool LONG, bool LAG>
__device__ __forceinline__ void run_mixed_range_item(const TabuLaunchArgs &a, int64_t pos,
                                                     uint8_t *lds) {
    const int64_t w = a.order ? (int64_t)a.order[pos] : pos;
    if constexpr (LONG)
        run_mixed_long_item<TRACE>(a, w, lds);
    else
        run_mixed_item<TRACE, LAG>(a, w, lds);
}

// LONG selects the N > 128 range (four wavefronts per SIMD is a hint for the
// short range only, whose default launch is one walk per workgroup).
template <int WPG, bool PERSIST, bool TRACE, bool LONG, bool LAG>
__global__ __launch_bounds__(64 * WPG) __attribute__((amdgpu_waves_per_eu(WPG == 1 && !PERSIST && !LONG && !LAG ? 4 : 1))) void tabu_kernel_mixed(TabuLaunchArgs a, int64_t begin,
                                                              int64_t end, uint32_t *counter) {
    constexpr int kLds = LONG ? walk_lds_bytes<4>()
                              : (LAG ? (walk_lds_bytes<2, true>() > walk_lds_bytes<1>()
                                            ? walk_lds_bytes<2, true>()
                                            : walk_lds_bytes<1>())
                                     : kMixedLds);
    __shared__ __attribute__((aligned(16))) uint8_t lds_all[WPG][kLds];
    const int wave = threadIdx.x >> 6;
    uint8_t *lds = lds_all[wave];
    if constexpr (PERSIST) {
        for (int64_t pos = begin + next_work(counter); pos < end;
             pos = begin + next_work(counter))
            run_mixed_range_item<TRACE, LONG, LAG>(a, pos, lds);
    } else {
        const int64_t pos = begin + (int64_t)blockIdx.x * WPG + wave;
        if (pos < end) run_mixed_range_item<TRACE, LONG, LAG>(a, pos, lds);
    }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Processing order of W walks, longest first, from their lengths in device
// memory (LABS_MIN_N <= ns[w] <= LABS_MAX_N, checked by the host): one
// workgroup counts the lengths in LDS, turns the counts into the first
// position of each length (descending N), then every walk takes the next
// position of its length.  Walks of one length land in an order that
// depends on the atomics' timing; results do not depend on the order.
constexpr int kOrderThreads = 1024;
__global__ __launch_bounds__(kOrderThreads) void order_by_length_kernel(
    const int32_t *__restrict__ ns, int64_t W, int32_t *__restrict__ order) {
    __shared__ int32_t next[LABS_MAX_N + 1];
    for (int n = threadIdx.x; n <= LABS_MAX_N; n += kOrderThreads) next[n] = 0;
    __syncthreads();
    for (int64_t w = threadIdx.x; w < W; w += kOrderThreads) atomicAdd(&next[ns[w]], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t pos = 0;
        for (int n = LABS_MAX_N; n >= 0; --n) {
            const int32_t c = next[n];
            next[n] = pos;
            pos += c;
        }
    }
    __syncthreads();
    for (int64_t w = threadIdx.x; w < W; w += kOrderThreads)
        order[atomicAdd(&next[ns[w]], 1)] = (int32_t)w;
}

// Scratch of the allocation-free tabu batch: the queue heads
// (kNoAllocHeadBytes), then the per-walk lengths and the processing order
// (kNoAllocMaxWalks int32 each).  Each device holds its own copy for the
// life of the process; host code reaches it only through the address
// returned by noalloc_scratch_address, never through this name.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

}  // namespace

hipError_t noalloc_scratch_address(int device, void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        // the caller has made `device` current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_order_by_length(const int32_t *ns, int64_t W, int32_t *order, hipStream_t s) {
    if (W <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_by_length_kernel, dim3(1), dim3(kOrderThreads), 0, s, ns, W, order);
    return hipGetLastError();
}

namespace {

// Work-items of one launch at most (a grid's x extent in work-items is a
// 32-bit count): a grid of one workgroup per few positions that would pass
// it runs as consecutive launches over sub-ranges of the positions.
constexpr int64_t kMaxLaunchItems = int64_t(1) << 30;

// launch(b, e, grid) for consecutive sub-ranges [b, e) of [begin, end), with
// `per_group` positions per workgroup of `lanes` lanes.
template <typename F>
hipError_t launch_in_ranges(int64_t begin, int64_t end, int per_group, int lanes, F &&launch) {
    const int64_t step = kMaxLaunchItems / lanes * per_group;
    for (int64_t b = begin; b < end; b += step) {
        const int64_t e = std::min(end, b + step);
        launch(b, e, (unsigned)((e - b + per_group - 1) / per_group));
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_energy(const int8_t *seqs, const int32_t *ns, int32_t n_uniform,
                         int32_t stride, int64_t count, int32_t *out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    constexpr int WPG = 4;
    return launch_in_ranges(0, count, WPG, 64 * WPG, [&](int64_t b, int64_t e, unsigned grid) {
        hipLaunchKernelGGL(energy_kernel<WPG>, dim3(grid), dim3(64 * WPG), 0, s,
                           seqs + b * (int64_t)stride, ns ? ns + b : nullptr, n_uniform, stride,
                           e - b, out + b);
    });
}

namespace {

template <int NW, int NB, int WPG, bool TRACE, bool LAG>
hipError_t launch_tabu_part_t(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                              uint32_t *counter, hipStream_t s) {
    if (groups > 0) {
        hipError_t e = launch_fill_u32(counter, 0u, 1, s);
        if (e != hipSuccess) return e;
        const int64_t need = (end - begin + WPG - 1) / WPG;
        hipLaunchKernelGGL((tabu_kernel<NW, NB, WPG, true, TRACE, LAG>),
                           dim3((unsigned)std::min<int64_t>(groups, need)), dim3(64 * WPG), 0, s, a,
                           begin, end, counter);
    } else {
        return launch_in_ranges(begin, end, WPG, 64 * WPG, [&](int64_t b, int64_t e, unsigned grid) {
            hipLaunchKernelGGL((tabu_kernel<NW, NB, WPG, false, TRACE, LAG>), dim3(grid),
                               dim3(64 * WPG), 0, s, a, b, e, counter);
        });
    }
    return hipGetLastError();
}

template <int NW, int NB, int WPG, bool LAG = (NW == 1)>
hipError_t launch_tabu_part(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                            uint32_t *counter, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    return a.trace != nullptr
               ? launch_tabu_part_t<NW, NB, WPG, true, LAG>(a, begin, end, groups, counter, s)
               : launch_tabu_part_t<NW, NB, WPG, false, LAG>(a, begin, end, groups, counter, s);
}

template <int WPG, bool TRACE, bool LONG, bool LAG>
hipError_t launch_mixed_t(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                          uint32_t *counter, hipStream_t s) {
    if (groups > 0) {
        hipError_t e = launch_fill_u32(counter, 0u, 1, s);
        if (e != hipSuccess) return e;
        const int64_t need = (end - begin + WPG - 1) / WPG;
        hipLaunchKernelGGL((tabu_kernel_mixed<WPG, true, TRACE, LONG, LAG>),
                           dim3((unsigned)std::min<int64_t>(groups, need)), dim3(64 * WPG), 0, s, a,
                           begin, end, counter);
    } else {
        return launch_in_ranges(begin, end, WPG, 64 * WPG, [&](int64_t b, int64_t e, unsigned grid) {
            hipLaunchKernelGGL((tabu_kernel_mixed<WPG, false, TRACE, LONG, LAG>), dim3(grid),
                               dim3(64 * WPG), 0, s, a, b, e, counter);
        });
    }
    return hipGetLastError();
}

template <int WPG, bool LONG, bool LAG>
hipError_t launch_mixed(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                        uint32_t *counter, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    return a.trace != nullptr
               ? launch_mixed_t<WPG, true, LONG, LAG>(a, begin, end, groups, counter, s)
               : launch_mixed_t<WPG, false, LONG, LAG>(a, begin, end, groups, counter, s);
}

template <bool TRACE, bool LAG>
hipError_t launch_split_t(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                          uint32_t *counter, hipStream_t s) {
    if (groups > 0) {
        hipError_t e = launch_fill_u32(counter, 0u, 1, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((tabu_kernel_split<true, TRACE, LAG>),
                           dim3((unsigned)std::min<int64_t>(groups, end - begin)), dim3(128), 0, s,
                           a, begin, end, counter);
    } else {
        return launch_in_ranges(begin, end, 1, 128, [&](int64_t b, int64_t e, unsigned grid) {
            hipLaunchKernelGGL((tabu_kernel_split<false, TRACE, LAG>), dim3(grid), dim3(128), 0, s,
                               a, b, e, counter);
        });
    }
    return hipGetLastError();
}

template <bool LAG>
hipError_t launch_split(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                        uint32_t *counter, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    return a.trace != nullptr ? launch_split_t<true, LAG>(a, begin, end, groups, counter, s)
                              : launch_split_t<false, LAG>(a, begin, end, groups, counter, s);
}

template <int G, int WAVES, bool TRACE>
hipError_t launch_group_t(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                          uint32_t *counter, hipStream_t s) {
    const int64_t need = (end - begin + G * WAVES - 1) / (G * WAVES);
    if (groups > 0) {
        hipError_t e = launch_fill_u32(counter, 0u, 1, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((tabu_kernel_group<G, WAVES, true, TRACE>),
                           dim3((unsigned)std::min<int64_t>(groups, need)), dim3(64 * WAVES), 0, s,
                           a, begin, end, counter);
    } else {
        return launch_in_ranges(begin, end, G * WAVES, 64 * WAVES,
                                [&](int64_t b, int64_t e, unsigned grid) {
            hipLaunchKernelGGL((tabu_kernel_group<G, WAVES, false, TRACE>), dim3(grid),
                               dim3(64 * WAVES), 0, s, a, b, e, counter);
        });
    }
    return hipGetLastError();
}

template <int G, int WAVES>
hipError_t launch_group(const TabuLaunchArgs &a, int64_t begin, int64_t end, int groups,
                        uint32_t *counter, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    if constexpr (WAVES > 2) {
        return hipErrorInvalidValue;  // 32 or 16 lanes per walk: 64- or 128-lane workgroups
    } else {
        return a.trace != nullptr
                   ? launch_group_t<G, WAVES, true>(a, begin, end, groups, counter, s)
                   : launch_group_t<G, WAVES, false>(a, begin, end, groups, counter, s);
    }
}

// One launch per launch group (walk_launch_groups), group g on streams[g]
// with the queue head of its first class (32 words apart).
template <int WPG, bool LAG>
hipError_t launch_tabu_wpg(const TabuLaunchArgs &a, const WalkLaunch &l, const hipStream_t *st) {
    static_assert(kWalkClasses == 8, "one launcher per class below");
    const int64_t *ce = a.class_end;
    const WalkGroups wg = walk_launch_groups(ce, l.split, l.lanes);
    hipError_t e = hipSuccess;
    for (int g = 0; g < wg.n && e == hipSuccess; ++g) {
        const int f = wg.first[g], z = wg.last[g], kind = wg.kind[g];
        const int64_t begin = f ? ce[f - 1] : 0, end = ce[z];
        uint32_t *q = a.counter + 32 * f;
        const int groups = kind == kKindSplit ? l.split_groups : l.groups;
        if (kind == kKindGroup2)
            e = launch_group<2, WPG>(a, begin, end, groups, q, st[g]);
        else if (kind == kKindGroup4)
            e = launch_group<4, WPG>(a, begin, end, groups, q, st[g]);
        else if (kind == kKindSplit)
            e = launch_split<LAG>(a, begin, end, groups, q, st[g]);
        else if (f == 0 && z == 1)
            e = launch_mixed<WPG, true, false>(a, begin, end, groups, q, st[g]);
        else if (f == 0)
            e = launch_tabu_part<4, 16, WPG>(a, begin, end, groups, q, st[g]);
        else if (f == 1)
            e = launch_tabu_part<4, 12, WPG>(a, begin, end, groups, q, st[g]);
        else if (z > f)  // several classes of N <= 128 in one launch
            e = launch_mixed<WPG, false, LAG>(a, begin, end, groups, q, st[g]);
        else if (f == 2)
            e = launch_tabu_part<2, 8, WPG, LAG>(a, begin, end, groups, q, st[g]);
        else if (f == 3)
            e = launch_tabu_part<2, 6, WPG, LAG>(a, begin, end, groups, q, st[g]);
        else if (f == 4)
            e = launch_tabu_part<1, 4, WPG>(a, begin, end, groups, q, st[g]);
        else if (f == 5)
            e = launch_tabu_part<1, 3, WPG>(a, begin, end, groups, q, st[g]);
        else if (f == 6)
            e = launch_tabu_part<1, 2, WPG>(a, begin, end, groups, q, st[g]);
        else
            e = launch_tabu_part<1, 1, WPG>(a, begin, end, groups, q, st[g]);
    }
    return e;
}

}  // namespace

hipError_t launch_tabu(const TabuLaunchArgs &a, const WalkLaunch &l, const hipStream_t *streams) {
    if (a.W <= 0) return hipSuccess;
    // every launch range lies inside the processing order [0, W)
    int64_t prev = 0;
    for (int c = 0; c < kWalkClasses; ++c) {
        if (a.class_end[c] < prev || a.class_end[c] > a.W) return hipErrorInvalidValue;
        prev = a.class_end[c];
    }
    if (prev != a.W) return hipErrorInvalidValue;
    switch (l.waves_per_group * 2 + (l.lag ? 1 : 0)) {
    case 2: return launch_tabu_wpg<1, false>(a, l, streams);
    case 3: return launch_tabu_wpg<1, true>(a, l, streams);
    case 4: return launch_tabu_wpg<2, false>(a, l, streams);
    case 5: return launch_tabu_wpg<2, true>(a, l, streams);
    case 8: return launch_tabu_wpg<4, false>(a, l, streams);
    case 9: return launch_tabu_wpg<4, true>(a, l, streams);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t grid = (count + 255) / 256;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)grid), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

}  // namespace liblabs
