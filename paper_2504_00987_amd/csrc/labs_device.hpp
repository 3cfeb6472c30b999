// Device building blocks of liblabs (gfx950): counter-based RNG, wavefront
// primitives, 128-bit sequence masks and the bit-sliced tabu walk.
//
// One tabu walk (Alg. 2 / Alg. 4 of arXiv:2504.00987) runs on one 64-lane
// wavefront.  The sequence is a wave-uniform bit mask (bit i set <=> s_i = -1)
// held in scalar registers; lane l owns neighbour j = l (and j = l + 64 when
// N > 64) and lag k = l + 1 (and k = l + 65).  The autocorrelation table C_k
// (Eq. 1) lives one entry per lane and is exposed to every lane as eight
// wave-uniform bit planes (two's complement, built with ballots), so the
// score of neighbour j,
//
//     dE_j = 4 * ( sum_k t_jk^2  -  s_j * sum_k t_jk C_k ),
//     t_jk = s_{j+k} + s_{j-k}   (terms outside the sequence are 0),
//
// is evaluated with AND + popcount over 64-bit words instead of one
// multiply-add per lag: sum_k t_jk C_k = PS(N-1-j) + PS(j)
// - 2 * sum_p w_p * popcount((R_j | L_j) & plane_p), with R_j / L_j the
// neighbour's right / left windows of set bits, PS the prefix sums of C and
// w_p the plane weights.  Planes that only repeat the sign bit are skipped.
// The flip of s_j changes C_k by -2 s_j t_jk (the paper's O(N) "one row and
// column" update of Sec. III.C), applied lane-parallel.  All arithmetic is
// exact int32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <limits.h>

#include "labs_internal.h"

namespace liblabs {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// ---------------------------------------------------------------------------
enum : uint32_t {
    kTagStart = 1,  // random start of a stand-alone walk
    kTagStep = 2,   // per tabu step: tie-break word 0, tenure word 1
    kTagLen = 3,    // per walk: random walk length, word 0
    kTagInit = 4,   // per population member: initial sequence
    kTagGen = 5,    // per generation: crossover, parents, cut, replacement
    kTagMut = 6     // per generation: mutation words
};

struct Draw4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Draw4 philox10(uint32_t x0, uint32_t x1, uint32_t x2,
                                          uint32_t x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a0 = x0, a2 = x2;
        x0 = __umulhi(0xCD9E8D57u, a2) ^ x1 ^ k0;
        x2 = __umulhi(0xD2511F53u, a0) ^ x3 ^ k1;
        x1 = 0xCD9E8D57u * a2;
        x3 = 0xD2511F53u * a0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {x0, x1, x2, x3};
}

// Uniform integer in [0, range) from a 32-bit word: (u * range) >> 32.
__device__ __forceinline__ uint32_t below(uint32_t u, uint32_t range) {
    return __umulhi(u, range);
}

// ---------------------------------------------------------------------------
// Wavefront primitives (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int rank_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int readlane(int v, int l) {
    return __builtin_amdgcn_readlane(v, l);
}

__device__ __forceinline__ uint32_t readlane_u(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// A wave-uniform 64-bit value, read from the first lane into scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Orders this wavefront's LDS accesses across lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP controls (GFX9 encoding).
#define LABS_DPP_QUAD_1032 0xB1
#define LABS_DPP_QUAD_2301 0x4E
#define LABS_DPP_ROW_SHR(n) (0x110 + (n))
#define LABS_DPP_ROW_MIRROR 0x140
#define LABS_DPP_ROW_HALF_MIRROR 0x141
#define LABS_DPP_ROW_BCAST15 0x142
#define LABS_DPP_ROW_BCAST31 0x143

// Minimum over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ int wave_min(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, LABS_DPP_QUAD_1032, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, LABS_DPP_QUAD_2301, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, LABS_DPP_ROW_HALF_MIRROR, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, LABS_DPP_ROW_MIRROR, 0xf, 0xf, false));
    const int a = readlane(v, 0), b = readlane(v, 16), c = readlane(v, 32), d = readlane(v, 48);
    return min(min(a, b), min(c, d));
}

// Bitwise OR over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ int wave_or(int v) {
    v |= __builtin_amdgcn_update_dpp(0, v, LABS_DPP_QUAD_1032, 0xf, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0, v, LABS_DPP_QUAD_2301, 0xf, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_HALF_MIRROR, 0xf, 0xf, false);
    v |= __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_MIRROR, 0xf, 0xf, false);
    return readlane(v, 0) | readlane(v, 16) | readlane(v, 32) | readlane(v, 48);
}

// Sum over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_QUAD_1032, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_QUAD_2301, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_HALF_MIRROR, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_MIRROR, 0xf, 0xf, false);
    return readlane(v, 0) + readlane(v, 16) + readlane(v, 32) + readlane(v, 48);
}

// Inclusive prefix sum over lanes 0..63 (lane l receives v_0 + ... + v_l).
__device__ __forceinline__ int wave_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_SHR(1), 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_SHR(2), 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_SHR(4), 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_SHR(8), 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_BCAST15, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_BCAST31, 0xc, 0xf, false);
    return v;
}

// ---------------------------------------------------------------------------
// Sequence masks: 64-bit for N <= 64, 128-bit for N <= 128.
// ---------------------------------------------------------------------------
struct M128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ uint64_t m_and(uint64_t a, uint64_t b) { return a & b; }
__device__ __forceinline__ uint64_t m_or(uint64_t a, uint64_t b) { return a | b; }
__device__ __forceinline__ uint64_t m_xor(uint64_t a, uint64_t b) { return a ^ b; }
__device__ __forceinline__ uint64_t m_not(uint64_t a) { return ~a; }
__device__ __forceinline__ bool m_eq(uint64_t a, uint64_t b) { return a == b; }
__device__ __forceinline__ int m_popc(uint64_t a) { return __popcll(a); }
// a >> sh for 0 <= sh <= 64 (64 gives 0).
__device__ __forceinline__ uint64_t m_shr(uint64_t a, int sh) {
    return sh >= 64 ? 0ull : (a >> sh);
}
// Bits [0, n) set, 0 <= n <= 64.
__device__ __forceinline__ uint64_t m_low(uint64_t, int n) {
    return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}
__device__ __forceinline__ int m_bit(uint64_t a, int i) { return (int)((a >> i) & 1ull); }
__device__ __forceinline__ uint64_t m_onebit(uint64_t, int i) { return 1ull << i; }

__device__ __forceinline__ M128 m_and(M128 a, M128 b) { return {a.lo & b.lo, a.hi & b.hi}; }
__device__ __forceinline__ M128 m_or(M128 a, M128 b) { return {a.lo | b.lo, a.hi | b.hi}; }
__device__ __forceinline__ M128 m_xor(M128 a, M128 b) { return {a.lo ^ b.lo, a.hi ^ b.hi}; }
__device__ __forceinline__ M128 m_not(M128 a) { return {~a.lo, ~a.hi}; }
__device__ __forceinline__ bool m_eq(M128 a, M128 b) { return a.lo == b.lo && a.hi == b.hi; }
__device__ __forceinline__ int m_popc(M128 a) { return __popcll(a.lo) + __popcll(a.hi); }
// a >> sh for 0 <= sh <= 128.
__device__ __forceinline__ M128 m_shr(M128 a, int sh) {
    M128 r;
    if (sh >= 64) {
        r.lo = sh >= 128 ? 0ull : (a.hi >> (sh - 64));
        r.hi = 0ull;
    } else if (sh == 0) {
        r = a;
    } else {
        r.lo = (a.lo >> sh) | (a.hi << (64 - sh));
        r.hi = a.hi >> sh;
    }
    return r;
}
__device__ __forceinline__ M128 m_low(M128, int n) {
    M128 r;
    if (n >= 128) {
        r.lo = ~0ull; r.hi = ~0ull;
    } else if (n >= 64) {
        r.lo = ~0ull; r.hi = (1ull << (n - 64)) - 1ull;
    } else {
        r.lo = (1ull << n) - 1ull; r.hi = 0ull;
    }
    return r;
}
__device__ __forceinline__ int m_bit(M128 a, int i) {
    return i < 64 ? (int)((a.lo >> i) & 1ull) : (int)((a.hi >> (i - 64)) & 1ull);
}
__device__ __forceinline__ M128 m_onebit(M128, int i) {
    M128 r;
    r.lo = i < 64 ? (1ull << i) : 0ull;
    r.hi = i < 64 ? 0ull : (1ull << (i - 64));
    return r;
}

template <int NW> struct MaskOf;
template <> struct MaskOf<1> { using type = uint64_t; };
template <> struct MaskOf<2> { using type = M128; };

__device__ __forceinline__ uint64_t mask_from(uint64_t lo, uint64_t) { return lo; }
__device__ __forceinline__ M128 mask_from(uint64_t lo, uint64_t hi, M128) { return {lo, hi}; }
__device__ __forceinline__ uint64_t mask_lo(uint64_t a) { return a; }
__device__ __forceinline__ uint64_t mask_hi(uint64_t) { return 0ull; }
__device__ __forceinline__ uint64_t mask_lo(M128 a) { return a.lo; }
__device__ __forceinline__ uint64_t mask_hi(M128 a) { return a.hi; }

// Half-width companion of a mask (the shorter window of a neighbour).
template <int NW> struct SmallOf;
template <> struct SmallOf<1> { using type = uint32_t; };
template <> struct SmallOf<2> { using type = uint64_t; };

__device__ __forceinline__ uint32_t low_half(uint64_t a) { return (uint32_t)a; }
__device__ __forceinline__ uint64_t low_half(M128 a) { return a.lo; }
__device__ __forceinline__ int s_popc(uint32_t a) { return __popc(a); }
__device__ __forceinline__ int s_popc(uint64_t a) { return __popcll(a); }
// Bits [0, n) of a half-width word, 0 <= n < its width.
__device__ __forceinline__ uint32_t s_low(uint32_t, int n) { return (1u << n) - 1u; }
__device__ __forceinline__ uint64_t s_low(uint64_t, int n) { return (1ull << n) - 1ull; }

// acc + popcount(big & plane) + popcount(small & low half of plane), as a
// chain of popcount-accumulate operations.
__device__ __forceinline__ int plane_count(uint64_t big, uint32_t small, uint64_t P, int acc) {
    acc = __popc(small & (uint32_t)P) + acc;
    acc = __popc((uint32_t)(big >> 32) & (uint32_t)(P >> 32)) + acc;
    return __popc((uint32_t)big & (uint32_t)P) + acc;
}
__device__ __forceinline__ int plane_count(M128 big, uint64_t small, M128 P, int acc) {
    acc = __popc((uint32_t)small & (uint32_t)P.lo) + acc;
    acc = __popc((uint32_t)(small >> 32) & (uint32_t)(P.lo >> 32)) + acc;
    acc = __popc((uint32_t)big.hi & (uint32_t)P.hi) + acc;
    acc = __popc((uint32_t)(big.hi >> 32) & (uint32_t)(P.hi >> 32)) + acc;
    acc = __popc((uint32_t)(big.lo >> 32) & (uint32_t)(P.lo >> 32)) + acc;
    return __popc((uint32_t)big.lo & (uint32_t)P.lo) + acc;
}

template <int NW>
__device__ __forceinline__ typename MaskOf<NW>::type make_mask(uint64_t lo, uint64_t hi) {
    if constexpr (NW == 1) {
        return lo;
    } else {
        return M128{lo, hi};
    }
}

// ---------------------------------------------------------------------------
// Walk schedule: maxIter and the tenure range.
// ---------------------------------------------------------------------------
struct Schedule {
    int T, lo, hi;
};

__device__ __forceinline__ Schedule make_schedule(const RuleParams &r, int N, uint32_t k0,
                                                  uint32_t k1, uint32_t entity, uint32_t gen) {
    Schedule s;
    if (r.steps_rule == 0) {
        s.T = r.steps_a;
    } else if (r.steps_rule == 1) {
        s.T = r.steps_a * N;
    } else {
        const Draw4 d = philox10(entity, gen, 0u, kTagLen, k0, k1);
        s.T = N / 2 + (int)below(d.w0, (uint32_t)(N + 1));
    }
    if (r.tenure_rule == 0) {
        s.lo = r.lo_num * N / r.lo_den + r.lo_add;
        s.hi = r.hi_num * N / r.hi_den + r.hi_add;
    } else {
        s.lo = s.T / 10;
        s.hi = 3 * s.T / 25;
    }
    return s;
}

// ---------------------------------------------------------------------------
// Energy of a sequence mask, computed by the whole wavefront (lane l owns
// lags l+1 and l+65): C_k = (N-k) - 2 * popcount((M ^ (M >> k)) & low(N-k)).
// ---------------------------------------------------------------------------
template <typename Mask>
__device__ __forceinline__ int lag_corr(Mask M, int N, int k) {
    return (N - k) - 2 * m_popc(m_and(m_xor(M, m_shr(M, k)), m_low(M, N - k)));
}

// Energy of one mask computed by a single lane (lane-serial, O(N) popcounts).
template <typename Mask>
__device__ __forceinline__ int lane_energy(Mask M, int N) {
    int e = 0;
    for (int k = 1; k < N; ++k) {
        const int c = lag_corr(M, N, k);
        e += c * c;
    }
    return e;
}

// ---------------------------------------------------------------------------
// The tabu walk.
// ---------------------------------------------------------------------------
template <int NW>
struct WalkResult {
    typename MaskOf<NW>::type best;
    int best_e;
    int final_e;
};

// Bit plane p of the lane-held table C (two's complement): bit k-1 is bit p
// of C_k.
template <int NW>
__device__ __forceinline__ typename MaskOf<NW>::type plane(const int (&C)[NW], int p) {
    const uint64_t lo = ballot(((C[0] >> p) & 1) != 0);
    uint64_t hi = 0ull;
    if constexpr (NW == 2) hi = ballot(((C[1] >> p) & 1) != 0);
    return make_mask<NW>(lo, hi);
}

// Number q of planes needed: every C_k lies in [-2^(q-1), 2^(q-1)), so the
// offset values C_k + 2^(q-1) are q-bit unsigned numbers.
template <int NW>
__device__ __forceinline__ int planes_needed(const int (&C)[NW]) {
    int x = C[0] ^ (C[0] >> 31);
    if constexpr (NW == 2) x |= C[1] ^ (C[1] >> 31);
    const int o = wave_or(x);
    return o == 0 ? 1 : 33 - __clz(o);
}

// Lane l receives bit l of a wave-uniform 64-bit mask.
__device__ __forceinline__ bool lane_bit(uint64_t mask) {
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// Runs one walk of sch.T steps from mask M0 (bits >= N must be clear).
//   ps     per-wavefront LDS scratch of 129 ints (prefix sums of C)
//   trace  optional: trace[t-1] = flipped index (written by lane 0)
// Every lane of the wavefront must call this with identical uniform inputs.
template <int NW>
__device__ __forceinline__ WalkResult<NW> tabu_walk(const int N, const typename MaskOf<NW>::type M0,
                                    const Schedule sch, const int aspiration,
                                    const uint32_t k0, const uint32_t k1,
                                    const uint32_t entity, const uint32_t gen,
                                    int *__restrict__ ps, int16_t *__restrict__ trace) {
    using Mask = typename MaskOf<NW>::type;
    using Small = typename SmallOf<NW>::type;
    const int lane = lane_id();
    // The sequence is wave-uniform; pinning it to scalar registers keeps the
    // per-move mask arithmetic on the scalar unit.
    Mask M = make_mask<NW>(uniform64(mask_lo(M0)), uniform64(mask_hi(M0)));

    // Reversed sequence: bit i of Mr is bit N-1-i of M.
    Mask Mr;
    {
        const uint64_t lo = ballot(lane < N && m_bit(M, N - 1 - lane));
        uint64_t hi = 0ull;
        if constexpr (NW == 2) hi = ballot(lane + 64 < N && m_bit(M, N - 65 - lane));
        Mr = make_mask<NW>(lo, hi);
    }

    // C_k for the lags this lane owns (Eq. 1) and the energy (Eq. 2).
    int C[NW];
    int sq = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int k = lane + 1 + 64 * w;
        C[w] = k < N ? lag_corr(M, N, k) : 0;
        sq += C[w] * C[w];
    }
    int E = wave_sum(sq);

    int tabu[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) tabu[w] = 0;
    Mask best = M;
    int bestE = E;

    ps[0] = 0;  // every lane stores the same value
    uint32_t dr0 = 0u, dr1 = 0u;

    for (int t = 1; t <= sch.T; ++t) {
        const int slot = (t - 1) & 63;
        if (slot == 0) {
            // draws for steps t .. t+63, one step per lane
            const Draw4 d = philox10(entity, gen, (uint32_t)(t + lane), kTagStep, k0, k1);
            dr0 = d.w0;
            dr1 = d.w1;
        }

        // Prefix sums PS(x) = sum_{k<=x} C_k, x = 0..N-1, into LDS.
        wave_sync();
        {
            const int s0 = wave_scan(C[0]);
            ps[1 + lane] = s0;
            if constexpr (NW == 2) {
                const int s1 = wave_scan(C[1]) + readlane(s0, 63);
                ps[65 + lane] = s1;
            }
        }
        wave_sync();

        // Score the neighbours this lane owns.  Neighbour j's right window
        // has N-1-j meaningful bits and its left window j; the longer one
        // ("big") needs the full mask width, the shorter ("small") at most
        // half of it, so each plane costs 3 (N <= 64) or 6 (N <= 128) words.
        // Lanes past the sequence compute on empty windows and are masked
        // out at the end, so the loop has no lane-dependent branch.
        Mask big[NW];
        Small small[NW];
        int bs[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int j = lane + 64 * w;
            const bool in = j < N;
            const Mask R = m_shr(M, j + 1);                  // bit k-1: s_{j+k} = -1
            const Mask L = m_shr(Mr, in ? N - j : 64 * NW);  // bit k-1: s_{j-k} = -1
            const bool right_big = N - 1 - j >= j;
            big[w] = right_big ? R : L;
            small[w] = low_half(right_big ? L : R);
            bs[w] = 0;
        }
        // Offset-binary planes: with D_k = C_k + 2^(q-1) in [0, 2^q),
        // sum_k x_k C_k = sum_p 2^p popc(x & plane_p(D)) - 2^(q-1) popc(x).
        const int q = planes_needed<NW>(C);
        const int off = 1 << (q - 1);
        int D[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) D[w] = C[w] + off;
#pragma unroll
        for (int p = 7; p >= 0; --p) {  // Horner: bs = 2 bs + count_p
            if (p < q) {
                const Mask P = plane<NW>(D, p);
#pragma unroll
                for (int w = 0; w < NW; ++w) bs[w] = plane_count(big[w], small[w], P, 2 * bs[w]);
            }
        }
#pragma unroll
        for (int w = 0; w < NW; ++w)  // bs = sum_k (bR_k + bL_k) C_k
            bs[w] -= off * (m_popc(big[w]) + s_popc(small[w]));
        int key[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int j = lane + 64 * w;
            const bool in = j < N;
            const int nb = in ? min(N - 1 - j, j) : 0;  // lags with both sides inside
            const int u = nb - 2 * s_popc((low_half(big[w]) ^ small[w]) & s_low(small[w], nb));
            const int v = ps[in ? N - 1 - j : 0] + ps[in ? j : 0] - 2 * bs[w];
            const int sj = 1 - 2 * m_bit(M, in ? j : 0);
            const int cand = E + 4 * (N - 1 + 2 * u - sj * v);
            const bool admissible = tabu[w] < t || (aspiration && cand < bestE);
            key[w] = in && admissible ? cand : INT_MAX;
        }

        // Admissible minimum, ties broken by the step's draw.
        int kmin = key[0];
        if constexpr (NW == 2) kmin = min(kmin, key[1]);
        const int m = wave_min(kmin);
        const uint64_t T0 = ballot(key[0] == m);
        uint64_t T1 = 0ull;
        if constexpr (NW == 2) T1 = ballot(key[1] == m);
        const int c0 = __popcll(T0);
        const int c = c0 + __popcll(T1);
        const uint32_t u0 = readlane_u(dr0, slot);
        const uint32_t u1 = readlane_u(dr1, slot);
        int r = (int)below(u0, (uint32_t)c);
        int pick;
        if (r < c0) {
            const uint64_t sel = ballot(lane_bit(T0) && rank_below(T0) == r);
            pick = __builtin_ctzll(sel);
        } else {
            r -= c0;
            const uint64_t sel = ballot(lane_bit(T1) && rank_below(T1) == r);
            pick = 64 + __builtin_ctzll(sel);
        }

        // Apply the move: tenure, sequence, energy, best.
        const int tenure = sch.lo + (int)below(u1, (uint32_t)(sch.hi - sch.lo + 1));
        tabu[0] = pick == lane ? t + tenure : tabu[0];
        if constexpr (NW == 2) tabu[1] = pick == lane + 64 ? t + tenure : tabu[1];
        const int sm = 1 - 2 * m_bit(M, pick);
        M = m_xor(M, m_onebit(M, pick));
        Mr = m_xor(Mr, m_onebit(Mr, N - 1 - pick));
        E = m;
        if (E < bestE) {
            bestE = E;
            best = M;
        }
        if (trace != nullptr) trace[t - 1] = (int16_t)pick;  // uniform store

        // C_k -= 2 s_pick t_pick,k for every lag (lane-parallel).  The
        // windows of the flipped index are wave-uniform: lag k (bit k-1) of
        // Rn / Ln says s_{pick+k} / s_{pick-k} = -1, of Rp / Lp that it is +1
        // (both clear past the ends, so lags >= N keep C_k = 0).
        {
            const Mask Rn = m_shr(M, pick + 1);
            const Mask Ln = m_shr(Mr, N - pick);
            const Mask Rp = m_and(m_low(M, N - 1 - pick), m_not(Rn));
            const Mask Lp = m_and(m_low(M, pick), m_not(Ln));
            const int k2 = -2 * sm;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint64_t rn = w == 0 ? mask_lo(Rn) : mask_hi(Rn);
                const uint64_t ln = w == 0 ? mask_lo(Ln) : mask_hi(Ln);
                const uint64_t rp = w == 0 ? mask_lo(Rp) : mask_hi(Rp);
                const uint64_t lp = w == 0 ? mask_lo(Lp) : mask_hi(Lp);
                const int sa = lane_bit(rn) ? -1 : (lane_bit(rp) ? 1 : 0);
                const int sb = lane_bit(ln) ? -1 : (lane_bit(lp) ? 1 : 0);
                C[w] += k2 * (sa + sb);
            }
        }
    }

    WalkResult<NW> res;
    res.best = best;
    res.best_e = bestE;
    res.final_e = E;
    return res;
}

}  // namespace liblabs
