// Device building blocks of liblabs (gfx950): counter-based RNG, wavefront
// primitives, sequence masks of up to 256 bits and the tabu walk.
//
// One tabu walk (Alg. 2 / Alg. 4 of arXiv:2504.00987) runs on one 64-lane
// wavefront (or two, for N <= 128 when few walks share the device).  The
// sequence is a wave-uniform bit mask (bit i set <=> s_i = -1) held in
// scalar registers; lane l owns neighbours j = l + 64h and lags k = j + 1.
// The score of neighbour j is
//
//     dE_j = 4 * ( sum_k t_jk^2  -  s_j * sum_k t_jk C_k ),
//     t_jk = s_{j+k} + s_{j-k}   (terms outside the sequence are 0),
//
// (flipping s_j changes C_k of Eq. 1 by -2 s_j t_jk), and sum_k t_jk^2 is
// N - 1 + 2 u_j with u_j = sum_k s_{j+k} s_{j-k}, which each lane keeps per
// neighbour: a move changes one of its terms.  sum_k t_jk C_k is a run of
// packed 4-way int8 dot products against C_k mirrored in LDS as int8 (as
// C_k >> 1 for N > 128, the parity part added from two wave-uniform sums).
// Two LDS layouts hold the t_jk:
//   lag form     row j holds t_j1 .. t_j64 (t_j128) as int8; a move rewrites
//                one byte per row (N <= 64, and N <= 128 where occupancy
//                does not depend on LDS);
//   record form  the sequence forwards (P) and reversed (Q) as 16-byte
//                records, record x holding bytes x .. x+15, so that every
//                lane's right window s_{j+1..} and left window s_{j-1..} is a
//                run of aligned 16-byte reads; a move rewrites one byte in
//                each of the 16 records that hold s_pick.
// After a move, C_k is updated lane-parallel (the paper's O(N) update of one
// "row and column", Sec. III.C).  All arithmetic is exact int32.
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
#define LABS_DPP_ROW_MIRROR 0x140
#define LABS_DPP_ROW_HALF_MIRROR 0x141
#define LABS_DPP_ROW_BCAST15 0x142
#define LABS_DPP_ROW_BCAST31 0x143

// Minimum over the 64 lanes, returned wave-uniform: row minima by DPP, then
// rows combined with the row broadcasts (lane 63 ends with the total).
__device__ __forceinline__ int wave_min(int v) {
    // the first four patterns give every lane a source: no fill value
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_QUAD_1032, 0xf, 0xf, true));
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_QUAD_2301, 0xf, 0xf, true));
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_ROW_HALF_MIRROR, 0xf, 0xf, true));
    v = min(v, __builtin_amdgcn_mov_dpp(v, LABS_DPP_ROW_MIRROR, 0xf, 0xf, true));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, LABS_DPP_ROW_BCAST15, 0xa, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, LABS_DPP_ROW_BCAST31, 0xc, 0xf, false));
    return readlane(v, 63);
}

// Sum over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_QUAD_1032, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_QUAD_2301, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_HALF_MIRROR, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, LABS_DPP_ROW_MIRROR, 0xf, 0xf, false);
    return readlane(v, 0) + readlane(v, 16) + readlane(v, 32) + readlane(v, 48);
}

// ---------------------------------------------------------------------------
// Sequence masks: 64-bit for N <= 64, 128-bit for N <= 128, 256-bit for
// N <= 256.
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
    return (int)(((i < 64 ? a.lo : a.hi) >> (i & 63)) & 1ull);
}
__device__ __forceinline__ M128 m_onebit(M128, int i) {
    const uint64_t b = 1ull << (i & 63);
    return {i < 64 ? b : 0ull, i < 64 ? 0ull : b};
}

// 256-bit masks for N <= 256 (four words, selected by value so that a
// variable word index never forces the mask out of registers).
struct M256 {
    uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ uint64_t m_word(const M256 &a, int i) {
    return i == 0 ? a.w0 : i == 1 ? a.w1 : i == 2 ? a.w2 : i == 3 ? a.w3 : 0ull;
}
__device__ __forceinline__ M256 m_and(M256 a, M256 b) {
    return {a.w0 & b.w0, a.w1 & b.w1, a.w2 & b.w2, a.w3 & b.w3};
}
__device__ __forceinline__ M256 m_or(M256 a, M256 b) {
    return {a.w0 | b.w0, a.w1 | b.w1, a.w2 | b.w2, a.w3 | b.w3};
}
__device__ __forceinline__ M256 m_xor(M256 a, M256 b) {
    return {a.w0 ^ b.w0, a.w1 ^ b.w1, a.w2 ^ b.w2, a.w3 ^ b.w3};
}
__device__ __forceinline__ M256 m_not(M256 a) { return {~a.w0, ~a.w1, ~a.w2, ~a.w3}; }
__device__ __forceinline__ bool m_eq(M256 a, M256 b) {
    return a.w0 == b.w0 && a.w1 == b.w1 && a.w2 == b.w2 && a.w3 == b.w3;
}
__device__ __forceinline__ int m_popc(M256 a) {
    return __popcll(a.w0) + __popcll(a.w1) + __popcll(a.w2) + __popcll(a.w3);
}
// a >> sh for 0 <= sh <= 256.
__device__ __forceinline__ M256 m_shr(M256 a, int sh) {
    const int q = sh >> 6, r = sh & 63;
    auto out = [&](int i) {
        const uint64_t lo = m_word(a, i + q);
        return r == 0 ? lo : (lo >> r) | (m_word(a, i + q + 1) << (64 - r));
    };
    return {out(0), out(1), out(2), out(3)};
}
__device__ __forceinline__ M256 m_low(M256, int n) {
    auto word = [&](int i) {
        const int b = n - 64 * i;
        return b >= 64 ? ~0ull : b <= 0 ? 0ull : ((1ull << b) - 1ull);
    };
    return {word(0), word(1), word(2), word(3)};
}
__device__ __forceinline__ int m_bit(M256 a, int i) {
    return (int)((m_word(a, i >> 6) >> (i & 63)) & 1ull);
}
__device__ __forceinline__ M256 m_onebit(M256, int i) {
    const int q = i >> 6;
    const uint64_t b = 1ull << (i & 63);
    return {q == 0 ? b : 0ull, q == 1 ? b : 0ull, q == 2 ? b : 0ull, q == 3 ? b : 0ull};
}

template <int NW> struct MaskOf;
template <> struct MaskOf<1> { using type = uint64_t; };
template <> struct MaskOf<2> { using type = M128; };
template <> struct MaskOf<4> { using type = M256; };

// Word h (0 <= h < 4) of a mask; words past its width are 0.
__device__ __forceinline__ uint64_t mask_word(uint64_t a, int h) { return h == 0 ? a : 0ull; }
__device__ __forceinline__ uint64_t mask_word(const M128 &a, int h) {
    return h == 0 ? a.lo : h == 1 ? a.hi : 0ull;
}
__device__ __forceinline__ uint64_t mask_word(const M256 &a, int h) { return m_word(a, h); }
template <typename Mask>
__device__ __forceinline__ uint64_t mask_lo(const Mask &a) { return mask_word(a, 0); }
template <typename Mask>
__device__ __forceinline__ uint64_t mask_hi(const Mask &a) { return mask_word(a, 1); }

// A mask of NW words from four words (words past NW are ignored).
template <int NW>
__device__ __forceinline__ typename MaskOf<NW>::type make_mask(uint64_t w0, uint64_t w1,
                                                               uint64_t w2 = 0ull,
                                                               uint64_t w3 = 0ull) {
    if constexpr (NW == 1) {
        return w0;
    } else if constexpr (NW == 2) {
        return M128{w0, w1};
    } else {
        return M256{w0, w1, w2, w3};
    }
}

// Mask of NW words stored at p[0 .. NW).
template <int NW>
__device__ __forceinline__ typename MaskOf<NW>::type load_mask(const uint64_t *p) {
    return make_mask<NW>(p[0], NW > 1 ? p[1] : 0ull, NW > 2 ? p[2] : 0ull, NW > 2 ? p[3] : 0ull);
}
template <int NW, typename Mask>
__device__ __forceinline__ void store_mask(uint64_t *p, const Mask &m) {
#pragma unroll
    for (int h = 0; h < NW; ++h) p[h] = mask_word(m, h);
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
        // PAPER: floor(N/2) + U[0, N]; RANGE: U[lo, hi] from the same word
        int lo = N / 2, span = N + 1;
        if (r.steps_rule == 3) {
            lo = r.slo_num * N / r.slo_den;
            span = r.shi_num * N / r.shi_den - lo + 1;
        }
        const Draw4 d = philox10(entity, gen, 0u, kTagLen, k0, k1);
        s.T = lo + (int)below(d.w0, (uint32_t)span);
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

// LDS layout of one walk of N > 64 (record form): P records, Q records
// (each run preceded by 15 spare records, so that the byte update after a
// move needs no bounds test; the Q run sits 0..15 records further on,
// depending on N, see below), plain P, plain Q, C bytes, and six words
// through which the two wavefronts of a split walk exchange their minima.
//   P[x] = s_x for x < N, 0 otherwise; Q is the reversed sequence,
//   Q[x] = s_{N-1-x} for x < N, 0 otherwise;
//   record x (16 bytes, at 16 x) holds P[x .. x+15], so a window starting
//   at any x is the records x, x+16, x+32, ...; lanes that read
//   consecutive starts touch consecutive 16-byte slots (no bank conflicts);
//   where the lanes switch from P windows (ascending starts) to Q windows
//   (descending), a 16-lane group would touch some 16-byte bank slot twice:
//   lanes j < m (P record j + 1) and j' >= m (Q record N - j') of the
//   group starting at g meet iff j + j' = dq + N - 1 (mod 16) for a Q run
//   shifted by dq records; the sums j + j' fill g + m .. g + m + 14, so
//   dq = m - N (mod 16) clears that group (m = (N + 1) / 2, the first lane
//   whose longer window is Q);
//   the plain copies hold P[0 .. LEN) and Q[0 .. LEN) for the C update;
//   CB[k-1] = C_k as int8 (N <= 128), or C_k >> 1 (N <= 256, where |C_k|
//   may reach 255; C_k = 2 (C_k >> 1) + ((N - k) & 1) since C_k is a sum of
//   N - k terms +-1).
// NREC covers the farthest record a window reads (start <= 64 NW, plus
// NBIG - 1 chunks); LEN the farthest byte the C update reads.
template <int NW> struct WalkLds;
template <> struct WalkLds<1> {
    static constexpr int NBIG = 4;  // lag form below
};
template <> struct WalkLds<2> {
    static constexpr int NBIG = 8, LEN = 256, CLEN = 128;
    static constexpr int NREC = 128 + 16 * (NBIG - 1) + 1;
};
template <> struct WalkLds<4> {
    static constexpr int NBIG = 16, LEN = 512, CLEN = 256;
    static constexpr int NREC = 256 + 16 * (NBIG - 1) + 1;
};
constexpr int kSpareRecords = 15;

// LDS layout of one walk of N <= 64 (lag form): 16 spare bytes, then row j
// (kLagRow bytes apart, so that 16-byte reads of consecutive rows are
// conflict-free) holding t_jk = s_{j+k} + s_{j-k} for k = 1..64 in bytes
// 0..63 (terms outside the sequence are 0) and 16 spare bytes; then
// CB[k-1] = C_k as int8.  The byte before each row is spare, so the update
// write of the lane whose neighbour was flipped (lag 0) lands there; rows
// j >= N are never read as neighbour data and take stray writes.
// (N <= 128: 64 NW rows of 64 NW + 16 bytes, C as 64 NW bytes, and six
// words through which the two wavefronts of a split walk exchange their
// minima.)  Last, the sequence as int8 with zeros around it: SP[q] = s_q
// for 0 <= q < N and 0 for the other q in -64 NW .. 128 NW - 1, which
// covers every q = 2j - p of two positions j, p < 64 NW.
template <int NW>
struct LagLds {
    static constexpr int ROW = 64 * NW + 16, BASE = 16;
    static constexpr int XCH = BASE + 64 * NW * ROW + 64 * NW;
    static constexpr int SPLO = XCH + 32, SP = SPLO + 64 * NW;
    static constexpr int BYTES = SP + 128 * NW;
};

template <int NW>
constexpr int record_lds_bytes() {
    // + 16 records of room for the Q run's shift, + the exchange words
    return 2 * 16 * (kSpareRecords + WalkLds<NW>::NREC) + 16 * 16 + 2 * WalkLds<NW>::LEN +
           WalkLds<NW>::CLEN + 32;
}

// LDS bytes of one walk: the lag form (LAG, N <= 128) or the record form.
// The lag form always serves N <= 64; for 64 < N <= 128 its 18 KB per walk
// halve the walks a CU holds, so only kernels whose occupancy is fixed by
// other means (batched memetic generations) choose it.
template <int NW, bool LAG = (NW == 1)>
constexpr int walk_lds_bytes() {
    static_assert(!LAG || NW <= 2, "the lag form covers N <= 128");
    if constexpr (LAG)
        return LagLds<NW>::BYTES;
    else
        return record_lds_bytes<NW>();
}
// Lane l receives bit l of a wave-uniform 64-bit mask.
__device__ __forceinline__ bool lane_bit(uint64_t mask) {
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// Four bytes P[x..x+3] of a sequence given as a mask (bit set <=> -1):
// 0x01 for +1, 0xFF for -1, 0 past the end.
template <typename Mask>
__device__ __forceinline__ uint32_t pack4(Mask M, int x, int N) {
    if (x >= N) return 0u;
    const uint32_t nib = (uint32_t)mask_lo(m_shr(M, x)) & 0xFu;
    const int cnt = min(N - x, 4);
    const uint32_t valid = cnt >= 4 ? 0x01010101u : (0x01010101u & ((1u << (8 * cnt)) - 1u));
    const uint32_t ones = (nib * 0x00204081u) & 0x01010101u;  // bit b -> byte b
    return valid | (ones * 0xFEu);
}

// |a - b| + c in one instruction, a wave-uniform.
__device__ __forceinline__ uint32_t absdiff_add_s(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(d) : "s"(a), "v"(b), "v"(c));
    return d;
}

// a * b + c for a, b of at most 24 significant bits (signed), where b
// comes straight from a dot-product instruction: a VALU read of a dot
// result needs three wait states, which the compiler cannot see to
// through inline assembly, so five are taken here first.
__device__ __forceinline__ int mad_i24_after_dot(int a, int b, int c) {
    int d;
    asm("s_nop 4\n\tv_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Two of them (a0 * b0 + c0, a1 * b1 + c1) after one such wait.
__device__ __forceinline__ void mad2_i24_after_dot(int a0, int b0, int c0, int a1, int b1, int c1,
                                                   int &d0, int &d1) {
    asm("s_nop 4\n\tv_mad_i32_i24 %0, %2, %3, %4\n\tv_mad_i32_i24 %1, %5, %6, %7"
        : "=&v"(d0), "=&v"(d1)
        : "v"(a0), "v"(b0), "v"(c0), "v"(a1), "v"(b1), "v"(c1));
}

// The same with b wave-uniform (a scalar operand).
__device__ __forceinline__ int mad_i24_s(int a, int b, int c) {
    int d;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
    return d;
}

// Byte accesses by LDS offset (the 32-bit address of the local address
// space, so that an offset computed in one instruction is the address).
typedef __attribute__((address_space(3))) int8_t lds_i8;
__device__ __forceinline__ uint32_t lds_offset(const void *p) {
    return (uint32_t)(uintptr_t)(const lds_i8 *)p;
}
__device__ __forceinline__ int lds_load_i8(uint32_t a) { return *(const lds_i8 *)(uintptr_t)a; }
__device__ __forceinline__ void lds_store_i8(uint32_t a, int v) {
    *(lds_i8 *)(uintptr_t)a = (int8_t)v;
}

// Bytewise a + b of four int8 lanes holding -1, 0 or +1 each (no carry
// crosses a byte: the low seven bits of each byte add to at most 0xFE).
__device__ __forceinline__ uint32_t add_bytes(uint32_t a, uint32_t b) {
    return ((a & 0x7F7F7F7Fu) + (b & 0x7F7F7F7Fu)) ^ ((a ^ b) & 0x80808080u);
}

// Four int8 lanes from bits x..x+3 of a 64-bit value of which the first n
// bits are valid (bit set <=> -1): 0x01 for +1, 0xFF for -1, 0 past n.
// Bits past n must be clear.
__device__ __forceinline__ uint32_t pack_bits4(uint64_t bits, int x, int n) {
    if (x >= n) return 0u;
    const uint32_t nib = (uint32_t)(bits >> x) & 0xFu;
    const int cnt = min(n - x, 4);
    const uint32_t valid = cnt >= 4 ? 0x01010101u : (0x01010101u & ((1u << (8 * cnt)) - 1u));
    const uint32_t ones = (nib * 0x00204081u) & 0x01010101u;  // bit b -> byte b
    return valid | (ones * 0xFEu);
}


__device__ __forceinline__ int dot16(const uint4 a, const uint4 b, int acc) {
    acc = __builtin_amdgcn_sdot4((int)a.x, (int)b.x, acc, false);
    acc = __builtin_amdgcn_sdot4((int)a.y, (int)b.y, acc, false);
    acc = __builtin_amdgcn_sdot4((int)a.z, (int)b.z, acc, false);
    return __builtin_amdgcn_sdot4((int)a.w, (int)b.w, acc, false);
}

// Orders the LDS accesses of the SPLIT wavefronts that run one walk (a
// wavefront fence for one, a workgroup barrier for two: the workgroup is
// exactly the walk's wavefronts).
template <int SPLIT>
__device__ __forceinline__ void walk_sync() {
    if constexpr (SPLIT == 1)
        wave_sync();
    else
        __syncthreads();
}

// One walk of N <= 64 NW (NW = 1 or 2) in the lag form on one wavefront,
// lane l owning neighbours j = l + 64h and lags k = j + 1 (h < NW).
// Neighbour j's sums are
//   v_j = sum_k t_jk C_k   (NB chunk dot products of its row against C),
//   u_j = sum_{k <= min(j, N-1-j)} s_{j+k} s_{j-k}   (kept per neighbour),
// since sum_k t_jk^2 = N - 1 + 2 u_j.  A move at p changes, for each j != p,
// only the lag k = |p - j| of row j: the other end of that pair is
// q = 2j - p, so t_jk becomes s_p + s_q (s_q = 0 outside the sequence) and
// u_j changes by -2 s_p(old) s_q when q is inside; C_k changes by
// -2 s_p(old) t_pk, read from row p, which the move leaves unchanged.
template <int NW, bool TRACE, int NB, int SPLIT = 1>
__device__ __forceinline__ WalkResult<NW> tabu_walk_lags(const int N_in,
                                                         const typename MaskOf<NW>::type M0,
                                                         const Schedule sch_in,
                                                         const int aspiration_in,
                                                         const uint32_t k0, const uint32_t k1,
                                                         const uint32_t entity, const uint32_t gen,
                                                         uint8_t *__restrict__ lds,
                                                         int16_t *__restrict__ trace,
                                                         const int part_in = 0) {
    static_assert(NW == 1 || NW == 2, "lag form: N <= 128");
    static_assert(SPLIT == 1 || (SPLIT == 2 && NW == 2), "two wavefronts per walk need N <= 128");
    static_assert(NB >= 1 && NB <= 4 * NW, "N <= 64 NW needs at most 4 NW 16-lag chunks");
    using Mask = typename MaskOf<NW>::type;
    constexpr int ROW = LagLds<NW>::ROW;
    constexpr int NL = NW / SPLIT;  // neighbours per lane
    const int lane = lane_id();
    const int part = SPLIT == 1 ? 0 : __builtin_amdgcn_readfirstlane(part_in);
    // register h of a lane holds neighbour j = lane + 64 half(h)
    auto half = [&](int h) { return SPLIT == 1 ? h : part; };
    const int N = __builtin_amdgcn_readfirstlane(N_in);
    const int aspiration = __builtin_amdgcn_readfirstlane(aspiration_in);
    Schedule sch;
    sch.T = __builtin_amdgcn_readfirstlane(sch_in.T);
    sch.lo = __builtin_amdgcn_readfirstlane(sch_in.lo);
    sch.hi = __builtin_amdgcn_readfirstlane(sch_in.hi);
    Mask M = make_mask<NW>(uniform64(mask_word(M0, 0)), uniform64(mask_word(M0, 1)));
    // bit i of Mr is bit N-1-i of M
    Mask Mr;
    {
        uint64_t r[2] = {0ull, 0ull};
#pragma unroll
        for (int h = 0; h < NW; ++h) {
            const int i = lane + 64 * h;
            r[h] = ballot(i < N && m_bit(M, N - 1 - i));
        }
        Mr = make_mask<NW>(r[0], r[1]);
    }

    uint8_t *const rows = lds + LagLds<NW>::BASE;
    int8_t *const CB = (int8_t *)(rows + 64 * NW * ROW);
    int *const XCH = (int *)(lds + LagLds<NW>::XCH);  // SPLIT: [part][min, tie lo, tie hi]

    // Row j: s_{j+k} is bit k-1 of R = M >> (j+1) (valid below N-1-j),
    // s_{j-k} bit k-1 of L = Mr >> (N-j) (valid below j).
    int u2[NL], ns[NL], C[NL], tabu[NL];  // 2 u_j, -s_j (set per step)
    bool asp[NL];
    uint32_t rowm1[NL];  // LDS offset of row j's byte k-1, minus k (k = 0: the spare byte)
    uint32_t spj[NL];    // LDS offset of SP[2j]
    int sq_e = 0;        // sum of C_k^2 over this lane's lags
    walk_sync<SPLIT>();
    for (int idx = lane + 64 * part; idx < 48 * NW; idx += 64 * SPLIT) {
        const int x = 4 * idx - 64 * NW;  // SP[x .. x+3]
        ((uint32_t *)(lds + LagLds<NW>::SPLO))[idx] = x < 0 ? 0u : pack4(M, x, N);
    }
#pragma unroll
    for (int h = 0; h < NL; ++h) {
        const int j = lane + 64 * half(h);
        const int nr = max(N - 1 - j, 0), nl = j < N ? j : 0;
        const Mask R = m_shr(m_shr(M, j), 1);
        const Mask L = j < N ? m_shr(m_shr(Mr, N - 1 - j), 1) : make_mask<NW>(0ull, 0ull);
        uint32_t *const row = (uint32_t *)(rows + ROW * j);
#pragma unroll
        for (int d = 0; d < 16 * NW; ++d) {
            const int x = 4 * d;  // a nibble never straddles two words
            row[d] = add_bytes(pack_bits4(mask_word(R, x >> 6), x & 63, nr - (x & ~63)),
                               pack_bits4(mask_word(L, x >> 6), x & 63, nl - (x & ~63)));
        }
        const int nu = min(nr, nl);
        u2[h] = 2 * (nu - 2 * m_popc(m_and(m_xor(R, L), m_low(R, nu))));
        // C_k of this lane's lag (Eq. 1) and its int8 mirror
        const int k = j + 1;
        C[h] = k < N ? lag_corr(M, N, k) : 0;
        CB[k - 1] = (int8_t)C[h];
        sq_e += C[h] * C[h];
        // lanes past the sequence are never admissible: infinite tenure
        // and no aspiration
        tabu[h] = j < N ? 0 : INT_MAX;
        asp[h] = aspiration && j < N;
        rowm1[h] = lds_offset(lds) + (uint32_t)(LagLds<NW>::BASE + ROW * j - 1);
        spj[h] = lds_offset(lds) + (uint32_t)(LagLds<NW>::SP + 2 * j);
    }
    int E = wave_sum(sq_e);
    if constexpr (SPLIT == 2) {
        XCH[3 * part] = E;  // uniform value, every lane
        walk_sync<SPLIT>();
        E += __builtin_amdgcn_readfirstlane(XCH[3 * (1 - part)]);
    }
    Mask best = M;
    int bestE = E;
    uint32_t dr0 = 0u;
    int expire = 0;  // lane l: step t0 + l plus that step's tenure

    uint4 tc[NL][NB];
    walk_sync<SPLIT>();
#pragma unroll
    for (int h = 0; h < NL; ++h)
#pragma unroll
        for (int r = 0; r < NB; ++r)
            tc[h][r] = ((const uint4 *)(rows + ROW * (lane + 64 * half(h))))[r];

    for (int t0 = 1; t0 <= sch.T; t0 += 64) {
        {
            const Draw4 d = philox10(entity, gen, (uint32_t)(t0 + lane), kTagStep, k0, k1);
            dr0 = d.w0;
            expire = t0 + lane + sch.lo + (int)below(d.w1, (uint32_t)(sch.hi - sch.lo + 1));
        }
        const int t_end = min(sch.T, t0 + 63);
        for (int t = t0; t <= t_end; ++t) {
            const int slot = t - t0;
            walk_sync<SPLIT>();  // the previous move's C and row bytes are visible
            uint4 cc[NB];
#pragma unroll
            for (int r = 0; r < NB; ++r) cc[r] = ((const uint4 *)CB)[r];

            // key d_j = 2 u_j - s_j v_j: candE_j = E + 4 (N - 1) + 4 d_j
            const int thr = ((bestE - E) >> 2) - (N - 1);
            int key[NL], v[NL], d[NL];
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                v[h] = 0;
#pragma unroll
                for (int r = 0; r < NB; ++r) v[h] = dot16(tc[h][r], cc[r], v[h]);
                ns[h] = lane_bit(mask_word(M, half(h))) ? 1 : -1;  // -s_j
            }
            if constexpr (NL == 2)  // |v| <= N^2
                mad2_i24_after_dot(ns[0], v[0], u2[0], ns[1], v[1], u2[1], d[0], d[1]);
            else
                d[0] = mad_i24_after_dot(ns[0], v[0], u2[0]);
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                const bool admissible = tabu[h] < t || (asp[h] && d[h] < thr);
                key[h] = admissible ? d[h] : INT_MAX;
            }
            int m;
            uint64_t T0, T1 = 0ull;
            if constexpr (SPLIT == 1) {
                int kmin = key[0];
                if constexpr (NW == 2) kmin = min(kmin, key[1]);
                m = wave_min(kmin);
                T0 = ballot(key[0] == m);
                if constexpr (NW == 2) T1 = ballot(key[1] == m);
            } else {
                // each wavefront's minimum and tie ballot, exchanged in LDS
                const int mine = wave_min(key[0]);
                const uint64_t tmine = ballot(key[0] == mine);
                XCH[3 * part] = mine;  // uniform values, every lane
                XCH[3 * part + 1] = (int)(uint32_t)tmine;
                XCH[3 * part + 2] = (int)(uint32_t)(tmine >> 32);
                walk_sync<SPLIT>();
                const int other = __builtin_amdgcn_readfirstlane(XCH[3 * (1 - part)]);
                const uint64_t tother =
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(XCH[3 * (1 - part) + 2]) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane(XCH[3 * (1 - part) + 1]);
                m = min(mine, other);
                const uint64_t a = mine == m ? tmine : 0ull;
                const uint64_t b = other == m ? tother : 0ull;
                T0 = part == 0 ? a : b;
                T1 = part == 0 ? b : a;
            }
            uint64_t tied = T0;
            int pick_base = 0;
            if constexpr (NW == 2) {
                if (T0 == 0ull) {
                    tied = T1;
                    pick_base = 64;
                }
            }
            // several tied moves: take the r-th, r from the step's first draw
            int c0 = __popcll(T0), count = NW == 2 ? c0 + __popcll(T1) : c0;
            asm("" : "+s"(count));  // a 32-bit scalar compare below
            if (count > 1) {
                int r = (int)below(readlane_u(dr0, slot), (uint32_t)count);
                tied = T0;
                pick_base = 0;
                if constexpr (NW == 2) {
                    if (r >= c0) {
                        tied = T1;
                        pick_base = 64;
                        r -= c0;
                    }
                }
                for (int i = 0; i < r; ++i) tied &= tied - 1ull;  // drop the r lowest
            }
            const int pick = pick_base + __builtin_ctzll(tied);

            const int tabu_new = readlane(expire, slot);  // t + tenure
            const bool neg = m_bit(M, pick);
            const int sm = neg ? -1 : 1;    // old s_pick
            const int k2 = neg ? 2 : -2;    // -2 s_pick(old)
            const int k4 = neg ? 4 : -4;
            M = m_xor(M, m_onebit(M, pick));
            E += 4 * (N - 1 + m);
            if (E < bestE) {
                bestE = E;
                best = M;
            }
            if constexpr (TRACE) {
                if (part == 0) trace[t - 1] = (int16_t)pick;  // uniform store
            }

            // Lag |pick - j| of row j has its other end at q = 2j - pick
            // (q >= N for j >= N), s_q = SP[q], and changes u_j by
            // -2 s_pick(old) s_q.  q = j only for j = pick, whose u is
            // unchanged: that lane reads s_pick(old) itself, and adds back
            // the -2 it takes; it also stores the new s_pick (its -s_j before
            // the move) into SP[pick] after the reads (with two wavefronts
            // the lane is on pick's owner; the other one reads other entries
            // only).  Each wavefront rewrites the rows of its own neighbours
            // (row pick, which another wavefront may read below, does not
            // change; for j = pick the write goes to the spare byte).
            // Both loads of the move depend on pick alone and go out together:
            // s_q, and t_pick,k of this lane's lags from row pick (which the
            // move leaves unchanged) for C_k -= 2 s_pick(old) t_pick,k.
            uint32_t qa[NL];
            int sq[NL], tpk[NL];
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                qa[h] = spj[h] - (uint32_t)pick;
                sq[h] = lds_load_i8(qa[h]);
                asm("" : "+v"(sq[h]));  // one sign-extending load
                tpk[h] = ((const int8_t *)rows)[ROW * pick + lane + 64 * half(h)];
            }
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                C[h] = mad_i24_s(tpk[h], k2, C[h]);
                CB[lane + 64 * half(h)] = (int8_t)C[h];
            }
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                const int j = lane + 64 * half(h);
                u2[h] = mad_i24_s(sq[h], k4, u2[h]);
                // t_jk = s_pick(new) + s_q into row j, byte |pick - j| - 1
                lds_store_i8(absdiff_add_s((uint32_t)pick, (uint32_t)j, rowm1[h]), sq[h] - sm);
                // lane pick (one neighbour per lane: the one-lane mask
                // straight from pick's bit; two: a compare is cheaper than
                // building the masks)
                if (NW == 1 ? lane_bit(1ull << pick) : j == pick) {
                    lds_store_i8(qa[h], ns[h]);
                    u2[h] += 4;
                    tabu[h] = tabu_new;
                }
            }
            wave_sync();  // own rows only
#pragma unroll
            for (int h = 0; h < NL; ++h)
#pragma unroll
                for (int r = 0; r < NB; ++r)
                    tc[h][r] = ((const uint4 *)(rows + ROW * (lane + 64 * half(h))))[r];
        }
    }

    WalkResult<NW> res;
    res.best = best;
    res.best_e = bestE;
    res.final_e = E;
    return res;
}

// Runs one walk of sch.T steps from mask M0 (bits >= N must be clear).
//   NW     neighbours per lane when one wavefront runs the walk: 1 for
//          N <= 64, 2 for N <= 128, 4 for N <= 256 (also fixes the mask
//          width and the LDS layout)
//   SPLIT  wavefronts per walk: 1, or 2 with NW = 2, wavefront `part`
//          (0 or 1) owning neighbours and lags 64 part .. 64 part + 63; the
//          two exchange their minima through LDS (two barriers per step)
//   lds    per-walk LDS scratch of walk_lds_bytes<NW>() bytes, 16-aligned
//   trace  with TRACE: trace[t-1] = flipped index
// Every lane of the walk's wavefronts must call this with identical uniform
// inputs (part aside).
template <int NW, bool TRACE, int SPLIT, int NB>
__device__ __forceinline__ WalkResult<NW> tabu_walk_records(const int N_in, const typename MaskOf<NW>::type M0,
                                                    const Schedule sch_in, const int aspiration_in,
                                                    const uint32_t k0, const uint32_t k1,
                                                    const uint32_t entity, const uint32_t gen,
                                                    uint8_t *__restrict__ lds,
                                                    int16_t *__restrict__ trace,
                                                    const int part_in = 0) {
    static_assert(SPLIT == 1 || (SPLIT == 2 && NW == 2), "two wavefronts per walk need N <= 128");
    static_assert(NW == 2 || NW == 4, "record form: mask widths of 128 or 256 bits");
    static_assert(NB >= 1 && NB <= WalkLds<NW>::NBIG, "chunk count beyond the layout");
    constexpr int NS = (NB + 1) / 2;  // chunks of the shorter window (N - 1 <= 16 NB)
    using Mask = typename MaskOf<NW>::type;
    using Cfg = WalkLds<NW>;
    constexpr int NL = NW / SPLIT;  // neighbours per lane
    const int lane = lane_id();
    // Wave-uniform parameters, pinned to scalar registers so that the step
    // loop is controlled by scalar branches.
    const int N = __builtin_amdgcn_readfirstlane(N_in);
    const int aspiration = __builtin_amdgcn_readfirstlane(aspiration_in);
    const int part = SPLIT == 1 ? 0 : __builtin_amdgcn_readfirstlane(part_in);
    Schedule sch;
    sch.T = __builtin_amdgcn_readfirstlane(sch_in.T);
    sch.lo = __builtin_amdgcn_readfirstlane(sch_in.lo);
    sch.hi = __builtin_amdgcn_readfirstlane(sch_in.hi);
    // The sequence is wave-uniform; pinning it to scalar registers keeps the
    // per-move mask arithmetic on the scalar unit.
    Mask M = make_mask<NW>(uniform64(mask_word(M0, 0)), uniform64(mask_word(M0, 1)),
                           uniform64(mask_word(M0, 2)), uniform64(mask_word(M0, 3)));

    // Reversed sequence: bit i of Mr is bit N-1-i of M.
    Mask Mr;
    {
        uint64_t r[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
        for (int h = 0; h < NW; ++h) {
            const int i = lane + 64 * h;
            r[h] = ballot(i < N && m_bit(M, N - 1 - i));
        }
        Mr = make_mask<NW>(r[0], r[1], r[2], r[3]);
    }
    // N <= 256 keeps C_k >> 1 in the int8 mirror; the parity part of
    // sum_k t_jk C_k is then sum_{k: N-k odd} t_jk = S_q - (N odd) s_j with
    // S_q the sum of s_i over positions i of parity q = (j + N - 1) mod 2
    // (every i != j in range is j + k or j - k for exactly one k, and
    // N - k odd <=> i = q mod 2).  S_0, S_1 are wave-uniform.
    constexpr bool kHalfC = NW == 4;
    int S0 = 0, S1 = 0;
    if constexpr (kHalfC) {
        constexpr uint64_t kEven = 0x5555555555555555ull;
        const M256 ev{kEven, kEven, kEven, kEven};
        const int neg0 = m_popc(m_and(M, ev)), neg1 = m_popc(m_and(M, m_not(ev)));
        S0 = (N + 1) / 2 - 2 * neg0;
        S1 = N / 2 - 2 * neg1;
    }

    constexpr int kRunBytes = 16 * (kSpareRecords + Cfg::NREC);
    const int dq = ((N + 1) / 2 - N) & 15;  // the Q run's shift in records
    uint8_t *const RP = lds + 16 * kSpareRecords;
    uint8_t *const RQ = RP + kRunBytes + 16 * dq;
    uint8_t *const PP = lds + 2 * kRunBytes + 16 * 16;
    uint8_t *const PQ = PP + Cfg::LEN;
    int8_t *const CB = (int8_t *)(PQ + Cfg::LEN);
    int *const XCH = (int *)(CB + Cfg::CLEN);  // SPLIT exchange: [part][min, tie lo, tie hi]

    // Fill the records (dword d of record x holds P[x + 4d .. x + 4d + 3])
    // and the plain copies.
    walk_sync<SPLIT>();
    for (int idx = lane + 64 * part; idx < 4 * Cfg::NREC; idx += 64 * SPLIT) {
        const int pos = (idx >> 2) + 4 * (idx & 3);
        ((uint32_t *)RP)[idx] = pack4(M, pos, N);
        ((uint32_t *)RQ)[idx] = pack4(Mr, pos, N);
    }
    for (int idx = lane + 64 * part; idx < Cfg::LEN / 4; idx += 64 * SPLIT) {
        ((uint32_t *)PP)[idx] = pack4(M, 4 * idx, N);
        ((uint32_t *)PQ)[idx] = pack4(Mr, 4 * idx, N);
    }

    // Register w of a lane holds neighbour j = lane + 64 h and lag
    // k = lane + 1 + 64 h, h = w (one wavefront) or part (two).
    auto half = [&](int w) { return SPLIT == 1 ? w : part; };

    // C_k for the lags this lane owns (Eq. 1), its int8 mirror, the energy.
    int C[NL];
    int sq = 0;
#pragma unroll
    for (int w = 0; w < NL; ++w) {
        const int k = lane + 1 + 64 * half(w);
        C[w] = k < N ? lag_corr(M, N, k) : 0;
        sq += C[w] * C[w];
        CB[k - 1] = (int8_t)(kHalfC ? C[w] >> 1 : C[w]);
    }
    int E = wave_sum(sq);
    if constexpr (SPLIT == 2) {
        XCH[3 * part] = E;  // uniform value, every lane
        walk_sync<SPLIT>();
        E += __builtin_amdgcn_readfirstlane(XCH[3 * (1 - part)]);
    }

    // Per-lane window addresses (fixed for the walk).  Neighbour j's right
    // window starts at P[j+1], its left window at Q[N-j]; the longer of the
    // two is read over all lags, the shorter over the first half.
    const uint8_t *big[NL];
    const uint8_t *small[NL];
#pragma unroll
    for (int w = 0; w < NL; ++w) {
        const int j = lane + 64 * half(w);
        const int xr = j + 1;
        // j >= N: an all-zero window, at a start that is a multiple of 16 so
        // that it shares no bank slot with lanes j < N of its group (all
        // lanes j >= N read the same address)
        const int xl = j < N ? N - j : (N + 15) & ~15;
        const uint8_t *right = RP + 16 * xr;
        const uint8_t *left = RQ + 16 * xl;
        const bool right_big = N - 1 - j >= j;
        big[w] = right_big ? right : left;
        small[w] = right_big ? left : right;
    }

    // The byte update after a move writes the new s_pick into the 16
    // records holding P[pick] (lanes 0..15: byte c of record pick - c), the
    // 16 holding Q[N-1-pick] (lanes 16..31) and the plain copies (lanes 32,
    // 33): offset from RP = upd_a + upd_b * pick.  Records down to -15 are
    // spare, so no lane tests bounds.
    int upd_a, upd_b;
    {
        const int c = lane & 15;
        const int pln = 2 * kRunBytes + 16 * 16 - 16 * kSpareRecords;  // PP - RP
        if (lane < 16) {
            upd_a = -15 * c;
            upd_b = 16;
        } else if (lane < 32) {
            upd_a = kRunBytes + 16 * dq + 16 * (N - 1) - 15 * c;
            upd_b = -16;
        } else if (lane == 32) {
            upd_a = pln;
            upd_b = 1;
        } else {
            upd_a = pln + Cfg::LEN + N - 1;
            upd_b = -1;
        }
    }
    const bool updater = part == 0 && lane < 34;

    // lanes past the sequence are never admissible: infinite tenure, and
    // zero windows give them d_j >= -ceil(N/2), never below the aspiration
    // threshold (at most -(N - 1), since bestE <= E)
    int tabu[NL];
#pragma unroll
    for (int w = 0; w < NL; ++w) tabu[w] = lane + 64 * half(w) < N ? 0 : INT_MAX;

    // u_j = sum_{k <= min(j, N-1-j)} s_{j+k} s_{j-k}: from the windows once,
    // then per move (a move at p changes only the term with k = |p - j|,
    // whose other end is q = 2j - p, by -2 s_p(old) s_q)
    int uj[NL];
    walk_sync<SPLIT>();
#pragma unroll
    for (int w = 0; w < NL; ++w) {
        int a = 0;
#pragma unroll
        for (int r = 0; r < NS; ++r)
            a = dot16(((const uint4 *)big[w])[16 * r], ((const uint4 *)small[w])[16 * r], a);
        uj[w] = a;
    }
    Mask best = M;
    int bestE = E;
    uint32_t dr0 = 0u;
    int expire = 0;  // lane l: step t0 + l plus that step's tenure

    // Window chunks of the current pivot, read at the top of each step (two
    // neighbours: the registers for earlier loads would cost occupancy; two
    // wavefronts: the other one's byte update must be visible first).  With
    // four neighbours per lane each neighbour's chunks are read where they
    // are used (all of them at once would not fit the register file).
    constexpr bool kPreload = NW != 4;
    constexpr int NLP = kPreload ? NL : 1;
    uint4 wb[NLP][NB];
    uint4 ws[NLP][NS];

    // Steps in blocks of 64: one Philox call per lane supplies the draws of
    // a block (read back with readlane), and the inner loop carries no
    // refill test.
    for (int t0 = 1; t0 <= sch.T; t0 += 64) {
        {
            const Draw4 d = philox10(entity, gen, (uint32_t)(t0 + lane), kTagStep, k0, k1);
            dr0 = d.w0;
            expire = t0 + lane + sch.lo + (int)below(d.w1, (uint32_t)(sch.hi - sch.lo + 1));
        }
        const int t_end = min(sch.T, t0 + 63);
        for (int t = t0; t <= t_end; ++t) {
            const int slot = t - t0;
            walk_sync<SPLIT>();  // the previous move's bytes are visible
            if constexpr (kPreload) {
#pragma unroll
                for (int w = 0; w < NL; ++w) {
#pragma unroll
                    for (int r = 0; r < NB; ++r) wb[w][r] = ((const uint4 *)big[w])[16 * r];
#pragma unroll
                    for (int r = 0; r < NS; ++r) ws[w][r] = ((const uint4 *)small[w])[16 * r];
                }
            }

            uint4 cc[NB];  // C_1 .. C_{16 NB} (wave-uniform)
#pragma unroll
            for (int r = 0; r < NB; ++r) cc[r] = ((const uint4 *)CB)[r];

            // Score the neighbours this lane owns.  The key is
            // d_j = 2 u_j - s_j v_j, so that candE_j = E + 4 (N - 1) + 4 d_j;
            // aspiration (candE_j < bestE) is d_j < thr.  Energies are all
            // congruent mod 4, so thr is exact.
            const int thr = ((bestE - E) >> 2) - (N - 1);
            // parity part (kHalfC): S_q - (N odd) s_j, q = (j + N - 1) mod 2 is
            // the same for all of this lane's neighbours
            const int Sq = ((lane + N - 1) & 1) ? S1 : S0;
            int key[NL];
#pragma unroll
            for (int w = 0; w < NL; ++w) {
                const int j = lane + 64 * half(w);
                int v = 0;  // sum_k t_jk C_k (kHalfC: sum_k t_jk (C_k >> 1))
                const int u = uj[w];
                if constexpr (kPreload) {
#pragma unroll
                    for (int r = 0; r < NB; ++r) {
                        v = dot16(wb[w][r], cc[r], v);
                        if (r < NS) v = dot16(ws[w][r], cc[r], v);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < NB; ++r) {
                        v = dot16(((const uint4 *)big[w])[16 * r], cc[r], v);
                        if (r < NS) v = dot16(((const uint4 *)small[w])[16 * r], cc[r], v);
                    }
                }
                const bool neg = lane_bit(mask_word(M, half(w)));  // s_j = -1
                int d;
                if constexpr (kHalfC) {
                    // v_j = 2 v + S_q - (N odd) s_j, so
                    // 2 u - s_j v_j = 2 u - s_j (2 v + S_q) + (N odd)
                    const int vq = 2 * v + Sq;
                    d = 2 * u + (neg ? vq : -vq) + (N & 1);
                } else {
                    d = 2 * u + (neg ? v : -v);  // 2 u_j - s_j v_j
                }
                const bool admissible = tabu[w] < t || (aspiration && d < thr);
                key[w] = admissible ? d : INT_MAX;
            }

            // Admissible minimum, ties broken by the step's draw: the r-th
            // (ascending) of the tied moves, r = (u0 * count) >> 32.
            int m;
            uint64_t T0, T1 = 0ull, T2 = 0ull, T3 = 0ull;
            if constexpr (SPLIT == 1) {
                int kmin = key[0];
                if constexpr (NW >= 2) kmin = min(kmin, key[1]);
                if constexpr (NW == 4) kmin = min(kmin, min(key[2], key[3]));
                m = wave_min(kmin);
                T0 = ballot(key[0] == m);
                if constexpr (NW >= 2) T1 = ballot(key[1] == m);
                if constexpr (NW == 4) {
                    T2 = ballot(key[2] == m);
                    T3 = ballot(key[3] == m);
                }
            } else {
                const int mine = wave_min(key[0]);
                const uint64_t tmine = ballot(key[0] == mine);
                XCH[3 * part] = mine;  // uniform values, every lane
                XCH[3 * part + 1] = (int)(uint32_t)tmine;
                XCH[3 * part + 2] = (int)(uint32_t)(tmine >> 32);
                walk_sync<SPLIT>();
                const int other = __builtin_amdgcn_readfirstlane(XCH[3 * (1 - part)]);
                const uint64_t tother =
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(XCH[3 * (1 - part) + 2]) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane(XCH[3 * (1 - part) + 1]);
                m = min(mine, other);
                const uint64_t a = mine == m ? tmine : 0ull;
                const uint64_t b = other == m ? tother : 0ull;
                T0 = part == 0 ? a : b;
                T1 = part == 0 ? b : a;
            }
            int pick;
            if constexpr (NW == 4) {
                // the r-th tied move over the four 64-neighbour words (r = 0
                // when only one is tied: the first word with a tied move)
                int c0 = __popcll(T0), c1 = __popcll(T1), c2 = __popcll(T2), c3 = __popcll(T3);
                asm("" : "+s"(c0), "+s"(c1), "+s"(c2), "+s"(c3));  // 32-bit scalar arithmetic
                const int count = c0 + c1 + c2 + c3;
                int r = 0;
                if (count > 1) r = (int)below(readlane_u(dr0, slot), (uint32_t)count);
                uint64_t tied;
                int base;
                if (r < c0) {
                    tied = T0;
                    base = 0;
                } else if (r < c0 + c1) {
                    tied = T1;
                    base = 64;
                    r -= c0;
                } else if (r < c0 + c1 + c2) {
                    tied = T2;
                    base = 128;
                    r -= c0 + c1;
                } else {
                    tied = T3;
                    base = 192;
                    r -= c0 + c1 + c2;
                }
                for (int i = 0; i < r; ++i) tied &= tied - 1ull;  // drop the r lowest
                pick = base + __builtin_ctzll(tied);
            } else {
                uint64_t tied = T0;
                int pick_base = 0;
                if constexpr (NW == 2) {
                    if (T0 == 0ull) {
                        tied = T1;
                        pick_base = 64;
                    }
                }
                // several tied moves: take the r-th, r from the step's first draw
                int c0 = __popcll(T0), count = c0 + __popcll(T1);
                asm("" : "+s"(c0), "+s"(count));  // 32-bit scalar arithmetic
                if (count > 1) {
                    int r = (int)below(readlane_u(dr0, slot), (uint32_t)count);
                    tied = T0;
                    pick_base = 0;
                    if constexpr (NW == 2) {
                        if (r >= c0) {
                            tied = T1;
                            pick_base = 64;
                            r -= c0;
                        }
                    }
                    for (int i = 0; i < r; ++i) tied &= tied - 1ull;  // drop the r lowest
                }
                pick = pick_base + __builtin_ctzll(tied);
            }

            // Apply the move: tenure, sequence, energy, best.
            const int tabu_new = readlane(expire, slot);  // t + tenure
            const bool neg = m_bit(M, pick);
            const int sm = neg ? -1 : 1;  // old s_pick
            const int k2 = neg ? 2 : -2;  // -2 s_pick(old)
            // lane pick (a one-lane mask straight from pick's bit) in
            // register w = pick >> 6 (one wavefront) or on wavefront part
            auto is_pick = [&](int w) {
                return lane_bit((pick >> 6) == half(w) ? 1ull << (pick & 63) : 0ull);
            };
#pragma unroll
            for (int w = 0; w < NL; ++w) tabu[w] = is_pick(w) ? tabu_new : tabu[w];
            M = m_xor(M, m_onebit(M, pick));
            E += 4 * (N - 1 + m);
            if constexpr (kHalfC) {
                if (pick & 1)
                    S1 -= 2 * sm;
                else
                    S0 -= 2 * sm;
            }
            if (E < bestE) {
                bestE = E;
                best = M;
            }
            if constexpr (TRACE) {
                if (part == 0) trace[t - 1] = (int16_t)pick;  // uniform store
            }

            // New s_pick into every record and plain copy that holds it.
            if (updater) RP[upd_a + upd_b * pick] = (uint8_t)(int8_t)(-sm);
            if constexpr (SPLIT == 1) wave_sync();  // lane pick reads P[pick] below

            // C_k -= 2 s_pick t_pick,k for every lag (lane-parallel):
            // s_{pick+k} = P[pick+k] and s_{pick-k} = Q[N-1-pick+k] are bytes of
            // the plain copies, zero past the ends (position pick itself is not
            // read, so the other wavefront's byte update cannot race with it).
            {
#pragma unroll
                for (int w = 0; w < NL; ++w) {
                    const int k = lane + 1 + 64 * half(w);
                    const int t_k = (int)((const int8_t *)PP)[pick + k] +
                                    (int)((const int8_t *)PQ)[N - 1 - pick + k];
                    C[w] += k2 * t_k;
                    CB[k - 1] = (int8_t)(kHalfC ? C[w] >> 1 : C[w]);
                }
            }

            // u_j += -2 s_pick(old) s_q with s_q = P[q], q = 2j - pick: q >= N
            // reads a zero, and so does q < 0 (index LEN + q >= N); j = pick,
            // whose u does not change, reads the new s_pick = -s_pick(old)
            // (one wavefront: the byte update above is in program order),
            // so that lane takes back the 2 it adds.  Two wavefronts: the
            // other one may be writing P[pick], which lane pick then skips.
#pragma unroll
            for (int w = 0; w < NL; ++w) {
                const int jw = lane + 64 * half(w);
                const int q = 2 * jw - pick;
                const int sq = (int)((const int8_t *)PP)[q & (Cfg::LEN - 1)];
                if constexpr (SPLIT == 1) {
                    uj[w] += k2 * sq;
                    if (is_pick(w)) uj[w] -= 2;
                } else {
                    uj[w] += jw != pick ? k2 * sq : 0;
                }
            }
        }
    }

    WalkResult<NW> res;
    res.best = best;
    res.best_e = bestE;
    res.final_e = E;
    return res;
}

// Runs one walk of sch.T steps from mask M0 (bits >= N must be clear): the
// lag form when LAG (N <= 128), the record form otherwise
// (arguments as above; lds holds walk_lds_bytes<NW, LAG>() bytes).
template <int NW, bool TRACE = false, int SPLIT = 1, int NB = WalkLds<NW>::NBIG,
          bool LAG = (NW == 1)>
__device__ __forceinline__ WalkResult<NW> tabu_walk(const int N_in,
                                                    const typename MaskOf<NW>::type M0,
                                                    const Schedule sch_in, const int aspiration_in,
                                                    const uint32_t k0, const uint32_t k1,
                                                    const uint32_t entity, const uint32_t gen,
                                                    uint8_t *__restrict__ lds,
                                                    int16_t *__restrict__ trace,
                                                    const int part_in = 0) {
    if constexpr (LAG) {
        static_assert(NW <= 2, "the lag form: N <= 128");
        return tabu_walk_lags<NW, TRACE, NB, SPLIT>(N_in, M0, sch_in, aspiration_in, k0, k1, entity,
                                                    gen, lds, trace, part_in);
    } else {
        return tabu_walk_records<NW, TRACE, SPLIT, NB>(N_in, M0, sch_in, aspiration_in, k0, k1,
                                                       entity, gen, lds, trace, part_in);
    }
}

}  // namespace liblabs
