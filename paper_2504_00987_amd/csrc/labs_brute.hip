// Exhaustive minima of Eq. (2) over all sequences of one length, and over
// the skew-symmetric ones of an odd length (Sec. II.C), for gfx950, and
// their launchers.
#include <algorithm>

#include "labs_device.hpp"
#include "labs_internal.h"

namespace liblabs {

namespace {


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

// Skew-symmetric sequences of odd length N = 2c + 1: lane g evaluates codes
// [g * per, (g + 1) * per) of the c free spins s_1..s_c (s_0 = +1); the
// other half is s_{c+i} = (-1)^i s_{c-i}.  Their C_k vanish for odd k, so E
// sums C_k^2 over even k only.  The code written back is the free-spin
// pattern F (bit i set <=> s_i = -1, i = 0..c).
template <int NW>
__device__ __forceinline__ typename MaskOf<NW>::type skew_mask(uint64_t F, int c) {
    // R_i = F_{c-i}; bit c + i of the sequence is R_i ^ (i odd), i = 1..c
    const uint64_t R = __builtin_bitreverse64(F) >> (63 - c);
    const uint64_t hiF = ((c >= 63 ? ~0ull : ((1ull << (c + 1)) - 1ull)) & ~1ull);
    const uint64_t U = (R ^ 0xAAAAAAAAAAAAAAAAull) & hiF;
    const uint64_t lo = F | (U << c);
    if constexpr (NW == 1) {
        return lo;
    } else {
        const uint64_t hi = c == 0 ? 0ull : (U >> (64 - c));
        return make_mask<NW>(lo, hi);
    }
}

template <int NW>
__global__ __launch_bounds__(256) void skew_bruteforce_kernel(int N, uint64_t per, uint64_t total,
                                                              int32_t *part_e, int64_t *part_count,
                                                              uint64_t *part_code) {
    using Mask = typename MaskOf<NW>::type;
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t wave = g >> 6;
    const int c = (N - 1) / 2;
    uint64_t c0 = g * per, c1 = c0 + per;
    if (c0 > total) c0 = total;
    if (c1 > total) c1 = total;
    int best = INT_MAX;
    int64_t cnt = 0;
    uint64_t best_code = ~0ull;
    for (uint64_t code = c0; code < c1; ++code) {
        const uint64_t F = code << 1;
        const Mask M = skew_mask<NW>(F, c);
        int e = 0;
        for (int k = 2; k < N; k += 2) {
            const int ck = lag_corr(M, N, k);
            e += ck * ck;
        }
        if (e < best) {
            best = e;
            cnt = 1;
            best_code = F;
        } else if (e == best) {
            ++cnt;
        }
    }
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
    part_code[wave] = code >> 1;  // the reduction shifts it back
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

// The skew-symmetric search has 2^c codes, c = (n - 1) / 2: the lane count
// of an exhaustive search over c + 1 spins.
int64_t skew_brute_waves(int n) { return brute_waves((n - 1) / 2 + 1); }

hipError_t launch_skew_bruteforce(int n, const BruteParts &p, hipStream_t s) {
    const int c = (n - 1) / 2;
    const uint64_t total = 1ull << c;
    const uint64_t lanes = brute_lanes(c + 1);
    const uint64_t per = (total + lanes - 1) / lanes;
    const unsigned blocks = (unsigned)(lanes / 256 > 0 ? lanes / 256 : 1);
    const unsigned threads = (unsigned)(lanes < 256 ? lanes : 256);
    if (n <= 64)
        hipLaunchKernelGGL(skew_bruteforce_kernel<1>, dim3(blocks), dim3(threads), 0, s, n, per,
                           total, p.part_e, p.part_count, p.part_code);
    else
        hipLaunchKernelGGL(skew_bruteforce_kernel<2>, dim3(blocks), dim3(threads), 0, s, n, per,
                           total, p.part_e, p.part_count, p.part_code);
    hipLaunchKernelGGL(bruteforce_reduce_kernel, dim3(1), dim3(64), 0, s, (int64_t)(lanes >> 6), p);
    return hipGetLastError();
}

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

}  // namespace liblabs
