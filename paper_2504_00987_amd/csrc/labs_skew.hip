// Deviation from skew-symmetry d(S) (App. A of arXiv:2504.00987) for a batch
// of sequences, for gfx950, and its launcher.
//
// Skew-symmetry of an odd-length sequence t, m = 2c + 1 (Sec. II.C):
// t_{c+i} = (-1)^i t_{c-i} for i = 1..c; n_non-skew(t) counts the pairs that
// break it.  d(S) is the least n_non-skew over one rotation of S (its first
// r elements moved to the end) followed, for even N, by one deletion: odd N
// has N candidates, even N has N * N (rotation r, deleted position q).
//
// One wavefront per sequence.  The sequence is copied twice into LDS, so
// rotation r reads position k at S2[r + k] without a modulo; lane l scores
// candidates l, l + 64, ... and the wavefront takes the minimum.
#include <algorithm>

#include "../../include/liblabs.h"
#include "labs_device.hpp"
#include "labs_internal.h"

namespace liblabs {

namespace {

template <int WPG>
__global__ __launch_bounds__(64 * WPG) void skew_deviation_kernel(
    const int8_t *__restrict__ seqs, const int32_t *__restrict__ ns, int32_t n_uniform,
    int32_t stride, int64_t count, int32_t *__restrict__ out) {
    __shared__ int8_t buf[WPG][2 * LABS_MAX_N];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t b = (int64_t)blockIdx.x * WPG + wave;
    if (b >= count) return;  // whole wavefronts only: no workgroup barrier below
    const int N = ns ? ns[b] : n_uniform;
    const int8_t *row = seqs + b * (int64_t)stride;
    int8_t *S2 = buf[wave];
    for (int k = lane; k < 2 * N; k += 64) S2[k] = row[k < N ? k : k - N];
    wave_sync();

    int best = N;
    if (N & 1) {
        const int c = (N - 1) / 2;
        for (int r = lane; r < N; r += 64) {
            const int8_t *t = S2 + r + c;
            int cnt = 0;
            for (int i = 1; i <= c; ++i) {
                const int a = t[i], l = t[-i];
                cnt += a != ((i & 1) ? -l : l);
            }
            best = min(best, cnt);
        }
    } else {
        // Del(Rot(S; r); q + 1): position p of the odd sequence is element
        // p + (p >= q) of the rotation
        const int c = N / 2 - 1;
        for (int cand = lane; cand < N * N; cand += 64) {
            const int r = cand / N, q = cand - r * N;
            const int8_t *t = S2 + r;
            int cnt = 0;
            for (int i = 1; i <= c; ++i) {
                const int p1 = c + i, p2 = c - i;
                const int a = t[p1 + (p1 >= q)], l = t[p2 + (p2 >= q)];
                cnt += a != ((i & 1) ? -l : l);
            }
            best = min(best, cnt);
        }
    }
    out[b] = wave_min(best);  // uniform value, every lane
}

}  // namespace

hipError_t launch_skew_deviation(const int8_t *seqs, const int32_t *ns, int32_t n_uniform,
                                 int32_t stride, int64_t count, int32_t *out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    constexpr int WPG = 4;
    // at most 2^30 work-items per launch (a grid's x extent in work-items is
    // a 32-bit count): larger batches run as consecutive launches
    constexpr int64_t kRowsPerLaunch = (int64_t(1) << 30) / 64;
    for (int64_t b0 = 0; b0 < count; b0 += kRowsPerLaunch) {
        const int64_t n = std::min(kRowsPerLaunch, count - b0);
        hipLaunchKernelGGL(skew_deviation_kernel<WPG>, dim3((unsigned)((n + WPG - 1) / WPG)),
                           dim3(64 * WPG), 0, s, seqs + b0 * (int64_t)stride, ns ? ns + b0 : nullptr,
                           n_uniform, stride, n, out + b0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace liblabs
