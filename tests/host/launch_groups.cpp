// Host-side launch logic of the batched walks, printed for the CPU tests:
// the length class of every N, the launch groups of every set of present
// classes under each launch form, and the layout of the kernel arguments.
// Built with the host compiler against the library's internal header; no
// GPU code runs.
#include <cstddef>
#include <cstdio>

#include "../../paper_2504_00987_amd/csrc/labs_internal.h"

using namespace liblabs;

int main() {
    std::printf("classes %d\n", kWalkClasses);
    for (int c = 0; c < kWalkClasses; ++c) std::printf("maxn %d %d\n", c, kClassMaxN[c]);
    for (int n = LABS_MIN_N; n <= LABS_MAX_N; ++n) std::printf("class %d %d\n", n, walk_class(n));
    std::printf("class_end_slots %zu\n", sizeof(((TabuLaunchArgs *)nullptr)->class_end) / sizeof(int64_t));
    std::printf("k0_after_class_end %d\n",
                (int)(offsetof(TabuLaunchArgs, k0) >=
                      offsetof(TabuLaunchArgs, class_end) + kWalkClasses * sizeof(int64_t)));
    // every subset of present classes, as a batch of one walk per present class
    for (int mask = 0; mask < (1 << kWalkClasses); ++mask)
        for (int split = 0; split < 2; ++split)
            for (int lanes : {64, 32, 16}) {
                int64_t ce[kWalkClasses];
                int64_t end = 0;
                for (int c = 0; c < kWalkClasses; ++c) ce[c] = end += (mask >> c) & 1;
                const WalkGroups g = walk_launch_groups(ce, split != 0, lanes);
                std::printf("groups %d %d %d %d", mask, split, lanes, g.n);
                for (int i = 0; i < g.n; ++i) std::printf(" %d:%d:%d", g.first[i], g.last[i], g.kind[i]);
                std::printf("\n");
            }
    return 0;
}
