// Host build of both packed layouts' two directions: for widths 64 and 128, every packed
// element's canonical source (h16_packed_source, f32_packed_source) against the targets each
// canonical parameter lists (h16_packed_targets with the stored scales, f32_packed_targets).
// Prints "W mismatches params elements listed" for the 16-bit layout, then the same with a
// leading 32 for the FP32 layout.
#include <cstdio>
#include <set>
#include <utility>
#include <vector>

#include "nirc_h16.hpp"

int main() {
    for (int W : {64, 128}) {
        const nirc::H16Layout L{W};
        const int64_t np = nirc::n_params(W);
        std::vector<std::set<int>> fwd(np);
        int used = 0;
        for (int e = 0; e < L.total(); ++e) {
            const int64_t s = nirc::h16_packed_source(W, e);
            if (s >= 0) {
                fwd[s].insert(e);
                ++used;
            }
        }
        int bad = 0, listed = 0;
        for (int64_t i = 0; i < np; ++i) {
            int e[6];
            float sc[6];
            const int n = nirc::h16_packed_targets(W, i, e, sc);
            std::set<int> got;
            for (int k = 0; k < n; ++k) {
                got.insert(e[k]);
                if (e[k] < 0 || e[k] >= L.total() || sc[k] != nirc::h16_packed_scale(W, e[k])) ++bad;
            }
            listed += n;
            if (got != fwd[i] || (int)got.size() != n) ++bad;
        }
        std::printf("%d %d %lld %d %d\n", W, bad, (long long)np, used, listed);
    }
    for (int W : {64, 128}) {
        const nirc::F32Layout L{W};
        const int64_t np = nirc::n_params(W);
        std::vector<std::set<int>> fwd(np);
        int used = 0;
        for (int e = 0; e < L.total(); ++e) {
            const int64_t s = nirc::f32_packed_source(W, e);
            if (s >= 0) {
                fwd[s].insert(e);
                ++used;
            }
        }
        int bad = 0, listed = 0;
        for (int64_t i = 0; i < np; ++i) {
            int e[2];
            const int n = nirc::f32_packed_targets(W, i, e);
            std::set<int> got;
            for (int k = 0; k < n; ++k) {
                got.insert(e[k]);
                if (e[k] < 0 || e[k] >= L.total()) ++bad;
            }
            listed += n;
            if (got != fwd[i] || (int)got.size() != n) ++bad;
        }
        std::printf("32 %d %d %lld %d %d\n", W, bad, (long long)np, used, listed);
    }
    return 0;
}
