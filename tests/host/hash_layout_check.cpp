// Host build of the hash-grid model's packed 16-bit layout: prints, for every packed element, its
// section-relative position and canonical source (or -1), so that the test can check coverage.
#include <cstdio>

#include "nirc_hash.hpp"

int main() {
    std::printf("%d %d %d %d %d\n", nirc::kHashPacked, nirc::kHashSecD, nirc::kHashRest, nirc::kHashSecTS,
                nirc::hash_sec(nirc::SEC_T0));
    for (int e = 0; e < nirc::kHashPacked; ++e) std::printf("%lld\n", (long long)nirc::hash_packed_source(e));
    return 0;
}
