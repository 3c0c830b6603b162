// Host build of the hash-grid model's packed layouts (16-bit, then FP32): prints, for every packed
// element, its canonical source (or -1), so that the test can check coverage.
#include <cstdio>

#include "nirc_hash.hpp"

int main() {
    std::printf("%d %d %d %d %d\n", nirc::kHashPacked, nirc::kHashSecD, nirc::kHashRest, nirc::kHashSecTS,
                nirc::hash_sec(nirc::SEC_T0));
    for (int e = 0; e < nirc::kHashPacked; ++e) std::printf("%lld\n", (long long)nirc::hash_packed_source(e));
    std::printf("%d %d %d\n", nirc::kHash32Packed, nirc::kHash32S + nirc::kHash32D, nirc::kHash32TS);
    for (int e = 0; e < nirc::kHash32Packed; ++e) std::printf("%lld\n", (long long)nirc::hash_packed_source32(e));
    return 0;
}
