// Host build of the device's spherical harmonics: reads directions (x y z per line) from stdin
// and prints the 25 values for each.
#include <cstdio>

#include "nirc_hash.hpp"

int main() {
    float x, y, z;
    while (std::scanf("%f %f %f", &x, &y, &z) == 3) {
        float Y[25];
        nirc::sh25(x, y, z, Y);
        for (int i = 0; i < 25; ++i) std::printf("%.9e%c", Y[i], i == 24 ? '\n' : ' ');
    }
    return 0;
}
