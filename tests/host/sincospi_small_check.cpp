// Host build of the encoding's sin/cos(pi t): 4M seeded arguments t = 2^k v (v uniform in
// [-1, 1], k = 0..7) against the FP64 library, and the multiples of 1/2 (exact values expected).
#include <cmath>
#include <cstdio>
#include <random>

#include "nirc_device.hpp"

int main() {
    std::mt19937 gen(1);
    std::uniform_real_distribution<float> U(-1.0f, 1.0f);
    double max_s = 0.0, max_c = 0.0;
    for (int it = 0; it < (1 << 22); ++it) {
        const float t = std::ldexp(U(gen), it & 7);
        float s, c;
        nirc::sincospi_small(t, s, c);
        max_s = std::fmax(max_s, std::fabs((double)s - std::sin(M_PI * (double)t)));
        max_c = std::fmax(max_c, std::fabs((double)c - std::cos(M_PI * (double)t)));
    }
    int inexact = 0;
    for (int h = -256; h <= 256; ++h) {   // t = h / 2
        float s, c;
        nirc::sincospi_small(0.5f * (float)h, s, c);
        const int q = ((h % 4) + 4) % 4;
        const float es = q == 1 ? 1.0f : q == 3 ? -1.0f : 0.0f, ec = q == 0 ? 1.0f : q == 2 ? -1.0f : 0.0f;
        if (s != es || c != ec) ++inexact;
    }
    std::printf("%.6e %.6e %d\n", max_s, max_c, inexact);
    return 0;
}
