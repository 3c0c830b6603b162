// Host build of the direction sampler's sin/cos(2 pi u): every 24-bit uniform u = k 2^-24 is
// evaluated and compared with the FP64 library functions; prints the largest absolute errors.
#include <cmath>
#include <cstdio>

#include "nirc_device.hpp"

int main() {
    double max_s = 0.0, max_c = 0.0;
    for (unsigned k = 0; k < (1u << 24); ++k) {
        const float u = (float)k * 0x1p-24f;
        float s, c;
        nirc::sincos_turns(u, s, c);
        const double a = 2.0 * M_PI * (double)u;
        max_s = std::fmax(max_s, std::fabs((double)s - std::sin(a)));
        max_c = std::fmax(max_c, std::fabs((double)c - std::cos(a)));
    }
    std::printf("%.6e %.6e\n", max_s, max_c);
    return 0;
}
