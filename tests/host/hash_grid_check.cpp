// Host build of the kernels' grid lookup (cell, corner entries and weights, fetch and blend):
// reads a table and positions from binary files, prints the 24 grid values of every position
// (lane groups 0..3, levels 3g..3g+2, two features each), in canonical order 2 l + f.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "nirc_hash.hpp"

int main(int argc, char **argv) {
    if (argc != 6) return 2;
    nirc_hash_grid grid{std::atoi(argv[3]), std::atoi(argv[4]), (float)std::atof(argv[5])};
    nirc::HashGridArgs args;
    const int64_t entries = nirc::hash_grid_setup(grid, &args);
    if (entries <= 0) return 3;
    std::vector<float2> table((size_t)entries);
    FILE *ft = std::fopen(argv[1], "rb");
    if (!ft || std::fread(table.data(), sizeof(float2), table.size(), ft) != table.size()) return 4;
    std::fclose(ft);
    FILE *fp = std::fopen(argv[2], "rb");
    if (!fp) return 5;
    float x[3];
    long mismatch = 0;
    double max_w = 0.0;
    while (std::fread(x, sizeof(float), 3, fp) == 3) {
        for (int g = 0; g < 4; ++g) {
            float v[6];
            nirc::hash_values6(args.lv, args.tmask, table.data(), x[0], x[1], x[2], g, v);
            for (int j = 0; j < 6; ++j) std::printf("%.9e%c", v[j], (g == 3 && j == 5) ? '\n' : ' ');
            // the training scatter's per-corner entries and weights (hash_entry) against the fetch:
            // same features corner by corner, and the same blend
            float2 t[24];
            nirc::hash_fetch24(args.lv, args.tmask, table.data(), x[0], x[1], x[2], g, t);
            for (int k = 0; k < 3; ++k) {
                const nirc::HashLevel lv = args.lv[3 * g + k];
                const nirc::HashCell h = nirc::hash_cell(x[0], x[1], x[2], lv.res);
                double a = 0.0;
                for (int c = 0; c < 8; ++c) {
                    float w;
                    const uint32_t e = nirc::hash_entry(lv, args.tmask, h, c, w);
                    if (table[e].x != t[8 * k + c].x || table[e].y != t[8 * k + c].y) ++mismatch;
                    a += (double)w * table[e].x;
                }
                max_w = std::fmax(max_w, std::fabs(a - (double)v[2 * k]));
            }
        }
    }
    std::fclose(fp);
    std::fprintf(stderr, "%ld %.3e\n", mismatch, max_w);
    return 0;
}
