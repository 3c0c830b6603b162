// Host build of the kernels' grid lookup (cell, corner entries and weights, fetch and blend):
// reads a table and positions from binary files, prints the 24 grid values of every position
// (lane groups 0..3, levels 3g..3g+2, two features each), in canonical order 2 l + f.
#include <cstdio>
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
    while (std::fread(x, sizeof(float), 3, fp) == 3) {
        for (int g = 0; g < 4; ++g) {
            float v[6];
            nirc::hash_values6(args.lv, args.tmask, table.data(), x[0], x[1], x[2], g, v);
            for (int j = 0; j < 6; ++j) std::printf("%.9e%c", v[j], (g == 3 && j == 5) ? '\n' : ' ');
        }
    }
    std::fclose(fp);
    return 0;
}
