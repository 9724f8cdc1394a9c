// Host build of the GPU path's geometry (csrc/geometry.hpp) for the
// CPU test-suite: writes every entry of A (ray-driven, mode "ray") or of A^T
// (voxel-driven, mode "voxel") as binary records {int32 row, int32 col,
// float64 length} to the file named on the command line.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../paper_2009_07226_amd/csrc/geometry.hpp"

int main(int argc, char **argv) {
    if (argc != 6) return 2;
    const bool ray = std::strcmp(argv[1], "ray") == 0;
    const int N = std::atoi(argv[2]), M = std::atoi(argv[3]), C = std::atoi(argv[4]);
    FILE *f = std::fopen(argv[5], "wb");
    if (!f) return 3;
    struct Rec { int32_t r, c; double v; };
    if (ray) {
        for (int k = 0; k < M; ++k)
            for (int c = 0; c < C; ++c)
                xct::trace_ray(N, M, C, k, c, [&](int i, int j, double len) {
                    Rec q{k * C + c, i * N + j, len};
                    std::fwrite(&q, sizeof q, 1, f);
                });
    } else {
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                xct::trace_voxel(N, M, C, i, j, [&](int k, int c, double len) {
                    Rec q{i * N + j, k * C + c, len};
                    std::fwrite(&q, sizeof q, 1, f);
                });
    }
    std::fclose(f);
    return 0;
}
