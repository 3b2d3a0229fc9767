// Brute-force check of the chunked population layout and its gather span on
// random periodic images, for the tile height the image gets and for fixed
// ones: every element a node's step touches (pull sources,
// bounce-back own populations, own stores) must lie inside the population
// array and within [chunk_base - slack, chunk_base + reach) of its chunk, and
// the node order must be a permutation of the fluid voxels.  Exit status 0
// when every case holds.
#include "lbm_host.hpp"
#include <cstdio>
#include <random>
#include <vector>
using namespace lbm;
int main() {
    std::mt19937 rng(5);
    int bad = 0, cases = 0;
    for (int it = 0; it < 300; ++it) {
        int nx = 1 + rng() % 40, ny = 1 + rng() % 40, nz = 1 + rng() % 90;
        double phi = (rng() % 100) / 100.0;
        std::vector<uint8_t> g((size_t)nx * ny * nz);
        std::uniform_real_distribution<double> U(0, 1);
        for (auto& v : g) v = U(rng) < phi ? 0 : 1;
        int64_t nf = count_fluid(g.data(), nx, ny, nz);
        if (nf == 0) continue;
        ++cases;
        int64_t np = padded(nf);
        for (int tz : {node_tile_z(g.data(), nx, ny, nz), 1, 2, 3, 16})  // the image's height and fixed ones
        for (int S : {19, 20}) {  // 19 populations, and 20 values per node as a check of the layout's generality
            std::vector<int32_t> t((size_t)18 * np, -1);
            build_table(g.data(), nx, ny, nz, nf, np, t.data(), tz);
            auto st = row_starts(g.data(), nx, ny, nz, tz);
            GatherSpan sp = gather_span(st, ny, nz, tz, S);
            const int64_t E = (int64_t)S * kChunk;
            for (int64_t n = 0; n < nf; ++n) {
                int64_t cb = (n / kChunk) * E;
                auto check = [&](int64_t e) {
                    int64_t rel = e - cb + sp.slack;
                    if (rel < 0 || rel >= sp.slack + sp.reach || e < 0 || e >= S * np) {
                        if (bad < 10) printf("BAD S=%d n=%lld e=%lld cb=%lld slack=%lld reach=%lld dims %d %d %d\n",
                                             S, (long long)n, (long long)e, (long long)cb, (long long)sp.slack,
                                             (long long)sp.reach, nx, ny, nz);
                        ++bad;
                    }
                };
                check(state_elem(0, n, S));
                check(state_elem(S - 1, n, S));
                for (int i = 1; i < 19; ++i) {
                    int32_t s = t[(size_t)(i - 1) * np + n];
                    check(s >= 0 ? state_elem(i, s, S) : state_elem(opposite(i), n, S));
                    check(s >= 0 ? state_elem(S - 1, s, S) : state_elem(S - 1, n, S));
                    check(state_elem(i, n, S));
                }
            }
        }
        // node order is a permutation of the fluid voxels
        std::vector<int64_t> vox(nf);
        fluid_voxels(g.data(), nx, ny, nz, vox.data());
        std::vector<char> seen((size_t)nx * ny * nz, 0);
        for (auto v : vox) { if (g[v] != 0 || seen[v]) { ++bad; } seen[v] = 1; }
    }
    // The tile height of an image is the tallest candidate whose span fits
    // 32-bit byte offsets with 4-byte elements: on a fully fluid 512^3 box
    // (134 M nodes) 32 planes fit and 64 do not.
    {
        const int n = 512;
        std::vector<uint8_t> g((size_t)n * n * n, 0);
        const int tz = node_tile_z(g.data(), n, n, n);
        auto fits = [&](int h) {
            GatherSpan sp = gather_span(row_starts(g.data(), n, n, n, h), n, n, h, 19);
            return (double)(sp.slack + sp.reach) * 4 < 4294967296.0;
        };
        printf("512^3 fluid box: tile height %d\n", tz);
        if (tz != 32 || !fits(32) || fits(64)) ++bad;
    }
    // ... and whose rows y -/+ 1 stay within the bitmap index's 18-bit base
    // differences, (h + 1) nx + 1 < 2^17: 4095-voxel rows allow 16 planes,
    // however small the span.
    {
        const int nx = 4095, ny = 3, nz = 200;
        std::vector<uint8_t> g((size_t)nx * ny * nz, 0);
        const int tz = node_tile_z(g.data(), nx, ny, nz);
        printf("4095 x 3 x 200 fluid box: tile height %d\n", tz);
        if (tz != 16) ++bad;
    }
    printf("cases %d bad %d\n", cases, bad);
    return bad != 0;
}
