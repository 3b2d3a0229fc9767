// Brute-force check of the bitmap neighbour index on random periodic images:
// for every fluid node, the pull sources decoded from its packed coordinate
// and the nine row records around it (one record per row: fluid bits, the
// next word's bits, node number before the word, fluid count of the row)
// must equal the sources of the plain neighbour table -- the node at x - c_i,
// or -1 where that voxel is solid.  The decode below is a CPU model of the
// step kernel's: the window of voxels x - 1, x, x + 1 is three bits of the
// row string starting at padded position x, their node numbers follow from
// a population count, and the x wrap uses the row's fluid count.  Exit
// status 0 when every case holds.
#include "lbm_host.hpp"
#include <cstdio>
#include <random>
#include <vector>
using namespace lbm;

namespace {
struct Row3 {
    int64_t rm, r0, rp;
    uint32_t bits;
};
Row3 decode(const RowRec& w, int x, int nx) {
    const uint32_t sh = (uint32_t)x & 31u;
    const uint64_t pair = ((uint64_t)w.next << 32) | w.bits;
    Row3 r;
    r.bits = (uint32_t)(pair >> sh) & 7u;
    const uint32_t below = (uint32_t)__builtin_popcount(sh == 0 ? 0u : (w.bits & ((1u << sh) - 1u)));
    r.r0 = (int64_t)w.base + below + (r.bits & 1u);
    r.rm = r.r0 - 1 + (x == 0 ? w.count : 0);
    r.rp = r.r0 + ((r.bits >> 1) & 1u) - (x == nx - 1 ? w.count : 0);
    return r;
}
// source node of the voxel at offset dx (-1, 0, +1) in the decoded row, or -1
int64_t pick(const Row3& w, int dx) {
    if (!((w.bits >> (dx + 1)) & 1u)) return -1;
    return dx < 0 ? w.rm : (dx == 0 ? w.r0 : w.rp);
}
}  // namespace

int main() {
    std::mt19937 rng(11);
    int bad = 0, cases = 0;
    const int edge_nx[] = {1, 2, 3, 29, 30, 31, 32, 33, 34, 62, 63, 64, 65, 66, 95, 96, 97};
    for (int it = 0; it < 400; ++it) {
        int nx = it < 17 ? edge_nx[it] : 1 + (int)(rng() % 100);
        int ny = 1 + (int)(rng() % 9), nz = 1 + (int)(rng() % 40);
        double phi = (rng() % 100) / 100.0;
        std::vector<uint8_t> g((size_t)nx * ny * nz);
        std::uniform_real_distribution<double> U(0, 1);
        for (auto& v : g) v = U(rng) < phi ? 0 : 1;
        int64_t nf = count_fluid(g.data(), nx, ny, nz);
        if (nf == 0) continue;
        CoordBits cb = coord_bits(nx, ny, nz);
        if (!cb.fits()) continue;
        ++cases;
        int64_t np = padded(nf);
        std::vector<int32_t> t((size_t)18 * np, -1);
        build_table(g.data(), nx, ny, nz, nf, np, t.data());
        BitmapIndex bm;
        build_bitmap(g.data(), nx, ny, nz, nf, &bm);
        const int R = bm.recs_per_row;
        if ((int64_t)bm.rec.size() != (int64_t)ny * nz * R) { ++bad; continue; }
        for (int64_t n = 0; n < nf; ++n) {
            const uint32_t c = bm.coords[n];
            const int x = (int)(c & ((1u << cb.bx) - 1u));
            const int y = (int)((c >> cb.bx) & ((1u << cb.by) - 1u));
            const int z = (int)((uint64_t)c >> (cb.bx + cb.by));
            auto row = [&](int dy, int dz) {
                const int yy = (y + dy + ny) % ny, zz = (z + dz + nz) % nz;
                return decode(bm.rec[((int64_t)zz * ny + yy) * R + (x >> 5)], x, nx);
            };
            for (int i = 1; i < 19; ++i) {
                // the source voxel is x - c_i
                const int64_t got = pick(row(-kC[i][1], -kC[i][2]), -kC[i][0]);
                const int64_t want = t[(size_t)(i - 1) * np + n];
                if (got != want) {
                    if (bad < 10)
                        printf("BAD dims %d %d %d node %lld (x %d y %d z %d) dir %d got %lld want %lld\n", nx, ny, nz,
                               (long long)n, x, y, z, i, (long long)got, (long long)want);
                    ++bad;
                }
            }
        }
    }
    printf("cases %d bad %d\n", cases, bad);
    return bad != 0;
}
