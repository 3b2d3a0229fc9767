// Brute-force check of the bitmap neighbour index on random periodic images:
// for every fluid node, the pull sources decoded from its packed coordinate
// and the records of its nine rows must equal the sources of the plain
// neighbour table -- the node at x - c_i, or -1 where that voxel is solid --
// and every record load must lie inside the record array.  The decode below
// is a CPU model of the step kernel's: entry (z, y, w) holds the 8-byte
// records of word w of rows y - 1, y, y + 1 of plane z; a node reads the
// entries (z - 1, y, w), (z, y, w), (z + 1, y, w) with w = x / 18; the window
// of voxels x - 1, x, x + 1 is three bits of a record starting at position
// x mod 18, node numbers follow from a population count, and the x wrap uses
// the row's fluid count.  With symmetry planes on the y and/or z faces
// (build_bitmap's mirror_y; the kernel reads plane z itself for z - 1 at
// z = 0 and for z + 1 at z = nz - 1 when the z faces are mirrors) the source
// of a pull that leaves the box through such a face is the voxel reached by
// the step's other components, the image's own boundary layer; every node's
// decoded sources are compared with that rule written out here.  Exit status
// 0 when every case holds.
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
    const uint32_t sh = (uint32_t)(x % kWordStep);
    const int64_t count = (int64_t)(w.lo >> 20);
    Row3 r;
    r.bits = (w.lo >> sh) & 7u;
    const uint32_t below = (uint32_t)__builtin_popcount(w.lo & ((1u << sh) - 1u));
    r.r0 = (int64_t)w.base + below + (r.bits & 1u);
    r.rm = r.r0 - 1 + (x == 0 ? count : 0);
    r.rp = r.r0 + ((r.bits >> 1) & 1u) - (x == nx - 1 ? count : 0);
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
    const int edge_nx[] = {1, 2, 3, 16, 17, 18, 19, 20, 35, 36, 37, 38, 53, 54, 55, 56, 57};
    for (int it = 0; it < 400; ++it) {
        int nx = it < 17 ? edge_nx[it] : 1 + (int)(rng() % 100);
        int ny = 1 + (int)(rng() % 9), nz = 1 + (int)(rng() % 40);
        double phi = (rng() % 100) / 100.0;
        if (it == 17 || it == 18) {  // the longest rows the 12-bit count holds, nearly or fully fluid
            nx = kBitmapMaxNx;
            ny = 2;
            nz = 3;
            phi = it == 17 ? 0.97 : 1.0;
        }
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
        // node number of every voxel (-1 solid), for the mirrored sources
        std::vector<int64_t> node((size_t)nx * ny * nz, -1);
        {
            std::vector<int64_t> vox(nf);
            fluid_voxels(g.data(), nx, ny, nz, vox.data());
            for (int64_t n = 0; n < nf; ++n) node[vox[n]] = n;
        }
        for (int mirror = 0; mirror < 4; ++mirror) {
        const bool my = mirror & 1, mz = mirror & 2;
        BitmapIndex bm;
        build_bitmap(g.data(), nx, ny, nz, nf, &bm, my);
        const int W = bm.words;
        const int64_t bytes = (int64_t)bm.rec.size() * 8;
        if (W != words_per_row(nx) || (int64_t)bm.rec.size() != (int64_t)nz * ny * W * 3) { ++bad; continue; }
        for (int64_t n = 0; n < nf; ++n) {
            const uint32_t c = bm.coords[n];
            const int x = (int)(c & ((1u << cb.bx) - 1u));
            const int y = (int)((c >> cb.bx) & ((1u << cb.by) - 1u));
            const int z = (int)((uint64_t)c >> (cb.bx + cb.by));
            // the kernel's byte offsets: entry (zz, y, w), 16 then 8 bytes
            RowRec rows[3][3];  // [plane z-1, z, z+1][row y-1, y, y+1]
            for (int dz = -1; dz <= 1; ++dz) {
                int zz = (z + dz + nz) % nz;
                if (mz && (z + dz < 0 || z + dz >= nz)) zz = z;   // ghost plane: the boundary plane itself
                const int64_t o = (((int64_t)zz * ny + y) * W + x / kWordStep) * 24;
                if (o < 0 || o + 24 > bytes || o % 8 != 0) {
                    if (bad < 10) printf("OUT dims %d %d %d node %lld offset %lld bytes %lld\n", nx, ny, nz,
                                         (long long)n, (long long)o, (long long)bytes);
                    ++bad;
                    continue;
                }
                for (int k = 0; k < 3; ++k) rows[dz + 1][k] = bm.rec[o / 8 + k];
            }
            for (int i = 1; i < 19; ++i) {
                // the source voxel is x - c_i
                const Row3 r = decode(rows[1 - kC[i][2]][1 - kC[i][1]], x, nx);
                const int64_t got = pick(r, -kC[i][0]);
                int64_t want = t[(size_t)(i - 1) * np + n];
                if (my || mz) {
                    int sx = (x - kC[i][0] + nx) % nx, sy = y - kC[i][1], sz = z - kC[i][2];
                    sy = sy < 0 || sy >= ny ? (my ? y : (sy + ny) % ny) : sy;
                    sz = sz < 0 || sz >= nz ? (mz ? z : (sz + nz) % nz) : sz;
                    want = node[sx + (int64_t)nx * (sy + (int64_t)ny * sz)];
                }
                if (got != want) {
                    if (bad < 10)
                        printf("BAD dims %d %d %d mirror %d node %lld (x %d y %d z %d) dir %d got %lld want %lld\n",
                               nx, ny, nz, mirror, (long long)n, x, y, z, i, (long long)got, (long long)want);
                    ++bad;
                }
            }
        }
        }
    }
    printf("cases %d bad %d\n", cases, bad);
    return bad != 0;
}
