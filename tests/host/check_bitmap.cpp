// Brute-force check of the bitmap neighbour index on random periodic images:
// for every fluid node, the pull sources decoded from its packed coordinate
// and the entries of its three planes must equal the sources of the plain
// neighbour table -- the node at x - c_i, or -1 where that voxel is solid --
// and every load must lie inside its array.  The decode below is a CPU model
// of the step kernel's: entry (z, y, w) holds word w's 20 bits of rows y - 1,
// y, y + 1 of plane z, the base of the word in row y and the 18-bit
// differences to the bases in rows y - 1 and y + 1; a node reads the entries
// (z - 1, y, w), (z, y, w), (z + 1, y, w) with w = x / 18, across the
// periodic y wrap the wrapped row's bases from one slot of the wrap array, and
// at the x wrap the five rows' fluid counts from one slot of the count array;
// the window of voxels x - 1, x, x + 1 is three bits starting
// at position x mod 18 and node numbers follow from a population count.  With
// symmetry planes on the y and/or z faces (build_bitmap's mirror_y and
// mirror_z; the kernel reads plane z itself for z - 1 at z = 0 and for z + 1 at z = nz - 1 when the
// z faces are mirrors) the source of a pull that leaves the box through such a
// face is the voxel reached by the step's other components, the image's own
// boundary layer; every node's decoded sources are compared with that rule
// written out here.  Exit status 0 when every case holds.
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
Row3 decode(uint32_t lo, int64_t base, int64_t count, int x, int nx) {
    const uint32_t sh = (uint32_t)(x % kWordStep);
    Row3 r;
    r.bits = (lo >> sh) & 7u;
    const uint32_t below = (uint32_t)__builtin_popcount(lo & ((1u << sh) - 1u));
    r.r0 = base + below + (r.bits & 1u);
    r.rm = r.r0 - 1 + (x == 0 ? count : 0);
    r.rp = r.r0 + ((r.bits >> 1) & 1u) - (x == nx - 1 ? count : 0);
    return r;
}
int64_t sext18(uint32_t v) { return (int64_t)((int32_t)(v << 14) >> 14); }
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
        if (it == 17 || it == 18) {  // the longest rows the bitmap index holds, nearly or fully fluid
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
        build_bitmap(g.data(), nx, ny, nz, nf, &bm, my, mz);
        const int W = bm.words;
        const int64_t nent = (int64_t)nz * ny * W;
        const int64_t nwrap = (int64_t)nz * 2 * W, nrow = (int64_t)nz * ny;
        if (W != words_per_row(nx) || !bm.fits || (int64_t)bm.ent.size() != nent * 4 ||
            (int64_t)bm.wrap.size() != nwrap * 4 || (int64_t)bm.count.size() != nrow * 4) { ++bad; continue; }
        auto in = [&](int64_t i, int64_t size, const char* what, int64_t n) {
            if (i >= 0 && i < size) return true;
            if (bad < 10) printf("OUT %s dims %d %d %d node %lld index %lld size %lld\n", what, nx, ny, nz,
                                 (long long)n, (long long)i, (long long)size);
            ++bad;
            return false;
        };
        for (int64_t n = 0; n < nf; ++n) {
            const uint32_t c = bm.coords[n];
            const int x = (int)(c & ((1u << cb.bx) - 1u));
            const int y = (int)((c >> cb.bx) & ((1u << cb.by) - 1u));
            const int z = (int)((uint64_t)c >> (cb.bx + cb.by));
            const int w = x / kWordStep;
            // the kernel's loads: three entries, the wrapped rows' bases, the counts
            int64_t ek[3];
            uint32_t E[3][4];
            bool ok = true;
            for (int k = 0; k < 3; ++k) {
                const int dz = k - 1;
                int zz = (z + dz + nz) % nz;
                if (mz && (z + dz < 0 || z + dz >= nz)) zz = z;   // ghost plane: the boundary plane itself
                ek[k] = ((int64_t)zz * ny + y) * W + w;
                ok = ok && in(ek[k], nent, "entry", n);
                if (ok)
                    for (int q = 0; q < 4; ++q) E[k][q] = bm.ent[(size_t)ek[k] * 4 + q];
            }
            if (!ok) continue;
            const bool ywrap = ny > 1 && !my;
            const bool wm = ywrap && y == 0, wp = ywrap && y == ny - 1;
            int64_t fb[3] = {0, 0, 0};
            if (wm || wp) {
                const int64_t i = ((int64_t)z * 2 + (wm ? 0 : 1)) * W + w;
                if (in(i, nwrap, "wrap", n))
                    for (int k = 0; k < 3; ++k) fb[k] = (int32_t)bm.wrap[(size_t)i * 4 + k];
            }
            int64_t cnt[5] = {0, 0, 0, 0, 0};
            if (x == 0 || x == nx - 1) {
                const int64_t i = (int64_t)z * ny + y;
                if (in(i, nrow, "count", n)) {
                    const uint32_t* v = &bm.count[(size_t)i * 4];
                    cnt[0] = v[0] & 0xffffu;
                    cnt[1] = v[0] >> 16;
                    cnt[2] = v[1] & 0xffffu;
                    cnt[3] = v[1] >> 16;
                    cnt[4] = v[2];
                }
            }
            // rows[plane z-1, z, z+1][row y-1, y, y+1]
            Row3 rows[3][3];
            for (int k = 0; k < 3; ++k) {
                const int64_t b0 = (int32_t)E[k][3];
                const int64_t dm = sext18((E[k][0] >> 20) | ((E[k][2] >> 20) & 63u) << 12);
                const int64_t dp = sext18((E[k][1] >> 20) | ((E[k][2] >> 26) & 63u) << 12);
                const int64_t cm = k == 1 ? cnt[1] : 0, c0 = k == 1 ? cnt[0] : (k == 0 ? cnt[3] : cnt[4]),
                              cp = k == 1 ? cnt[2] : 0;
                rows[k][0] = decode(E[k][0] & 0xfffffu, wm ? fb[k] : b0 + dm, cm, x, nx);
                rows[k][1] = decode(E[k][1] & 0xfffffu, b0, c0, x, nx);
                rows[k][2] = decode(E[k][2] & 0xfffffu, wp ? fb[k] : b0 + dp, cp, x, nx);
            }
            for (int i = 1; i < 19; ++i) {
                // the source voxel is x - c_i
                const Row3& r = rows[1 - kC[i][2]][1 - kC[i][1]];
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
