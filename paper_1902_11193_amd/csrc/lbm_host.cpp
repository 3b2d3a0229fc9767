// Host-side setup for liblbm: relaxation rates (Table 2 of Rao & Schaefer,
// arXiv:1902.11193) and compaction of the segmented image into the fluid-node
// list with its neighbour index.
#include "lbm_host.hpp"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <thread>

namespace lbm {

const int kC[19][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};

// Table 2.  s_nu = 1/tau on the shear moments in every set.  With s = s_nu:
//   a = 8 (2 - s) / (8 - s)    (Set A kinetic rates; s_q, s_m of Set B; s_q of Set D)
//   b = 4 (2 - s) / (4 + s)    (s_m of Set D)
//   e = 2 (2 - s) / (4 Lambda s - s + 2)   (odd rates of Set E, Eq. Magic param)
// Set C uses the constants of d'Humieres et al. 2002 (the values in Table 2).
std::string rates(int set, double tau, double Lambda, RateClasses* out, RateClasses* dtau,
                  RateClasses* dlam) {
    if (!std::isfinite(tau) || !(tau > 0.5)) return "tau must be finite and > 1/2";
    if (set < 0 || set > 5) return "relaxation_set must be 0 (SRT) .. 5 (Set E)";
    if (set == 5 && (!std::isfinite(Lambda) || !(Lambda > 0)))
        return "Set E needs a finite Lambda > 0";
    const double s = 1.0 / tau, dsdt = -1.0 / (tau * tau);
    const double a = 8 * (2 - s) / (8 - s), da = -48.0 / ((8 - s) * (8 - s));
    const double b = 4 * (2 - s) / (4 + s), db = -24.0 / ((4 + s) * (4 + s));
    RateClasses r{}, dt{}, dl{};
    r.s_nu = s;
    dt.s_nu = dsdt;
    switch (set) {
        case 0:  // SRT
            r = {s, s, s, s, s, s};
            dt = {dsdt, dsdt, dsdt, dsdt, dsdt, dsdt};
            break;
        case 1:  // Set A
            r = {a, a, a, s, a, a};
            dt = {da * dsdt, da * dsdt, da * dsdt, dsdt, da * dsdt, da * dsdt};
            break;
        case 2:  // Set B
            r = {s, s, a, s, s, a};
            dt = {dsdt, dsdt, da * dsdt, dsdt, dsdt, da * dsdt};
            break;
        case 3:  // Set C
            r = {1.19, 1.4, 1.2, s, 1.4, 1.98};
            dt = {0, 0, 0, dsdt, 0, 0};
            break;
        case 4:  // Set D
            r = {s, s, a, s, s, b};
            dt = {dsdt, dsdt, da * dsdt, dsdt, dsdt, db * dsdt};
            break;
        case 5: {  // Set E
            const double den = 4 * Lambda * s - s + 2;
            const double e = 2 * (2 - s) / den;
            const double de_ds = -16.0 * Lambda / (den * den);
            const double de_dl = -8.0 * s * (2 - s) / (den * den);
            r = {s, s, e, s, s, e};
            dt = {dsdt, dsdt, de_ds * dsdt, dsdt, dsdt, de_ds * dsdt};
            dl = {0, 0, de_dl, 0, 0, de_dl};
            break;
        }
    }
    const double all[6] = {r.s_e, r.s_eps, r.s_q, r.s_nu, r.s_pi, r.s_m};
    for (double v : all)
        if (!(v > 0 && v < 2)) return "a relaxation rate falls outside (0, 2)";
    if (out) *out = r;
    if (dtau) *dtau = dt;
    if (dlam) *dlam = dl;
    return "";
}

void rates_to_moments(const RateClasses& r, double s[19]) {
    const double v[19] = {0,      r.s_e,  r.s_eps, 0,      r.s_q,  0,      r.s_q,
                          0,      r.s_q,  r.s_nu,  r.s_pi, r.s_nu, r.s_pi, r.s_nu,
                          r.s_nu, r.s_nu, r.s_m,   r.s_m,  r.s_m};
    std::copy(v, v + 19, s);
}

std::string check_dims(int nx, int ny, int nz) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return "dimensions must be positive";
    if ((int64_t)nx * ny * nz > (int64_t)1 << 40) return "image too large";
    return "";
}

namespace {
int nthreads_for(int64_t work) {
    unsigned hw = std::thread::hardware_concurrency();
    int t = (int)std::min<unsigned>(hw ? hw : 4, 16);
    if (work < (1 << 20)) t = 1;
    return t;
}

// Run f(z0, z1) over [0, nz) in parallel slabs.
template <class F>
void parallel_slabs(int nz, int64_t work, F&& f) {
    int t = std::min(nthreads_for(work), nz);
    if (t <= 1) {
        f(0, nz);
        return;
    }
    std::vector<std::thread> th;
    for (int k = 0; k < t; ++k) {
        int z0 = (int)((int64_t)nz * k / t), z1 = (int)((int64_t)nz * (k + 1) / t);
        th.emplace_back([=, &f] { f(z0, z1); });
    }
    for (auto& x : th) x.join();
}

int bits_for(int n) {
    int b = 0;
    while ((1ll << b) < n) ++b;
    return b;
}

// Number of fluid voxels before each z-slab (exclusive prefix), size nz + 1.
std::vector<int64_t> slab_offsets(const uint8_t* g, int nx, int ny, int nz) {
    std::vector<int64_t> cnt(nz + 1, 0);
    const int64_t plane = (int64_t)nx * ny;
    parallel_slabs(nz, plane * nz, [&](int z0, int z1) {
        for (int z = z0; z < z1; ++z) {
            int64_t c = 0;
            const uint8_t* p = g + plane * z;
            for (int64_t i = 0; i < plane; ++i) c += (p[i] == 0);
            cnt[z + 1] = c;
        }
    });
    for (int z = 0; z < nz; ++z) cnt[z + 1] += cnt[z];
    return cnt;
}
}  // namespace

namespace {
// Fluid voxels of every row r = z * ny + y.
std::vector<int64_t> row_counts(const uint8_t* g, int nx, int ny, int nz) {
    const int64_t rows = (int64_t)ny * nz;
    std::vector<int64_t> cnt(rows, 0);
    parallel_slabs(nz, rows * nx, [&](int z0, int z1) {
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < ny; ++y) {
                const uint8_t* p = g + ((int64_t)z * ny + y) * nx;
                int64_t c = 0;
                for (int x = 0; x < nx; ++x) c += (p[x] == 0);
                cnt[(int64_t)z * ny + y] = c;
            }
    });
    return cnt;
}

// First node of every row in the order with z-tiles of tile_z planes.
std::vector<int64_t> order_rows(const std::vector<int64_t>& cnt, int ny, int nz, int tile_z) {
    const int64_t rows = (int64_t)ny * nz;
    std::vector<int64_t> start(rows + 1, 0);
    int64_t n = 0;
    const int T = (nz + tile_z - 1) / tile_z;
    for (int p = 0; p < T; ++p) {
        const int z0 = tile_at(p, T) * tile_z;
        for (int y = 0; y < ny; ++y)
            for (int z = z0; z < std::min(nz, z0 + tile_z); ++z) {
                const int64_t r = (int64_t)z * ny + y;
                start[r] = n;
                n += cnt[r];
            }
    }
    start[rows] = n;
    return start;
}

// The tallest of kNodeTileHeights whose gather span fits 32-bit byte offsets
// with 4-byte elements, else with 2-byte ones, else the shortest; and whose
// rows y - 1, y + 1 stay close enough for the bitmap index's base
// differences: (h + 1) nx + 1 < 2^(kDeltaBits - 1).
int tile_from_counts(const std::vector<int64_t>& cnt, int nx, int ny, int nz) {
    const int64_t lim = (int64_t)1 << (kDeltaBits - 1);
    for (const int elem : {4, 2})
        for (const int h : kNodeTileHeights) {
            if (((int64_t)std::min(h, nz) + 1) * nx + 1 >= lim) continue;
            const GatherSpan g = gather_span(order_rows(cnt, ny, nz, h), ny, nz, h, 19);
            if ((double)(g.slack + g.reach) * elem < 4294967296.0 && g.slack < ((int64_t)1 << 32)) return h;
        }
    return 1;
}
}  // namespace

int node_tile_z(const uint8_t* g, int nx, int ny, int nz) {
    return tile_from_counts(row_counts(g, nx, ny, nz), nx, ny, nz);
}

std::vector<int64_t> row_starts(const uint8_t* g, int nx, int ny, int nz, int tile_z) {
    return order_rows(row_counts(g, nx, ny, nz), ny, nz, tile_z);
}

NodeOrder node_order(const uint8_t* g, int nx, int ny, int nz) {
    const std::vector<int64_t> cnt = row_counts(g, nx, ny, nz);
    NodeOrder o;
    o.tile_z = tile_from_counts(cnt, nx, ny, nz);
    o.start = order_rows(cnt, ny, nz, o.tile_z);
    return o;
}

std::vector<int64_t> row_starts(const uint8_t* g, int nx, int ny, int nz) {
    return node_order(g, nx, ny, nz).start;
}

GatherSpan gather_span(const std::vector<int64_t>& start, int ny, int nz, int tile_z, int S) {
    const int T = (nz + tile_z - 1) / tile_z;
    const int64_t total = start[(int64_t)ny * nz];
    // first node of the tile at each position, and one past its last
    std::vector<int64_t> first(T), last(T);
    for (int p = 0; p < T; ++p) first[p] = start[(int64_t)tile_at(p, T) * tile_z * ny];
    for (int p = 0; p < T; ++p) last[p] = p + 1 < T ? first[p + 1] : total;
    const int64_t E = (int64_t)S * kChunk;
    auto chunk_lo = [&](int64_t node) { return node / kChunk * E; };
    auto chunk_hi = [&](int64_t node) { return (node / kChunk + 1) * E; };
    GatherSpan g{0, 0};
    for (int p = 0; p < T; ++p) {
        if (last[p] <= first[p]) continue;
        const int t = tile_at(p, T);
        int64_t lo = INT64_MAX, hi = 0;
        for (int d = -1; d <= 1; ++d) {
            const int q = tile_pos(((t + d) % T + T) % T, T);
            if (last[q] <= first[q]) continue;
            lo = std::min(lo, chunk_lo(first[q]));
            hi = std::max(hi, chunk_hi(last[q] - 1));
        }
        g.slack = std::max(g.slack, chunk_lo(last[p] - 1) - lo);
        g.reach = std::max(g.reach, hi - chunk_lo(first[p]));
    }
    return g;
}

int64_t count_fluid(const uint8_t* g, int nx, int ny, int nz) {
    return slab_offsets(g, nx, ny, nz)[nz];
}

CoordBits coord_bits(int nx, int ny, int nz) {
    return CoordBits{bits_for(nx), bits_for(ny), bits_for(nz)};
}

void build_table(const uint8_t* g, int nx, int ny, int nz, int64_t nf, int64_t stride,
                 int32_t* table, int tile_z) {
    const int64_t plane = (int64_t)nx * ny, vol = plane * nz;
    std::vector<int32_t> node(vol);
    auto start = tile_z > 0 ? row_starts(g, nx, ny, nz, tile_z) : row_starts(g, nx, ny, nz);
    parallel_slabs(nz, vol, [&](int z0, int z1) {
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < ny; ++y) {
                const int64_t r = (int64_t)z * ny + y;
                int64_t n = start[r];
                for (int64_t v = r * nx; v < (r + 1) * nx; ++v) node[v] = g[v] == 0 ? (int32_t)n++ : -1;
            }
    });
    parallel_slabs(nz, vol * 18, [&](int z0, int z1) {
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t v = x + (int64_t)nx * (y + (int64_t)ny * z);
                    const int32_t n = node[v];
                    if (n < 0) continue;
                    for (int i = 1; i < 19; ++i) {
                        // pull source x - c_i, periodic
                        int sx = x - kC[i][0], sy = y - kC[i][1], sz = z - kC[i][2];
                        sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
                        sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
                        sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
                        table[(int64_t)(i - 1) * stride + n] =
                            node[sx + (int64_t)nx * (sy + (int64_t)ny * sz)];
                    }
                }
    });
    (void)nf;
}

void build_bitmap(const uint8_t* g, int nx, int ny, int nz, int64_t nf, BitmapIndex* out, bool mirror_y,
                  bool mirror_z) {
    const int W = words_per_row(nx);
    const int64_t rows = (int64_t)ny * nz;
    out->words = W;
    out->bits = coord_bits(nx, ny, nz);
    out->coords.assign(nf, 0);
    out->ent.assign((size_t)rows * W * 4, 0u);
    out->wrap.assign((size_t)nz * 2 * W * 4, 0u);
    out->count.assign((size_t)rows * 4, 0u);
    std::vector<uint32_t> bits_of((size_t)rows * W, 0u), count_of((size_t)rows, 0u);
    std::vector<int32_t> base_of((size_t)rows * W, 0);
    auto start = row_starts(g, nx, ny, nz);
    const int bx = out->bits.bx, by = out->bits.by;
    // every row word's bits and base, every row's count, every node's coordinate
    parallel_slabs(nz, rows * nx, [&](int z0, int z1) {
        std::vector<uint8_t> pad(nx + 2);
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < ny; ++y) {
                const int64_t r = (int64_t)z * ny + y;
                const uint8_t* p = g + r * nx;
                const int64_t rowstart = start[r];
                int64_t n = rowstart;
                for (int x = 0; x < nx; ++x) pad[x + 1] = p[x] == 0;
                pad[0] = pad[nx];
                pad[nx + 1] = pad[1];
                uint32_t count = 0;
                for (int x = 0; x < nx; ++x) count += pad[x + 1];
                count_of[r] = count;
                int64_t before = 0;  // fluid voxels at real positions [1, kWordStep w)
                for (int w = 0; w < W; ++w) {
                    uint32_t bits = 0;
                    for (int b = 0; b < kWordStep + 2; ++b) {
                        const int q = kWordStep * w + b;
                        if (q < nx + 2 && pad[q]) bits |= 1u << b;
                    }
                    bits_of[r * W + w] = bits;
                    base_of[r * W + w] = (int32_t)(rowstart + before - (w == 0 ? pad[0] : 0));
                    for (int b = 0; b < kWordStep; ++b) {
                        const int q = kWordStep * w + b;
                        if (q >= 1 && q <= nx) before += pad[q];
                    }
                }
                for (int x = 0; x < nx; ++x)
                    if (p[x] == 0)
                        out->coords[n++] =
                            (uint32_t)x | ((uint32_t)y << bx) | ((uint32_t)z << (bx + by));
            }
    });
    // the neighbouring rows: y - 1 and y + 1 periodic in y, or, with symmetry
    // planes on the y faces, row 0 its own row y - 1 and row ny - 1 its own
    // row y + 1 (their ghost images); likewise the planes z - 1 and z + 1.
    // Across the periodic y wrap the kernel reads the bases from `wrap` and
    // the entry's difference is left 0.
    const int64_t lim = (int64_t)1 << (kDeltaBits - 1);
    std::atomic<bool> fits{true};
    parallel_slabs(nz, rows * W, [&](int z0, int z1) {
        for (int z = z0; z < z1; ++z) {
            const int zm = z == 0 ? (mirror_z ? 0 : nz - 1) : z - 1;
            const int zp = z == nz - 1 ? (mirror_z ? nz - 1 : 0) : z + 1;
            for (int y = 0; y < ny; ++y) {
                const int ym = y == 0 ? (mirror_y ? 0 : ny - 1) : y - 1;
                const int yp = y == ny - 1 ? (mirror_y ? ny - 1 : 0) : y + 1;
                const bool wm = ny > 1 && !mirror_y && y == 0, wp = ny > 1 && !mirror_y && y == ny - 1;
                const int64_t r = (int64_t)z * ny + y, rm = (int64_t)z * ny + ym, rp = (int64_t)z * ny + yp;
                uint32_t* cn = &out->count[(size_t)r * 4];
                cn[0] = count_of[r] | count_of[rm] << 16;
                cn[1] = count_of[rp] | count_of[(int64_t)zm * ny + y] << 16;
                cn[2] = count_of[(int64_t)zp * ny + y];
                for (int w = 0; w < W; ++w) {
                    const int64_t b0 = base_of[r * W + w];
                    const int64_t dm = wm ? 0 : base_of[rm * W + w] - b0;
                    const int64_t dp = wp ? 0 : base_of[rp * W + w] - b0;
                    if (dm < -lim || dm >= lim || dp < -lim || dp >= lim) fits = false;
                    const uint32_t um = (uint32_t)dm, up = (uint32_t)dp;
                    uint32_t* e = &out->ent[(size_t)(r * W + w) * 4];
                    e[0] = bits_of[rm * W + w] | (um & 0xfffu) << 20;
                    e[1] = bits_of[r * W + w] | (up & 0xfffu) << 20;
                    e[2] = bits_of[rp * W + w] | ((um >> 12) & 63u) << 20 | ((up >> 12) & 63u) << 26;
                    e[3] = (uint32_t)b0;
                }
            }
            // the rows across the y wrap: row ny - 1 for y = 0 (side 0), row 0 for y = ny - 1 (side 1)
            for (int side = 0; side < 2; ++side) {
                const int yw = side == 0 ? ny - 1 : 0;
                for (int w = 0; w < W; ++w) {
                    uint32_t* v = &out->wrap[(((size_t)z * 2 + side) * W + w) * 4];
                    v[0] = (uint32_t)base_of[((int64_t)zm * ny + yw) * W + w];
                    v[1] = (uint32_t)base_of[((int64_t)z * ny + yw) * W + w];
                    v[2] = (uint32_t)base_of[((int64_t)zp * ny + yw) * W + w];
                }
            }
        }
    });
    out->fits = fits;
}

void boundary_image(const uint8_t* g, int nx, int ny, int nz, int pad, bool mirror_y, bool mirror_z,
                    uint8_t* out) {
    const int ox = nx + 2 * pad, oy = mirror_y ? 2 * ny : ny, oz = mirror_z ? 2 * nz : nz;
    parallel_slabs(oz, (int64_t)ox * oy * oz, [&](int z0, int z1) {
        for (int z = z0; z < z1; ++z) {
            const int sz = z < nz ? z : 2 * nz - 1 - z;   // reflected copy beyond the z face
            for (int y = 0; y < oy; ++y) {
                const int sy = y < ny ? y : 2 * ny - 1 - y;
                uint8_t* row = out + ((int64_t)z * oy + y) * ox;
                const uint8_t* src = g + ((int64_t)sz * ny + sy) * nx;
                for (int x = 0; x < pad; ++x) row[x] = 0;
                for (int x = 0; x < nx; ++x) row[pad + x] = src[x];
                for (int x = pad + nx; x < ox; ++x) row[x] = 0;
            }
        }
    });
}

void neighbor_nodes(const uint8_t* g, int nx, int ny, int nz, const int64_t* nodes, int64_t count,
                    int32_t* out) {
    const auto start = row_starts(g, nx, ny, nz);
    const int64_t rows = (int64_t)ny * nz;
    // rows holding fluid, sorted by their first node number (distinct starts)
    std::vector<int64_t> order;
    for (int64_t r = 0; r < rows; ++r) {
        const uint8_t* p = g + r * nx;
        for (int x = 0; x < nx; ++x)
            if (p[x] == 0) {
                order.push_back(r);
                break;
            }
    }
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return start[a] < start[b]; });
    auto node_at = [&](int x, int y, int z) -> int32_t {  // node number of a voxel, -1 if solid
        const int64_t r = (int64_t)z * ny + y;
        const uint8_t* p = g + r * nx;
        if (p[x] != 0) return -1;
        int64_t k = 0;
        for (int q = 0; q < x; ++q) k += (p[q] == 0);
        return (int32_t)(start[r] + k);
    };
    for (int64_t k = 0; k < count; ++k) {
        const int64_t n = nodes[k];
        // the fluid row with the largest first node <= n holds node n
        const auto it = std::upper_bound(order.begin(), order.end(), n,
                                         [&](int64_t v, int64_t r) { return v < start[r]; });
        const int64_t r = *(it - 1);
        const int z = (int)(r / ny), y = (int)(r % ny);
        int64_t want = n - start[r];
        const uint8_t* p = g + r * nx;
        int x = 0;
        for (;; ++x)
            if (p[x] == 0 && want-- == 0) break;
        for (int i = 1; i < 19; ++i) {
            int sx = x - kC[i][0], sy = y - kC[i][1], sz = z - kC[i][2];
            sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
            sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
            sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
            out[(int64_t)(i - 1) * count + k] = node_at(sx, sy, sz);
        }
    }
}

void fluid_voxels(const uint8_t* g, int nx, int ny, int nz, int64_t* out) {
    auto start = row_starts(g, nx, ny, nz);
    parallel_slabs(nz, (int64_t)nx * ny * nz, [&](int z0, int z1) {
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < ny; ++y) {
                const int64_t r = (int64_t)z * ny + y;
                int64_t n = start[r];
                for (int x = 0; x < nx; ++x)
                    if (g[r * nx + x] == 0) out[n++] = r * nx + x;
            }
    });
}

}  // namespace lbm
