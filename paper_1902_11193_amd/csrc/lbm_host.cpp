// Host-side setup for liblbm: relaxation rates (Table 2 of Rao & Schaefer,
// arXiv:1902.11193) and compaction of the segmented image into the fluid-node
// list with its neighbour index.
#include "lbm_host.hpp"

#include <algorithm>
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

int64_t count_fluid(const uint8_t* g, int nx, int ny, int nz) {
    return slab_offsets(g, nx, ny, nz)[nz];
}

CoordBits coord_bits(int nx, int ny, int nz) {
    return CoordBits{bits_for(nx), bits_for(ny), bits_for(nz)};
}

void build_table(const uint8_t* g, int nx, int ny, int nz, int64_t nf, int64_t stride,
                 int32_t* table) {
    const int64_t plane = (int64_t)nx * ny, vol = plane * nz;
    std::vector<int32_t> node(vol);
    auto off = slab_offsets(g, nx, ny, nz);
    parallel_slabs(nz, vol, [&](int z0, int z1) {
        int64_t n = off[z0];
        for (int64_t v = plane * z0; v < plane * z1; ++v) node[v] = g[v] == 0 ? (int32_t)n++ : -1;
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

void build_bitmap(const uint8_t* g, int nx, int ny, int nz, int64_t nf, BitmapIndex* out) {
    const int W = (nx + 63) / 64;
    const int64_t rows = (int64_t)ny * nz;
    out->words_per_row = W;
    out->bits = coord_bits(nx, ny, nz);
    out->coords.assign(nf, 0);
    out->rowbits.assign(rows * W, 0);
    out->wordbase.assign(rows * W, 0);
    auto off = slab_offsets(g, nx, ny, nz);
    const int bx = out->bits.bx, by = out->bits.by;
    parallel_slabs(nz, rows * nx, [&](int z0, int z1) {
        int64_t n = off[z0];
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < ny; ++y) {
                const int64_t r = (int64_t)z * ny + y;
                const uint8_t* p = g + r * nx;
                for (int w = 0; w < W; ++w) {
                    out->wordbase[r * W + w] = (int32_t)n;
                    uint64_t bits = 0;
                    for (int b = 0; b < 64 && 64 * w + b < nx; ++b) {
                        const int x = 64 * w + b;
                        if (p[x] == 0) {
                            bits |= 1ull << b;
                            out->coords[n++] = (uint32_t)x | ((uint32_t)y << bx) |
                                               ((uint32_t)z << (bx + by));
                        }
                    }
                    out->rowbits[r * W + w] = bits;
                }
            }
    });
}

void fluid_voxels(const uint8_t* g, int nx, int ny, int nz, int64_t* out) {
    const int64_t vol = (int64_t)nx * ny * nz;
    int64_t n = 0;
    for (int64_t v = 0; v < vol; ++v)
        if (g[v] == 0) out[n++] = v;
}

}  // namespace lbm
