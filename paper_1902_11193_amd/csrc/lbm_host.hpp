// Host-side setup for liblbm: relaxation rates and compaction of the voxel
// image into the fluid-node list with its neighbour index.  Plain C++, no HIP.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace lbm {

// Velocity order used everywhere in the library (pairs 2k-1, 2k opposite).
extern const int kC[19][3];
inline int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Rates of Table 2 for a set at (tau, Lambda), grouped by class, with their
// derivatives.  Returns an empty string when valid, else the reason.
struct RateClasses {
    double s_e, s_eps, s_q, s_nu, s_pi, s_m;
};
std::string rates(int set, double tau, double Lambda, RateClasses* s, RateClasses* ds_dtau,
                  RateClasses* ds_dLambda);
void rates_to_moments(const RateClasses& r, double s[19]);

// Shape checks common to every entry point.
std::string check_dims(int nx, int ny, int nz);

int64_t count_fluid(const uint8_t* geom, int nx, int ny, int nz);

// Bit widths of the packed voxel coordinate x | y << bx | z << (bx + by).
struct CoordBits {
    int bx, by, bz;
    bool fits() const { return bx + by + bz <= 32; }
};
CoordBits coord_bits(int nx, int ny, int nz);

// Padded node count: the fluid list rounded up to a multiple of 256.
inline int64_t padded(int64_t nf) { return (nf + 255) / 256 * 256; }

// Pull-source table [18][stride], entry (i-1)*stride + n; -1 = solid source.
void build_table(const uint8_t* geom, int nx, int ny, int nz, int64_t nf, int64_t stride,
                 int32_t* table);

// Bitmap index: packed coordinate per node, fluid bits per 64-voxel word of
// every (y, z) row, and the node number of the first fluid voxel at or after
// each word.
struct BitmapIndex {
    int words_per_row = 0;
    CoordBits bits{};
    std::vector<uint32_t> coords;    // [nf]
    std::vector<uint64_t> rowbits;   // [ny * nz * words_per_row]
    std::vector<int32_t> wordbase;   // [ny * nz * words_per_row]
};
void build_bitmap(const uint8_t* geom, int nx, int ny, int nz, int64_t nf, BitmapIndex* out);

// Linear voxel id of every fluid node (raster order).
void fluid_voxels(const uint8_t* geom, int nx, int ny, int nz, int64_t* out);

}  // namespace lbm
