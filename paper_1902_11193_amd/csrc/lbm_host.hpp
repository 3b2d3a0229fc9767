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

// Node order of the compacted fluid list: the (y, z) rows of the image are
// taken in z-tiles of tile_z planes -- tile, then y, then z inside the tile --
// and the fluid voxels of each row in increasing x.  Rows that are neighbours
// in y or z then sit at most tile_z rows apart in the list (except across
// tile faces).  The tiles themselves are folded: tile t of T comes at
// position 2t when 2t < T, else at 2(T - 1 - t) + 1 (order 0, T-1, 1, T-2,
// ...), so tiles that touch in z, across the periodic wrap too, are at most
// two positions apart and every gather stays near its node.
//
// The gathers across a tile face reach a tile two positions away, whose lines
// no cache still holds, and the same lines are fetched again when that tile
// is stepped; within a tile a neighbour row tile_z rows back was fetched
// moments before (by another XCD, possibly, from the MALL).  So the tiles are
// as tall as the 32-bit gather offsets allow: node_tile_z takes the tallest
// height of kNodeTileHeights whose gather span fits with 4-byte elements
// (else with 2-byte ones) and with (h + 1) nx + 1 < 2^17 (the bitmap index's
// base differences, below).  (512^3 rock, FP32 storage: 0.767 ms per step with
// 16-plane tiles, 0.745 with 64, 0.738 with 96 or 128; the 16-bit storages
// within 0.5%.)  The choice depends on the image alone, so every storage and
// every call that orders the nodes agrees on it.
constexpr int kNodeTileHeights[] = {128, 64, 32, 16, 8, 4, 2, 1};
inline int tile_at(int p, int T) { return (p & 1) ? T - 1 - (p >> 1) : (p >> 1); }
inline int tile_pos(int t, int T) { return 2 * t < T ? 2 * t : 2 * (T - 1 - t) + 1; }
int node_tile_z(const uint8_t* geom, int nx, int ny, int nz);

// Node number of the first fluid voxel of every row r = z * ny + y
// (entry ny * nz holds the fluid count), in the image's order (node_tile_z),
// or with the given tile height.
std::vector<int64_t> row_starts(const uint8_t* geom, int nx, int ny, int nz);
std::vector<int64_t> row_starts(const uint8_t* geom, int nx, int ny, int nz, int tile_z);
struct NodeOrder {
    int tile_z;
    std::vector<int64_t> start;  // row_starts with that height
};
NodeOrder node_order(const uint8_t* geom, int nx, int ny, int nz);

// Padded node count: the fluid list rounded up to a multiple of kChunk.
constexpr int kChunk = 256;
inline int64_t padded(int64_t nf) { return (nf + kChunk - 1) / kChunk * kChunk; }

// Population layout in device memory: the kChunk nodes of chunk q = n / kChunk
// keep their S values back to back (S = 19 populations; FP16 with a reference
// keeps the references in a per-node array after the chunks), element (i, n)
// at q * S * kChunk + i * kChunk + n % kChunk.
inline int64_t state_elem(int i, int64_t n, int S = 19) {
    return (n / kChunk) * ((int64_t)S * kChunk) + (int64_t)i * kChunk + n % kChunk;
}

// The step kernels address a chunk's gathers as 32-bit byte offsets from a
// base `slack` elements below the chunk.  From the tile structure of the node
// order (row_starts with tile height tile_z), gather_span bounds how far below its chunk (slack) and
// how far past its start (reach) a chunk's gathered elements can lie; the
// offsets fit when (slack + reach) * element size < 2^32.
struct GatherSpan {
    int64_t slack, reach;  // elements
};
GatherSpan gather_span(const std::vector<int64_t>& start, int ny, int nz, int tile_z, int S = 19);

// Pull-source table [18][stride], entry (i-1)*stride + n; -1 = solid source;
// nodes in the image's order, or with tiles of tile_z planes when tile_z > 0.
void build_table(const uint8_t* geom, int nx, int ny, int nz, int64_t nf, int64_t stride,
                 int32_t* table, int tile_z = 0);

// Bitmap index.  Every (y, z) row of the image is a padded bit string of
// nx + 2 positions: position x + 1 holds voxel x, position 0 repeats voxel
// nx - 1 and position nx + 1 repeats voxel 0 (the periodic wrap).  Word w of a
// row covers positions kWordStep w .. kWordStep w + 19: consecutive words
// overlap by two positions, so the window x .. x + 2 (voxels x - 1, x, x + 1)
// of voxel x lies inside word x / kWordStep.  The base of a row word is the
// node number counting the row's real voxels before it (minus the left pad
// bit on word 0).  For every row (y, z) and word w one 16-byte entry holds the
// 20 bits of word w of rows y - 1, y, y + 1 (periodic in y) of plane z, the
// base of the word in row y, and the bases in rows y - 1 and y + 1 as 18-bit
// differences dm, dp from it:
//   e[0] = bits(y - 1) | (dm & 0xfff) << 20
//   e[1] = bits(y)     | (dp & 0xfff) << 20
//   e[2] = bits(y + 1) | ((dm >> 12) & 63) << 20 | ((dp >> 12) & 63) << 26
//   e[3] = base(y)
// so a node reads its nine rows with three 16-byte loads, entries (z - 1, y,
// w), (z, y, w), (z + 1, y, w), and the nodes of a row read consecutive
// entries.  Two things stay outside the entries, each one load for the nodes
// that need it: for the rows y = 0 and y = ny - 1, `wrap` (z, side, w) holds
// the bases of word w in the row across the periodic y wrap (row ny - 1 for
// side 0, row 0 for side 1) in planes z - 1, z, z + 1, a tile apart in the
// node order; and `count` (z, y) holds the fluid counts of rows (y, z),
// (y - 1, z), (y + 1, z), (y, z - 1), (y, z + 1) as 16-bit fields {c0 | c1 << 16,
// c2 | c3 << 16, c4, 0}, which the x wrap needs at x = 0 and x = nx - 1.  Every
// other difference is at most (h + 1) nx + 1 for z-tiles of h planes, below
// 2^17 with node_tile_z's height.  Each node also keeps its packed voxel
// coordinate.
constexpr int kWordStep = 18;
constexpr int kDeltaBits = 18;
inline int words_per_row(int nx) { return (nx - 1) / kWordStep + 1; }
constexpr int kBitmapMaxNx = 4095;
struct BitmapIndex {
    int words = 0;  // words per row
    CoordBits bits{};
    bool fits = true;              // every used difference fits kDeltaBits
    std::vector<uint32_t> coords;  // [nf]
    std::vector<uint32_t> ent;     // [nz][ny][words][4]
    std::vector<uint32_t> wrap;    // [nz][2][words][4]
    std::vector<uint32_t> count;   // [nz][ny][4]
};
// mirror_y: symmetry planes on the y faces (Sec. 2.3): row y - 1 of row 0 and
// row y + 1 of row ny - 1 are those rows themselves (their ghost images)
// instead of the periodic neighbours.  mirror_z: likewise plane z - 1 of
// plane 0 and plane z + 1 of plane nz - 1 (for the counts and wrap bases; the
// kernel picks the planes of the entries itself).
void build_bitmap(const uint8_t* geom, int nx, int ny, int nz, int64_t nf, BitmapIndex* out,
                  bool mirror_y = false, bool mirror_z = false);

// Non-periodic image stacks (Sec. 2.3): `pad` fluid-only layers before and
// after the image along x, then the image reflected across its y and/or z
// faces, so that those faces become symmetry (mirror) planes of the periodic
// box.  out is [nz'][ny'][nx'] with nx' = nx + 2 pad, ny' = ny (x2 when
// mirror_y), nz' = nz (x2 when mirror_z).
void boundary_image(const uint8_t* geom, int nx, int ny, int nz, int pad, bool mirror_y, bool mirror_z,
                    uint8_t* out);

// Pull sources [18][count] (entry (i-1)*count + k; -1 = solid source) of the
// given nodes only, found from the row starts without the full table.
void neighbor_nodes(const uint8_t* geom, int nx, int ny, int nz, const int64_t* nodes, int64_t count,
                    int32_t* out);

// Linear voxel id x + nx (y + ny z) of every fluid node, in node order.
void fluid_voxels(const uint8_t* geom, int nx, int ny, int nz, int64_t* out);

}  // namespace lbm
