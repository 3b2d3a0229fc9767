// gfx950 kernels of liblbm: one fused D3Q19 MRT stream-collide step over the
// compacted fluid-node list, its discrete adjoint, and small helpers.
//
// Method: Rao & Schaefer, arXiv:1902.11193 -- lattice Boltzmann equation
// (Sec. 2, Eq. LBE), MRT collision in moment space (Sec. 2.1.1, Eqs. MRT
// Collision, MRT Equi, MRT params), Guo forcing (Eqs. MRT-LBE,
// Guo_Forcing), halfway bounce-back and a periodic body-force-driven box
// (Sec. 2.3), volume-averaged velocity for Darcy's law (Eq. perm_calc).
//
// Design for CDNA4: every fluid node is one lane of a wave64; populations are
// stored chunk by chunk, the 256 nodes of a chunk (one block's share of a
// sweep) keeping their 19 populations back to back, so a chunk's 19 stores
// are one contiguous run and its gathers fall in a few nearby runs rather
// than 19 separate arrays; the 19x19 transform M and its inverse M^T diag(1/|row|^2) are
// written out as integer-coefficient adds on pair sums/differences of
// opposite populations (no MFMA: at ~0.4 kflop per node-update against
// ~150 bytes of traffic this is an HBM-bound stencil, not a contraction).
// Storage holds deviations f_i - w_i rho0 (FP32, scaled FP16, BF16, or FP16
// relative to a per-node reference density); all
// arithmetic is FP32; the mean-velocity reduction is FP64 and deterministic
// (fixed per-block node ranges, fixed reduction trees).
#include "lbm_kernels.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <type_traits>
#include <utility>

namespace lbm {
namespace {

// Reduction scratch of contexts set up with lbm_setup_static: every GPU holds
// its own copy.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (static_scratch below).
static __device__ __align__(256) unsigned char scratch[kReductionBytes];

constexpr int kThreads = 256;

__host__ __device__ constexpr int cdir(int i, int a) {
    constexpr int t[19][3] = {
        {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
        {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
        {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    return t[i][a];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// index of c_i with its components along the axes in `mask` (bit a: axis a) negated
__host__ __device__ constexpr int mirrored(int i, int mask) {
    int want[3] = {cdir(i, 0), cdir(i, 1), cdir(i, 2)};
    for (int a = 0; a < 3; ++a)
        if (mask >> a & 1) want[a] = -want[a];
    for (int j = 0; j < 19; ++j)
        if (cdir(j, 0) == want[0] && cdir(j, 1) == want[1] && cdir(j, 2) == want[2]) return j;
    return -1;
}
// lattice weights w_i: 1/3 rest, 1/18 axis (i = 1..6), 1/36 diagonal
__host__ __device__ constexpr float wgt(int i) { return i == 0 ? 1.f / 3.f : (i <= 6 ? 1.f / 18.f : 1.f / 36.f); }

template <class F, int... I>
__device__ __forceinline__ void unroll_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F&& f) {
    unroll_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------------------------ codecs
// Storage of deviations f_i - w_i rho0: cvt decodes a stored value, enc
// encodes one (FP16 carries a power-of-two scale; BF16 rounds to nearest even).
struct CodecF32 {
    using T = float;
    static constexpr int kSlots = 19;    // values kept per node
    static constexpr bool kRef = false;  // populations stored relative to a reference density
    static __device__ __forceinline__ float cvt(T v, float) { return v; }
    static __device__ __forceinline__ T enc(float v, float) { return v; }
};
struct CodecF16 {
    using T = _Float16;
    static constexpr int kSlots = 19;
    static constexpr bool kRef = false;
    static __device__ __forceinline__ float cvt(T v, float inv) { return (float)v * inv; }
    static __device__ __forceinline__ T enc(float v, float s) { return (_Float16)(v * s); }
};
struct CodecBF16 {
    using T = uint16_t;
    static constexpr int kSlots = 19;
    static constexpr bool kRef = false;
    static __device__ __forceinline__ float cvt(T v, float inv) {
        return __uint_as_float((uint32_t)v << 16) * inv;
    }
    // round to nearest even (NaN stays NaN): one hardware conversion on gfx950
    static __device__ __forceinline__ T enc(float v, float s) { return __builtin_bit_cast(T, (__bf16)(v * s)); }
};

// FP16 relative to a per-node reference density: a node stores, besides its
// populations, r = fp16(drho) in the state's reference array (one FP16 per
// node in node order, after the chunks), and each population as
// 2^e (f_i - w_i rho0 - w_i r).  A reader adds w_i r of the node the value
// came from.  Writer and reader use the same stored r, so the reference is
// exact; what FP16 rounds is only the velocity and non-equilibrium part,
// not the density (pressure) deviation that dominates f - w rho0 in poorly
// connected rock.
struct CodecF16R {
    using T = _Float16;
    static constexpr int kSlots = 19;
    static constexpr bool kRef = true;
    static __device__ __forceinline__ float cvt(T v, float inv) { return (float)v * inv; }
    static __device__ __forceinline__ T enc(float v, float s) { return (_Float16)(v * s); }
};

// ------------------------------------------------------------------ addressing
// Loads through a wave-uniform base pointer and a 32-bit byte offset: the
// compiler emits global loads with a scalar base and one VGPR offset, so no
// 64-bit address arithmetic runs per lane.
template <class T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void st_off(T* base, uint32_t byte_off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// Streaming store: the next step reads these values only after the whole
// population array (gigabytes) has gone through the caches, so they are
// written without displacing cached lines the gathers still reuse.
template <class T>
__device__ __forceinline__ void st_stream(T* base, uint32_t byte_off, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off));
}

// ------------------------------------------------------------------ layout
// Element (i, m) of a population array sits at node_elem(m) + i * kThreads:
// chunk q = m / 256 owns elements [q * S * 256, (q + 1) * S * 256), S = 19
// values per node (FP16 with a reference keeps the references in a separate
// per-node array after the chunks).
constexpr uint32_t kChunkElems = 19u * kThreads;
template <int S = 19>
__device__ __forceinline__ uint32_t node_elem(uint32_t m) {
    return m + (m >> 8) * ((uint32_t)(S - 1) * kThreads);  // = (m / 256) * S * 256 + m % 256
}

// Gathers of one chunk go through a wave-uniform base pointer placed `slack`
// elements below the chunk's first element, with one 32-bit byte offset per
// lane; the host checks (gather_span) that every element a chunk gathers lies
// within 2^32 bytes above that base.  Offsets are formed modulo 2^32, which
// is exact for values that fit.
template <class T, int S = 19>
__device__ __forceinline__ const T* chunk_base(const T* p, uint32_t chunk, uint32_t slack) {
    return p + ((int64_t)chunk * (S * kThreads) - (int64_t)slack);
}
// Byte offset, from the base of chunk cbe / kChunkElems, of the population
// pulled in direction i: population i of the source node m, or, when the
// source voxel is solid (m < 0), population opp(i) of the node itself (en =
// node_elem of the node; halfway bounce-back).
template <class T, int I, int S = 19>
__device__ __forceinline__ uint32_t pull_offset(int32_t m, uint32_t en, uint32_t kb) {
    // both candidates, then a bitwise select: no branch per direction
    const uint32_t pulled = node_elem<S>((uint32_t)m) + (uint32_t)I * kThreads;
    const uint32_t own = en + (uint32_t)opp(I) * kThreads;
    const uint32_t wall = (uint32_t)(m >> 31);  // all ones when m < 0
    return ((pulled & ~wall) | (own & wall)) * (uint32_t)sizeof(T) + kb;
}
// kb of a chunk: (slack - first element of the chunk) * sizeof(T), mod 2^32
template <class T, int S = 19>
__device__ __forceinline__ uint32_t chunk_kb(uint32_t chunk, uint32_t slack) {
    return (slack - chunk * (uint32_t)(S * kThreads)) * (uint32_t)sizeof(T);
}
// Offsets of the 19 populations gathered into node n of chunk `chunk`
// (off[0]: its own rest population) from the pull sources s.
template <class T, int S = 19>
__device__ __forceinline__ void gather_offsets(const int32_t s[19], uint32_t n, uint32_t chunk,
                                               uint32_t slack, uint32_t off[19]) {
    const uint32_t en = node_elem<S>(n), kb = chunk_kb<T, S>(chunk, slack);
    off[0] = en * (uint32_t)sizeof(T) + kb;
    unroll<18>([&](auto k) {
        constexpr int i = decltype(k)::value + 1;
        off[i] = pull_offset<T, i, S>(s[i], en, kb);
    });
}

// ------------------------------------------------------------------ indices
// An index yields, for node n, the pull sources s[i] (i = 1..18): the node
// at x_n - c_i, or -1 when that voxel is solid (halfway bounce-back there),
// and from them the 19 gather offsets of the step (offsets).  The adjoint
// reads the sources transposed, s[opp(i)] being the node at x_n + c_i.
//
// Both indices split into load (issue the memory reads for a node) and
// resolve (arithmetic on what was read), so a caller can overlap the reads of
// one node with the population traffic of another.

// Wall links of a node as a bit mask (bit i: the voxel at x - c_i is solid).
__device__ __forceinline__ uint32_t wall_bits(const int32_t s[19]) {
    uint32_t b = 0;
    unroll<18>([&](auto k) {
        constexpr int i = decltype(k)::value + 1;
        b |= (uint32_t)(s[i] < 0) << i;
    });
    return b;
}

// Device table of pull sources [18][stride] (entry -1: solid source).
struct TableIdx {
    const int32_t* __restrict__ t;
    uint32_t stride;
    using Pre = uint32_t;  // nothing to fetch ahead
    __device__ __forceinline__ Pre prefetch(uint32_t) const { return 0u; }
    struct Raw {
        int32_t t[19];
    };
    template <bool BRANCH = true>
    __device__ __forceinline__ void load(uint32_t n, Pre, Raw& r) const {
        unroll<18>([&](auto k) {
            constexpr int i = decltype(k)::value + 1;
            r.t[i] = ld_off(t + (size_t)(i - 1) * stride, n * 4u);
        });
    }
    __device__ __forceinline__ void sources(const Raw& r, Pre, int32_t s[19]) const {
        unroll<18>([&](auto k) {
            constexpr int i = decltype(k)::value + 1;
            s[i] = r.t[i];
        });
    }
    // gather offsets of node n (chunk `chunk`) and, if WB, its wall links
    // (symmetry planes need the bitmap index)
    template <class T, int S, bool WB, bool SYM = false>
    __device__ __forceinline__ void offsets(const Raw& r, Pre p, uint32_t n, uint32_t chunk,
                                            uint32_t slack, uint32_t off[19], uint32_t& wb) const {
        static_assert(!SYM, "symmetry planes are built for the bitmap index");
        int32_t s[19];
        sources(r, p, s);
        gather_offsets<T, S>(s, n, chunk, slack, off);
        if constexpr (WB) wb = wall_bits(s);
    }
    // F16R: byte offset in the reference array of the node each value comes
    // from (the source, or the node itself at a wall), one load per direction
    struct RefPlan {
        uint32_t ro[19];
    };
    template <class T, int S>
    __device__ __forceinline__ void offsets_ref(const Raw& r, Pre p, uint32_t n, uint32_t chunk, uint32_t slack,
                                                uint32_t off[19], uint32_t& wb, RefPlan& plan) const {
        int32_t s[19];
        sources(r, p, s);
        gather_offsets<T, S>(s, n, chunk, slack, off);
        wb = wall_bits(s);
        plan.ro[0] = n * (uint32_t)sizeof(T);
        unroll<18>([&](auto k) {
            constexpr int i = decltype(k)::value + 1;
            plan.ro[i] = (uint32_t)(s[i] < 0 ? (int32_t)n : s[i]) * (uint32_t)sizeof(T);
        });
    }
    template <class T>
    struct RefLoads {
        T v[19];
    };
    template <class T, int S>
    __device__ __forceinline__ void issue_refs(const RefPlan& plan, const T* rb, uint32_t, const uint32_t*,
                                               uint32_t, uint32_t, RefLoads<T>& L) const {
        unroll<19>([&](auto k) {
            constexpr int i = decltype(k)::value;
            L.v[i] = ld_off(rb, plan.ro[i]);
        });
    }
    template <class T>
    __device__ __forceinline__ void finish_refs(const RefPlan&, uint32_t, const RefLoads<T>& L, T rr[19]) const {
        unroll<19>([&](auto k) {
            constexpr int i = decltype(k)::value;
            rr[i] = L.v[i];
        });
    }
    // both gathers of the reverse step (see BitmapIdx::offsets_adj)
    template <class T, int S>
    __device__ __forceinline__ void offsets_adj(const Raw& r, Pre p, uint32_t n, uint32_t chunk,
                                                uint32_t slack, uint32_t of[19], uint32_t ob[19]) const {
        int32_t s[19];
        sources(r, p, s);
        const uint32_t en = node_elem<S>(n), kb = chunk_kb<T, S>(chunk, slack);
        of[0] = ob[0] = en * (uint32_t)sizeof(T) + kb;
        unroll<18>([&](auto k) {
            constexpr int i = decltype(k)::value + 1;
            of[i] = pull_offset<T, i, S>(s[i], en, kb);
            ob[i] = pull_offset<T, i, S>(s[opp(i)], en, kb);
        });
    }
};

// Row words of the padded bit strings built on the host: word w of a row
// covers padded positions 18 w .. 18 w + 19 (position x + 1 is voxel x, the
// two ends repeat the opposite voxel: periodic x), so the window of voxel x
// lies in word x / 18.  Entry (z, y, w), 16 bytes: the 20 bits of word w of
// rows y - 1, y, y + 1 of plane z, the node base of the word in row y and, as
// 18-bit differences from it split over the bits' spare high bits, the bases
// in rows y - 1 and y + 1.  A node reads the entries of planes z - 1, z,
// z + 1: three 16-byte loads.  Across the periodic y wrap (row y - 1 of
// y = 0, row y + 1 of y = ny - 1) the bases come from one 12-byte slot of the
// wrap array, and the x wrap (x = 0 or nx - 1) takes the fluid counts of the
// five rows it crosses from one 12-byte slot of the count array; only nodes
// there read them.
constexpr uint32_t kWordStep = 18;
// (a & mask) | (b & ~mask) in one instruction
__device__ __forceinline__ uint32_t bit_select(uint32_t mask, uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(mask), "v"(a), "v"(b));
    return r;
}
struct BitmapIdx {
    const uint32_t* __restrict__ coords;
    const uint4* __restrict__ ent;
    const uint4* __restrict__ wraps;   // [nz][2][R]: bases in planes z - 1, z, z + 1 of the row across the y wrap
    const uint4* __restrict__ counts;  // [nz][ny]: 16-bit counts of rows (y, z), (y - 1, z), (y + 1, z), (y, z -/+ 1)
    uint32_t nx, ny, nz, R, bx, by;  // R: words per row
    // entry offsets from plane z to the plane read as z - 1 at z = 0 and as
    // z + 1 at z = nz - 1: the periodic wrap, or 0 (the plane itself, its
    // ghost image) with symmetry planes on the z faces
    uint32_t zlo, zhi;
    uint32_t sym;  // symmetry planes: bit 0 on the y faces, bit 1 on the z faces

    // voxels x - 1, x, x + 1 of a row: fluid bits (bit 0..2) and node numbers
    struct Row3 {
        int32_t rm, r0, rp;
        uint32_t bits;
    };
    // lo: the word's 20 bits (higher bits ignored); base: node number before
    // the word; count: the row's fluid voxels (read at x = 0 and nx - 1 only)
    __device__ __forceinline__ Row3 decode(uint32_t lo, int32_t base, uint32_t count, uint32_t x, bool x_first,
                                           bool x_last) const {
        const uint32_t sh = x - (x / kWordStep) * kWordStep;
        Row3 r;
        r.bits = __builtin_amdgcn_ubfe(lo, sh, 3u);   // padded positions x..x+2
        const int32_t below = (int32_t)__popc(__builtin_amdgcn_ubfe(lo, 0u, sh));
        r.r0 = base + below + (int32_t)(r.bits & 1u);
        r.rm = r.r0 - 1 + (x_first ? (int32_t)count : 0);
        r.rp = r.r0 + (int32_t)((r.bits >> 1) & 1u) - (x_last ? (int32_t)count : 0);
        return r;
    }
    using Pre = uint32_t;  // the node's packed coordinate, loaded ahead of use
    __device__ __forceinline__ Pre prefetch(uint32_t n) const { return ld_off(coords, n * 4u); }
    // 1 on the plane x = 0, 2 on x = nx - 1, else 0
    __device__ __forceinline__ uint32_t x_face(Pre c) const {
        const uint32_t x = c & ((1u << bx) - 1u);
        return x == 0 ? 1u : (x == nx - 1 ? 2u : 0u);
    }
    // rows y - 1 of y = 0 and y + 1 of y = ny - 1 lie across the periodic y wrap
    __device__ __forceinline__ bool y_wraps() const { return ny > 1u && !(sym & 1u); }
    struct Raw {
        uint4 a[3];       // entries of planes z - 1, z, z + 1
        uint32_t cn[3];   // x = 0 or nx - 1: the five rows' counts, 16 bits each
        int32_t fb[3];    // across the y wrap: base of the wrapped row's word in planes z - 1, z, z + 1
    };
    // 12 bytes at a 16-byte slot
    static __device__ __forceinline__ void load12(const uint4* p, uint32_t v[3]) {
        typedef uint32_t V3 __attribute__((ext_vector_type(3), aligned(16)));
        const V3 t = *reinterpret_cast<const V3*>(p);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
    }
    // the 18-bit base differences of rows y - 1 (dm) and y + 1 (dp)
    static __device__ __forceinline__ int32_t sext18(uint32_t v) { return (int32_t)(v << 14) >> 14; }
    static __device__ __forceinline__ int32_t dm(const uint4& e) {
        return sext18((e.x >> 20) | ((e.z >> 20) & 63u) << 12);
    }
    static __device__ __forceinline__ int32_t dp(const uint4& e) {
        return sext18((e.y >> 20) | ((e.z >> 26) & 63u) << 12);
    }
    // issue the entry loads of the node with packed coordinate c and its count
    // and wrap slots (in bounds for every node; used only on the x or y wrap).
    // BRANCH: the slots only when a node of the wave lies on either wrap,
    // under one wave-uniform branch; the steps take it (loading the slots in
    // every wave cost the 512^3 rock's FP16 step 4%, FP32 0.5%).  The adjoint
    // loads them always: at one wave per SIMD the branch cost the 128^3
    // pack's reverse step 8% (the 512^3 rock's 0.3%).
    template <bool BRANCH = true>
    __device__ __forceinline__ void load(uint32_t, Pre c, Raw& r) const {
        const uint32_t x = c & ((1u << bx) - 1u);
        const uint32_t y = (c >> bx) & ((1u << by) - 1u);
        const uint32_t z = (uint32_t)((uint64_t)c >> (bx + by));
        const uint32_t plane = ny * R;                          // entries per plane
        const uint32_t e = (z * ny + y) * R + x / kWordStep;    // entry (z, y, w)
        const uint32_t em = e + (z == 0 ? zlo : 0u - plane);
        const uint32_t ep = e + (z == nz - 1 ? zhi : plane);
        __builtin_amdgcn_sched_barrier(0);
        r.a[0] = ent[em];
        r.a[1] = ent[e];
        r.a[2] = ent[ep];
        auto slots = [&] {
            load12(counts + (z * ny + y), r.cn);
            uint32_t v[3];
            load12(wraps + ((z * 2u + (y == 0u ? 0u : 1u)) * R + x / kWordStep), v);
            unroll<3>([&](auto k) { r.fb[decltype(k)::value] = (int32_t)v[decltype(k)::value]; });
        };
        if constexpr (BRANCH) {
            unroll<3>([&](auto k) {
                r.cn[decltype(k)::value] = 0u;
                r.fb[decltype(k)::value] = 0;
            });
            if (__builtin_amdgcn_ballot_w64(x == 0u || x == nx - 1u || y == 0u || y == ny - 1u) != 0) slots();
        } else {
            slots();
        }
    }
    // Calls put(I, row, which) for the 18 directions I of node c: the source
    // voxel x - c_I is voxel x + which (which = -1, 0, +1) of the decoded
    // row `row` (Row3: node numbers and fluid bits of voxels x - 1 .. x + 1).
    // The nine rows are numbered 0 own, 1 y - 1, 2 y + 1, 3 z - 1, 4 z + 1,
    // 5 (y - 1, z - 1), 6 (y + 1, z + 1), 7 (y - 1, z + 1), 8 (y + 1, z - 1);
    // direction i pulls from voxel x + which_of(i) of row row_of(i).
    static __host__ __device__ constexpr int row_of(int i) {
        constexpr int t[19] = {0, 0, 0, 1, 2, 3, 4, 1, 2, 2, 1, 3, 4, 4, 3, 5, 6, 7, 8};
        return t[i];
    }
    static __host__ __device__ constexpr int which_of(int i) {
        constexpr int t[19] = {0, -1, 1, 0, 0, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 0, 0};
        return t[i];
    }
    template <class Put>
    __device__ __forceinline__ void visit(const Raw& r, Pre c, Put&& put) const {
        using std::integral_constant;
        const uint32_t x = c & ((1u << bx) - 1u);
        const uint32_t y = (c >> bx) & ((1u << by) - 1u);
        const bool xf = x == 0, xl = x == nx - 1;
        const bool wm = y_wraps() && y == 0u, wp = y_wraps() && y == ny - 1u;
        // bases of rows y - 1 and y + 1 in the entry of plane k
        auto bm = [&](int k) { return wm ? r.fb[k] : (int32_t)r.a[k].w + dm(r.a[k]); };
        auto bp = [&](int k) { return wp ? r.fb[k] : (int32_t)r.a[k].w + dp(r.a[k]); };
        // source x' = x - c_x: c_x = +1 reads x - 1 (which -1), c_x = -1 reads x + 1
        const Row3 o = decode(r.a[1].y, (int32_t)r.a[1].w, r.cn[0] & 0xffffu, x, xf, xl);
        put(integral_constant<int, 1>{}, o, -1);
        put(integral_constant<int, 2>{}, o, +1);
        const Row3 a = decode(r.a[1].x, bm(1), r.cn[0] >> 16, x, xf, xl);   // c_y = +1
        put(integral_constant<int, 3>{}, a, 0);
        put(integral_constant<int, 7>{}, a, -1);
        put(integral_constant<int, 10>{}, a, +1);
        const Row3 b = decode(r.a[1].z, bp(1), r.cn[1] & 0xffffu, x, xf, xl);   // c_y = -1
        put(integral_constant<int, 4>{}, b, 0);
        put(integral_constant<int, 8>{}, b, +1);
        put(integral_constant<int, 9>{}, b, -1);
        const Row3 d = decode(r.a[0].y, (int32_t)r.a[0].w, r.cn[1] >> 16, x, xf, xl);   // c_z = +1
        put(integral_constant<int, 5>{}, d, 0);
        put(integral_constant<int, 11>{}, d, -1);
        put(integral_constant<int, 14>{}, d, +1);
        const Row3 e = decode(r.a[2].y, (int32_t)r.a[2].w, r.cn[2], x, xf, xl);   // c_z = -1
        put(integral_constant<int, 6>{}, e, 0);
        put(integral_constant<int, 12>{}, e, +1);
        put(integral_constant<int, 13>{}, e, -1);
        // the corner rows only give voxel x, which needs no count
        put(integral_constant<int, 15>{}, decode(r.a[0].x, bm(0), 0u, x, false, false), 0);   // y - 1, z - 1
        put(integral_constant<int, 16>{}, decode(r.a[2].z, bp(2), 0u, x, false, false), 0);   // y + 1, z + 1
        put(integral_constant<int, 17>{}, decode(r.a[2].x, bm(2), 0u, x, false, false), 0);   // y - 1, z + 1
        put(integral_constant<int, 18>{}, decode(r.a[0].z, bp(0), 0u, x, false, false), 0);   // y + 1, z - 1
    }
    // node number of voxel x + which of a decoded row, and all ones when it is fluid
    static __device__ __forceinline__ uint32_t src_node(const Row3& w, int which) {
        return (uint32_t)(which < 0 ? w.rm : (which == 0 ? w.r0 : w.rp));
    }
    static __device__ __forceinline__ uint32_t src_fluid(const Row3& w, int which) {
        return (uint32_t)__builtin_amdgcn_sbfe((int32_t)w.bits, (uint32_t)(which + 1), 1u);
    }
    // Gather offsets of node n straight from the decoded rows: for each
    // direction the fluid bit of the source voxel selects, bitwise, between
    // the pulled population and the node's own opposite one, so no node
    // number -1 is formed and tested.  WB: also the wall links as a mask.
    //
    // SYM: symmetry planes on the y and/or z faces (Sec. 2.3).  A pull that
    // would leave the box through such a face reads the ghost row or plane,
    // the boundary layer itself (the entries and zlo / zhi), and takes the
    // population whose velocity is mirrored in that axis: the mirror image
    // of the flow on the other side of the plane sends it back.
    template <class T, int S, bool WB, bool SYM = false>
    __device__ __forceinline__ void offsets(const Raw& r, Pre c, uint32_t n, uint32_t chunk,
                                            uint32_t slack, uint32_t off[19], uint32_t& wb) const {
        constexpr uint32_t sz = sizeof(T);
        const uint32_t kb = chunk_kb<T, S>(chunk, slack);
        const uint32_t ekb = node_elem<S>(n) * sz + kb;
        off[0] = ekb;
        uint32_t walls = 0;
        // nodes on a mirrored face: pulls with c_y = +1 leave through y = 0, ...
        bool y0 = false, y1 = false, z0 = false, z1 = false;
        if constexpr (SYM) {
            const uint32_t y = (c >> bx) & ((1u << by) - 1u);
            const uint32_t z = (uint32_t)((uint64_t)c >> (bx + by));
            y0 = (sym & 1u) && y == 0;
            y1 = (sym & 1u) && y == ny - 1;
            z0 = (sym & 2u) && z == 0;
            z1 = (sym & 2u) && z == nz - 1;
        }
        visit(r, c, [&](auto I, const Row3& w, int which) {
            constexpr int i = decltype(I)::value;
            const uint32_t fluid = src_fluid(w, which);
            uint32_t pop = (uint32_t)i * kThreads * sz;
            if constexpr (SYM) {
                constexpr int cy = cdir(i, 1), cz = cdir(i, 2);
                const bool my = cy > 0 ? y0 : (cy < 0 ? y1 : false);
                const bool mz = cz > 0 ? z0 : (cz < 0 ? z1 : false);
                constexpr uint32_t py = (uint32_t)mirrored(i, 2) * kThreads * sz;
                constexpr uint32_t pz = (uint32_t)mirrored(i, 4) * kThreads * sz;
                constexpr uint32_t pyz = (uint32_t)mirrored(i, 6) * kThreads * sz;
                pop = my ? (mz ? pyz : py) : (mz ? pz : pop);
            }
            const uint32_t pulled = node_elem<S>(src_node(w, which)) * sz + (kb + pop);
            const uint32_t own = ekb + (uint32_t)opp(i) * kThreads * sz;
            off[i] = bit_select(fluid, pulled, own);
            if constexpr (WB) walls |= ~fluid & (1u << i);
        });
        if constexpr (WB) wb = walls;
    }
    // Both gathers of the reverse step of node n.  of[i]: the forward pull,
    // population i of the node at x - c_i, or the node's own opp(i) at a
    // wall.  ob[i]: its transpose, population i of the node at x + c_i (the
    // source of direction opp(i)), or the node's own opp(i) when that voxel
    // is solid: the value the forward pull of the wall link opp(i) had taken
    // from this node.
    template <class T, int S>
    __device__ __forceinline__ void offsets_adj(const Raw& r, Pre c, uint32_t n, uint32_t chunk,
                                                uint32_t slack, uint32_t of[19], uint32_t ob[19]) const {
        constexpr uint32_t sz = sizeof(T);
        const uint32_t kb = chunk_kb<T, S>(chunk, slack);
        const uint32_t ekb = node_elem<S>(n) * sz + kb;
        of[0] = ob[0] = ekb;
        visit(r, c, [&](auto I, const Row3& w, int which) {
            constexpr int i = decltype(I)::value;
            constexpr int j = opp(i);
            const uint32_t fluid = src_fluid(w, which);
            const uint32_t src = node_elem<S>(src_node(w, which)) * sz + kb;
            of[i] = bit_select(fluid, src + (uint32_t)i * kThreads * sz, ekb + (uint32_t)j * kThreads * sz);
            ob[j] = bit_select(fluid, src + (uint32_t)j * kThreads * sz, ekb + (uint32_t)i * kThreads * sz);
        });
    }

    // F16R: the references of the nodes a step pulls from.  The sources in
    // one row are voxels x - 1 .. x + 1, nodes r0 - 1 .. r0 + 1 (node numbers
    // run along a row), so one 8-byte window of the reference array per row,
    // starting at the even node (r0 - 1) & ~1 (4-byte aligned), holds them:
    // nine loads instead of nineteen.  Across the periodic x wrap (x = 0 or
    // nx - 1) the source at x -/+ 1 is the row's last / first node, outside the
    // window; issue_refs fetches those few separately.
    struct RefPlan {
        uint32_t ro[9];  // byte offset of each row's window in the reference array
        uint64_t pos;    // bits 2i, 2i + 1: position of value i's source node in its row's window
        uint32_t xw;     // bit 0: x == 0, bit 1: x == nx - 1, with nx >= 3 (sources across the wrap)
    };
    template <class T, int S>
    __device__ __forceinline__ void offsets_ref(const Raw& r, Pre c, uint32_t n, uint32_t chunk, uint32_t slack,
                                                uint32_t off[19], uint32_t& wb, RefPlan& plan) const {
        constexpr uint32_t sz = sizeof(T);
        const uint32_t kb = chunk_kb<T, S>(chunk, slack);
        const uint32_t ekb = node_elem<S>(n) * sz + kb;
        off[0] = ekb;
        uint32_t walls = 0, e[9];
        uint64_t pos = 0;
        visit(r, c, [&](auto I, const Row3& w, int which) {
            constexpr int i = decltype(I)::value;
            constexpr int R = row_of(i);
            const uint32_t fluid = src_fluid(w, which);
            const uint32_t node = src_node(w, which);
            const uint32_t pulled = node_elem<S>(node) * sz + (kb + (uint32_t)i * kThreads * sz);
            off[i] = bit_select(fluid, pulled, ekb + (uint32_t)opp(i) * kThreads * sz);
            walls |= ~fluid & (1u << i);
            if constexpr (i == 1 || i == 3 || i == 4 || i == 5 || i == 6 || i >= 15) {  // first visit of row R
                const uint32_t r0 = (uint32_t)w.r0;
                e[R] = (r0 == 0u ? 0u : r0 - 1u) & ~1u;
                plan.ro[R] = e[R] * sz;
            }
            pos |= (uint64_t)((node - e[R]) & 3u) << (2 * i);
        });
        pos |= (uint64_t)((n - e[0]) & 3u);   // the node itself, in its own row's window
        wb = walls;
        plan.pos = pos;
        // one or two voxels per row: the wrapped sources are the node itself
        // or its neighbour, inside the window
        const uint32_t x = c & ((1u << bx) - 1u);
        plan.xw = nx < 3 ? 0u : (x == 0 ? 1u : (x == nx - 1 ? 2u : 0u));
    }
    // Loads in flight for node n (issue_refs, before the next node's offsets
    // overwrite the plan), then rr[i] = reference of the node value i came
    // from, its own at a wall (finish_refs, with node n's plan and walls).
    template <class T>
    struct RefLoads {
        uint64_t win[9];
        T wrap[5];  // across the x wrap: sources of c_x = +1 (x = 0) or c_x = -1 (x = nx - 1)
    };
    template <class T, int S>
    __device__ __forceinline__ void issue_refs(const RefPlan& plan, const T* rb, uint32_t wb, const uint32_t* off,
                                               uint32_t chunk, uint32_t slack, RefLoads<T>& L) const {
        typedef uint32_t U2 __attribute__((ext_vector_type(2), aligned(4)));
        unroll<9>([&](auto k) {
            constexpr int R = decltype(k)::value;
            const U2 v = ld_off(reinterpret_cast<const U2*>(rb), plan.ro[R]);
            L.win[R] = (uint64_t)v.x | ((uint64_t)v.y << 32);
        });
        if (plan.xw) {
            // Node m of a pulled value i from its offset: the load reads element
            // chunk * S * 256 - slack + off / sizeof(T) of the state (64-bit:
            // states pass 4 GiB), which is node_elem(m) + i * 256.
            const bool left = plan.xw & 1u;  // x = 0: c_x = +1 pulls the row's last node
            unroll<5>([&](auto k) {
                constexpr int a = 2 * decltype(k)::value + 1;          // 1, 7, 9, 11, 13 ...
                constexpr int il = a == 1 ? 1 : a + 4, ir = il + 1;    // ... and 2, 8, 10, 12, 14
                const int i = left ? il : ir;
                if (!((wb >> i) & 1u)) {
                    const uint32_t o = left ? off[il] : off[ir];
                    const uint64_t ne = (uint64_t)chunk * (S * kThreads) - slack + o / (uint32_t)sizeof(T) -
                                        (uint64_t)i * kThreads;
                    const uint32_t m = (uint32_t)(ne / (S * kThreads)) * kThreads + (uint32_t)(ne % (S * kThreads));
                    L.wrap[decltype(k)::value] = ld_off(rb, m * (uint32_t)sizeof(T));
                }
            });
        }
    }
    template <class T>
    __device__ __forceinline__ void finish_refs(const RefPlan& plan, uint32_t wb, const RefLoads<T>& L,
                                                T rr[19]) const {
        auto pick = [&](int R, int i) -> T {
            const uint32_t q = (uint32_t)(plan.pos >> (2 * i)) & 3u;
            return __builtin_bit_cast(T, (uint16_t)(L.win[R] >> (16u * q)));
        };
        const T own = pick(0, 0);
        rr[0] = own;
        unroll<18>([&](auto k) {
            constexpr int i = decltype(k)::value + 1;
            T v = pick(row_of(i), i);
            if constexpr (i <= 14 && i != 3 && i != 4 && i != 5 && i != 6) {
                // the x-wrapped sources
                constexpr int slot = i <= 2 ? 0 : (i - 5) / 2;
                constexpr unsigned side = (i & 1) ? 1u : 2u;
                if (plan.xw == side) v = L.wrap[slot];
            }
            rr[i] = ((wb >> i) & 1u) ? own : v;
        });
    }
};
static_assert(BitmapIdx::row_of(7) == 1 && BitmapIdx::which_of(7) == -1 && BitmapIdx::row_of(9) == 2 &&
                  BitmapIdx::which_of(9) == -1 && BitmapIdx::row_of(13) == 4 && BitmapIdx::which_of(13) == -1 &&
                  BitmapIdx::row_of(14) == 3 && BitmapIdx::which_of(14) == 1,
              "row_of / which_of follow BitmapIdx::visit");

// ------------------------------------------------------------------ moments
// Moments of 19 values in the paper's order (rho, e, eps, jx, qx, jy, qy, jz,
// qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz): the rows of
// d'Humieres et al. (2002) evaluated on pair sums P_k = f_{2k-1} + f_{2k}
// (even rows) and differences D_k = f_{2k-1} - f_{2k} (odd rows).
struct Mom {
    float rho, e, eps, jx, qx, jy, qy, jz, qz, pxx, pixx, pww, piww, pxy, pyz, pxz, mx, my, mz;
};

__device__ __forceinline__ Mom moments(const float f[19]) {
    const float P1 = f[1] + f[2], P2 = f[3] + f[4], P3 = f[5] + f[6];
    const float P4 = f[7] + f[8], P5 = f[9] + f[10], P6 = f[11] + f[12], P7 = f[13] + f[14];
    const float P8 = f[15] + f[16], P9 = f[17] + f[18];
    const float D1 = f[1] - f[2], D2 = f[3] - f[4], D3 = f[5] - f[6];
    const float D4 = f[7] - f[8], D5 = f[9] - f[10], D6 = f[11] - f[12], D7 = f[13] - f[14];
    const float D8 = f[15] - f[16], D9 = f[17] - f[18];
    const float Pa = P1 + P2 + P3;               // |c|^2 = 1
    const float Pxy = P4 + P5, Pxz = P6 + P7, Pyz = P8 + P9;
    const float Pd = Pxy + Pxz + Pyz;            // |c|^2 = 2
    Mom m;
    m.rho = f[0] + Pa + Pd;
    m.e = -30.f * f[0] - 11.f * Pa + 8.f * Pd;
    m.eps = 12.f * f[0] - 4.f * Pa + Pd;
    m.pxx = 2.f * P1 - P2 - P3 + Pxy + Pxz - 2.f * Pyz;
    m.pixx = -4.f * P1 + 2.f * (P2 + P3) + Pxy + Pxz - 2.f * Pyz;
    m.pww = P2 - P3 + Pxy - Pxz;
    m.piww = -2.f * (P2 - P3) + Pxy - Pxz;
    m.pxy = P4 - P5;
    m.pxz = P6 - P7;
    m.pyz = P8 - P9;
    const float sx = D4 + D5 + D6 + D7, sy = D4 - D5 + D8 + D9, sz = D6 - D7 + D8 - D9;
    m.jx = D1 + sx;
    m.qx = -4.f * D1 + sx;
    m.jy = D2 + sy;
    m.qy = -4.f * D2 + sy;
    m.jz = D3 + sz;
    m.qz = -4.f * D3 + sz;
    m.mx = D4 + D5 - D6 - D7;
    m.my = -D4 + D5 + D8 + D9;
    m.mz = D6 - D7 - D8 + D9;
    return m;
}

// f_i += sum_k M_ki h_k  (h in moment order; M^T applied on pair halves).
__device__ __forceinline__ void add_back(float f[19], const Mom& h) {
    f[0] += h.rho - 30.f * h.e + 12.f * h.eps;
    const float base1 = h.rho - 11.f * h.e - 4.f * h.eps;
    const float Ex = base1 + 2.f * h.pxx - 4.f * h.pixx;
    const float Eyz = base1 - h.pxx + 2.f * h.pixx;
    const float Ey = Eyz + h.pww - 2.f * h.piww;
    const float Ez = Eyz - h.pww + 2.f * h.piww;
    const float base2 = h.rho + 8.f * h.e + h.eps;
    const float Exy = base2 + h.pxx + h.pixx + h.pww + h.piww;
    const float Exz = base2 + h.pxx + h.pixx - h.pww - h.piww;
    const float Eyz2 = base2 - 2.f * h.pxx - 2.f * h.pixx;
    const float Ox = h.jx - 4.f * h.qx, Oy = h.jy - 4.f * h.qy, Oz = h.jz - 4.f * h.qz;
    const float ax = h.jx + h.qx, ay = h.jy + h.qy, az = h.jz + h.qz;
    const float O4 = ax + ay + h.mx - h.my;
    const float O5 = ax - ay + h.mx + h.my;
    const float O6 = ax + az - h.mx + h.mz;
    const float O7 = ax - az - h.mx - h.mz;
    const float O8 = ay + az + h.my - h.mz;
    const float O9 = ay - az + h.my + h.mz;
    f[1] += Ex + Ox;            f[2] += Ex - Ox;
    f[3] += Ey + Oy;            f[4] += Ey - Oy;
    f[5] += Ez + Oz;            f[6] += Ez - Oz;
    f[7] += Exy + h.pxy + O4;   f[8] += Exy + h.pxy - O4;
    f[9] += Exy - h.pxy + O5;   f[10] += Exy - h.pxy - O5;
    f[11] += Exz + h.pxz + O6;  f[12] += Exz + h.pxz - O6;
    f[13] += Exz - h.pxz + O7;  f[14] += Exz - h.pxz - O7;
    f[15] += Eyz2 + h.pyz + O8; f[16] += Eyz2 + h.pyz - O8;
    f[17] += Eyz2 - h.pyz + O9; f[18] += Eyz2 - h.pyz - O9;
}

// Squared row norms of M: 19, 2394, 252, 10, 40, 36, 72, 12, 24, 4, 8.
constexpr float kInvE = 1.f / 2394.f, kInvEps = 1.f / 252.f, kInvJ = 1.f / 10.f,
                kInvQ = 1.f / 40.f, kInvPxx = 1.f / 36.f, kInvPixx = 1.f / 72.f,
                kInvPww = 1.f / 12.f, kInvPiww = 1.f / 24.f, kInvP = 1.f / 4.f, kInvM = 1.f / 8.f;

// Post-collision moment increments (m* - m) of the MRT collision with Guo
// forcing: dm_k = -s_k (m_k - m_eq_k) + (1 - s_k/2) mF_k, where m_eq uses the
// shifted momentum j = sum f c + F/2 (rho0 = 1, incompressible form with the
// misprints of Eq. MRT Equi read as corrected) and mF = M F_i in closed form
// (mF = d m_eq / d j . F).  Returned scaled by 1/|row|^2, ready for add_back.
__device__ __forceinline__ Mom collide_increment(const Mom& m, float jx, float jy, float jz,
                                                 float Fx, float Fy, float Fz, const RatesF& r) {
    const float xx = jx * jx, yy = jy * jy, zz = jz * jz, jj = xx + yy + zz;
    const float uF = jx * Fx + jy * Fy + jz * Fz;
    const float pxx_eq = 2.f * xx - yy - zz, pww_eq = yy - zz;
    const float X = 2.f * jx * Fx - jy * Fy - jz * Fz, Wf = jy * Fy - jz * Fz;
    const float ge = 1.f - 0.5f * r.s_e, geps = 1.f - 0.5f * r.s_eps, gq = 1.f - 0.5f * r.s_q,
                gnu = 1.f - 0.5f * r.s_nu, gpi = 1.f - 0.5f * r.s_pi;
    Mom h;
    h.rho = 0.f;
    h.e = (-r.s_e * (m.e - (-11.f * m.rho + 19.f * jj)) + ge * 38.f * uF) * kInvE;
    h.eps = (-r.s_eps * (m.eps - (3.f * m.rho - 5.5f * jj)) - geps * 11.f * uF) * kInvEps;
    h.jx = Fx * kInvJ;
    h.jy = Fy * kInvJ;
    h.jz = Fz * kInvJ;
    const float tq = -2.f / 3.f;
    h.qx = (-r.s_q * (m.qx - tq * jx) + gq * tq * Fx) * kInvQ;
    h.qy = (-r.s_q * (m.qy - tq * jy) + gq * tq * Fy) * kInvQ;
    h.qz = (-r.s_q * (m.qz - tq * jz) + gq * tq * Fz) * kInvQ;
    h.pxx = (-r.s_nu * (m.pxx - pxx_eq) + gnu * 2.f * X) * kInvPxx;
    h.pixx = (-r.s_pi * (m.pixx + 0.5f * pxx_eq) - gpi * X) * kInvPixx;
    h.pww = (-r.s_nu * (m.pww - pww_eq) + gnu * 2.f * Wf) * kInvPww;
    h.piww = (-r.s_pi * (m.piww + 0.5f * pww_eq) - gpi * Wf) * kInvPiww;
    h.pxy = (-r.s_nu * (m.pxy - jx * jy) + gnu * (jx * Fy + jy * Fx)) * kInvP;
    h.pyz = (-r.s_nu * (m.pyz - jy * jz) + gnu * (jy * Fz + jz * Fy)) * kInvP;
    h.pxz = (-r.s_nu * (m.pxz - jx * jz) + gnu * (jx * Fz + jz * Fx)) * kInvP;
    h.mx = -r.s_m * m.mx * kInvM;
    h.my = -r.s_m * m.my * kInvM;
    h.mz = -r.s_m * m.mz * kInvM;
    return h;
}

// ------------------------------------------------------------------ Zou-He
// Pressure boundaries on the x faces (Sec. 2.3, 3.1).  On the plane x = 0
// (side 1) the populations with c_x = +1, on x = nx - 1 (side 2) those with
// c_x = -1, arrive from outside the image; they are rebuilt from the known
// ones so that the node has the prescribed density deviation (drho_in /
// drho_out), no transverse velocity, equal non-equilibrium parts of the
// opposite pair along x, and diagonals that cancel the transverse momentum of
// the in-plane populations.  f holds deviations (the w rho0 parts cancel).
__device__ __forceinline__ void zou_he(float f[19], uint32_t side, float drho_in, float drho_out) {
    const float H0 = f[0] + (f[3] + f[4]) + (f[5] + f[6]) + (f[15] + f[16]) + (f[17] + f[18]);
    const float Ny = 0.5f * ((f[3] - f[4]) + (f[15] - f[16]) + (f[17] - f[18]));
    const float Nz = 0.5f * ((f[5] - f[6]) + (f[15] - f[16]) - (f[17] - f[18]));
    // Both faces' values, then selects: with two branches that store to
    // different elements the compiler turned f into a stack array.
    const bool in = side == 1u;
    const float ju_in = drho_in - (H0 + 2.f * (f[2] + f[8] + f[10] + f[12] + f[14]));
    const float ju_out = (H0 + 2.f * (f[1] + f[7] + f[9] + f[11] + f[13])) - drho_out;
    const float ju = in ? ju_in : ju_out;
    const float j3 = ju * (1.f / 3.f), j6 = ju * (1.f / 6.f);
    const float a1 = f[2] + j3, a7 = f[8] + j6 - Ny, a9 = f[10] + j6 + Ny, a11 = f[12] + j6 - Nz,
                a13 = f[14] + j6 + Nz;
    const float b2 = f[1] - j3, b8 = f[7] - j6 + Ny, b10 = f[9] - j6 - Ny, b12 = f[11] - j6 + Nz,
                b14 = f[13] - j6 - Nz;
    f[1] = in ? a1 : f[1];
    f[7] = in ? a7 : f[7];
    f[9] = in ? a9 : f[9];
    f[11] = in ? a11 : f[11];
    f[13] = in ? a13 : f[13];
    f[2] = in ? f[2] : b2;
    f[8] = in ? f[8] : b8;
    f[10] = in ? f[10] : b10;
    f[12] = in ? f[12] : b12;
    f[14] = in ? f[14] : b14;
}

// ------------------------------------------------------------------ TRT
// Two-relaxation-time collision (Sec. 2.1.2) applied link-wise, for two-rate
// sets (SRT, B, E): every even non-conserved moment relaxes at sp = s_nu and
// every odd one at sm = s_q.  Per opposite pair (a, b = opp(a)) the symmetric
// part (f_a + f_b)/2 relaxes towards that of the incompressible equilibrium
// e_a = w_a [drho + 3 c.j + 9/2 (c.j)^2 - 3/2 j.j] and gains (1 - sp/2) times
// that of Guo's source w_a [3 (c - u).F + 9 (c.u)(c.F)]; the antisymmetric
// part does the same at sm.  With the shifted j in the equilibrium this is the
// MRT collision of those rates: the momentum gets sm F/2 from the relaxation
// and (1 - sm/2) F from the source.  f holds deviations f - w rho0 on entry
// and exit; returns the shifted momentum and drho for the reduction.
struct TrtOut {
    float jx, jy, jz, rho;
};
__device__ __forceinline__ TrtOut collide_trt(float f[19], float Fx, float Fy, float Fz, float sp,
                                              float sm) {
    float S[10], D[10];
    unroll<9>([&](auto k) {
        constexpr int a = 2 * decltype(k)::value + 1;
        S[a >> 1] = f[a] + f[a + 1];
        D[a >> 1] = f[a] - f[a + 1];
    });
    // pairs: 0 x, 1 y, 2 z, 3 (1,1,0), 4 (1,-1,0), 5 (1,0,1), 6 (1,0,-1), 7 (0,1,1), 8 (0,1,-1)
    const float rho = f[0] + ((S[0] + S[1] + S[2]) + ((S[3] + S[4]) + (S[5] + S[6]) + (S[7] + S[8])));
    const float jx = D[0] + (D[3] + D[4]) + (D[5] + D[6]) + 0.5f * Fx;
    const float jy = D[1] + (D[3] - D[4]) + (D[7] + D[8]) + 0.5f * Fy;
    const float jz = D[2] + (D[5] - D[6]) + (D[7] - D[8]) + 0.5f * Fz;
    const float jj = jx * jx + jy * jy + jz * jz, uF = jx * Fx + jy * Fy + jz * Fz;
    const float gp = 1.f - 0.5f * sp, gm = 1.f - 0.5f * sm;
    const float A0 = sp * (rho - 1.5f * jj) - 3.f * gp * uF;   // per-node part of the symmetric update
    const float a1 = 0.5f * (1.f - sp), a2 = 0.5f * (1.f - sm), c45 = 4.5f * sp, g9 = 9.f * gp;
    f[0] = (1.f - sp) * f[0] + (1.f / 3.f) * A0;
    auto pair = [&](int a, float w, float cj, float cF) {
        const float P = (c45 * cj + g9 * cF) * cj + A0;
        const float hp = a1 * S[a >> 1] + w * P;
        const float hm = a2 * D[a >> 1] + 3.f * w * (sm * cj + gm * cF);
        f[a] = hp + hm;
        f[a + 1] = hp - hm;
    };
    constexpr float w1 = 1.f / 18.f, w2 = 1.f / 36.f;
    pair(1, w1, jx, Fx);
    pair(3, w1, jy, Fy);
    pair(5, w1, jz, Fz);
    pair(7, w2, jx + jy, Fx + Fy);
    pair(9, w2, jx - jy, Fx - Fy);
    pair(11, w2, jx + jz, Fx + Fz);
    pair(13, w2, jx - jz, Fx - Fz);
    pair(15, w2, jy + jz, Fy + Fz);
    pair(17, w2, jy - jz, Fy - Fz);
    return TrtOut{jx, jy, jz, rho};
}

// ------------------------------------------------------------------ reductions
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* out) {
    __shared__ double red[kThreads / 64][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Which window position a block takes.  A sweep goes through the chunks in
// windows of G = gridDim.x; logical block lb takes chunks lb, lb + G, ...
// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8),
// each with its own L2.  The map below hands each XCD runs of kXcdRun
// consecutive chunks of the window: the rows that neighbour a node lie a few
// chunks away in the node order, so most of its gathers hit the L2 of the XCD
// that reads them, while all XCDs still work inside one window of the node
// list and share the MALL and the DRAM pages it covers.  (Measured on a 512^3
// rock at 5 blocks per CU: runs of 16-32 chunks +3% FP32 over plain
// round-robin, runs of 64 equal, 128 -3%; a contiguous eighth of the list per
// XCD -6%.  At one block per CU, where 256 blocks make runs of 32 the whole
// window of each XCD: plain round-robin -4%, bands of 2 to 16 windows per
// XCD -2% to -10%.)  A grid that is not a multiple of 8 kXcdRun keeps
// plain round-robin.  The map is a bijection of [0, G).
constexpr uint32_t kXcdRun = 32;
__device__ __forceinline__ uint32_t logical_block() {
    const uint32_t G = gridDim.x, b = blockIdx.x;
    if (G % (8u * kXcdRun) != 0) return b;
    const uint32_t xcd = b & 7u, j = b >> 3;
    return ((j / kXcdRun) * 8u + xcd) * kXcdRun + j % kXcdRun;
}

// Fixed-order FP64 sum of per-block partials [grid][K] into out[0..K-1], by
// one whole block: strided per-thread sums, then the block_sum tree.
template <int K>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partials, int grid,
                                                double* __restrict__ out) {
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < grid; b += kThreads)
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] += partials[(int64_t)b * K + k];
    block_sum<K>(s, out);
}

template <int K>
__global__ void __launch_bounds__(kThreads)
k_finalize(const double* __restrict__ partials, int grid, double* __restrict__ out) {
    reduce_partials<K>(partials, grid, out);
}

// Reduce per-block partials [grid][4] of one step into the next slot of the
// ring of per-step sums, the slot being the device counter *ctr (steps
// reduced so far) modulo kRingSlots, then advance the counter.  Run by one
// whole block; keeping the slot on the device lets a captured sequence of
// steps replay with unchanged arguments.
__device__ __forceinline__ void reduce_into_ring(const double* __restrict__ partials, int grid,
                                                 double* __restrict__ ring, uint32_t* __restrict__ ctr) {
    const uint32_t slot = ctr[0];
    reduce_partials<4>(partials, grid, ring + (size_t)(slot % kRingSlots) * 4);
    __syncthreads();
    if (threadIdx.x == 0) ctr[0] = slot + 1u;
}

__global__ void __launch_bounds__(kThreads)
k_finalize_ring(const double* __restrict__ partials, int grid, double* __restrict__ ring,
                uint32_t* __restrict__ ctr) {
    reduce_into_ring(partials, grid, ring, ctr);
}

// ------------------------------------------------------------------ step
// FW: full-way bounce-back (Sec. 2.3).  A population sent into a wall comes
// back one step later than with the halfway wall, so at a wall link the node
// takes fh_opp(i) of two steps ago.  `wall` keeps, per node and population p,
// the fh_p this node had one step ago (same layout as a state): at a wall link
// in direction i the node reads slot opp(i) there and writes back the fh_opp(i)
// the halfway gather brought (the previous step's); only the node itself
// touches its slots.
// ZH: Zou-He pressure boundaries on the x faces (bitmap index only, which
// knows each node's x).  SYM: symmetry planes on the y / z faces (bitmap
// index, BitmapIdx::offsets).
// The plain MRT step fits 96 VGPRs without spilling, so 5 blocks of it fit a
// CU, which the 16-bit storages use (FP32 storage launches one block per CU);
// the reference-density, link-wise TRT, full-way and symmetry variants would
// spill there and keep the compiler's choice.
template <class C, class Ix, bool FIELD, bool TRT, bool FW, bool ZH = false, bool SYM = false>
__global__ void __launch_bounds__(kThreads, (C::kRef || TRT || FW || SYM) ? 1 : 5)
k_step(const typename C::T* __restrict__ src, typename C::T* __restrict__ dst, Ix ix,
       uint32_t slack, uint32_t nf, RatesF r, float Fx0, float Fy0, float Fz0,
       const float* __restrict__ field, float scale, float inv, double* __restrict__ partials,
       const double* __restrict__ prev_partials, double* __restrict__ ring, uint32_t* __restrict__ ctr,
       float* __restrict__ wall,
       float drho_in = 0.f, float drho_out = 0.f) {
    using T = typename C::T;
    constexpr int S = C::kSlots;
    constexpr bool REF = C::kRef;
    // The previous step's block partials are reduced here, by the first block,
    // so a time step is a single launch; kernel order makes them visible.
    if (prev_partials != nullptr && blockIdx.x == 0) {
        reduce_into_ring(prev_partials, gridDim.x, ring, ctr);
        __syncthreads();
    }
    const uint32_t lb = logical_block();
    const uint32_t chunks = (nf + kThreads - 1) / kThreads;
    const uint32_t G = gridDim.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // Software pipeline over this block's chunks c, c + G, c + 2G, ...: while
    // the populations of node n are gathered, the neighbour index of the next
    // node n1 is resolved and the coordinate of the one after (n2) is
    // fetched, so each iteration waits for memory once.  Node numbers past
    // the list are clamped to the last node for loads; what such a lane
    // stores goes to its own padded slot (below).
    auto node_of = [&](uint32_t cc) { return min(cc * kThreads + threadIdx.x, nf - 1); };
    uint32_t c = lb;
    if (c < chunks) {
        uint32_t n = node_of(c), n1 = node_of(c + G);
        typename Ix::Pre pre1 = ix.prefetch(n1);
        uint32_t off[19];
        uint32_t wb = 0;    // wall links of node n (FW, REF)
        uint32_t side = 0;  // pressure face of node n (ZH only)
        typename Ix::RefPlan plan;  // REF: where the references of node n's sources are
        // REF: the reference arrays after the chunks of the two states
        const T* rsrc = src + (size_t)chunks * (S * kThreads);
        T* rdst = dst + (size_t)chunks * (S * kThreads);
        auto resolve = [&](const typename Ix::Raw& raw, typename Ix::Pre p, uint32_t node, uint32_t chunk) {
            if constexpr (REF)
                ix.template offsets_ref<T, S>(raw, p, node, chunk, slack, off, wb, plan);
            else
                ix.template offsets<T, S, FW, SYM>(raw, p, node, chunk, slack, off, wb);
        };
        {
            const typename Ix::Pre p0 = ix.prefetch(n);
            typename Ix::Raw raw;
            ix.load(n, p0, raw);
            resolve(raw, p0, n, c);
            if constexpr (ZH) side = ix.x_face(p0);
        }
        for (;;) {
            // (1) index loads of the next node, (2) population loads of this
            // node and the coordinate two nodes ahead, (3) decode the index
            // while the populations are in flight, (4) collide and store.
            __builtin_amdgcn_sched_barrier(0);
            typename Ix::Raw raw;
            ix.load(n1, pre1, raw);
            __builtin_amdgcn_sched_barrier(0);
            const T* gb = chunk_base<T, S>(src, c, slack);
            T fr[19];
            unroll<19>([&](auto k) {
                constexpr int i = decltype(k)::value;
                fr[i] = ld_off(gb, off[i]);
            });
            // REF: the reference density of the node each value came from: the
            // source node, or the node itself at a wall
            typename Ix::template RefLoads<T> refl;
            if constexpr (REF) ix.template issue_refs<T, S>(plan, rsrc, wb, off, c, slack, refl);
            const typename Ix::RefPlan plan_n = plan;
            float wv[19];
            float* wc = FW ? wall + (size_t)c * kChunkElems : nullptr;
            // a lane's own slot in chunk c: node c * 256 + lane, or for a lane
            // past the list a padded slot that no other lane reads or writes
            const uint32_t own = threadIdx.x * 4u;
            if constexpr (FW) {
                unroll<18>([&](auto k) {
                    constexpr int i = decltype(k)::value + 1;
                    wv[i] = ld_off(wc + opp(i) * kThreads, own);
                });
            }
            const typename Ix::Pre pre2 = ix.prefetch(node_of(c + 2 * G));
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t wb_n = wb, side_n = side;
            {
                resolve(raw, pre1, n1, c + G);
                if constexpr (ZH) side = ix.x_face(pre1);
            }
            __builtin_amdgcn_sched_barrier(0);
            T rr[19];
            if constexpr (REF) ix.finish_refs(plan_n, wb_n, refl, rr);
            float f[19];
            unroll<19>([&](auto k) {
                constexpr int i = decltype(k)::value;
                f[i] = C::cvt(fr[i], inv);
                if constexpr (REF) f[i] += wgt(i) * (float)rr[i];
            });
            if constexpr (FW) {
                // wall link i: use the value of two steps ago, keep this one
                unroll<18>([&](auto k) {
                    constexpr int i = decltype(k)::value + 1;
                    const bool w = (wb_n >> i) & 1u;
                    const float halfway = f[i];
                    f[i] = w ? wv[i] : halfway;
                    wv[i] = w ? halfway : wv[i];
                });
                unroll<18>([&](auto k) {
                    constexpr int i = decltype(k)::value + 1;
                    st_off(wc + opp(i) * kThreads, own, wv[i]);
                });
            }
            if constexpr (ZH) {
                if (side_n != 0u) zou_he(f, side_n, drho_in, drho_out);
            }
            float Fx = Fx0, Fy = Fy0, Fz = Fz0;
            if (FIELD) {
                Fx = field[n];
                Fy = field[nf + n];
                Fz = field[2 * nf + n];
            }
            float jx, jy, jz, drho;
            if constexpr (TRT) {
                const TrtOut o = collide_trt(f, Fx, Fy, Fz, r.s_nu, r.s_q);
                jx = o.jx;
                jy = o.jy;
                jz = o.jz;
                drho = o.rho;
            } else {
                const Mom m = moments(f);
                jx = m.jx + 0.5f * Fx;
                jy = m.jy + 0.5f * Fy;
                jz = m.jz + 0.5f * Fz;
                drho = m.rho;
                add_back(f, collide_increment(m, jx, jy, jz, Fx, Fy, Fz, r));
            }
            // Lanes past the list carry n = nf - 1 for their loads and write
            // their results to their own padded slots (element lane of the
            // last chunk), which nothing reads, so the stores stay
            // unconditional (no branch for the compiler to sink the gathers
            // into); the reduction leaves them out.
            const bool live = c * kThreads + threadIdx.x < nf;
            acc[0] += live ? (double)jx : 0.0;
            acc[1] += live ? (double)jy : 0.0;
            acc[2] += live ? (double)jz : 0.0;
            acc[3] += live ? (double)drho : 0.0;
            T* db = dst + (size_t)c * (S * kThreads);
            const uint32_t so = threadIdx.x * (uint32_t)sizeof(T);
            if constexpr (REF) {
                // the node's new reference: its density deviation, which the
                // collision conserves, rounded to the stored type
                const T r_new = (T)drho;
                const float rf = (float)r_new;
                st_stream(rdst + (size_t)c * kThreads, so, r_new);
                unroll<19>([&](auto k) {
                    constexpr int i = decltype(k)::value;
                    st_stream(db + i * kThreads, so, C::enc(f[i] - wgt(i) * rf, scale));
                });
            } else {
                unroll<19>([&](auto k) {
                    constexpr int i = decltype(k)::value;
                    st_stream(db + i * kThreads, so, C::enc(f[i], scale));
                });
            }
            c += G;
            if (c >= chunks) break;
            n = n1;
            n1 = node_of(c + G);
            pre1 = pre2;
        }
    }
    block_sum<4>(acc, partials + (size_t)lb * 4);
}

__global__ void k_zero(uint32_t* p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <class C>
__global__ void k_rescale(typename C::T* p, int64_t count, float factor) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        p[i] = C::enc(C::cvt(p[i], 1.f), factor);
    }
}

// ------------------------------------------------------------------ adjoint
// Quadratic part of the j-derivative of the equilibrium moments, contracted
// with moment-space weights w: G_a(v, w) = sum_l w_l d m_eq_l / d j_a at j = v.
struct Vec3 {
    float x, y, z;
};
__device__ __forceinline__ Vec3 gquad(float vx, float vy, float vz, const Mom& w) {
    Vec3 g;
    const float ee = 38.f * w.e - 11.f * w.eps;
    g.x = ee * vx + 4.f * vx * w.pxx - 2.f * vx * w.pixx + vy * w.pxy + vz * w.pxz;
    g.y = ee * vy - 2.f * vy * w.pxx + vy * w.pixx + 2.f * vy * w.pww - vy * w.piww +
          vx * w.pxy + vz * w.pyz;
    g.z = ee * vz - 2.f * vz * w.pxx + vz * w.pixx - 2.f * vz * w.pww + vz * w.piww +
          vy * w.pyz + vx * w.pxz;
    return g;
}

// Reverse step n at every node:
//   b = P^T a^{n+1}            (transpose of the pull stream: gather from x + c_i)
//   f = P fh^{n-1}             (the forward's gathered populations of step n)
//   a^n = b + M^T nu,  nu = (d dm / d m)^T D^-1 M b
// plus the rate-class and body-force sensitivities b^T dC/ds, b^T dC/dF.
// The body-force sensitivity of the node is added to an FP32 accumulator
// [3][stride] (written, not added, when `first`: the first reverse step of a
// checkpoint segment); the host folds it into the FP64 total once per segment,
// so an FP32 sum runs over at most one segment.  Each accumulator value is
// touched once per step, so it is read and written with non-temporal
// accesses that leave L2 to the gathered lines.  Software pipeline as in
// k_step: the index entries of the next node are loaded and decoded while
// this node's 38 gathers are in flight.  It is launched with one block per
// compute unit (its two gathered arrays make it bound by L2 misses, not by
// latency), where the registers this pipeline needs (151) cost no occupancy.
// Tail lanes as in k_step: lanes past the list load node nf - 1 and store to
// their own padded slots.
template <class Ix, bool FIELD>
__global__ void __launch_bounds__(kThreads)
k_adjoint(const float* __restrict__ ain, float* __restrict__ aout, const float* __restrict__ st,
          Ix ix, uint32_t slack, uint32_t nf, RatesF r, float Fx0, float Fy0, float Fz0,
          const float* __restrict__ field, float* __restrict__ dkdF, uint32_t stride, int first,
          double* __restrict__ partials) {
    const uint32_t lb = logical_block();
    const uint32_t chunks = (nf + kThreads - 1) / kThreads;
    const uint32_t G = gridDim.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    auto node_of = [&](uint32_t cc) { return min(cc * kThreads + threadIdx.x, nf - 1); };
    uint32_t c = lb;
    if (c < chunks) {
        uint32_t n = node_of(c), n1 = node_of(c + G);
        typename Ix::Pre pre1 = ix.prefetch(n1);
        uint32_t of[19], ob[19];
        {
            const typename Ix::Pre p0 = ix.prefetch(n);
            typename Ix::Raw raw;
            ix.template load<false>(n, p0, raw);
            ix.template offsets_adj<float, 19>(raw, p0, n, c, slack, of, ob);
        }
        for (;;) {
            __builtin_amdgcn_sched_barrier(0);
            typename Ix::Raw raw;
            ix.template load<false>(n1, pre1, raw);
            __builtin_amdgcn_sched_barrier(0);
            // f: the forward's pulls; b: the transposed pulls
            const float* sb = chunk_base(st, c, slack);
            const float* ab = chunk_base(ain, c, slack);
            float f[19], b[19];
            unroll<19>([&](auto k) {
                constexpr int i = decltype(k)::value;
                f[i] = ld_off(sb, of[i]);
                b[i] = ld_off(ab, ob[i]);
            });
            const uint32_t e = c * kThreads + threadIdx.x;   // this lane's slot
            float d[3] = {0.f, 0.f, 0.f};
            if (!first) {
                d[0] = __builtin_nontemporal_load(dkdF + e);
                d[1] = __builtin_nontemporal_load(dkdF + stride + e);
                d[2] = __builtin_nontemporal_load(dkdF + 2 * stride + e);
            }
            float Fx = Fx0, Fy = Fy0, Fz = Fz0;
            if (FIELD) {
                Fx = field[n];
                Fy = field[nf + n];
                Fz = field[2 * nf + n];
            }
            const typename Ix::Pre pre2 = ix.prefetch(node_of(c + 2 * G));
            __builtin_amdgcn_sched_barrier(0);
            ix.template offsets_adj<float, 19>(raw, pre1, n1, c + G, slack, of, ob);
            __builtin_amdgcn_sched_barrier(0);

            const Mom m = moments(f);
            const float jx = m.jx + 0.5f * Fx, jy = m.jy + 0.5f * Fy, jz = m.jz + 0.5f * Fz;
            const float xx = jx * jx, yy = jy * jy, zz = jz * jz, jj = xx + yy + zz;
            const float uF = jx * Fx + jy * Fy + jz * Fz;
            const float pxx_eq = 2.f * xx - yy - zz, pww_eq = yy - zz;
            const float X = 2.f * jx * Fx - jy * Fy - jz * Fz, Wf = jy * Fy - jz * Fz;
            Mom mu = moments(b);
            mu.rho *= 1.f / 19.f;
            mu.e *= kInvE;
            mu.eps *= kInvEps;
            mu.jx *= kInvJ;
            mu.jy *= kInvJ;
            mu.jz *= kInvJ;
            mu.qx *= kInvQ;
            mu.qy *= kInvQ;
            mu.qz *= kInvQ;
            mu.pxx *= kInvPxx;
            mu.pixx *= kInvPixx;
            mu.pww *= kInvPww;
            mu.piww *= kInvPiww;
            mu.pxy *= kInvP;
            mu.pyz *= kInvP;
            mu.pxz *= kInvP;
            mu.mx *= kInvM;
            mu.my *= kInvM;
            mu.mz *= kInvM;
            // rate-class sensitivities: mu_l * (-(m_l - m_eq_l) - mF_l / 2)
            const bool live = e < nf;
            const float tq = -2.f / 3.f;
            const float a0 = mu.e * (-(m.e - (-11.f * m.rho + 19.f * jj)) - 19.f * uF);
            const float a1 = mu.eps * (-(m.eps - (3.f * m.rho - 5.5f * jj)) + 5.5f * uF);
            const float a2 = mu.qx * (-(m.qx - tq * jx) + Fx / 3.f) + mu.qy * (-(m.qy - tq * jy) + Fy / 3.f) +
                             mu.qz * (-(m.qz - tq * jz) + Fz / 3.f);
            const float a3 = mu.pxx * (-(m.pxx - pxx_eq) - X) + mu.pww * (-(m.pww - pww_eq) - Wf) +
                             mu.pxy * (-(m.pxy - jx * jy) - 0.5f * (jx * Fy + jy * Fx)) +
                             mu.pyz * (-(m.pyz - jy * jz) - 0.5f * (jy * Fz + jz * Fy)) +
                             mu.pxz * (-(m.pxz - jx * jz) - 0.5f * (jx * Fz + jz * Fx));
            const float a4 = mu.pixx * (-(m.pixx + 0.5f * pxx_eq) + 0.5f * X) +
                             mu.piww * (-(m.piww + 0.5f * pww_eq) + 0.5f * Wf);
            const float a5 = -(mu.mx * m.mx + mu.my * m.my + mu.mz * m.mz);
            acc[0] += live ? (double)a0 : 0.0;
            acc[1] += live ? (double)a1 : 0.0;
            acc[2] += live ? (double)a2 : 0.0;
            acc[3] += live ? (double)a3 : 0.0;
            acc[4] += live ? (double)a4 : 0.0;
            acc[5] += live ? (double)a5 : 0.0;
            // c_l = s_l mu_l (equilibrium path), d_l = (1 - s_l/2) mu_l (source path)
            Mom cw, dw;
            cw.e = r.s_e * mu.e;       dw.e = (1.f - 0.5f * r.s_e) * mu.e;
            cw.eps = r.s_eps * mu.eps; dw.eps = (1.f - 0.5f * r.s_eps) * mu.eps;
            cw.pxx = r.s_nu * mu.pxx;  dw.pxx = (1.f - 0.5f * r.s_nu) * mu.pxx;
            cw.pixx = r.s_pi * mu.pixx; dw.pixx = (1.f - 0.5f * r.s_pi) * mu.pixx;
            cw.pww = r.s_nu * mu.pww;  dw.pww = (1.f - 0.5f * r.s_nu) * mu.pww;
            cw.piww = r.s_pi * mu.piww; dw.piww = (1.f - 0.5f * r.s_pi) * mu.piww;
            cw.pxy = r.s_nu * mu.pxy;  dw.pxy = (1.f - 0.5f * r.s_nu) * mu.pxy;
            cw.pyz = r.s_nu * mu.pyz;  dw.pyz = (1.f - 0.5f * r.s_nu) * mu.pyz;
            cw.pxz = r.s_nu * mu.pxz;  dw.pxz = (1.f - 0.5f * r.s_nu) * mu.pxz;
            const float cqx = r.s_q * mu.qx, cqy = r.s_q * mu.qy, cqz = r.s_q * mu.qz;
            const float gq = 1.f - 0.5f * r.s_q;
            const Vec3 gjc = gquad(jx, jy, jz, cw);
            const Vec3 gFd = gquad(Fx, Fy, Fz, dw);
            const Vec3 gjd = gquad(jx, jy, jz, dw);
            Mom nu;
            nu.rho = -11.f * cw.e + 3.f * cw.eps;
            nu.jx = gjc.x + gFd.x + tq * cqx;
            nu.jy = gjc.y + gFd.y + tq * cqy;
            nu.jz = gjc.z + gFd.z + tq * cqz;
            nu.e = -r.s_e * mu.e;
            nu.eps = -r.s_eps * mu.eps;
            nu.qx = -r.s_q * mu.qx;
            nu.qy = -r.s_q * mu.qy;
            nu.qz = -r.s_q * mu.qz;
            nu.pxx = -r.s_nu * mu.pxx;
            nu.pixx = -r.s_pi * mu.pixx;
            nu.pww = -r.s_nu * mu.pww;
            nu.piww = -r.s_pi * mu.piww;
            nu.pxy = -r.s_nu * mu.pxy;
            nu.pyz = -r.s_nu * mu.pyz;
            nu.pxz = -r.s_nu * mu.pxz;
            nu.mx = -r.s_m * mu.mx;
            nu.my = -r.s_m * mu.my;
            nu.mz = -r.s_m * mu.mz;
            // body force: F enters through the shift j = m_j + F/2, through
            // mF = (d m_eq / d j) F, and directly as the momentum source.
            d[0] += 0.5f * nu.jx + gjd.x + tq * gq * mu.qx + mu.jx;
            d[1] += 0.5f * nu.jy + gjd.y + tq * gq * mu.qy + mu.jy;
            d[2] += 0.5f * nu.jz + gjd.z + tq * gq * mu.qz + mu.jz;
            __builtin_nontemporal_store(d[0], dkdF + e);
            __builtin_nontemporal_store(d[1], dkdF + stride + e);
            __builtin_nontemporal_store(d[2], dkdF + 2 * stride + e);
            add_back(b, nu);
            float* ob_ = aout + (size_t)c * kChunkElems;
            unroll<19>([&](auto k) {
                constexpr int i = decltype(k)::value;
                st_stream(ob_ + i * kThreads, threadIdx.x * 4u, b[i]);
            });
            c += G;
            if (c >= chunks) break;
            n = n1;
            n1 = node_of(c + G);
            pre1 = pre2;
        }
    }
    double part[6];
    block_sum<6>(acc, part);
    if ((int)threadIdx.x < 6) partials[(size_t)lb * 6 + threadIdx.x] += part[threadIdx.x];
}

// dk_dF[a][n] += acc[a][n] (FP64 total += one segment's FP32 sum), n < nf.
__global__ void k_fold(double* __restrict__ d, const float* __restrict__ acc, int64_t nf, int64_t stride) {
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nf;
         n += (int64_t)gridDim.x * blockDim.x) {
        d[n] += (double)acc[n];
        d[nf + n] += (double)acc[stride + n];
        d[2 * nf + n] += (double)acc[2 * stride + n];
    }
}

__global__ void k_seed(float* adj, int64_t nf, int axis, float kappa) {
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nf;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = (n / kThreads) * kChunkElems + (n % kThreads);
        for (int i = 0; i < 19; ++i) adj[e + (int64_t)i * kThreads] = kappa * (float)cdir(i, axis);
    }
}

__global__ void k_add_uniform(double* d, int64_t nf, double vx, double vy, double vz) {
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nf;
         n += (int64_t)gridDim.x * blockDim.x) {
        d[n] += vx;
        d[nf + n] += vy;
        d[2 * nf + n] += vz;
    }
}

int grid_for(int64_t n) {
    int64_t g = (n + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

TableIdx table_view(const IndexView& v) { return TableIdx{v.table, (uint32_t)v.stride}; }
BitmapIdx bitmap_view(const IndexView& v) {
    const uint32_t plane = (uint32_t)v.ny * (uint32_t)v.R;         // entries per plane
    const uint32_t wrap = (uint32_t)(v.nz - 1) * plane;
    const bool mz = (v.sym & 2) != 0;
    return BitmapIdx{v.coords, static_cast<const uint4*>(v.ent), static_cast<const uint4*>(v.wrap),
                     static_cast<const uint4*>(v.count), (uint32_t)v.nx, (uint32_t)v.ny,
                     (uint32_t)v.nz, (uint32_t)v.R, (uint32_t)v.bx, (uint32_t)v.by,
                     mz ? 0u : wrap, mz ? 0u : 0u - wrap, (uint32_t)v.sym};
}

template <class C, class Ix, bool TRT, bool FW, bool SYM = false>
hipError_t step_launch(const StepLaunch& a, Ix ix, hipStream_t s) {
    using T = typename C::T;
    const T* src = static_cast<const T*>(a.src);
    T* dst = static_cast<T*>(a.dst);
    if (a.field)
        hipLaunchKernelGGL((k_step<C, Ix, true, TRT, FW, false, SYM>), dim3(a.grid), dim3(kThreads), 0, s, src, dst,
                           ix, (uint32_t)a.idx.slack, (uint32_t)a.nf, a.rates, a.F[0], a.F[1], a.F[2], a.field,
                           a.scale, a.inv_scale, a.partials, a.prev_partials, a.ring, a.ctr, a.wall, 0.f, 0.f);
    else
        hipLaunchKernelGGL((k_step<C, Ix, false, TRT, FW, false, SYM>), dim3(a.grid), dim3(kThreads), 0, s, src,
                           dst, ix, (uint32_t)a.idx.slack, (uint32_t)a.nf, a.rates, a.F[0], a.F[1], a.F[2], nullptr,
                           a.scale, a.inv_scale, a.partials, a.prev_partials, a.ring, a.ctr, a.wall, 0.f, 0.f);
    return hipGetLastError();
}

// Zou-He pressure faces: FP32 storage, bitmap index, uniform (zero) force,
// halfway bounce-back.
template <bool TRT>
hipError_t step_pressure(const StepLaunch& a, BitmapIdx ix, hipStream_t s) {
    hipLaunchKernelGGL((k_step<CodecF32, BitmapIdx, false, TRT, false, true>), dim3(a.grid), dim3(kThreads), 0, s,
                       static_cast<const float*>(a.src), static_cast<float*>(a.dst), ix, (uint32_t)a.idx.slack,
                       (uint32_t)a.nf, a.rates, a.F[0], a.F[1], a.F[2], nullptr, a.scale, a.inv_scale, a.partials,
                       a.prev_partials, a.ring, a.ctr, nullptr, a.drho_in, a.drho_out);
    return hipGetLastError();
}

// Full-way bounce-back is built for FP32 storage only; symmetry planes for
// FP32 storage and the bitmap index, without pressure faces.
template <class C, class Ix, bool TRT>
hipError_t step_with(const StepLaunch& a, Ix ix, hipStream_t s) {
    if (a.pressure) {
        if constexpr (std::is_same<C, CodecF32>::value && std::is_same<Ix, BitmapIdx>::value) {
            if (!a.wall && !a.field && !a.idx.sym) return step_pressure<TRT>(a, ix, s);
        }
        return hipErrorInvalidValue;
    }
    if (a.idx.sym) {
        if constexpr (std::is_same<C, CodecF32>::value && std::is_same<Ix, BitmapIdx>::value) {
            if (a.wall) return step_launch<C, Ix, TRT, true, true>(a, ix, s);
            return step_launch<C, Ix, TRT, false, true>(a, ix, s);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (std::is_same<C, CodecF32>::value) {
        if (a.wall) return step_launch<C, Ix, TRT, true>(a, ix, s);
    } else {
        if (a.wall) return hipErrorInvalidValue;
    }
    return step_launch<C, Ix, TRT, false>(a, ix, s);
}

template <class C, bool TRT>
hipError_t step_codec(const StepLaunch& a, hipStream_t s) {
    if (a.idx.kind == kTable) return step_with<C, TableIdx, TRT>(a, table_view(a.idx), s);
    return step_with<C, BitmapIdx, TRT>(a, bitmap_view(a.idx), s);
}

template <bool TRT>
hipError_t step_collision(const StepLaunch& a, hipStream_t s) {
    switch (a.storage) {
        case kF32: return step_codec<CodecF32, TRT>(a, s);
        case kF16: return step_codec<CodecF16, TRT>(a, s);
        case kBF16: return step_codec<CodecBF16, TRT>(a, s);
        case kF16R: return step_codec<CodecF16R, TRT>(a, s);
    }
    return hipErrorInvalidValue;
}

template <class Ix>
hipError_t adjoint_with(const AdjLaunch& a, Ix ix, hipStream_t s) {
    if (a.field)
        hipLaunchKernelGGL((k_adjoint<Ix, true>), dim3(a.grid), dim3(kThreads), 0, s, a.adj_in,
                           a.adj_out, a.state, ix, (uint32_t)a.idx.slack, (uint32_t)a.nf, a.rates,
                           a.F[0], a.F[1], a.F[2], a.field, a.dk_acc, (uint32_t)a.acc_stride, (int)a.first,
                           a.partials);
    else
        hipLaunchKernelGGL((k_adjoint<Ix, false>), dim3(a.grid), dim3(kThreads), 0, s, a.adj_in,
                           a.adj_out, a.state, ix, (uint32_t)a.idx.slack, (uint32_t)a.nf, a.rates,
                           a.F[0], a.F[1], a.F[2], nullptr, a.dk_acc, (uint32_t)a.acc_stride, (int)a.first,
                           a.partials);
    return hipGetLastError();
}

}  // namespace

hipError_t static_scratch(void** ptr) {
    constexpr int kDevices = 64;
    static std::mutex mu;
    static void* addr[kDevices] = {};
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return he;
    if (dev < 0 || dev >= kDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (he != hipSuccess) return he;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_step(const StepLaunch& a, hipStream_t s) {
    return a.collision == kTrt ? step_collision<true>(a, s) : step_collision<false>(a, s);
}

hipError_t step_occupancy(int storage, int index_kind, int collision, int* blocks_per_cu) {
    auto q = [&](const void* k) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kThreads, 0);
    };
#define LBM_OCC(C, I, R) q(reinterpret_cast<const void*>(&k_step<C, I, false, R, false>))
#define LBM_OCC2(R)                                                     \
    if (index_kind == kTable) {                                         \
        if (storage == kF32) return LBM_OCC(CodecF32, TableIdx, R);     \
        if (storage == kF16) return LBM_OCC(CodecF16, TableIdx, R);     \
        if (storage == kF16R) return LBM_OCC(CodecF16R, TableIdx, R);   \
        return LBM_OCC(CodecBF16, TableIdx, R);                         \
    }                                                                   \
    if (storage == kF32) return LBM_OCC(CodecF32, BitmapIdx, R);        \
    if (storage == kF16) return LBM_OCC(CodecF16, BitmapIdx, R);        \
    if (storage == kF16R) return LBM_OCC(CodecF16R, BitmapIdx, R);      \
    return LBM_OCC(CodecBF16, BitmapIdx, R);
    if (collision == kTrt) {
        LBM_OCC2(true)
    }
    LBM_OCC2(false)
#undef LBM_OCC2
#undef LBM_OCC
}

hipError_t launch_finalize(const double* partials, int grid, double* ring, uint32_t* ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_ring, dim3(1), dim3(kThreads), 0, s, partials, grid, ring, ctr);
    return hipGetLastError();
}

hipError_t launch_finalize6(const double* partials, int grid, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize<6>, dim3(1), dim3(kThreads), 0, s, partials, grid, out);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s) {
    const int64_t words = (bytes + 3) / 4;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(words)), dim3(kThreads), 0, s,
                       static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

hipError_t launch_rescale(int storage, void* p, int64_t count, float factor, hipStream_t s) {
    const dim3 g(grid_for(count)), b(kThreads);
    switch (storage) {
        case kF32:
            hipLaunchKernelGGL(k_rescale<CodecF32>, g, b, 0, s, static_cast<float*>(p), count, factor);
            break;
        case kF16:
            hipLaunchKernelGGL(k_rescale<CodecF16>, g, b, 0, s, static_cast<_Float16*>(p), count,
                               factor);
            break;
        case kBF16:
            hipLaunchKernelGGL(k_rescale<CodecBF16>, g, b, 0, s, static_cast<uint16_t*>(p), count,
                               factor);
            break;
        case kF16R:
            hipLaunchKernelGGL(k_rescale<CodecF16R>, g, b, 0, s, static_cast<_Float16*>(p), count,
                               factor);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const AdjLaunch& a, hipStream_t s) {
    if (a.idx.kind == kTable) return adjoint_with(a, table_view(a.idx), s);
    return adjoint_with(a, bitmap_view(a.idx), s);
}

hipError_t launch_fold(double* dk_dF, const float* acc, int64_t nf, int64_t stride, hipStream_t s) {
    hipLaunchKernelGGL(k_fold, dim3(grid_for(nf)), dim3(kThreads), 0, s, dk_dF, acc, nf, stride);
    return hipGetLastError();
}

hipError_t launch_adjoint_seed(float* adj, int64_t nf, int axis, float kappa,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_seed, dim3(grid_for(nf)), dim3(kThreads), 0, s, adj, nf, axis,
                       kappa);
    return hipGetLastError();
}

hipError_t launch_add_uniform(double* d, int64_t nf, double vx, double vy, double vz,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_add_uniform, dim3(grid_for(nf)), dim3(kThreads), 0, s, d, nf, vx, vy, vz);
    return hipGetLastError();
}

}  // namespace lbm
