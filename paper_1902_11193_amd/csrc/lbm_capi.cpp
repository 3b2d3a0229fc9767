// C-ABI of liblbm (declarations and contracts in include/lbm.h).
#include "lbm.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_host.hpp"
#include "lbm_kernels.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(LBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr int kRing = (int)lbm::kRingSlots;
constexpr int kGraphSteps = 32;  // steps per captured graph (even: the buffers return to place)
using lbm::kMaxGrid;
using lbm::align256;
constexpr double kW[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};

double weight(int i) {
    const int q = lbm::kC[i][0] * lbm::kC[i][0] + lbm::kC[i][1] * lbm::kC[i][1] +
                  lbm::kC[i][2] * lbm::kC[i][2];
    return kW[q];
}

size_t elem_size(int storage) { return storage == LBM_F32 ? 4 : 2; }
// values per node in the chunks of a state: the 19 populations
constexpr int kSlots = 19;
// LBM_F16R: the state's reference array follows its chunks, one FP16 per
// node in node order, np + 4 entries (a kernel reads 8-byte windows of it
// that may start up to two entries before the last node)
int64_t ref_elems(int storage, int64_t np) { return storage == LBM_F16R ? np + 4 : 0; }
// bytes of one state, before alignment
size_t state_bytes(int storage, int64_t np) {
    return ((size_t)kSlots * np + (size_t)ref_elems(storage, np)) * elem_size(storage);
}

// Workspace layout (byte offsets, each 256-aligned).
struct Layout {
    size_t A, B, table, coords, ent, wrap, count, partials, ring, total;
};

Layout layout(int64_t np, int64_t nf, int storage, int index_kind, int nx, int ny, int nz) {
    Layout L{};
    size_t off = 0;
    const size_t state = align256(state_bytes(storage, np));
    L.A = off;
    off += state;
    L.B = off;
    off += state;
    if (index_kind == LBM_INDEX_TABLE) {
        L.table = off;
        off += align256((size_t)18 * np * 4);
    } else {
        const size_t words = (size_t)ny * nz * lbm::words_per_row(nx);
        L.coords = off;
        off += align256((size_t)std::max<int64_t>(nf, 1) * 4);
        L.ent = off;
        off += align256(words * 16);
        L.wrap = off;
        off += align256((size_t)nz * 2 * lbm::words_per_row(nx) * 16);
        L.count = off;
        off += align256((size_t)ny * nz * 16);
    }
    // the reduction scratch, kReductionBytes at the end (lbm_setup_static
    // contexts keep it in the static array instead)
    L.partials = off;  // two buffers: steps alternate between them
    off += 2 * lbm::kPartialBytes;
    L.ring = off;  // ring of per-step sums, then the device counter of steps reduced
    off += align256((size_t)kRing * 4 * 8 + sizeof(uint32_t));
    L.total = off;
    return L;
}
static_assert(LBM_REDUCTION_BYTES == lbm::kReductionBytes, "header and layout disagree on the reduction scratch");

std::string check_common(const uint8_t* geom, int nx, int ny, int nz, int storage,
                         int index_kind) {
    if (!geom) return "geometry is NULL";
    std::string e = lbm::check_dims(nx, ny, nz);
    if (!e.empty()) return e;
    if (storage < LBM_F32 || storage > LBM_F16R) return "storage must be LBM_F32, LBM_F16, LBM_BF16 or LBM_F16R";
    if (index_kind != LBM_INDEX_TABLE && index_kind != LBM_INDEX_BITMAP)
        return "index_kind must be LBM_INDEX_TABLE or LBM_INDEX_BITMAP";
    return "";
}

// The gathers of a chunk are 32-bit byte offsets from one base (gather_span).
std::string check_span(const lbm::GatherSpan& g, int storage) {
    const double bytes = (double)(g.slack + g.reach) * (double)elem_size(storage);
    if (bytes >= 4294967296.0 || g.slack >= ((int64_t)1 << 32))
        return "the image is too large for 32-bit gather offsets (" + std::to_string((int64_t)bytes) +
               " bytes around a chunk); use a smaller image or 16-bit storage";
    return "";
}

// FP16 / BF16 host encoders (round to nearest even).
uint16_t to_bf16(float v) {
    uint32_t u;
    std::memcpy(&u, &v, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
float from_bf16(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float v;
    std::memcpy(&v, &u, 4);
    return v;
}

}  // namespace

struct lbm_ctx {
    int nx, ny, nz;
    int64_t nf, np;
    double tau, Lambda;
    int set;
    double g[3];
    int axis;
    int storage, index_kind;
    int collision;
    int wall_mode;      // LBM_WALL_HALFWAY or LBM_WALL_FULLWAY
    float* wallbuf;     // full-way delay line (caller's workspace), state layout
    bool pressure;      // Zou-He pressure faces on x = 0 and x = nx - 1
    double rho_in, rho_out;
    int cus;
    lbm::RateClasses rates, ds_dtau, ds_dLambda;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    Layout L;
    lbm::GatherSpan span;
    void* cur;   // state after the last step
    void* nxt;
    lbm::IndexView idx;
    int grid;
    double* partials[2];
    double* ring;
    uint32_t* ctr;      // steps reduced into the ring so far (device, after the ring)
    int64_t steps;
    bool pending;  // the last step's partials are not yet reduced into the ring
    const float* field;
    int exponent;
    std::vector<uint8_t> geom;
    // captured kGraphSteps-step sequences, by (cur buffer, step parity); any
    // change of what a step launch bakes in drops them
    bool graphs;
    hipStream_t cap_stream;
    hipGraphExec_t gexec[4];
    int static_dev;  // device whose static reduction scratch this context holds, or -1
    double adj_ms[3];  // last lbm_adjoint: forward, recompute and reverse milliseconds
    bool adj_timed;
    ~lbm_ctx();
};

namespace {

lbm::RatesF rates_f(const lbm::RateClasses& r) {
    return lbm::RatesF{(float)r.s_e, (float)r.s_eps, (float)r.s_q,
                       (float)r.s_nu, (float)r.s_pi, (float)r.s_m};
}

float scale_of(const lbm_ctx* c) { return std::ldexp(1.0f, c->exponent); }

// One forward step from `src` to `dst` with partial sums into `partials`;
// when prev_partials is non-null the same launch reduces them into the next
// ring slot (the device counter's).
hipError_t step_raw(lbm_ctx* c, const void* src, void* dst, double* partials,
                    const double* prev_partials = nullptr, hipStream_t stream = nullptr) {
    lbm::StepLaunch a{};
    a.storage = c->storage;
    a.collision = c->collision;
    a.wall = c->wall_mode == LBM_WALL_FULLWAY ? c->wallbuf : nullptr;
    a.pressure = c->pressure;
    a.drho_in = (float)(c->rho_in - 1.0);
    a.drho_out = (float)(c->rho_out - 1.0);
    a.src = src;
    a.dst = dst;
    a.idx = c->idx;
    a.nf = c->nf;
    a.rates = rates_f(c->rates);
    a.F[0] = (float)c->g[0];
    a.F[1] = (float)c->g[1];
    a.F[2] = (float)c->g[2];
    a.field = c->field;
    a.scale = scale_of(c);
    a.inv_scale = 1.0f / a.scale;
    a.grid = c->grid;
    a.partials = partials;
    a.prev_partials = prev_partials;
    a.ring = c->ring;
    a.ctr = c->ctr;
    return lbm::launch_step(a, stream ? stream : c->stream);
}

void drop_graphs(lbm_ctx* c) {
    for (auto& g : c->gexec)
        if (g) {
            hipGraphExecDestroy(g);
            g = nullptr;
        }
}

hipError_t zero_ring(lbm_ctx* c) {
    return lbm::launch_zero(c->ring, (int64_t)kRing * 4 * 8 + (int64_t)sizeof(uint32_t), c->stream);
}

// The graph of kGraphSteps steps from the current buffers and step parity,
// with the previous step's partials pending (captured on first use).
hipGraphExec_t graph_for(lbm_ctx* c) {
    const int key = (c->cur == c->ws + c->L.A ? 0 : 2) + (int)(c->steps & 1);
    if (c->gexec[key]) return c->gexec[key];
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        return nullptr;
    }
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    void* cur = c->cur;
    void* nxt = c->nxt;
    hipError_t he = hipSuccess;
    for (int k = 0; k < kGraphSteps && he == hipSuccess; ++k) {
        const int64_t t = c->steps + k;
        he = step_raw(c, cur, nxt, c->partials[t & 1], c->partials[(t - 1) & 1], c->cap_stream);
        std::swap(cur, nxt);
    }
    hipGraph_t graph = nullptr;
    const hipError_t he2 = hipStreamEndCapture(c->cap_stream, &graph);
    if (he != hipSuccess || he2 != hipSuccess || !graph) {
        if (graph) hipGraphDestroy(graph);
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (he != hipSuccess) return nullptr;
    c->gexec[key] = exec;
    return exec;
}

// One resident wave of blocks: every block starts at once and walks the
// chunk list with stride `grid` (a multiple of the XCD count when >= 64),
// so the chunks in flight form a window of `grid` consecutive chunks.  With
// FP32 storage one block per compute unit: that step is bound by the L2
// misses of its gathers, not by latency, and the narrowest window serves
// them best (512^3 rock: 0.833 ms with 5 blocks per unit, 0.827 with 2,
// 0.769 with 1).  The 16-bit storages, bound by the loads they can keep in
// flight, take every block that fits (1 per unit: FP16 0.575 -> 0.670 ms).
hipError_t choose_grid(lbm_ctx* c) {
    int per_cu = 0;
    hipError_t he = lbm::step_occupancy(c->storage, c->index_kind, c->collision, &per_cu);
    if (he != hipSuccess) return he;
    if (c->storage == LBM_F32) per_cu = 1;
    const int64_t chunks = (c->nf + 255) / 256;
    int64_t G = std::min<int64_t>(chunks, (int64_t)std::max(c->cus, 1) * std::max(per_cu, 1));
    if (G >= 64) G -= G % 8;
    c->grid = (int)std::min<int64_t>(G, kMaxGrid);
    return hipSuccess;
}

// The rates form a two-relaxation-time set: one rate on every even
// non-conserved moment (e, eps, p, pi) and one on every odd one (q, m).
bool two_rate(const lbm::RateClasses& r) {
    return r.s_e == r.s_nu && r.s_eps == r.s_nu && r.s_pi == r.s_nu && r.s_m == r.s_q;
}

// Step n (0-based) writes partials[n % 2]; its launch also reduces the
// partials of step n-1 into the ring.  With a step pending, runs of
// kGraphSteps steps replay a captured graph (one launch call instead of
// kGraphSteps; the launches and their arguments are the same).
int do_steps(lbm_ctx* c, int n) {
    int k = 0;
    while (k < n) {
        if (c->graphs && c->pending && n - k >= kGraphSteps) {
            hipGraphExec_t g = graph_for(c);
            if (g) {
                HIP_TRY(hipGraphLaunch(g, c->stream));
                c->steps += kGraphSteps;  // even: cur and nxt are back in place
                k += kGraphSteps;
                continue;
            }
            c->graphs = false;  // capture not available: plain launches from here on
        }
        const int64_t t = c->steps;
        const double* prev = c->pending ? c->partials[(t - 1) & 1] : nullptr;
        HIP_TRY(step_raw(c, c->cur, c->nxt, c->partials[t & 1], prev));
        std::swap(c->cur, c->nxt);
        ++c->steps;
        c->pending = true;
        ++k;
    }
    return LBM_OK;
}

// Reduce the last step's partials if that has not happened yet.
int flush(lbm_ctx* c) {
    if (!c->pending) return LBM_OK;
    HIP_TRY(lbm::launch_finalize(c->partials[(c->steps - 1) & 1], c->grid, c->ring, c->ctr, c->stream));
    c->pending = false;
    return LBM_OK;
}

int read_slot(lbm_ctx* c, int64_t step_index, double out[4]) {
    int rc = flush(c);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(out, c->ring + (step_index % kRing) * 4, 4 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

double volume(const lbm_ctx* c) { return (double)c->nx * c->ny * c->nz; }
double viscosity(const lbm_ctx* c) { return (c->tau - 0.5) / 3.0; }

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_velocities(int c[19][3]) {
    if (!c) return fail(LBM_EINVAL, "c is NULL");
    for (int i = 0; i < 19; ++i)
        for (int a = 0; a < 3; ++a) c[i][a] = lbm::kC[i][a];
    return LBM_OK;
}

int lbm_rates(int set, double tau, double Lambda, double s[19], double ds_dtau[19],
              double ds_dLambda[19]) {
    lbm::RateClasses r{}, dt{}, dl{};
    std::string e = lbm::rates(set, tau, Lambda, &r, &dt, &dl);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    if (s) lbm::rates_to_moments(r, s);
    if (ds_dtau) lbm::rates_to_moments(dt, ds_dtau);
    if (ds_dLambda) lbm::rates_to_moments(dl, ds_dLambda);
    return LBM_OK;
}

int lbm_workspace_query(const uint8_t* geometry, int nx, int ny, int nz, int storage,
                        int index_kind, size_t* bytes, int64_t* n_fluid) {
    std::string e = check_common(geometry, nx, ny, nz, storage, index_kind);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    const int64_t nf = lbm::count_fluid(geometry, nx, ny, nz);
    if (n_fluid) *n_fluid = nf;
    if (nf == 0) return fail(LBM_ENOFLUID, "the image has no fluid voxel");
    if (nf >= ((int64_t)1 << 31) - 256) return fail(LBM_ERANGE, "more than 2^31 fluid nodes");
    if (index_kind == LBM_INDEX_BITMAP && !lbm::coord_bits(nx, ny, nz).fits())
        return fail(LBM_ERANGE, "packed voxel coordinates need more than 32 bits");
    if (index_kind == LBM_INDEX_BITMAP && nx > lbm::kBitmapMaxNx)
        return fail(LBM_ERANGE, "the bitmap index holds rows of at most 4095 voxels");
    if (index_kind == LBM_INDEX_BITMAP && (int64_t)ny * nz * lbm::words_per_row(nx) >= ((int64_t)1 << 32))
        return fail(LBM_ERANGE, "the bitmap index holds fewer than 2^32 row words");
    {
        const lbm::NodeOrder o = lbm::node_order(geometry, nx, ny, nz);
        e = check_span(lbm::gather_span(o.start, ny, nz, o.tile_z, kSlots), storage);
    }
    if (!e.empty()) return fail(LBM_ERANGE, e);
    if (bytes) *bytes = layout(lbm::padded(nf), nf, storage, index_kind, nx, ny, nz).total;
    return LBM_OK;
}

int lbm_neighbor_table(const uint8_t* geometry, int nx, int ny, int nz, int32_t* table,
                       int64_t n_fluid) {
    std::string e = check_common(geometry, nx, ny, nz, LBM_F32, LBM_INDEX_TABLE);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    if (!table) return fail(LBM_EINVAL, "table is NULL");
    const int64_t nf = lbm::count_fluid(geometry, nx, ny, nz);
    if (nf != n_fluid) return fail(LBM_EINVAL, "n_fluid does not match the image");
    if (nf == 0) return fail(LBM_ENOFLUID, "the image has no fluid voxel");
    lbm::build_table(geometry, nx, ny, nz, nf, nf, table);
    return LBM_OK;
}

int lbm_neighbor_nodes(const uint8_t* geometry, int nx, int ny, int nz, const int64_t* nodes, int64_t count,
                       int32_t* table) {
    std::string e = check_common(geometry, nx, ny, nz, LBM_F32, LBM_INDEX_TABLE);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    if (count < 0 || (count > 0 && (!nodes || !table))) return fail(LBM_EINVAL, "NULL argument or count < 0");
    const int64_t nf = lbm::count_fluid(geometry, nx, ny, nz);
    for (int64_t k = 0; k < count; ++k)
        if (nodes[k] < 0 || nodes[k] >= nf) return fail(LBM_EINVAL, "node number out of range");
    lbm::neighbor_nodes(geometry, nx, ny, nz, nodes, count, table);
    return LBM_OK;
}

int lbm_node_order(const uint8_t* geometry, int nx, int ny, int nz, int64_t* voxel,
                   int64_t n_fluid) {
    std::string e = check_common(geometry, nx, ny, nz, LBM_F32, LBM_INDEX_TABLE);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    if (!voxel) return fail(LBM_EINVAL, "voxel is NULL");
    const int64_t nf = lbm::count_fluid(geometry, nx, ny, nz);
    if (nf != n_fluid) return fail(LBM_EINVAL, "n_fluid does not match the image");
    lbm::fluid_voxels(geometry, nx, ny, nz, voxel);
    return LBM_OK;
}

int lbm_boundary_dims(int nx, int ny, int nz, int pad, int mirror_y, int mirror_z, int* onx, int* ony,
                      int* onz) {
    std::string e = lbm::check_dims(nx, ny, nz);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    if (pad < 0 || pad > (1 << 20)) return fail(LBM_EINVAL, "pad must be in [0, 2^20]");
    if (!onx || !ony || !onz) return fail(LBM_EINVAL, "NULL argument");
    const int64_t ox = (int64_t)nx + 2 * (int64_t)pad, oy = mirror_y ? 2 * (int64_t)ny : ny,
                  oz = mirror_z ? 2 * (int64_t)nz : nz;
    if (ox > INT32_MAX || oy > INT32_MAX || oz > INT32_MAX) return fail(LBM_ERANGE, "extents overflow int");
    e = lbm::check_dims((int)ox, (int)oy, (int)oz);
    if (!e.empty()) return fail(LBM_ERANGE, e);
    *onx = (int)ox;
    *ony = (int)oy;
    *onz = (int)oz;
    return LBM_OK;
}

int lbm_boundary_image(const uint8_t* geometry, int nx, int ny, int nz, int pad, int mirror_y, int mirror_z,
                       uint8_t* out) {
    if (!geometry || !out) return fail(LBM_EINVAL, "NULL argument");
    int ox, oy, oz;
    int rc = lbm_boundary_dims(nx, ny, nz, pad, mirror_y, mirror_z, &ox, &oy, &oz);
    if (rc) return rc;
    lbm::boundary_image(geometry, nx, ny, nz, pad, mirror_y != 0, mirror_z != 0, out);
    return LBM_OK;
}

}  // extern "C"

namespace {

// Contexts holding a GPU's static reduction scratch (lbm_setup_static), by device.
constexpr int kStaticDevices = 64;
std::mutex g_static_mu;
const lbm_ctx* g_static_owner[kStaticDevices] = {};

}  // namespace

lbm_ctx::~lbm_ctx() {
    for (auto& g : gexec)
        if (g) hipGraphExecDestroy(g);
    if (cap_stream) hipStreamDestroy(cap_stream);
    if (static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_owner[static_dev] == this) g_static_owner[static_dev] = nullptr;
    }
}

namespace {

// lbm_setup and lbm_setup_static: with use_static the reduction scratch is
// the current GPU's static array instead of the workspace's last
// LBM_REDUCTION_BYTES.
int setup_impl(lbm_ctx** ctx, const uint8_t* geometry, int nx, int ny, int nz, double tau, double Lambda,
               int relaxation_set, const double g[3], int storage, int index_kind, void* workspace,
               size_t workspace_bytes, void* hip_stream, bool use_static) {
    if (!ctx) return fail(LBM_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    std::string e = check_common(geometry, nx, ny, nz, storage, index_kind);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    if (!g) return fail(LBM_EINVAL, "g is NULL");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(g[a])) return fail(LBM_EINVAL, "g must be finite");
    lbm::RateClasses r{}, dt{}, dl{};
    e = lbm::rates(relaxation_set, tau, Lambda, &r, &dt, &dl);
    if (!e.empty()) return fail(LBM_EINVAL, e);
    size_t need = 0;
    int64_t nf = 0;
    int rc = lbm_workspace_query(geometry, nx, ny, nz, storage, index_kind, &need, &nf);
    if (rc != LBM_OK) return rc;
    if (!workspace) return fail(LBM_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(LBM_EWORKSPACE, "workspace must be 256-byte aligned");
    if (use_static) need -= LBM_REDUCTION_BYTES;  // the reduction scratch is the tail of the layout
    if (workspace_bytes < need)
        return fail(LBM_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");

    // ---- everything below may call HIP
    void* red = nullptr;  // the static reduction scratch, when used
    int dev = 0;
    if (use_static) {
        hipError_t he = hipGetDevice(&dev);
        if (he != hipSuccess) return fail(LBM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
        if (dev < 0 || dev >= kStaticDevices) return fail(LBM_ERANGE, "device ordinal beyond the static scratch table");
        he = lbm::static_scratch(&red);
        if (he != hipSuccess)
            return fail(LBM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(he));
    }
    auto* c = new lbm_ctx();
    c->static_dev = -1;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->nf = nf;
    c->np = lbm::padded(nf);
    c->tau = tau;
    c->Lambda = Lambda;
    c->set = relaxation_set;
    for (int a = 0; a < 3; ++a) c->g[a] = g[a];
    c->axis = 0;
    for (int a = 1; a < 3; ++a)
        if (std::fabs(g[a]) > std::fabs(g[c->axis])) c->axis = a;
    c->storage = storage;
    c->index_kind = index_kind;
    c->rates = r;
    c->ds_dtau = dt;
    c->ds_dLambda = dl;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char*>(workspace);
    c->ws_bytes = workspace_bytes;
    c->L = layout(c->np, nf, storage, index_kind, nx, ny, nz);
    c->cur = c->ws + c->L.A;
    c->nxt = c->ws + c->L.B;
    char* rbase = use_static ? static_cast<char*>(red) : c->ws + c->L.partials;  // partials, then the ring
    c->partials[0] = reinterpret_cast<double*>(rbase);
    c->partials[1] = c->partials[0] + lbm::kPartialBytes / 8;
    c->pending = false;
    c->ring = reinterpret_cast<double*>(rbase + (c->L.ring - c->L.partials));
    c->ctr = reinterpret_cast<uint32_t*>(c->ring + (size_t)kRing * 4);
    c->graphs = true;
    c->cap_stream = nullptr;
    for (auto& g : c->gexec) g = nullptr;
    c->steps = 0;
    c->field = nullptr;
    c->geom.assign(geometry, geometry + (size_t)nx * ny * nz);
    {
        const lbm::NodeOrder o = lbm::node_order(geometry, nx, ny, nz);
        c->span = lbm::gather_span(o.start, ny, nz, o.tile_z, kSlots);
    }
    double gmax = std::max({std::fabs(g[0]), std::fabs(g[1]), std::fabs(g[2])});
    // FP16 scale: plain deviations hold the density deviation, which grows to
    // ~1e2-1e3 g in rock; the referenced ones hold velocity-sized values only
    c->exponent = 0;
    if (storage == LBM_F16 && gmax > 0) c->exponent = (int)std::lround(-std::log2(gmax)) - 4;
    if (storage == LBM_F16R && gmax > 0) c->exponent = (int)std::lround(-std::log2(gmax)) + 2;
    if (c->exponent < 0) c->exponent = 0;

    c->collision = LBM_COLLIDE_MRT;
    c->wall_mode = LBM_WALL_HALFWAY;
    c->wallbuf = nullptr;
    c->pressure = false;
    c->rho_in = c->rho_out = 1.0;
    c->cus = 0;
    auto cleanup = [&](int code) {
        delete c;
        return code;
    };
    if (use_static) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_owner[dev])
            return cleanup(fail(LBM_EBUSY, "the static reduction scratch of device " + std::to_string(dev) +
                                               " is held by another live context (lbm_destroy it first)"));
        g_static_owner[dev] = c;
        c->static_dev = dev;
    }
    hipError_t he = hipGetDevice(&dev);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (he != hipSuccess) return cleanup(fail(LBM_EHIP, std::string("device query: ") + hipGetErrorString(he)));
    he = choose_grid(c);
    if (he != hipSuccess) return cleanup(fail(LBM_EHIP, std::string("occupancy query: ") + hipGetErrorString(he)));

    lbm::IndexView& v = c->idx;
    v.kind = index_kind;
    v.stride = c->np;
    v.slack = c->span.slack;
    std::vector<int32_t> table;
    lbm::BitmapIndex bm;
    if (index_kind == LBM_INDEX_TABLE) {
        table.assign((size_t)18 * c->np, -1);
        lbm::build_table(geometry, nx, ny, nz, nf, c->np, table.data());
        v.table = reinterpret_cast<const int32_t*>(c->ws + c->L.table);
        he = hipMemcpyAsync(c->ws + c->L.table, table.data(), table.size() * 4,
                            hipMemcpyHostToDevice, c->stream);
    } else {
        lbm::build_bitmap(geometry, nx, ny, nz, nf, &bm);
        if (!bm.fits)
            return cleanup(fail(LBM_ERANGE, "the bitmap index's row-base differences exceed 18 bits"));
        v.coords = reinterpret_cast<const uint32_t*>(c->ws + c->L.coords);
        v.ent = c->ws + c->L.ent;
        v.wrap = c->ws + c->L.wrap;
        v.count = c->ws + c->L.count;
        v.nx = nx;
        v.ny = ny;
        v.nz = nz;
        v.R = bm.words;
        v.bx = bm.bits.bx;
        v.by = bm.bits.by;
        he = hipMemcpyAsync(c->ws + c->L.coords, bm.coords.data(), bm.coords.size() * 4,
                            hipMemcpyHostToDevice, c->stream);
        if (he == hipSuccess)
            he = hipMemcpyAsync(c->ws + c->L.ent, bm.ent.data(), bm.ent.size() * 4, hipMemcpyHostToDevice,
                                c->stream);
        if (he == hipSuccess)
            he = hipMemcpyAsync(c->ws + c->L.wrap, bm.wrap.data(), bm.wrap.size() * 4, hipMemcpyHostToDevice,
                                c->stream);
        if (he == hipSuccess)
            he = hipMemcpyAsync(c->ws + c->L.count, bm.count.data(), bm.count.size() * 4, hipMemcpyHostToDevice,
                                c->stream);
    }
    if (he == hipSuccess) he = lbm::launch_zero(c->ws + c->L.A, (int64_t)(c->L.B - c->L.A) * 2, c->stream);
    if (he == hipSuccess) he = zero_ring(c);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return cleanup(fail(LBM_EHIP, std::string("setup upload: ") + hipGetErrorString(he)));
    *ctx = c;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_setup(lbm_ctx** ctx, const uint8_t* geometry, int nx, int ny, int nz, double tau,
              double Lambda, int relaxation_set, const double g[3], int storage, int index_kind,
              void* workspace, size_t workspace_bytes, void* hip_stream) {
    return setup_impl(ctx, geometry, nx, ny, nz, tau, Lambda, relaxation_set, g, storage, index_kind, workspace,
                      workspace_bytes, hip_stream, false);
}

int lbm_setup_static(lbm_ctx** ctx, const uint8_t* geometry, int nx, int ny, int nz, double tau,
                     double Lambda, int relaxation_set, const double g[3], int storage, int index_kind,
                     void* workspace, size_t workspace_bytes, void* hip_stream) {
    return setup_impl(ctx, geometry, nx, ny, nz, tau, Lambda, relaxation_set, g, storage, index_kind, workspace,
                      workspace_bytes, hip_stream, true);
}

int lbm_step(lbm_ctx* c, int n) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    return do_steps(c, n);
}

int64_t lbm_steps_done(const lbm_ctx* c) { return c ? c->steps : -1; }
int64_t lbm_n_fluid(const lbm_ctx* c) { return c ? c->nf : -1; }

int lbm_mean_velocity(lbm_ctx* c, double u[3]) {
    if (!c || !u) return fail(LBM_EINVAL, "NULL argument");
    if (c->steps == 0) {
        u[0] = u[1] = u[2] = 0.0;
        return LBM_OK;
    }
    double s[4];
    int rc = read_slot(c, c->steps - 1, s);
    if (rc) return rc;
    for (int a = 0; a < 3; ++a) u[a] = s[a] / volume(c);
    if (!std::isfinite(u[0]) || !std::isfinite(u[1]) || !std::isfinite(u[2]) || !std::isfinite(s[3]))
        return fail(LBM_ENAN, "mean velocity or mass is not finite");
    return LBM_OK;
}

int lbm_permeability(lbm_ctx* c, double k[3]) {
    if (!c || !k) return fail(LBM_EINVAL, "NULL argument");
    double u[3];
    int rc = lbm_mean_velocity(c, u);
    if (rc) return rc;
    if (c->pressure) {
        // Eq. perm_calc: grad p = c_s^2 (rho_in - rho_out) / (nx - 1) between the faces
        const double gp = (c->rho_in - c->rho_out) / 3.0 / (c->nx - 1);
        k[0] = viscosity(c) * u[0] / gp;
        k[1] = k[2] = NAN;
        return LBM_OK;
    }
    for (int a = 0; a < 3; ++a) k[a] = c->g[a] != 0 ? viscosity(c) * u[a] / c->g[a] : NAN;
    return LBM_OK;
}

int lbm_mass(lbm_ctx* c, double* m) {
    if (!c || !m) return fail(LBM_EINVAL, "NULL argument");
    double dm = 0.0;
    const int rc = lbm_mass_deviation(c, &dm);
    if (rc) return rc;
    *m = (double)c->nf + dm;  // rho0 = 1
    return LBM_OK;
}

int lbm_mass_deviation(lbm_ctx* c, double* dm) {
    if (!c || !dm) return fail(LBM_EINVAL, "NULL argument");
    if (c->steps == 0) {
        *dm = 0.0;
        return LBM_OK;
    }
    double s[4];
    int rc = read_slot(c, c->steps - 1, s);
    if (rc) return rc;
    *dm = s[3];
    if (!std::isfinite(*dm)) return fail(LBM_ENAN, "mass is not finite");
    return LBM_OK;
}

int lbm_history(lbm_ctx* c, int count, double* u) {
    if (!c || !u) return fail(LBM_EINVAL, "NULL argument");
    if (count < 0 || count > kRing || count > c->steps)
        return fail(LBM_EINVAL, "count must be in [0, min(1024, steps done)]");
    std::vector<double> ring((size_t)kRing * 4);
    int rc = flush(c);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(ring.data(), c->ring, ring.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int t = 0; t < count; ++t) {
        const int64_t step = c->steps - count + t;
        for (int a = 0; a < 3; ++a) u[3 * t + a] = ring[(step % kRing) * 4 + a] / volume(c);
    }
    return LBM_OK;
}

int lbm_run_to_steady(lbm_ctx* c, double eps, int check_every, int max_steps, int* steps,
                      double k[3], int* converged) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!(eps > 0) || check_every < 1 || check_every > kRing - 1 || max_steps < 0)
        return fail(LBM_EINVAL, "need eps > 0, 1 <= check_every < 1024, max_steps >= 0");
    if (c->g[c->axis] == 0 && !c->pressure) return fail(LBM_EINVAL, "no body force and no pressure drop");
    int done = 0, conv = 0;
    std::vector<double> h;
    while (done < max_steps && !conv) {
        const int n = std::min(check_every, max_steps - done);
        int rc = do_steps(c, n);
        if (rc) return rc;
        done += n;
        const int m = (int)std::min<int64_t>(c->steps, n + 1);
        h.assign((size_t)3 * m, 0.0);
        rc = lbm_history(c, m, h.data());
        if (rc) return rc;
        for (int t = 1; t < m; ++t) {
            const double a = h[3 * (t - 1) + c->axis], b = h[3 * t + c->axis];
            if (!std::isfinite(b)) return fail(LBM_ENAN, "mean velocity is not finite");
            if (c->steps - (m - 1 - t) >= 2 && std::fabs(b - a) < eps * std::fabs(b)) conv = 1;
        }
    }
    if (steps) *steps = done;
    if (converged) *converged = conv;
    if (k) {
        int rc = lbm_permeability(c, k);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_get_state(lbm_ctx* c, double* f) {
    if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
    const int S = kSlots;
    std::vector<char> raw(state_bytes(c->storage, c->np));
    HIP_TRY(hipMemcpyAsync(raw.data(), c->cur, raw.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const double inv = 1.0 / std::ldexp(1.0, c->exponent);
    const _Float16* h16 = reinterpret_cast<const _Float16*>(raw.data());
    const _Float16* ref = h16 + (size_t)S * c->np;  // LBM_F16R: the reference array
    for (int i = 0; i < 19; ++i) {
        const double w = weight(i);
        for (int64_t n = 0; n < c->nf; ++n) {
            const size_t at = (size_t)lbm::state_elem(i, n, S);
            double d;
            if (c->storage == LBM_F32)
                d = reinterpret_cast<const float*>(raw.data())[at];
            else if (c->storage == LBM_F16)
                d = (double)(float)h16[at] * inv;
            else if (c->storage == LBM_F16R)
                d = (double)((float)h16[at] * (float)inv + (float)w * (float)ref[n]);
            else
                d = (double)from_bf16(reinterpret_cast<const uint16_t*>(raw.data())[at]);
            f[(size_t)i * c->nf + n] = w + d;
        }
    }
    return LBM_OK;
}

int lbm_get_state_nodes(lbm_ctx* c, const int64_t* nodes, int64_t count, double* f) {
    if (!c || (count > 0 && (!nodes || !f)) || count < 0) return fail(LBM_EINVAL, "NULL argument or count < 0");
    for (int64_t k = 0; k < count; ++k)
        if (nodes[k] < 0 || nodes[k] >= c->nf) return fail(LBM_EINVAL, "node number out of range");
    const size_t es = elem_size(c->storage);
    const int S = kSlots;
    const size_t chunk_bytes = (size_t)S * lbm::kChunk * es;
    std::vector<char> buf(chunk_bytes);
    std::vector<_Float16> rbuf(lbm::kChunk);  // LBM_F16R: the chunk's references
    const double inv = 1.0 / std::ldexp(1.0, c->exponent);
    int64_t loaded = -1;
    for (int64_t k = 0; k < count; ++k) {
        const int64_t n = nodes[k], q = n / lbm::kChunk;
        if (q != loaded) {  // the node's chunk holds its populations
            HIP_TRY(hipMemcpyAsync(buf.data(), static_cast<char*>(c->cur) + (size_t)q * chunk_bytes, chunk_bytes,
                                   hipMemcpyDeviceToHost, c->stream));
            if (c->storage == LBM_F16R)
                HIP_TRY(hipMemcpyAsync(rbuf.data(),
                                       static_cast<char*>(c->cur) + ((size_t)S * c->np + (size_t)q * lbm::kChunk) * es,
                                       lbm::kChunk * es, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            loaded = q;
        }
        const int64_t m = n % lbm::kChunk;
        const _Float16* h16 = reinterpret_cast<const _Float16*>(buf.data());
        for (int i = 0; i < 19; ++i) {
            const size_t at = (size_t)lbm::state_elem(i, m, S);
            double d;
            if (c->storage == LBM_F32)
                d = reinterpret_cast<const float*>(buf.data())[at];
            else if (c->storage == LBM_F16)
                d = (double)(float)h16[at] * inv;
            else if (c->storage == LBM_F16R)
                d = (double)((float)h16[at] * (float)inv + (float)weight(i) * (float)rbuf[m]);
            else
                d = (double)from_bf16(reinterpret_cast<const uint16_t*>(buf.data())[at]);
            f[(size_t)i * count + k] = weight(i) + d;
        }
    }
    return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, const double* f) {
    if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
    const int S = kSlots;
    std::vector<char> raw(state_bytes(c->storage, c->np), 0);
    const double sc = std::ldexp(1.0, c->exponent);
    _Float16* h16 = reinterpret_cast<_Float16*>(raw.data());
    std::vector<float> ref;
    if (c->storage == LBM_F16R) {  // each node's reference: its density deviation in FP16
        ref.resize(c->nf);
        for (int64_t n = 0; n < c->nf; ++n) {
            double d = -1.0;
            for (int i = 0; i < 19; ++i) d += f[(size_t)i * c->nf + n];
            const _Float16 r = (_Float16)(float)d;
            h16[(size_t)S * c->np + n] = r;
            ref[n] = (float)r;
        }
    }
    for (int i = 0; i < 19; ++i) {
        const double w = weight(i);
        for (int64_t n = 0; n < c->nf; ++n) {
            const size_t at = (size_t)lbm::state_elem(i, n, S);
            const double d = f[(size_t)i * c->nf + n] - w;
            if (c->storage == LBM_F32)
                reinterpret_cast<float*>(raw.data())[at] = (float)d;
            else if (c->storage == LBM_F16)
                h16[at] = (_Float16)(float)(d * sc);
            else if (c->storage == LBM_F16R)
                h16[at] = (_Float16)(float)((d - w * (double)ref[n]) * sc);
            else
                reinterpret_cast<uint16_t*>(raw.data())[at] = to_bf16((float)d);
        }
    }
    HIP_TRY(hipMemcpyAsync(c->cur, raw.data(), raw.size(), hipMemcpyHostToDevice, c->stream));
    if (c->wall_mode == LBM_WALL_FULLWAY)  // the state one step older starts equal to it
        HIP_TRY(hipMemcpyAsync(c->wallbuf, c->cur, raw.size(), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(zero_ring(c));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->steps = 0;
    c->pending = false;
    return LBM_OK;
}

int lbm_fluid_index(lbm_ctx* c, int64_t* voxel) {
    if (!c || !voxel) return fail(LBM_EINVAL, "NULL argument");
    lbm::fluid_voxels(c->geom.data(), c->nx, c->ny, c->nz, voxel);
    return LBM_OK;
}

int lbm_set_force_field(lbm_ctx* c, const float* g_device) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->pressure && g_device) return fail(LBM_EINVAL, "a force field cannot be combined with pressure faces");
    c->field = g_device;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_set_collision(lbm_ctx* c, int collision) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (collision != LBM_COLLIDE_MRT && collision != LBM_COLLIDE_TRT)
        return fail(LBM_EINVAL, "collision must be LBM_COLLIDE_MRT or LBM_COLLIDE_TRT");
    if (collision == LBM_COLLIDE_TRT && !two_rate(c->rates))
        return fail(LBM_EINVAL, "the link-wise TRT collision needs a two-rate set (SRT, Set B or Set E)");
    if (c->pending) {
        int rc = flush(c);  // the pending partials were written with the current grid
        if (rc) return rc;
    }
    const int old = c->collision, old_grid = c->grid;
    c->collision = collision;
    drop_graphs(c);
    hipError_t he = choose_grid(c);
    if (he != hipSuccess) {
        c->collision = old;
        c->grid = old_grid;
        return fail(LBM_EHIP, std::string("occupancy query: ") + hipGetErrorString(he));
    }
    return LBM_OK;
}

int lbm_wall_workspace_query(lbm_ctx* c, size_t* bytes) {
    if (!c || !bytes) return fail(LBM_EINVAL, "NULL argument");
    *bytes = align256((size_t)19 * c->np * 4);
    return LBM_OK;
}

int lbm_set_wall(lbm_ctx* c, int mode, void* workspace, size_t workspace_bytes) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (mode == LBM_WALL_HALFWAY) {
        c->wall_mode = mode;
        c->wallbuf = nullptr;
        drop_graphs(c);
        return LBM_OK;
    }
    if (mode != LBM_WALL_FULLWAY) return fail(LBM_EINVAL, "mode must be LBM_WALL_HALFWAY or LBM_WALL_FULLWAY");
    if (c->storage != LBM_F32) return fail(LBM_EINVAL, "full-way bounce-back needs FP32 storage");
    if (c->pressure) return fail(LBM_EINVAL, "full-way bounce-back cannot be combined with pressure faces");
    const size_t need = align256((size_t)19 * c->np * 4);
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(LBM_EWORKSPACE, "wall workspace NULL or not 256-byte aligned");
    if (workspace_bytes < need) return fail(LBM_EWORKSPACE, "wall workspace too small: need " + std::to_string(need));
    c->wallbuf = static_cast<float*>(workspace);
    // the state one step older than the current one starts equal to it
    HIP_TRY(hipMemcpyAsync(c->wallbuf, c->cur, (size_t)19 * c->np * 4, hipMemcpyDeviceToDevice, c->stream));
    c->wall_mode = mode;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_set_pressure(lbm_ctx* c, int enable, double rho_in, double rho_out) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!enable) {
        c->pressure = false;
        drop_graphs(c);
        return LBM_OK;
    }
    if (!std::isfinite(rho_in) || !std::isfinite(rho_out) || !(rho_in > 0) || !(rho_out > 0) || rho_in == rho_out)
        return fail(LBM_EINVAL, "need finite, positive and different rho_in, rho_out");
    if (c->storage != LBM_F32 || c->index_kind != LBM_INDEX_BITMAP)
        return fail(LBM_EINVAL, "pressure faces need FP32 storage and the bitmap index");
    if (c->g[0] != 0 || c->g[1] != 0 || c->g[2] != 0 || c->field)
        return fail(LBM_EINVAL, "pressure faces need a context without body force");
    if (c->wall_mode != LBM_WALL_HALFWAY) return fail(LBM_EINVAL, "pressure faces need halfway bounce-back");
    if (c->idx.sym) return fail(LBM_EINVAL, "pressure faces cannot be combined with symmetry planes");
    if (c->nx < 3) return fail(LBM_EINVAL, "pressure faces need nx >= 3");
    c->pressure = true;
    drop_graphs(c);
    c->rho_in = rho_in;
    c->rho_out = rho_out;
    c->axis = 0;
    return LBM_OK;
}

int lbm_set_symmetry(lbm_ctx* c, int mirror_y, int mirror_z) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    const int sym = (mirror_y ? 1 : 0) | (mirror_z ? 2 : 0);
    if (sym && c->index_kind != LBM_INDEX_BITMAP) return fail(LBM_EINVAL, "symmetry planes need the bitmap index");
    if (sym && c->storage != LBM_F32) return fail(LBM_EINVAL, "symmetry planes need FP32 storage");
    if (sym && c->pressure) return fail(LBM_EINVAL, "symmetry planes cannot be combined with pressure faces");
    if (sym == c->idx.sym) return LBM_OK;
    // the entries hold ghost rows beyond mirrored y faces, the counts and wrap
    // bases the ghost rows and planes (the kernel picks the entries' z ghost
    // planes itself)
    lbm::BitmapIndex bm;
    lbm::build_bitmap(c->geom.data(), c->nx, c->ny, c->nz, c->nf, &bm, (sym & 1) != 0, (sym & 2) != 0);
    if (!bm.fits) return fail(LBM_ERANGE, "the bitmap index's row-base differences exceed 18 bits");
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.ent, bm.ent.data(), bm.ent.size() * 4, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.wrap, bm.wrap.data(), bm.wrap.size() * 4, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.count, bm.count.data(), bm.count.size() * 4, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->idx.sym = sym;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_set_graphs(lbm_ctx* c, int enable) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    c->graphs = enable != 0;
    if (!c->graphs) drop_graphs(c);
    return LBM_OK;
}

int lbm_set_storage_exponent(lbm_ctx* c, int e) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->storage != LBM_F16 && c->storage != LBM_F16R) return LBM_OK;
    if (e < -60 || e > 60) return fail(LBM_EINVAL, "exponent out of range [-60, 60]");
    const float factor = std::ldexp(1.0f, e - c->exponent);
    // the populations only; LBM_F16R's references are not scaled
    HIP_TRY(lbm::launch_rescale(c->storage, c->cur, (int64_t)kSlots * c->np, factor, c->stream));
    c->exponent = e;
    drop_graphs(c);
    return LBM_OK;
}

// ---------------------------------------------------------------- adjoint
namespace {
// Events on the stream between the phases of a run; phase k of a mark lasts
// until the next mark.  The events are destroyed with the timer.
struct PhaseTimer {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    hipError_t mark(int k, hipStream_t s) {
        hipEvent_t e = nullptr;
        hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) return he;
        ev.push_back(e);
        kind.push_back(k);
        return hipEventRecord(e, s);
    }
    // after the stream has drained: milliseconds per phase kind (< n)
    hipError_t totals(double* ms, int n) const {
        for (int k = 0; k < n; ++k) ms[k] = 0.0;
        for (size_t i = 0; i + 1 < ev.size(); ++i) {
            float t = 0.f;
            hipError_t he = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
            if (he != hipSuccess) return he;
            if (kind[i] >= 0 && kind[i] < n) ms[kind[i]] += t;
        }
        return hipSuccess;
    }
    ~PhaseTimer() {
        for (auto e : ev) hipEventDestroy(e);
    }
};
enum { kPhaseForward = 0, kPhaseRecompute = 1, kPhaseReverse = 2, kPhaseOther = 3 };

struct AdjLayout {
    size_t snaps, seg, adjA, adjB, acc, part6, scratch4, out6, total;
    int nsnap;
};
AdjLayout adj_layout(const lbm_ctx* c, int n_steps, int K) {
    AdjLayout a{};
    const size_t state = align256((size_t)19 * c->np * 4);
    a.nsnap = std::max(1, (n_steps - 1 + K - 1) / K);
    size_t off = 0;
    a.snaps = off;
    off += state * a.nsnap;
    a.seg = off;
    off += state * (size_t)std::max(K - 1, 0);
    a.adjA = off;
    off += state;
    a.adjB = off;
    off += state;
    a.acc = off;  // FP32 body-force sensitivity of one segment, [3][np]
    off += align256((size_t)3 * c->np * 4);
    a.part6 = off;
    off += align256((size_t)kMaxGrid * 6 * 8);
    a.scratch4 = off;
    off += align256((size_t)kMaxGrid * 4 * 8);
    a.out6 = off;
    off += 256;
    a.total = off;
    return a;
}
}  // namespace

int lbm_adjoint_workspace_query(lbm_ctx* c, int n_steps, int K, size_t* bytes) {
    if (!c || !bytes) return fail(LBM_EINVAL, "NULL argument");
    if (n_steps < 1 || K < 1) return fail(LBM_EINVAL, "need n_steps >= 1 and checkpoint_every >= 1");
    *bytes = adj_layout(c, n_steps, K).total;
    return LBM_OK;
}

int lbm_adjoint(lbm_ctx* c, int N, int K, void* workspace, size_t workspace_bytes, double* k_out,
                double* dk_dtau, double* dk_dLambda, double* dk_dg) {
    if (!c || !dk_dtau || !dk_dLambda || !dk_dg) return fail(LBM_EINVAL, "NULL argument");
    if (c->storage != LBM_F32) return fail(LBM_EINVAL, "the adjoint needs FP32 storage");
    if (c->wall_mode != LBM_WALL_HALFWAY) return fail(LBM_EINVAL, "the adjoint is built for halfway bounce-back");
    if (c->pressure || c->idx.sym)
        return fail(LBM_EINVAL, "the adjoint is built for the body-force-driven periodic box");
    if (N < 1 || K < 1) return fail(LBM_EINVAL, "need n_steps >= 1 and checkpoint_every >= 1");
    if (c->g[c->axis] == 0) return fail(LBM_EINVAL, "no body force");
    const AdjLayout A = adj_layout(c, N, K);
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(LBM_EWORKSPACE, "adjoint workspace NULL or not 256-byte aligned");
    if (workspace_bytes < A.total)
        return fail(LBM_EWORKSPACE, "adjoint workspace too small: need " + std::to_string(A.total));
    char* ws = static_cast<char*>(workspace);
    const size_t state = align256((size_t)19 * c->np * 4);
    auto snap = [&](int s) { return (float*)(ws + A.snaps + state * s); };
    auto seg = [&](int t) { return (float*)(ws + A.seg + state * (t - 1)); };  // t >= 1
    double* part6 = (double*)(ws + A.part6);
    double* scratch4 = (double*)(ws + A.scratch4);
    double* out6 = (double*)(ws + A.out6);

    c->adj_timed = false;
    PhaseTimer timer;
    // forward from rest to step N, keeping fh^{sK}
    HIP_TRY(timer.mark(kPhaseForward, c->stream));
    HIP_TRY(lbm::launch_zero(c->cur, (int64_t)19 * c->np * 4, c->stream));
    HIP_TRY(zero_ring(c));
    c->steps = 0;
    c->pending = false;
    for (int n = 0; n < N; ++n) {
        if (n % K == 0 && n / K < A.nsnap && n <= N - 1)
            HIP_TRY(hipMemcpyAsync(snap(n / K), c->cur, (size_t)19 * c->np * 4,
                                   hipMemcpyDeviceToDevice, c->stream));
        int rc = do_steps(c, 1);
        if (rc) return rc;
    }
    HIP_TRY(timer.mark(kPhaseOther, c->stream));
    double u[3];
    int rc = lbm_mean_velocity(c, u);
    if (rc) return rc;
    const double gref = c->g[c->axis], V = volume(c), nu = viscosity(c);
    const double k = nu * u[c->axis] / gref;

    // reverse sweep
    float* a_in = (float*)(ws + A.adjA);
    float* a_out = (float*)(ws + A.adjB);
    HIP_TRY(lbm::launch_adjoint_seed(a_in, c->nf, c->axis, (float)(nu / (gref * V)), c->stream));
    HIP_TRY(lbm::launch_zero(part6, (int64_t)kMaxGrid * 6 * 8, c->stream));
    HIP_TRY(lbm::launch_zero(dk_dg, (int64_t)3 * c->nf * 8, c->stream));
    lbm::AdjLaunch al{};
    al.idx = c->idx;
    al.nf = c->nf;
    al.rates = rates_f(c->rates);
    for (int a = 0; a < 3; ++a) al.F[a] = (float)c->g[a];
    al.field = c->field;
    al.dk_acc = (float*)(ws + A.acc);
    al.acc_stride = c->np;
    al.grid = c->grid;
    al.partials = part6;
    const int nrev = N - 1;  // reverse steps n = N-1 .. 1
    for (int s = (nrev + K - 1) / K - 1; s >= 0; --s) {
        const int n0 = s * K;                        // segment start: fh^{n0}
        const int n1 = std::min((s + 1) * K, nrev);  // last reverse step of the segment
        // recompute fh^{n0+1} .. fh^{n1-1}
        HIP_TRY(timer.mark(kPhaseRecompute, c->stream));
        for (int t = 1; t < n1 - n0; ++t) {
            const void* src = t == 1 ? (const void*)snap(s) : (const void*)seg(t - 1);
            HIP_TRY(step_raw(c, src, seg(t), scratch4));
        }
        HIP_TRY(timer.mark(kPhaseReverse, c->stream));
        for (int n = n1; n > n0; --n) {
            al.adj_in = a_in;
            al.adj_out = a_out;
            al.state = (n - 1 - n0) == 0 ? snap(s) : seg(n - 1 - n0);
            al.first = n == n1;
            HIP_TRY(lbm::launch_adjoint_step(al, c->stream));
            std::swap(a_in, a_out);
        }
        HIP_TRY(timer.mark(kPhaseOther, c->stream));
        // the segment's FP32 force sensitivities into the FP64 total
        if (n1 > n0) HIP_TRY(lbm::launch_fold(dk_dg, al.dk_acc, c->nf, c->np, c->stream));
    }
    // readout's direct dependence on F through the shift u = (sum f c + F/2)
    double dv[3] = {0, 0, 0};
    dv[c->axis] = nu / (2.0 * gref * V);
    HIP_TRY(lbm::launch_add_uniform(dk_dg, c->nf, dv[0], dv[1], dv[2], c->stream));
    HIP_TRY(lbm::launch_finalize6(part6, c->grid, out6, c->stream));
    double cls[6];
    HIP_TRY(hipMemcpyAsync(cls, out6, sizeof(cls), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const lbm::RateClasses& dt = c->ds_dtau;
    const lbm::RateClasses& dl = c->ds_dLambda;
    const double via_t = cls[0] * dt.s_e + cls[1] * dt.s_eps + cls[2] * dt.s_q + cls[3] * dt.s_nu +
                         cls[4] * dt.s_pi + cls[5] * dt.s_m;
    const double via_l = cls[0] * dl.s_e + cls[1] * dl.s_eps + cls[2] * dl.s_q + cls[3] * dl.s_nu +
                         cls[4] * dl.s_pi + cls[5] * dl.s_m;
    *dk_dtau = via_t + u[c->axis] / (3.0 * gref);  // nu = (tau - 1/2)/3 in k
    *dk_dLambda = c->set == LBM_SET_E ? via_l : 0.0;
    if (k_out) *k_out = k;
    HIP_TRY(timer.totals(c->adj_ms, 3));
    c->adj_timed = true;
    return LBM_OK;
}

int lbm_adjoint_timing(const lbm_ctx* c, double ms[3]) {
    if (!c || !ms) return fail(LBM_EINVAL, "NULL argument");
    if (!c->adj_timed) return fail(LBM_EINVAL, "no lbm_adjoint has completed on this context");
    for (int k = 0; k < 3; ++k) ms[k] = c->adj_ms[k];
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) { delete c; }

}  // extern "C"
