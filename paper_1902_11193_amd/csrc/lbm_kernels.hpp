// Launch interface of the gfx950 kernels (host-callable, no HIP types beyond
// the stream).  Implemented in lbm_kernels.hip.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace lbm {

enum Storage : int { kF32 = 0, kF16 = 1, kBF16 = 2, kF16R = 3 };
enum IndexKind : int { kTable = 0, kBitmap = 1 };
enum Collision : int { kMrt = 0, kTrt = 1 };
// Slots of the ring of per-step sums (ux, uy, uz, drho) kept on the device.
constexpr uint32_t kRingSlots = 1024;
// Most blocks a step launch uses (its per-block partial sums are sized for it).
constexpr int kMaxGrid = 8192;
// The reduction scratch of a context: two buffers of per-block partial sums
// (double[kMaxGrid][4] each, 256-byte aligned) and the ring with its step
// counter, in that order; the tail of a workspace, or the static array.
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kPartialBytes = align256((size_t)kMaxGrid * 4 * 8);
constexpr size_t kReductionBytes = 2 * kPartialBytes + align256((size_t)kRingSlots * 4 * 8 + 4);

// Device address of the current GPU's static reduction scratch (one array
// of kReductionBytes per GPU, kept until the process ends), looked up once
// per device.
hipError_t static_scratch(void** ptr);

struct RatesF {
    float s_e, s_eps, s_q, s_nu, s_pi, s_m;
};

// Device view of the neighbour index.
struct IndexView {
    int kind;
    int64_t stride;             // padded node count np (row stride of the table)
    int64_t slack;              // elements between a chunk's gather base and the chunk (gather_span)
    const int32_t* table;       // kTable: [18][stride] pull sources, -1 = solid
    const uint32_t* coords;     // kBitmap: [nf] packed voxel coordinates
    const void* ent;            // kBitmap: [nz][ny][R] 16-byte entries (rows y - 1, y, y + 1)
    const void* wrap;           // kBitmap: [nz][2][R] 16-byte slots: bases of the rows across the y wrap
    const void* count;          // kBitmap: [nz][ny] 16-byte slots: the x wrap's row counts
    int nx, ny, nz, R, bx, by;  // kBitmap geometry; R = words per row
    int sym;                    // kBitmap: symmetry planes, bit 0 on the y faces, bit 1 on the z faces
                                // (the entries then hold the y ghost rows)
};

struct StepLaunch {
    int storage;
    int collision;        // kMrt: moment space, any set; kTrt: link-wise, two-rate sets only
    const void* src;      // deviations (storage type), chunked: element (i, n) at state_elem(i, n)
    void* dst;            // same layout
    IndexView idx;
    int64_t nf;
    RatesF rates;
    float F[3];           // uniform force density
    const float* field;   // optional [3][nf] accelerations (rho0 = 1), or nullptr
    float scale, inv_scale;
    int grid;             // number of blocks (fixed per context)
    double* partials;     // [grid][4] written by this step
    const double* prev_partials;  // [grid][4] of the previous step, reduced by block 0 into
                                  // ring slot (*ctr % kRingSlots), then ++*ctr; nullptr: nothing pending
    double* ring;                 // [kRingSlots][4] per-step sums
    uint32_t* ctr;                // steps reduced so far (device)
    float* wall;          // full-way bounce-back: per-node fh of the previous step (state layout,
                          // FP32 storage only), or nullptr for halfway bounce-back
    bool pressure;        // Zou-He pressure faces at x = 0 and x = nx - 1 (FP32, bitmap, no field)
    float drho_in, drho_out;  // their density deviations rho - rho0
};

// One fused step: gather with halfway bounce-back, MRT + Guo collision, store,
// and per-block FP64 partial sums of (ux, uy, uz, drho).
hipError_t launch_step(const StepLaunch& a, hipStream_t s);

// Resident blocks per compute unit of the step kernel for this storage/index/collision.
hipError_t step_occupancy(int storage, int index_kind, int collision, int* blocks_per_cu);

// Sum the per-block partials in fixed order into ring slot (*ctr % kRingSlots), ++*ctr.
hipError_t launch_finalize(const double* partials, int grid, double* ring, uint32_t* ctr, hipStream_t s);

// Fill count elements of `bytes_per_elem` size with zero bits.
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s);

// Multiply every stored deviation by `factor` (storage-exponent change).
hipError_t launch_rescale(int storage, void* p, int64_t count, float factor, hipStream_t s);

// ---------------------------------------------------------------- adjoint
struct AdjLaunch {
    const float* adj_in;   // a^{n+1}: adjoint of the gathered populations of step n+1 (state layout)
    float* adj_out;        // a^n
    const float* state;    // fh^{n-1}: FP32 deviations (state layout)
    IndexView idx;
    int64_t nf;
    RatesF rates;
    float F[3];
    const float* field;
    float* dk_acc;         // [3][acc_stride] FP32 body-force sensitivity of the current segment:
                           // written by the step with `first`, added to by the others
    int64_t acc_stride;    // >= padded node count
    bool first;
    int grid;
    double* partials;      // [grid][6] accumulated in place: rate-class sensitivities
};
hipError_t launch_adjoint_step(const AdjLaunch& a, hipStream_t s);

// dk_dF[a][n] += acc[a][n] for n < nf (one segment's FP32 sums into the FP64 total).
hipError_t launch_fold(double* dk_dF, const float* acc, int64_t nf, int64_t stride, hipStream_t s);

// a^N seed: element (i, n) = kappa * c_i[axis] for fluid nodes (state layout).
hipError_t launch_adjoint_seed(float* adj, int64_t nf, int axis, float kappa,
                               hipStream_t s);

// out[k] = sum over blocks of partials[b][k], k < 6, fixed order.
hipError_t launch_finalize6(const double* partials, int grid, double* out, hipStream_t s);

// dk_dF[a][n] += v[a] for every node (direct terms of the readout).
hipError_t launch_add_uniform(double* dk_dF, int64_t nf, double vx, double vy, double vz,
                              hipStream_t s);

}  // namespace lbm
