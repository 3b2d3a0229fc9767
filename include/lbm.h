/*
 * liblbm -- D3Q19 multiple-relaxation-time lattice-Boltzmann permeability
 * solver for segmented voxel images on AMD Instinct MI355X (gfx950).
 *
 * Method: Rao & Schaefer, "Lattice Boltzmann Models for Micro-tomographic
 * Pore-spaces" (arXiv:1902.11193).  One time step is the lattice Boltzmann
 * equation (Sec. 2, Eq. LBE) with the MRT collision of Sec. 2.1.1
 * (Eqs. MRT Collision, MRT Equi, MRT params), Guo body forcing
 * (Eqs. MRT-LBE, Guo_Forcing), halfway bounce-back at solid voxels in a
 * periodic box driven by a uniform body force (Sec. 2.3), and the Darcy
 * permeability k_j = nu <u_j> / g_j (Sec. 3, Eq. perm_calc) with the
 * steady-state test of Eq. convergence.
 *
 * Conventions shared by every call
 *   - geometry: uint8 [nz][ny][nx], x fastest; 0 = fluid, any other value =
 *     solid.  The box is periodic in all three axes.
 *   - Only fluid voxels carry populations.  They are numbered 0..n_fluid-1,
 *     the "compacted fluid list", in node order: the (y, z) rows of the image
 *     taken in z-tiles of h planes (tile, then y, then z inside the tile),
 *     the fluid voxels of each row in increasing x.  The T = ceil(nz / h)
 *     tiles come folded, t = 0, T-1, 1, T-2, ..., so tiles that touch in z
 *     (periodic wrap included) are near each other in the list.  h is the
 *     tallest of 128, 64, 32, ..., 1 planes for which the populations
 *     gathered around any 256-node chunk span less than 4 GiB in FP32 (else
 *     in a 16-bit storage); it depends on the image alone.  Every per-node
 *     array of this interface (state, force field, gradients, neighbour
 *     table) uses this order; lbm_node_order gives the voxel of each node.
 *   - Velocity order i = 0..18 (pairs i, i+1 for odd i are opposite):
 *       0:( 0, 0, 0)
 *       1:( 1, 0, 0)  2:(-1, 0, 0)  3:( 0, 1, 0)  4:( 0,-1, 0)
 *       5:( 0, 0, 1)  6:( 0, 0,-1)  7:( 1, 1, 0)  8:(-1,-1, 0)
 *       9:( 1,-1, 0) 10:(-1, 1, 0) 11:( 1, 0, 1) 12:(-1, 0,-1)
 *      13:( 1, 0,-1) 14:(-1, 0, 1) 15:( 0, 1, 1) 16:( 0,-1,-1)
 *      17:( 0, 1,-1) 18:( 0,-1, 1)
 *     with weights 1/3, 1/18 (|c|^2 = 1), 1/36 (|c|^2 = 2); rho0 = 1.
 *   - State: post-collision populations after the last step.  On the device
 *     they are stored as deviations f_i - w_i rho0 in FP32, FP16 or BF16
 *     (FP16 scaled by a power of two), or for LBM_F16R as FP16 deviations
 *     from a per-node reference density (below); collision arithmetic is
 *     FP32; the mean velocity and mass are reduced in FP64.
 *   - Step n = gather (pull stream with halfway bounce-back), then collide.
 *     <u>_n is the volume average (sum over fluid / (nx ny nz)) of the
 *     shifted velocity (sum_i f_i c_i + F/2) / rho0 of the populations
 *     gathered at step n.  The state starts at rest, f_i = w_i rho0.
 *   - Memory: the library allocates no device memory.  The caller passes a
 *     device workspace (size from lbm_workspace_query) that must outlive the
 *     context.  All device work is enqueued on the caller's HIP stream.
 *   - Errors: every int-returning call returns LBM_OK (0) or a negative code;
 *     lbm_last_error() gives a message (thread-local).  Arguments are checked
 *     before any HIP call is made.
 */
#ifndef LIBLBM_H
#define LIBLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)     /* bad argument (dims, tau <= 1/2, non-finite, set, rates outside (0,2)) */
#define LBM_ENOFLUID (-2)   /* the image has no fluid voxel */
#define LBM_EWORKSPACE (-3) /* workspace missing, too small or misaligned (needs 256-byte alignment) */
#define LBM_EHIP (-4)       /* a HIP runtime call failed; message has the HIP error string */
#define LBM_ENAN (-5)       /* non-finite mean velocity or mass: the run diverged or overflowed */
#define LBM_ERANGE (-6)     /* image too large for the index or gather layout */
#define LBM_EBUSY (-7)      /* the GPU's static reduction scratch is held by another live context */

/* Bytes of reduction scratch at the end of the workspace lbm_workspace_query
 * sizes: per-block partial sums of the mean velocity and the ring of per-step
 * sums.  lbm_setup_static keeps them in a static array instead. */
#define LBM_REDUCTION_BYTES 557312

/* Relaxation-rate sets of Table 2 (Sec. 2.2). */
#define LBM_SRT 0
#define LBM_SET_A 1
#define LBM_SET_B 2
#define LBM_SET_C 3
#define LBM_SET_D 4
#define LBM_SET_E 5

/* Storage type of the population deviations.
 * LBM_F32, LBM_F16, LBM_BF16: f_i - w_i rho0 (FP16 scaled by 2^e).
 * LBM_F16R: FP16 with a reference density per node.  A node also stores
 *   r = fp16(rho - rho0) of its own populations (in an array of one FP16 per
 *   node after the populations of the state), and each population as
 *   2^e (f_i - w_i rho0 - w_i r); the node that pulls a value adds w_i r of
 *   the node it came from.  Both sides use the same stored r, so nothing is
 *   lost to the reference; FP16 rounds only the velocity and
 *   non-equilibrium part.  In rock that part is orders of magnitude smaller
 *   than the density deviation that plain FP16 must carry.  20 values per
 *   node (80 bytes per node-update moved instead of 76). */
#define LBM_F32 0
#define LBM_F16 1
#define LBM_BF16 2
#define LBM_F16R 3

/* Neighbour layout used by the gather.
 * LBM_INDEX_TABLE:  int32 [18][n_pad] table of pull-source nodes (-1 = wall),
 *                   72 bytes per fluid node.
 * LBM_INDEX_BITMAP: one packed uint32 voxel coordinate per node plus, for
 *                   every (y, z) row and every 18 voxels of it, a 16-byte
 *                   entry (the 20 fluid bits of that word in rows y - 1, y,
 *                   y + 1 of the plane, the node number before the word in
 *                   row y and the differences to those of rows y - 1 and
 *                   y + 1), small slots for the rows across the periodic y
 *                   wrap and the fluid counts the periodic x wrap needs; the
 *                   source node of a link is found by a population count.
 *                   4 bytes per node + about 0.94 bytes per voxel.  Needs
 *                   ceil(log2 nx) + ceil(log2 ny) + ceil(log2 nz) <= 32,
 *                   nx <= 4095 and fewer than 2^32 row words
 *                   (ny nz ceil(nx / 18)). */
#define LBM_INDEX_TABLE 0
#define LBM_INDEX_BITMAP 1

/* Collision kernels (lbm_set_collision).
 * LBM_COLLIDE_MRT: the moment-space collision of Sec. 2.1.1 (Eq. MRT-LBE),
 *                  any relaxation set.  The default.
 * LBM_COLLIDE_TRT: the same map written link-wise on opposite pairs (the
 *                  two-relaxation-time form of Sec. 2.1.2), for sets whose
 *                  even non-conserved moments share one rate and odd ones
 *                  another: SRT, Set B, Set E.  Equal to MRT up to rounding. */
#define LBM_COLLIDE_MRT 0
#define LBM_COLLIDE_TRT 1

/* Wall schemes (lbm_set_wall).
 * LBM_WALL_HALFWAY: the wall midway between a fluid and a solid voxel; a
 *                   population sent into it returns at the next step.  The
 *                   default, and the scheme every other statement here uses.
 * LBM_WALL_FULLWAY: the paper's full-way bounce-back (Sec. 2.3): the
 *                   population travels to the solid voxel, turns there at the
 *                   next collision and returns one step later than halfway.
 *                   The steady state at fluid nodes is the same. */
#define LBM_WALL_HALFWAY 0
#define LBM_WALL_FULLWAY 1

typedef struct lbm_ctx lbm_ctx;

/* Host only.  The velocity order above: c[i][0..2] = (cx, cy, cz). */
int lbm_velocities(int c[19][3]);

/* Host only.  The 19 diagonal entries of the relaxation matrix S
 * (Eq. MRT params) for a set of Table 2 at (tau, Lambda); Lambda is read only
 * for LBM_SET_E (Eq. Magic param).  Moment order: rho, e, eps, jx, qx, jy,
 * qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz.  Also returns
 * d s / d tau and d s / d Lambda when the pointers are non-NULL. */
int lbm_rates(int relaxation_set, double tau, double Lambda, double s[19],
              double ds_dtau[19], double ds_dLambda[19]);

/* Host only.  Counts fluid voxels and the device workspace the context
 * needs.  Fails with LBM_ENOFLUID / LBM_ERANGE / LBM_EINVAL as lbm_setup.
 * LBM_ERANGE: 2^31 or more fluid nodes; with the bitmap index, packed
 * coordinates over 32 bits, nx above 4095 or 2^32 row words or more; or the
 * populations gathered around one 256-node chunk
 * spanning 4 GiB or more in the chosen storage (up to five z-tiles of fluid
 * nodes, with the tile height of the node order, at 76 bytes each for FP32,
 * 38 for FP16/BF16/F16R). */
int lbm_workspace_query(const uint8_t* geometry, int nx, int ny, int nz, int storage,
                        int index_kind, size_t* bytes, int64_t* n_fluid);

/* Host only.  Non-periodic image stacks (Sec. 2.3, the paper's sphere-pack
 * setup): `pad` fluid-only layers are added before and after the image along
 * x, the driven axis, and with mirror_y / mirror_z the image is reflected
 * across its y / z faces.  In the periodic box this gives, the reflected faces
 * are symmetry (mirror) planes (zero normal velocity, zero normal gradients)
 * and the padding separates outlet from inlet.  lbm_boundary_dims returns
 * the new extents: nx + 2 pad, ny (2 ny with mirror_y), nz (2 nz with
 * mirror_z).  lbm_boundary_image writes the new uint8 image
 * [onz][ony][onx] to `out` (caller-owned, host).  The flow in the original
 * image is that of the new box for x in [pad, pad + nx), y < ny, z < nz; the
 * superficial <u_x> is the same over the whole new box, so lbm_permeability
 * of a context built on it is that of the padded sample with the body force
 * on every fluid voxel, as in the paper.  LBM_EINVAL: bad extents, pad
 * outside [0, 2^20], NULL pointers; LBM_ERANGE: new extents too large. */
int lbm_boundary_dims(int nx, int ny, int nz, int pad, int mirror_y, int mirror_z, int* onx, int* ony,
                      int* onz);
int lbm_boundary_image(const uint8_t* geometry, int nx, int ny, int nz, int pad, int mirror_y, int mirror_z,
                       uint8_t* out);

/* Host only (no GPU needed).  Pull sources of selected nodes, as in
 * lbm_neighbor_table but for nodes[count] only (node numbers in node order):
 * table[18][count] int32, entry (i-1)*count + k, -1 where the source voxel is
 * solid.  Caller-owned host arrays.  LBM_EINVAL for a node out of range. */
int lbm_neighbor_nodes(const uint8_t* geometry, int nx, int ny, int nz, const int64_t* nodes, int64_t count,
                       int32_t* table);

/* Host only (no GPU needed).  Linear voxel id x + nx (y + ny z) of every
 * node, in node order: voxel[n_fluid] int64, owned by the caller. */
int lbm_node_order(const uint8_t* geometry, int nx, int ny, int nz, int64_t* voxel,
                   int64_t n_fluid);

/* Host only (no GPU needed).  The pull-source table of the compacted fluid
 * list: table[(i-1) * n_fluid + n] = node at x_n - c_i (periodic), or -1 when
 * that voxel is solid (halfway bounce-back), for i = 1..18.  `table` holds
 * 18 * n_fluid int32 and is owned by the caller. */
int lbm_neighbor_table(const uint8_t* geometry, int nx, int ny, int nz, int32_t* table,
                       int64_t n_fluid);

/* The problem of Sec. 2 and Sec. 3 (Eq. LBE, with Eq. MRT-LBE for the
 * forced MRT collision): a segmented image, the relaxation time tau (the
 * viscosity nu = (tau - 1/2)/3), a relaxation set of Table 2 with the magic
 * parameter Lambda of Eq. Magic param (Set E), and a body force driving the
 * flow (Sec. 2.3).  Builds the context: copies and compacts the geometry
 * (borrowed for the call only; the solid voxels carry no work, Sec. 3),
 * computes the rates, uploads the index to `workspace` and sets the state to
 * rest.  g[3] is the body-force acceleration (lattice units); F = rho0 g acts
 * on every fluid node.  Errors: LBM_EINVAL (NULL ctx, geometry or g, bad
 * extents, tau <= 1/2, a set outside 0..5, Lambda <= 0 for Set E, a rate
 * outside (0, 2), non-finite g), LBM_ENOFLUID, LBM_ERANGE,
 * LBM_EWORKSPACE (NULL, not 256-byte aligned, smaller than
 * lbm_workspace_query's bytes), LBM_EHIP; *ctx is NULL on error.  `hip_stream` is a hipStream_t (NULL =
 * the default stream).  Returns the context in *ctx (owned by the caller,
 * freed with lbm_destroy).  Synchronises the stream before returning. */
int lbm_setup(lbm_ctx** ctx, const uint8_t* geometry, int nx, int ny, int nz, double tau,
              double Lambda, int relaxation_set, const double g[3], int storage, int index_kind,
              void* workspace, size_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate device memory at this point (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same as lbm_setup, except that the reduction scratch (LBM_REDUCTION_BYTES:
 * two buffers of per-block partial sums and the ring of per-step sums) lives
 * in a static device array of that size compiled into the library, one per
 * GPU, held until the process ends, instead of at the end of `workspace`.
 * `workspace` needs only lbm_workspace_query's bytes minus
 * LBM_REDUCTION_BYTES; the library makes no device allocation.  One live
 * context per GPU may hold the array: a second call on the same device
 * returns LBM_EBUSY until the first context is destroyed.  The array keeps
 * what the last context left in it; setup clears the ring and its step
 * counter.  Launches that overlap on one GPU from outside the owning
 * context's stream order would race on the array; the owning context's own
 * calls are ordered on its stream.  Other errors as lbm_setup. */
int lbm_setup_static(lbm_ctx** ctx, const uint8_t* geometry, int nx, int ny, int nz, double tau,
                     double Lambda, int relaxation_set, const double g[3], int storage, int index_kind,
                     void* workspace, size_t workspace_bytes, void* hip_stream);

/* Advances n >= 0 time steps of Eq. LBE (Sec. 2): per step every fluid node
 * pulls f_i from x - c_i (halfway bounce-back where that voxel is solid),
 * collides in moment space (Eq. MRT-LBE with the equilibria of Eq. MRT Equi
 * and Guo's source, Eq. Guo_Forcing) and stores the result; the same launch
 * sums the node velocities for <u>_n.  Asynchronous on the context's stream.
 * LBM_EINVAL for n < 0, LBM_EHIP if a launch fails. */
int lbm_step(lbm_ctx* ctx, int n);

/* Steps taken since setup (or since the last lbm_set_state). */
int64_t lbm_steps_done(const lbm_ctx* ctx);

/* Mean velocity <u>_n of the last step (FP64), the volume average of
 * Eq. perm_calc.  Synchronises the stream.  LBM_ENAN if it is not finite.
 * Before the first step: zeros. */
int lbm_mean_velocity(lbm_ctx* ctx, double u[3]);

/* k_j = nu <u_j>_n / g_j with nu = (tau - 1/2)/3 (Eq. perm_calc); NaN where
 * g_j == 0.  Synchronises the stream. */
int lbm_permeability(lbm_ctx* ctx, double k[3]);

/* Sum over fluid nodes of the density deviation rho - rho0 at the last step
 * (FP64); the collision leaves rho unrelaxed (s_0 = 0 in Table 2) and the
 * stream with bounce-back moves populations without loss, so it stays at
 * rounding level. */
int lbm_mass_deviation(lbm_ctx* ctx, double* dm);

/* Total mass sum_fluid rho = n_fluid rho0 + lbm_mass_deviation (rho0 = 1),
 * at the last step (n_fluid before the first).  Synchronises the stream. */
int lbm_mass(lbm_ctx* ctx, double* m);

/* Per-step mean velocities (Eq. perm_calc) of the last `count` steps (count
 * <= 1024 and <= steps done), oldest first, into u[count][3] (host): the
 * history the test of Eq. convergence reads.  Synchronises. */
int lbm_history(lbm_ctx* ctx, int count, double* u);

/* Steps in chunks of `check_every` until the per-step relative change of
 * k along the largest |g| component falls below eps (Eq. convergence) or
 * max_steps have run.  *steps = steps taken in this call, k = last k,
 * *converged = 1 when the test held at some step of the last chunk.
 * The test is the paper's, as printed: it can hold at a turning point of an
 * early overshoot, and on geometries where k keeps a neutral period-2
 * oscillation it may never hold; the mean of two successive lbm_history
 * entries converges in that case. */
int lbm_run_to_steady(lbm_ctx* ctx, double eps, int check_every, int max_steps, int* steps,
                      double k[3], int* converged);

/* Host.  The state of selected nodes only (full populations f_i, FP64,
 * f[19][count], entry i*count + k), read chunk by chunk from the device:
 * for sampled checks of images too large to copy whole.  Synchronises. */
int lbm_get_state_nodes(lbm_ctx* ctx, const int64_t* nodes, int64_t count, double* f);

/* Host copies of the state, the post-collision populations of Eq. LBE:
 * full populations f_i = w_i rho0 + deviation in FP64, layout
 * [19][n_fluid] (host memory owned by the caller).
 * lbm_set_state also resets the step count and the mean-velocity history.
 * Synchronise the stream. */
int lbm_get_state(lbm_ctx* ctx, double* f);
int lbm_set_state(lbm_ctx* ctx, const double* f);

/* Linear voxel id (x + nx (y + ny z)) of every fluid node, host int64 [n_fluid]. */
int lbm_fluid_index(lbm_ctx* ctx, int64_t* voxel);

/* Optional per-node body force, the F of Eq. MRT-LBE and Eq. Guo_Forcing
 * varying from node to node: a device FP32 array [3][n_fluid] of
 * accelerations owned by the caller, read by every later step (it must stay
 * alive and unchanged until replaced).  NULL returns to the uniform g of
 * lbm_setup.  k keeps dividing by the g of lbm_setup. */
int lbm_set_force_field(lbm_ctx* ctx, const float* g_device);

int64_t lbm_n_fluid(const lbm_ctx* ctx);

/* Host + enqueue.  Chooses the collision kernel for the following steps
 * (LBM_COLLIDE_MRT or LBM_COLLIDE_TRT, see above); flushes a pending
 * reduction first.  LBM_EINVAL for an unknown kind or for TRT with a set that
 * is not two-rate (A, C, D); the context is then unchanged. */
int lbm_set_collision(lbm_ctx* ctx, int collision);

/* Host + enqueue.  Chooses the wall scheme for the following steps.
 * LBM_WALL_FULLWAY needs FP32 storage and a device workspace of
 * lbm_wall_workspace_query bytes (256-byte aligned, caller-owned, must outlive
 * the mode): it holds every node's populations of one step earlier, and is
 * initialised to the current state (as is again by lbm_set_state).
 * LBM_WALL_HALFWAY releases it (workspace may be NULL).  Errors: LBM_EINVAL
 * (unknown mode, storage other than FP32), LBM_EWORKSPACE.  lbm_adjoint refuses a
 * context in full-way mode. */
int lbm_wall_workspace_query(lbm_ctx* ctx, size_t* bytes);
int lbm_set_wall(lbm_ctx* ctx, int mode, void* workspace, size_t workspace_bytes);

/* Host only.  Pressure-driven flow (Sec. 2.3, 3.1): with enable != 0 the box
 * is no longer periodic in x; the fluid nodes of the planes x = 0 and
 * x = nx - 1 get Zou-He pressure boundaries at densities rho_in and rho_out
 * (rho0 = 1): the populations arriving from outside the image are rebuilt
 * from the known ones for that density, zero transverse velocity and equal
 * non-equilibrium parts of the opposite pair along x.  lbm_permeability then
 * returns k_x = nu <u_x> / grad p with grad p = (rho_in - rho_out) / 3 /
 * (nx - 1) (Eq. perm_calc; k_y, k_z NaN), and lbm_run_to_steady tests k_x.
 * Needs FP32 storage, the bitmap index, g = (0, 0, 0) at lbm_setup, no force
 * field, halfway bounce-back and nx >= 3 (else LBM_EINVAL; rho_in, rho_out
 * finite, positive, different).  enable = 0 returns to the periodic box.
 * lbm_adjoint refuses a context with pressure faces. */
int lbm_set_pressure(lbm_ctx* ctx, int enable, double rho_in, double rho_out);

/* Host + device upload.  Symmetry (mirror) planes on the faces normal to y
 * and/or z (Sec. 2.3, the lateral planes of the paper's sphere-pack setup):
 * the box is no longer periodic across those faces; a population that a
 * step would pull from beyond such a face comes from the boundary layer's own
 * voxel reached by the other components of c_i, with its velocity mirrored in
 * that axis (zero normal velocity and zero normal gradients at the plane,
 * half a voxel outside the layer).  Halfway (or full-way) bounce-back applies
 * where that voxel is solid.  The same problem as lbm_boundary_image's
 * reflected image, without its 2x (4x) nodes.  Needs the bitmap index and
 * FP32 storage, no pressure faces (else LBM_EINVAL); rebuilds the index
 * entries (synchronises the stream).  (0, 0) returns to the periodic box.
 * lbm_adjoint refuses a context with symmetry planes. */
int lbm_set_symmetry(lbm_ctx* ctx, int mirror_y, int mirror_z);

/* Host only.  With enable != 0 (the default), lbm_step and
 * lbm_run_to_steady run stretches of 32 steps, once a step is pending, by
 * replaying a HIP graph captured from the same launches on first use (one
 * launch call per 32 steps: small images are otherwise launch-bound).  The
 * results are identical to plain launches, which enable = 0 selects.  Any
 * change of collision, wall, pressure, force field or storage exponent drops
 * the captured graphs. */
int lbm_set_graphs(lbm_ctx* ctx, int enable);

/* FP16 storage keeps 2^e (f_i - w_i rho0); e defaults to
 * round(-log2 max|g|) - 4, and for LBM_F16R to round(-log2 max|g|) + 2
 * (its values are velocity-sized).  May be changed at any time (the state is
 * rescaled; LBM_F16R's reference slot is not scaled).  Ignored for FP32 /
 * BF16 storage, where e = 0. */
int lbm_set_storage_exponent(lbm_ctx* ctx, int e);

/* Discrete adjoint (an extension beyond the paper's method): exact
 * derivatives of k_N (the permeability after N = n_steps steps from rest,
 * along the largest |g| component) with respect to tau, Lambda and the
 * per-node body-force acceleration, by reverse time stepping with
 * two-level checkpointing: a snapshot every `checkpoint_every` steps, the
 * steps of one segment recomputed and kept while it is reversed.
 * Re-runs the forward from rest; the context's state afterwards is the
 * state after n_steps steps.  Needs FP32 storage.
 * Workspace: size from lbm_adjoint_workspace_query, device, caller-owned.
 * dk_dg: device FP64 [3][n_fluid] (caller-owned), overwritten.
 * dk_dLambda is 0 unless the set is LBM_SET_E. */
int lbm_adjoint_workspace_query(lbm_ctx* ctx, int n_steps, int checkpoint_every, size_t* bytes);
int lbm_adjoint(lbm_ctx* ctx, int n_steps, int checkpoint_every, void* workspace,
                size_t workspace_bytes, double* k, double* dk_dtau, double* dk_dLambda,
                double* dk_dg);

/* Host only.  Where the last completed lbm_adjoint on this context spent its
 * GPU time, measured with HIP events on its stream: ms[0] the forward run
 * from rest with its snapshots, ms[1] the recomputation of the checkpoint
 * segments, ms[2] the reverse steps.  LBM_EINVAL before any. */
int lbm_adjoint_timing(const lbm_ctx* ctx, double ms[3]);

void lbm_destroy(lbm_ctx* ctx);

/* Message of the last failing call on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBLBM_H */
