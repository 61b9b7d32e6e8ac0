/*
 * ltm.h -- C ABI of the light-transport camera model library (libltm.so).
 *
 * The library computes, on an AMD MI355X (gfx950), the matrix-free camera
 * operator y = A x of McGaffin, Chen, Fessler and Sick, "A practical light
 * transport system model for chemiluminescence distribution reconstruction"
 * (arXiv 1812.03358), its exact transpose x = A^T y, and the penalized
 * nonnegative least-squares reconstruction of the paper's reconstruction
 * section.
 *
 * Conventions shared by every entry point
 *   - Pointers named x, y, w, ws, ... are DEVICE pointers (hipMalloc'ed or
 *     torch CUDA tensors).  Descriptors and parameter structs are host
 *     memory.  Streams are hipStream_t passed as void* (NULL = null stream).
 *   - The library never allocates device memory: every buffer, including
 *     the workspace a plan needs, is provided by the caller.  Plans and
 *     solvers own host memory only.
 *   - Calls are asynchronous on the given stream unless stated otherwise.
 *     Outputs are overwritten, never accumulated into.
 *   - Layouts: a volume x is float32 [nz][ny][nx] (x fastest), voxel (i,j,k)
 *     centred at ((i + 1/2 - nx/2) d, (j + 1/2 - ny/2) d, (k + 1/2 - nz/2) d)
 *     in world millimetres (the voxel basis of the paper's object-model
 *     section); y holds the cameras' images one after another, each
 *     float32 [det_nv][det_nu] with u (the s axis) fastest (the paper stores
 *     light fields column-major with s fastest).
 *   - Every function returns an ltm_status.  On failure nothing has been
 *     launched and ltm_last_error() returns a message (thread-local).  No C++
 *     exception crosses this interface.
 */
#ifndef LTM_H
#define LTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LTM_ABI_VERSION 4u

typedef enum ltm_status {
    LTM_OK = 0,
    LTM_ERR_INVALID = 1,      /* bad descriptor, size or argument */
    LTM_ERR_DEVICE = 2,       /* a HIP call failed */
    LTM_ERR_NUMERIC = 3,      /* non-finite value met by the solver */
    LTM_ERR_WORKSPACE = 4,    /* workspace missing or too small */
    LTM_ERR_UNSUPPORTED = 5   /* valid request the library does not implement */
} ltm_status;

enum { LTM_SINGLE_LENS = 0u, LTM_PLENOPTIC = 1u, LTM_PLENOPTIC_HEX = 2u };
enum { LTM_FORWARD = 0u, LTM_ADJOINT = 1u };

/* Voxel grid centred at the world origin (object-model section: pillbox
 * voxels of edge pitch_mm; here sampled by trilinear interpolation between
 * voxel centres).  Each of nx, ny, nz must be at least 2. */
typedef struct ltm_grid {
    uint32_t nx, ny, nz, reserved;
    double pitch_mm;
} ltm_grid;

/* One camera.  Optics follow the paper's camera-model section: a thin main
 * lens (focal length f_main, aperture radius r_main) at camera depth 0, with
 *   single lens: the detector at depth -d_det;
 *   plenoptic:   a square microlens array at depth -d_mla (lenslets of
 *                radius r_mla, focal length f_mla, pitch det_nu/mla_nu
 *                pixels) and the detector d_mla_det behind it;
 *   hexagonal plenoptic (the simulated plenoptic table as listed): a
 *                hexagonal array of mla_nu lenslets per row and mla_nv rows
 *                of touching lenslets (pitch 2 r_mla, row spacing
 *                sqrt(3) r_mla; rows at odd distance from row mla_nv/2
 *                shifted by r_mla along s; lenslet (i, j) at
 *                s = (i - (mla_nu-1)/2 + shift) 2 r_mla,
 *                t = (j - (mla_nv-1)/2) sqrt(3) r_mla) whose lenslets have
 *                three focal lengths f_hex_mm[type], type = (q - r) mod 3 in
 *                hexagonal axial coordinates (r = j - mla_nv/2,
 *                q = i + shift - r/2), so that neighbours differ.  A pixel
 *                sums the light through every lenslet (the sum over
 *                microlenses of the plenoptic-camera section).  The library
 *                visits, per pixel, the 3 x 3 lenslets around it (nearest
 *                row +-1, nearest lenslet of each row +-1) and rejects
 *                cameras for which light could arrive from farther:
 *                (e hd + e (r_main + k r_mla)) / (1 + e) must stay below
 *                1.5 sqrt(3) r_mla, with e = d_mla_det/d_mla, hd the
 *                detector's half diagonal (pixel centres) and k the largest
 *                |1 + d_mla/d_mla_det - d_mla/f|.  rays_u*rays_v <= 7.
 * Rays are traced from each pixel centre through rays_u x rays_v angular
 * samples -- the centres of a grid over the aperture's bounding square
 * (main lens for single-lens cameras, the pixel's own lenslet for square
 * plenoptic ones, each visited lenslet for hexagonal ones); samples outside
 * the circular aperture, or a plenoptic ray that misses the main lens, are
 * occluded but still count in the 1/R mean.
 * Each ray is integrated with `samples` midpoint samples over its segment
 * inside the grid.  Camera point (s,t,z) is world point
 * lens_center + s e_s + t e_t + z e_z, axes = {e_s, e_t, e_z} (orthonormal,
 * right-handed), and the scene is at z > 0. */
typedef struct ltm_camera {
    uint32_t kind;              /* LTM_SINGLE_LENS, LTM_PLENOPTIC or LTM_PLENOPTIC_HEX */
    uint32_t det_nu, det_nv;    /* detector pixels */
    uint32_t mla_nu, mla_nv;    /* plenoptic only: lenslets (square: det_n* multiples) */
    uint32_t rays_u, rays_v;    /* angular samples per pixel, R = rays_u*rays_v <= 64 */
    uint32_t samples;           /* S >= 1 */
    double pixel_pitch_mm;
    double f_main_mm, r_main_mm;
    double d_det_mm;            /* single lens only */
    double d_mla_mm, d_mla_det_mm, f_mla_mm, r_mla_mm;  /* plenoptic only */
    double axes[9];
    double lens_center_mm[3];
    double f_hex_mm[3];         /* hexagonal plenoptic only: focal length per lenslet type */
} ltm_camera;

/* How one camera's rays are grouped into workgroups.  A tile is a block of
 * tile_u x tile_v lenslets (for single-lens and hexagonal plenoptic
 * cameras, blocks of block_u x block_v pixels play the lenslets' role).  Its pixels are split
 * over `splits` workgroups.  `order` holds flags: bit 0 clear puts one
 * lenslet's pixels on adjacent lanes, set walks adjacent lanes across
 * lenslets; bit 1 stops lanes from starting their angular-sample loop at
 * different samples; bit 2 (adjoint) accumulates the brick in FP32 before the
 * FP64 flush; bit 3 (adjoint) staggers the lanes' walks along their rays;
 * bit 4 (adjoint) merges consecutive samples of one trilinear cell in
 * registers before the LDS atomics; bit 5 (adjoint) instead keeps two planes
 * of corner sums across the ray's dominant axis, so a step along that axis
 * flushes 4 corners, not 8; bit 6 (with bit 3) makes the staggered starting
 * offsets even, so rays that advance half a voxel per sample along that axis
 * cross its cell planes on the same iterations.  Each workgroup
 * marches its rays through consecutive slabs of chunk_mm camera depth,
 * staging the voxels the slab's rays touch in an LDS brick of at most
 * brick_floats floats (a slab whose brick does not fit uses global memory).
 * Tilings change speed only: every tiling computes the same samples. */
typedef struct ltm_tiling {
    uint32_t tile_u, tile_v;
    uint32_t block_u, block_v;
    uint32_t order;
    uint32_t splits;
    uint32_t brick_floats;      /* 0: no LDS staging */
    uint32_t groups_per_cu;     /* 0: as many workgroups per CU as registers and LDS allow;
                                   k in 2..8: at most k (each group reserves more LDS than it
                                   uses, 160 KiB / (k + 1) + 512 bytes) -- fewer waves per CU */
    double chunk_mm;
} ltm_tiling;

typedef struct ltm_plan ltm_plan;

uint32_t ltm_abi_version(void);
const char* ltm_last_error(void);

/* Validate the descriptors and build a plan (host memory only).  Errors:
 * LTM_ERR_INVALID for zero or too-small sizes, a detector that is not a
 * multiple of the lenslet count, non-positive focal lengths, radii or
 * distances, axes that are not a right-handed orthonormal frame, R > 64 or
 * S = 0. */
ltm_status ltm_plan_create(const ltm_grid* grid, const ltm_camera* cams, uint32_t n_cam,
                           ltm_plan** out);
void ltm_plan_destroy(ltm_plan* plan);

/* N = nx*ny*nz voxels and M = total pixels over all cameras. */
ltm_status ltm_plan_sizes(const ltm_plan* plan, uint64_t* n_voxels, uint64_t* n_meas);

/* Device workspace the plan needs (tile and brick tables), in bytes. */
ltm_status ltm_plan_workspace_bytes(const ltm_plan* plan, uint64_t* bytes);

/* Bind a caller-owned device workspace and fill its tables on `stream`.  The
 * workspace must stay valid while the plan is used.  Must be called before
 * ltm_project / ltm_backproject, and again after ltm_plan_set_tiling.
 * Cameras on their default tilings adapt the slab depth here: while more
 * than 1% of a tiling's slabs have voxel boxes too large for LDS, the slab
 * depth halves (at most three times; ltm_plan_get_tiling reports the
 * result), which reads the tables back and synchronizes `stream`.
 * Tilings set with ltm_plan_set_tiling are used as given. */
ltm_status ltm_plan_bind_workspace(ltm_plan* plan, void* ws, uint64_t bytes, void* stream);

ltm_status ltm_plan_get_tiling(const ltm_plan* plan, uint32_t direction, uint32_t camera,
                               ltm_tiling* out);
/* Replace one camera's tiling for one direction.  The plan becomes unbound:
 * query the workspace size and bind again. */
ltm_status ltm_plan_set_tiling(ltm_plan* plan, uint32_t direction, uint32_t camera,
                               const ltm_tiling* tiling);

/* Number of rays of one camera (over all pixels and angular samples) that are
 * unoccluded and cross the grid; each carries `samples` valid samples.  Uses
 * the plan's workspace and synchronizes the stream. */
ltm_status ltm_plan_valid_rays(ltm_plan* plan, uint32_t camera, uint64_t* rays, void* stream);

/* View subsets (the paper's view-subset acceleration): from now on project,
 * backproject and ltm_plan_valid_rays use only angular samples
 * r = ru + rays_u * rv with r mod n_subsets == index, averaged over the
 * subset -- the subset operator scaled by K/|S|.  n_subsets = 1 restores the
 * full operator.  The setting belongs to the plan (not thread-safe). */
ltm_status ltm_plan_set_ray_subset(ltm_plan* plan, uint32_t n_subsets, uint32_t index);

/* y = A x: ray integrals of the trilinear interpolant of x, averaged over
 * each pixel's angular samples (measurement-formation section; radiance as a
 * line integral through the object, object-model section).  x: N floats,
 * y: M floats (overwritten).  FP32 arithmetic, per-pixel sums in FP64. */
ltm_status ltm_project(ltm_plan* plan, const float* x, float* y, void* stream);

/* x = A^T y with the same samples and weights as ltm_project (the adjoint
 * the paper's adjoint-operations section requires).  y: M floats,
 * x: N floats (overwritten).  Each sample's eight weighted values are
 * rounded to FP32 and summed into an FP64 accumulator in the plan's
 * workspace, which is rounded to FP32 once at the end. */
ltm_status ltm_backproject(ltm_plan* plan, const float* y, float* x, void* stream);

/* For callers that cannot allocate device memory at the call (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * ltm_backproject with the FP64 accumulator taken from a fixed array the
 * library holds on each GPU (2^23 doubles = 64 MiB, reserved when the
 * library's code is loaded on that GPU and kept until the process ends)
 * instead of from the plan's workspace.  Same kernels, samples and weights,
 * so the same result as ltm_backproject.  The plan must still be bound (its
 * tile tables live in the workspace); y, x and the stream are as for
 * ltm_backproject, on the current device.  Errors: LTM_ERR_INVALID when the
 * plan has more than 2^23 = 8388608 voxels (checked before anything else
 * than the null arguments, with no device call), LTM_ERR_WORKSPACE when the
 * plan is unbound, LTM_ERR_DEVICE when the array's address cannot be read.
 * Allocates nothing: the first call on a GPU only looks the array's address
 * up.  Every call on one GPU shares that GPU's array; each call clears the
 * part it uses on its stream first, so calls ordered on one stream are
 * safe, while calls that overlap on one GPU (other streams, other threads)
 * race and give wrong results. */
ltm_status ltm_backproject_noalloc(ltm_plan* plan, const float* y, float* x, void* stream);

/* ---------------------------------------------------------------------- */
/* Tilings chosen by measurement (an addition to the paper's method, whose
 * own kernels had fixed shapes).  A tiling changes only how rays are grouped,
 * staged and summed, so any tiling whose output matches the current one may
 * be used.  For every camera and direction, ltm_autotune runs each candidate
 * on a one-camera copy of the plan (the full operator, whatever view subset
 * the plan is set to), on x (forward) or on the camera's block of y
 * (adjoint); a candidate whose output differs from the current tiling's by
 * more than 1e-6 relative L2 is rejected before it is timed.  The survivors
 * are timed with HIP events on `stream` (median of `reps` runs after one
 * untimed run).  Stage 1 searches tile size, lane order flags, slab depth
 * and brick size (ltm_autotune_candidates lists them); stage 2 tries
 * groups_per_cu = 2 and 3 on the three fastest.  The fastest passing tiling
 * (the current one if nothing beats it) is set on the plan.
 * cache_path (may be NULL): a text file of tilings keyed by GPU
 * architecture, grid and camera descriptor.  A camera found there runs only
 * its cached tiling, through the same parity gate, against the current one;
 * searched results are added to the file (written to path.tmp, then renamed).
 * ms (host, may be NULL): 4 doubles per camera -- forward best and current
 * ms, adjoint best and current ms.
 * Workspace: ltm_autotune_workspace_bytes (device, 256-byte aligned; the
 * plan's own workspace is not touched).  The plan must be bound; it is left
 * UNBOUND when any tiling changed -- query its workspace size and bind again.
 * Synchronizes the stream many times. */
ltm_status ltm_autotune_candidates(const ltm_plan* plan, uint32_t direction, uint32_t camera,
                                   ltm_tiling* out, uint32_t capacity, uint32_t* count);
ltm_status ltm_autotune_workspace_bytes(const ltm_plan* plan, uint64_t* bytes);
ltm_status ltm_autotune(ltm_plan* plan, const float* x, const float* y, void* ws, uint64_t bytes,
                        const char* cache_path, uint32_t reps, double* ms, void* stream);

/* ---------------------------------------------------------------------- */
/* Reconstruction: the paper's reconstruction-algorithm table (FISTA with a
 * diagonal majorizer) for
 *   min_{x>=0} sum_c 1/2 ||A_c x - g_c y_c||^2_{W_c} + nu ||x||_1 + R(x),
 * R(x) = beta/2 sum_j sum_{l in N_j} psi(x_j - x_l) over the 26 neighbours
 * present in the grid, psi(t) = t^2/2 or delta^2 (sqrt(1 + (t/delta)^2) - 1).
 * The majorizer is diag(sum_c A_c^T W_c A_c 1) + c_R beta (the paper uses
 * 26 beta; 36 is the largest eigenvalue of the 26-neighbour Laplacian),
 * with a zero step where it vanishes.  Gains g_1 = 1 and, when enabled,
 * g_c = y_c^T W_c p_c / y_c^T W_c y_c (c >= 2); otherwise all gains are 1.
 * Vectors are FP32; inner products, gains, the momentum scalar t and the
 * residual are FP64 on the device. */
enum { LTM_PSI_QUADRATIC = 0u, LTM_PSI_HYPERBOLA = 1u };

typedef struct ltm_solver_params {
    uint32_t momentum;          /* 1: FISTA, 0: projected gradient */
    uint32_t gains;             /* 1: estimate g_c for c >= 2 */
    uint32_t psi_kind;
    uint32_t n_subsets;         /* > 1: iteration n uses angular-sample subset n mod n_subsets
                                   (view-subset acceleration); the majorizer uses all samples */
    double beta, delta, nu, c_r;
    /* Stop rule of ltm_solver_solve (the algorithm table's loop runs for N_iter
     * iterations; a residual target ends it earlier): */
    double rho_target;          /* stop once rho(x) <= rho_target; 0 runs max_iter iterations */
    uint32_t max_iter;          /* N_iter: at most this many iterations per solve (>= 1) */
    uint32_t check_every;       /* iterations between residual checks, one host sync each (>= 1) */
} ltm_solver_params;

typedef struct ltm_solver ltm_solver;

/* Device workspace a solver needs: 4 volumes, 2 images and FP64 scalars. */
ltm_status ltm_solver_workspace_bytes(const ltm_plan* plan, uint64_t* bytes);

/* Create a solver on a bound plan.  y (M floats) and w (M floats, or NULL
 * for W = I) must stay valid while the solver is used.  Computes the
 * majorizer on `stream`.  The iterate starts at 0. */
ltm_status ltm_solver_create(ltm_plan* plan, const ltm_solver_params* params,
                             const float* y, const float* w, void* ws, uint64_t ws_bytes,
                             void* stream, ltm_solver** out);
void ltm_solver_destroy(ltm_solver* solver);

/* Restart from x0 (N floats on the device, or NULL for zero): x = z = x0,
 * t = 1, gains reset. */
ltm_status ltm_solver_reset(ltm_solver* solver, const float* x0, void* stream);

/* Restart from a candidate start x0 (N floats on the device, e.g. a learned
 * estimate of the volume), judged by the plain solver.  x0 is scaled by the
 * least-squares factor of its image, alpha = <A x0, y>_W / ||A x0||_W^2 (camera
 * 1 only when gains are estimated, since the other cameras' gains absorb any
 * scale), costing one projection.  At that scale rho(alpha x0)^2 = 1 - cos^2 of
 * the angle between A x0 and y (gains off), below rho(0) = 1 whenever the two
 * correlate positively.  The start is rejected -- the solver restarts from
 * x = 0 instead -- when x0 holds a non-finite value, when alpha is not finite
 * and positive (no positive correlation, or A x0 = 0), or when rho(alpha x0)
 * is not below 1.  Outputs (host, any may be NULL): alpha, rho(alpha x0) (1
 * when rejected) and accepted (1 or 0).
 * Synchronizes the stream.  x0 is only read. */
ltm_status ltm_solver_reset_warm(ltm_solver* solver, const float* x0, double* alpha, double* rho,
                                 uint32_t* accepted, void* stream);

/* Run n_iter iterations.  Asynchronous; no host synchronization. */
ltm_status ltm_solver_step(ltm_solver* solver, uint32_t n_iter, void* stream);

/* Run the algorithm from the current state until the stop rule of the
 * parameters: every check_every iterations the monitored residual (at the
 * extrapolated point) is read; once it is at or below rho_target the residual
 * of x itself is computed (one extra projection) and the solve stops when that
 * too is at or below the target.  Otherwise it stops after max_iter
 * iterations, reporting the residual of x.  Outputs (host): iterations run in
 * this call, converged (1 or 0) and rho(x).  Synchronizes once per check.
 * Returns LTM_ERR_NUMERIC as soon as a residual is not finite. */
ltm_status ltm_solver_solve(ltm_solver* solver, uint32_t* iterations, uint32_t* converged,
                            double* rho, void* stream);

/* Copy the current iterate x (N floats) into `x`. */
ltm_status ltm_solver_get_x(const ltm_solver* solver, float* x, void* stream);

/* Relative data residual of the last iteration, rho = ||p - g y||_W / ||g y||_W
 * with p = A z at that iteration's extrapolated point, and the iteration
 * count.  Synchronizes the stream.  Returns LTM_ERR_NUMERIC if rho is not
 * finite. */
ltm_status ltm_solver_residual(ltm_solver* solver, double* rho, uint32_t* iterations,
                               void* stream);

/* Relative data residual of the current iterate x itself (one extra
 * projection).  Synchronizes the stream. */
ltm_status ltm_solver_residual_x(ltm_solver* solver, double* rho, void* stream);

/* Checkpoint: copy the iterate x and the extrapolated point z (N floats
 * each, device) and return FISTA's t, the iteration count and the n_cam
 * current gains (host array, or NULL).  Synchronizes the stream. */
ltm_status ltm_solver_save(const ltm_solver* solver, float* x, float* z, double* t,
                           uint32_t* iterations, double* gains, void* stream);

/* Resume from a checkpoint written by ltm_solver_save (t >= 1).  Gains may be
 * NULL to keep the current ones.  Synchronizes the stream. */
ltm_status ltm_solver_load(ltm_solver* solver, const float* x, const float* z, double t,
                           uint32_t iterations, const double* gains, void* stream);

/* Gradient of R at z added into g:  g += beta sum_{l in N_j} psi'(z_j - z_l).
 * z, g: N floats on the device. */
ltm_status ltm_reg_grad_add(const ltm_grid* grid, uint32_t psi_kind, double beta, double delta,
                            const float* z, float* g, void* stream);

/* ---------------------------------------------------------------------- */
/* Batched sweeps.  Several bound plans -- for instance the time frames of a
 * sequence, each with its own grid size and cameras -- are projected by ONE
 * persistent launch and backprojected by another.  Each workgroup takes
 * (plan, camera, tile) items from a device counter, costliest first, so
 * uneven frames share the GPU without a launch per camera.  The sweep
 * allocates nothing, never synchronizes with the host and records no memset,
 * so it can be captured in a hipGraph (ltm_batch_graph_capture) and
 * replayed.  A batch records each member plan's tables, tilings, view
 * subset and workspace when it is created and bound: after any of them
 * changes (ltm_plan_set_tiling, ltm_plan_bind_workspace,
 * ltm_plan_set_ray_subset to another subset), ltm_batch_bind and every
 * launch entry point, graph launch included, return LTM_ERR_WORKSPACE
 * without launching; create the batch again. */
typedef struct ltm_batch ltm_batch;

ltm_status ltm_batch_create(ltm_plan* const* plans, uint32_t n_plans, ltm_batch** out);
void ltm_batch_destroy(ltm_batch* batch);
ltm_status ltm_batch_workspace_bytes(const ltm_batch* batch, uint64_t* bytes);

/* Bind a device workspace and, per plan k, its buffers: x_in[k] (N_k floats,
 * read by the forward), y[k] (M_k floats, written by the forward and read by
 * the adjoint) and x_out[k] (N_k floats, written by the adjoint).  The three
 * arguments are host arrays of n_plans device pointers.  Synchronizes. */
ltm_status ltm_batch_bind(ltm_batch* batch, void* ws, uint64_t bytes, const float* const* x_in,
                          float* const* y, float* const* x_out, void* stream);

/* y_k = A_k x_in_k for every plan. */
ltm_status ltm_batch_project(ltm_batch* batch, void* stream);
/* x_out_k = A_k^T y_k for every plan. */
ltm_status ltm_batch_backproject(ltm_batch* batch, void* stream);
/* Both, forward first. */
ltm_status ltm_batch_sweep(ltm_batch* batch, void* stream);

/* Capture one ltm_batch_sweep on `stream` (not the null stream) into a
 * graph owned by the batch; replay it with ltm_batch_graph_launch. */
ltm_status ltm_batch_graph_capture(ltm_batch* batch, void* stream);
ltm_status ltm_batch_graph_launch(ltm_batch* batch, void* stream);

/* ---------------------------------------------------------------------- */
/* Learned warm start: building blocks of a 3-D convolutional encoder-decoder
 * that maps A^T y to a starting volume for the solver (an addition to the
 * paper's method; the zero-start solver remains the reference).
 * Activations are BF16 channels-last [d][h][w][c] (uint16 storage); weights
 * keep an FP32 master copy [cout][taps * cin] (tap = dz*9 + dy*3 + dx,
 * offsets -1..1, ci fastest) packed to BF16 by ltm_nn_pack_weights.
 * Convolutions are "same" size with zero padding, run on MFMA with BF16
 * operands and FP32 accumulation.  All pointers are device pointers; every
 * call is asynchronous on `stream` and allocates nothing. */
typedef struct ltm_nn_conv {
    uint32_t ksize;       /* 1 or 3 */
    uint32_t d, h, w;     /* output grid */
    uint32_t c0, c1;      /* input channels read from in0, then in1 (concatenation); c1 may be 0.
                             Multiples of 8, or c0 = 1 alone */
    uint32_t cout;        /* output channels, <= 128 */
    uint32_t upsample;    /* 1: the input grid is the output grid halved (nearest 2x upsampling) */
    uint32_t relu;        /* 1: ReLU after the bias */
    uint32_t out_f32;     /* 1: FP32 outputs, else BF16 */
    uint32_t split;       /* output channels [0, split) -> out, [split, cout) -> out2 */
    uint32_t reserved;
} ltm_nn_conv;

/* Element counts of the two packed BF16 weight layouts of a layer. */
ltm_status ltm_nn_packed_sizes(uint32_t cout, uint32_t cin, uint32_t ksize, uint64_t* fwd_elems,
                               uint64_t* bwd_elems);
/* FP32 master weights -> packed forward (and, if w_bwd != NULL, input-gradient) BF16 layouts. */
ltm_status ltm_nn_pack_weights(const float* w, uint32_t cout, uint32_t cin, uint32_t ksize,
                               uint16_t* w_fwd, uint16_t* w_bwd, void* stream);
/* out = act(conv(concat(in0, in1)) + bias). */
ltm_status ltm_nn_conv3d_forward(const ltm_nn_conv* c, const uint16_t* in0, const uint16_t* in1,
                                 const uint16_t* w_fwd, const float* bias, void* out, void* out2,
                                 void* stream);
/* Input gradient of the conv described by c: dx0 (c0 channels) and dx1 (c1
 * channels) in FP32, from dy (BF16, the gradient at the pre-activation).
 * For an upsampling conv the result is on the output grid: reduce it with
 * ltm_nn_upsample2_backward. */
ltm_status ltm_nn_conv3d_dgrad(const ltm_nn_conv* c, const uint16_t* dy, const uint16_t* w_bwd,
                               float* dx0, float* dx1, void* stream);
/* dw += weight gradient (FP32 [cout][taps * cin]) from the layer input and dy. */
ltm_status ltm_nn_conv3d_wgrad(const ltm_nn_conv* c, const uint16_t* in0, const uint16_t* in1,
                               const uint16_t* dy, float* dw, void* stream);
/* 2x2x2 max pooling of a [d][h][w][c] grid; arg records the winning child. */
ltm_status ltm_nn_maxpool2(const uint16_t* x, uint16_t* y, uint8_t* arg, uint32_t d, uint32_t h,
                           uint32_t w, uint32_t c, void* stream);
/* dx += the pooled gradient routed to the winning children (dx on the fine grid). */
ltm_status ltm_nn_maxpool2_backward(const float* dy, const uint8_t* arg, float* dx, uint32_t d,
                                    uint32_t h, uint32_t w, uint32_t c, void* stream);
/* Backward of nearest 2x upsampling: d_low (= or +=) sum over each 2x2x2 block of d_high;
 * d, h, w are the fine grid. */
ltm_status ltm_nn_upsample2_backward(const float* d_high, float* d_low, uint32_t d, uint32_t h,
                                     uint32_t w, uint32_t c, uint32_t accumulate, void* stream);
/* g = d_out * (out > 0) (or d_out when relu = 0) as BF16; d_bias += per-channel sums (may be NULL). */
ltm_status ltm_nn_relu_backward(const float* d_out, const uint16_t* out, uint32_t relu, uint16_t* g,
                                float* d_bias, uint64_t n, uint32_t c, void* stream);
/* loss += mean((x - target)^2) (FP64 scalar), grad = 2 (x - target) / n. */
ltm_status ltm_nn_mse(const float* x, const float* target, float* grad, double* loss, uint64_t n,
                      void* stream);
/* One bias-corrected Adam step (step >= 1) on FP32 weights; g is cleared. */
ltm_status ltm_nn_adam(float* w, float* g, float* m, float* v, uint64_t n, double lr, double beta1,
                       double beta2, double eps, uint32_t step, void* stream);
/* y = x / max|x| as BF16 (the network input from A^T y); scratch: one uint32. */
ltm_status ltm_nn_prep_input(const float* x, uint16_t* y, uint32_t* scratch, uint64_t n, void* stream);
/* a += b (FP32). */
ltm_status ltm_nn_add(float* a, const float* b, uint64_t n, void* stream);

/* ------------------------------------------------------------------------ */
/* The paper's own discretization (light-field discretization, light
 * transport, object-model, camera-model and rotated-perspective sections;
 * Dirac and pillbox transport tables), for a single-lens camera at any
 * azimuth phi about the grid's y axis (e_t = +y), with the lens on the camera
 * axis through the grid centre.  With phi = 90 q + phi', |phi'| <= 45 deg (q
 * the nearest integer, half-way cases to even), the volume is first turned
 * by q quarter turns about y, an exact permutation of voxels that swaps the
 * x and z extents for odd q: the turned volume at p' is the volume at
 * R(90 q) p', R the rotation from camera to world axes.  A posed camera then
 * rotates the turned volume by phi' into its axes as the paper does, with
 * phi' in place of phi below: with c = cos phi the voxels scale
 * to (pitch/c, pitch, pitch c) along (s, t, depth), then a z shear
 * (z += -sin(phi) c x) and an x shear (x += tan(phi) z) resample the
 * coefficients, each the L2 projection of the sheared boxes (a piecewise
 * quadratic kernel); the rotated grid grows to nz' = nz + 2 ceil(|sin c| nx
 * / (2 c^2)) + 2 slices and to nx' = nx + 2 k + 2 columns, the least k whose
 * outermost column centre lies at least dx + |tan| dz / 2 beyond the volume's
 * rotated image (a column holding only zeros is left out; dx, dz the rotated
 * voxel sizes), and never more than nx + 2 ceil(|tan| nz' c^2 / 2) + 2.
 * The (rotated) volume is collapsed into its slices; slice iz at camera
 * depth z = distance + (iz + 1/2 - nz'/2) dz radiates the light field
 * dz * x[iz] for every angular cell.  The angular plane is the main
 * lens, divided into rays_u x rays_v cells (each 1..64) of size
 * 2 r_main / rays_* over its bounding square; cells whose centre lies
 * outside the lens disc are masked.  Each cell's transport is the Kronecker product of an s and a
 * t factor whose entries are the table's blur kernel integrated over the
 * source voxel; pixel i reads
 *   y_i = (dz / (K V^d)) sum_slices sum_cells [B_s (x) B_t] x_slice,
 * K = rays_u * rays_v, V^d the detector basis volume of the table (the
 * paper's sqrt(V^d) sum over cells replaced by the mean over cells, a global
 * scale).  A^T uses the same FP32 entries.  Accumulation is FP64 per output.
 * The library evaluates the entries in FP64 once, at bind time, into banded
 * FP32 tables in the workspace.
 *
 * A square-array plenoptic camera (LTM_PLENOPTIC, posed as above, the
 * volume rotated the same way) takes the paper's factorized plenoptic model
 * instead: every slice is transported
 * onto the lenslet-array plane (d_mla behind the main lens; array pixels of
 * the detector's pitch, det_nu / mla_nu per lenslet) per angular cell; the
 * aperture mask keeps array pixels whose centre lies inside their lenslet's
 * disc of radius r_mla (the occluder rasterized on the array grid), scaled by
 * 1 / V^a; each lenslet then transports its own pixels onto the detector
 * d_mla_det behind it (lenslet focal length f_mla).  The array stage is
 * separable per cell, so both stages are banded s and t factor tables.
 * y = norm sum_cells B^d_cell (mask . f^a_cell) / V^d with norm = d0s d0t /
 * ((d_mla + d_mla_det - d_mla d_mla_det / f_mla)^2 (2 r_mla / d_mla_det)^2):
 * the pixel integral over dp^2 times the solid angle of the lenslet's
 * bounding square.  Workspace: the tables plus three FP32 intermediates,
 * nz * rays_v * det_nv * nx (slices filtered along t), cells * det_nv *
 * det_nu (the masked array-plane light field), and the same again (after
 * the lenslet t stage), plus the two rotated volumes of a posed camera and
 * the turned volume when q != 0. */
enum { LTM_BASIS_DIRAC = 0u, LTM_BASIS_PILLBOX = 1u };

typedef struct ltm_xport ltm_xport;

ltm_status ltm_xport_create(const ltm_grid* grid, const ltm_camera* camera, uint32_t basis,
                            ltm_xport** out);
void ltm_xport_destroy(ltm_xport* t);
/* Workspace for the banded tables and the nz * rays_v * det_nv * nx FP32
 * intermediate of the two filtering passes (plenoptic: the three above). */
ltm_status ltm_xport_workspace_bytes(const ltm_xport* t, uint64_t* bytes);
/* Binds caller-owned device memory (>= workspace_bytes, 256-byte aligned)
 * and uploads the tables; synchronizes the stream. */
ltm_status ltm_xport_bind_workspace(ltm_xport* t, void* workspace, uint64_t bytes, void* stream);
/* y (det_nv x det_nu) = A x; x[nz][ny][nx]. */
ltm_status ltm_xport_project(ltm_xport* t, const float* x, float* y, void* stream);
/* x = A^T y (overwrites x). */
ltm_status ltm_xport_backproject(ltm_xport* t, const float* y, float* x, void* stream);
/* Band widths of the four tables: t-factor rows, s-factor rows (cells of
 * one row summed), and their transposes; for the plenoptic model those of
 * the slice-to-array stage (t, s, s transposed, t transposed). */
ltm_status ltm_xport_bands(const ltm_xport* t, uint32_t bands[4]);

#ifdef __cplusplus
}
#endif
#endif /* LTM_H */
