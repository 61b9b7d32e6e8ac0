// Internal types shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ltm.h"

namespace ltm {

constexpr int kThreads = 256;      // workgroup size of every ray kernel
constexpr int kMaxRays = 64;       // R limit per pixel
constexpr int kMaxBrickFloats = 16384;  // brick words (4 bytes)
constexpr int kMaxLdsBytes = 65536;     // dynamic LDS of one march workgroup
constexpr int kLdsPerCu = 163840;       // LDS of one gfx950 compute unit
constexpr int kMaxRayList = 8192;       // valid rays one workgroup may own
// voxels of the fixed FP64 accumulator behind ltm_backproject_noalloc
constexpr uint64_t kScratchVoxels = uint64_t(1) << 23;

// Per-tile record: camera depth (relative to the anchor plane) where the
// tile's first slab starts, and its number of slabs.
struct TileRec {
    float z_start;
    int n_chunks;
};

// Per-(tile, slab) record: voxel box [lo, lo + dim) staged in LDS, or
// lds == 0 when it does not fit (the slab then reads/writes global memory).
struct BrickRec {
    int lo[3];
    int dim[3];
    int lds;
    float base;   // lo.x + dim.x * (lo.y + dim.y * lo.z): flat index of lo
};

// Everything a kernel needs about one camera, in FP32 except the FP64
// main-aperture test.  Built on the host in FP64 and rounded once.
//
// A ray of pixel (iu, iv), angular sample (ru, rv) is written with
//   cu = lenslet index + 1/2 - mu/2, du = pixel index + 1/2 - nu/2,
//   g  = (2 ru + 1)/Ru - 1 (aperture grid cell centre in [-1, 1]);
// its lateral position on the anchor plane (the camera-depth plane through
// the grid centre) and its slope after the main lens are linear in them:
//   sigma = Ac cu + Ad du + Ag g,   slope = Bc cu + Bd du + Bg g,
// and likewise for t with (cv, dv, g_t).  In voxel-index coordinates the
// ray is q(z') = qA + z' dq with z' the camera depth relative to the anchor,
//   qA = CA + sigma Es + tau Et,   dq = slope_s Es + slope_t Et + Ez.
//
// Hexagonal plenoptic cameras also loop over the 3 x 3 lenslets around each
// pixel: rv runs over 9 grv (lenslet-major), the angular grid is ru x grv,
// cu/cv are the visited lenslet's position in pitches (s) and row spacings
// (t), Ac/Bc/Lc and Act/Bct/Lct scale them, and the g terms depend on the
// lenslet's type (hAg, hBg, hLg).  For the other kinds grv = rv, Act = Ac,
// Bct = Bc and Lct = Lc.
struct CamDev {
    int kind, nu, nv, mu, mv, ku, kv, ru, rv, S;
    int grv;              // angular-grid rows (rv / 9 for hexagonal cameras)
    int n[3];
    float Ac, Ad, Ag, Bc, Bd, Bg;
    float Act, Bct;
    float hAg[3], hBg[3];
    float rowf, colf;     // hexagonal: pixel pitch / row spacing, pixel pitch / lenslet pitch
    int hmu, hmv, hmid;   // hexagonal: lenslets per row, rows, mla_nv / 2 (unshifted row parity)
    float CA[3], Es[3], Et[3], Ez[3];
    float zlo;            // lens plane: z' >= zlo
    float invR;
    float inv_ru, inv_rv;
    int need_aperture;    // plenoptic: FP64 main-lens test per ray
    double Lc, Ld, Lg, r2;  // main-lens crossing s_L = Lc cu + Ld du + Lg g; r_main^2
    double Lct, hLg[3];
    // tiling
    int tile_u, tile_v, order, splits;
    int rotate;           // lanes start their aperture-sample loop at lane mod R
    int adj_f32;          // adjoint: FP32 LDS brick (flushed into the FP64 accumulator)
    int skew;             // adjoint: lanes start their sample walk at staggered offsets
    int merge;            // adjoint: merge consecutive samples of one cell in registers
    int window;           // adjoint: two planes of corner sums along the ray's dominant axis
    int groups_per_cu;    // 0, or the most workgroups one CU may hold (LDS reservation)
    int sub_n, sub_i;     // angular-sample subset: keep r with r mod sub_n == sub_i
    int items, items_per_split, tiles_u, tiles_v, n_tiles;
    int brick_cap;        // LDS brick capacity in voxels (FP32 forward, FP64 adjoint)
    int max_chunks;
    float chunk;
    const TileRec* tiles;
    const BrickRec* bricks;
    uint64_t y_off;
};

// One (plan, camera) of a batch: its constants and the buffers it reads and
// writes (x: the plan's input volume, y: its image block, xacc: the plan's
// FP64 adjoint accumulator).
struct BatchCam {
    CamDev cam;
    const float* x;
    float* y;
    double* xacc;
};
constexpr int kTileBits = 20;   // work item = (batch camera << 20) | tile

struct CamHost {
    ltm_camera desc;
    ltm_tiling tiling[2];
    CamDev dev;                 // constants without table pointers / tiling
    uint64_t npix;
    uint64_t y_off;
    // workspace offsets (bytes) of this camera's tables, per direction
    uint64_t tiles_off[2], bricks_off[2];
    int n_tiles[2], max_chunks[2];
    // default tilings adapt their slab depth at bind time (down to
    // chunk_floor, which sizes the brick table); explicit tilings do not
    bool adapt[2];
    double chunk_floor[2];
};

}  // namespace ltm

struct ltm_plan {
    ltm_grid grid;
    std::vector<ltm::CamHost> cams;
    uint64_t n_vox = 0, n_meas = 0;
    uint64_t ws_bytes = 0;
    uint64_t counter_off = 0;   // 256-byte scratch word for ltm_plan_valid_rays
    uint64_t accum_off = 0;     // N doubles: FP64 accumulator of the adjoint
    uint32_t sub_n = 1, sub_i = 0;   // current angular-sample subset
    char* ws = nullptr;
    bool bound = false;
    // bumped whenever the tables a launch reads may change (tiling, workspace
    // binding), so that batches built on the plan can detect it
    uint64_t generation = 0;
};

namespace ltm {

// error reporting (thread-local message)
ltm_status fail(ltm_status s, const std::string& msg);
ltm_status hip_fail(hipError_t e, const char* what);
void clear_error();

// descriptor checks shared by every operator built from grid and cameras
ltm_status validate_cameras(const ltm_grid* g, const ltm_camera* cams, uint32_t n_cam);

// kernel launchers (ltm_project.hip)
hipError_t launch_setup(const CamDev& c, int dir, hipStream_t s);
hipError_t launch_project(const CamDev& c, const float* x, float* y, hipStream_t s);
hipError_t launch_backproject(const CamDev& c, const float* y, double* x, hipStream_t s);
hipError_t launch_fill64(double* p, uint64_t n, hipStream_t s);
// device address of the current GPU's fixed accumulator (kScratchVoxels doubles)
hipError_t scratch_accumulator(double** out);
hipError_t launch_to_f32(const double* a, float* b, uint64_t n, hipStream_t s);
// out[0] = sum (a - b)^2, out[1] = sum b^2 in FP64 (out: 2 doubles, cleared first)
hipError_t launch_diff_sumsq(const float* a, const float* b, uint64_t n, double* out, hipStream_t s);
hipError_t launch_fill(float* p, uint64_t n, float v, hipStream_t s);
hipError_t launch_count(const CamDev& c, unsigned long long* counter, hipStream_t s);
size_t march_lds_bytes(const CamDev& c, int dir);
hipError_t launch_batch(const BatchCam* cams, const uint32_t* items, uint32_t n_items,
                        unsigned int* counter, int dir, int blocks, size_t lds, hipStream_t s);
int batch_blocks_per_cu(int dir, size_t lds);

// tiling limits (ltm_plan.cpp); sets the error message on failure
ltm_status check_tiling(const ltm_grid& g, const ltm_camera& c, const ltm_tiling& t);

// the camera's constants with the tables of one direction bound
CamDev bound_dev(const ltm_plan* p, const CamHost& c, int dir);

}  // namespace ltm
