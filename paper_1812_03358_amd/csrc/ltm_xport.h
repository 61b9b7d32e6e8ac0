// Internal types of the light-field transport operator (the paper's own
// discretization): banded FP32 factor tables and the filtering launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ltm {

// One banded table family: for each of `pairs` (slice, angular row) pairs and
// each of `rows` output rows, the first nonzero column `start` and `width`
// weights stored weight-major: w[(pair * width + k) * rows + row] multiplies
// column start + k (zero padded past the band).
struct BandDev {
    const int32_t* start;
    const float* w;
    int rows, width;
};

struct XportDev {
    int nx, ny, nz, nu, nv, kt;   // grid, detector, angular rows
    BandDev bt;    // t factor:      rows = detector rows,    columns = voxel rows (y)
    BandDev cs;    // s factor sum:  rows = detector columns, columns = voxel columns (x)
    BandDev cst;   // transpose of cs: rows = voxel columns,  columns = detector columns
    BandDev btt;   // transpose of bt: rows = voxel rows,     columns = detector rows
    float* mid;    // nz * kt * nv * nx intermediate
};

// Rotation of the volume into a posed camera's axes (scaling plus two
// shears, each an L2-projected 1-D resampling): natural grid (nz1, ny, nx1)
// -> z-sheared (nz, ny, nx1) -> x-sheared (nz, ny, nx), the transport's grid.
struct ShearDev {
    int nx1, nz1, nx, ny, nz;
    BandDev ez;    // per natural column x1: rows = sheared z,  columns = natural z
    BandDev ezt;   // transpose:             rows = natural z,  columns = sheared z
    BandDev ex;    // per sheared row z:     rows = rotated x,  columns = natural x
    BandDev ext;   // transpose:             rows = natural x,  columns = rotated x
    float* r1;     // z-sheared volume
    float* xr;     // rotated volume
};

// Factorized plenoptic transport (square lenslet array): slices -> array
// plane per angular cell, the aperture mask, then each lenslet -> detector.
// Cells are listed row by row (kt outer); cell_first[kt] .. cell_first[kt+1]
// are the active cells of angular row kt.
struct PlenDev {
    int nx, ny, nz;          // grid
    int na_u, na_v;          // array-plane pixels
    int nu, nv;              // detector
    int ks, kt, cells;       // angular columns, rows, active cells
    int row_cells_max;       // most active cells in one angular row
    const int32_t* cell_ks;
    const int32_t* cell_kt;
    const int32_t* cell_first;
    BandDev bt1;   // per (slice, kt): rows = array rows,    columns = voxel rows
    BandDev bs1;   // per (slice, ks): rows = array columns, columns = voxel columns (x dz)
    BandDev bt2;   // per kt:          rows = detector rows, columns = array rows
    BandDev bs2;   // per ks:          rows = detector cols, columns = array columns (x norm / V^d)
    BandDev bt1t, bs1t, bt2t, bs2t;   // transposes
    const float* mask;       // array pixel inside its lenslet's disc, / V^a
    float* m1;               // [slice][kt][array row][x]
    float* fa;               // [cell][array row][array col]
    float* m2;               // [cell][detector row][array col]
};

hipError_t launch_plen_project(const PlenDev& d, const float* x, float* y, hipStream_t s);
hipError_t launch_plen_backproject(const PlenDev& d, const float* y, float* x, hipStream_t s);

hipError_t launch_xport_project(const XportDev& d, const float* x, float* y, hipStream_t s);
hipError_t launch_xport_backproject(const XportDev& d, const float* y, float* x, hipStream_t s);
hipError_t launch_shear_forward(const ShearDev& r, const float* x, hipStream_t s);
hipError_t launch_shear_adjoint(const ShearDev& r, float* x, hipStream_t s);
// q quarter turns about y of a volume on the grid (nz, ny, nx): dst on the
// turned grid (nx, ny, nz for odd q), dst(p') = src(R(90 q) p').
hipError_t launch_turn(const float* src, float* dst, int nx, int ny, int nz, int q, hipStream_t s);

}  // namespace ltm
