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

hipError_t launch_xport_project(const XportDev& d, const float* x, float* y, hipStream_t s);
hipError_t launch_xport_backproject(const XportDev& d, const float* y, float* x, hipStream_t s);

}  // namespace ltm
