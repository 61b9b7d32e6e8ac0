// Solver state shared by the host code and the solver kernels.
#pragma once

#include "ltm_internal.h"

namespace ltm {

// FP64 scalar slots in device memory
enum {
    SC_T = 0,       // FISTA t
    SC_MOM = 1,     // (t - 1) / t+ of the last iteration
    SC_RHO = 2,     // relative data residual at the last iteration's z
    SC_ITER = 3,    // iterations done
    SC_RHOX = 4,    // relative data residual at x (ltm_solver_residual_x)
    SC_BAD = 5,     // non-finite values of a candidate start (ltm_solver_reset_warm)
    SC_CAM = 8      // per-camera arrays follow, n_cam entries each:
};
enum { SC_PP = 0, SC_YP = 1, SC_YY = 2, SC_GAMMA = 3, SC_NCAMARR = 4 };

struct SolverDev {
    float *x, *z, *g, *dinv, *p, *r;
    const float *y, *w;
    double* sc;
    uint64_t* cam_off;        // n_cam + 1 image offsets
    int n_cam, blocks_per_cam, gains, momentum;
    uint64_t N, M;
};

hipError_t launch_reg_grad(const ltm_grid& g, int kind, double beta, double delta, const float* z,
                           float* out, hipStream_t s);
hipError_t solver_launch_reduce(const SolverDev& d, const float* p, hipStream_t s);
hipError_t solver_launch_yy(const SolverDev& d, hipStream_t s);
hipError_t solver_launch_scalars(const SolverDev& d, hipStream_t s);
hipError_t solver_launch_rho_x(const SolverDev& d, hipStream_t s);
hipError_t solver_launch_residual(const SolverDev& d, const float* p, float* r, hipStream_t s);
hipError_t solver_launch_update(const SolverDev& d, float nu, hipStream_t s);
hipError_t solver_launch_dinv(const SolverDev& d, float add, hipStream_t s);
hipError_t solver_launch_reset(const SolverDev& d, hipStream_t s);
hipError_t launch_copy(float* dst, const float* src, uint64_t n, hipStream_t s);
hipError_t launch_mul(float* a, const float* w, uint64_t n, hipStream_t s);
hipError_t launch_scale_copy(float* dst, const float* src, float a, uint64_t n, hipStream_t s);
hipError_t launch_count_nonfinite(const float* v, uint64_t n, double* count, hipStream_t s);

}  // namespace ltm

struct ltm_solver {
    ltm_plan* plan = nullptr;
    ltm_solver_params prm{};
    ltm::SolverDev d{};
    std::vector<uint64_t> cam_off;
    uint32_t iter = 0;        // host count of iterations (selects the view subset)
};
