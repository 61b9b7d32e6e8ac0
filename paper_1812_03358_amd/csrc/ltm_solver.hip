// gfx950 kernels of the reconstruction algorithm (the paper's
// reconstruction-algorithm table: FISTA with a diagonal majorizer) and of the
// edge-preserving regularizer gradient.  Vectors are FP32; inner products,
// gains, the momentum scalar t and the data residual are FP64 on the device,
// so an iteration never waits for the host.
#include "ltm_internal.h"
#include "ltm_solver.h"

namespace ltm {

namespace {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Per-camera sums over the image: sum W p^2 and sum W y p (FP64).  One block
// handles a contiguous range of one camera's pixels; block sums are added
// into the scalar slots with FP64 atomics.
__global__ __launch_bounds__(kRedThreads) void k_reduce(const float* __restrict__ p,
                                                        const float* __restrict__ y,
                                                        const float* __restrict__ w,
                                                        const uint64_t* __restrict__ cam_off,
                                                        int n_cam, int blocks_per_cam,
                                                        double* __restrict__ sc)
{
    __shared__ double red[2][kRedThreads / 64];
    const int cam = blockIdx.x / blocks_per_cam;
    const int part = blockIdx.x % blocks_per_cam;
    const uint64_t lo = cam_off[cam], hi = cam_off[cam + 1];
    double spp = 0.0, syp = 0.0;
    for (uint64_t i = lo + (uint64_t)part * kRedThreads + threadIdx.x; i < hi;
         i += (uint64_t)blocks_per_cam * kRedThreads) {
        const double wi = w ? (double)w[i] : 1.0;
        const double pi = (double)p[i];
        spp += wi * pi * pi;
        syp += wi * (double)y[i] * pi;
    }
    spp = wave_sum(spp);
    syp = wave_sum(syp);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = spp;
        red[1][wave] = syp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < kRedThreads / 64; ++k) {
            a += red[0][k];
            b += red[1][k];
        }
        unsafeAtomicAdd(&sc[SC_CAM + SC_PP * n_cam + cam], a);
        unsafeAtomicAdd(&sc[SC_CAM + SC_YP * n_cam + cam], b);
    }
}

// sum W y^2 per camera (once, at creation).
__global__ __launch_bounds__(kRedThreads) void k_reduce_yy(const float* __restrict__ y,
                                                           const float* __restrict__ w,
                                                           const uint64_t* __restrict__ cam_off,
                                                           int n_cam, int blocks_per_cam,
                                                           double* __restrict__ sc)
{
    __shared__ double red[kRedThreads / 64];
    const int cam = blockIdx.x / blocks_per_cam;
    const int part = blockIdx.x % blocks_per_cam;
    const uint64_t lo = cam_off[cam], hi = cam_off[cam + 1];
    double s = 0.0;
    for (uint64_t i = lo + (uint64_t)part * kRedThreads + threadIdx.x; i < hi;
         i += (uint64_t)blocks_per_cam * kRedThreads) {
        const double wi = w ? (double)w[i] : 1.0;
        s += wi * (double)y[i] * (double)y[i];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int k = 0; k < kRedThreads / 64; ++k) a += red[k];
        unsafeAtomicAdd(&sc[SC_CAM + SC_YY * n_cam + cam], a);
    }
}

// Clear the per-iteration sums.
__global__ void k_scalars_clear(double* sc, int n_cam)
{
    for (int k = threadIdx.x; k < n_cam; k += blockDim.x) {
        sc[SC_CAM + SC_PP * n_cam + k] = 0.0;
        sc[SC_CAM + SC_YP * n_cam + k] = 0.0;
    }
}

// Gains, residual and the momentum scalars of one iteration (one thread).
//   g_1 = 1; g_c = (y_c^T W p_c) / (y_c^T W y_c) for c >= 2 when gains are on.
//   rho^2 = sum_c ||p_c - g_c y_c||_W^2 / sum_c ||g_c y_c||_W^2
//   t+ = (1 + sqrt(1 + 4 t^2)) / 2, momentum (t - 1) / t+ (0 without FISTA).
__global__ void k_scalars_step(double* sc, int n_cam, int gains, int momentum)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double num = 0.0, den = 0.0;
    for (int c = 0; c < n_cam; ++c) {
        const double pp = sc[SC_CAM + SC_PP * n_cam + c];
        const double yp = sc[SC_CAM + SC_YP * n_cam + c];
        const double yy = sc[SC_CAM + SC_YY * n_cam + c];
        double g = 1.0;
        if (gains && c > 0) g = yy > 0.0 ? yp / yy : 0.0;
        sc[SC_CAM + SC_GAMMA * n_cam + c] = g;
        num += pp - 2.0 * g * yp + g * g * yy;
        den += g * g * yy;
    }
    if (num < 0.0) num = 0.0;   // cancellation at a tiny residual
    if (!isfinite(num) || !isfinite(den))
        sc[SC_RHO] = __builtin_nan("");   // non-finite data or iterate: reported to the host
    else
        sc[SC_RHO] = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
    const double t = sc[SC_T];
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    sc[SC_MOM] = momentum ? (t - 1.0) / tn : 0.0;
    sc[SC_T] = tn;
    sc[SC_ITER] += 1.0;
}

// Residual of the iterate x itself (gains re-estimated for p = A x).
__global__ void k_scalars_rho_x(double* sc, int n_cam, int gains)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double num = 0.0, den = 0.0;
    for (int c = 0; c < n_cam; ++c) {
        const double pp = sc[SC_CAM + SC_PP * n_cam + c];
        const double yp = sc[SC_CAM + SC_YP * n_cam + c];
        const double yy = sc[SC_CAM + SC_YY * n_cam + c];
        double g = 1.0;
        if (gains && c > 0) g = yy > 0.0 ? yp / yy : 0.0;
        num += pp - 2.0 * g * yp + g * g * yy;
        den += g * g * yy;
    }
    if (num < 0.0) num = 0.0;
    if (!isfinite(num) || !isfinite(den))
        sc[SC_RHOX] = __builtin_nan("");
    else
        sc[SC_RHOX] = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
}

// r = W (p - g_c y) on every camera's pixels.
__global__ void k_residual(const float* __restrict__ p, const float* __restrict__ y,
                           const float* __restrict__ w, const uint64_t* __restrict__ cam_off,
                           int n_cam, const double* __restrict__ sc, float* __restrict__ r,
                           uint64_t M)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int c = 0;
        while (c + 1 < n_cam && i >= cam_off[c + 1]) ++c;
        const float g = (float)sc[SC_CAM + SC_GAMMA * n_cam + c];
        float v = p[i] - g * y[i];
        if (w) v *= w[i];
        r[i] = v;
    }
}

// Majorizer inverse: dinv = 1 / (D + c_R beta), 0 where that vanishes.
__global__ void k_dinv(float* __restrict__ d, uint64_t n, float add)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float v = d[i] + add;
        d[i] = v > 0.0f ? 1.0f / v : 0.0f;
    }
}

// w = [z - dinv g]_+,  x+ = [w - nu]_+,  z+ = x+ + mom (x+ - x).
__global__ void k_update(float* __restrict__ x, float* __restrict__ z,
                         const float* __restrict__ g, const float* __restrict__ dinv,
                         const double* __restrict__ sc, float nu, uint64_t n)
{
    const float mom = (float)sc[SC_MOM];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float zi = z[i];
        const float wv = fmaxf(fmaf(-dinv[i], g[i], zi), 0.0f);
        const float xn = fmaxf(wv - nu, 0.0f);
        const float xo = x[i];
        x[i] = xn;
        z[i] = fmaf(mom, xn - xo, xn);
    }
}

__global__ void k_copy(float* __restrict__ dst, const float* __restrict__ src, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_mul(float* __restrict__ a, const float* __restrict__ w, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        a[i] *= w[i];
}

// dst = a * src.
__global__ void k_scale_copy(float* __restrict__ dst, const float* __restrict__ src, float a, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = a * src[i];
}

// Number of non-finite values of v, added into *count (FP64 slot; one atomic
// per block).
__global__ __launch_bounds__(kRedThreads) void k_nonfinite(const float* __restrict__ v, uint64_t n,
                                                           double* __restrict__ count)
{
    __shared__ unsigned int red[kRedThreads / 64];
    unsigned int c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kRedThreads)
        c += isfinite(v[i]) ? 0u : 1u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int t = 0;
        for (int k = 0; k < kRedThreads / 64; ++k) t += red[k];
        if (t) unsafeAtomicAdd(count, (double)t);
    }
}

__global__ void k_slot_zero(double* slot) { if (threadIdx.x == 0 && blockIdx.x == 0) *slot = 0.0; }

__global__ void k_scalars_reset(double* sc, int n_cam, int gains)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc[SC_T] = 1.0;
    sc[SC_MOM] = 0.0;
    sc[SC_RHO] = INFINITY;
    sc[SC_ITER] = 0.0;
    for (int c = 0; c < n_cam; ++c)
        sc[SC_CAM + SC_GAMMA * n_cam + c] = (c == 0 || !gains) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- regularizer
// g_j += beta sum_{l in N_j} psi'(z_j - z_l) over the 26 neighbours inside the
// grid.  A block owns an 8 x 8 x 4 voxel tile and stages it with a one-voxel
// halo in LDS (voxels outside the grid are flagged absent).
constexpr int RX = 8, RY = 8, RZ = 4;

__device__ __forceinline__ float dpsi(float t, int kind, float inv_delta2)
{
    if (kind == LTM_PSI_QUADRATIC) return t;
    return t * rsqrtf(fmaf(t * t, inv_delta2, 1.0f));
}

__global__ __launch_bounds__(RX* RY* RZ) void k_reg_grad(const float* __restrict__ z,
                                                         float* __restrict__ g, int nx, int ny,
                                                         int nz, int kind, float beta,
                                                         float inv_delta2)
{
    __shared__ float tile[RZ + 2][RY + 2][RX + 2];
    const int bx = blockIdx.x * RX, by = blockIdx.y * RY, bz = blockIdx.z * RZ;
    const int tid = threadIdx.x;
    const float absent = __builtin_nanf("");
    for (int e = tid; e < (RX + 2) * (RY + 2) * (RZ + 2); e += RX * RY * RZ) {
        const int lx = e % (RX + 2), ly = (e / (RX + 2)) % (RY + 2), lz = e / ((RX + 2) * (RY + 2));
        const int gx = bx + lx - 1, gy = by + ly - 1, gz = bz + lz - 1;
        float v = absent;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
            v = z[(size_t)gx + (size_t)nx * ((size_t)gy + (size_t)ny * gz)];
        tile[lz][ly][lx] = v;
    }
    __syncthreads();
    const int lx = tid % RX, ly = (tid / RX) % RY, lz = tid / (RX * RY);
    const int gx = bx + lx, gy = by + ly, gz = bz + lz;
    if (gx >= nx || gy >= ny || gz >= nz) return;
    const float zc = tile[lz + 1][ly + 1][lx + 1];
    float acc = 0.0f;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                if (dx == 1 && dy == 1 && dz == 1) continue;
                const float zl = tile[lz + dz][ly + dy][lx + dx];
                if (zl == zl) acc += dpsi(zc - zl, kind, inv_delta2);   // skip absent
            }
    const size_t j = (size_t)gx + (size_t)nx * ((size_t)gy + (size_t)ny * gz);
    g[j] = fmaf(beta, acc, g[j]);
}

unsigned grid1(uint64_t n)
{
    uint64_t b = (n + 255) / 256;
    return (unsigned)(b > 16384 ? 16384 : (b ? b : 1));
}

}  // namespace

hipError_t launch_reg_grad(const ltm_grid& gr, int kind, double beta, double delta, const float* z,
                           float* g, hipStream_t s)
{
    dim3 grid((gr.nx + RX - 1) / RX, (gr.ny + RY - 1) / RY, (gr.nz + RZ - 1) / RZ);
    const float inv_d2 = delta > 0 ? (float)(1.0 / (delta * delta)) : 0.0f;
    hipLaunchKernelGGL(k_reg_grad, grid, dim3(RX * RY * RZ), 0, s, z, g, (int)gr.nx, (int)gr.ny,
                       (int)gr.nz, kind, (float)beta, inv_d2);
    return hipGetLastError();
}

hipError_t solver_launch_reduce(const SolverDev& d, const float* p, hipStream_t s)
{
    hipLaunchKernelGGL(k_scalars_clear, dim3(1), dim3(64), 0, s, d.sc, d.n_cam);
    hipLaunchKernelGGL(k_reduce, dim3(d.n_cam * d.blocks_per_cam), dim3(kRedThreads), 0, s, p, d.y,
                       d.w, d.cam_off, d.n_cam, d.blocks_per_cam, d.sc);
    return hipGetLastError();
}

hipError_t solver_launch_yy(const SolverDev& d, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_yy, dim3(d.n_cam * d.blocks_per_cam), dim3(kRedThreads), 0, s, d.y,
                       d.w, d.cam_off, d.n_cam, d.blocks_per_cam, d.sc);
    return hipGetLastError();
}

hipError_t solver_launch_scalars(const SolverDev& d, hipStream_t s)
{
    hipLaunchKernelGGL(k_scalars_step, dim3(1), dim3(64), 0, s, d.sc, d.n_cam, d.gains, d.momentum);
    return hipGetLastError();
}

hipError_t solver_launch_rho_x(const SolverDev& d, hipStream_t s)
{
    hipLaunchKernelGGL(k_scalars_rho_x, dim3(1), dim3(64), 0, s, d.sc, d.n_cam, d.gains);
    return hipGetLastError();
}

hipError_t solver_launch_residual(const SolverDev& d, const float* p, float* r, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, dim3(grid1(d.M)), dim3(256), 0, s, p, d.y, d.w, d.cam_off,
                       d.n_cam, d.sc, r, d.M);
    return hipGetLastError();
}

hipError_t solver_launch_update(const SolverDev& d, float nu, hipStream_t s)
{
    hipLaunchKernelGGL(k_update, dim3(grid1(d.N)), dim3(256), 0, s, d.x, d.z, d.g, d.dinv, d.sc, nu,
                       d.N);
    return hipGetLastError();
}

hipError_t solver_launch_dinv(const SolverDev& d, float add, hipStream_t s)
{
    hipLaunchKernelGGL(k_dinv, dim3(grid1(d.N)), dim3(256), 0, s, d.dinv, d.N, add);
    return hipGetLastError();
}

hipError_t solver_launch_reset(const SolverDev& d, hipStream_t s)
{
    hipLaunchKernelGGL(k_scalars_reset, dim3(1), dim3(64), 0, s, d.sc, d.n_cam, d.gains);
    return hipGetLastError();
}

hipError_t launch_copy(float* dst, const float* src, uint64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(grid1(n)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_scale_copy(float* dst, const float* src, float a, uint64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_copy, dim3(grid1(n)), dim3(256), 0, s, dst, src, a, n);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* v, uint64_t n, double* count, hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_zero, dim3(1), dim3(64), 0, s, count);
    hipLaunchKernelGGL(k_nonfinite, dim3(grid1(n)), dim3(kRedThreads), 0, s, v, n, count);
    return hipGetLastError();
}

hipError_t launch_mul(float* a, const float* w, uint64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_mul, dim3(grid1(n)), dim3(256), 0, s, a, w, n);
    return hipGetLastError();
}

}  // namespace ltm
