// Light-field transport operator (the paper's Dirac / pillbox transport for a
// head-on single-lens camera) as separable filtering passes on gfx950.
//
// Forward, per (slice iz, angular row kt):
//   minor pass  M[iz][kt][v][ix] = sum_iy Bt(iz,kt)[v][iy] x[iz][iy][ix]
//   major pass  y[v][u]          = sum_{iz,kt} sum_ix Cs(iz,kt)[u][ix] M[iz][kt][v][ix]
// where Cs(iz,kt) is the sum of the s factors of the row's unmasked cells
// (the cells of one angular row share their t factor).  The adjoint runs the
// transposed tables in the opposite order.  Every output has one writer
// (no atomics): the minor passes write one intermediate value per thread and
// the major passes accumulate a whole output in FP64 registers.
#include <algorithm>

#include "ltm_xport.h"

namespace ltm {

namespace {

constexpr int kBlock = 256;
constexpr int kRowsPerThread = 1;   // forward major pass: detector rows per thread

// M[p][v][ix] = sum_k bt.w[p][k][v] * x[iz][start + k][ix],  p = iz * kt + kt_i
__global__ __launch_bounds__(kBlock) void k_minor_fwd(XportDev d, const float* __restrict__ x)
{
    const size_t total = (size_t)d.nz * d.kt * d.nv * d.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ix = (int)(i % d.nx);
        const size_t r = i / d.nx;
        const int v = (int)(r % d.nv);
        const size_t p = r / d.nv;
        const size_t iz = p / d.kt;
        const int st = d.bt.start[p * d.nv + v];
        const float* w = d.bt.w + p * d.bt.width * (size_t)d.nv + v;
        const float* xs = x + iz * d.ny * (size_t)d.nx + ix;
        float acc = 0.0f;
        for (int k = 0; k < d.bt.width; ++k) {
            const int iy = st + k;
            if (iy < d.ny) acc = fmaf(w[(size_t)k * d.nv], xs[(size_t)iy * d.nx], acc);
        }
        d.mid[i] = acc;
    }
}

// y[v][u] for kRowsPerThread consecutive rows v of one column u.
__global__ __launch_bounds__(kBlock) void k_major_fwd(XportDev d, float* __restrict__ y)
{
    const int vblocks = (d.nv + kRowsPerThread - 1) / kRowsPerThread;
    const size_t total = (size_t)vblocks * d.nu;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int u = (int)(i % d.nu);
        const int v0 = (int)(i / d.nu) * kRowsPerThread;
        double acc[kRowsPerThread];
#pragma unroll
        for (int r = 0; r < kRowsPerThread; ++r) acc[r] = 0.0;
        const size_t pairs = (size_t)d.nz * d.kt;
        for (size_t p = 0; p < pairs; ++p) {
            const int st = d.cs.start[p * d.nu + u];
            const float* w = d.cs.w + p * d.cs.width * (size_t)d.nu + u;
            const float* m = d.mid + p * d.nv * (size_t)d.nx;
            for (int k = 0; k < d.cs.width; ++k) {
                const int ix = st + k;
                if (ix >= d.nx) break;
                const float c = w[(size_t)k * d.nu];
#pragma unroll
                for (int r = 0; r < kRowsPerThread; ++r)
                    if (v0 + r < d.nv) acc[r] += (double)(c * m[(size_t)(v0 + r) * d.nx + ix]);
            }
        }
#pragma unroll
        for (int r = 0; r < kRowsPerThread; ++r)
            if (v0 + r < d.nv) y[(size_t)(v0 + r) * d.nu + u] = (float)acc[r];
    }
}

// Same as k_major_fwd (one row per thread) with the band width fixed at
// compile time: the padded weights are zero, so the column index is clamped
// instead of tested, and the pair loop unrolls so that the independent table
// and intermediate loads of several pairs are in flight together.
template <int W>
__global__ __launch_bounds__(kBlock) void k_major_fwd_w(XportDev d, float* __restrict__ y)
{
    const size_t total = (size_t)d.nv * d.nu;
    const size_t pairs = (size_t)d.nz * d.kt;
    const size_t pstride = (size_t)d.nv * d.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int u = (int)(i % d.nu);
        const int v = (int)(i / d.nu);
        const float* mrow = d.mid + (size_t)v * d.nx;
        double acc = 0.0;
#pragma unroll 4
        for (size_t p = 0; p < pairs; ++p) {
            const int st = d.cs.start[p * d.nu + u];
            const float* w = d.cs.w + p * W * (size_t)d.nu + u;
            const float* m = mrow + p * pstride;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int ix = min(st + k, d.nx - 1);
                acc += (double)(w[(size_t)k * d.nu] * m[ix]);
            }
        }
        y[i] = (float)acc;
    }
}

// Same as k_major_adj with the loop bound fixed at compile time (W >= the
// table's width; the terms past the width are skipped).
template <int W>
__global__ __launch_bounds__(kBlock) void k_major_adj_w(XportDev d, const float* __restrict__ y)
{
    const size_t total = (size_t)d.nz * d.kt * d.nv * d.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ix = (int)(i % d.nx);
        const size_t r = i / d.nx;
        const int v = (int)(r % d.nv);
        const size_t p = r / d.nv;
        const int wd = d.cst.width;
        const int st = d.cst.start[p * d.nx + ix];
        const float* w = d.cst.w + p * wd * (size_t)d.nx + ix;
        const float* yr = y + (size_t)v * d.nu;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (k < wd) {
                const int u = min(st + k, d.nu - 1);
                acc += (double)(w[(size_t)k * d.nx] * yr[u]);
            }
        }
        d.mid[i] = (float)acc;
    }
}

// Adjoint major pass with the image rows staged in LDS: a workgroup takes
// `rows` detector rows (staged once, coalesced) and a chunk of (slice, row)
// pairs; a thread holds one (pair, voxel column)'s band weights in registers
// and applies them to every staged row.  The image gathers hit LDS instead
// of scattered global loads.  W >= the table's width (terms past it skipped).
template <int W>
__global__ __launch_bounds__(kBlock) void k_major_adj_lds(XportDev d, const float* __restrict__ y,
                                                          int rows, int pchunk)
{
    extern __shared__ float ys[];
    const int v0 = blockIdx.x * rows;
    const int nr = min(rows, d.nv - v0);
    for (int i = threadIdx.x; i < nr * d.nu; i += kBlock) ys[i] = y[(size_t)v0 * d.nu + i];
    __syncthreads();
    const size_t pairs = (size_t)d.nz * d.kt;
    const size_t pb = (size_t)blockIdx.y * pchunk;
    const size_t pe = pb + pchunk < pairs ? pb + pchunk : pairs;
    const int wd = d.cst.width;
    const size_t items = (pe - pb) * d.nx;
    for (size_t it = threadIdx.x; it < items; it += kBlock) {
        const size_t p = pb + it / d.nx;
        const int ix = (int)(it % d.nx);
        const int st = d.cst.start[p * d.nx + ix];
        const float* wp = d.cst.w + p * wd * (size_t)d.nx + ix;
        float w[W];
        int col[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            w[k] = k < wd ? wp[(size_t)k * d.nx] : 0.0f;
            col[k] = min(st + k, d.nu - 1);
        }
        float* out = d.mid + (p * d.nv + v0) * (size_t)d.nx + ix;
        for (int r = 0; r < nr; ++r) {
            const float* yr = ys + r * d.nu;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (k < wd) acc += (double)(w[k] * yr[col[k]]);
            out[(size_t)r * d.nx] = (float)acc;
        }
    }
}

// M[p][v][ix] = sum_k cst.w[p][k][ix] * y[v][start + k]
__global__ __launch_bounds__(kBlock) void k_major_adj(XportDev d, const float* __restrict__ y)
{
    const size_t total = (size_t)d.nz * d.kt * d.nv * d.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ix = (int)(i % d.nx);
        const size_t r = i / d.nx;
        const int v = (int)(r % d.nv);
        const size_t p = r / d.nv;
        const int st = d.cst.start[p * d.nx + ix];
        const float* w = d.cst.w + p * d.cst.width * (size_t)d.nx + ix;
        const float* yr = y + (size_t)v * d.nu;
        double acc = 0.0;
        for (int k = 0; k < d.cst.width; ++k) {
            const int u = st + k;
            if (u < d.nu) acc += (double)(w[(size_t)k * d.nx] * yr[u]);
        }
        d.mid[i] = (float)acc;
    }
}

// x[iz][iy][ix] = sum_kt sum_k btt.w[p][k][iy] * M[p][start + k][ix]
__global__ __launch_bounds__(kBlock) void k_minor_adj(XportDev d, float* __restrict__ x)
{
    const size_t total = (size_t)d.nz * d.ny * d.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ix = (int)(i % d.nx);
        const size_t r = i / d.nx;
        const int iy = (int)(r % d.ny);
        const size_t iz = r / d.ny;
        double acc = 0.0;
        for (int kt = 0; kt < d.kt; ++kt) {
            const size_t p = iz * d.kt + kt;
            const int st = d.btt.start[p * d.ny + iy];
            const float* w = d.btt.w + p * d.btt.width * (size_t)d.ny + iy;
            const float* m = d.mid + p * d.nv * (size_t)d.nx + ix;
            for (int k = 0; k < d.btt.width; ++k) {
                const int v = st + k;
                if (v < d.nv) acc += (double)(w[(size_t)k * d.ny] * m[(size_t)v * d.nx]);
            }
        }
        x[i] = (float)acc;
    }
}

// ---------------------------------------------------------------- shears
// r1[z][y][x1] = sum_k ez.w[x1][k][z] * x[start + k][y][x1]
__global__ __launch_bounds__(kBlock) void k_shear_z(ShearDev r, const float* __restrict__ x)
{
    const size_t total = (size_t)r.nz * r.ny * r.nx1;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int x1 = (int)(i % r.nx1);
        const size_t q = i / r.nx1;
        const int y = (int)(q % r.ny);
        const int z = (int)(q / r.ny);
        const int st = r.ez.start[(size_t)x1 * r.nz + z];
        const float* w = r.ez.w + (size_t)x1 * r.ez.width * r.nz + z;
        double acc = 0.0;
        for (int k = 0; k < r.ez.width; ++k) {
            const int zs = st + k;
            if (zs < r.nz1) acc += (double)(w[(size_t)k * r.nz] * x[((size_t)zs * r.ny + y) * r.nx1 + x1]);
        }
        r.r1[i] = (float)acc;
    }
}

// xr[z][y][x] = sum_k ex.w[z][k][x] * r1[z][y][start + k]
__global__ __launch_bounds__(kBlock) void k_shear_x(ShearDev r)
{
    const size_t total = (size_t)r.nz * r.ny * r.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int x = (int)(i % r.nx);
        const size_t q = i / r.nx;
        const int z = (int)(q / r.ny);
        const int st = r.ex.start[(size_t)z * r.nx + x];
        const float* w = r.ex.w + (size_t)z * r.ex.width * r.nx + x;
        const float* row = r.r1 + q * r.nx1;
        double acc = 0.0;
        for (int k = 0; k < r.ex.width; ++k) {
            const int xs = st + k;
            if (xs < r.nx1) acc += (double)(w[(size_t)k * r.nx] * row[xs]);
        }
        r.xr[i] = (float)acc;
    }
}

// r1[z][y][x1] = sum_k ext.w[z][k][x1] * xr[z][y][start + k]
__global__ __launch_bounds__(kBlock) void k_shear_x_t(ShearDev r)
{
    const size_t total = (size_t)r.nz * r.ny * r.nx1;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int x1 = (int)(i % r.nx1);
        const size_t q = i / r.nx1;
        const int z = (int)(q / r.ny);
        const int st = r.ext.start[(size_t)z * r.nx1 + x1];
        const float* w = r.ext.w + (size_t)z * r.ext.width * r.nx1 + x1;
        const float* row = r.xr + q * r.nx;
        double acc = 0.0;
        for (int k = 0; k < r.ext.width; ++k) {
            const int xs = st + k;
            if (xs < r.nx) acc += (double)(w[(size_t)k * r.nx1] * row[xs]);
        }
        r.r1[i] = (float)acc;
    }
}

// x[z1][y][x1] = sum_k ezt.w[x1][k][z1] * r1[start + k][y][x1]
__global__ __launch_bounds__(kBlock) void k_shear_z_t(ShearDev r, float* __restrict__ x)
{
    const size_t total = (size_t)r.nz1 * r.ny * r.nx1;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int x1 = (int)(i % r.nx1);
        const size_t q = i / r.nx1;
        const int y = (int)(q % r.ny);
        const int z1 = (int)(q / r.ny);
        const int st = r.ezt.start[(size_t)x1 * r.nz1 + z1];
        const float* w = r.ezt.w + (size_t)x1 * r.ezt.width * r.nz1 + z1;
        double acc = 0.0;
        for (int k = 0; k < r.ezt.width; ++k) {
            const int zs = st + k;
            if (zs < r.nz) acc += (double)(w[(size_t)k * r.nz1] * r.r1[((size_t)zs * r.ny + y) * r.nx1 + x1]);
        }
        x[i] = (float)acc;
    }
}

unsigned grid_for(size_t n)
{
    const size_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}

}  // namespace

hipError_t launch_xport_project(const XportDev& d, const float* x, float* y, hipStream_t s)
{
    const size_t nm = (size_t)d.nz * d.kt * d.nv * d.nx;
    hipLaunchKernelGGL(k_minor_fwd, dim3(grid_for(nm)), dim3(kBlock), 0, s, d, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t ny = (size_t)((d.nv + kRowsPerThread - 1) / kRowsPerThread) * d.nu;
    const dim3 g(grid_for(ny)), b(kBlock);
    switch (d.cs.width) {
    case 1: hipLaunchKernelGGL(k_major_fwd_w<1>, g, b, 0, s, d, y); break;
    case 2: hipLaunchKernelGGL(k_major_fwd_w<2>, g, b, 0, s, d, y); break;
    case 3: hipLaunchKernelGGL(k_major_fwd_w<3>, g, b, 0, s, d, y); break;
    case 4: hipLaunchKernelGGL(k_major_fwd_w<4>, g, b, 0, s, d, y); break;
    default: hipLaunchKernelGGL(k_major_fwd, g, b, 0, s, d, y); break;
    }
    return hipGetLastError();
}

hipError_t launch_shear_forward(const ShearDev& r, const float* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_shear_z, dim3(grid_for((size_t)r.nz * r.ny * r.nx1)), dim3(kBlock), 0, s, r, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_shear_x, dim3(grid_for((size_t)r.nz * r.ny * r.nx)), dim3(kBlock), 0, s, r);
    return hipGetLastError();
}

hipError_t launch_shear_adjoint(const ShearDev& r, float* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_shear_x_t, dim3(grid_for((size_t)r.nz * r.ny * r.nx1)), dim3(kBlock), 0, s, r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_shear_z_t, dim3(grid_for((size_t)r.nz1 * r.ny * r.nx1)), dim3(kBlock), 0, s, r, x);
    return hipGetLastError();
}

hipError_t launch_xport_backproject(const XportDev& d, const float* y, float* x, hipStream_t s)
{
    const size_t nm = (size_t)d.nz * d.kt * d.nv * d.nx;
    const dim3 g(grid_for(nm)), b(kBlock);
    const int rows = std::min(16, 16384 / std::max(1, d.nu));     // <= 64 KiB of staged rows
    const size_t pairs = (size_t)d.nz * d.kt;
    const int pchunk = 32;
    const dim3 gl((unsigned)((d.nv + rows - 1) / std::max(1, rows)),
                  (unsigned)((pairs + pchunk - 1) / pchunk));
    const size_t lds = (size_t)std::max(1, rows) * d.nu * sizeof(float);
    if (rows >= 1 && gl.y < 65536 && d.cst.width <= 8)
        hipLaunchKernelGGL(k_major_adj_lds<8>, gl, b, lds, s, d, y, rows, pchunk);
    else if (rows >= 1 && gl.y < 65536 && d.cst.width <= 16)
        hipLaunchKernelGGL(k_major_adj_lds<16>, gl, b, lds, s, d, y, rows, pchunk);
    else if (rows >= 1 && gl.y < 65536 && d.cst.width <= 24)
        hipLaunchKernelGGL(k_major_adj_lds<24>, gl, b, lds, s, d, y, rows, pchunk);
    else if (d.cst.width <= 24)
        hipLaunchKernelGGL(k_major_adj_w<24>, g, b, 0, s, d, y);
    else
        hipLaunchKernelGGL(k_major_adj, g, b, 0, s, d, y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t nx = (size_t)d.nz * d.ny * d.nx;
    hipLaunchKernelGGL(k_minor_adj, dim3(grid_for(nx)), dim3(kBlock), 0, s, d, x);
    return hipGetLastError();
}

}  // namespace ltm
