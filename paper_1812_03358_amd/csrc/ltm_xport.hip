// Light-field transport operator (the paper's Dirac / pillbox transport for a
// head-on single-lens camera) as separable filtering passes on gfx950.
//
// Forward, per (slice iz, angular row kt):
//   minor pass  M[iz][kt][v][ix] = sum_iy Bt(iz,kt)[v][iy] x[iz][iy][ix]
//   major pass  y[v][u]          = sum_{iz,kt} sum_ix Cs(iz,kt)[u][ix] M[iz][kt][v][ix]
// where Cs(iz,kt) is the sum of the s factors of the row's unmasked cells
// (the cells of one angular row share their t factor).  The adjoint runs the
// transposed tables in the opposite order.  Every output has one writer
// (no atomics): a minor-pass thread writes its own intermediate values and a
// major-pass thread accumulates whole outputs in FP64 registers.
//
// A posed camera wraps these passes in quarter turns of the volume and the
// rotation's z and x shears; the
// factorized plenoptic model chains two such separable stages (slices onto
// the lenslet-array plane, the mask, each lenslet onto the detector).
#include <algorithm>

#include "ltm_xport.h"

namespace ltm {

namespace {

constexpr int kBlock = 256;
constexpr int kRowsPerThread = 1;   // forward major pass: detector rows per thread

// Row kernels: grid y walks the output rows (the row's coordinates, band
// start and weights are then uniform across the workgroup and decoded once),
// threads the row's columns.
struct RowGrid {
    dim3 g, b;
};

RowGrid row_grid(size_t rows, int cols)
{
    const int bs = cols >= kBlock ? kBlock : ((cols + 63) / 64) * 64;
    const unsigned gx = (unsigned)((cols + bs - 1) / bs);
    const unsigned gy = (unsigned)(rows < 65535 ? (rows ? rows : 1) : 65535);
    return {dim3(gx, gy), dim3((unsigned)bs)};
}

constexpr int kMinorRows = 8;   // minor passes: output rows per thread

// mid[p][v][ix] = sum_k bt.w[p][k][v] * x[iz][start + k][ix], p = (iz, kt):
// a thread takes column ix of kMinorRows consecutive rows v of one pair, so
// that the rows' table and volume loads are in flight together; each output
// is still summed over k in order.
__global__ __launch_bounds__(kBlock) void k_minor_fwd(XportDev d, const float* __restrict__ x)
{
    constexpr int R = kMinorRows;
    const int ix = blockIdx.x * blockDim.x + threadIdx.x;
    if (ix >= d.nx) return;
    const int vb = (d.nv + R - 1) / R;
    const size_t groups = (size_t)d.nz * d.kt * vb;
    for (size_t g = blockIdx.y; g < groups; g += gridDim.y) {
        const int v0 = (int)(g % vb) * R;
        const size_t p = g / vb;
        const size_t iz = p / d.kt;
        const float* xs = x + iz * d.ny * (size_t)d.nx + ix;
        const int32_t* st = d.bt.start + p * d.nv;
        const float* w = d.bt.w + p * d.bt.width * (size_t)d.nv;
        int s0[R];
        float acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            s0[r] = st[min(v0 + r, d.nv - 1)];
            acc[r] = 0.0f;
        }
        for (int k = 0; k < d.bt.width; ++k) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int iy = s0[r] + k;
                if (iy < d.ny)
                    acc[r] = fmaf(w[(size_t)k * d.nv + min(v0 + r, d.nv - 1)], xs[(size_t)iy * d.nx], acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (v0 + r < d.nv) d.mid[(p * d.nv + v0 + r) * d.nx + ix] = acc[r];
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

// R consecutive floats of an LDS row group (16-, 8- or 4-byte aligned).
template <int R>
__device__ __forceinline__ void lds_rows(const float* p, float (&v)[R])
{
    if constexpr (R % 4 == 0) {
#pragma unroll
        for (int i = 0; i < R; i += 4) {
            const float4 q = *reinterpret_cast<const float4*>(p + i);
            v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
        }
    } else if constexpr (R == 2) {
        const float2 q = *reinterpret_cast<const float2*>(p);
        v[0] = q.x; v[1] = q.y;
    } else {
        v[0] = p[0];
    }
}

constexpr int kBlockF = 1024;   // LDS-staged major passes: 16 waves share one staged block
constexpr int kGroup = 4;       // plenoptic stage 1: terms of kGroup slices summed in FP32, then in FP64

// k_major_fwd with the intermediate staged in LDS: a workgroup of kBlockF
// threads takes R detector rows and kBlockF detector columns; per chunk of zc
// (slice, angular row) pairs it stages the R rows of every pair once
// (coalesced; the R rows of one voxel column adjacent so one LDS read serves
// all R; W - 1 zero columns past the last so the band needs no clamp), and a
// thread applies its column's band weights, loaded once per pair, to the R
// staged rows.  Each product is rounded to FP32 and summed in FP64, as in
// the adjoint's passes, so that A and A^T round the same products alike.
// W is the table's width.
template <int R, int W>
__global__ __launch_bounds__(kBlockF) void k_major_fwd_lds(XportDev d, float* __restrict__ y, int zc)
{
    extern __shared__ float4 ms4[];
    float* ms = reinterpret_cast<float*>(ms4);             // [pair of the chunk][nx + W - 1][R]
    const int nvb = (d.nv + R - 1) / R;
    const int v0 = (blockIdx.x % nvb) * R;
    const int u = (blockIdx.x / nvb) * kBlockF + threadIdx.x;
    const bool live = u < d.nu;
    const int nr = min(R, d.nv - v0);
    const int pairs = d.nz * d.kt;
    const int pitch = (d.nx + W - 1) * R;                  // floats per staged pair
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    const int lane = threadIdx.x & 63;
    for (int p0 = 0; p0 < pairs; p0 += zc) {
        const int npc = min(zc, pairs - p0);
        __syncthreads();                                   // the previous chunk is consumed
        // one wave per staged row, lanes along it; loads from clamped (valid)
        // addresses, then a select, so a wave's loads are in flight together
        for (int row = threadIdx.x >> 6; row < npc * R; row += kBlockF / 64) {
            const int p = row / R, r = row % R;
            const float* src = d.mid + ((size_t)(p0 + p) * d.nv + v0 + min(r, nr - 1)) * d.nx;
            float* dst = ms + p * pitch + r;
#pragma unroll 4
            for (int ix = lane; ix < d.nx + W - 1; ix += 64) {
                const float v = src[min(ix, d.nx - 1)];
                dst[ix * R] = r < nr && ix < d.nx ? v : 0.0f;
            }
        }
        __syncthreads();
        if (!live) continue;
#pragma unroll 4
        for (int p = 0; p < npc; ++p) {
            // 32-bit table offsets (the launcher checks the tables' sizes)
            const int pp = p0 + p;
            const int s0 = d.cs.start[pp * d.nu + u];
            const int wo = pp * W * d.nu + u;
            const float* mz = ms + p * pitch + s0 * R;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const float wk = d.cs.w[wo + k * d.nu];
                float m[R];
                lds_rows<R>(mz + k * R, m);
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += (double)(wk * m[r]);
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nr) y[(size_t)(v0 + r) * d.nu + u] = (float)acc[r];
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
// of scattered global loads.  W >= the table's width (terms past it
// skipped).
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

// x[iz][iy][ix] = sum_kt sum_k btt.w[p][k][iy] * M[p][start + k][ix]:
// angular rows four at a time, each with its own FP64 partial sum, so that
// their table and intermediate loads are in flight together.
__global__ __launch_bounds__(kBlock) void k_minor_adj(XportDev d, float* __restrict__ x)
{
    constexpr int G = 4;
    const size_t total = (size_t)d.nz * d.ny * d.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ix = (int)(i % d.nx);
        const size_t r = i / d.nx;
        const int iy = (int)(r % d.ny);
        const size_t iz = r / d.ny;
        double acc = 0.0;
        for (int kt0 = 0; kt0 < d.kt; kt0 += G) {
            int st[G];
            const float* w[G];
            const float* m[G];
            double part[G];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                // rows past the last repeat it with no terms (st = nv)
                const bool live = kt0 + j < d.kt;
                const size_t p = iz * d.kt + (live ? kt0 + j : d.kt - 1);
                st[j] = live ? d.btt.start[p * d.ny + iy] : d.nv;
                w[j] = d.btt.w + p * d.btt.width * (size_t)d.ny + iy;
                m[j] = d.mid + p * d.nv * (size_t)d.nx + ix;
                part[j] = 0.0;
            }
            for (int k = 0; k < d.btt.width; ++k) {
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int v = st[j] + k;
                    if (v < d.nv) part[j] += (double)(w[j][(size_t)k * d.ny] * m[j][(size_t)v * d.nx]);
                }
            }
            acc += (part[0] + part[1]) + (part[2] + part[3]);
        }
        x[i] = (float)acc;
    }
}

// ---------------------------------------------------------------- shears
// r1[z][y][x1] = sum_k ez.w[x1][k][z] * x[start + k][y][x1]
__global__ __launch_bounds__(kBlock) void k_shear_z(ShearDev r, const float* __restrict__ x)
{
    const int x1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (x1 >= r.nx1) return;
    const size_t rows = (size_t)r.nz * r.ny;
    for (size_t q = blockIdx.y; q < rows; q += gridDim.y) {
        const size_t i = q * r.nx1 + x1;
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
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= r.nx) return;
    const size_t rows = (size_t)r.nz * r.ny;
    for (size_t q = blockIdx.y; q < rows; q += gridDim.y) {
        const size_t i = q * r.nx + x;
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
    const int x1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (x1 >= r.nx1) return;
    const size_t rows = (size_t)r.nz * r.ny;
    for (size_t q = blockIdx.y; q < rows; q += gridDim.y) {
        const size_t i = q * r.nx1 + x1;
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
    const int x1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (x1 >= r.nx1) return;
    const size_t rows = (size_t)r.nz1 * r.ny;
    for (size_t q = blockIdx.y; q < rows; q += gridDim.y) {
        const size_t i = q * r.nx1 + x1;
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

// ---------------------------------------------------------------- quarter turns
// dst on the turned grid, dst(p') = src(R(90 q) p') with R the rotation about
// y.  With the natural grid (nz, ny, nx): q = 1 reads src[nz-1-x'][y][z'],
// q = 3 reads src[x'][y][nx-1-z'] (x and z extents swap), q = 2 reads
// src[nz-1-z'][y][nx-1-x'].  Odd turns transpose each y plane through a
// padded LDS tile so that reads and writes both run along rows.
constexpr int kTurn = 32;

__global__ __launch_bounds__(256) void k_turn_odd(const float* __restrict__ src, float* __restrict__ dst,
                                                  int nx, int ny, int nz, int q)
{
    __shared__ float tile[kTurn][kTurn + 1];
    const int nxq = nz, nzq = nx;                       // turned grid
    const int b0 = blockIdx.x * kTurn, a0 = blockIdx.y * kTurn, y = blockIdx.z;
    const int tx = threadIdx.x & (kTurn - 1), ty = threadIdx.x / kTurn;
    // tile[b][a] = dst[a0 + a][b0 + b]: lanes walk a, a source row
    for (int k = ty; k < kTurn; k += 256 / kTurn) {
        const int a = a0 + tx, b = b0 + k;
        if (a < nzq && b < nxq) {
            const int zs = q == 1 ? nz - 1 - b : b;
            const int xs = q == 1 ? a : nx - 1 - a;
            tile[k][tx] = src[((size_t)zs * ny + y) * nx + xs];
        }
    }
    __syncthreads();
    // lanes walk b, a destination row
    for (int k = ty; k < kTurn; k += 256 / kTurn) {
        const int a = a0 + k, b = b0 + tx;
        if (a < nzq && b < nxq) dst[((size_t)a * ny + y) * nxq + b] = tile[tx][k];
    }
}

__global__ __launch_bounds__(kBlock) void k_turn_half(const float* __restrict__ src, float* __restrict__ dst,
                                                      int nx, int ny, int nz)
{
    const size_t total = (size_t)nz * ny * nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int x = (int)(i % nx);
        const size_t r = i / nx;
        const int y = (int)(r % ny);
        const int z = (int)(r / ny);
        dst[i] = src[((size_t)(nz - 1 - z) * ny + y) * nx + (nx - 1 - x)];
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
    {
        const RowGrid rg = row_grid((size_t)d.nz * d.kt * ((d.nv + kMinorRows - 1) / kMinorRows), d.nx);
        hipLaunchKernelGGL(k_minor_fwd, rg.g, rg.b, 0, s, d, x);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // LDS-staged pass for band widths up to 4 while 4 rows of one pair fit 64 KiB
    {
        constexpr int R = 4;
        const int w = std::max(1, d.cs.width);
        const int zc = 65536 / ((d.nx + w - 1) * R * (int)sizeof(float));
        const int nvb = (d.nv + R - 1) / R, nub = (d.nu + kBlockF - 1) / kBlockF;
        const size_t lds = (size_t)std::max(1, zc) * (d.nx + w - 1) * R * sizeof(float);
        const dim3 gs((unsigned)((size_t)nvb * nub)), bf(kBlockF);
        if (zc >= 1 && d.cs.width <= 4 && (size_t)d.nz * d.kt * d.cs.width * d.nu < (1u << 31)) {
            switch (d.cs.width) {
            case 1: hipLaunchKernelGGL((k_major_fwd_lds<R, 1>), gs, bf, lds, s, d, y, zc); break;
            case 2: hipLaunchKernelGGL((k_major_fwd_lds<R, 2>), gs, bf, lds, s, d, y, zc); break;
            case 3: hipLaunchKernelGGL((k_major_fwd_lds<R, 3>), gs, bf, lds, s, d, y, zc); break;
            default: hipLaunchKernelGGL((k_major_fwd_lds<R, 4>), gs, bf, lds, s, d, y, zc); break;
            }
            return hipGetLastError();
        }
    }
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

hipError_t launch_turn(const float* src, float* dst, int nx, int ny, int nz, int q, hipStream_t s)
{
    q = ((q % 4) + 4) % 4;
    if (q == 0)
        return hipMemcpyAsync(dst, src, (size_t)nx * ny * nz * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (q == 2) {
        hipLaunchKernelGGL(k_turn_half, dim3(grid_for((size_t)nx * ny * nz)), dim3(kBlock), 0, s,
                           src, dst, nx, ny, nz);
    } else {
        if (ny > 65535 || (nx + kTurn - 1) / kTurn > 65535) return hipErrorInvalidValue;
        const dim3 g((unsigned)((nz + kTurn - 1) / kTurn), (unsigned)((nx + kTurn - 1) / kTurn), (unsigned)ny);
        hipLaunchKernelGGL(k_turn_odd, g, dim3(256), 0, s, src, dst, nx, ny, nz, q);
    }
    return hipGetLastError();
}

hipError_t launch_shear_forward(const ShearDev& r, const float* x, hipStream_t s)
{
    {
        const RowGrid rg = row_grid((size_t)r.nz * r.ny, r.nx1);
        hipLaunchKernelGGL(k_shear_z, rg.g, rg.b, 0, s, r, x);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const RowGrid rg = row_grid((size_t)r.nz * r.ny, r.nx);
        hipLaunchKernelGGL(k_shear_x, rg.g, rg.b, 0, s, r);
    }
    return hipGetLastError();
}

hipError_t launch_shear_adjoint(const ShearDev& r, float* x, hipStream_t s)
{
    {
        const RowGrid rg = row_grid((size_t)r.nz * r.ny, r.nx1);
        hipLaunchKernelGGL(k_shear_x_t, rg.g, rg.b, 0, s, r);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const RowGrid rg = row_grid((size_t)r.nz1 * r.ny, r.nx1);
        hipLaunchKernelGGL(k_shear_z_t, rg.g, rg.b, 0, s, r, x);
    }
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
    hipLaunchKernelGGL(k_minor_adj, dim3(grid_for((size_t)d.nz * d.ny * d.nx)), dim3(kBlock), 0, s, d, x);
    return hipGetLastError();
}


// ------------------------------------------------ factorized plenoptic model
namespace {

__device__ __forceinline__ double band_dot(const BandDev& b, size_t tab, int row, const float* src,
                                           size_t stride, int ncols)
{
    const int st = b.start[tab * b.rows + row];
    const float* w = b.w + tab * b.width * (size_t)b.rows + row;
    double acc = 0.0;
    for (int k = 0; k < b.width; ++k) {
        const int c = st + k;
        if (c < ncols) acc += (double)(w[(size_t)k * b.rows] * src[(size_t)c * stride]);
    }
    return acc;
}

// FA[c][va][ua] = mask[va][ua] * sum_iz sum_k bs1[iz, ks_c][ua][k] M1[iz][kt_c][va][st + k]
__global__ __launch_bounds__(kBlock) void k_pl_major1(PlenDev d)
{
    const size_t total = (size_t)d.cells * d.na_v * d.na_u;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ua = (int)(i % d.na_u);
        const size_t q = i / d.na_u;
        const int va = (int)(q % d.na_v);
        const int c = (int)(q / d.na_v);
        const int ks = d.cell_ks[c], kt = d.cell_kt[c];
        double acc = 0.0;
        for (int iz = 0; iz < d.nz; ++iz) {
            const float* row = d.m1 + (((size_t)iz * d.kt + kt) * d.na_v + va) * d.nx;
            acc += band_dot(d.bs1, (size_t)iz * d.ks + ks, ua, row, 1, d.nx);
        }
        d.fa[i] = (float)acc * d.mask[(size_t)va * d.na_u + ua];
    }
}

// k_pl_major1 with the table width W fixed at compile time and the slice
// loop unrolled, so the loads of several slices are in flight together.
template <int W>
__global__ __launch_bounds__(kBlock) void k_pl_major1_w(PlenDev d)
{
    const size_t total = (size_t)d.cells * d.na_v * d.na_u;
    const size_t zstride = (size_t)d.kt * d.na_v * d.nx;
    const size_t sstride = (size_t)d.ks * d.na_u;             // start: next slice
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ua = (int)(i % d.na_u);
        const size_t q = i / d.na_u;
        const int va = (int)(q % d.na_v);
        const int c = (int)(q / d.na_v);
        const int ks = d.cell_ks[c], kt = d.cell_kt[c];
        const float* row = d.m1 + ((size_t)kt * d.na_v + va) * d.nx;
        const int32_t* st = d.bs1.start + (size_t)ks * d.na_u + ua;
        const float* w = d.bs1.w + (size_t)ks * W * d.na_u + ua;
        double acc = 0.0;
#pragma unroll 8
        for (int iz = 0; iz < d.nz; ++iz) {
            const int s0 = st[iz * sstride];
            const float* wz = w + iz * sstride * W;
            const float* rz = row + iz * zstride;
#pragma unroll
            for (int k = 0; k < W; ++k)
                acc += (double)(wz[(size_t)k * d.na_u] * rz[min(s0 + k, d.nx - 1)]);
        }
        d.fa[i] = (float)acc * d.mask[(size_t)va * d.na_u + ua];
    }
}


// k_pl_major1 with the intermediate staged in LDS: a workgroup of kBlockF
// threads takes R array rows of one angular row kt and kBlockF output columns
// of that row (columns run over the row's cells, then the array columns); per
// chunk of zc slices it stages the R rows of every slice once (coalesced, the
// R rows of one voxel column adjacent so one LDS read serves all R, W - 1
// zero columns past the last so the band needs no clamp), and a thread
// applies its column's band weights, loaded once per slice, to the R staged
// rows.  Sums: FP32 over the terms of kGroup consecutive slices, FP64 across
// groups.  W is the table's width.
template <int R, int W>
__global__ __launch_bounds__(kBlockF) void k_pl_major1_lds(PlenDev d, int zc, int ncb)
{
    extern __shared__ float4 ms4[];
    float* ms = reinterpret_cast<float*>(ms4);             // [slice of the chunk][nx + W - 1][R]
    const int nvb = (d.na_v + R - 1) / R;
    const int kt = blockIdx.x / (nvb * ncb);
    const int rem = blockIdx.x % (nvb * ncb);
    const int va0 = (rem / ncb) * R;
    const int j = (rem % ncb) * kBlockF + threadIdx.x;
    const int nr = min(R, d.na_v - va0);
    const int c0 = d.cell_first[kt];
    const int ncols = (d.cell_first[kt + 1] - c0) * d.na_u;
    if ((rem % ncb) * kBlockF >= ncols) return;            // uniform over the workgroup
    const bool live = j < ncols;
    const int ua = live ? j % d.na_u : 0;
    const int ks = live ? d.cell_ks[c0 + j / d.na_u] : 0;
    const int pitch = (d.nx + W - 1) * R;                  // floats per staged slice
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    // 32-bit table offsets (the launcher checks the tables' sizes)
    const int sstep = d.ks * d.na_u;
    const int so = ks * d.na_u + ua;
    const int lane = threadIdx.x & 63;
    for (int z0 = 0; z0 < d.nz; z0 += zc) {
        const int nzc = min(zc, d.nz - z0);
        __syncthreads();                                   // the previous chunk is consumed
        // one wave per staged row, lanes along it; loads from clamped (valid)
        // addresses, then a select, so a wave's loads are in flight together
        for (int row = threadIdx.x >> 6; row < nzc * R; row += kBlockF / 64) {
            const int z = row / R, r = row % R;
            const float* src =
                d.m1 + (((size_t)(z0 + z) * d.kt + kt) * d.na_v + va0 + min(r, nr - 1)) * d.nx;
            float* dst = ms + z * pitch + r;
#pragma unroll 4
            for (int ix = lane; ix < d.nx + W - 1; ix += 64) {
                const float v = src[min(ix, d.nx - 1)];
                dst[ix * R] = r < nr && ix < d.nx ? v : 0.0f;
            }
        }
        __syncthreads();
        if (!live) continue;
        for (int z = 0; z < nzc; z += kGroup) {
            float part[R];
#pragma unroll
            for (int r = 0; r < R; ++r) part[r] = 0.0f;
#pragma unroll
            for (int g = 0; g < kGroup; ++g) {
                if (z + g >= nzc) break;
                const int zs = so + (z0 + z + g) * sstep;
                const int s0 = d.bs1.start[zs];
                const int wo = zs + (zs - ua) * (W - 1);   // (table * W) * na_u + ua
                const float* mz = ms + (z + g) * pitch + s0 * R;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const float wk = d.bs1.w[wo + k * d.na_u];
                    float m[R];
                    lds_rows<R>(mz + k * R, m);
#pragma unroll
                    for (int r = 0; r < R; ++r) part[r] = fmaf(wk, m[r], part[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += (double)part[r];
        }
    }
    if (!live) return;
    const int c = c0 + j / d.na_u;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < nr)
            d.fa[((size_t)c * d.na_v + va0 + r) * d.na_u + ua] =
                (float)acc[r] * d.mask[(size_t)(va0 + r) * d.na_u + ua];
}

// M2[c][vd][ua] = sum_k bt2[kt_c][vd][k] FA[c][st + k][ua]
__global__ __launch_bounds__(kBlock) void k_pl_minor2(PlenDev d)
{
    constexpr int R = kMinorRows;
    const int ua = blockIdx.x * blockDim.x + threadIdx.x;
    if (ua >= d.na_u) return;
    const int vb = (d.nv + R - 1) / R;
    const size_t groups = (size_t)d.cells * vb;
    for (size_t g = blockIdx.y; g < groups; g += gridDim.y) {
        const int v0 = (int)(g % vb) * R;
        const int c = (int)(g / vb);
        const float* col = d.fa + (size_t)c * d.na_v * d.na_u + ua;
        const size_t tab = (size_t)d.cell_kt[c];
        const int32_t* st = d.bt2.start + tab * d.bt2.rows;
        const float* w = d.bt2.w + tab * d.bt2.width * (size_t)d.bt2.rows;
        int s0[R];
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            s0[r] = st[min(v0 + r, d.nv - 1)];
            acc[r] = 0.0;
        }
        for (int k = 0; k < d.bt2.width; ++k) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int va = s0[r] + k;
                if (va < d.na_v)
                    acc[r] += (double)(w[(size_t)k * d.bt2.rows + min(v0 + r, d.nv - 1)] *
                                       col[(size_t)va * d.na_u]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (v0 + r < d.nv) d.m2[((size_t)c * d.nv + v0 + r) * d.na_u + ua] = (float)acc[r];
    }
}

// y[vd][ud] = sum_c sum_k bs2[ks_c][ud][k] M2[c][vd][st + k]
// (kMinorRows detector rows per thread share the column's band; each output
// sums a cell's band in order, then the cells in order)
__global__ __launch_bounds__(kBlock) void k_pl_major2(PlenDev d, float* __restrict__ y)
{
    constexpr int R = kMinorRows;
    const int ud = blockIdx.x * blockDim.x + threadIdx.x;
    if (ud >= d.nu) return;
    const int vb = (d.nv + R - 1) / R;
    for (int g = blockIdx.y; g < vb; g += gridDim.y) {
        const int v0 = g * R;
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int c = 0; c < d.cells; ++c) {
            const size_t tab = (size_t)d.cell_ks[c];
            const int st = d.bs2.start[tab * d.bs2.rows + ud];
            const float* w = d.bs2.w + tab * d.bs2.width * (size_t)d.bs2.rows + ud;
            const float* m = d.m2 + (size_t)c * d.nv * d.na_u;
            double part[R];
#pragma unroll
            for (int r = 0; r < R; ++r) part[r] = 0.0;
            for (int k = 0; k < d.bs2.width; ++k) {
                const int col = st + k;
                if (col >= d.na_u) break;
                const float wk = w[(size_t)k * d.bs2.rows];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    part[r] += (double)(wk * m[(size_t)min(v0 + r, d.nv - 1) * d.na_u + col]);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += part[r];
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (v0 + r < d.nv) y[(size_t)(v0 + r) * d.nu + ud] = (float)acc[r];
    }
}

// M2[c][vd][ua] = sum_k bs2t[ks_c][ua][k] y[vd][st + k]
// (kMinorRows detector rows per thread share the array column's band)
__global__ __launch_bounds__(kBlock) void k_pl_major2_t(PlenDev d, const float* __restrict__ y)
{
    constexpr int R = kMinorRows;
    const int ua = blockIdx.x * blockDim.x + threadIdx.x;
    if (ua >= d.na_u) return;
    const int vb = (d.nv + R - 1) / R;
    const size_t groups = (size_t)d.cells * vb;
    for (size_t g = blockIdx.y; g < groups; g += gridDim.y) {
        const int v0 = (int)(g % vb) * R;
        const int c = (int)(g / vb);
        const size_t tab = (size_t)d.cell_ks[c];
        const int st = d.bs2t.start[tab * d.bs2t.rows + ua];
        const float* w = d.bs2t.w + tab * d.bs2t.width * (size_t)d.bs2t.rows + ua;
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int k = 0; k < d.bs2t.width; ++k) {
            const int col = st + k;
            if (col >= d.nu) break;
            const float wk = w[(size_t)k * d.bs2t.rows];
#pragma unroll
            for (int r = 0; r < R; ++r)
                acc[r] += (double)(wk * y[(size_t)min(v0 + r, d.nv - 1) * d.nu + col]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (v0 + r < d.nv) d.m2[((size_t)c * d.nv + v0 + r) * d.na_u + ua] = (float)acc[r];
    }
}

// FA[c][va][ua] = mask[va][ua] * sum_k bt2t[kt_c][va][k] M2[c][st + k][ua]
__global__ __launch_bounds__(kBlock) void k_pl_minor2_t(PlenDev d)
{
    constexpr int R = kMinorRows;
    const int ua = blockIdx.x * blockDim.x + threadIdx.x;
    if (ua >= d.na_u) return;
    const int vb = (d.na_v + R - 1) / R;
    const size_t groups = (size_t)d.cells * vb;
    for (size_t g = blockIdx.y; g < groups; g += gridDim.y) {
        const int v0 = (int)(g % vb) * R;
        const int c = (int)(g / vb);
        const float* col = d.m2 + (size_t)c * d.nv * d.na_u + ua;
        const size_t tab = (size_t)d.cell_kt[c];
        const int32_t* st = d.bt2t.start + tab * d.bt2t.rows;
        const float* w = d.bt2t.w + tab * d.bt2t.width * (size_t)d.bt2t.rows;
        int s0[R];
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            s0[r] = st[min(v0 + r, d.na_v - 1)];
            acc[r] = 0.0;
        }
        for (int k = 0; k < d.bt2t.width; ++k) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int vd = s0[r] + k;
                if (vd < d.nv)
                    acc[r] += (double)(w[(size_t)k * d.bt2t.rows + min(v0 + r, d.na_v - 1)] *
                                       col[(size_t)vd * d.na_u]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (v0 + r < d.na_v) {
                const size_t i = ((size_t)c * d.na_v + v0 + r) * d.na_u + ua;
                d.fa[i] = (float)acc[r] * d.mask[(size_t)(v0 + r) * d.na_u + ua];
            }
    }
}

// M1[iz][kt][va][ix] = sum_{c in row kt} sum_k bs1t[iz, ks_c][ix][k] FA[c][va][st + k]
__global__ __launch_bounds__(kBlock) void k_pl_major1_t(PlenDev d)
{
    const size_t total = (size_t)d.nz * d.kt * d.na_v * d.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ix = (int)(i % d.nx);
        size_t q = i / d.nx;
        const int va = (int)(q % d.na_v);
        q /= d.na_v;
        const int kt = (int)(q % d.kt);
        const int iz = (int)(q / d.kt);
        double acc = 0.0;
        for (int c = d.cell_first[kt]; c < d.cell_first[kt + 1]; ++c) {
            const float* row = d.fa + ((size_t)c * d.na_v + va) * d.na_u;
            acc += band_dot(d.bs1t, (size_t)iz * d.ks + d.cell_ks[c], ix, row, 1, d.na_u);
        }
        d.m1[i] = (float)acc;
    }
}

// k_pl_major1_t with the loop bound W >= the table width fixed at compile
// time (terms past the width are skipped).
template <int W>
__global__ __launch_bounds__(kBlock) void k_pl_major1_t_w(PlenDev d)
{
    const size_t total = (size_t)d.nz * d.kt * d.na_v * d.nx;
    const int wd = d.bs1t.width;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int ix = (int)(i % d.nx);
        size_t q = i / d.nx;
        const int va = (int)(q % d.na_v);
        q /= d.na_v;
        const int kt = (int)(q % d.kt);
        const int iz = (int)(q / d.kt);
        double acc = 0.0;
        for (int c = d.cell_first[kt]; c < d.cell_first[kt + 1]; ++c) {
            const size_t tab = (size_t)iz * d.ks + d.cell_ks[c];
            const int s0 = d.bs1t.start[tab * d.nx + ix];
            const float* w = d.bs1t.w + tab * wd * (size_t)d.nx + ix;
            const float* row = d.fa + ((size_t)c * d.na_v + va) * d.na_u;
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (k < wd) acc += (double)(w[(size_t)k * d.nx] * row[min(s0 + k, d.na_u - 1)]);
        }
        d.m1[i] = (float)acc;
    }
}

// k_pl_major1_t with the array-plane rows staged in LDS: a workgroup takes
// R array rows of one angular row kt (the rows of all its cells, staged once,
// coalesced, the R rows of one array column adjacent so one LDS read serves
// all R) and a chunk of slices; a thread takes one (slice, voxel column), loads each
// cell's band weights once and applies them to the R staged rows.  Sums:
// FP32 over one cell's band, FP64 across cells.  W >= the table's width
// (terms past it skipped).
constexpr int kBlockT = 1024;   // 16 waves share one staged row block

template <int R, int W>
__global__ __launch_bounds__(kBlockT) void k_pl_major1_t_lds(PlenDev d, int zchunk)
{
    extern __shared__ float4 fs4[];
    float* fs = reinterpret_cast<float*>(fs4);             // [cell of the row][na_u][R]
    const int nvb = (d.na_v + R - 1) / R;
    const int kt = blockIdx.x / nvb;
    const int va0 = (blockIdx.x % nvb) * R;
    const int nr = min(R, d.na_v - va0);
    const int c0 = d.cell_first[kt], nc = d.cell_first[kt + 1] - c0;
    const int pitch = d.na_u * R;                          // floats per staged cell
    // one wave per staged row, lanes along it; loads from valid rows, then a
    // select, so a wave's loads are in flight together
    const int lane = threadIdx.x & 63;
    for (int row = threadIdx.x >> 6; row < nc * R; row += kBlockT / 64) {
        const int c = row / R, r = row % R;
        const float* src = d.fa + ((size_t)(c0 + c) * d.na_v + va0 + min(r, nr - 1)) * d.na_u;
        float* dst = fs + c * pitch + r;
#pragma unroll 4
        for (int ua = lane; ua < d.na_u; ua += 64) {
            const float v = src[ua];
            dst[ua * R] = r < nr ? v : 0.0f;
        }
    }
    __syncthreads();
    const int iz0 = blockIdx.y * zchunk;
    const int iz1 = min(d.nz, iz0 + zchunk);
    const int wd = d.bs1t.width;
    const int items = (iz1 - iz0) * d.nx;
    for (int it = threadIdx.x; it < items; it += kBlockT) {
        const int iz = iz0 + it / d.nx;
        const int ix = it % d.nx;
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll 2
        for (int c = 0; c < nc; ++c) {
            // 32-bit table offsets (the launcher checks the tables' sizes)
            const int tab = iz * d.ks + d.cell_ks[c0 + c];
            const int s0 = d.bs1t.start[tab * d.nx + ix];
            const int wo = tab * wd * d.nx + ix;
            const float* fc = fs + c * pitch;
            float part[R];
#pragma unroll
            for (int r = 0; r < R; ++r) part[r] = 0.0f;
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (k < wd) {
                    const float wk = d.bs1t.w[wo + k * d.nx];
                    float f[R];
                    lds_rows<R>(fc + min(s0 + k, d.na_u - 1) * R, f);
#pragma unroll
                    for (int r = 0; r < R; ++r) part[r] = fmaf(wk, f[r], part[r]);
                }
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += (double)part[r];
        }
        float* out = d.m1 + (((size_t)iz * d.kt + kt) * d.na_v + va0) * d.nx + ix;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r < nr) out[(size_t)r * d.nx] = (float)acc[r];
    }
}

template <int R>
void launch_major1_t_lds(const PlenDev& p, int wb, int zchunk, dim3 g, hipStream_t s)
{
    const size_t lds = (size_t)std::max(1, p.row_cells_max) * R * p.na_u * sizeof(float);
    if (wb == 8)
        hipLaunchKernelGGL((k_pl_major1_t_lds<R, 8>), g, dim3(kBlockT), lds, s, p, zchunk);
    else if (wb == 16)
        hipLaunchKernelGGL((k_pl_major1_t_lds<R, 16>), g, dim3(kBlockT), lds, s, p, zchunk);
    else
        hipLaunchKernelGGL((k_pl_major1_t_lds<R, 24>), g, dim3(kBlockT), lds, s, p, zchunk);
}

// Stage-1 major pass of A: the LDS-staged kernel for table widths up to 4
// while 4 rows of one slice fit 64 KiB, else the global-gather kernels.
void launch_major1(const PlenDev& p, hipStream_t s)
{
    constexpr int R = 4;
    const int w = std::max(1, p.bs1.width);
    const int zc = 65536 / ((p.nx + w - 1) * R * (int)sizeof(float));    // slices per 64 KiB chunk
    const int nvb = (p.na_v + R - 1) / R;
    const int ncb = (int)(((size_t)p.row_cells_max * p.na_u + kBlockF - 1) / kBlockF);
    const size_t nblocks = (size_t)p.kt * nvb * ncb;
    const size_t lds = (size_t)std::max(1, zc) * (p.nx + w - 1) * R * sizeof(float);
    const bool staged = zc >= 1 && nblocks < (1u << 31) && (size_t)p.row_cells_max * p.na_u < (1u << 31) &&
                        (size_t)p.nz * p.ks * p.bs1.width * p.na_u < (1u << 31);
    const dim3 gs((unsigned)nblocks), bf(kBlockF), b(kBlock);
    const dim3 g1(grid_for((size_t)p.cells * p.na_v * p.na_u));
    switch (staged ? p.bs1.width : -p.bs1.width) {
    case 1: hipLaunchKernelGGL((k_pl_major1_lds<R, 1>), gs, bf, lds, s, p, zc, ncb); break;
    case 2: hipLaunchKernelGGL((k_pl_major1_lds<R, 2>), gs, bf, lds, s, p, zc, ncb); break;
    case 3: hipLaunchKernelGGL((k_pl_major1_lds<R, 3>), gs, bf, lds, s, p, zc, ncb); break;
    case 4: hipLaunchKernelGGL((k_pl_major1_lds<R, 4>), gs, bf, lds, s, p, zc, ncb); break;
    case -1: hipLaunchKernelGGL(k_pl_major1_w<1>, g1, b, 0, s, p); break;
    case -2: hipLaunchKernelGGL(k_pl_major1_w<2>, g1, b, 0, s, p); break;
    case -3: hipLaunchKernelGGL(k_pl_major1_w<3>, g1, b, 0, s, p); break;
    case -4: hipLaunchKernelGGL(k_pl_major1_w<4>, g1, b, 0, s, p); break;
    default: hipLaunchKernelGGL(k_pl_major1, g1, b, 0, s, p); break;
    }
}

// Stage-1 major pass of A^T: the LDS-staged kernel while R >= 1 rows of every
// cell of one angular row fit 64 KiB, else the global-gather kernels.
void launch_major1_t(const PlenDev& p, hipStream_t s)
{
    const int wb = p.bs1t.width <= 8 ? 8 : p.bs1t.width <= 16 ? 16 : 24;
    int R = 8;
    while (R >= 1 && (size_t)p.row_cells_max * R * p.na_u * sizeof(float) > 65536) R /= 2;
    if (R >= 1 && p.bs1t.width <= 24 && (size_t)p.nz * p.ks * p.bs1t.width * p.nx < (1u << 31)) {
        const int nvb = (p.na_v + R - 1) / R;
        const int zsplit = std::max(1, std::min(p.nz, (1024 + p.kt * nvb - 1) / (p.kt * nvb)));
        const int zchunk = (p.nz + zsplit - 1) / zsplit;
        const dim3 g((unsigned)(p.kt * nvb), (unsigned)((p.nz + zchunk - 1) / zchunk));
        switch (R) {
        case 8: launch_major1_t_lds<8>(p, wb, zchunk, g, s); return;
        case 4: launch_major1_t_lds<4>(p, wb, zchunk, g, s); return;
        case 2: launch_major1_t_lds<2>(p, wb, zchunk, g, s); return;
        default: launch_major1_t_lds<1>(p, wb, zchunk, g, s); return;
        }
    }
    const dim3 g1(grid_for((size_t)p.nz * p.kt * p.na_v * p.nx)), b(kBlock);
    if (p.bs1t.width <= 8)
        hipLaunchKernelGGL(k_pl_major1_t_w<8>, g1, b, 0, s, p);
    else if (p.bs1t.width <= 16)
        hipLaunchKernelGGL(k_pl_major1_t_w<16>, g1, b, 0, s, p);
    else if (p.bs1t.width <= 24)
        hipLaunchKernelGGL(k_pl_major1_t_w<24>, g1, b, 0, s, p);
    else
        hipLaunchKernelGGL(k_pl_major1_t, g1, b, 0, s, p);
}

}  // namespace

hipError_t launch_plen_project(const PlenDev& p, const float* x, float* y, hipStream_t s)
{
    // stage 1 minor pass: the transport's t filter onto the array plane
    XportDev d{};
    d.nx = p.nx; d.ny = p.ny; d.nz = p.nz; d.nu = p.na_u; d.nv = p.na_v; d.kt = p.kt;
    d.bt = p.bt1;
    d.mid = p.m1;
    {
        const RowGrid rg = row_grid((size_t)d.nz * d.kt * ((d.nv + kMinorRows - 1) / kMinorRows), d.nx);
        hipLaunchKernelGGL(k_minor_fwd, rg.g, rg.b, 0, s, d, x);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_major1(p, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        const RowGrid rg = row_grid((size_t)p.cells * ((p.nv + kMinorRows - 1) / kMinorRows), p.na_u);
        hipLaunchKernelGGL(k_pl_minor2, rg.g, rg.b, 0, s, p);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        const RowGrid rg = row_grid((size_t)((p.nv + kMinorRows - 1) / kMinorRows), p.nu);
        hipLaunchKernelGGL(k_pl_major2, rg.g, rg.b, 0, s, p, y);
    }
    return hipGetLastError();
}

hipError_t launch_plen_backproject(const PlenDev& p, const float* y, float* x, hipStream_t s)
{
    {
        const RowGrid rg = row_grid((size_t)p.cells * ((p.nv + kMinorRows - 1) / kMinorRows), p.na_u);
        hipLaunchKernelGGL(k_pl_major2_t, rg.g, rg.b, 0, s, p, y);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const RowGrid rg = row_grid((size_t)p.cells * ((p.na_v + kMinorRows - 1) / kMinorRows), p.na_u);
        hipLaunchKernelGGL(k_pl_minor2_t, rg.g, rg.b, 0, s, p);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    launch_major1_t(p, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // stage 1 minor pass transposed: sums the angular rows per voxel
    XportDev d{};
    d.nx = p.nx; d.ny = p.ny; d.nz = p.nz; d.nu = p.na_u; d.nv = p.na_v; d.kt = p.kt;
    d.btt = p.bt1t;
    d.mid = p.m1;
    hipLaunchKernelGGL(k_minor_adj, dim3(grid_for((size_t)p.nz * p.ny * p.nx)), dim3(kBlock), 0, s, d, x);
    return hipGetLastError();
}

}  // namespace ltm
