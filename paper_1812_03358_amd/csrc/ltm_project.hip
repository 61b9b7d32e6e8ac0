// gfx950 kernels of the camera operator y = A x and its transpose.
//
// A ray of a pixel is traced back through the camera's lenses (the affine
// propagation and thin-lens maps of the paper's optics table, composed per
// its camera-model section), clipped to the voxel box and integrated with S
// midpoint samples of the trilinear interpolant (line-integral radiance of
// the object-model section).  The pixel value is the mean over its R
// angular samples (measurement-formation section).  The transpose uses the
// same samples and weights, so it is the exact adjoint (adjoint-operations
// section).
//
// Work decomposition (not the paper's: its separable filtering kernels are
// replaced by a ray march): one workgroup owns a tile of pixels; it walks
// the tile's rays through slabs of camera depth, staging the voxels a slab
// touches in an LDS brick (forward: gather from LDS; adjoint: LDS float
// atomics, then one global atomic flush per brick voxel).  The brick of
// every (tile, slab) is computed once per plan by k_setup.
#include "ltm_internal.h"

#include <algorithm>
#include <cfloat>
#include <mutex>

// Fixed FP64 adjoint accumulator of ltm_backproject_noalloc (kScratchVoxels
// doubles, 64 MiB per GPU, held until the process ends).  Host code never
// passes this name to a kernel: it is a host-side stand-in there, and the
// device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) double scratch[ltm::kScratchVoxels];

namespace ltm {

// Device address of this GPU's copy of `scratch`, looked up once per device
// (with that device current) and kept.
hipError_t scratch_accumulator(double** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

namespace {

struct Ray {
    float qA[3], dq[3];
    float z0, z1, h, inv_h, w;
};

// Pixel of one work item of a tile, or false for a ragged item.
__device__ __forceinline__ bool item_pixel(const CamDev& c, int tile, int item, int& iu, int& iv)
{
    if (item >= c.items_per_split) return false;
    const int split = tile % c.splits;
    const int blk = tile / c.splits;
    const int it = split * c.items_per_split + item;
    if (it >= c.items) return false;
    const int tu = blk % c.tiles_u, tv = blk / c.tiles_u;
    const int tl = c.tile_u * c.tile_v, kk = c.ku * c.kv;
    int lid, pid;
    if ((c.order & 1) == 0) {
        lid = it / kk;
        pid = it - lid * kk;
    } else {
        pid = it / tl;
        lid = it - pid * tl;
    }
    const int lu = tu * c.tile_u + lid % c.tile_u;
    const int lv = tv * c.tile_v + lid / c.tile_u;
    if (lu >= c.mu || lv >= c.mv) return false;
    iu = lu * c.ku + pid % c.ku;
    iv = lv * c.kv + pid / c.ku;
    return iu < c.nu && iv < c.nv;
}

// Geometry of ray (ru, rv) of pixel (iu, iv).  Returns false when the ray is
// occluded (aperture grid sample outside the unit disc, or a plenoptic ray
// missing the main lens -- decided in FP64) or misses the voxel box.
__device__ __forceinline__ bool make_ray(const CamDev& c, int iu, int iv, int ru, int rv, Ray& r)
{
    // hexagonal cameras: rv = lenslet * grv + angular row (3 x 3 lenslets)
    int nb = 0;
    if (c.kind == LTM_PLENOPTIC_HEX) {
        nb = rv / c.grv;
        rv -= nb * c.grv;
    }
    const int a = 2 * ru + 1 - c.ru, b = 2 * rv + 1 - c.grv;
    if ((long long)a * a * c.grv * c.grv + (long long)b * b * c.ru * c.ru >
        (long long)c.ru * c.ru * c.grv * c.grv)
        return false;
    if (c.sub_n > 1 && (ru + c.ru * rv) % c.sub_n != c.sub_i) return false;
    const float gs = (float)a / (float)c.ru;
    const float gt = (float)b / (float)c.grv;
    const float du = (float)iu + 0.5f - 0.5f * (float)c.nu;
    const float dv = (float)iv + 0.5f - 0.5f * (float)c.nv;
    float cu = 0.0f, cv = 0.0f, Ag = c.Ag, Bg = c.Bg;
    double Lg = c.Lg;
    if (c.kind == LTM_PLENOPTIC) {
        cu = (float)(iu / c.ku) + 0.5f - 0.5f * (float)c.mu;
        cv = (float)(iv / c.kv) + 0.5f - 0.5f * (float)c.mv;
    } else if (c.kind == LTM_PLENOPTIC_HEX) {
        // nearest row +-1, then that row's nearest lenslet +-1
        const int j = (int)rintf(fmaf(dv, c.rowf, 0.5f * (float)(c.hmv - 1))) + nb / 3 - 1;
        if (j < 0 || j >= c.hmv) return false;
        const int rr = j - c.hmid;
        const int odd = rr & 1;
        const float shift = 0.5f * (float)odd - 0.5f * (float)(c.hmu - 1);
        const int i = (int)rintf(fmaf(du, c.colf, -shift)) + nb % 3 - 1;
        if (i < 0 || i >= c.hmu) return false;
        cu = (float)i + shift;                          // exact half-integers
        cv = (float)j - 0.5f * (float)(c.hmv - 1);
        int type = ((2 * i + odd - rr) / 2 - rr) % 3;
        type += type < 0 ? 3 : 0;
        Ag = type == 0 ? c.hAg[0] : (type == 1 ? c.hAg[1] : c.hAg[2]);
        Bg = type == 0 ? c.hBg[0] : (type == 1 ? c.hBg[1] : c.hBg[2]);
        Lg = type == 0 ? c.hLg[0] : (type == 1 ? c.hLg[1] : c.hLg[2]);
    }
    if (c.need_aperture) {
        const double sL = c.Lc * (double)cu + c.Ld * (double)du + Lg * (double)gs;
        const double tL = c.Lct * (double)cv + c.Ld * (double)dv + Lg * (double)gt;
        if (sL * sL + tL * tL > c.r2) return false;
    }
    const float sig = fmaf(c.Ac, cu, fmaf(c.Ad, du, Ag * gs));
    const float tau = fmaf(c.Act, cv, fmaf(c.Ad, dv, Ag * gt));
    const float us = fmaf(c.Bc, cu, fmaf(c.Bd, du, Bg * gs));
    const float vs = fmaf(c.Bct, cv, fmaf(c.Bd, dv, Bg * gt));
    float zl = c.zlo, zh = FLT_MAX;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.qA[k] = fmaf(sig, c.Es[k], fmaf(tau, c.Et[k], c.CA[k]));
        r.dq[k] = fmaf(us, c.Es[k], fmaf(vs, c.Et[k], c.Ez[k]));
        const float lo = -0.5f, hi = (float)c.n[k] - 0.5f;
        if (r.dq[k] != 0.0f) {
            const float t1 = (lo - r.qA[k]) / r.dq[k];
            const float t2 = (hi - r.qA[k]) / r.dq[k];
            zl = fmaxf(zl, fminf(t1, t2));
            zh = fminf(zh, fmaxf(t1, t2));
        } else if (r.qA[k] < lo || r.qA[k] > hi) {
            return false;
        }
    }
    if (!(zh > zl)) return false;
    r.z0 = zl;
    r.z1 = zh;
    r.h = (zh - zl) / (float)c.S;
    r.inv_h = (float)c.S / (zh - zl);
    r.w = r.h * sqrtf(fmaf(us, us, fmaf(vs, vs, 1.0f))) * c.invR;
    return true;
}

// First sample index m with z' >= z (samples sit at z0 + (m + 1/2) h).
__device__ __forceinline__ int sample_bound(const Ray& r, float z, int S)
{
    const float t = ceilf(fmaf(z - r.z0, r.inv_h, -0.5f));
    return (int)fminf(fmaxf(t, 0.0f), (float)S);
}

__device__ __forceinline__ float slab_edge(const TileRec& t, int k, float chunk)
{
    return fmaf((float)k, chunk, t.z_start);
}

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(v, lo, hi);
}

// Trilinear cell of sample position q: clamp to [0, n-1], cell origin
// i = min(floor(q), n-2) and fraction f = q - i (identical in every kernel).
// floor(clamp(q, 0, nextbelow(n-1))) equals min(floor(clamp(q, 0, n-1)), n-2)
// for every q, without a separate min.
struct Cell {
    float i[3], f[3];
};

struct Bounds {
    float nm1[3], nm1m[3];   // n - 1 and the largest float below it
};

__device__ __forceinline__ Bounds bounds_of(const int n[3])
{
    Bounds b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        b.nm1[k] = (float)(n[k] - 1);
        b.nm1m[k] = __int_as_float(__float_as_int(b.nm1[k]) - 1);
    }
    return b;
}

__device__ __forceinline__ Cell cell_of(float qx, float qy, float qz, const Bounds& bd)
{
    Cell s;
    const float q[3] = {qx, qy, qz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float qc = clampf(q[k], 0.0f, bd.nm1[k]);
        s.i[k] = floorf(clampf(q[k], 0.0f, bd.nm1m[k]));
        s.f[k] = qc - s.i[k];
    }
    return s;
}

// The same trilinear cell inside an LDS brick that carries one replicated
// layer outside the grid on every side (index -1 holds voxel 0, index n holds
// voxel n-1): the clamps drop out.  For q in the outer half-voxel shell the
// interpolation mixes a voxel with its own copy, a + f (a - a) = a exactly,
// which is the clamped value; inside it is the same cell as cell_of.
__device__ __forceinline__ Cell cell_of_padded(float qx, float qy, float qz)
{
    Cell s;
    const float q[3] = {qx, qy, qz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s.i[k] = floorf(q[k]);
        s.f[k] = q[k] - s.i[k];
    }
    return s;
}

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ float tri(float c000, float c100, float c010, float c110, float c001,
                                     float c101, float c011, float c111, const Cell& s)
{
    const float x00 = lerp(c000, c100, s.f[0]);
    const float x10 = lerp(c010, c110, s.f[0]);
    const float x01 = lerp(c001, c101, s.f[0]);
    const float x11 = lerp(c011, c111, s.f[0]);
    return lerp(lerp(x00, x10, s.f[1]), lerp(x01, x11, s.f[1]), s.f[2]);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Block-wide min (is_max = false) or max over kThreads lanes.
__device__ float block_reduce(float v, bool is_max, float* red)
{
    v = is_max ? wave_max(v) : wave_min(v);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    float r = red[0];
#pragma unroll
    for (int k = 1; k < kThreads / 64; ++k) r = is_max ? fmaxf(r, red[k]) : fminf(r, red[k]);
    return r;
}

// ---------------------------------------------------------------- setup
// One workgroup per tile: the camera-depth range of the tile's rays, then
// for each slab the voxel box its samples can touch (with one voxel of
// margin against rounding).
__global__ __launch_bounds__(kThreads) void k_setup(CamDev c, TileRec* tiles, BrickRec* bricks)
{
    __shared__ float red[kThreads / 64];
    const int tile = blockIdx.x;
    float zmin = FLT_MAX, zmax = -FLT_MAX;
    for (int item = threadIdx.x; item < c.items_per_split; item += kThreads) {
        int iu, iv;
        if (!item_pixel(c, tile, item, iu, iv)) continue;
        for (int rv = 0; rv < c.rv; ++rv)
            for (int ru = 0; ru < c.ru; ++ru) {
                Ray r;
                if (!make_ray(c, iu, iv, ru, rv, r)) continue;
                zmin = fminf(zmin, r.z0);
                zmax = fmaxf(zmax, r.z1);
            }
    }
    zmin = block_reduce(zmin, false, red);
    zmax = block_reduce(zmax, true, red);
    TileRec t;
    t.z_start = zmin;
    t.n_chunks = 0;
    if (zmax > zmin) {
        const float span = (zmax - zmin) / c.chunk;
        t.n_chunks = (int)fminf(fmaxf(ceilf(span), 1.0f), (float)c.max_chunks);
    }
    if (threadIdx.x == 0) tiles[tile] = t;
    const float nm1[3] = {(float)(c.n[0] - 1), (float)(c.n[1] - 1), (float)(c.n[2] - 1)};
    for (int ch = 0; ch < t.n_chunks; ++ch) {
        const float za = slab_edge(t, ch, c.chunk);
        const float zb = (ch == t.n_chunks - 1) ? FLT_MAX : slab_edge(t, ch + 1, c.chunk);
        float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
        for (int item = threadIdx.x; item < c.items_per_split; item += kThreads) {
            int iu, iv;
            if (!item_pixel(c, tile, item, iu, iv)) continue;
            for (int rv = 0; rv < c.rv; ++rv)
                for (int ru = 0; ru < c.ru; ++ru) {
                    Ray r;
                    if (!make_ray(c, iu, iv, ru, rv, r)) continue;
                    const float a = fmaxf(za, r.z0), b = fminf(zb, r.z1);
                    if (a > b) continue;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const float pa = clampf(fmaf(a, r.dq[k], r.qA[k]), 0.0f, nm1[k]);
                        const float pb = clampf(fmaf(b, r.dq[k], r.qA[k]), 0.0f, nm1[k]);
                        lo[k] = fminf(lo[k], fminf(pa, pb));
                        hi[k] = fmaxf(hi[k], fmaxf(pa, pb));
                    }
                }
        }
        BrickRec br;
        long long vol = 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float l = block_reduce(lo[k], false, red);
            const float h = block_reduce(hi[k], true, red);
            int il = 0, ih = 1;
            if (h >= l) {
                // one replicated layer past the grid on each side (-1 .. n)
                il = max(-1, (int)floorf(l) - 1);
                ih = min(c.n[k], (int)floorf(h) + 2);
                ih = max(ih, il + 1);
            }
            br.lo[k] = il;
            br.dim[k] = ih - il + 1;
            vol *= br.dim[k];
        }
        br.lds = (vol <= (long long)c.brick_cap) ? 1 : 0;
        br.base = (float)br.lo[0] + (float)br.dim[0] * ((float)br.lo[1] + (float)br.dim[1] * (float)br.lo[2]);
        if (threadIdx.x == 0) bricks[(size_t)tile * c.max_chunks + ch] = br;
    }
}

// ---------------------------------------------------------------- brick I/O
__device__ __forceinline__ size_t gindex(const int n[3], int x, int y, int z)
{
    return (size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * (size_t)z);
}

// Brick words are visited plane by plane.  Lane t owns one point (x, y) of the
// brick's z-planes and a first plane z0, and steps through z by zq, so that
// with fewer plane points than lanes the lanes split the planes between them;
// the point's coordinates and clamped row offset are worked out once, and
// the z clamp is the same for every lane.  Consecutive lanes read
// consecutive x.
struct BrickWalk {
    int plane, zq, z0, p;
    size_t off, nxy;   // clamped (x, y) offset and the grid's z stride
};

// Lanes t < plane * zq take part; exact for t, p < 2^20: (t + 1/2)/d is at
// least 1/(2 d) away from an integer.
__device__ __forceinline__ bool brick_walk(const BrickRec& b, const int n[3], int t, BrickWalk& w)
{
    w.plane = b.dim[0] * b.dim[1];
    w.zq = w.plane >= kThreads ? 1 : kThreads / w.plane;
    if (t >= w.plane * w.zq) return false;
    w.z0 = (int)(((float)t + 0.5f) / (float)w.plane);
    w.p = t - w.z0 * w.plane;
    const int ly = (int)(((float)w.p + 0.5f) / (float)b.dim[0]), lx = w.p - ly * b.dim[0];
    const int gx = min(max(b.lo[0] + lx, 0), n[0] - 1), gy = min(max(b.lo[1] + ly, 0), n[1] - 1);
    w.off = (size_t)gx + (size_t)n[0] * gy;
    w.nxy = (size_t)n[0] * n[1];
    return true;
}

constexpr int kStageLoads = 4;

__device__ void stage_brick(const BrickRec& b, const int n[3], const float* __restrict__ x,
                            float* brick)
{
    for (int t = threadIdx.x;; t += kThreads) {
        BrickWalk w;
        if (!brick_walk(b, n, t, w)) break;
        const float* row = x + w.off;
        // kStageLoads loads in flight; the clamped z keeps those past the
        // brick in the grid, and only the brick's planes are stored
        for (int lz = w.z0; lz < b.dim[2]; lz += kStageLoads * w.zq) {
            float v[kStageLoads];
#pragma unroll
            for (int u = 0; u < kStageLoads; ++u) {
                const int gz = min(max(b.lo[2] + lz + u * w.zq, 0), n[2] - 1);
                v[u] = row[w.nxy * gz];
            }
#pragma unroll
            for (int u = 0; u < kStageLoads; ++u)
                if (lz + u * w.zq < b.dim[2]) brick[w.p + w.plane * (lz + u * w.zq)] = v[u];
        }
    }
}

template <typename T>
__device__ void zero_brick(const BrickRec& b, T* brick)
{
    const int vol = b.dim[0] * b.dim[1] * b.dim[2];
    for (int e = threadIdx.x; e < vol; e += kThreads) brick[e] = (T)0;
}

template <typename T>
__device__ void flush_brick(const BrickRec& b, const int n[3], T* brick, double* __restrict__ x)
{
    for (int t = threadIdx.x;; t += kThreads) {
        BrickWalk w;
        if (!brick_walk(b, n, t, w)) break;
        double* row = x + w.off;
        for (int lz = w.z0; lz < b.dim[2]; lz += w.zq) {
            const double v = (double)brick[w.p + w.plane * lz];
            if (v == 0.0) continue;
            const int gz = min(max(b.lo[2] + lz, 0), n[2] - 1);
            unsafeAtomicAdd(&row[w.nxy * gz], v);
        }
    }
}

// ---------------------------------------------------------------- marching
struct March {
    float qs[3], st[3];
};

__device__ __forceinline__ March march_of(const Ray& r)
{
    March m;
    const float zc = fmaf(0.5f, r.h, r.z0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        m.qs[k] = fmaf(zc, r.dq[k], r.qA[k]);
        m.st[k] = r.h * r.dq[k];
    }
    return m;
}

__device__ __forceinline__ double gather_lds(const March& mr, int m0, int m1, const BrickRec& b,
                                             const float* brick, const Bounds& bd)
{
    const float dx = (float)b.dim[0], dxy = (float)(b.dim[0] * b.dim[1]);
    const int sx = b.dim[0], sxy = b.dim[0] * b.dim[1];
    const float maxi = (float)(b.dim[0] * b.dim[1] * b.dim[2] - 1 - (1 + sx + sxy));
    double acc = 0.0;
    // samples are summed in FP32 groups of up to 8, each group added in FP64
    for (int g0 = m0; g0 < m1; g0 += 8) {
        const float fend = (float)min(g0 + 8, m1);
        float part = 0.0f;
        for (float fm = (float)g0; fm < fend; fm += 1.0f) {
            const Cell s = cell_of_padded(fmaf(fm, mr.st[0], mr.qs[0]), fmaf(fm, mr.st[1], mr.qs[1]),
                                   fmaf(fm, mr.st[2], mr.qs[2]));
            const float fi = fmaf(s.i[2], dxy, fmaf(s.i[1], dx, s.i[0])) - b.base;
            const int i0 = (int)clampf(fi, 0.0f, maxi);
            const float* p = brick + i0;
            part += tri(p[0], p[1], p[sx], p[sx + 1], p[sxy], p[sxy + 1], p[sxy + sx], p[sxy + sx + 1], s);
        }
        acc += (double)part;
    }
    return acc;
}

__device__ __forceinline__ double gather_global(const March& mr, int m0, int m1, const int n[3],
                                                const float* __restrict__ x, const Bounds& bd)
{
    const size_t sx = (size_t)n[0], sxy = (size_t)n[0] * n[1];
    double acc = 0.0;
    for (int g0 = m0; g0 < m1; g0 += 8) {
        const float fend = (float)min(g0 + 8, m1);
        float part = 0.0f;
        for (float fm = (float)g0; fm < fend; fm += 1.0f) {
            const Cell s = cell_of(fmaf(fm, mr.st[0], mr.qs[0]), fmaf(fm, mr.st[1], mr.qs[1]),
                                   fmaf(fm, mr.st[2], mr.qs[2]), bd);
            const float* p = x + gindex(n, (int)s.i[0], (int)s.i[1], (int)s.i[2]);
            part += tri(p[0], p[1], p[sx], p[sx + 1], p[sxy], p[sxy + 1], p[sxy + sx], p[sxy + sx + 1], s);
        }
        acc += (double)part;
    }
    return acc;
}

template <typename T, typename Add>
__device__ __forceinline__ void scatter8(T* p, size_t sx, size_t sxy, const Cell& s, float v,
                                         Add add)
{
    const float gx = 1.0f - s.f[0], gy = 1.0f - s.f[1], gz = 1.0f - s.f[2];
    const float z0 = v * gz, z1 = v * s.f[2];
    const float a00 = gy * z0, a10 = s.f[1] * z0, a01 = gy * z1, a11 = s.f[1] * z1;
    add(p, gx * a00);
    add(p + 1, s.f[0] * a00);
    add(p + sx, gx * a10);
    add(p + sx + 1, s.f[0] * a10);
    add(p + sxy, gx * a01);
    add(p + sxy + 1, s.f[0] * a01);
    add(p + sxy + sx, gx * a11);
    add(p + sxy + sx + 1, s.f[0] * a11);
}

// Scatter one ray's samples [m0, m1) into the LDS brick.  With skew, lane
// l walks the samples starting at offset (l mod 64) * count / 64 and wraps,
// so rays of one narrow bundle are at different depths at any moment and
// their LDS atomics do not collide on the same voxels.
template <typename T>
__device__ __forceinline__ void scatter_lds(const March& mr, int m0, int m1, const BrickRec& b,
                                            T* brick, const Bounds& bd, float v, bool skew)
{
    const float dx = (float)b.dim[0], dxy = (float)(b.dim[0] * b.dim[1]);
    const int sx = b.dim[0], sxy = b.dim[0] * b.dim[1];
    const float maxi = (float)(b.dim[0] * b.dim[1] * b.dim[2] - 1 - (1 + sx + sxy));
    const int cnt = m1 - m0;
    int m = m0;
    if (skew) m += (int)(((threadIdx.x & 63) * (unsigned)cnt) >> 6);
    for (int k = 0; k < cnt; ++k) {
        const float fm = (float)m;
        const Cell s = cell_of_padded(fmaf(fm, mr.st[0], mr.qs[0]), fmaf(fm, mr.st[1], mr.qs[1]),
                               fmaf(fm, mr.st[2], mr.qs[2]));
        const float fi = fmaf(s.i[2], dxy, fmaf(s.i[1], dx, s.i[0])) - b.base;
        const int i0 = (int)clampf(fi, 0.0f, maxi);
        scatter8(brick + i0, (size_t)sx, (size_t)sxy, s, v, [](T* q, float a) { atomicAdd(q, (T)a); });
        ++m;
        m = m == m1 ? m0 : m;
    }
}

// As scatter_lds, but a lane keeps the 8 corner weights of its current cell
// in registers while consecutive samples stay in that cell, and issues the
// LDS atomics only when the cell changes (rays advance about half a voxel
// per sample, so cells repeat).
template <typename T>
__device__ __forceinline__ void scatter_lds_merged(const March& mr, int m0, int m1, const BrickRec& b,
                                                   T* brick, const Bounds& bd, float v, bool skew)
{
    const float dx = (float)b.dim[0], dxy = (float)(b.dim[0] * b.dim[1]);
    const int sx = b.dim[0], sxy = b.dim[0] * b.dim[1];
    const float maxi = (float)(b.dim[0] * b.dim[1] * b.dim[2] - 1 - (1 + sx + sxy));
    const int cnt = m1 - m0;
    int m = m0;
    if (skew) m += (int)(((threadIdx.x & 63) * (unsigned)cnt) >> 6);
    int cur = -1;
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    auto flush = [&](int i0) {
        T* p = brick + i0;
        const int off[8] = {0, 1, sx, sx + 1, sxy, sxy + 1, sxy + sx, sxy + sx + 1};
#pragma unroll
        for (int k = 0; k < 8; ++k) atomicAdd(p + off[k], (T)a[k]);
    };
    for (int k = 0; k < cnt; ++k) {
        const float fm = (float)m;
        const Cell s = cell_of_padded(fmaf(fm, mr.st[0], mr.qs[0]), fmaf(fm, mr.st[1], mr.qs[1]),
                               fmaf(fm, mr.st[2], mr.qs[2]));
        const float fi = fmaf(s.i[2], dxy, fmaf(s.i[1], dx, s.i[0])) - b.base;
        const int i0 = (int)clampf(fi, 0.0f, maxi);
        const float gx = 1.0f - s.f[0], gy = 1.0f - s.f[1], gz = 1.0f - s.f[2];
        const float z0 = v * gz, z1 = v * s.f[2];
        const float a00 = gy * z0, a10 = s.f[1] * z0, a01 = gy * z1, a11 = s.f[1] * z1;
        const float w[8] = {gx * a00, s.f[0] * a00, gx * a10, s.f[0] * a10,
                            gx * a01, s.f[0] * a01, gx * a11, s.f[0] * a11};
        // flush the previous cell's sums when the cell changes, then restart
        // (keep = 0) or continue (keep = 1) them without a divergent branch
        const bool change = i0 != cur;
        if (change && cur >= 0) flush(cur);
        const float keep = change ? 0.0f : 1.0f;
        cur = i0;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = fmaf(keep, a[j], w[j]);
        ++m;
        m = m == m1 ? m0 : m;
    }
    if (cur >= 0) flush(cur);
}

// As scatter_lds_merged, but a lane keeps two planes of corner sums across
// the ray's dominant axis c (the 2 x 2 corners in the other two axes, at the
// cell's low and high c): when a sample moves one cell along c, only the
// plane left behind is flushed (4 atomics) and the other becomes the new
// cell's low (or high) plane; any other move flushes both planes.  Rays
// advance about half a voxel per sample, mostly along c, so most cell
// changes flush 4 corners instead of 8.
//
// A wave runs the flush code whenever any of its lanes changes cell, so the
// cost follows how many iterations see a change in some lane.  With skew = 2
// the lanes' staggered starting offsets are even: rays that cross the whole
// grid along c advance exactly half a voxel per sample and cross c-planes at
// samples of one parity, so even offsets keep their c-crossings on the same
// iterations while the lanes still sit at different depths.
template <typename T>
__device__ __forceinline__ void scatter_lds_window(const March& mr, int m0, int m1, const BrickRec& b,
                                                   T* brick, float v, int skew)
{
    const int sx = b.dim[0], sxy = b.dim[0] * b.dim[1];
    const float maxi = (float)(b.dim[0] * b.dim[1] * b.dim[2] - 1 - (1 + sx + sxy));
    // dominant axis c and the other two (a, b), per lane, by selects so that
    // nothing leaves registers: c = x -> (a, b) = (y, z); c = y -> (x, z);
    // c = z -> (x, y)
    const float ax = fabsf(mr.st[0]), ay = fabsf(mr.st[1]), az = fabsf(mr.st[2]);
    const int c = (az >= ax && az >= ay) ? 2 : (ay >= ax ? 1 : 0);
    const int sa = c == 0 ? sx : 1, sb = c == 2 ? sx : sxy, sc = c == 0 ? 1 : (c == 1 ? sx : sxy);
    const float qa0 = c == 0 ? mr.qs[1] : mr.qs[0], da = c == 0 ? mr.st[1] : mr.st[0];
    const float qb0 = c == 2 ? mr.qs[1] : mr.qs[2], db = c == 2 ? mr.st[1] : mr.st[2];
    const float qc0 = c == 0 ? mr.qs[0] : (c == 1 ? mr.qs[1] : mr.qs[2]);
    const float dc = c == 0 ? mr.st[0] : (c == 1 ? mr.st[1] : mr.st[2]);
    const float fsa = (float)sa, fsb = (float)sb, fsc = (float)sc, nbase = -b.base;
    // byte strides of the corners from a cell's low corner
    char* const bytes = reinterpret_cast<char*>(brick);
    const int ba = sa * (int)sizeof(T), bb = sb * (int)sizeof(T), bab = ba + bb;
    const int bc = sc * (int)sizeof(T);
    const int cnt = m1 - m0;
    int off = 0;
    if (skew) {
        off = (int)(((threadIdx.x & 63) * (unsigned)cnt) >> 6);
        if (skew == 2) off &= ~1;
    }
    // the cell's LDS index: exact integer arithmetic in FP32 (brick indices < 2^24)
    auto cell = [&](float fm, float& fa, float& fb, float& fc) {
        const float qa = fmaf(fm, da, qa0), qb = fmaf(fm, db, qb0), qc = fmaf(fm, dc, qc0);
        const float ca = floorf(qa), cb = floorf(qb), cc = floorf(qc);
        fa = qa - ca;
        fb = qb - cb;
        fc = qc - cc;
        const float fi = fmaf(cc, fsc, fmaf(cb, fsb, fmaf(ca, fsa, nbase)));
        return (int)clampf(fi, 0.0f, maxi);
    };
    float lo[4] = {0.f, 0.f, 0.f, 0.f}, hi[4] = {0.f, 0.f, 0.f, 0.f};
    auto flush4 = [&](int i, const float (&p)[4]) {
        char* q = bytes + i * (int)sizeof(T);
        atomicAdd(reinterpret_cast<T*>(q), (T)p[0]);
        atomicAdd(reinterpret_cast<T*>(q + ba), (T)p[1]);
        atomicAdd(reinterpret_cast<T*>(q + bb), (T)p[2]);
        atomicAdd(reinterpret_cast<T*>(q + bab), (T)p[3]);
    };
    // a ray whose dominant coordinate falls (dc < 0) is walked from its last
    // sample back, so along c the window only ever moves up; the positions
    // are the same fmaf(m, d, q0) as the forward's, visited in reverse
    const bool rev = dc < 0.0f;
    const float finc = rev ? -1.0f : 1.0f;
    const float fstart = rev ? (float)(m1 - 1) : (float)m0, fend = rev ? (float)(m0 - 1) : (float)m1;
    // the window starts at the first visited sample's cell
    float fm = rev ? (float)(m1 - 1 - off) : (float)(m0 + off);
    float fa, fb, fc;
    int cur = cell(fm, fa, fb, fc);
    auto step = [&](float fm) {
        const int i0 = cell(fm, fa, fb, fc);
        if (i0 != cur) {
            // one cell up along c: plane cur is complete and the upper plane
            // becomes the lower one; any other move (a, b changed, or the
            // wrap back to the first sample) flushes both planes
            const bool up = i0 == cur + sc;
            flush4(cur, lo);
            if (!up) flush4(cur + sc, hi);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                lo[j] = up ? hi[j] : 0.0f;
                hi[j] = 0.0f;
            }
            cur = i0;
        }
        const float ga = 1.0f - fa, gb = 1.0f - fb;
        const float vh = v * fc, vl = v - vh;
        const float w[4] = {ga * gb, fa * gb, ga * fb, fa * fb};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            lo[j] = fmaf(vl, w[j], lo[j]);
            hi[j] = fmaf(vh, w[j], hi[j]);
        }
    };
    // the sample index counts in FP32 (exact below 2^24) from the lane's
    // offset and wraps at the end of [m0, m1) back to its start: every lane
    // runs cnt iterations, so a wave's lanes stay busy together
    for (int k = 0; k < cnt; ++k) {
        step(fm);
        fm += finc;
        fm = fm == fend ? fstart : fm;
    }
    if (cnt > 0) {
        flush4(cur, lo);
        flush4(cur + sc, hi);
    }
}

__device__ __forceinline__ void scatter_global(const March& mr, int m0, int m1, const int n[3],
                                               double* __restrict__ x, const Bounds& bd, float v)
{
    const size_t sx = (size_t)n[0], sxy = (size_t)n[0] * n[1];
    for (int m = m0; m < m1; ++m) {
        const float fm = (float)m;
        const Cell s = cell_of(fmaf(fm, mr.st[0], mr.qs[0]), fmaf(fm, mr.st[1], mr.qs[1]),
                               fmaf(fm, mr.st[2], mr.qs[2]), bd);
        double* p = x + gindex(n, (int)s.i[0], (int)s.i[1], (int)s.i[2]);
        scatter8(p, sx, sxy, s, v, [](double* q, float a) { unsafeAtomicAdd(q, (double)a); });
    }
}

// ---------------------------------------------------------------- A x, A^T y
// Dynamic LDS of a march workgroup: the tile's compacted ray list (one
// uint32 per valid ray: item | aperture sample << 16), one FP64 word per
// pixel item (forward: the pixel's running sum; adjoint: its y value), then
// the brick.
struct Smem {
    uint32_t* list;
    double* item;
    unsigned char* brick;
};

__device__ __forceinline__ Smem smem_of(unsigned char* base, const CamDev& c)
{
    Smem m;
    m.list = reinterpret_cast<uint32_t*>(base);
    const int list_bytes = ((c.items_per_split * c.ru * c.rv * 4) + 15) & ~15;
    const int item_bytes = ((c.items_per_split * 8) + 15) & ~15;
    m.item = reinterpret_cast<double*>(base + list_bytes);
    m.brick = base + list_bytes + item_bytes;
    return m;
}

// Order-preserving compaction of the tile's valid rays into the LDS list.
// Pass (k, j) offers ray (j + rot) mod R of item k*kThreads + lane; the
// valid ones are appended in lane order, so a wave later marches rays that
// were neighbours in the tile.  Returns the list length (block-uniform).
template <bool kAdj>
__device__ int build_ray_list(const CamDev& c, int tile, const Smem& m, int* wsum)
{
    const int R = c.ru * c.rv;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rot = c.rotate ? (int)(threadIdx.x % (unsigned)R) : 0;
    int total = 0;
    for (int base = 0; base < c.items_per_split; base += kThreads) {
        const int item = base + threadIdx.x;
        int iu = 0, iv = 0;
        const bool have = item_pixel(c, tile, item, iu, iv);
        const bool lit = have && (!kAdj || m.item[item] != 0.0);
        for (int j = 0; j < R; ++j) {
            int rr = j + rot;
            rr = rr >= R ? rr - R : rr;
            bool ok = false;
            if (lit) {
                const int rv = rr / c.ru, ru = rr - rv * c.ru;
                Ray r;
                ok = make_ray(c, iu, iv, ru, rv, r);
            }
            const unsigned long long bal = __ballot(ok);
            const int pre = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wsum[wave] = __popcll(bal);
            __syncthreads();
            int off = total, all = 0;
#pragma unroll
            for (int w = 0; w < kThreads / 64; ++w) {
                off += (w < wave) ? wsum[w] : 0;
                all += wsum[w];
            }
            if (ok) m.list[off + pre] = (uint32_t)item | ((uint32_t)rr << 16);
            total += all;
            __syncthreads();
        }
    }
    return total;
}

// One tile of one camera: compact its rays, march them slab by slab, and
// write the tile's pixels (forward) or flush its bricks (adjoint).  Shared by
// the one-camera launch and the persistent batch kernel.
template <bool kAdj>
__device__ void march_tile(const CamDev& c, int tile, const float* __restrict__ in,
                           float* __restrict__ yout, double* __restrict__ xacc,
                           unsigned char* smem, int* wsum)
{
    const Smem m = smem_of(smem, c);
    const TileRec t = c.tiles[tile];
    const Bounds bd = bounds_of(c.n);

    // per-item words: forward sums start at 0, the adjoint reads y once
    for (int item = threadIdx.x; item < c.items_per_split; item += kThreads) {
        double v = 0.0;
        if (kAdj) {
            int iu, iv;
            if (item_pixel(c, tile, item, iu, iv)) v = (double)in[c.y_off + (size_t)iv * c.nu + iu];
        }
        m.item[item] = v;
    }
    __syncthreads();
    const int nrays = t.n_chunks > 0 ? build_ray_list<kAdj>(c, tile, m, wsum) : 0;

    // a lane's rays of the first two passes are the same in every slab, so
    // their set-up (make_ray, exact and slab-independent) is kept for the
    // whole tile instead of being redone per slab (later passes, for tiles
    // of more than 2 x 256 rays, redo it)
    Ray rp[2];
    int itemp[2] = {0, 0};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int e0 = p * kThreads, left = nrays - e0;
        if (left <= 0) break;
        const int parts = (kAdj || left >= kThreads) ? 1 : kThreads / left;
        if ((int)threadIdx.x < parts * min(left, kThreads)) {
            const int e = parts == 1 ? e0 + (int)threadIdx.x : e0 + (int)threadIdx.x % left;
            const uint32_t id = m.list[e];
            itemp[p] = (int)(id & 0xffffu);
            const int rr = (int)(id >> 16);
            int iu, iv;
            item_pixel(c, tile, itemp[p], iu, iv);
            const int rv = rr / c.ru, ru = rr - rv * c.ru;
            make_ray(c, iu, iv, ru, rv, rp[p]);
        }
    }

    for (int ch = 0; ch < t.n_chunks && nrays > 0; ++ch) {
        const BrickRec b = c.bricks[(size_t)tile * c.max_chunks + ch];
        const float za = slab_edge(t, ch, c.chunk);
        const float zb = slab_edge(t, ch + 1, c.chunk);
        const bool last = ch == t.n_chunks - 1;
        if (b.lds) {
            __syncthreads();
            if (kAdj) {
                if (c.adj_f32)
                    zero_brick(b, reinterpret_cast<float*>(m.brick));
                else
                    zero_brick(b, reinterpret_cast<double*>(m.brick));
            } else {
                stage_brick(b, c.n, in, reinterpret_cast<float*>(m.brick));
            }
            __syncthreads();
        }
        // whole passes give each lane one ray.  In the forward, a last,
        // partial pass of `left` rays splits each of them into kThreads / left
        // pieces of its sample range, so all waves share it instead of a few
        // lanes running whole rays (the pieces' sums meet in the pixel's FP64
        // LDS word).  The adjoint keeps whole rays: its plane window costs a
        // set-up and up to 8 closing atomics per piece, too much for pieces of
        // a few samples (measured slower), and 4 pieces of a last pass of at
        // most 64 rays, one per wave, measured no faster: other workgroups
        // fill the idle SIMDs.
        for (int e0 = 0; e0 < nrays; e0 += kThreads) {
            const int left = nrays - e0;
            const int parts = (kAdj || left >= kThreads) ? 1 : kThreads / left;
            if ((int)threadIdx.x >= parts * min(left, kThreads)) continue;
            const int e = parts == 1 ? e0 + (int)threadIdx.x : e0 + (int)threadIdx.x % left;
            const int part = parts == 1 ? 0 : (int)threadIdx.x / left;
            int item;
            Ray r;
            if (e0 == 0) {
                item = itemp[0];
                r = rp[0];
            } else if (e0 == kThreads) {
                item = itemp[1];
                r = rp[1];
            } else {
                const uint32_t id = m.list[e];
                item = (int)(id & 0xffffu);
                const int rr = (int)(id >> 16);
                int iu, iv;
                item_pixel(c, tile, item, iu, iv);
                const int rv = rr / c.ru, ru = rr - rv * c.ru;
                make_ray(c, iu, iv, ru, rv, r);
            }
            int m0 = sample_bound(r, za, c.S);
            int m1 = last ? c.S : sample_bound(r, zb, c.S);
            if (parts > 1 && m1 > m0) {
                const int len = m1 - m0;
                const int a = m0 + (len * part) / parts, b = m0 + (len * (part + 1)) / parts;
                m0 = a;
                m1 = b;
            }
            if (m0 >= m1) continue;
            const March mr = march_of(r);
            if (!kAdj) {
                const double s = b.lds ? gather_lds(mr, m0, m1, b, reinterpret_cast<const float*>(m.brick), bd)
                                       : gather_global(mr, m0, m1, c.n, in, bd);
                atomicAdd(&m.item[item], s * (double)r.w);
            } else {
                const float v = (float)m.item[item] * r.w;
                if (!b.lds)
                    scatter_global(mr, m0, m1, c.n, xacc, bd, v);
                else if (c.window && c.adj_f32)
                    scatter_lds_window(mr, m0, m1, b, reinterpret_cast<float*>(m.brick), v, c.skew);
                else if (c.window)
                    scatter_lds_window(mr, m0, m1, b, reinterpret_cast<double*>(m.brick), v, c.skew);
                else if (c.merge && c.adj_f32)
                    scatter_lds_merged(mr, m0, m1, b, reinterpret_cast<float*>(m.brick), bd, v, c.skew);
                else if (c.merge)
                    scatter_lds_merged(mr, m0, m1, b, reinterpret_cast<double*>(m.brick), bd, v, c.skew);
                else if (c.adj_f32)
                    scatter_lds(mr, m0, m1, b, reinterpret_cast<float*>(m.brick), bd, v, c.skew);
                else
                    scatter_lds(mr, m0, m1, b, reinterpret_cast<double*>(m.brick), bd, v, c.skew);
            }
        }
        if (kAdj && b.lds) {
            __syncthreads();
            if (c.adj_f32)
                flush_brick(b, c.n, reinterpret_cast<float*>(m.brick), xacc);
            else
                flush_brick(b, c.n, reinterpret_cast<double*>(m.brick), xacc);
        }
    }
    if (!kAdj) {
        __syncthreads();
        for (int item = threadIdx.x; item < c.items_per_split; item += kThreads) {
            int iu, iv;
            if (item_pixel(c, tile, item, iu, iv))
                yout[c.y_off + (size_t)iv * c.nu + iu] = (float)m.item[item];
        }
    }
    __syncthreads();   // the caller may reuse the LDS for the next tile
}

// Bounded to 5 waves per SIMD (at most 96 VGPRs): with adjoint bricks of up to
// 6144 floats, 5 workgroups share a CU's LDS, which hides more of the LDS
// atomics' latency than the few spilled registers cost.
template <bool kAdj>
__global__ __launch_bounds__(kThreads, 5) void k_march(CamDev c, const float* __restrict__ in,
                                                    float* __restrict__ yout,
                                                    double* __restrict__ xacc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wsum[kThreads / 64];
    march_tile<kAdj>(c, blockIdx.x, in, yout, xacc, smem, wsum);
}

// Persistent sweep over many (plan, camera, tile) items: each workgroup
// takes the next item from a global counter until the list is exhausted
// (every workgroup reaches the exit once the counter passes n_items).
// Items are ordered by decreasing estimated cost.
template <bool kAdj>
__global__ __launch_bounds__(kThreads, 5) void k_batch(const BatchCam* __restrict__ cams,
                                                    const uint32_t* __restrict__ items,
                                                    uint32_t n_items,
                                                    unsigned int* __restrict__ counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wsum[kThreads / 64];
    __shared__ uint32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t k = next;
        __syncthreads();
        if (k >= n_items) break;
        const uint32_t it = items[k];
        const int pc = __builtin_amdgcn_readfirstlane((int)(it >> kTileBits));
        const int tile = __builtin_amdgcn_readfirstlane((int)(it & ((1u << kTileBits) - 1u)));
        const BatchCam& bc = cams[pc];
        if (kAdj)
            march_tile<true>(bc.cam, tile, bc.y, nullptr, bc.xacc, smem, wsum);
        else
            march_tile<false>(bc.cam, tile, bc.x, bc.y, nullptr, smem, wsum);
    }
}

__global__ void k_zero_u32(unsigned int* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

__global__ void k_fill(float* p, uint64_t n, float v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Valid-ray count: one thread per pixel, block sum, one atomic per block.
__global__ __launch_bounds__(kThreads) void k_count(CamDev c, unsigned long long* counter)
{
    __shared__ unsigned int red[kThreads / 64];
    unsigned int cnt = 0;
    const long long npix = (long long)c.nu * c.nv;
    for (long long p = (long long)blockIdx.x * kThreads + threadIdx.x; p < npix;
         p += (long long)gridDim.x * kThreads) {
        const int iu = (int)(p % c.nu), iv = (int)(p / c.nu);
        for (int rv = 0; rv < c.rv; ++rv)
            for (int ru = 0; ru < c.ru; ++ru) {
                Ray r;
                cnt += make_ray(c, iu, iv, ru, rv, r) ? 1u : 0u;
            }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kThreads / 64; ++k) t += red[k];
        atomicAdd(counter, t);
    }
}

__global__ void k_fill64(double* p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// out[0] += sum (a - b)^2, out[1] += sum b^2 (FP64; the autotuner's parity gate)
__global__ void k_diff_sumsq(const float* __restrict__ a, const float* __restrict__ b, uint64_t n,
                             double* __restrict__ out)
{
    double d2 = 0.0, b2 = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double bv = b[i];
        const double dv = (double)a[i] - bv;
        d2 += dv * dv;
        b2 += bv * bv;
    }
    for (int off = 32; off > 0; off >>= 1) {
        d2 += __shfl_down(d2, off, 64);
        b2 += __shfl_down(b2, off, 64);
    }
    __shared__ double part[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wave] = d2;
        part[1][wave] = b2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int waves = (blockDim.x + 63) >> 6;
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < waves; ++w) {
            s0 += part[0][w];
            s1 += part[1][w];
        }
        atomicAdd(out, s0);
        atomicAdd(out + 1, s1);
    }
}

unsigned grid_for(uint64_t n)
{
    uint64_t blocks = (n + 255) / 256;
    return (unsigned)(blocks > 8192 ? 8192 : (blocks ? blocks : 1));
}


}  // namespace

hipError_t launch_fill(float* p, uint64_t n, float v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_count(const CamDev& c, unsigned long long* counter, hipStream_t s)
{
    const long long npix = (long long)c.nu * c.nv;
    long long blocks = (npix + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_count, dim3((unsigned)blocks), dim3(kThreads), 0, s, c, counter);
    return hipGetLastError();
}

hipError_t launch_setup(const CamDev& c, int dir, hipStream_t s)
{
    (void)dir;
    hipLaunchKernelGGL(k_setup, dim3(c.n_tiles), dim3(kThreads), 0, s, c,
                       const_cast<TileRec*>(c.tiles), const_cast<BrickRec*>(c.bricks));
    return hipGetLastError();
}

size_t march_lds_bytes(const CamDev& c, int dir)
{
    const size_t list_bytes = ((size_t)c.items_per_split * c.ru * c.rv * 4 + 15) & ~size_t(15);
    const size_t item_bytes = ((size_t)c.items_per_split * 8 + 15) & ~size_t(15);
    const size_t brick_bytes = (size_t)c.brick_cap * ((dir == LTM_ADJOINT && !c.adj_f32) ? 8 : 4);
    size_t lds = list_bytes + item_bytes + brick_bytes;
    if (c.groups_per_cu >= 2) {
        // reserve enough that k + 1 groups cannot share one CU's LDS
        const size_t cap = (size_t)kLdsPerCu / (size_t)(c.groups_per_cu + 1) + 512;
        lds = std::max(lds, (cap + 15) & ~size_t(15));
    }
    return lds;
}

hipError_t launch_project(const CamDev& c, const float* x, float* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_march<false>, dim3(c.n_tiles), dim3(kThreads),
                       march_lds_bytes(c, LTM_FORWARD), s, c, x, y, nullptr);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchCam* cams, const uint32_t* items, uint32_t n_items,
                        unsigned int* counter, int dir, int blocks, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counter, 1);
    if (dir == LTM_ADJOINT)
        hipLaunchKernelGGL(k_batch<true>, dim3(blocks), dim3(kThreads), lds, s, cams, items, n_items,
                           counter);
    else
        hipLaunchKernelGGL(k_batch<false>, dim3(blocks), dim3(kThreads), lds, s, cams, items, n_items,
                           counter);
    return hipGetLastError();
}

int batch_blocks_per_cu(int dir, size_t lds)
{
    int n = 0;
    hipError_t e = dir == LTM_ADJOINT
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<true>, kThreads, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<false>, kThreads, lds);
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_fill64(double* p, uint64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill64, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_diff_sumsq(const float* a, const float* b, uint64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill64, dim3(1), dim3(64), 0, s, out, (uint64_t)2);
    unsigned blocks = grid_for(n);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_diff_sumsq, dim3(blocks), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* a, float* b, uint64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

hipError_t launch_backproject(const CamDev& c, const float* y, double* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_march<true>, dim3(c.n_tiles), dim3(kThreads),
                       march_lds_bytes(c, LTM_ADJOINT), s, c, y, nullptr, x);
    return hipGetLastError();
}

}  // namespace ltm
