// Host side of the camera operator: descriptor validation, the FP64 ray
// constants of each camera, tilings, workspace layout and the C ABI of
// project / backproject.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "ltm_internal.h"

namespace ltm {

namespace {
thread_local std::string g_err;

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

uint64_t align256(uint64_t v) { return (v + 255u) & ~uint64_t(255u); }

// Lateral crossing of the main lens sL, slope after it u2 and position on
// the anchor plane sigma = sL + dA u2, for one of s/t, as functions of the
// lenslet-centre index cu, the pixel index du and the aperture sample g.
// The camera chain (single lens: detector -> lens; plenoptic: detector ->
// lenslet -> main lens) is linear in (cu, du, g) with no constant term, so
// evaluating it at unit inputs gives its coefficients.
struct Chain {
    double sL, u2, sigma;
};

Chain chain(const ltm_camera& c, double dA, double cu, double du, double g, double f_hex = 0.0)
{
    Chain r;
    const double p = c.pixel_pitch_mm;
    if (c.kind == LTM_PLENOPTIC_HEX) {
        const double cm = cu;                           // lenslet centre, mm
        const double a = cm + c.r_mla_mm * g;           // sample on that lenslet
        const double sd = du * p;
        const double u = (a - sd) / c.d_mla_det_mm;     // detector -> MLA
        const double u1 = u - (a - cm) / f_hex;         // refraction by its type
        r.sL = a + u1 * c.d_mla_mm;
        r.u2 = u1 - r.sL / c.f_main_mm;
    } else if (c.kind == LTM_SINGLE_LENS) {
        const double a = c.r_main_mm * g;              // aperture sample on the lens
        const double sd = du * p;                       // pixel centre
        const double u = (a - sd) / c.d_det_mm;         // propagation D
        r.u2 = u - a / c.f_main_mm;                     // thin-lens refraction
        r.sL = a;
    } else {
        const double P = (double)(c.det_nu / c.mla_nu) * p;  // lenslet pitch
        const double cm = cu * P;                       // lenslet centre
        const double a = cm + c.r_mla_mm * g;           // sample on the lenslet
        const double sd = du * p;
        const double u = (a - sd) / c.d_mla_det_mm;     // detector -> MLA
        const double u1 = u - (a - cm) / c.f_mla_mm;    // lenslet refraction
        r.sL = a + u1 * c.d_mla_mm;                     // MLA -> main lens
        r.u2 = u1 - r.sL / c.f_main_mm;                 // main-lens refraction
    }
    r.sigma = r.sL + dA * r.u2;
    return r;
}

ltm_status validate(const ltm_grid* g, const ltm_camera* cams, uint32_t n_cam)
{
    if (!g || !cams) return fail(LTM_ERR_INVALID, "null descriptor");
    if (n_cam == 0) return fail(LTM_ERR_INVALID, "no cameras");
    if (g->nx < 2 || g->ny < 2 || g->nz < 2)
        return fail(LTM_ERR_INVALID, "grid needs at least 2 voxels per axis");
    if ((uint64_t)g->nx * g->ny * g->nz > (1ull << 31))
        return fail(LTM_ERR_INVALID, "grid larger than 2^31 voxels");
    if (!(g->pitch_mm > 0.0) || !std::isfinite(g->pitch_mm))
        return fail(LTM_ERR_INVALID, "grid pitch must be positive");
    for (uint32_t i = 0; i < n_cam; ++i) {
        const ltm_camera& c = cams[i];
        const std::string who = "camera " + std::to_string(i) + ": ";
        if (c.kind != LTM_SINGLE_LENS && c.kind != LTM_PLENOPTIC && c.kind != LTM_PLENOPTIC_HEX)
            return fail(LTM_ERR_INVALID, who + "unknown kind");
        if (c.det_nu == 0 || c.det_nv == 0) return fail(LTM_ERR_INVALID, who + "empty detector");
        if ((uint64_t)c.det_nu * c.det_nv > (1ull << 30))
            return fail(LTM_ERR_INVALID, who + "detector larger than 2^30 pixels");
        if (c.rays_u == 0 || c.rays_v == 0 || c.rays_u * c.rays_v > (uint32_t)kMaxRays)
            return fail(LTM_ERR_INVALID, who + "need 1 <= rays_u*rays_v <= 64");
        if (c.samples == 0 || c.samples > (1u << 20))
            return fail(LTM_ERR_INVALID, who + "need 1 <= samples <= 2^20");
        if (!(c.pixel_pitch_mm > 0) || !(c.f_main_mm > 0) || !(c.r_main_mm > 0))
            return fail(LTM_ERR_INVALID, who + "pitch, focal length and radius must be positive");
        if (c.kind == LTM_SINGLE_LENS) {
            if (!(c.d_det_mm > 0)) return fail(LTM_ERR_INVALID, who + "d_det must be positive");
        } else if (c.kind == LTM_PLENOPTIC_HEX) {
            if (c.mla_nu == 0 || c.mla_nv == 0 || c.mla_nu > 65536 || c.mla_nv > 65536)
                return fail(LTM_ERR_INVALID, who + "need 1..65536 lenslets per row and rows");
            if (!(c.d_mla_mm > 0) || !(c.d_mla_det_mm > 0) || !(c.r_mla_mm > 0))
                return fail(LTM_ERR_INVALID, who + "lenslet distances and radius must be positive");
            if (9 * c.rays_u * c.rays_v > (uint32_t)kMaxRays)
                return fail(LTM_ERR_INVALID, who + "hexagonal cameras need rays_u*rays_v <= 7");
            double kmax = 0.0;
            for (int t = 0; t < 3; ++t) {
                const double f = c.f_hex_mm[t];
                if (!(f > 0) || !std::isfinite(f))
                    return fail(LTM_ERR_INVALID, who + "lenslet focal lengths must be positive");
                kmax = std::max(kmax, std::fabs(1.0 + c.d_mla_mm / c.d_mla_det_mm - c.d_mla_mm / f));
            }
            // a pixel d lit through lenslet c satisfies
            // |d - c| <= (e |d| + e (r_main + k r_mla)) / (1 + e); the 3 x 3
            // visited lenslets hold every lenslet closer than 1.5 row spacings
            const double e = c.d_mla_det_mm / c.d_mla_mm;
            const double hd = 0.5 * c.pixel_pitch_mm *
                              std::hypot((double)c.det_nu - 1.0, (double)c.det_nv - 1.0);
            const double reach = (e * hd + e * (c.r_main_mm + kmax * c.r_mla_mm)) / (1.0 + e);
            if (!(reach < 1.5 * std::sqrt(3.0) * c.r_mla_mm))
                return fail(LTM_ERR_INVALID, who + "light could reach pixels from beyond the "
                                                   "3 x 3 lenslets around them");
        } else {
            if (c.mla_nu == 0 || c.mla_nv == 0 || c.det_nu % c.mla_nu || c.det_nv % c.mla_nv)
                return fail(LTM_ERR_INVALID, who + "detector must be a multiple of the lenslet count");
            if (!(c.d_mla_mm > 0) || !(c.d_mla_det_mm > 0) || !(c.f_mla_mm > 0) || !(c.r_mla_mm > 0))
                return fail(LTM_ERR_INVALID, who + "lenslet distances, focal length and radius must be positive");
        }
        const double* e = c.axes;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double d = dot3(e + 3 * a, e + 3 * b) - (a == b ? 1.0 : 0.0);
                if (!(std::fabs(d) < 1e-9)) return fail(LTM_ERR_INVALID, who + "axes not orthonormal");
            }
        const double cx[3] = {e[1] * e[5] - e[2] * e[4], e[2] * e[3] - e[0] * e[5],
                              e[0] * e[4] - e[1] * e[3]};
        if (!(dot3(cx, e + 6) > 0.999999)) return fail(LTM_ERR_INVALID, who + "axes not right-handed");
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(c.lens_center_mm[a])) return fail(LTM_ERR_INVALID, who + "bad lens centre");
    }
    return LTM_OK;
}

// Rays each pixel visits: R, or 9 R for hexagonal cameras (3 x 3 lenslets).
uint64_t rays_per_pixel(const ltm_camera& c)
{
    const uint64_t R = (uint64_t)c.rays_u * c.rays_v;
    return c.kind == LTM_PLENOPTIC_HEX ? 9 * R : R;
}

// The optical axis lies along none of the grid's axes.
bool oblique(const ltm_camera& c)
{
    const double* ez = c.axes + 6;
    return std::fabs(ez[0]) < 1.0 - 1e-9 && std::fabs(ez[1]) < 1.0 - 1e-9 && std::fabs(ez[2]) < 1.0 - 1e-9;
}

ltm_tiling default_tiling(const ltm_grid& g, const ltm_camera& c, int dir)
{
    // Defaults from tiling sweeps on MI355X (the autotuner refines them):
    //  * forward: lanes of one lenslet / pixel block on adjacent lanes read
    //    the same LDS words (a bundle is a fraction of a voxel wide); no
    //    rotation of the starting angular sample; ~1-4k rays per group;
    //  * adjoint: staggered sample walks and two-plane windows along the
    //    rays' dominant axis (bits 3, 5) break the LDS atomic collisions of
    //    converging bundles and halve the atomics per cell step (4-14%
    //    faster than merged cells, bit 4, on the benchmark workloads); with many rays per
    //    pixel, lanes also walk across lenslets / blocks (bit 0) and the slabs
    //    get thinner.  The square-array plenoptic camera with R <= 4 keeps
    //    4x4 lenslets and 256 pixels per group (fastest on the 128^3 case).
    ltm_tiling t{};
    const uint64_t R = rays_per_pixel(c);
    const bool pl = c.kind == LTM_PLENOPTIC;
    const uint64_t k = pl ? (uint64_t)(c.det_nu / c.mla_nu) * (c.det_nv / c.mla_nv) : 0;
    t.block_u = t.block_v = 16;
    t.brick_floats = 8192;
    if (dir == LTM_FORWARD) {
        t.order = 2;
        t.brick_floats = 4096;
        t.tile_u = t.tile_v = pl ? (R <= 4 ? 2 : 1) : 1;
        t.chunk_mm = (c.kind == LTM_SINGLE_LENS ? 32.0 : 64.0) * g.pitch_mm;
        const uint64_t items = (uint64_t)t.tile_u * t.tile_v * (pl ? k : 256);
        const uint64_t target = R <= 4 ? 1024 : 4096;    // rays per group
        t.splits = 1;
        while (t.splits < items && items / t.splits * R > target) t.splits *= 2;
    } else if (pl && R <= 4 && oblique(c)) {
        // an optical axis oblique to the grid: bundles cross the slabs
        // diagonally, so smaller tiles and thinner slabs keep the bricks in
        // LDS, and lanes walk across lenslets (2.2-2.4 ms against 3.8-4.2 ms
        // for 2048^2 cameras at 30 and 60 deg on a 256^3 grid)
        t.tile_u = t.tile_v = 2;
        t.order = 1 | 2 | 8 | 32;
        t.chunk_mm = 16.0 * g.pitch_mm;
        t.splits = (uint32_t)std::max<uint64_t>(1, 4 * k / 256);    // 256 pixels per group
        t.brick_floats = 6144;   // 5 groups per CU (1.51 -> 1.48 ms at 30 deg on 128^3)
    } else if (pl && R <= 4) {
        t.tile_u = t.tile_v = 4;
        t.order = 2 | 8 | 32;
        t.chunk_mm = 32.0 * g.pitch_mm;
        t.splits = (uint32_t)std::max<uint64_t>(1, 16 * k / 256);   // 256 pixels per group
        t.brick_floats = 6144;   // 5 groups per CU (0.90 -> 0.86 ms on 128^3)
    } else {
        t.tile_u = t.tile_v = 2;
        t.block_u = t.block_v = 8;
        t.order = (c.kind == LTM_PLENOPTIC_HEX ? 0 : 1) | 2 | 8 | 32;
        t.chunk_mm = (c.kind == LTM_PLENOPTIC_HEX ? 32.0 : 16.0) * g.pitch_mm;
        const uint64_t items = 4 * (pl ? k : 64);
        t.splits = 1;
        while (t.splits < items && items / t.splits * R > 4096) t.splits *= 2;
    }
    // shrink until the ray list, pixel sums and brick fit one workgroup:
    // too many rays or pixels per group -> more splits (the brick keeps its
    // size: a smaller brick spills slabs to global memory); LDS overflow ->
    // shrink the larger of the ray list (more splits) and the brick
    const uint64_t ku = c.kind == LTM_PLENOPTIC ? c.det_nu / c.mla_nu : t.block_u;
    const uint64_t kv = c.kind == LTM_PLENOPTIC ? c.det_nv / c.mla_nv : t.block_v;
    const uint64_t items = (uint64_t)t.tile_u * t.tile_v * ku * kv;
    for (int guard = 0; guard < 64 && check_tiling(g, c, t) != LTM_OK; ++guard) {
        const uint64_t per = (items + t.splits - 1) / t.splits;
        if (per > 8ull * kThreads || per * R > (uint64_t)kMaxRayList) {
            t.splits *= 2;
        } else if (per * R >= t.brick_floats && per > 1) {
            t.splits *= 2;
        } else {
            t.brick_floats /= 2;
        }
    }
    clear_error();
    return t;
}

// Fill the FP32/FP64 ray constants of one camera (tiling-independent part).
void camera_constants(const ltm_grid& g, const ltm_camera& c, CamDev& d)
{
    std::memset(&d, 0, sizeof(d));
    d.kind = (int)c.kind;
    d.nu = (int)c.det_nu;
    d.nv = (int)c.det_nv;
    const bool hex = c.kind == LTM_PLENOPTIC_HEX;
    d.ru = (int)c.rays_u;
    d.grv = (int)c.rays_v;
    d.rv = hex ? 9 * (int)c.rays_v : (int)c.rays_v;
    d.S = (int)c.samples;
    d.n[0] = (int)g.nx;
    d.n[1] = (int)g.ny;
    d.n[2] = (int)g.nz;
    const double* es = c.axes;
    const double* et = c.axes + 3;
    const double* ez = c.axes + 6;
    const double* L = c.lens_center_mm;
    // anchor plane: the camera-depth plane through the grid centre (origin)
    const double dA = -dot3(L, ez);
    const double fh = hex ? c.f_hex_mm[0] : 0.0;
    const Chain k_c = chain(c, dA, 1, 0, 0, fh), k_d = chain(c, dA, 0, 1, 0, fh),
                k_g = chain(c, dA, 0, 0, 1, fh);
    const bool pl = c.kind != LTM_SINGLE_LENS;
    // hexagonal: cu counts lenslet pitches along s, cv row spacings along t
    const double hp = 2.0 * c.r_mla_mm, hh = std::sqrt(3.0) * c.r_mla_mm;
    const double cs = hex ? hp : 1.0, ct = hex ? hh : 1.0;
    d.Ac = pl ? (float)(k_c.sigma * cs) : 0.0f;
    d.Bc = pl ? (float)(k_c.u2 * cs) : 0.0f;
    d.Act = pl ? (float)(k_c.sigma * ct) : 0.0f;
    d.Bct = pl ? (float)(k_c.u2 * ct) : 0.0f;
    d.Ad = (float)k_d.sigma;
    d.Bd = (float)k_d.u2;
    d.Ag = (float)k_g.sigma;
    d.Bg = (float)k_g.u2;
    for (int t = 0; t < 3; ++t) {
        const Chain k = hex ? chain(c, dA, 0, 0, 1, c.f_hex_mm[t]) : k_g;
        d.hAg[t] = (float)k.sigma;
        d.hBg[t] = (float)k.u2;
        d.hLg[t] = k.sL;
    }
    if (hex) {
        d.rowf = (float)(c.pixel_pitch_mm / hh);
        d.colf = (float)(c.pixel_pitch_mm / hp);
        d.hmid = (int)(c.mla_nv / 2);
        d.hmu = (int)c.mla_nu;
        d.hmv = (int)c.mla_nv;
    }
    const double nn[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
    for (int a = 0; a < 3; ++a) {
        d.CA[a] = (float)((L[a] + dA * ez[a]) / g.pitch_mm + 0.5 * nn[a] - 0.5);
        d.Es[a] = (float)(es[a] / g.pitch_mm);
        d.Et[a] = (float)(et[a] / g.pitch_mm);
        d.Ez[a] = (float)(ez[a] / g.pitch_mm);
    }
    d.zlo = (float)(-dA);
    d.invR = (float)(1.0 / ((double)c.rays_u * c.rays_v));
    d.inv_ru = (float)(1.0 / c.rays_u);
    d.inv_rv = (float)(1.0 / c.rays_v);
    d.need_aperture = pl ? 1 : 0;
    d.Lc = pl ? k_c.sL * cs : 0.0;
    d.Lct = pl ? k_c.sL * ct : 0.0;
    d.Ld = k_d.sL;
    d.Lg = k_g.sL;
    d.r2 = c.r_main_mm * c.r_main_mm;
}

// Tiling-dependent fields.
void apply_tiling(const ltm_grid& g, const ltm_camera& c, const ltm_tiling& t, CamDev& d,
                  int& n_tiles, int& max_chunks, double chunk_floor)
{
    if (c.kind == LTM_PLENOPTIC) {
        d.ku = (int)(c.det_nu / c.mla_nu);
        d.kv = (int)(c.det_nv / c.mla_nv);
        d.mu = (int)c.mla_nu;
        d.mv = (int)c.mla_nv;
    } else {
        d.ku = (int)t.block_u;
        d.kv = (int)t.block_v;
        d.mu = (int)((c.det_nu + t.block_u - 1) / t.block_u);
        d.mv = (int)((c.det_nv + t.block_v - 1) / t.block_v);
    }
    d.tile_u = (int)t.tile_u;
    d.tile_v = (int)t.tile_v;
    d.order = (int)t.order;
    d.rotate = (t.order & 2) ? 0 : 1;
    d.adj_f32 = (t.order & 4) ? 1 : 0;
    d.skew = (t.order & 8) ? ((t.order & 64) ? 2 : 1) : 0;
    d.merge = (t.order & 16) ? 1 : 0;
    d.window = (t.order & 32) ? 1 : 0;
    d.groups_per_cu = (int)t.groups_per_cu;
    d.splits = (int)t.splits;
    d.items = d.tile_u * d.tile_v * d.ku * d.kv;
    d.items_per_split = (d.items + d.splits - 1) / d.splits;
    d.tiles_u = (d.mu + d.tile_u - 1) / d.tile_u;
    d.tiles_v = (d.mv + d.tile_v - 1) / d.tile_v;
    d.n_tiles = d.tiles_u * d.tiles_v * d.splits;
    d.brick_cap = (int)t.brick_floats;
    d.chunk = (float)t.chunk_mm;
    const double diag = g.pitch_mm * std::sqrt((double)g.nx * g.nx + (double)g.ny * g.ny +
                                               (double)g.nz * g.nz);
    d.max_chunks = (int)std::ceil(diag / std::min(chunk_floor, t.chunk_mm)) + 2;
    n_tiles = d.n_tiles;
    max_chunks = d.max_chunks;
}

void layout(ltm_plan* p)
{
    uint64_t off = 0;
    for (auto& c : p->cams) {
        for (int dir = 0; dir < 2; ++dir) {
            CamDev tmp = c.dev;
            apply_tiling(p->grid, c.desc, c.tiling[dir], tmp, c.n_tiles[dir], c.max_chunks[dir],
                         c.chunk_floor[dir]);
            c.tiles_off[dir] = off;
            off = align256(off + sizeof(TileRec) * (uint64_t)c.n_tiles[dir]);
            c.bricks_off[dir] = off;
            off = align256(off + sizeof(BrickRec) * (uint64_t)c.n_tiles[dir] * c.max_chunks[dir]);
        }
    }
    p->counter_off = off;
    off += 256;
    p->accum_off = off;
    off = align256(off + sizeof(double) * p->n_vox);
    p->ws_bytes = off;
}

}  // namespace

ltm_status check_tiling(const ltm_grid& g, const ltm_camera& c, const ltm_tiling& t)
{
    // the kernels form brick indices as FP32 sums of a grid coordinate times a
    // brick stride (at most brick_floats); every such product must stay an
    // exact FP32 integer
    const uint64_t nmax = std::max<uint64_t>(g.nx, std::max<uint64_t>(g.ny, g.nz)) + 2;
    if (nmax * std::max<uint64_t>(t.brick_floats, 1) >= (1ull << 24))
        return fail(LTM_ERR_INVALID, "grid axis times brick_floats must stay below 2^24");
    if (t.tile_u == 0 || t.tile_v == 0 || t.splits == 0)
        return fail(LTM_ERR_INVALID, "tiling sizes must be positive");
    if (c.kind != LTM_PLENOPTIC && (t.block_u == 0 || t.block_v == 0))
        return fail(LTM_ERR_INVALID, "single-lens and hexagonal tilings need block sizes");
    if (t.order > 127) return fail(LTM_ERR_INVALID, "tiling order flags must be 0..127");
    if (t.groups_per_cu == 1 || t.groups_per_cu > 8)
        return fail(LTM_ERR_INVALID, "groups_per_cu must be 0 or 2..8");
    if (t.brick_floats > (uint32_t)kMaxBrickFloats)
        return fail(LTM_ERR_INVALID, "brick larger than 64 KiB of LDS");
    if (!(t.chunk_mm > 0) || !std::isfinite(t.chunk_mm))
        return fail(LTM_ERR_INVALID, "chunk_mm must be positive");
    const uint64_t ku = c.kind == LTM_PLENOPTIC ? c.det_nu / c.mla_nu : t.block_u;
    const uint64_t kv = c.kind == LTM_PLENOPTIC ? c.det_nv / c.mla_nv : t.block_v;
    const uint64_t items = (uint64_t)t.tile_u * t.tile_v * ku * kv;
    const uint64_t per = (items + t.splits - 1) / t.splits;
    if (per == 0 || per > 8ull * kThreads)
        return fail(LTM_ERR_INVALID, "a workgroup may own at most 2048 pixels of a tile");
    const uint64_t R = rays_per_pixel(c);
    if (per * R > (uint64_t)kMaxRayList)
        return fail(LTM_ERR_INVALID, "a workgroup may own at most 8192 rays (pixels x R)");
    const uint64_t lds = ((per * R * 4 + 15) & ~15ull) + ((per * 8 + 15) & ~15ull) +
                         (uint64_t)t.brick_floats * 4;
    if (lds > (uint64_t)kMaxLdsBytes)
        return fail(LTM_ERR_INVALID, "ray list, pixel sums and brick exceed 64 KiB of LDS");
    if (items > (1ull << 30)) return fail(LTM_ERR_INVALID, "tile too large");
    return LTM_OK;
}

ltm_status validate_cameras(const ltm_grid* g, const ltm_camera* cams, uint32_t n_cam)
{
    return validate(g, cams, n_cam);
}

ltm_status fail(ltm_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

ltm_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return LTM_ERR_DEVICE;
}

void clear_error() { g_err.clear(); }

CamDev bound_dev(const ltm_plan* p, const CamHost& c, int dir)
{
    CamDev d = c.dev;
    int nt, mc;
    apply_tiling(p->grid, c.desc, c.tiling[dir], d, nt, mc, c.chunk_floor[dir]);
    if (dir == LTM_ADJOINT && !d.adj_f32) d.brick_cap /= 2;   // FP64 brick in the same LDS budget
    if (p->sub_n > 1) {
        // mean over the subset's samples: the view-subset operator (K/|S|) A_S
        const int R = d.ru * d.grv;
        int ns = 0;
        for (int r = 0; r < R; ++r) ns += (r % (int)p->sub_n == (int)p->sub_i);
        d.sub_n = (int)p->sub_n;
        d.sub_i = (int)p->sub_i;
        d.invR = ns > 0 ? (float)(1.0 / ns) : 0.0f;
    } else {
        d.sub_n = 1;
        d.sub_i = 0;
    }
    d.tiles = reinterpret_cast<const TileRec*>(p->ws + c.tiles_off[dir]);
    d.bricks = reinterpret_cast<const BrickRec*>(p->ws + c.bricks_off[dir]);
    d.y_off = c.y_off;
    return d;
}

const char* last_error() { return g_err.c_str(); }

}  // namespace ltm

using namespace ltm;

extern "C" {

uint32_t ltm_abi_version(void) { return LTM_ABI_VERSION; }

const char* ltm_last_error(void) { return ltm::last_error(); }

ltm_status ltm_plan_create(const ltm_grid* grid, const ltm_camera* cams, uint32_t n_cam,
                           ltm_plan** out)
{
    if (!out) return fail(LTM_ERR_INVALID, "null output pointer");
    *out = nullptr;
    ltm_status s = validate(grid, cams, n_cam);
    if (s != LTM_OK) return s;
    ltm_plan* p = new (std::nothrow) ltm_plan();
    if (!p) return fail(LTM_ERR_INVALID, "out of host memory");
    p->grid = *grid;
    p->n_vox = (uint64_t)grid->nx * grid->ny * grid->nz;
    uint64_t yoff = 0;
    for (uint32_t i = 0; i < n_cam; ++i) {
        CamHost c{};
        c.desc = cams[i];
        for (int dir = 0; dir < 2; ++dir) {
            c.tiling[dir] = default_tiling(*grid, cams[i], dir);
            c.adapt[dir] = true;
            c.chunk_floor[dir] = c.tiling[dir].chunk_mm / 8.0;
        }
        camera_constants(*grid, cams[i], c.dev);
        c.npix = (uint64_t)cams[i].det_nu * cams[i].det_nv;
        c.y_off = yoff;
        yoff += c.npix;
        p->cams.push_back(c);
    }
    p->n_meas = yoff;
    layout(p);
    clear_error();
    *out = p;
    return LTM_OK;
}

void ltm_plan_destroy(ltm_plan* plan) { delete plan; }

ltm_status ltm_plan_sizes(const ltm_plan* p, uint64_t* n_voxels, uint64_t* n_meas)
{
    if (!p) return fail(LTM_ERR_INVALID, "null plan");
    if (n_voxels) *n_voxels = p->n_vox;
    if (n_meas) *n_meas = p->n_meas;
    return LTM_OK;
}

ltm_status ltm_plan_workspace_bytes(const ltm_plan* p, uint64_t* bytes)
{
    if (!p || !bytes) return fail(LTM_ERR_INVALID, "null argument");
    *bytes = p->ws_bytes;
    return LTM_OK;
}

ltm_status ltm_plan_bind_workspace(ltm_plan* p, void* ws, uint64_t bytes, void* stream)
{
    if (!p) return fail(LTM_ERR_INVALID, "null plan");
    if (!ws || bytes < p->ws_bytes)
        return fail(LTM_ERR_WORKSPACE, "workspace of " + std::to_string(p->ws_bytes) +
                                           " bytes required");
    if (reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(LTM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    p->ws = static_cast<char*>(ws);
    p->bound = false;
    ++p->generation;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<TileRec> tiles;
    std::vector<BrickRec> bricks;
    for (auto& c : p->cams)
        for (int dir = 0; dir < 2; ++dir) {
            for (;;) {
                const CamDev d = bound_dev(p, c, dir);
                hipError_t e = launch_setup(d, dir, s);
                if (e != hipSuccess) return hip_fail(e, "tile setup");
                if (!c.adapt[dir] || c.tiling[dir].chunk_mm * 0.5 < c.chunk_floor[dir] * 0.999) break;
                // default tilings: halve the slab depth while more than 1% of the
                // used slabs have voxel boxes too large for LDS (global memory is
                // many times slower, oblique poses need thinner slabs)
                tiles.resize(d.n_tiles);
                bricks.resize((size_t)d.n_tiles * d.max_chunks);
                e = hipMemcpyAsync(tiles.data(), d.tiles, tiles.size() * sizeof(TileRec),
                                   hipMemcpyDeviceToHost, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(bricks.data(), d.bricks, bricks.size() * sizeof(BrickRec),
                                       hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_fail(e, "tile setup readback");
                uint64_t used = 0, spill = 0;
                for (int t = 0; t < d.n_tiles; ++t)
                    for (int ch = 0; ch < tiles[t].n_chunks; ++ch) {
                        ++used;
                        spill += bricks[(size_t)t * d.max_chunks + ch].lds ? 0 : 1;
                    }
                if (spill * 100 <= used) break;
                c.tiling[dir].chunk_mm *= 0.5;
            }
        }
    p->bound = true;
    clear_error();
    return LTM_OK;
}

ltm_status ltm_plan_get_tiling(const ltm_plan* p, uint32_t dir, uint32_t cam, ltm_tiling* out)
{
    if (!p || !out) return fail(LTM_ERR_INVALID, "null argument");
    if (dir > 1 || cam >= p->cams.size()) return fail(LTM_ERR_INVALID, "bad direction or camera");
    *out = p->cams[cam].tiling[dir];
    return LTM_OK;
}

ltm_status ltm_plan_set_tiling(ltm_plan* p, uint32_t dir, uint32_t cam, const ltm_tiling* t)
{
    if (!p || !t) return fail(LTM_ERR_INVALID, "null argument");
    if (dir > 1 || cam >= p->cams.size()) return fail(LTM_ERR_INVALID, "bad direction or camera");
    ltm_status s = check_tiling(p->grid, p->cams[cam].desc, *t);
    if (s != LTM_OK) return s;
    p->cams[cam].tiling[dir] = *t;
    p->cams[cam].adapt[dir] = false;
    p->cams[cam].chunk_floor[dir] = t->chunk_mm;
    layout(p);
    p->bound = false;
    p->ws = nullptr;
    ++p->generation;
    clear_error();
    return LTM_OK;
}

ltm_status ltm_plan_valid_rays(ltm_plan* p, uint32_t cam, uint64_t* rays, void* stream)
{
    if (!p || !rays) return fail(LTM_ERR_INVALID, "null argument");
    if (cam >= p->cams.size()) return fail(LTM_ERR_INVALID, "bad camera");
    if (!p->bound) return fail(LTM_ERR_WORKSPACE, "plan has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* ctr = reinterpret_cast<unsigned long long*>(p->ws + p->counter_off);
    hipError_t e = hipMemsetAsync(ctr, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) e = launch_count(bound_dev(p, p->cams[cam], LTM_FORWARD), ctr, s);
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, ctr, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "count rays");
    *rays = h;
    return LTM_OK;
}

ltm_status ltm_plan_set_ray_subset(ltm_plan* p, uint32_t n_subsets, uint32_t index)
{
    if (!p) return fail(LTM_ERR_INVALID, "null plan");
    if (n_subsets == 0 || n_subsets > (uint32_t)kMaxRays || (n_subsets > 1 && index >= n_subsets))
        return fail(LTM_ERR_INVALID, "need 1 <= n_subsets <= 64 and index < n_subsets");
    p->sub_n = n_subsets;
    p->sub_i = n_subsets > 1 ? index : 0;
    return LTM_OK;
}

ltm_status ltm_project(ltm_plan* p, const float* x, float* y, void* stream)
{
    if (!p || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (!p->bound) return fail(LTM_ERR_WORKSPACE, "plan has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (auto& c : p->cams) {
        hipError_t e = launch_project(bound_dev(p, c, LTM_FORWARD), x, y, s);
        if (e != hipSuccess) return hip_fail(e, "project");
    }
    return LTM_OK;
}

ltm_status ltm_backproject(ltm_plan* p, const float* y, float* x, void* stream)
{
    if (!p || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (!p->bound) return fail(LTM_ERR_WORKSPACE, "plan has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* acc = reinterpret_cast<double*>(p->ws + p->accum_off);
    hipError_t e = launch_fill64(acc, p->n_vox, s);
    if (e != hipSuccess) return hip_fail(e, "zero accumulator");
    for (auto& c : p->cams) {
        e = launch_backproject(bound_dev(p, c, LTM_ADJOINT), y, acc, s);
        if (e != hipSuccess) return hip_fail(e, "backproject");
    }
    e = launch_to_f32(acc, x, p->n_vox, s);
    if (e != hipSuccess) return hip_fail(e, "convert");
    return LTM_OK;
}

ltm_status ltm_backproject_noalloc(ltm_plan* p, const float* y, float* x, void* stream)
{
    if (!p || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (p->n_vox > kScratchVoxels)
        return fail(LTM_ERR_INVALID, "volume of " + std::to_string(p->n_vox) +
                                         " voxels exceeds the fixed accumulator's " +
                                         std::to_string(kScratchVoxels));
    if (!p->bound) return fail(LTM_ERR_WORKSPACE, "plan has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* acc = nullptr;
    hipError_t e = scratch_accumulator(&acc);
    if (e != hipSuccess) return hip_fail(e, "fixed accumulator address");
    e = launch_fill64(acc, p->n_vox, s);
    if (e != hipSuccess) return hip_fail(e, "zero accumulator");
    for (auto& c : p->cams) {
        e = launch_backproject(bound_dev(p, c, LTM_ADJOINT), y, acc, s);
        if (e != hipSuccess) return hip_fail(e, "backproject");
    }
    e = launch_to_f32(acc, x, p->n_vox, s);
    if (e != hipSuccess) return hip_fail(e, "convert");
    return LTM_OK;
}

}  // extern "C"
