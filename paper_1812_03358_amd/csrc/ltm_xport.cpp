// Host side of the light-field transport operator: validation, the FP64
// evaluation of the transport tables' entries, banded FP32 tables and their
// exact transposes, workspace layout.
//
// Optics of a head-on single-lens camera, rays running from the detector
// into the scene along camera depth z (propagation T_d: s' = s + d u;
// refraction R_f: u' = u - s/f).  A slice at depth z reaches the angular
// plane (the lens) through X^{0q} = (T_z R_f)^{-1}: s_L = s - z u, and the
// detector D behind the lens through X^{pq} = T_D^{-1} X^{0q}:
//   s_d = (1 - D/F) s + (D z / F - z - D) u;
// the detector reaches the angular plane through X^{0d} = T_D.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ltm_internal.h"
#include "ltm_xport.h"

struct ltm_xport {
    ltm_grid grid;
    ltm_camera cam;
    uint32_t basis;
    int kt;                        // angular rows (rays_v)
    // host tables (FP32 values, built once)
    struct Band {
        int rows = 0, width = 0;
        std::vector<int32_t> start;   // pairs * rows
        std::vector<float> w;         // pairs * width * rows (weight-major)
    } bt, cs, cst, btt;
    // posed cameras: rotation of the natural grid into the camera's axes
    bool rot = false;
    int nxr = 0, nyr = 0, nzr = 0;          // transport grid (rotated, or the natural one)
    Band ez, ezt, ex, ext;
    uint64_t off_bt_s = 0, off_bt_w = 0, off_cs_s = 0, off_cs_w = 0, off_cst_s = 0, off_cst_w = 0,
             off_btt_s = 0, off_btt_w = 0, off_mid = 0, ws_bytes = 0;
    uint64_t off_ez_s = 0, off_ez_w = 0, off_ezt_s = 0, off_ezt_w = 0, off_ex_s = 0, off_ex_w = 0,
             off_ext_s = 0, off_ext_w = 0, off_r1 = 0, off_xr = 0;
    char* ws = nullptr;
    bool bound = false;
};

namespace ltm {
namespace {

// One axis of the transport from a slice to the detector for one angular
// cell: the blur kernel g (Dirac: a box on [tau1, tau2); pillbox: a trapezoid
// on tau1..tau4), its height h and magnification mag = 1/alpha.
struct Kernel1D {
    int basis;
    double tau[4];
    double h, mag;
};

Kernel1D kernel_of(int basis, double z, double D, double F, double sk, double d0, double dp)
{
    const double qss = 1.0, qsu = -z, qbar = 0.0;                  // X^{0q}
    const double pss = 1.0 - D / F, psu = D * z / F - z - D, pbar = 0.0;  // X^{pq}
    Kernel1D k{};
    k.basis = basis;
    if (basis == LTM_BASIS_DIRAC) {
        const double alpha = pss - qss * psu / qsu;
        const double beta = pbar + psu * (sk - qbar) / qsu;
        const double a = (0.5 * dp - beta) / alpha, b = (-0.5 * dp - beta) / alpha;
        k.tau[0] = k.tau[1] = std::min(a, b);
        k.tau[2] = k.tau[3] = std::max(a, b);
        k.h = d0 / std::fabs(qsu);
        k.mag = 1.0 / alpha;
    } else {
        const double alpha = pss - psu * qss / qsu;
        const double beta = psu / qsu;
        const double gamma = pbar - psu * qbar / qsu;
        int n = 0;
        for (double sp : {1.0, -1.0})
            for (double s0 : {1.0, -1.0})
                k.tau[n++] = (sp * 0.5 * dp - beta * (sk - s0 * 0.5 * d0) - gamma) / alpha;
        std::sort(k.tau, k.tau + 4);
        k.h = psu == 0.0 ? std::fabs(d0 / qsu) : std::min(std::fabs(d0 / qsu), std::fabs(dp / psu));
        k.mag = 1.0 / alpha;
    }
    return k;
}

// Antiderivative of g from -infinity (g rises linearly on [t0, t1], is 1 on
// [t1, t2] and falls linearly on [t2, t3]; a zero-width ramp is a step).
double G(const Kernel1D& k, double x)
{
    const double t0 = k.tau[0], t1 = k.tau[1], t2 = k.tau[2], t3 = k.tau[3];
    const double up = 0.5 * (t1 - t0), flat = t2 - t1, down = 0.5 * (t3 - t2);
    if (x <= t0) return 0.0;
    if (x <= t1) return 0.5 * (x - t0) * (x - t0) / (t1 - t0);
    if (x <= t2) return up + (x - t1);
    if (x <= t3) {
        const double r = x - t2;
        return up + flat + r - 0.5 * r * r / (t3 - t2);
    }
    return up + flat + down;
}

// Entries of one factor row: destination centre si; source cells of size dq
// with left edges (j - n/2) dq, j = 0..n-1.  Appends (j, value) pairs.
void factor_row(const Kernel1D& k, double si, double dq, int n, double scale,
                std::vector<std::pair<int, double>>& out)
{
    const double c = k.mag * si;
    const double lo = (c + k.tau[0]) / dq + 0.5 * n, hi = (c + k.tau[3]) / dq + 0.5 * n;
    const int j0 = std::max(0, (int)std::floor(lo) - 1), j1 = std::min(n - 1, (int)std::floor(hi) + 1);
    for (int j = j0; j <= j1; ++j) {
        const double a = (j - 0.5 * n) * dq - c;
        const double v = k.h * (G(k, a + dq) - G(k, a)) * scale;
        if (v != 0.0) out.emplace_back(j, v);
    }
}

double axis_volume(int basis, double D, double dp, double d0)
{
    const double ss = 1.0, su = D;                                   // X^{0d} = T_D
    if (basis == LTM_BASIS_DIRAC) return dp * std::fabs(d0 / su);
    const double m = std::max(d0 / (2.0 * std::fabs(su)), dp * std::fabs(ss / su) / 2.0);
    const double h = std::min(dp, d0 / std::fabs(ss));
    return 2.0 * m * h;
}

using Rows = std::vector<std::vector<std::pair<int, double>>>;   // per row: (column, value)

// Pack per-(pair, row) sparse rows into a banded FP32 table.
void pack(const std::vector<Rows>& pairs, int rows, ltm_xport::Band& b)
{
    int width = 1;
    for (const Rows& pr : pairs)
        for (const auto& r : pr)
            if (!r.empty()) width = std::max(width, r.back().first - r.front().first + 1);
    b.rows = rows;
    b.width = width;
    b.start.assign(pairs.size() * rows, 0);
    b.w.assign(pairs.size() * (size_t)width * rows, 0.0f);
    for (size_t p = 0; p < pairs.size(); ++p)
        for (int r = 0; r < rows; ++r) {
            const auto& e = pairs[p][r];
            if (e.empty()) continue;
            const int st = e.front().first;
            b.start[p * rows + r] = st;
            for (const auto& kv : e)
                b.w[(p * width + (kv.first - st)) * (size_t)rows + r] = (float)kv.second;
        }
}

// Exact transpose of a banded table (same FP32 values): columns -> rows.
void transpose(const ltm_xport::Band& a, int pairs, int cols, ltm_xport::Band& t)
{
    std::vector<Rows> tp(pairs, Rows(cols));
    for (int p = 0; p < pairs; ++p)
        for (int r = 0; r < a.rows; ++r)
            for (int k = 0; k < a.width; ++k) {
                const float v = a.w[((size_t)p * a.width + k) * a.rows + r];
                const int c = a.start[(size_t)p * a.rows + r] + k;
                if (v != 0.0f && c < cols) tp[p][c].emplace_back(r, (double)v);
            }
    pack(tp, cols, t);
}

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// Rotated perspectives: the L2 projection of boxes of size h displaced by
// shift + t, t uniform over [-width/2, width/2] (the shear across the
// column's other coordinate), onto boxes of size h: the mean of the box
// overlap fraction hat(d) = max(0, 1 - |d|) over the window, a piecewise
// quadratic in d = (zi - zj + shift) / h.
double hat_integral(double d)
{
    if (d <= -1.0) return 0.0;
    if (d <= 0.0) return 0.5 * (d + 1.0) * (d + 1.0);
    if (d < 1.0) return 1.0 - 0.5 * (1.0 - d) * (1.0 - d);
    return 1.0;
}

double shear_entry(double zi, double zj, double h, double shift, double width)
{
    const double d = (zi - zj + shift) / h;
    if (width == 0.0) return std::max(0.0, 1.0 - std::fabs(d));
    const double w = width / h;
    return (hat_integral(d + 0.5 * w) - hat_integral(d - 0.5 * w)) / w;
}

// One column of a shear: rows = output centres zi, columns = input centres zj.
Rows shear_rows(int n_out, int n_in, double h, double shift, double width)
{
    Rows rows(n_out);
    for (int i = 0; i < n_out; ++i) {
        const double zi = (i + 0.5 - 0.5 * n_out) * h;
        for (int j = 0; j < n_in; ++j) {
            const double v = shear_entry(zi, (j + 0.5 - 0.5 * n_in) * h, h, shift, width);
            if (v != 0.0) rows[i].emplace_back(j, v);
        }
    }
    return rows;
}

}  // namespace
}  // namespace ltm

using namespace ltm;

extern "C" {

ltm_status ltm_xport_create(const ltm_grid* g, const ltm_camera* c, uint32_t basis, ltm_xport** out)
{
    if (!g || !c || !out) return fail(LTM_ERR_INVALID, "null argument");
    *out = nullptr;
    if (basis > LTM_BASIS_PILLBOX) return fail(LTM_ERR_INVALID, "basis must be Dirac or pillbox");
    // the cell grid may be finer than the ray operator's R <= 64
    if (c->rays_u == 0 || c->rays_v == 0 || c->rays_u > 64 || c->rays_v > 64)
        return fail(LTM_ERR_INVALID, "need 1 <= rays_u, rays_v <= 64 angular cells");
    ltm_camera one = *c;
    one.rays_u = one.rays_v = 1;
    ltm_status st = validate_cameras(g, &one, 1);
    if (st != LTM_OK) return st;
    if (c->kind != LTM_SINGLE_LENS)
        return fail(LTM_ERR_UNSUPPORTED, "the transport operator models single-lens cameras");
    // pose: azimuth phi about the grid's y axis, |phi| <= 45 deg, the lens on
    // the camera axis through the grid centre
    const double* es = c->axes;
    const double* et = c->axes + 3;
    const double* ez = c->axes + 6;
    if (std::fabs(et[1] - 1.0) > 1e-12 || std::fabs(es[1]) > 1e-12 || std::fabs(ez[1]) > 1e-12)
        return fail(LTM_ERR_UNSUPPORTED, "the transport operator needs an azimuth pose (e_t = +y)");
    const double phi = std::atan2(ez[0], ez[2]);
    if (std::fabs(phi) > 0.25 * M_PI + 1e-12)
        return fail(LTM_ERR_UNSUPPORTED, "the transport operator's shear rotation needs |phi| <= 45 deg");
    const double L = -(c->lens_center_mm[0] * ez[0] + c->lens_center_mm[1] * ez[1] +
                       c->lens_center_mm[2] * ez[2]);
    for (int a = 0; a < 3; ++a)
        if (std::fabs(c->lens_center_mm[a] + L * ez[a]) > 1e-9 * std::fabs(L))
            return fail(LTM_ERR_UNSUPPORTED, "the transport operator needs the lens on the camera axis through the grid centre");
    const double cphi = std::cos(phi), sphi = std::sin(phi);
    const bool rot = std::fabs(sphi) > 1e-15;
    const double sa = -sphi * cphi, sb = sphi / cphi;           // S_z: z += sa x, S_x: x += sb z
    const double d = g->pitch_mm;
    const double hx = rot ? d / cphi : d, hy = d, hz = rot ? d * cphi : d;
    int nzr = (int)g->nz, nxr = (int)g->nx;
    if (rot) {
        nzr = (int)g->nz + 2 * (int)std::ceil(0.5 * std::fabs(sa) * g->nx * hx / hz) + 2;
        nxr = (int)g->nx + 2 * (int)std::ceil(0.5 * std::fabs(sb) * nzr * hz / hx) + 2;
    }
    if (!(L - 0.5 * nzr * hz > 0.0))
        return fail(LTM_ERR_INVALID, "every slice must lie in front of the lens");
    const uint64_t mid = (uint64_t)nzr * c->rays_v * c->det_nv * (uint64_t)nxr;
    if (mid > (1ull << 34)) return fail(LTM_ERR_INVALID, "intermediate larger than 2^34 values");
    ltm_xport* t = new ltm_xport();
    t->grid = *g;
    t->cam = *c;
    t->basis = basis;
    t->kt = (int)c->rays_v;
    t->rot = rot;
    t->nxr = nxr;
    t->nyr = (int)g->ny;
    t->nzr = nzr;

    // transport on the (rotated) grid: voxel sizes hx (s), hy (t), hz (depth)
    const int nx = nxr, ny = (int)g->ny, nz = nzr;
    const int nu = (int)c->det_nu, nv = (int)c->det_nv, Ks = (int)c->rays_u, Kt = (int)c->rays_v;
    const double dp = c->pixel_pitch_mm, D = c->d_det_mm, F = c->f_main_mm;
    const double r = c->r_main_mm, d0s = 2.0 * r / Ks, d0t = 2.0 * r / Kt;
    const double Vd = axis_volume((int)basis, D, dp, d0s) * axis_volume((int)basis, D, dp, d0t);
    const double scale = hz / ((double)Ks * Kt * Vd);
    std::vector<Rows> bt_pairs, cs_pairs;
    bt_pairs.reserve((size_t)nz * Kt);
    cs_pairs.reserve((size_t)nz * Kt);
    std::vector<std::pair<int, double>> tmp;
    for (int iz = 0; iz < nz; ++iz) {
        const double z = L + (iz + 0.5 - 0.5 * nz) * hz;
        for (int kt = 0; kt < Kt; ++kt) {
            const double tk = (kt + 0.5) * d0t - r;
            // t factor (shared by the row's cells; unit scale)
            Rows bt(nv);
            const Kernel1D kt1 = kernel_of((int)basis, z, D, F, tk, d0t, dp);
            for (int v = 0; v < nv; ++v) factor_row(kt1, (v + 0.5 - 0.5 * nv) * dp, hy, ny, 1.0, bt[v]);
            // s factors of the row's unmasked cells, summed, with the scale
            std::vector<std::vector<double>> dense(nu);
            std::vector<int> lo(nu, nx), hi(nu, -1);
            for (int ks = 0; ks < Ks; ++ks) {
                const double sk = (ks + 0.5) * d0s - r;
                if (sk * sk + tk * tk > r * r) continue;              // aperture mask
                const Kernel1D k1 = kernel_of((int)basis, z, D, F, sk, d0s, dp);
                for (int u = 0; u < nu; ++u) {
                    tmp.clear();
                    factor_row(k1, (u + 0.5 - 0.5 * nu) * dp, hx, nx, scale, tmp);
                    if (dense[u].empty() && !tmp.empty()) dense[u].assign(nx, 0.0);
                    for (const auto& kv : tmp) {
                        dense[u][kv.first] += kv.second;
                        lo[u] = std::min(lo[u], kv.first);
                        hi[u] = std::max(hi[u], kv.first);
                    }
                }
            }
            Rows cs(nu);
            for (int u = 0; u < nu; ++u)
                for (int j = lo[u]; j <= hi[u]; ++j)
                    if (dense[u][j] != 0.0) cs[u].emplace_back(j, dense[u][j]);
            bt_pairs.push_back(std::move(bt));
            cs_pairs.push_back(std::move(cs));
        }
    }
    pack(bt_pairs, nv, t->bt);
    pack(cs_pairs, nu, t->cs);
    const int pairs = nz * Kt;
    transpose(t->cs, pairs, nx, t->cst);
    transpose(t->bt, pairs, ny, t->btt);
    if (rot) {
        // E^z per natural x column (shift sa * x, spread |sa| hx), then E^x
        // per sheared z row (shift sb * z, spread |sb| hz)
        const int nx1 = (int)g->nx, nz1 = (int)g->nz;
        std::vector<Rows> ezp, exp_;
        for (int x1 = 0; x1 < nx1; ++x1)
            ezp.push_back(shear_rows(nzr, nz1, hz, sa * (x1 + 0.5 - 0.5 * nx1) * hx, std::fabs(sa) * hx));
        for (int z = 0; z < nzr; ++z)
            exp_.push_back(shear_rows(nxr, nx1, hx, sb * (z + 0.5 - 0.5 * nzr) * hz, std::fabs(sb) * hz));
        pack(ezp, nzr, t->ez);
        pack(exp_, nxr, t->ex);
        transpose(t->ez, nx1, nz1, t->ezt);
        transpose(t->ex, nzr, nx1, t->ext);
    }
    uint64_t off = 0;
    auto place = [&](uint64_t& o, uint64_t bytes) { o = off; off = align256(off + bytes); };
    place(t->off_bt_s, t->bt.start.size() * 4);
    place(t->off_bt_w, t->bt.w.size() * 4);
    place(t->off_cs_s, t->cs.start.size() * 4);
    place(t->off_cs_w, t->cs.w.size() * 4);
    place(t->off_cst_s, t->cst.start.size() * 4);
    place(t->off_cst_w, t->cst.w.size() * 4);
    place(t->off_btt_s, t->btt.start.size() * 4);
    place(t->off_btt_w, t->btt.w.size() * 4);
    place(t->off_mid, mid * 4);
    if (rot) {
        place(t->off_ez_s, t->ez.start.size() * 4);
        place(t->off_ez_w, t->ez.w.size() * 4);
        place(t->off_ezt_s, t->ezt.start.size() * 4);
        place(t->off_ezt_w, t->ezt.w.size() * 4);
        place(t->off_ex_s, t->ex.start.size() * 4);
        place(t->off_ex_w, t->ex.w.size() * 4);
        place(t->off_ext_s, t->ext.start.size() * 4);
        place(t->off_ext_w, t->ext.w.size() * 4);
        place(t->off_r1, (uint64_t)nzr * g->ny * g->nx * 4);
        place(t->off_xr, (uint64_t)nzr * g->ny * nxr * 4);
    }
    t->ws_bytes = off;
    *out = t;
    clear_error();
    return LTM_OK;
}

void ltm_xport_destroy(ltm_xport* t) { delete t; }

ltm_status ltm_xport_workspace_bytes(const ltm_xport* t, uint64_t* bytes)
{
    if (!t || !bytes) return fail(LTM_ERR_INVALID, "null argument");
    *bytes = t->ws_bytes;
    return LTM_OK;
}

ltm_status ltm_xport_bands(const ltm_xport* t, uint32_t bands[4])
{
    if (!t || !bands) return fail(LTM_ERR_INVALID, "null argument");
    bands[0] = (uint32_t)t->bt.width;
    bands[1] = (uint32_t)t->cs.width;
    bands[2] = (uint32_t)t->cst.width;
    bands[3] = (uint32_t)t->btt.width;
    return LTM_OK;
}

ltm_status ltm_xport_bind_workspace(ltm_xport* t, void* ws, uint64_t bytes, void* stream)
{
    if (!t || !ws) return fail(LTM_ERR_INVALID, "null argument");
    if (bytes < t->ws_bytes) return fail(LTM_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(LTM_ERR_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    struct Up { uint64_t off; const void* src; size_t n; } ups[] = {
        {t->off_bt_s, t->bt.start.data(), t->bt.start.size() * 4},
        {t->off_bt_w, t->bt.w.data(), t->bt.w.size() * 4},
        {t->off_cs_s, t->cs.start.data(), t->cs.start.size() * 4},
        {t->off_cs_w, t->cs.w.data(), t->cs.w.size() * 4},
        {t->off_cst_s, t->cst.start.data(), t->cst.start.size() * 4},
        {t->off_cst_w, t->cst.w.data(), t->cst.w.size() * 4},
        {t->off_btt_s, t->btt.start.data(), t->btt.start.size() * 4},
        {t->off_btt_w, t->btt.w.data(), t->btt.w.size() * 4},
        {t->off_ez_s, t->ez.start.data(), t->ez.start.size() * 4},
        {t->off_ez_w, t->ez.w.data(), t->ez.w.size() * 4},
        {t->off_ezt_s, t->ezt.start.data(), t->ezt.start.size() * 4},
        {t->off_ezt_w, t->ezt.w.data(), t->ezt.w.size() * 4},
        {t->off_ex_s, t->ex.start.data(), t->ex.start.size() * 4},
        {t->off_ex_w, t->ex.w.data(), t->ex.w.size() * 4},
        {t->off_ext_s, t->ext.start.data(), t->ext.start.size() * 4},
        {t->off_ext_w, t->ext.w.data(), t->ext.w.size() * 4}};
    for (const Up& u : ups) {
        if (u.n == 0) continue;
        hipError_t e = hipMemcpyAsync(base + u.off, u.src, u.n, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "upload transport tables");
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "upload transport tables");
    t->ws = base;
    t->bound = true;
    return LTM_OK;
}

}  // extern "C"

namespace {

ltm::XportDev dev_of(const ltm_xport* t)
{
    ltm::XportDev d{};
    d.nx = t->nxr;
    d.ny = t->nyr;
    d.nz = t->nzr;
    d.nu = (int)t->cam.det_nu;
    d.nv = (int)t->cam.det_nv;
    d.kt = t->kt;
    auto band = [&](const ltm_xport::Band& b, uint64_t so, uint64_t wo) {
        ltm::BandDev r;
        r.start = reinterpret_cast<const int32_t*>(t->ws + so);
        r.w = reinterpret_cast<const float*>(t->ws + wo);
        r.rows = b.rows;
        r.width = b.width;
        return r;
    };
    d.bt = band(t->bt, t->off_bt_s, t->off_bt_w);
    d.cs = band(t->cs, t->off_cs_s, t->off_cs_w);
    d.cst = band(t->cst, t->off_cst_s, t->off_cst_w);
    d.btt = band(t->btt, t->off_btt_s, t->off_btt_w);
    d.mid = reinterpret_cast<float*>(t->ws + t->off_mid);
    return d;
}

ltm::ShearDev shear_of(const ltm_xport* t)
{
    ltm::ShearDev r{};
    r.nx1 = (int)t->grid.nx;
    r.nz1 = (int)t->grid.nz;
    r.nx = t->nxr;
    r.ny = t->nyr;
    r.nz = t->nzr;
    auto band = [&](const ltm_xport::Band& b, uint64_t so, uint64_t wo) {
        ltm::BandDev q;
        q.start = reinterpret_cast<const int32_t*>(t->ws + so);
        q.w = reinterpret_cast<const float*>(t->ws + wo);
        q.rows = b.rows;
        q.width = b.width;
        return q;
    };
    r.ez = band(t->ez, t->off_ez_s, t->off_ez_w);
    r.ezt = band(t->ezt, t->off_ezt_s, t->off_ezt_w);
    r.ex = band(t->ex, t->off_ex_s, t->off_ex_w);
    r.ext = band(t->ext, t->off_ext_s, t->off_ext_w);
    r.r1 = reinterpret_cast<float*>(t->ws + t->off_r1);
    r.xr = reinterpret_cast<float*>(t->ws + t->off_xr);
    return r;
}

}  // namespace

extern "C" {

ltm_status ltm_xport_project(ltm_xport* t, const float* x, float* y, void* stream)
{
    if (!t || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (!t->bound) return fail(LTM_ERR_WORKSPACE, "transport operator has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (t->rot) {
        const ltm::ShearDev r = shear_of(t);
        e = launch_shear_forward(r, x, s);
        if (e == hipSuccess) e = launch_xport_project(dev_of(t), r.xr, y, s);
    } else {
        e = launch_xport_project(dev_of(t), x, y, s);
    }
    return e == hipSuccess ? LTM_OK : hip_fail(e, "transport project");
}

ltm_status ltm_xport_backproject(ltm_xport* t, const float* y, float* x, void* stream)
{
    if (!t || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (!t->bound) return fail(LTM_ERR_WORKSPACE, "transport operator has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (t->rot) {
        const ltm::ShearDev r = shear_of(t);
        e = launch_xport_backproject(dev_of(t), y, r.xr, s);
        if (e == hipSuccess) e = launch_shear_adjoint(r, x, s);
    } else {
        e = launch_xport_backproject(dev_of(t), y, x, s);
    }
    return e == hipSuccess ? LTM_OK : hip_fail(e, "transport backproject");
}

}  // extern "C"
