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
    ltm_grid grid;                 // the grid after the quarter turns (natural when q = 0)
    ltm_camera cam;
    uint32_t basis;
    int kt;                        // angular rows (rays_v)
    // host tables (FP32 values, built once)
    struct Band {
        int rows = 0, width = 0;
        std::vector<int32_t> start;   // pairs * rows
        std::vector<float> w;         // pairs * width * rows (weight-major)
    } bt, cs, cst, btt;
    // posed cameras: q quarter turns of the volume about y (x and z extents
    // swap for odd q), then the shear rotation of the remaining |phi'| <= 45 deg
    int q = 0;                     // 0..3
    int nx0 = 0, nz0 = 0;          // natural grid columns and slices
    uint64_t off_turn = 0;         // the turned volume (when q != 0)
    bool rot = false;
    int nxr = 0, nyr = 0, nzr = 0;          // transport grid (rotated, or the natural one)
    Band ez, ezt, ex, ext;
    // factorized plenoptic model (square lenslet array)
    bool plen = false;
    int na_u = 0, na_v = 0, ncells = 0, ks = 0;
    std::vector<int32_t> cell_ks, cell_kt, cell_first;
    std::vector<float> mask;
    Band bt1, bs1, bt2, bs2, bt1t, bs1t, bt2t, bs2t;
    uint64_t off_pl[20] = {};
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

// One axis of an affine ray map (s' = ss s + su u + bar), or the 3x3 form
// on (s, u, 1) for compositions.
struct Aff {
    double m[3][3];
};

Aff aff_mul(const Aff& a, const Aff& b)
{
    Aff r{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) r.m[i][j] += a.m[i][k] * b.m[k][j];
    return r;
}

Aff aff_inv(const Aff& a)
{
    // [[A, t], [0, 1]]^-1 = [[A^-1, -A^-1 t], [0, 1]]
    const double det = a.m[0][0] * a.m[1][1] - a.m[0][1] * a.m[1][0];
    Aff r{};
    r.m[0][0] = a.m[1][1] / det;
    r.m[0][1] = -a.m[0][1] / det;
    r.m[1][0] = -a.m[1][0] / det;
    r.m[1][1] = a.m[0][0] / det;
    r.m[0][2] = -(r.m[0][0] * a.m[0][2] + r.m[0][1] * a.m[1][2]);
    r.m[1][2] = -(r.m[1][0] * a.m[0][2] + r.m[1][1] * a.m[1][2]);
    r.m[2][2] = 1.0;
    return r;
}

Aff aff_T(double d) { return Aff{{{1.0, d, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}}}; }
Aff aff_R(double f, double c) { return Aff{{{1.0, 0.0, 0.0}, {-1.0 / f, 1.0, c / f}, {0.0, 0.0, 1.0}}}; }

Kernel1D kernel_affine(int basis, const Aff& Xpq, const Aff& X0q, double sk, double d0, double dp);

Kernel1D kernel_of(int basis, double z, double D, double F, double sk, double d0, double dp)
{
    Aff X0q{{{1.0, -z, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}}};
    Aff Xpq{{{1.0 - D / F, D * z / F - z - D, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}}};
    return kernel_affine(basis, Xpq, X0q, sk, d0, dp);
}

Kernel1D kernel_affine(int basis, const Aff& Xpq, const Aff& X0q, double sk, double d0, double dp)
{
    const double qss = X0q.m[0][0], qsu = X0q.m[0][1], qbar = X0q.m[0][2];
    const double pss = Xpq.m[0][0], psu = Xpq.m[0][1], pbar = Xpq.m[0][2];
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

// Entries of one factor row over source cells [j0, j1) of size dq whose
// left edges are at (j - n/2) dq (a sub-block of a lattice of n cells).
void factor_row_block(const Kernel1D& k, double si, double dq, int n, int j0, int j1, double scale,
                      std::vector<std::pair<int, double>>& out)
{
    const double c = k.mag * si;
    for (int j = j0; j < j1; ++j) {
        const double a = (j - 0.5 * n) * dq - c;
        const double v = k.h * (G(k, a + dq) - G(k, a)) * scale;
        if (v != 0.0) out.emplace_back(j, v);
    }
}

double axis_volume_affine(int basis, const Aff& X0p, double dp, double d0)
{
    const double ss = X0p.m[0][0], su = X0p.m[0][1];
    if (basis == LTM_BASIS_DIRAC) return dp * std::fabs(d0 / su);
    const double m = std::max(d0 / (2.0 * std::fabs(su)), dp * std::fabs(ss / su) / 2.0);
    const double h = std::min(dp, d0 / std::fabs(ss));
    return 2.0 * m * h;
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

namespace {

// Rotation of a posed camera's volume into its axes: the z shear E^z per
// natural x column (shift sa x, spread |sa| hx) and the x shear E^x per
// sheared z row (shift sb z, spread |sb| hz), with exact transposes.
void build_shears(ltm_xport* t, const ltm_grid* g, double sa, double sb, double hx, double hz)
{
    const int nx1 = (int)g->nx, nz1 = (int)g->nz, nzr = t->nzr, nxr = t->nxr;
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

// Workspace places of the shear tables and the two rotated volumes.
void place_shears(ltm_xport* t, const ltm_grid* g, uint64_t& off)
{
    auto place = [&](uint64_t& o, uint64_t bytes) { o = off; off = align256(off + bytes); };
    place(t->off_ez_s, t->ez.start.size() * 4);
    place(t->off_ez_w, t->ez.w.size() * 4);
    place(t->off_ezt_s, t->ezt.start.size() * 4);
    place(t->off_ezt_w, t->ezt.w.size() * 4);
    place(t->off_ex_s, t->ex.start.size() * 4);
    place(t->off_ex_w, t->ex.w.size() * 4);
    place(t->off_ext_s, t->ext.start.size() * 4);
    place(t->off_ext_w, t->ext.w.size() * 4);
    place(t->off_r1, (uint64_t)t->nzr * g->ny * g->nx * 4);
    place(t->off_xr, (uint64_t)t->nzr * g->ny * t->nxr * 4);
}

// The quarter turns of a posed camera: the natural grid's extents and a
// workspace place for the turned volume, after the operator's other places.
void add_turn(ltm_xport* t, int q, const ltm_grid& gq)
{
    t->q = q;
    t->nx0 = (int)((q & 1) ? gq.nz : gq.nx);
    t->nz0 = (int)((q & 1) ? gq.nx : gq.nz);
    if (q == 0) return;
    t->off_turn = t->ws_bytes;
    t->ws_bytes = align256(t->ws_bytes + (uint64_t)gq.nx * gq.ny * gq.nz * 4);
}

// The factorized plenoptic model (camera-model section, plenoptic camera):
// slices -> array plane per angular cell, the rasterized aperture mask, then
// each lenslet -> detector.  Array pixels: the detector's pixel pitch, k per
// lenslet.  Tables hold the table entries with the slice thickness folded into
// the s factor of stage 1 and the measurement normalization (the pixel
// integral divided by dp^2 times the lenslet bounding square's solid angle
// (2 r / D_d)^2, over V^d) into the s factor of stage 2.  A posed camera
// takes the transport grid of the rotated volume (anisotropic voxels).
struct Pose {
    bool rot;
    double sa, sb;          // z shear (z += sa x) and x shear (x += sb z)
    double hx, hy, hz;      // voxel sizes on the transport grid (s, t, depth)
    int nxr, nzr;           // transport grid columns and slices
};

ltm_status create_plenoptic(const ltm_grid* g, const ltm_camera* c, uint32_t basis, double L,
                            const Pose& ps, ltm_xport** out)
{
    const int nx = ps.nxr, ny = (int)g->ny, nz = ps.nzr;
    const double hx = ps.hx, hy = ps.hy, hz = ps.hz;
    const int nu = (int)c->det_nu, nv = (int)c->det_nv, mu = (int)c->mla_nu, mv = (int)c->mla_nv;
    const int ka = nu / mu;
    if (nv / mv != ka)
        return fail(LTM_ERR_UNSUPPORTED, "the factorized plenoptic transport needs square lenslets "
                                         "(det_nu / mla_nu == det_nv / mla_nv)");
    const int Ks = (int)c->rays_u, Kt = (int)c->rays_v;
    const double dp = c->pixel_pitch_mm, P = ka * dp, da = dp;
    const double r = c->r_main_mm, d0s = 2.0 * r / Ks, d0t = 2.0 * r / Kt;
    const double Dm = c->d_mla_mm, Dd = c->d_mla_det_mm;
    if (!(L - 0.5 * nz * hz > 0.0)) return fail(LTM_ERR_INVALID, "every slice must lie in front of the lens");
    const uint64_t m1 = (uint64_t)nz * Kt * nv * (uint64_t)nx;
    if (m1 > (1ull << 34) || (uint64_t)Ks * Kt * nv * (uint64_t)nu > (1ull << 34))
        return fail(LTM_ERR_INVALID, "intermediates larger than 2^34 values");
    ltm_xport* t = new ltm_xport();
    t->grid = *g;
    t->cam = *c;
    t->basis = basis;
    t->plen = true;
    t->rot = ps.rot;
    t->nxr = nx;
    t->nyr = ny;
    t->nzr = nz;
    t->kt = Kt;
    t->ks = Ks;
    t->na_u = nu;
    t->na_v = nv;
    const int na_u = nu, na_v = nv;
    // active cells, row by row
    t->cell_first.push_back(0);
    for (int kt = 0; kt < Kt; ++kt) {
        const double tk = (kt + 0.5) * d0t - r;
        for (int ks = 0; ks < Ks; ++ks) {
            const double sk = (ks + 0.5) * d0s - r;
            if (sk * sk + tk * tk > r * r) continue;
            t->cell_ks.push_back(ks);
            t->cell_kt.push_back(kt);
        }
        t->cell_first.push_back((int32_t)t->cell_ks.size());
    }
    t->ncells = (int)t->cell_ks.size();
    const Aff X0a = aff_T(Dm);
    const Aff X0d = aff_mul(aff_mul(X0a, aff_R(c->f_mla_mm, 0.0)), aff_T(Dd));
    const double Va = axis_volume_affine((int)basis, X0a, da, d0s) * axis_volume_affine((int)basis, X0a, da, d0t);
    const double Vd = axis_volume_affine((int)basis, X0d, dp, d0s) * axis_volume_affine((int)basis, X0d, dp, d0t);
    const double omega = (2.0 * c->r_mla_mm / Dd) * (2.0 * c->r_mla_mm / Dd);
    const double norm = d0s * d0t / (X0d.m[0][1] * X0d.m[0][1] * omega);
    // mask: array pixel centre inside its lenslet's aperture disc, over V^a
    t->mask.assign((size_t)na_v * na_u, 0.0f);
    for (int va = 0; va < na_v; ++va)
        for (int ua = 0; ua < na_u; ++ua) {
            const double sa = (ua + 0.5 - 0.5 * na_u) * da, ta = (va + 0.5 - 0.5 * na_v) * da;
            const double cs = (ua / ka + 0.5 - 0.5 * mu) * P, ct = (va / ka + 0.5 - 0.5 * mv) * P;
            if ((sa - cs) * (sa - cs) + (ta - ct) * (ta - ct) <= c->r_mla_mm * c->r_mla_mm)
                t->mask[(size_t)va * na_u + ua] = (float)(1.0 / Va);
        }
    // stage 1: per (slice, kt) t factor and per (slice, ks) s factor
    std::vector<Rows> bt1, bs1;
    for (int iz = 0; iz < nz; ++iz) {
        const double z = L + (iz + 0.5 - 0.5 * nz) * hz;
        const Aff X0q = aff_inv(aff_mul(aff_T(z), aff_R(c->f_main_mm, 0.0)));
        const Aff Xaq = aff_mul(aff_inv(X0a), X0q);
        for (int kt = 0; kt < Kt; ++kt) {
            const Kernel1D k1 = kernel_affine((int)basis, Xaq, X0q, (kt + 0.5) * d0t - r, d0t, da);
            Rows rows(na_v);
            for (int va = 0; va < na_v; ++va) factor_row(k1, (va + 0.5 - 0.5 * na_v) * da, hy, ny, 1.0, rows[va]);
            bt1.push_back(std::move(rows));
        }
        for (int ks = 0; ks < Ks; ++ks) {
            const Kernel1D k1 = kernel_affine((int)basis, Xaq, X0q, (ks + 0.5) * d0s - r, d0s, da);
            Rows rows(na_u);
            for (int ua = 0; ua < na_u; ++ua) factor_row(k1, (ua + 0.5 - 0.5 * na_u) * da, hx, nx, hz, rows[ua]);
            bs1.push_back(std::move(rows));
        }
    }
    // stage 2: per angular column / row, each lenslet's block of array pixels
    // onto the detector (every lenslet whose block meets the kernel's support)
    auto stage2 = [&](int K, double d0, int nd, int nl, std::vector<Rows>& outv, double scale) {
        for (int kk = 0; kk < K; ++kk) {
            const double sk = (kk + 0.5) * d0 - r;
            std::vector<Kernel1D> kern(nl);
            for (int l = 0; l < nl; ++l) {
                const double cl = (l + 0.5 - 0.5 * nl) * P;
                const Aff X0dl = aff_mul(aff_mul(X0a, aff_R(c->f_mla_mm, cl)), aff_T(Dd));
                kern[l] = kernel_affine((int)basis, aff_mul(aff_inv(X0dl), X0a), X0a, sk, d0, dp);
            }
            Rows rows(nd);
            for (int i = 0; i < nd; ++i) {
                const double si = (i + 0.5 - 0.5 * nd) * dp;
                for (int l = 0; l < nl; ++l) {
                    const double c0 = kern[l].mag * si;
                    const double lo = (l * ka - 0.5 * nl * ka) * da - c0, hi = lo + ka * da;
                    if (hi <= kern[l].tau[0] || lo >= kern[l].tau[3]) continue;
                    factor_row_block(kern[l], si, da, nl * ka, l * ka, (l + 1) * ka, scale, rows[i]);
                }
            }
            outv.push_back(std::move(rows));
        }
    };
    std::vector<Rows> bt2, bs2;
    stage2(Kt, d0t, nv, mv, bt2, 1.0);
    stage2(Ks, d0s, nu, mu, bs2, norm / Vd);
    pack(bt1, na_v, t->bt1);
    pack(bs1, na_u, t->bs1);
    pack(bt2, nv, t->bt2);
    pack(bs2, nu, t->bs2);
    transpose(t->bt1, nz * Kt, ny, t->bt1t);
    transpose(t->bs1, nz * Ks, nx, t->bs1t);
    transpose(t->bt2, Kt, na_v, t->bt2t);
    transpose(t->bs2, Ks, na_u, t->bs2t);
    uint64_t off = 0;
    auto place = [&](int i, uint64_t bytes) { t->off_pl[i] = off; off = align256(off + bytes); };
    const ltm_xport::Band* bands[8] = {&t->bt1, &t->bs1, &t->bt2, &t->bs2, &t->bt1t, &t->bs1t, &t->bt2t, &t->bs2t};
    for (int i = 0; i < 8; ++i) {
        place(2 * i, bands[i]->start.size() * 4);
        place(2 * i + 1, bands[i]->w.size() * 4);
    }
    place(16, (t->cell_ks.size() + t->cell_kt.size() + t->cell_first.size()) * 4);
    place(17, t->mask.size() * 4);
    place(18, m1 * 4 + (uint64_t)t->ncells * na_v * na_u * 4);      // M1, then FA
    place(19, (uint64_t)t->ncells * nv * na_u * 4);                 // M2
    if (ps.rot) {
        build_shears(t, g, ps.sa, ps.sb, hx, hz);
        place_shears(t, g, off);
    }
    t->ws_bytes = off;
    *out = t;
    clear_error();
    return LTM_OK;
}

}  // namespace

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
    if (c->kind != LTM_SINGLE_LENS && c->kind != LTM_PLENOPTIC)
        return fail(LTM_ERR_UNSUPPORTED, "the transport operator models single-lens and square-array plenoptic cameras");
    // pose: azimuth phi about the grid's y axis, the lens on the camera axis
    // through the grid centre; phi = 90 q + phi' with |phi'| <= 45 deg
    const double* es = c->axes;
    const double* et = c->axes + 3;
    const double* ez = c->axes + 6;
    if (std::fabs(et[1] - 1.0) > 1e-12 || std::fabs(es[1]) > 1e-12 || std::fabs(ez[1]) > 1e-12)
        return fail(LTM_ERR_UNSUPPORTED, "the transport operator needs an azimuth pose (e_t = +y)");
    const double phi0 = std::atan2(ez[0], ez[2]);
    // nearest q; the azimuth read back from the axes carries rounding, so
    // half-way cases within 1e-9 of a quarter are taken to even exactly
    const double tq = phi0 / (0.5 * M_PI), fq = std::floor(tq);
    const int q = std::fabs(tq - fq - 0.5) < 1e-9 ? (int)fq + ((int)fq & 1) : (int)std::nearbyint(tq);
    const double phi = phi0 - 0.5 * M_PI * q;
    // the volume turned by q quarter turns is what a camera at phi' sees
    ltm_grid gq = *g;
    if (q & 1) std::swap(gq.nx, gq.nz);
    g = &gq;
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
        // The x shear of the whole z-sheared box is wider than the image of the
        // volume itself, a rotated rectangle: a column x1 (centre c1) is nonzero
        // after the z shear only within |z - sa c1| < (nz hz + hz + |sa| hx) / 2,
        // and (1 + sa sb) = cos^2 phi, so after the x shear every nonzero cell
        // centre lies within |x| <= m.  Cells beyond that only ever hold zeros;
        // the grid keeps the parity of nx (the same cell centres) and the
        // outermost centre at least hx + |sb| hz / 2 beyond m.
        const double ua = std::fabs(sa), ub = std::fabs(sb);
        const double m = (0.5 * g->nx * hx - 0.5 * hx) * (1.0 - ua * ub) +
                         ub * (0.5 * g->nz * hz + 0.5 * hz + 0.5 * ua * hx);
        const double need = 2.0 * (m + hx + 0.5 * ub * hz) / hx + 1.0;
        const int k = std::max(0, (int)std::ceil(0.5 * (need - (double)g->nx - 2.0)));
        nxr = std::min(nxr, (int)g->nx + 2 * k + 2);
    }
    const int qm = ((q % 4) + 4) % 4;
    if (c->kind == LTM_PLENOPTIC) {
        const Pose ps{rot, sa, sb, hx, hy, hz, nxr, nzr};
        st = create_plenoptic(g, c, basis, L, ps, out);
        if (st == LTM_OK) add_turn(*out, qm, gq);
        return st;
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
    if (rot) build_shears(t, g, sa, sb, hx, hz);
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
    if (rot) place_shears(t, g, off);
    t->ws_bytes = off;
    add_turn(t, qm, gq);
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
    const bool p = t->plen;
    bands[0] = (uint32_t)(p ? t->bt1.width : t->bt.width);
    bands[1] = (uint32_t)(p ? t->bs1.width : t->cs.width);
    bands[2] = (uint32_t)(p ? t->bs1t.width : t->cst.width);
    bands[3] = (uint32_t)(p ? t->bt1t.width : t->btt.width);
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
    std::vector<Up> all;
    if (t->plen) {
        const ltm_xport::Band* bands[8] = {&t->bt1, &t->bs1, &t->bt2, &t->bs2,
                                           &t->bt1t, &t->bs1t, &t->bt2t, &t->bs2t};
        for (int i = 0; i < 8; ++i) {
            all.push_back({t->off_pl[2 * i], bands[i]->start.data(), bands[i]->start.size() * 4});
            all.push_back({t->off_pl[2 * i + 1], bands[i]->w.data(), bands[i]->w.size() * 4});
        }
        const size_t nc = t->cell_ks.size(), nf = t->cell_first.size();
        all.push_back({t->off_pl[16], t->cell_ks.data(), nc * 4});
        all.push_back({t->off_pl[16] + nc * 4, t->cell_kt.data(), nc * 4});
        all.push_back({t->off_pl[16] + 2 * nc * 4, t->cell_first.data(), nf * 4});
        all.push_back({t->off_pl[17], t->mask.data(), t->mask.size() * 4});
        if (t->rot)
            for (int i = 8; i < 16; ++i) all.push_back(ups[i]);   // the shear tables
    } else {
        all.assign(std::begin(ups), std::end(ups));
    }
    for (const Up& u : all) {
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

ltm::PlenDev plen_of(const ltm_xport* t)
{
    ltm::PlenDev d{};
    d.nx = t->nxr;
    d.ny = t->nyr;
    d.nz = t->nzr;
    d.na_u = t->na_u;
    d.na_v = t->na_v;
    d.nu = (int)t->cam.det_nu;
    d.nv = (int)t->cam.det_nv;
    d.ks = t->ks;
    d.kt = t->kt;
    d.cells = t->ncells;
    d.row_cells_max = 0;
    for (size_t k = 0; k + 1 < t->cell_first.size(); ++k)
        d.row_cells_max = std::max(d.row_cells_max, t->cell_first[k + 1] - t->cell_first[k]);
    const int32_t* cl = reinterpret_cast<const int32_t*>(t->ws + t->off_pl[16]);
    d.cell_ks = cl;
    d.cell_kt = cl + t->ncells;
    d.cell_first = cl + 2 * t->ncells;
    auto band = [&](const ltm_xport::Band& b, int i) {
        ltm::BandDev q;
        q.start = reinterpret_cast<const int32_t*>(t->ws + t->off_pl[2 * i]);
        q.w = reinterpret_cast<const float*>(t->ws + t->off_pl[2 * i + 1]);
        q.rows = b.rows;
        q.width = b.width;
        return q;
    };
    d.bt1 = band(t->bt1, 0);
    d.bs1 = band(t->bs1, 1);
    d.bt2 = band(t->bt2, 2);
    d.bs2 = band(t->bs2, 3);
    d.bt1t = band(t->bt1t, 4);
    d.bs1t = band(t->bs1t, 5);
    d.bt2t = band(t->bt2t, 6);
    d.bs2t = band(t->bs2t, 7);
    d.mask = reinterpret_cast<const float*>(t->ws + t->off_pl[17]);
    d.m1 = reinterpret_cast<float*>(t->ws + t->off_pl[18]);
    d.fa = d.m1 + (size_t)d.nz * d.kt * d.na_v * d.nx;
    d.m2 = reinterpret_cast<float*>(t->ws + t->off_pl[19]);
    return d;
}

}  // namespace

extern "C" {

ltm_status ltm_xport_project(ltm_xport* t, const float* x, float* y, void* stream)
{
    if (!t || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (!t->bound) return fail(LTM_ERR_WORKSPACE, "transport operator has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    // quarter turns, then the shear rotation, then the head-on transport
    if (t->q) {
        float* xq = reinterpret_cast<float*>(t->ws + t->off_turn);
        e = launch_turn(x, xq, t->nx0, t->nyr, t->nz0, t->q, s);
        x = xq;
    }
    if (e == hipSuccess && t->rot) {
        const ltm::ShearDev r = shear_of(t);
        e = launch_shear_forward(r, x, s);
        x = r.xr;
    }
    if (e == hipSuccess)
        e = t->plen ? launch_plen_project(plen_of(t), x, y, s) : launch_xport_project(dev_of(t), x, y, s);
    return e == hipSuccess ? LTM_OK : hip_fail(e, "transport project");
}

ltm_status ltm_xport_backproject(ltm_xport* t, const float* y, float* x, void* stream)
{
    if (!t || !x || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (!t->bound) return fail(LTM_ERR_WORKSPACE, "transport operator has no bound workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the transposes in reverse order: transport, shears, quarter turns
    float* xq = t->q ? reinterpret_cast<float*>(t->ws + t->off_turn) : x;
    const ltm::ShearDev r = t->rot ? shear_of(t) : ltm::ShearDev{};
    float* xt = t->rot ? r.xr : xq;
    hipError_t e = t->plen ? launch_plen_backproject(plen_of(t), y, xt, s)
                           : launch_xport_backproject(dev_of(t), y, xt, s);
    if (e == hipSuccess && t->rot) e = launch_shear_adjoint(r, xq, s);
    // the turn by -q on the turned grid is the inverse permutation
    if (e == hipSuccess && t->q)
        e = launch_turn(xq, x, (int)t->grid.nx, t->nyr, (int)t->grid.nz, (4 - t->q) % 4, s);
    return e == hipSuccess ? LTM_OK : hip_fail(e, "transport backproject");
}

}  // extern "C"
