// Host side of the reconstruction algorithm (the paper's reconstruction-
// algorithm table) and of the regularizer entry point.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "ltm_internal.h"
#include "ltm_solver.h"

namespace ltm {
namespace {

uint64_t align256(uint64_t v) { return (v + 255u) & ~uint64_t(255u); }

struct Layout {
    uint64_t x, z, g, dinv, p, r, sc, cam_off, total;
};

Layout solver_layout(const ltm_plan* p)
{
    Layout L{};
    const uint64_t N = p->n_vox, M = p->n_meas, nc = p->cams.size();
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.x = take(4 * N);
    L.z = take(4 * N);
    L.g = take(4 * N);
    L.dinv = take(4 * N);
    L.p = take(4 * M);
    L.r = take(4 * M);
    L.sc = take(8 * (SC_CAM + SC_NCAMARR * nc));
    L.cam_off = take(8 * (nc + 1));
    L.total = off;
    return L;
}

// One iteration: p = A z, gains and residual, r = W(p - g y), g = A^T r,
// g += grad R(z), then the projected (accelerated) update.
ltm_status iterate(ltm_solver* s, hipStream_t st)
{
    SolverDev& d = s->d;
    const uint32_t ns = s->prm.n_subsets > 1 ? s->prm.n_subsets : 1;
    ltm_plan_set_ray_subset(s->plan, ns, ns > 1 ? s->iter % ns : 0);
    ltm_status e = ltm_project(s->plan, d.z, d.p, st);
    if (e != LTM_OK) return e;
    hipError_t h = solver_launch_reduce(d, d.p, st);
    if (h == hipSuccess) h = solver_launch_scalars(d, st);
    if (h == hipSuccess) h = solver_launch_residual(d, d.p, d.r, st);
    if (h != hipSuccess) return hip_fail(h, "solver residual");
    e = ltm_backproject(s->plan, d.r, d.g, st);
    if (e != LTM_OK) return e;
    if (s->prm.beta > 0.0) {
        h = launch_reg_grad(s->plan->grid, (int)s->prm.psi_kind, s->prm.beta, s->prm.delta, d.z, d.g, st);
        if (h != hipSuccess) return hip_fail(h, "regularizer");
    }
    h = solver_launch_update(d, (float)s->prm.nu, st);
    if (h != hipSuccess) return hip_fail(h, "solver update");
    ltm_plan_set_ray_subset(s->plan, 1, 0);
    ++s->iter;
    return LTM_OK;
}

}  // namespace
}  // namespace ltm

using namespace ltm;

extern "C" {

ltm_status ltm_solver_workspace_bytes(const ltm_plan* p, uint64_t* bytes)
{
    if (!p || !bytes) return fail(LTM_ERR_INVALID, "null argument");
    *bytes = solver_layout(p).total;
    return LTM_OK;
}

ltm_status ltm_solver_create(ltm_plan* plan, const ltm_solver_params* prm, const float* y,
                             const float* w, void* ws, uint64_t ws_bytes, void* stream,
                             ltm_solver** out)
{
    if (!out) return fail(LTM_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!plan || !prm || !y) return fail(LTM_ERR_INVALID, "null argument");
    if (prm->psi_kind > LTM_PSI_HYPERBOLA) return fail(LTM_ERR_INVALID, "unknown potential");
    if (prm->n_subsets > 64) return fail(LTM_ERR_INVALID, "at most 64 view subsets");
    if (!(prm->beta >= 0.0) || !(prm->nu >= 0.0) || !(prm->c_r >= 0.0) || !std::isfinite(prm->beta) ||
        !std::isfinite(prm->nu) || !std::isfinite(prm->c_r))
        return fail(LTM_ERR_INVALID, "beta, nu and c_R must be finite and nonnegative");
    if (prm->psi_kind == LTM_PSI_HYPERBOLA && !(prm->delta > 0.0 && std::isfinite(prm->delta)))
        return fail(LTM_ERR_INVALID, "the hyperbola potential needs delta > 0");
    if (!(prm->rho_target >= 0.0) || !std::isfinite(prm->rho_target))
        return fail(LTM_ERR_INVALID, "rho_target must be finite and nonnegative");
    if (!plan->bound) return fail(LTM_ERR_WORKSPACE, "plan has no bound workspace");
    const Layout L = solver_layout(plan);
    if (!ws || ws_bytes < L.total)
        return fail(LTM_ERR_WORKSPACE, "solver workspace of " + std::to_string(L.total) +
                                           " bytes required");
    if (reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(LTM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    ltm_solver* s = new (std::nothrow) ltm_solver();
    if (!s) return fail(LTM_ERR_INVALID, "out of host memory");
    ltm_plan_set_ray_subset(plan, 1, 0);   // the majorizer uses every angular sample
    s->plan = plan;
    s->prm = *prm;
    char* b = static_cast<char*>(ws);
    SolverDev& d = s->d;
    d.x = reinterpret_cast<float*>(b + L.x);
    d.z = reinterpret_cast<float*>(b + L.z);
    d.g = reinterpret_cast<float*>(b + L.g);
    d.dinv = reinterpret_cast<float*>(b + L.dinv);
    d.p = reinterpret_cast<float*>(b + L.p);
    d.r = reinterpret_cast<float*>(b + L.r);
    d.sc = reinterpret_cast<double*>(b + L.sc);
    d.cam_off = reinterpret_cast<uint64_t*>(b + L.cam_off);
    d.y = y;
    d.w = w;
    d.n_cam = (int)plan->cams.size();
    d.gains = prm->gains ? 1 : 0;
    d.momentum = prm->momentum ? 1 : 0;
    d.N = plan->n_vox;
    d.M = plan->n_meas;
    uint64_t maxpix = 0;
    s->cam_off.push_back(0);
    for (auto& c : plan->cams) {
        s->cam_off.push_back(c.y_off + c.npix);
        if (c.npix > maxpix) maxpix = c.npix;
    }
    uint64_t bpc = (maxpix + 255) / 256;
    d.blocks_per_cam = (int)(bpc > 512 ? 512 : (bpc ? bpc : 1));

    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t h = hipMemcpyAsync(d.cam_off, s->cam_off.data(), 8 * s->cam_off.size(),
                                  hipMemcpyHostToDevice, st);
    // sum W y^2 per camera: zero the slots, then reduce
    if (h == hipSuccess) h = hipMemsetAsync(d.sc, 0, 8 * (SC_CAM + SC_NCAMARR * d.n_cam), st);
    if (h == hipSuccess) h = solver_launch_yy(d, st);
    if (h == hipSuccess) h = solver_launch_reset(d, st);
    // majorizer D = A^T W A 1 (cameras stacked), then dinv = 1/(D + c_R beta)
    if (h == hipSuccess) h = launch_fill(d.x, d.N, 1.0f, st);
    if (h != hipSuccess) {
        delete s;
        return hip_fail(h, "solver setup");
    }
    ltm_status e = ltm_project(plan, d.x, d.p, st);
    if (e == LTM_OK && w) {
        h = launch_mul(d.p, w, d.M, st);
        if (h != hipSuccess) e = hip_fail(h, "majorizer weights");
    }
    if (e == LTM_OK) e = ltm_backproject(plan, d.p, d.dinv, st);
    if (e == LTM_OK) {
        h = solver_launch_dinv(d, (float)(prm->c_r * prm->beta), st);
        if (h == hipSuccess) h = launch_fill(d.x, d.N, 0.0f, st);
        if (h == hipSuccess) h = launch_fill(d.z, d.N, 0.0f, st);
        if (h != hipSuccess) e = hip_fail(h, "majorizer");
    }
    if (e != LTM_OK) {
        delete s;
        return e;
    }
    // the host copy of cam_off must outlive the asynchronous upload
    h = hipStreamSynchronize(st);
    if (h != hipSuccess) {
        delete s;
        return hip_fail(h, "solver setup");
    }
    clear_error();
    *out = s;
    return LTM_OK;
}

void ltm_solver_destroy(ltm_solver* s) { delete s; }

ltm_status ltm_solver_reset(ltm_solver* s, const float* x0, void* stream)
{
    if (!s) return fail(LTM_ERR_INVALID, "null solver");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t h;
    if (x0) {
        h = launch_copy(s->d.x, x0, s->d.N, st);
        if (h == hipSuccess) h = launch_copy(s->d.z, x0, s->d.N, st);
    } else {
        h = launch_fill(s->d.x, s->d.N, 0.0f, st);
        if (h == hipSuccess) h = launch_fill(s->d.z, s->d.N, 0.0f, st);
    }
    if (h == hipSuccess) h = solver_launch_reset(s->d, st);
    if (h != hipSuccess) return hip_fail(h, "solver reset");
    s->iter = 0;
    return LTM_OK;
}

ltm_status ltm_solver_reset_warm(ltm_solver* s, const float* x0, double* alpha_out, double* rho_out,
                                 uint32_t* accepted, void* stream)
{
    if (!s || !x0) return fail(LTM_ERR_INVALID, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    SolverDev& d = s->d;
    const int nc = d.n_cam;
    // non-finite values of x0, then p = A x0 and its per-camera sums
    hipError_t h = launch_count_nonfinite(x0, d.N, d.sc + SC_BAD, st);
    if (h != hipSuccess) return hip_fail(h, "warm start check");
    ltm_plan_set_ray_subset(s->plan, 1, 0);
    ltm_status e = ltm_project(s->plan, x0, d.p, st);
    if (e != LTM_OK) return e;
    h = solver_launch_reduce(d, d.p, st);
    std::vector<double> sc(SC_CAM + SC_NCAMARR * nc);
    if (h == hipSuccess) h = hipMemcpyAsync(sc.data(), d.sc, 8 * sc.size(), hipMemcpyDeviceToHost, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) return hip_fail(h, "warm start check");
    const double* pp = &sc[SC_CAM + SC_PP * nc];
    const double* yp = &sc[SC_CAM + SC_YP * nc];
    const double* yy = &sc[SC_CAM + SC_YY * nc];
    // least-squares scale of the image: camera 1 alone when the other
    // cameras' gains are estimated (a gain absorbs any scale), else all
    double spp = 0.0, syp = 0.0;
    for (int c = 0; c < (d.gains ? 1 : nc); ++c) {
        spp += pp[c];
        syp += yp[c];
    }
    const double alpha = spp > 0.0 ? syp / spp : 0.0;
    // rho(alpha x0) from the sums: p -> alpha p, gains re-estimated for it
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nc; ++c) {
        double g = 1.0;
        if (d.gains && c > 0) g = yy[c] > 0.0 ? alpha * yp[c] / yy[c] : 0.0;
        num += alpha * alpha * pp[c] - 2.0 * g * alpha * yp[c] + g * g * yy[c];
        den += g * g * yy[c];
    }
    double rho = den > 0.0 ? std::sqrt(std::max(num, 0.0) / den) : INFINITY;
    const bool ok = sc[SC_BAD] == 0.0 && std::isfinite(alpha) && alpha > 0.0 && std::isfinite(rho) &&
                    rho < 1.0;
    if (ok) {
        h = launch_scale_copy(d.x, x0, (float)alpha, d.N, st);
        if (h == hipSuccess) h = launch_copy(d.z, d.x, d.N, st);
    } else {
        rho = 1.0;
        h = launch_fill(d.x, d.N, 0.0f, st);
        if (h == hipSuccess) h = launch_fill(d.z, d.N, 0.0f, st);
    }
    if (h == hipSuccess) h = solver_launch_reset(d, st);
    if (h != hipSuccess) return hip_fail(h, "warm start reset");
    s->iter = 0;
    if (alpha_out) *alpha_out = alpha;
    if (rho_out) *rho_out = rho;
    if (accepted) *accepted = ok ? 1u : 0u;
    clear_error();
    return LTM_OK;
}

ltm_status ltm_solver_solve(ltm_solver* s, uint32_t* iterations, uint32_t* converged, double* rho,
                            void* stream)
{
    if (!s) return fail(LTM_ERR_INVALID, "null solver");
    const uint32_t cap = s->prm.max_iter, every = s->prm.check_every;
    if (cap == 0 || every == 0) return fail(LTM_ERR_INVALID, "max_iter and check_every must be >= 1");
    const double target = s->prm.rho_target;
    uint32_t it = 0;
    bool conv = false;
    double r = INFINITY;
    while (it < cap) {
        const uint32_t n = std::min(every, cap - it);
        ltm_status e = ltm_solver_step(s, n, stream);
        if (e != LTM_OK) return e;
        it += n;
        double rz = INFINITY;
        e = ltm_solver_residual(s, &rz, nullptr, stream);
        if (e != LTM_OK) return e;
        if (target > 0.0 && rz <= target) {
            e = ltm_solver_residual_x(s, &r, stream);
            if (e != LTM_OK) return e;
            if (r <= target) {
                conv = true;
                break;
            }
        }
    }
    if (!conv) {
        ltm_status e = ltm_solver_residual_x(s, &r, stream);
        if (e != LTM_OK) return e;
    }
    if (iterations) *iterations = it;
    if (converged) *converged = conv ? 1u : 0u;
    if (rho) *rho = r;
    return LTM_OK;
}

ltm_status ltm_solver_step(ltm_solver* s, uint32_t n_iter, void* stream)
{
    if (!s) return fail(LTM_ERR_INVALID, "null solver");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (uint32_t k = 0; k < n_iter; ++k) {
        ltm_status e = iterate(s, st);
        if (e != LTM_OK) return e;
    }
    return LTM_OK;
}

ltm_status ltm_solver_get_x(const ltm_solver* s, float* x, void* stream)
{
    if (!s || !x) return fail(LTM_ERR_INVALID, "null argument");
    hipError_t h = launch_copy(x, s->d.x, s->d.N, static_cast<hipStream_t>(stream));
    if (h != hipSuccess) return hip_fail(h, "copy x");
    return LTM_OK;
}

ltm_status ltm_solver_residual(ltm_solver* s, double* rho, uint32_t* iterations, void* stream)
{
    if (!s) return fail(LTM_ERR_INVALID, "null solver");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double h4[4];
    hipError_t h = hipMemcpyAsync(h4, s->d.sc, sizeof(h4), hipMemcpyDeviceToHost, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) return hip_fail(h, "read residual");
    if (rho) *rho = h4[SC_RHO];
    if (iterations) *iterations = (uint32_t)h4[SC_ITER];
    if (h4[SC_ITER] > 0 && !std::isfinite(h4[SC_RHO]))
        return fail(LTM_ERR_NUMERIC, "non-finite data residual");
    return LTM_OK;
}

ltm_status ltm_solver_residual_x(ltm_solver* s, double* rho, void* stream)
{
    if (!s || !rho) return fail(LTM_ERR_INVALID, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    ltm_plan_set_ray_subset(s->plan, 1, 0);
    ltm_status e = ltm_project(s->plan, s->d.x, s->d.p, st);
    if (e != LTM_OK) return e;
    hipError_t h = solver_launch_reduce(s->d, s->d.p, st);
    if (h == hipSuccess) h = solver_launch_rho_x(s->d, st);
    double v = 0.0;
    if (h == hipSuccess) h = hipMemcpyAsync(&v, s->d.sc + SC_RHOX, 8, hipMemcpyDeviceToHost, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) return hip_fail(h, "residual of x");
    *rho = v;
    if (!std::isfinite(v)) return fail(LTM_ERR_NUMERIC, "non-finite data residual");
    return LTM_OK;
}

ltm_status ltm_solver_save(const ltm_solver* s, float* x, float* z, double* t, uint32_t* iterations,
                           double* gains, void* stream)
{
    if (!s || !x || !z || !t || !iterations) return fail(LTM_ERR_INVALID, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nc = s->d.n_cam;
    std::vector<double> sc(SC_CAM + SC_NCAMARR * nc);
    hipError_t h = launch_copy(x, s->d.x, s->d.N, st);
    if (h == hipSuccess) h = launch_copy(z, s->d.z, s->d.N, st);
    if (h == hipSuccess) h = hipMemcpyAsync(sc.data(), s->d.sc, 8 * sc.size(), hipMemcpyDeviceToHost, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) return hip_fail(h, "save solver state");
    *t = sc[SC_T];
    *iterations = (uint32_t)sc[SC_ITER];
    if (gains)
        for (int c = 0; c < nc; ++c) gains[c] = sc[SC_CAM + SC_GAMMA * nc + c];
    return LTM_OK;
}

ltm_status ltm_solver_load(ltm_solver* s, const float* x, const float* z, double t,
                           uint32_t iterations, const double* gains, void* stream)
{
    if (!s || !x || !z) return fail(LTM_ERR_INVALID, "null argument");
    if (!(t >= 1.0) || !std::isfinite(t)) return fail(LTM_ERR_INVALID, "FISTA t must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nc = s->d.n_cam;
    std::vector<double> sc(SC_CAM + SC_NCAMARR * nc);
    hipError_t h = hipMemcpyAsync(sc.data(), s->d.sc, 8 * sc.size(), hipMemcpyDeviceToHost, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) return hip_fail(h, "load solver state");
    sc[SC_T] = t;
    sc[SC_ITER] = (double)iterations;
    s->iter = iterations;
    sc[SC_MOM] = 0.0;
    if (gains)
        for (int c = 0; c < nc; ++c) sc[SC_CAM + SC_GAMMA * nc + c] = gains[c];
    h = launch_copy(s->d.x, x, s->d.N, st);
    if (h == hipSuccess) h = launch_copy(s->d.z, z, s->d.N, st);
    if (h == hipSuccess) h = hipMemcpyAsync(s->d.sc, sc.data(), 8 * sc.size(), hipMemcpyHostToDevice, st);
    if (h == hipSuccess) h = hipStreamSynchronize(st);
    if (h != hipSuccess) return hip_fail(h, "load solver state");
    return LTM_OK;
}

ltm_status ltm_reg_grad_add(const ltm_grid* grid, uint32_t psi_kind, double beta, double delta,
                            const float* z, float* g, void* stream)
{
    if (!grid || !z || !g) return fail(LTM_ERR_INVALID, "null argument");
    if (grid->nx == 0 || grid->ny == 0 || grid->nz == 0) return fail(LTM_ERR_INVALID, "empty grid");
    if (psi_kind > LTM_PSI_HYPERBOLA) return fail(LTM_ERR_INVALID, "unknown potential");
    if (psi_kind == LTM_PSI_HYPERBOLA && !(delta > 0.0)) return fail(LTM_ERR_INVALID, "delta must be > 0");
    if (!(beta >= 0.0)) return fail(LTM_ERR_INVALID, "beta must be >= 0");
    hipError_t h = launch_reg_grad(*grid, (int)psi_kind, beta, delta, z, g, static_cast<hipStream_t>(stream));
    if (h != hipSuccess) return hip_fail(h, "regularizer");
    return LTM_OK;
}

}  // extern "C"
