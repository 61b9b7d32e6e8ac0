/*
 * FP64 reference of the ray-driven camera operator A and its transpose.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this code; the product library never does.  It
 * shares no header, helper or constant with the HIP path: every struct and
 * formula here is written out again from the paper.
 *
 * What it computes (per camera, cameras stacked):
 *   ray optics   -- the affine maps of the paper's table of optical
 *                   transformations: propagation s' = s + d u and thin-lens
 *                   refraction u' = u - (s - s0)/f, composed detector -> scene
 *                   (single-lens and plenoptic camera models);
 *   lenslets     -- square array, each pixel seeing only through the
 *                   lenslet above it; or hexagonal array of three focal
 *                   lengths (table of the simulated plenoptic camera), each
 *                   pixel summing the light of every lenslet of the array
 *                   (the sum over microlenses of the plenoptic-camera
 *                   section), checked here by brute force over all lenslets;
 *   occlusion    -- a ray is kept only if it passes inside the lenslet
 *                   aperture and the main-lens aperture (occlusion masks of
 *                   the occlusion and plenoptic-camera sections; closed
 *                   aperture, |t| <= 1/2 convention of the rect function);
 *   object       -- a voxel grid centred at the world origin; the radiance
 *                   along a ray is the line integral of the object (object
 *                   model section), evaluated with S midpoint samples of the
 *                   trilinear interpolant of the voxel values, clamped to the
 *                   edge inside the grid and zero outside;
 *   measurement  -- a pixel reads the mean over its R angular samples (the
 *                   sum over angular basis functions of the measurement
 *                   formation section, one Dirac sample per ray).
 * A^T is the same loops scattering instead of gathering.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no -ffast-math: IEEE FP64 is the
 * point of this file).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz, pad;
    double pitch;                 /* voxel edge, mm */
} orc_grid;

typedef struct {
    int32_t kind;                 /* 0 single lens, 1 plenoptic, 2 hexagonal plenoptic */
    int32_t nu, nv;               /* detector pixels (u = s direction fastest) */
    int32_t mu, mv;               /* lenslets (plenoptic) */
    int32_t ru, rv;               /* angular samples per pixel: ru x rv grid */
    int32_t samples;              /* S samples per ray */
    double pixel_pitch;
    double f_main, r_main;        /* main lens focal length and radius */
    double d_det;                 /* single lens: lens -> detector distance */
    double d_mla, d_mla_det;      /* plenoptic: lens -> MLA, MLA -> detector */
    double f_mla, r_mla;          /* lenslet focal length and radius */
    double axes[9];               /* e_s, e_t, e_z in world coordinates */
    double lens[3];               /* main-lens centre in world coordinates */
    double f_hex[3];              /* hexagonal array: focal length of each lenslet type */
} orc_camera;

/* Hexagonal lenslet array: mu lenslets per row, mv rows, touching discs of
 * radius r (pitch p = 2r, row spacing p sqrt(3)/2).  Rows whose distance
 * from row mv/2 is odd are shifted by p/2 along s.  Lenslet (i, j) has
 * hexagonal axial coordinates (q, r) with s/p = q + r/2 + const and r = j -
 * mv/2; its type (q - r) mod 3 differs from each of its six neighbours'. */
void orc_hex_lenslet(const orc_camera* c, int i, int j, double* cs, double* ct, int* type)
{
    const double p = 2.0 * c->r_mla, h = p * sqrt(3.0) / 2.0;
    const int r = j - c->mv / 2;
    const int odd = r & 1;
    *cs = (i - 0.5 * (c->mu - 1) + 0.5 * odd) * p;
    *ct = (j - 0.5 * (c->mv - 1)) * h;
    const int q2 = 2 * i + odd - r;                /* 2q, always even */
    *type = (((q2 / 2 - r) % 3) + 3) % 3;
}

/* Number of light paths per (pixel, angular sample): one lenslet (or the
 * lens) for kinds 0 and 1, every lenslet of the array for kind 2. */
int orc_paths(const orc_camera* c) { return c->kind == 2 ? c->mu * c->mv : 1; }

/* ------------------------------------------------------------------------ */
/* Ray optics.  A ray is (s,u,t,v) with u = ds/dz.  Starting on the detector
 * (pixel centre, aperture sample), the maps are applied in the order light
 * travels backwards: propagate to the aperture plane, refract, propagate,
 * refract.  The result is the ray leaving the main lens (z = 0) towards the
 * scene, returned in world coordinates as origin O and direction w with
 * w . e_z = 1 (so the ray parameter is the camera depth z).              */
int orc_trace_path(const orc_camera* c, int iu, int iv, int path, int ru, int rv,
                   double O[3], double w[3])
{
    const double gs = (2.0 * ru + 1.0) / c->ru - 1.0;   /* aperture grid cell centre */
    const double gt = (2.0 * rv + 1.0) / c->rv - 1.0;   /* in [-1, 1]               */
    const double sd = (iu + 0.5 - 0.5 * c->nu) * c->pixel_pitch;
    const double td = (iv + 0.5 - 0.5 * c->nv) * c->pixel_pitch;
    int valid = (gs * gs + gt * gt <= 1.0);
    double s0, t0, u2, v2;

    if (c->kind == 0) {
        /* aperture sample on the main lens, detector at distance D behind it */
        const double as = c->r_main * gs, at = c->r_main * gt;
        const double u = (as - sd) / c->d_det;           /* T_D slope */
        const double v = (at - td) / c->d_det;
        u2 = u - as / c->f_main;                         /* R_f about the axis */
        v2 = v - at / c->f_main;
        s0 = as;
        t0 = at;
    } else if (c->kind == 2) {
        /* angular sample on lenslet `path`, refracted by that lenslet's type */
        double cs, ct;
        int type;
        orc_hex_lenslet(c, path % c->mu, path / c->mu, &cs, &ct, &type);
        const double f = c->f_hex[type];
        const double as = cs + c->r_mla * gs, at = ct + c->r_mla * gt;
        const double u = (as - sd) / c->d_mla_det;
        const double v = (at - td) / c->d_mla_det;
        const double u1 = u - (as - cs) / f;
        const double v1 = v - (at - ct) / f;
        s0 = as + u1 * c->d_mla;
        t0 = at + v1 * c->d_mla;
        if (s0 * s0 + t0 * t0 > c->r_main * c->r_main) valid = 0;
        u2 = u1 - s0 / c->f_main;
        v2 = v1 - t0 / c->f_main;
    } else {
        const int ku = c->nu / c->mu, kv = c->nv / c->mv;
        const int lu = iu / ku, lv = iv / kv;             /* this pixel's lenslet */
        const double cs = (lu + 0.5 - 0.5 * c->mu) * (ku * c->pixel_pitch);
        const double ct = (lv + 0.5 - 0.5 * c->mv) * (kv * c->pixel_pitch);
        const double as = cs + c->r_mla * gs;            /* sample on the lenslet */
        const double at = ct + c->r_mla * gt;
        const double u = (as - sd) / c->d_mla_det;       /* detector -> MLA */
        const double v = (at - td) / c->d_mla_det;
        const double u1 = u - (as - cs) / c->f_mla;      /* lenslet refraction */
        const double v1 = v - (at - ct) / c->f_mla;
        s0 = as + u1 * c->d_mla;                          /* MLA -> main lens */
        t0 = at + v1 * c->d_mla;
        if (s0 * s0 + t0 * t0 > c->r_main * c->r_main) valid = 0;  /* main aperture */
        u2 = u1 - s0 / c->f_main;                         /* main-lens refraction */
        v2 = v1 - t0 / c->f_main;
    }
    const double* es = c->axes;
    const double* et = c->axes + 3;
    const double* ez = c->axes + 6;
    for (int a = 0; a < 3; ++a) {
        O[a] = c->lens[a] + s0 * es[a] + t0 * et[a];
        w[a] = u2 * es[a] + v2 * et[a] + ez[a];
    }
    return valid;
}

int orc_trace(const orc_camera* c, int iu, int iv, int ru, int rv, double O[3], double w[3])
{
    return orc_trace_path(c, iu, iv, 0, ru, rv, O, w);
}

/* Segment of the ray inside the grid's box [-n dx/2, n dx/2]^3, restricted to
 * the scene side of the lens (z >= 0).  Returns 1 and [z0, z1] on a hit. */
int orc_clip(const orc_grid* g, const double O[3], const double w[3], double zr[2])
{
    const int n[3] = {g->nx, g->ny, g->nz};
    double lo = 0.0, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double h = 0.5 * n[a] * g->pitch;
        if (w[a] == 0.0) {
            if (O[a] < -h || O[a] > h) return 0;
            continue;
        }
        double ta = (-h - O[a]) / w[a], tb = (h - O[a]) / w[a];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    zr[0] = lo;
    zr[1] = hi;
    return hi > lo;
}

/* Trilinear interpolation weights of world point P: the 8 voxel indices and
 * weights.  Voxel (i,j,k) has its centre at ((i + 1/2 - nx/2) dx, ...). */
static void corners(const orc_grid* g, const double P[3], int64_t idx[8], double wt[8])
{
    const int n[3] = {g->nx, g->ny, g->nz};
    int i[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double q = P[a] / g->pitch + 0.5 * n[a] - 0.5;
        if (q < 0.0) q = 0.0;
        if (q > n[a] - 1.0) q = n[a] - 1.0;
        int ia = (int)floor(q);
        if (ia > n[a] - 2) ia = n[a] - 2;
        i[a] = ia;
        f[a] = q - ia;
    }
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const int k = cx + 2 * cy + 4 * cz;
                idx[k] = (int64_t)(i[0] + cx) +
                         (int64_t)g->nx * ((int64_t)(i[1] + cy) + (int64_t)g->ny * (i[2] + cz));
                wt[k] = (cx ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) *
                        (cz ? f[2] : 1.0 - f[2]);
            }
}

/* Line integral of one ray with S midpoint samples; returns 0 for a miss. */
static double ray_integral(const orc_grid* g, const double* x, const double O[3],
                           const double w[3], int S)
{
    double zr[2];
    if (!orc_clip(g, O, w, zr)) return 0.0;
    const double len = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) * (zr[1] - zr[0]);
    const double hz = (zr[1] - zr[0]) / S;
    double acc = 0.0;
    for (int m = 0; m < S; ++m) {
        const double z = zr[0] + (m + 0.5) * hz;
        const double P[3] = {O[0] + z * w[0], O[1] + z * w[1], O[2] + z * w[2]};
        int64_t idx[8];
        double wt[8];
        corners(g, P, idx, wt);
        for (int k = 0; k < 8; ++k) acc += wt[k] * x[idx[k]];
    }
    return acc * (len / S);
}

static void ray_scatter(const orc_grid* g, double* x, const double O[3], const double w[3],
                        int S, double val)
{
    double zr[2];
    if (!orc_clip(g, O, w, zr)) return;
    const double len = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) * (zr[1] - zr[0]);
    const double hz = (zr[1] - zr[0]) / S;
    const double v = val * (len / S);
    for (int m = 0; m < S; ++m) {
        const double z = zr[0] + (m + 0.5) * hz;
        const double P[3] = {O[0] + z * w[0], O[1] + z * w[1], O[2] + z * w[2]};
        int64_t idx[8];
        double wt[8];
        corners(g, P, idx, wt);
        for (int k = 0; k < 8; ++k) x[idx[k]] += wt[k] * v;
    }
}

/* Angular-sample subsets (the paper's view-subset acceleration): subset
 * `idx` of `nsub` holds the samples r = ru + Ru*rv with r mod nsub == idx
 * (every nsub-th sample in lexicographic order).  Its operator is the mean
 * over the subset, i.e. the paper's (K/|S|) A_S.  nsub <= 1 is the full set. */
static int in_subset(int r, int nsub, int idx) { return nsub <= 1 || r % nsub == idx; }

static int subset_size(int R, int nsub, int idx)
{
    if (nsub <= 1) return R;
    int n = 0;
    for (int r = 0; r < R; ++r) n += (r % nsub == idx);
    return n;
}

static double pixel_subset(const orc_grid* g, const orc_camera* c, const double* x, int iu, int iv,
                           int nsub, int idx)
{
    const int R = c->ru * c->rv;
    double acc = 0.0;
    for (int path = 0; path < orc_paths(c); ++path)
        for (int rv = 0; rv < c->rv; ++rv)
            for (int ru = 0; ru < c->ru; ++ru) {
                double O[3], w[3];
                if (!in_subset(ru + c->ru * rv, nsub, idx)) continue;
                if (!orc_trace_path(c, iu, iv, path, ru, rv, O, w)) continue;
                acc += ray_integral(g, x, O, w, c->samples);
            }
    return acc / subset_size(R, nsub, idx);
}

/* y_i of one pixel of one camera: mean over its R angular samples. */
double orc_pixel(const orc_grid* g, const orc_camera* c, const double* x, int iu, int iv)
{
    return pixel_subset(g, c, x, iu, iv, 1, 0);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* y = A_S x for angular-sample subset idx of nsub (nsub <= 1: all samples). */
void orc_project_subset(const orc_grid* g, const orc_camera* cams, int ncam, const double* x,
                        double* y, int nsub, int idx, int nthreads)
{
    set_threads(nthreads);
    int64_t off = 0;
    for (int ci = 0; ci < ncam; ++ci) {
        const orc_camera* c = &cams[ci];
        const int64_t np = (int64_t)c->nu * c->nv;
        double* yc = y + off;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t p = 0; p < np; ++p)
            yc[p] = pixel_subset(g, c, x, (int)(p % c->nu), (int)(p / c->nu), nsub, idx);
        off += np;
    }
}

/* y = A x for all cameras, y concatenated camera by camera, each (nv, nu). */
void orc_project(const orc_grid* g, const orc_camera* cams, int ncam,
                 const double* x, double* y, int nthreads)
{
    set_threads(nthreads);
    int64_t off = 0;
    for (int ci = 0; ci < ncam; ++ci) {
        const orc_camera* c = &cams[ci];
        const int64_t np = (int64_t)c->nu * c->nv;
        double* yc = y + off;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t p = 0; p < np; ++p)
            yc[p] = orc_pixel(g, c, x, (int)(p % c->nu), (int)(p / c->nu));
        off += np;
    }
}

/* y for a list of pixels of one camera (sampled checks at full size). */
void orc_project_pixels(const orc_grid* g, const orc_camera* c, const double* x,
                        const int64_t* pix, int64_t n, double* out, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k)
        out[k] = orc_pixel(g, c, x, (int)(pix[k] % c->nu), (int)(pix[k] / c->nu));
}

/* x = A_S^T y (nsub <= 1: A^T y).  Each thread scatters into a private FP64
 * volume; the volumes are then added in thread order, so the result depends
 * only on the thread count. */
void orc_backproject_subset(const orc_grid* g, const orc_camera* cams, int ncam,
                            const double* y, double* x, int nsub, int idx, int nthreads)
{
    set_threads(nthreads);
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    memset(x, 0, sizeof(double) * N);
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double* priv = (double*)calloc((size_t)nt * (size_t)N, sizeof(double));
    if (!priv) return;
    int64_t off = 0;
    for (int ci = 0; ci < ncam; ++ci) {
        const orc_camera* c = &cams[ci];
        const int64_t np = (int64_t)c->nu * c->nv;
        const int ns = subset_size(c->ru * c->rv, nsub, idx);
        const double* yc = y + off;
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* xt = priv + (size_t)tid * (size_t)N;
#pragma omp for schedule(static)
            for (int64_t p = 0; p < np; ++p) {
                if (yc[p] == 0.0) continue;
                const int iu = (int)(p % c->nu), iv = (int)(p / c->nu);
                for (int path = 0; path < orc_paths(c); ++path)
                    for (int rv = 0; rv < c->rv; ++rv)
                        for (int ru = 0; ru < c->ru; ++ru) {
                            double O[3], w[3];
                            if (!in_subset(ru + c->ru * rv, nsub, idx)) continue;
                            if (!orc_trace_path(c, iu, iv, path, ru, rv, O, w)) continue;
                            ray_scatter(g, xt, O, w, c->samples, yc[p] / ns);
                        }
            }
        }
        off += np;
    }
    for (int t = 0; t < nt; ++t) {
        const double* xt = priv + (size_t)t * (size_t)N;
        for (int64_t j = 0; j < N; ++j) x[j] += xt[j];
    }
    free(priv);
}

void orc_backproject(const orc_grid* g, const orc_camera* cams, int ncam,
                     const double* y, double* x, int nthreads)
{
    orc_backproject_subset(g, cams, ncam, y, x, 1, 0, nthreads);
}

/* Number of rays (over all pixels and angular samples) that are unoccluded
 * and hit the grid: the valid-sample count is this times S. */
int64_t orc_count_valid_rays(const orc_grid* g, const orc_camera* c, int nthreads)
{
    set_threads(nthreads);
    const int64_t np = (int64_t)c->nu * c->nv;
    int64_t count = 0;
#pragma omp parallel for reduction(+ : count) schedule(dynamic, 256)
    for (int64_t p = 0; p < np; ++p)
        for (int path = 0; path < orc_paths(c); ++path)
            for (int rv = 0; rv < c->rv; ++rv)
                for (int ru = 0; ru < c->ru; ++ru) {
                    double O[3], w[3], zr[2];
                    if (!orc_trace_path(c, (int)(p % c->nu), (int)(p / c->nu), path, ru, rv, O, w))
                        continue;
                    if (orc_clip(g, O, w, zr)) ++count;
                }
    return count;
}
