"""Pins of the oracle's ray optics and sampling against closed forms.

Each test checks the FP64 oracle against a property fixed by the paper's
optics or by plain mathematics, never against a retyped copy of its code:

* thin-lens focusing: all rays of a pixel meet at the detector's conjugate
  plane 1/d + 1/D = 1/f, at the inverted, magnified pixel position (the
  composition of the propagation and thin-lens maps of the optics table);
* plenoptic chain: rays leaving one lenslet point meet at the main-lens image
  of the MLA plane; rays of one pixel meet at the main-lens image of the
  lenslet's virtual image of that pixel; a ray through a lenslet centre is
  undeviated;
* occlusion: aperture samples outside the unit disc are dropped;
* uniform volume: y = intensity x chord, the chord found by bisection;
* an axis-aligned ray through voxel centres integrates to pitch x sum;
* trilinear sampling agrees with scipy.ndimage.map_coordinates;
* midpoint sampling converges at second order to the continuous integral;
* a 90 degree pose equals a permuted volume; a mirrored volume gives a
  mirrored image.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

from paper_1812_03358_amd import workloads as W


def _point_at_depth(O, w, depth):
    # w . e_z = 1 and O lies on the lens plane, so camera depth == ray parameter
    return O + depth * w


def test_ray_parameter_is_camera_depth(orc):
    cam = W.plenoptic_camera(64, 4, (2, 2), 16, phi_deg=37.0)
    ez = np.array(cam["axes"][6:9])
    L = np.array(cam["lens_center"])
    for (iu, iv, ru, rv) in [(0, 0, 0, 0), (17, 40, 1, 0), (63, 63, 1, 1)]:
        _, O, w = orc.trace(cam, iu, iv, ru, rv)
        assert abs(np.dot(w, ez) - 1.0) < 1e-14
        assert abs(np.dot(O - L, ez)) < 1e-12


@pytest.mark.parametrize("phi", [0.0, 30.0, 90.0])
def test_thin_lens_rays_focus_at_conjugate_plane(orc, phi):
    cam = W.single_lens_camera(16, (4, 4), 8, phi_deg=phi)
    f, D = cam["f_main"], cam["d_det"]
    d_img = 1.0 / (1.0 / f - 1.0 / D)          # lens equation
    es, et, ez = (np.array(cam["axes"][3 * k:3 * k + 3]) for k in range(3))
    L = np.array(cam["lens_center"])
    p = cam["pixel_pitch"]
    for iu, iv in [(0, 0), (5, 11), (15, 15), (8, 7)]:
        sd = (iu + 0.5 - 8) * p
        td = (iv + 0.5 - 8) * p
        expect = L + (-sd * d_img / D) * es + (-td * d_img / D) * et + d_img * ez
        for ru in range(4):
            for rv in range(4):
                _, O, w = orc.trace(cam, iu, iv, ru, rv)
                P = _point_at_depth(O, w, d_img)
                assert np.max(np.abs(P - expect)) < 1e-9


def test_thin_lens_aperture_occlusion(orc):
    # 4x4 aperture grid: cell centres (+-1/4, +-3/4); the 4 corners (3/4,3/4)
    # lie outside the unit disc, the other 12 inside.
    cam = W.single_lens_camera(8, (4, 4), 8)
    for iu, iv in [(0, 0), (3, 6)]:
        valid = [orc.trace(cam, iu, iv, ru, rv)[0] for rv in range(4) for ru in range(4)]
        assert sum(valid) == 12
        assert not valid[0] and not valid[3] and not valid[12] and not valid[15]


def _lenslet_centre(cam, lu, lv):
    k = cam["det_nu"] // cam["mla_nu"]
    P = k * cam["pixel_pitch"]
    return ((lu + 0.5 - cam["mla_nu"] / 2) * P, (lv + 0.5 - cam["mla_nv"] / 2) * P)


@pytest.mark.parametrize("phi", [0.0, 60.0])
def test_plenoptic_lenslet_point_images_to_mla_conjugate(orc, phi):
    cam = W.plenoptic_camera(64, 4, (2, 2), 8, phi_deg=phi)
    f, Dm = cam["f_main"], cam["d_mla"]
    d_c = 1.0 / (1.0 / f - 1.0 / Dm)           # conjugate of the MLA plane: 1680 mm
    es, et, ez = (np.array(cam["axes"][3 * k:3 * k + 3]) for k in range(3))
    L = np.array(cam["lens_center"])
    r = cam["r_mla"]
    k = 16
    for lu, lv in [(0, 0), (2, 1), (3, 3)]:
        cs, ct = _lenslet_centre(cam, lu, lv)
        for ru in range(2):
            for rv in range(2):
                gs, gt = (2 * ru + 1) / 2 - 1, (2 * rv + 1) / 2 - 1
                a_s, a_t = cs + r * gs, ct + r * gt
                expect = L + (-a_s * d_c / Dm) * es + (-a_t * d_c / Dm) * et + d_c * ez
                for pu in (0, 5, 15):
                    for pv in (0, 9, 15):
                        _, O, w = orc.trace(cam, lu * k + pu, lv * k + pv, ru, rv)
                        P = _point_at_depth(O, w, d_c)
                        assert np.max(np.abs(P - expect)) < 1e-9 * d_c


def test_plenoptic_pixel_rays_meet_at_image_of_virtual_pixel(orc):
    # The lenslet forms a virtual image of the pixel (object distance D_ud <
    # f_u); the main lens images that virtual point.  All aperture samples of
    # the pixel pass through the final image point.
    cam = W.plenoptic_camera(64, 4, (4, 4), 8, phi_deg=15.0)
    f, Dm, Dd, fu = cam["f_main"], cam["d_mla"], cam["d_mla_det"], cam["f_mla"]
    b = 1.0 / (1.0 / fu - 1.0 / Dd)            # negative: virtual image
    assert b < 0
    mag = -b / Dd                               # upright virtual magnification
    obj = Dm - b                                # its distance behind the main lens
    z_img = 1.0 / (1.0 / f - 1.0 / obj)
    es, et, ez = (np.array(cam["axes"][3 * k:3 * k + 3]) for k in range(3))
    L = np.array(cam["lens_center"])
    p = cam["pixel_pitch"]
    for iu, iv in [(3, 4), (20, 50), (63, 0)]:
        cs, ct = _lenslet_centre(cam, iu // 16, iv // 16)
        sd, td = (iu + 0.5 - 32) * p, (iv + 0.5 - 32) * p
        vs, vt = cs + mag * (sd - cs), ct + mag * (td - ct)
        expect = L + (-vs * z_img / obj) * es + (-vt * z_img / obj) * et + z_img * ez
        for ru in range(4):
            for rv in range(4):
                _, O, w = orc.trace(cam, iu, iv, ru, rv)
                P = _point_at_depth(O, w, z_img)
                assert np.max(np.abs(P - expect)) < 1e-9 * z_img


def test_plenoptic_lenslet_chief_ray_undeviated(orc):
    cam = W.plenoptic_camera(64, 4, (1, 1), 8)
    Dm, Dd = cam["d_mla"], cam["d_mla_det"]
    es, et = np.array(cam["axes"][0:3]), np.array(cam["axes"][3:6])
    L = np.array(cam["lens_center"])
    p = cam["pixel_pitch"]
    for iu, iv in [(0, 0), (7, 30), (40, 63)]:
        cs, ct = _lenslet_centre(cam, iu // 16, iv // 16)
        sd, td = (iu + 0.5 - 32) * p, (iv + 0.5 - 32) * p
        # straight line pixel -> lenslet centre, continued to the main lens
        s_lens = cs + (cs - sd) * Dm / Dd
        t_lens = ct + (ct - td) * Dm / Dd
        _, O, _ = orc.trace(cam, iu, iv, 0, 0)
        assert abs(np.dot(O - L, es) - s_lens) < 1e-12
        assert abs(np.dot(O - L, et) - t_lens) < 1e-12


def test_plenoptic_main_aperture_vignetting(orc):
    # valid <=> the ray crosses the main-lens plane inside radius r_main
    cam = W.plenoptic_camera(64, 4, (2, 2), 8)
    es, et = np.array(cam["axes"][0:3]), np.array(cam["axes"][3:6])
    L = np.array(cam["lens_center"])
    n_in = n_out = 0
    for iu in range(0, 64, 3):
        for iv in range(0, 64, 5):
            for ru in range(2):
                for rv in range(2):
                    v, O, _ = orc.trace(cam, iu, iv, ru, rv)
                    rad = math.hypot(np.dot(O - L, es), np.dot(O - L, et))
                    assert v == (rad <= cam["r_main"])
                    n_in += v
                    n_out += not v
    assert n_in > 0 and n_out > 0              # the geometry vignettes some rays


def _inside(g, P):
    h = 0.5 * np.array([g["nx"], g["ny"], g["nz"]]) * g["pitch"]
    return bool(np.all(np.abs(P) <= h))


def _bisect_chord(g, O, w, z_in):
    """Chord length by bisection of the inside-box predicate from a point
    known to be inside; independent of any slab computation."""
    def edge(direction):
        lo, hi = z_in, z_in + direction * 1e4
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _inside(g, O + mid * w):
                lo = mid
            else:
                hi = mid
        return lo
    z1 = edge(+1.0)
    z0 = max(edge(-1.0), 0.0)
    return (z1 - z0) * np.linalg.norm(w)


@pytest.mark.parametrize("which", ["thin", "plen"])
def test_uniform_volume_gives_intensity_times_chord(orc, which):
    if which == "thin":
        g = W.grid((9, 8, 7), 0.25)
        cam = W.single_lens_camera(12, (2, 2), 5, phi_deg=30.0)
    else:
        g = W.grid((10, 12, 9), 3.0)
        cam = W.plenoptic_camera(48, 3, (2, 2), 7, phi_deg=20.0)
    c = 0.7
    x = np.full(g["nx"] * g["ny"] * g["nz"], c)
    y = orc.project(g, [cam], x)
    R = cam["rays_u"] * cam["rays_v"]
    hits = 0
    for iv in range(cam["det_nv"]):
        for iu in range(cam["det_nu"]):
            acc = 0.0
            for rv in range(cam["rays_v"]):
                for ru in range(cam["rays_u"]):
                    v, O, w = orc.trace(cam, iu, iv, ru, rv)
                    if not v:
                        continue
                    hit, z0, z1 = orc.clip(g, O, w)
                    if hit:
                        hits += 1
                        assert _inside(g, O + 0.5 * (z0 + z1) * w)
                        acc += _bisect_chord(g, O, w, 0.5 * (z0 + z1))
                    else:
                        # a miss really misses: dense scan finds no inside point
                        zs = np.linspace(0, 2 * np.linalg.norm(cam["lens_center"]), 4001)
                        assert not any(_inside(g, O + z * w) for z in zs[::40])
            expect = c * acc / R
            assert abs(y[iv * cam["det_nu"] + iu] - expect) <= 1e-12 * max(1.0, expect)
    assert hits > 10


@pytest.mark.parametrize("phi,axis", [(0.0, "z"), (90.0, "x")])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_axis_ray_through_voxel_centres(orc, phi, axis, k):
    n = 9
    g = W.grid(n, 0.4)
    cam = W.single_lens_camera(65, (1, 1), n * k, phi_deg=phi)  # centre pixel on axis
    x = W.uniform_random((n, n, n), seed=5).astype(np.float64)
    y = orc.project(g, [cam], x.reshape(-1)).reshape(65, 65)
    c = n // 2
    line = x[:, c, c] if axis == "z" else x[c, c, :]
    assert abs(y[32, 32] - g["pitch"] * line.sum()) < 1e-13 * line.sum()


def _sample_points(g, O, w, z0, z1, S):
    z = z0 + (np.arange(S) + 0.5) * (z1 - z0) / S
    P = O[None, :] + z[:, None] * w[None, :]
    n = np.array([g["nx"], g["ny"], g["nz"]], dtype=np.float64)
    q = P / g["pitch"] + 0.5 * n - 0.5      # voxel centres on integers
    return q


def _library_ray_integral(g, vol, O, w, z0, z1, S):
    q = _sample_points(g, O, w, z0, z1, S)
    # map_coordinates on a (z, y, x) array; 'nearest' replicates the edge,
    # which is the clamp-to-edge of the voxel values
    vals = ndimage.map_coordinates(vol, [q[:, 2], q[:, 1], q[:, 0]], order=1, mode="nearest")
    return vals.sum() * (z1 - z0) * np.linalg.norm(w) / S


@pytest.mark.parametrize("which", ["thin", "plen"])
def test_trilinear_samples_match_map_coordinates(orc, which):
    if which == "thin":
        g = W.grid((11, 9, 10), 0.3)
        cam = W.single_lens_camera(10, (2, 1), 23, phi_deg=25.0)
    else:
        g = W.grid((12, 10, 11), 2.5)
        cam = W.plenoptic_camera(32, 2, (2, 2), 19, phi_deg=50.0)
    vol = W.uniform_random((g["nz"], g["ny"], g["nx"]), seed=9).astype(np.float64)
    y = orc.project(g, [cam], vol.reshape(-1))
    R = cam["rays_u"] * cam["rays_v"]
    checked = 0
    for iu, iv in [(0, 0), (3, 4), (5, 5), (9, 2), (7, 8), (4, 6)]:
        acc = 0.0
        for rv in range(cam["rays_v"]):
            for ru in range(cam["rays_u"]):
                v, O, w = orc.trace(cam, iu, iv, ru, rv)
                hit, z0, z1 = orc.clip(g, O, w)
                if v and hit:
                    acc += _library_ray_integral(g, vol, O, w, z0, z1, cam["samples"])
                    checked += 1
        assert abs(y[iv * cam["det_nu"] + iu] - acc / R) < 1e-12 * max(1.0, abs(acc))
    assert checked > 3


def test_midpoint_sampling_is_second_order(orc):
    g = W.grid(16, 1.0)
    vol = W.blobs(16, seed=3).astype(np.float64)
    cam = W.single_lens_camera(8, (1, 1), 8, phi_deg=20.0)
    # rays of a few pixels, distance chosen so they cross the volume
    errs = {}
    ref = {}
    for iu, iv in [(3, 4), (4, 4), (2, 5)]:
        _, O, w = orc.trace(cam, iu, iv, 0, 0)
        hit, z0, z1 = orc.clip(g, O, w)
        assert hit
        ref[(iu, iv)] = _library_ray_integral(g, vol, O, w, z0, z1, 1 << 18)
    Ss = (64, 128, 256, 512, 1024)
    for S in Ss:
        c = dict(cam, samples=S)
        y = orc.project(g, [c], vol.reshape(-1))
        errs[S] = sum(abs(y[iv * 8 + iu] - ref[(iu, iv)]) for iu, iv in ref)
    # The interpolant is piecewise cubic with kinks at cell faces, so single
    # ratios oscillate; the order fitted over four doublings is 2 for
    # midpoints (an end-point rule would give 1).
    order = math.log2(errs[Ss[0]] / errs[Ss[-1]]) / (len(Ss) - 1)
    assert 1.7 < order < 2.7, (order, errs)
    scaled = [errs[S] * S * S for S in Ss]
    assert max(scaled) / min(scaled) < 10.0, scaled


@pytest.mark.parametrize("which", ["thin", "plen"])
def test_pose_90_equals_permuted_volume(orc, which):
    n = 10
    if which == "thin":
        g = W.grid(n, 0.3)
        c0 = W.single_lens_camera(12, (2, 2), 17, phi_deg=0.0)
        c90 = W.single_lens_camera(12, (2, 2), 17, phi_deg=90.0)
    else:
        g = W.grid(n, 8.0)
        c0 = W.plenoptic_camera(32, 4, (2, 2), 17, phi_deg=0.0)
        c90 = W.plenoptic_camera(32, 4, (2, 2), 17, phi_deg=90.0)
    v90 = W.uniform_random((n, n, n), seed=21).astype(np.float64)
    # a camera at 90 degrees maps camera (s, t, z) to world (z - d, t, -s)
    v0 = np.flip(v90, axis=0).transpose(2, 1, 0).copy()
    y90 = orc.project(g, [c90], v90.reshape(-1))
    y0 = orc.project(g, [c0], v0.reshape(-1))
    assert np.max(np.abs(y90 - y0)) <= 1e-12 * np.max(np.abs(y0))
    assert np.max(y0) > 0


@pytest.mark.parametrize("which", ["thin", "plen"])
def test_mirrored_volume_gives_mirrored_image(orc, which):
    if which == "thin":
        g = W.grid((8, 9, 10), 0.3)
        cam = W.single_lens_camera(12, (2, 2), 13)
    else:
        g = W.grid((8, 9, 10), 8.0)
        cam = W.plenoptic_camera(32, 4, (2, 2), 13)
    v = W.uniform_random((10, 9, 8), seed=4).astype(np.float64)
    y = orc.project(g, [cam], v.reshape(-1)).reshape(cam["det_nv"], cam["det_nu"])
    ym = orc.project(g, [cam], v[:, :, ::-1].copy().reshape(-1)).reshape(y.shape)
    assert np.max(np.abs(ym - y[:, ::-1])) <= 1e-12 * np.max(np.abs(y))
