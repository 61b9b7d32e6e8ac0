"""Seeded synthetic inputs and camera/grid descriptions.

This module holds no arithmetic of the camera model itself: it only draws
random volumes and noise and lists geometry constants.  Both the FP64 oracle
(``oracle/``) and the HIP path read their inputs from here, so the two never
share any code that computes A, A^T or the solver.

Volumes are float32 arrays of shape (nz, ny, nx), x fastest, y vertical.
Index coordinates q in [0, n-1]^3 put voxel centres on integers.

Camera dicts use plain Python numbers; each side marshals them into its own
C struct.  Geometry constants follow the paper's simulated cameras:
  * single-lens camera: Table "Simulated single-lens camera configuration"
    (f = 30 mm, lens radius 5 mm, D = 31.3 mm, 5 um pixels);
  * plenoptic camera: Table "Simulated plenoptic camera configuration"
    (f = 105 mm, radius 4.5 mm, D_um = 112 mm, D_ud = 2.2 mm, lenslet radius
    100 um), read with a square lenslet grid, one lenslet focal length
    (3.0 mm, the middle of the three listed) and 16 px per 0.2 mm lenslet.
Each camera sits at the distance where its detector (single lens) or its
microlens array (plenoptic) is in focus on the volume centre.
"""
from __future__ import annotations

import math

import numpy as np

SINGLE_LENS = 0
PLENOPTIC = 1
PLENOPTIC_HEX = 2

# --------------------------------------------------------------------------
# geometry constants (mm)
# --------------------------------------------------------------------------
TL_F, TL_R, TL_D, TL_PITCH = 30.0, 5.0, 31.3, 0.005
PL_F, PL_R, PL_DMM, PL_DMD = 105.0, 4.5, 112.0, 2.2
PL_FMU, PL_RMU, PL_PMU = 3.0, 0.1, 0.2
PL_FHEX = (2.8, 3.0, 3.2)       # the three lenslet focal lengths of the table
PL_HEX_PIXEL = 0.005            # 5 um pixels of the table


def azimuth_axes(phi_deg: float):
    """Camera axes (e_s, e_t, e_z) for a camera rotated by phi about world y.

    e_z points from the lens into the scene; (e_s, e_t, e_z) is right-handed.
    """
    p = math.radians(phi_deg)
    c, s = math.cos(p), math.sin(p)
    # exact zeros/ones at multiples of 90 degrees keep poses exact
    if abs(c) < 1e-15:
        c = 0.0
    if abs(s) < 1e-15:
        s = 0.0
    return [c, 0.0, -s, 0.0, 1.0, 0.0, s, 0.0, c]


def _place(cam: dict, distance: float, phi_deg: float) -> dict:
    ax = azimuth_axes(phi_deg)
    ez = ax[6:9]
    cam["axes"] = ax
    cam["lens_center"] = [-distance * ez[0], -distance * ez[1], -distance * ez[2]]
    cam["phi_deg"] = phi_deg
    return cam


def single_lens_camera(det: int = 64, rays=(1, 1), samples: int = 64,
                       phi_deg: float = 0.0, det_v: int | None = None,
                       distance: float | None = None, r_main: float = TL_R) -> dict:
    """Single-lens camera of the paper's simulated single-lens table
    (r_main: the main-lens aperture radius, the table's 5 mm by default)."""
    if distance is None:
        distance = TL_F * TL_D / (TL_D - TL_F)  # detector conjugate plane
    cam = dict(kind=SINGLE_LENS, det_nu=det, det_nv=det if det_v is None else det_v,
               mla_nu=0, mla_nv=0, rays_u=rays[0], rays_v=rays[1],
               samples=samples, pixel_pitch=TL_PITCH, f_main=TL_F, r_main=r_main,
               d_det=TL_D, d_mla=0.0, d_mla_det=0.0, f_mla=0.0, r_mla=0.0)
    return _place(cam, distance, phi_deg)


def plenoptic_camera(det: int = 1024, mla: int = 64, rays=(2, 2), samples: int = 256,
                     phi_deg: float = 0.0, distance: float | None = None) -> dict:
    """Plenoptic camera of the paper's simulated plenoptic table (square MLA)."""
    if det % mla:
        raise ValueError("detector size must be a multiple of the lenslet count")
    k = det // mla
    if distance is None:
        distance = PL_F * PL_DMM / (PL_DMM - PL_F)  # MLA conjugate plane: 1680 mm
    cam = dict(kind=PLENOPTIC, det_nu=det, det_nv=det, mla_nu=mla, mla_nv=mla,
               rays_u=rays[0], rays_v=rays[1], samples=samples,
               pixel_pitch=PL_PMU / k, f_main=PL_F, r_main=PL_R, d_det=0.0,
               d_mla=PL_DMM, d_mla_det=PL_DMD, f_mla=PL_FMU, r_mla=PL_RMU)
    return _place(cam, distance, phi_deg)


def hex_plenoptic_camera(det: int = 2048, mla=None, rays=(2, 2), samples: int = 256,
                         phi_deg: float = 0.0, distance: float | None = None,
                         f_hex=PL_FHEX, r_main: float = PL_R) -> dict:
    """Plenoptic camera of the paper's simulated plenoptic table as listed:
    hexagonal array of touching 100 um lenslets of three focal lengths, 5 um
    pixels, every pixel summing the light of all lenslets.  ``mla`` =
    (lenslets per row, rows); the default covers the detector with one
    lenslet to spare on each side."""
    p = 2.0 * PL_RMU
    if mla is None:
        side = det * PL_HEX_PIXEL
        mla = (int(math.ceil(side / p)) + 1, int(math.ceil(side / (p * math.sqrt(3) / 2))) + 1)
    if distance is None:
        distance = PL_F * PL_DMM / (PL_DMM - PL_F)
    cam = dict(kind=PLENOPTIC_HEX, det_nu=det, det_nv=det, mla_nu=int(mla[0]), mla_nv=int(mla[1]),
               rays_u=rays[0], rays_v=rays[1], samples=samples, pixel_pitch=PL_HEX_PIXEL,
               f_main=PL_F, r_main=r_main, d_det=0.0, d_mla=PL_DMM, d_mla_det=PL_DMD,
               f_mla=f_hex[1], r_mla=PL_RMU, f_hex=[float(f) for f in f_hex])
    return _place(cam, distance, phi_deg)


def grid(n, pitch: float) -> dict:
    if isinstance(n, int):
        n = (n, n, n)
    return dict(nx=int(n[0]), ny=int(n[1]), nz=int(n[2]), pitch=float(pitch))


def n_pixels(cam: dict) -> int:
    return cam["det_nu"] * cam["det_nv"]


def n_rays(cam: dict) -> int:
    return n_pixels(cam) * cam["rays_u"] * cam["rays_v"]


# --------------------------------------------------------------------------
# volumes
# --------------------------------------------------------------------------
def blobs(n: int = 32, seed: int = 1, count: int = 3) -> np.ndarray:
    """Isotropic Gaussian blobs: centres U[0.3,0.7](n-1), sigma U[2,5] voxels,
    amplitude U[0.5,1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.3, 0.7, size=(count, 3)) * (n - 1)
    sig = rng.uniform(2.0, 5.0, size=count)
    amp = rng.uniform(0.5, 1.0, size=count)
    q = np.arange(n, dtype=np.float64)
    vol = np.zeros((n, n, n))
    for k in range(count):
        gx = np.exp(-0.5 * ((q - c[k, 0]) / sig[k]) ** 2)
        gy = np.exp(-0.5 * ((q - c[k, 1]) / sig[k]) ** 2)
        gz = np.exp(-0.5 * ((q - c[k, 2]) / sig[k]) ** 2)
        vol += amp[k] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return vol.astype(np.float32)


def _value_noise_axis(n: int, spacing: float):
    """Lattice cell index and smoothstep weight along one axis."""
    t = np.arange(n, dtype=np.float64) / spacing
    i = np.floor(t).astype(np.int64)
    f = t - i
    w = f * f * (3.0 - 2.0 * f)
    return i, w


def _value_noise(n: int, spacing: float, rng: np.random.Generator) -> np.ndarray:
    g = int(math.floor((n - 1) / spacing)) + 2
    lat = rng.uniform(-1.0, 1.0, size=(g, g, g))  # (z, y, x)
    i, w = _value_noise_axis(n, spacing)
    # separable smoothstep-weighted interpolation, x then y then z
    t = lat[:, :, i] * (1 - w) + lat[:, :, i + 1] * w          # (gz, gy, nx)
    t = t[:, i, :] * (1 - w)[None, :, None] + t[:, i + 1, :] * w[None, :, None]  # (gz, ny, nx)
    t = t[i] * (1 - w)[:, None, None] + t[i + 1] * w[:, None, None]             # (nz, ny, nx)
    return t


def flame(n: int = 128, seed: int = 2) -> np.ndarray:
    """Flame-like volume: 8 anisotropic Gaussian plumes stacked along y,
    modulated by 3 octaves of value-noise turbulence, clipped at 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = 8
    offx = rng.uniform(-0.03, 0.03, K)
    offz = rng.uniform(-0.03, 0.03, K)
    amp = rng.uniform(0.5, 1.0, K) * (1.0 - 0.5 * np.arange(K) / (K - 1))
    q = np.arange(n, dtype=np.float64)
    sv = 0.1 * n
    plume = np.zeros((n, n, n))
    for k in range(K):
        mx = (n - 1) / 2 + offx[k] * (n - 1)
        mz = (n - 1) / 2 + offz[k] * (n - 1)
        my = (0.15 + 0.1 * k) * (n - 1)
        sh = (0.04 + 0.06 * k / (K - 1)) * n
        gx = np.exp(-0.5 * ((q - mx) / sh) ** 2)
        gz = np.exp(-0.5 * ((q - mz) / sh) ** 2)
        gy = np.exp(-0.5 * ((q - my) / sv) ** 2)
        plume += amp[k] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    turb = np.zeros((n, n, n))
    for weight, div in ((1.0, 8), (0.5, 16), (0.25, 32)):
        turb += weight * _value_noise(n, n / div, rng)
    m = np.abs(turb).max()
    if m > 0:
        turb /= m
    vol = np.maximum(0.0, plume * (1.0 + 0.35 * turb))
    return vol.astype(np.float32)


def uniform_random(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape).astype(np.float32)


# --------------------------------------------------------------------------
# measurement noise (takes the clean image as input; draws only)
# --------------------------------------------------------------------------
def gaussian_noise(y_clean: np.ndarray, seed: int, level: float = 0.01) -> np.ndarray:
    """Additive Gaussian noise with sigma = level * ||y||_2 / sqrt(M)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y = np.asarray(y_clean, dtype=np.float64)
    sigma = level * np.linalg.norm(y) / math.sqrt(y.size)
    return (y + sigma * rng.standard_normal(y.shape)).astype(np.float32)


def poisson_noise(y_clean: np.ndarray, seed: int, peak: float = 1000.0) -> np.ndarray:
    """Poisson counts with the brightest pixel at `peak` counts, rescaled back."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y = np.asarray(y_clean, dtype=np.float64)
    mx = float(y.max())
    if mx <= 0:
        return y.astype(np.float32)
    counts = rng.poisson(np.maximum(y, 0.0) * (peak / mx))
    return (counts * (mx / peak)).astype(np.float32)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def config_thin_lens():
    """32^3 blobs, single-lens camera 64^2, 1 ray/pixel, 64 samples/ray."""
    return dict(name="thin_lens_32", grid=grid(32, 0.2),
                cameras=[single_lens_camera(64, (1, 1), 64)],
                volume=lambda: blobs(32, 1), noise_seed=11)


def config_plenoptic():
    """128^3 flame, plenoptic 1024^2 behind 64^2 lenslets, 2x2 rays, 256 samples."""
    return dict(name="plenoptic_128", grid=grid(128, 1.25),
                cameras=[plenoptic_camera(1024, 64, (2, 2), 256)],
                volume=lambda: flame(128, 2), noise_seed=12)


def config_batched(frames: int = 48, seed: int = 3):
    """48 frames with volumes of 96/128/160/192 (12 each, seeded order) x 4
    plenoptic cameras at 0/30/60/90 degrees, 1024^2 detectors, 2x2 rays,
    S = 2n samples per ray, 160 mm cube."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.repeat(np.array([96, 128, 160, 192]), frames // 4)
    rng.shuffle(sizes)
    out = []
    for f, n in enumerate(sizes.tolist()):
        out.append(dict(frame=f, grid=grid(n, 160.0 / n),
                        cameras=[plenoptic_camera(1024, 64, (2, 2), 2 * n, phi)
                                 for phi in (0.0, 30.0, 60.0, 90.0)],
                        volume_seed=300 + f))
    return out


def config_differentiable():
    """256^3 flame, 4 plenoptic cameras 2048^2 (128^2 lenslets), 2x1 rays, 512 samples."""
    return dict(name="differentiable_256", grid=grid(256, 1.25),
                cameras=[plenoptic_camera(2048, 128, (2, 1), 512, phi)
                         for phi in (0.0, 30.0, 60.0, 90.0)],
                volume=lambda: flame(256, 4))


def config_warm_start():
    """128^3 flames seen by 2 plenoptic cameras at 0 and 90 degrees."""
    return dict(name="warm_start_128", grid=grid(128, 1.25),
                cameras=[plenoptic_camera(1024, 64, (2, 2), 256, phi)
                         for phi in (0.0, 90.0)])


def config_hex_plenoptic():
    """The simulated plenoptic table as listed: 2048^2 px of 5 um behind a
    hexagonal 53 x 61 array of three focal lengths, light summed over all
    lenslets; 100^3 flame at 1 mm, 2x2 angular samples, 200 samples per ray."""
    return dict(name="hex_plenoptic_100", grid=grid(100, 1.0),
                cameras=[hex_plenoptic_camera(2048, None, (2, 2), 200)],
                volume=lambda: flame(100, 5), noise_seed=13)


def config_three_camera(n: int = 100, det_pl: int = 2048, mla: int = 128, det_tl: int = 1024,
                        rays=(8, 8), samples: int = 200):
    """One plenoptic camera head-on and two single-lens cameras at +-30 deg
    (the paper's three-camera experiment): 100^3 at 1 mm, an 8x8 angular grid
    per camera, no subsets.  ``gains`` are the planted gains that divide each
    camera's clean image (the first camera's is 1); per-pixel weights come
    from ``bayer_green_mask`` and ``damaged_mask``."""
    cams = [plenoptic_camera(det_pl, mla, rays, samples, 0.0),
            single_lens_camera(det_tl, rays, samples, 30.0),
            single_lens_camera(det_tl, rays, samples, -30.0)]
    return dict(name="three_camera_100", grid=grid(n, 100.0 / n), cameras=cams,
                volume=lambda: flame(n, 5), gains=[1.0, 0.8, 1.3])


def bayer_green_mask(nu: int, nv: int) -> np.ndarray:
    """1 on the green sites of an RGGB mosaic ((u + v) odd), else 0."""
    u = np.arange(nu)[None, :]
    v = np.arange(nv)[:, None]
    return (((u + v) % 2) == 1).astype(np.float32).reshape(-1)


def damaged_mask(nu: int, nv: int, box=(0.6, 0.8, 0.1, 0.3)) -> np.ndarray:
    """1 except a rectangular block (fractions u0, u1, v0, v1) set to 0."""
    m = np.ones((nv, nu), np.float32)
    u0, u1, v0, v1 = (int(box[0] * nu), int(box[1] * nu), int(box[2] * nv), int(box[3] * nv))
    m[v0:v1, u0:u1] = 0.0
    return m.reshape(-1)
