"""FP64 reference of the paper's own discretization: the L2-projected light
field transport with Dirac or pillbox angular bases, for a single-lens camera
looking head-on at a voxel volume collapsed into slices.

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``): imported by
tests/ and the benchmark's CPU leg, never by the product package.

What it computes, in the paper's notation:
  * optics    -- 3x3 affine ray maps on (s, u, 1) built from the propagation
                 T_d and the refraction R_f of the table of common affine
                 optical transformations; the angular plane is the main lens;
                 X^{0q} = (T_{z_q} o R_f)^{-1} for a slice at depth z_q,
                 X^{0d} = T_D for the detector, X^{pq} = (X^{0p})^{-1} o X^{0q}
                 (camera-model and light-transport sections);
  * transport -- the entries of B^{pq}_k from the Dirac and the pillbox
                 transport tables (blur kernel g, its breakpoints tau,
                 height h and magnification 1/alpha), integrated over the
                 source pixel; the s and t factors multiply (Kronecker
                 separability of the transport);
  * slices    -- each voxel slice of thickness dz radiates the light field
                 w_k = dz x_slice for every angular basis k (object-model
                 section, small-angle collapse);
  * occlusion -- angular cells whose centre lies outside the lens disc are
                 masked (occlusion section, the aperture rasterized on the
                 angular grid);
  * detector  -- f^d_k = B^{ds}_k w_k / V^d, and a pixel reads the mean over
                 the K angular cells of f^d_k.  The measurement section
                 writes sqrt(V^d) sum_k f^d_k; the constant is replaced by 1/K
                 so that the values share the units of the ray-driven
                 operator (mean over rays of line integrals), a global scale
                 the camera gains absorb.
The angular grid is Ks x Kt cells of size 2 r_main / K over the lens's
bounding square, as the ray-driven operator places its rays.
"""
from __future__ import annotations

import math

import numpy as np

DIRAC = 0
PILLBOX = 1


# --------------------------------------------------------------------------
# affine optics on (s, u, 1)
# --------------------------------------------------------------------------
def T(d: float) -> np.ndarray:
    """Propagation by d: s' = s + d u."""
    return np.array([[1.0, d, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def R(f: float, c: float = 0.0) -> np.ndarray:
    """Thin-lens refraction (focal length f, centre c): u' = u - (s - c)/f."""
    return np.array([[1.0, 0.0, 0.0], [-1.0 / f, 1.0, c / f], [0.0, 0.0, 1.0]])


def single_lens_maps(z_q: float, D: float, F: float):
    """(X^{0q}, X^{pq}, X^{0p}) for a slice at camera depth z_q, the detector
    D behind a lens of focal length F (rays run from the detector into the
    scene, z increasing)."""
    X0q = np.linalg.inv(T(z_q) @ R(F))
    X0p = T(D)
    Xpq = np.linalg.inv(X0p) @ X0q
    return X0q, Xpq, X0p


# --------------------------------------------------------------------------
# one-dimensional transport factors (the tables)
# --------------------------------------------------------------------------
def _overlap(a0, a1, b0, b1):
    return np.maximum(0.0, np.minimum(a1, b1) - np.maximum(a0, b0))


def _trapezoid_integral(lo, hi, t):
    """Integral over [lo, hi] of the trapezoid rising on [t1, t2], flat (1)
    on [t2, t3] and falling on [t3, t4]; vectorized over lo/hi."""
    t1, t2, t3, t4 = t

    def ramp_up(x):           # integral from t1 to x of (s - t1)/(t2 - t1), x in [t1, t2]
        return 0.5 * (x - t1) ** 2 / (t2 - t1) if t2 > t1 else 0.0 * x

    def ramp_dn(x):           # integral from t3 to x of 1 - (s - t3)/(t4 - t3)
        return ((x - t3) - 0.5 * (x - t3) ** 2 / (t4 - t3)) if t4 > t3 else 0.0 * x

    def G(x):                 # antiderivative from -inf
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros_like(x)
        m = (x > t1) & (x <= t2)
        out[m] = ramp_up(x[m])
        up = 0.5 * (t2 - t1)
        m = (x > t2) & (x <= t3)
        out[m] = up + (x[m] - t2)
        m = (x > t3) & (x <= t4)
        out[m] = up + (t3 - t2) + ramp_dn(x[m])
        m = x > t4
        out[m] = up + (t3 - t2) + 0.5 * (t4 - t3)
        return out

    return G(hi) - G(lo)


def transport_factor(basis: int, Xpq, X0q, sk: float, d0: float, si, dp: float, sj, dq: float,
                     axis: int = 0) -> np.ndarray:
    """[B^{pq}_{k,axis}]_{ij}: destination pixels centred at si (size dp) on
    plane p, source pixels centred at sj (size dq) on plane q, angular cell
    centred at sk (size d0) on the angular plane.  ``Xpq``/``X0q`` are the
    3x3 affine maps of that axis."""
    si = np.asarray(si, dtype=np.float64)
    sj = np.asarray(sj, dtype=np.float64)
    pss, psu, pbar = Xpq[0, 0], Xpq[0, 1], Xpq[0, 2]
    qss, qsu, qbar = X0q[0, 0], X0q[0, 1], X0q[0, 2]
    if basis == DIRAC:
        alpha = pss - qss * psu / qsu
        beta = pbar + psu * (sk - qbar) / qsu
        tau = np.sort([(0.5 * dp - beta) / alpha, (-0.5 * dp - beta) / alpha])
        h = d0 / abs(qsu)
        mag = 1.0 / alpha
        lo = si[:, None] * mag + tau[0]
        hi = si[:, None] * mag + tau[1]
        return h * _overlap(sj[None, :] - 0.5 * dq, sj[None, :] + 0.5 * dq, lo, hi)
    alpha = pss - psu * qss / qsu
    beta = psu / qsu
    gamma = pbar - psu * qbar / qsu
    tau = np.sort([(sp * 0.5 * dp - beta * (sk - s0 * 0.5 * d0) - gamma) / alpha
                   for sp in (1.0, -1.0) for s0 in (1.0, -1.0)])
    h = abs(d0 / qsu) if psu == 0.0 else min(abs(d0 / qsu), abs(dp / psu))
    mag = 1.0 / alpha
    lo = sj[None, :] - 0.5 * dq - si[:, None] * mag
    return h * _trapezoid_integral(lo, lo + dq, tau)


def detector_volume(basis: int, X0p, dp: float, d0: float) -> float:
    """One axis of V^p (the Dirac table's product form, or the pillbox
    table's 2 m h)."""
    ss, su = X0p[0, 0], X0p[0, 1]
    if basis == DIRAC:
        return dp * abs(d0 / su)
    m = max(d0 / (2.0 * abs(su)), dp * abs(ss / su) / 2.0)
    h = min(dp, d0 / abs(ss))
    return 2.0 * m * h


# --------------------------------------------------------------------------
# the camera operator
# --------------------------------------------------------------------------
def _check_head_on(cam: dict):
    if cam["kind"] != 0:
        raise ValueError("the transport operator models single-lens cameras")
    ax = np.asarray(cam["axes"], dtype=np.float64)
    if not np.array_equal(ax, np.eye(3).reshape(-1)) or cam["lens_center"][0] != 0.0 or \
            cam["lens_center"][1] != 0.0:
        raise ValueError("the transport operator needs a head-on camera on the z axis")


def angular_cells(cam: dict):
    """Centres (s_k, t_k) of the unmasked angular cells and the cell sizes."""
    Ks, Kt, r = cam["rays_u"], cam["rays_v"], cam["r_main"]
    d0s, d0t = 2.0 * r / Ks, 2.0 * r / Kt
    cells = []
    for kt in range(Kt):
        for ks in range(Ks):
            s = (ks + 0.5) * d0s - r
            t = (kt + 0.5) * d0t - r
            if s * s + t * t <= r * r:
                cells.append((s, t))
    return cells, d0s, d0t


def slice_factors(g: dict, cam: dict, basis: int):
    """Per slice iz and unmasked cell k: (Bs [nu, nx], Bt [nv, ny]) and the
    scale dz / (K V^d).  The grid pitch may be one size or (s, t, depth)
    sizes (the rotated grids of posed cameras)."""
    _check_head_on(cam)
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    pitch = g["pitch"]
    hx, hy, dx = (pitch, pitch, pitch) if np.isscalar(pitch) else pitch   # s, t, depth sizes
    nu, nv, dp = cam["det_nu"], cam["det_nv"], cam["pixel_pitch"]
    L = -cam["lens_center"][2]
    D, F = cam["d_det"], cam["f_main"]
    cells, d0s, d0t = angular_cells(cam)
    K = cam["rays_u"] * cam["rays_v"]
    si = (np.arange(nu) + 0.5 - 0.5 * nu) * dp
    ti = (np.arange(nv) + 0.5 - 0.5 * nv) * dp
    sj = (np.arange(nx) + 0.5 - 0.5 * nx) * hx
    tj = (np.arange(ny) + 0.5 - 0.5 * ny) * hy
    X0p = T(D)
    Vd = detector_volume(basis, X0p, dp, d0s) * detector_volume(basis, X0p, dp, d0t)
    scale = dx / (K * Vd)
    out = []
    for iz in range(nz):
        zq = L + (iz + 0.5 - 0.5 * nz) * dx
        X0q, Xpq, _ = single_lens_maps(zq, D, F)
        per = []
        for sk, tk in cells:
            Bs = transport_factor(basis, Xpq, X0q, sk, d0s, si, dp, sj, hx)
            Bt = transport_factor(basis, Xpq, X0q, tk, d0t, ti, dp, tj, hy)
            per.append((Bs, Bt))
        out.append(per)
    return out, scale


def project(g: dict, cam: dict, x, basis: int = PILLBOX) -> np.ndarray:
    """y = A x, image (nv, nu) flattened; x is (nz, ny, nx)."""
    x = np.asarray(x, dtype=np.float64).reshape(g["nz"], g["ny"], g["nx"])
    fac, scale = slice_factors(g, cam, basis)
    y = np.zeros((cam["det_nv"], cam["det_nu"]))
    for iz, per in enumerate(fac):
        for Bs, Bt in per:
            y += Bt @ x[iz] @ Bs.T
    return (scale * y).reshape(-1)


def backproject(g: dict, cam: dict, y, basis: int = PILLBOX) -> np.ndarray:
    """x = A^T y, volume (nz, ny, nx) flattened."""
    y = np.asarray(y, dtype=np.float64).reshape(cam["det_nv"], cam["det_nu"])
    fac, scale = slice_factors(g, cam, basis)
    x = np.zeros((g["nz"], g["ny"], g["nx"]))
    for iz, per in enumerate(fac):
        for Bs, Bt in per:
            x[iz] += Bt.T @ y @ Bs
    return (scale * x).reshape(-1)


# --------------------------------------------------------------------------
# rotated perspectives: scaling and shears with L2-projected resampling
# --------------------------------------------------------------------------
def _hat_antiderivative(d):
    """Integral from -inf to d of max(0, 1 - |t|)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.where(d <= -1.0, 0.0, 0.0)
    m = (d > -1.0) & (d <= 0.0)
    out = np.where(m, 0.5 * (d + 1.0) ** 2, out)
    m = (d > 0.0) & (d < 1.0)
    out = np.where(m, 1.0 - 0.5 * (1.0 - d) ** 2, out)
    return np.where(d >= 1.0, 1.0, out)


def shear_factor(zi, zj, h, shift, width):
    """[E]_{ij} for one column of a shear: the L2 projection onto boxes of
    size h (centres zi) of boxes of size h (centres zj) displaced by
    shift + t, t uniform over [-width/2, width/2] across the column's other
    coordinate: the mean over t of the box overlap h * hat(.) / h, a
    piecewise quadratic in (zi - zj + shift)."""
    d = (np.asarray(zi, np.float64)[:, None] - np.asarray(zj, np.float64)[None, :] + shift) / h
    if width == 0.0:
        return np.maximum(0.0, 1.0 - np.abs(d))
    w = width / h
    return (_hat_antiderivative(d + 0.5 * w) - _hat_antiderivative(d - 0.5 * w)) / w


def azimuth_shears(phi_deg: float):
    """Theta = D S_z S_x for a rotation about y by phi (|phi| <= 45 deg), in
    the x-z plane: D = diag(cos, 1/cos), S_z: z += a x with a = -sin cos,
    S_x: x += b z with b = tan.  Returns (cos, a, b)."""
    if abs(phi_deg) > 45.0 + 1e-9:
        raise ValueError("the three-shear rotation is used for |phi| <= 45 deg")
    p = math.radians(phi_deg)
    c, s = math.cos(p), math.sin(p)
    return c, -s * c, s / c


def rotated_grid(g: dict, phi_deg: float):
    """Voxel sizes and counts of the rotated coefficients (camera-aligned s,
    t, z'): sizes (d/cos, d, d cos); the shears widen the z' and s ranges so
    that the sheared support fits."""
    c, a, b = azimuth_shears(phi_deg)
    d = g["pitch"]
    hx, hz = d / c, d * c
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    nz2 = nz + 2 * int(math.ceil(0.5 * abs(a) * nx * hx / hz)) + 2
    nx3 = nx + 2 * int(math.ceil(0.5 * abs(b) * nz2 * hz / hx)) + 2
    return dict(hx=hx, hy=d, hz=hz, nx=nx3, ny=ny, nz=nz2, nx1=nx, nz1=nz, a=a, b=b, c=c)


def _centres(n, h):
    return (np.arange(n) + 0.5 - 0.5 * n) * h


def rotate_azimuth(g: dict, x, phi_deg: float):
    """x^r = E^x E^z x on the rotated grid (D only rescales the voxels):
    x is (nz, ny, nx) natural, the result (nz2, ny, nx3) in camera axes."""
    R = rotated_grid(g, phi_deg)
    x = np.asarray(x, np.float64).reshape(g["nz"], g["ny"], g["nx"])
    hx, hz, a, b = R["hx"], R["hz"], R["a"], R["b"]
    z1, z2 = _centres(R["nz1"], hz), _centres(R["nz"], hz)
    x1, x3 = _centres(R["nx1"], hx), _centres(R["nx"], hx)
    # E^z: per x column, shift a * x_c, spread |a| hx
    r = np.zeros((R["nz"], g["ny"], R["nx1"]))
    for ix, xc in enumerate(x1):
        E = shear_factor(z2, z1, hz, a * xc, abs(a) * hx)          # (nz2, nz1)
        r[:, :, ix] = E @ x[:, :, ix]
    # E^x: per z row, shift b * z_c, spread |b| hz
    out = np.zeros((R["nz"], g["ny"], R["nx"]))
    for iz, zc in enumerate(z2):
        E = shear_factor(x3, x1, hx, b * zc, abs(b) * hz)           # (nx3, nx1)
        out[iz] = r[iz] @ E.T
    return out, R


def rotate_azimuth_adjoint(g: dict, xr, phi_deg: float):
    """(E^x E^z)^T applied to rotated coefficients."""
    R = rotated_grid(g, phi_deg)
    xr = np.asarray(xr, np.float64).reshape(R["nz"], g["ny"], R["nx"])
    hx, hz, a, b = R["hx"], R["hz"], R["a"], R["b"]
    z1, z2 = _centres(R["nz1"], hz), _centres(R["nz"], hz)
    x1, x3 = _centres(R["nx1"], hx), _centres(R["nx"], hx)
    r = np.zeros((R["nz"], g["ny"], R["nx1"]))
    for iz, zc in enumerate(z2):
        E = shear_factor(x3, x1, hx, b * zc, abs(b) * hz)
        r[iz] = xr[iz] @ E
    out = np.zeros((g["nz"], g["ny"], g["nx"]))
    for ix, xc in enumerate(x1):
        E = shear_factor(z2, z1, hz, a * xc, abs(a) * hx)
        out[:, :, ix] = E.T @ r[:, :, ix]
    return out


def quarter_turns(phi_deg: float):
    """phi = 90 q + phi' with |phi'| <= 45 deg: the quarter turns q and phi'
    (rotated-perspective section: a rotation over 45 deg is a permutation,
    whole quarter turns, composed with a smaller rotation)."""
    q = int(round(phi_deg / 90.0))
    return q, phi_deg - 90.0 * q


def quarter_turn(g: dict, x, q: int):
    """The volume a camera at phi sees as if it stood at phi - 90 q: the
    value at p' is x(R(90 q) p'), R the rotation about y that maps camera
    axes (e_s, e_t, e_z) to world axes.  An exact permutation of voxels (with
    reversals); odd q swap the x and z extents.  Returns (x_q, g_q)."""
    x = np.asarray(x, np.float64).reshape(g["nz"], g["ny"], g["nx"])
    q %= 4
    if q == 0:
        return x.copy(), dict(g)
    if q == 2:
        return x[::-1, :, ::-1].copy(), dict(g)
    # x_q[iz'][iy][ix']: q = 1 reads x[nz-1-ix'][iy][iz'], q = 3 reads x[ix'][iy][nx-1-iz']
    t = np.transpose(x, (2, 1, 0))                       # t[ix][iy][iz] = x[iz][iy][ix]
    xq = t[:, :, ::-1] if q == 1 else t[::-1, :, :]
    return xq.copy(), dict(g, nx=g["nz"], nz=g["nx"])


def quarter_turn_adjoint(g: dict, xq, q: int):
    """The transpose (the inverse permutation) of ``quarter_turn``."""
    q %= 4
    gq = dict(g, nx=g["nz"], nz=g["nx"]) if q % 2 else dict(g)
    xq = np.asarray(xq, np.float64).reshape(gq["nz"], gq["ny"], gq["nx"])
    if q == 0:
        return xq.copy()
    if q == 2:
        return xq[::-1, :, ::-1].copy()
    t = xq[:, :, ::-1] if q == 1 else xq[::-1, :, :]     # back to t[ix][iy][iz]
    return np.transpose(t, (2, 1, 0)).copy()


def _camera_distance(cam: dict) -> float:
    L = np.asarray(cam["lens_center"], np.float64)
    ez = np.asarray(cam["axes"][6:9], np.float64)
    if abs(np.linalg.norm(L + np.dot(-L, ez) * ez)) > 1e-9 * np.linalg.norm(L):
        raise ValueError("the lens must lie on the camera axis through the grid centre")
    if abs(cam["axes"][4] - 1.0) > 1e-12:
        raise ValueError("only rotations about the grid's y axis (azimuth poses)")
    return float(-np.dot(L, ez))


def project_posed(g: dict, cam: dict, x, basis: int = PILLBOX) -> np.ndarray:
    """A x for a single-lens camera at azimuth phi: rotate the coefficients
    into the camera's axes (quarter turns, then the scaling and two shears of
    the remaining |phi'| <= 45 deg), then the head-on transport on the
    rotated grid's anisotropic voxels."""
    q, phi = quarter_turns(cam["phi_deg"])
    xq, gq = quarter_turn(g, x, q)
    xr, R = rotate_azimuth(gq, xq, phi)
    head = dict(cam, axes=[1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0],
                lens_center=[0.0, 0.0, -_camera_distance(cam)])
    gr = dict(nx=R["nx"], ny=R["ny"], nz=R["nz"], pitch=(R["hx"], R["hy"], R["hz"]))
    return project(gr, head, xr, basis)


def backproject_posed(g: dict, cam: dict, y, basis: int = PILLBOX) -> np.ndarray:
    q, phi = quarter_turns(cam["phi_deg"])
    gq = dict(g, nx=g["nz"], nz=g["nx"]) if q % 2 else dict(g)
    R = rotated_grid(gq, phi)
    head = dict(cam, axes=[1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0],
                lens_center=[0.0, 0.0, -_camera_distance(cam)])
    gr = dict(nx=R["nx"], ny=R["ny"], nz=R["nz"], pitch=(R["hx"], R["hy"], R["hz"]))
    xr = backproject(gr, head, y, basis)
    return quarter_turn_adjoint(g, rotate_azimuth_adjoint(gq, xr, phi), q).reshape(-1)


# --------------------------------------------------------------------------
# plenoptic camera: factorized transport through the lenslet array
# --------------------------------------------------------------------------
def plenoptic_maps(z_q: float, cam: dict, c_mu: float, f_mu: float):
    """Ray maps of the factorized plenoptic model (camera-model section):
    X^{0a} = T_{D_mu_m} (array plane -> lens), X^{0s} = (T_z R_F)^{-1}
    (slice -> lens), and through lenslet mu (centre c_mu, focal f_mu):
    X^{0d,mu} = X^{0a} R_mu T_{D_d_mu} (detector -> lens)."""
    X0a = T(cam["d_mla"])
    X0q = np.linalg.inv(T(z_q) @ R(cam["f_main"]))
    X0d = X0a @ R(f_mu, c_mu) @ T(cam["d_mla_det"])
    return X0a, X0q, X0d


def _volume_axis(basis, X0p, dp, d0):
    return detector_volume(basis, X0p, dp, d0)


def _plenoptic_parts(g: dict, cam: dict, basis: int, ka):
    if cam["kind"] != 1:
        raise ValueError("the factorized model is for square-array plenoptic cameras")
    _check_head_on(dict(cam, kind=0))
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    pitch = g["pitch"]
    hx, hy, dz = (pitch, pitch, pitch) if np.isscalar(pitch) else pitch   # s, t, depth sizes
    nu, nv, mu, mv = cam["det_nu"], cam["det_nv"], cam["mla_nu"], cam["mla_nv"]
    k = nu // mu
    ka = k if ka is None else ka
    P = k * cam["pixel_pitch"]                      # lenslet pitch
    da = P / ka                                     # array pixel
    na_u, na_v = mu * ka, mv * ka
    L = -cam["lens_center"][2]
    cells, d0s, d0t = angular_cells(cam)
    sa = (np.arange(na_u) + 0.5 - 0.5 * na_u) * da
    ta = (np.arange(na_v) + 0.5 - 0.5 * na_v) * da
    sj = (np.arange(nx) + 0.5 - 0.5 * nx) * hx
    tj = (np.arange(ny) + 0.5 - 0.5 * ny) * hy
    sd = (np.arange(nu) + 0.5 - 0.5 * nu) * cam["pixel_pitch"]
    td = (np.arange(nv) + 0.5 - 0.5 * nv) * cam["pixel_pitch"]
    cu = (np.arange(mu) + 0.5 - 0.5 * mu) * P
    cv = (np.arange(mv) + 0.5 - 0.5 * mv) * P
    own_u, own_v = np.arange(na_u) // ka, np.arange(na_v) // ka
    inside = ((sa - cu[own_u])[None, :] ** 2 + (ta - cv[own_v])[:, None] ** 2) <= cam["r_mla"] ** 2
    X0a = T(cam["d_mla"])
    Va = detector_volume(basis, X0a, da, d0s) * detector_volume(basis, X0a, da, d0t)
    _, _, X0d = plenoptic_maps(L, cam, 0.0, cam["f_mla"])
    Vd = detector_volume(basis, X0d, cam["pixel_pitch"], d0s) * \
        detector_volume(basis, X0d, cam["pixel_pitch"], d0t)
    omega = (2.0 * cam["r_mla"] / cam["d_mla_det"]) ** 2
    norm = d0s * d0t / (abs(X0d[0, 1]) ** 2 * omega)
    stage1 = []                                      # per cell: list over slices of (Bs, Bt)
    stage2 = []                                      # per cell: (Bs_full [nu, na_u], Bt_full [nv, na_v])
    for (sk, tk) in cells:
        per = []
        for iz in range(nz):
            zq = L + (iz + 0.5 - 0.5 * nz) * dz
            X0q = np.linalg.inv(T(zq) @ R(cam["f_main"]))
            Xaq = np.linalg.inv(X0a) @ X0q
            per.append((transport_factor(basis, Xaq, X0q, sk, d0s, sa, da, sj, hx),
                        transport_factor(basis, Xaq, X0q, tk, d0t, ta, da, tj, hy)))
        stage1.append(per)
        Bs2 = np.zeros((nu, na_u))
        Bt2 = np.zeros((nv, na_v))
        for lu in range(mu):
            _, _, X0d_s = plenoptic_maps(L, cam, cu[lu], cam["f_mla"])
            us = slice(lu * ka, (lu + 1) * ka)
            Bs2[:, us] = transport_factor(basis, np.linalg.inv(X0d_s) @ X0a, X0a, sk, d0s, sd,
                                          cam["pixel_pitch"], sa[us], da)
        for lv in range(mv):
            _, _, X0d_t = plenoptic_maps(L, cam, cv[lv], cam["f_mla"])
            vs = slice(lv * ka, (lv + 1) * ka)
            Bt2[:, vs] = transport_factor(basis, np.linalg.inv(X0d_t) @ X0a, X0a, tk, d0t, td,
                                          cam["pixel_pitch"], ta[vs], da)
        stage2.append((Bs2, Bt2))
    return dict(inside=inside, Va=Va, Vd=Vd, norm=norm, dz=dz, stage1=stage1, stage2=stage2,
                shape_a=(na_v, na_u), shape_d=(nv, nu), shape_x=(nz, ny, nx))


def project_plenoptic(g: dict, cam: dict, x, basis: int = PILLBOX, ka: int | None = None):
    """A x for a head-on square-array plenoptic camera in the paper's
    factorized form: every slice is transported onto the lenslet-array plane
    (array pixels of size pitch/ka, ka per lenslet; default the detector's
    pixels per lenslet), the mask keeps array pixels whose centre lies in a
    lenslet's aperture disc (the occluder rasterized on the array grid), and
    each lenslet transports its pixels onto the detector; f^a_k = B^{as}_k
    w_k / V^a, f^d_k = sum_mu B^{d mu}_k M_mu f^a_k / V^d.  Because each array
    column (row) belongs to one lenslet column (row), the lenslet stage is one
    separable banded transform per cell.  The pixel integral of the detector
    light field is sum_k f^d_k dp^2 d0s d0t / |X^{0d}_su X^{0d}_tv| (each
    cell integrated over the pixel's slopes); y divides it by dp^2 times the
    solid angle (2 r_mla / D_mu_d)^2 of the lenslet's bounding square, the
    angular domain the ray-driven operator averages over (for a single-lens
    camera the same rule, with (2 r_main / D)^2, is the mean over cells)."""
    Pp = _plenoptic_parts(g, cam, basis, ka)
    x = np.asarray(x, np.float64).reshape(Pp["shape_x"])
    y = np.zeros(Pp["shape_d"])
    for per, (Bs2, Bt2) in zip(Pp["stage1"], Pp["stage2"]):
        fa = np.zeros(Pp["shape_a"])
        for iz, (Bs, Bt) in enumerate(per):
            fa += Bt @ (Pp["dz"] * x[iz]) @ Bs.T
        fa = fa / Pp["Va"] * Pp["inside"]
        y += Bt2 @ fa @ Bs2.T / Pp["Vd"]
    return (y * Pp["norm"]).reshape(-1)


def backproject_plenoptic(g: dict, cam: dict, y, basis: int = PILLBOX, ka: int | None = None):
    """A^T y of ``project_plenoptic`` (the stages transposed in reverse)."""
    Pp = _plenoptic_parts(g, cam, basis, ka)
    y = np.asarray(y, np.float64).reshape(Pp["shape_d"]) * Pp["norm"]
    x = np.zeros(Pp["shape_x"])
    for per, (Bs2, Bt2) in zip(Pp["stage1"], Pp["stage2"]):
        fa = Bt2.T @ y @ Bs2 / Pp["Vd"]
        fa = fa / Pp["Va"] * Pp["inside"]
        for iz, (Bs, Bt) in enumerate(per):
            x[iz] += Pp["dz"] * (Bt.T @ fa @ Bs)
    return x.reshape(-1)


def _head_on_view(cam: dict):
    """The camera in its own axes (lens on the z axis at its distance)."""
    return dict(cam, axes=[1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0],
                lens_center=[0.0, 0.0, -_camera_distance(cam)])


def project_plenoptic_posed(g: dict, cam: dict, x, basis: int = PILLBOX, ka: int | None = None):
    """A x of the factorized plenoptic model for a square-array plenoptic
    camera at azimuth phi: the coefficients rotated into the camera's axes
    (quarter turns, then the scaling and two shears of the remaining
    |phi'| <= 45 deg), then the head-on factorized transport on the rotated
    grid's anisotropic voxels."""
    q, phi = quarter_turns(cam["phi_deg"])
    xq, gq = quarter_turn(g, x, q)
    xr, Rg = rotate_azimuth(gq, xq, phi)
    gr = dict(nx=Rg["nx"], ny=Rg["ny"], nz=Rg["nz"], pitch=(Rg["hx"], Rg["hy"], Rg["hz"]))
    return project_plenoptic(gr, _head_on_view(cam), xr, basis, ka)


def backproject_plenoptic_posed(g: dict, cam: dict, y, basis: int = PILLBOX, ka: int | None = None):
    """A^T y of ``project_plenoptic_posed``."""
    q, phi = quarter_turns(cam["phi_deg"])
    gq = dict(g, nx=g["nz"], nz=g["nx"]) if q % 2 else dict(g)
    Rg = rotated_grid(gq, phi)
    gr = dict(nx=Rg["nx"], ny=Rg["ny"], nz=Rg["nz"], pitch=(Rg["hx"], Rg["hy"], Rg["hz"]))
    xr = backproject_plenoptic(gr, _head_on_view(cam), y, basis, ka)
    return quarter_turn_adjoint(g, rotate_azimuth_adjoint(gq, xr, phi), q).reshape(-1)
