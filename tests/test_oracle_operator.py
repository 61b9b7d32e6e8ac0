"""Pins of the oracle's A and A^T as linear maps.

* A^T is the exact transpose of A: the explicit matrix built column by column
  from A e_j, transposed, equals the oracle's A^T on tiny grids (both camera
  kinds, non-cubic grids), and the dot-product identity holds to 1e-13;
* A is linear and maps nonnegative volumes to nonnegative images;
* the pixel-subset entry point agrees with the full projection;
* several cameras stack their images in order.
"""
import numpy as np
import pytest

from paper_1812_03358_amd import workloads as W


def _cams_small():
    return [W.single_lens_camera(4, (2, 2), 6, phi_deg=10.0),
            W.plenoptic_camera(8, 2, (2, 1), 5, phi_deg=35.0)]


@pytest.mark.parametrize("dims", [(4, 4, 4), (5, 6, 7)])
def test_explicit_matrix_transpose_equals_backprojection(orc, dims):
    g_tl = W.grid(dims, 0.25)
    g_pl = W.grid(dims, 12.0)
    for g, cam in [(g_tl, _cams_small()[0]), (g_pl, _cams_small()[1])]:
        N = dims[0] * dims[1] * dims[2]
        M = cam["det_nu"] * cam["det_nv"]
        A = np.zeros((M, N))
        for j in range(N):
            e = np.zeros(N)
            e[j] = 1.0
            A[:, j] = orc.project(g, [cam], e)
        assert np.count_nonzero(A) > 0.05 * A.size
        assert A.min() >= 0.0
        rng = np.random.default_rng(3)
        for _ in range(3):
            y = rng.uniform(-1, 1, M)
            xt = orc.backproject(g, [cam], y)
            assert np.max(np.abs(xt - A.T @ y)) <= 1e-14 * np.max(np.abs(A.T @ y)) * 10
        x = rng.uniform(0, 1, N)
        assert np.max(np.abs(orc.project(g, [cam], x) - A @ x)) <= 1e-13 * np.max(A @ x)


@pytest.mark.parametrize("nthreads", [1, 3])
def test_dot_product_identity(orc, nthreads):
    g = W.grid((10, 11, 12), 5.0)
    cams = [W.plenoptic_camera(32, 4, (2, 2), 21, phi_deg=p) for p in (0.0, 30.0, 90.0)]
    cams.append(W.single_lens_camera(16, (1, 1), 40, phi_deg=45.0,
                                     distance=W.TL_F * W.TL_D / (W.TL_D - W.TL_F) * 30))
    x = W.uniform_random(10 * 11 * 12, seed=7).astype(np.float64)
    y = W.uniform_random(sum(c["det_nu"] ** 2 for c in cams), seed=8).astype(np.float64)
    Ax = orc.project(g, cams, x, threads=nthreads)
    Aty = orc.backproject(g, cams, y, threads=nthreads)
    err = abs(np.dot(Ax, y) - np.dot(x, Aty)) / (np.linalg.norm(Ax) * np.linalg.norm(y))
    assert err < 1e-13
    assert np.linalg.norm(Ax) > 0


def test_linearity_and_positivity(orc):
    g = W.grid(12, 6.0)
    cams = [W.plenoptic_camera(32, 2, (2, 2), 30, phi_deg=20.0)]
    a = W.uniform_random(12 ** 3, seed=1).astype(np.float64)
    b = W.uniform_random(12 ** 3, seed=2, lo=-1, hi=1).astype(np.float64)
    ya, yb = orc.project(g, cams, a), orc.project(g, cams, b)
    y = orc.project(g, cams, 2.5 * a - 0.75 * b)
    assert np.max(np.abs(y - (2.5 * ya - 0.75 * yb))) <= 1e-13 * np.max(np.abs(y))
    assert ya.min() >= 0.0 and ya.max() > 0.0


def test_pixel_subset_matches_full_projection(orc):
    g = W.grid(16, 10.0)
    cam = W.plenoptic_camera(64, 4, (2, 2), 32, phi_deg=30.0)
    x = W.flame(16, seed=5).astype(np.float64)
    y = orc.project(g, [cam], x.reshape(-1))
    pix = np.array([0, 5, 64 * 31 + 17, 64 * 64 - 1, 1000])
    assert np.array_equal(orc.project_pixels(g, cam, x.reshape(-1), pix), y[pix])


def test_cameras_stack_in_order(orc):
    g = W.grid(8, 10.0)
    c1 = W.plenoptic_camera(16, 2, (1, 1), 9, phi_deg=0.0)
    c2 = W.plenoptic_camera(32, 2, (2, 2), 9, phi_deg=50.0)
    x = W.uniform_random(512, seed=3).astype(np.float64)
    y = orc.project(g, [c1, c2], x)
    assert np.array_equal(y[:256], orc.project(g, [c1], x))
    assert np.array_equal(y[256:], orc.project(g, [c2], x))
    yy = W.uniform_random(256 + 1024, seed=4).astype(np.float64)
    xb = orc.backproject(g, [c1, c2], yy, threads=1)
    xs = orc.backproject(g, [c1], yy[:256], threads=1) + orc.backproject(g, [c2], yy[256:], threads=1)
    assert np.max(np.abs(xb - xs)) <= 1e-14 * np.max(np.abs(xb))


def test_flame_volume_statistics():
    v = W.flame(32, seed=2)
    assert v.dtype == np.float32 and v.shape == (32, 32, 32)
    assert v.min() >= 0.0 and 0.3 < v.max() < 2.0
    # plumes stacked along y: the mass centre sits near the lateral centre
    q = np.arange(32)
    cx = (v.sum(axis=(0, 1)) * q).sum() / v.sum()
    cz = (v.sum(axis=(1, 2)) * q).sum() / v.sum()
    assert abs(cx - 15.5) < 3 and abs(cz - 15.5) < 3
    assert np.array_equal(v, W.flame(32, seed=2))           # seeded
    assert not np.array_equal(v, W.flame(32, seed=3))


@pytest.mark.parametrize("nsub", [2, 3, 4])
def test_view_subsets_partition_the_operator(orc, nsub):
    # the paper's view subsets: every nsub-th angular sample; the subset
    # operator is the mean over its samples, so sum_n |S_n|/K A_Sn = A
    g = W.grid((9, 10, 11), 12.0)
    cam = W.plenoptic_camera(32, 2, (2, 2), 19, phi_deg=25.0)
    x = W.uniform_random(9 * 10 * 11, seed=12).astype(np.float64)
    y = W.uniform_random(32 * 32, seed=13).astype(np.float64)
    R = 4
    sizes = [len([r for r in range(R) if r % nsub == n]) for n in range(nsub)]
    full = orc.project(g, [cam], x)
    acc = sum(sizes[n] / R * orc.project(g, [cam], x, subsets=nsub, subset=n) for n in range(nsub))
    assert np.max(np.abs(acc - full)) <= 1e-13 * np.max(full)
    accb = sum(sizes[n] / R * orc.backproject(g, [cam], y, subsets=nsub, subset=n) for n in range(nsub))
    assert np.max(np.abs(accb - orc.backproject(g, [cam], y))) <= 1e-12 * np.max(np.abs(accb))
    for n in range(nsub):
        Ax = orc.project(g, [cam], x, subsets=nsub, subset=n)
        Aty = orc.backproject(g, [cam], y, subsets=nsub, subset=n)
        assert abs(np.dot(Ax, y) - np.dot(x, Aty)) <= 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_view_subset_solver_decreases_residual(orc):
    g = W.grid(8, 20.0)
    cams = [W.plenoptic_camera(32, 2, (2, 2), 17, phi_deg=p) for p in (0.0, 90.0)]
    xt = W.flame(8, seed=4).astype(np.float64)
    y = orc.project(g, cams, xt.reshape(-1))
    s = orc.Solver(g, cams, [y[:1024], y[1024:]], subsets=2, momentum=False)
    r0 = s.residual(s.x)
    s.run(10)
    assert s.residual(s.x) < 0.5 * r0
