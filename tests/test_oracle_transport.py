"""Pins of the oracle's L2-projected light-field transport (the paper's
Dirac and pillbox transport tables, slice collapse, single-lens camera).

* each table entry equals the inner product it is defined by, integrated
  numerically: a 2-D midpoint rule over (s, u) for the pillbox basis, and
  the Dirac sifting over u followed by a midpoint rule over s for the Dirac
  basis, on random affine ray maps with decentred offsets;
* a uniform in-focus slice gives dz x K_in / K on every pixel inside its
  image, for both bases (normalization and magnification);
* A^T equals the explicit transpose of A;
* pillbox and Dirac converge to each other as the angular cells shrink;
* against the ray-driven oracle (independent code: rays, trilinear voxels,
  pixel centres) on a smooth volume: the same total light to 1e-4 and the
  same image to a few percent (the two discretize voxels and pixels
  differently);
* the optics composition: the in-focus slice has X^{pq}_su = 0 and
  magnification -D/z.
"""
import numpy as np
import pytest

from oracle import transport as X
from paper_1812_03358_amd import workloads as W


def _affine(rng):
    M = np.eye(3)
    M[0, 0], M[0, 1], M[0, 2] = rng.uniform(0.5, 1.5), rng.uniform(-3, 3), rng.uniform(-0.2, 0.2)
    M[1, 0], M[1, 1] = rng.uniform(-0.3, 0.3), rng.uniform(0.5, 1.5)
    return M


def _numeric_entry(basis, Xpq, X0q, sk, d0, si, dp, sj, dq, n=3000):
    s = sj - 0.5 * dq + (np.arange(n) + 0.5) * dq / n
    qss, qsu, qbar = X0q[0]
    pss, psu, pbar = Xpq[0]
    if basis == X.DIRAC:
        # sift: u where the ray lands on s_k, Jacobian d0 / |X0q_su|
        u = (sk - qbar - qss * s) / qsu
        sp = pss * s + psu * u + pbar
        inside = np.abs(sp - si) <= 0.5 * dp
        return inside.sum() * (dq / n) * d0 / abs(qsu)
    # pillbox: bound u by the angular cell, then a 2-D midpoint rule
    u0 = (sk - 0.5 * d0 - qbar - qss * s) / qsu
    u1 = (sk + 0.5 * d0 - qbar - qss * s) / qsu
    ulo, uhi = min(u0.min(), u1.min()), max(u0.max(), u1.max())
    uu = ulo + (np.arange(n) + 0.5) * (uhi - ulo) / n
    S, U = np.meshgrid(s, uu, indexing="ij")
    a = np.abs(qss * S + qsu * U + qbar - sk) <= 0.5 * d0
    b = np.abs(pss * S + psu * U + pbar - si) <= 0.5 * dp
    return (a & b).sum() * (dq / n) * ((uhi - ulo) / n)


@pytest.mark.parametrize("basis", [X.DIRAC, X.PILLBOX])
def test_table_entries_equal_their_inner_products(basis):
    rng = np.random.default_rng(7 + basis)
    checked = 0
    for trial in range(6):
        Xpq, X0q = _affine(rng), _affine(rng)
        sk, d0, dp, dq = rng.uniform(-1, 1), rng.uniform(0.2, 1.0), rng.uniform(0.2, 1.0), \
            rng.uniform(0.2, 1.0)
        sj = np.array([rng.uniform(-1, 1)])
        # destination pixels around the source pixel's image
        B = X.transport_factor(basis, Xpq, X0q, sk, d0, np.linspace(-4, 4, 41), dp, sj, dq)
        for i in np.flatnonzero(B[:, 0] > 0)[:4]:
            si = np.linspace(-4, 4, 41)[i]
            ref = _numeric_entry(basis, Xpq, X0q, sk, d0, si, dp, sj[0], dq)
            assert abs(B[i, 0] - ref) <= 3e-3 * max(B[:, 0].max(), 1e-12), (trial, i, B[i, 0], ref)
            checked += 1
        # and zeros where the inner product vanishes
        for i in np.flatnonzero(B[:, 0] == 0)[:2]:
            si = np.linspace(-4, 4, 41)[i]
            assert _numeric_entry(basis, Xpq, X0q, sk, d0, si, dp, sj[0], dq, n=800) <= \
                3e-3 * max(B[:, 0].max(), 1e-12)
    assert checked >= 10


def test_in_focus_maps():
    D, F = W.TL_D, W.TL_F
    z = F * D / (D - F)
    X0q, Xpq, X0p = X.single_lens_maps(z, D, F)
    assert abs(Xpq[0, 1]) < 1e-12 * z
    assert abs(Xpq[0, 0] + D / z) < 1e-12
    assert abs(X0q[0, 0] - 1.0) < 1e-12 and abs(X0q[0, 1] + z) < 1e-12 * z
    assert X0p[0, 1] == D and X0p[0, 0] == 1.0


@pytest.mark.parametrize("basis", [X.DIRAC, X.PILLBOX])
def test_uniform_in_focus_slice(basis):
    # one slice, exactly at the in-focus distance, far wider than the view
    cam = W.single_lens_camera(32, (6, 6), 8)
    g = W.grid((64, 64, 1), 0.5)
    x = np.full((1, 64, 64), 2.0)
    y = X.project(g, cam, x, basis)
    cells, _, _ = X.angular_cells(cam)
    expect = 0.5 * 2.0 * len(cells) / 36.0
    assert np.max(np.abs(y - expect)) <= 1e-12 * expect


def test_backprojection_is_the_transpose():
    g = W.grid((5, 4, 3), 1.0)
    cam = W.single_lens_camera(12, (3, 2), 4)
    for basis in (X.DIRAC, X.PILLBOX):
        N, M = 60, 144
        A = np.zeros((M, N))
        for j in range(N):
            e = np.zeros(N)
            e[j] = 1.0
            A[:, j] = X.project(g, cam, e, basis)
        assert np.count_nonzero(A) > 0.05 * A.size
        y = np.random.default_rng(2).uniform(-1, 1, M)
        ref = A.T @ y
        assert np.max(np.abs(X.backproject(g, cam, y, basis) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_pillbox_and_dirac_converge():
    g = W.grid(12, 2.0)
    x = W.blobs(12, seed=4, count=3)
    diffs = []
    for K in (2, 4, 8):
        cam = W.single_lens_camera(96, (K, K), 8)
        yd = X.project(g, cam, x, X.DIRAC)
        yp = X.project(g, cam, x, X.PILLBOX)
        diffs.append(np.linalg.norm(yp - yd) / np.linalg.norm(yd))
    assert diffs[0] > diffs[1] > diffs[2]
    assert diffs[2] < 0.5 * diffs[0]


@pytest.mark.parametrize("basis", [X.DIRAC, X.PILLBOX])
def test_agrees_with_ray_driven_oracle(orc, basis):
    g = W.grid(24, 1.0)
    cam = W.single_lens_camera(256, (4, 4), 96)
    x = W.blobs(24, seed=3, count=4)
    y1 = X.project(g, cam, x, basis)
    y0 = orc.project(g, [cam], x.astype(np.float64).reshape(-1))
    assert abs(y1.sum() / y0.sum() - 1.0) < 1e-4
    assert np.linalg.norm(y1 - y0) / np.linalg.norm(y0) < 0.08
