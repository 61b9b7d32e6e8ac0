"""GPU parity of the hexagonal three-focal-length plenoptic camera (light
summed over all lenslets) against the FP64 oracle, which sums over every
lenslet of the array by brute force.  Same bars as the other operators:
relative L2 <= 1e-5 for A x and A^T y, dot-product identity, exact
valid-ray counts; at the paper's full size (2048^2 detector, 53 x 61
lenslets, 100^3 at 1 mm) on sampled pixels and through the dot identity."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from dotbar import dot_bar
from paper_1812_03358_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def ltm():
    from paper_1812_03358_amd import ltm as L
    L.lib()
    return L


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32).reshape(-1)).cuda()


@pytest.mark.parametrize("rays,phis", [((2, 2), (0.0,)), ((2, 3), (0.0, 50.0)), ((1, 1), (25.0,))])
def test_hex_small_matches_oracle(orc, ltm, rays, phis):
    # 192 px of 5 um: a 7 x 8 hexagonal array, field of view ~14 mm
    g = W.grid((20, 22, 18), 0.7)
    cams = [W.hex_plenoptic_camera(192, None, rays, 29, phi_deg=p) for p in phis]
    x = W.flame(22, seed=4)[:18, :22, :20]
    M = sum(W.n_pixels(c) for c in cams)
    y = W.uniform_random(M, seed=6)
    plan = ltm.Plan(g, cams)
    Ax = plan.project(_dev(x)).cpu().numpy()
    Aty = plan.backproject(_dev(y)).cpu().numpy()
    ref_Ax = orc.project(g, cams, x.astype(np.float64).reshape(-1))
    ref_Aty = orc.backproject(g, cams, y.astype(np.float64))
    e1, e2 = rel_l2(Ax, ref_Ax), rel_l2(Aty, ref_Aty)
    x64, y64 = x.astype(np.float64).reshape(-1), y.astype(np.float64)
    dot = abs(Ax.astype(np.float64) @ y64 - x64 @ Aty.astype(np.float64)) / (
        np.linalg.norm(Ax) * np.linalg.norm(y64))
    print(f"hex rays={rays} phis={phis}: A {e1:.2e} A^T {e2:.2e} dot {dot:.2e}", flush=True)
    assert np.linalg.norm(ref_Ax) > 0
    assert e1 < TOL and e2 < TOL
    assert dot < dot_bar(x64, ref_Aty, y64, ref_Ax)
    for k, c in enumerate(cams):
        assert plan.valid_rays(k) == orc.count_valid_rays(g, c)


def test_hex_mixed_with_other_kinds(orc, ltm):
    g = W.grid(16, 0.8)
    cams = [W.hex_plenoptic_camera(160, None, (2, 2), 21, phi_deg=0.0),
            W.plenoptic_camera(96, 6, (2, 2), 21, phi_deg=90.0),
            W.single_lens_camera(48, (2, 2), 21, phi_deg=-40.0, distance=300.0)]
    x = W.flame(16, seed=8)
    y = W.uniform_random(sum(W.n_pixels(c) for c in cams), seed=9)
    plan = ltm.Plan(g, cams)
    Ax = plan.project(_dev(x)).cpu().numpy()
    Aty = plan.backproject(_dev(y)).cpu().numpy()
    e1 = rel_l2(Ax, orc.project(g, cams, x.astype(np.float64).reshape(-1)))
    e2 = rel_l2(Aty, orc.backproject(g, cams, y.astype(np.float64)))
    print(f"mixed kinds: A {e1:.2e} A^T {e2:.2e}", flush=True)
    assert e1 < TOL and e2 < TOL


def test_hex_subsets_match_oracle(orc, ltm):
    g = W.grid(16, 0.8)
    cams = [W.hex_plenoptic_camera(160, None, (2, 3), 17)]
    x = W.flame(16, seed=2)
    y = W.uniform_random(160 * 160, seed=3)
    plan = ltm.Plan(g, cams)
    for n in range(3):
        plan.set_ray_subset(3, n)
        Ax = plan.project(_dev(x)).cpu().numpy()
        Aty = plan.backproject(_dev(y)).cpu().numpy()
        assert rel_l2(Ax, orc.project(g, cams, x.astype(np.float64).reshape(-1), subsets=3,
                                      subset=n)) < TOL
        assert rel_l2(Aty, orc.backproject(g, cams, y.astype(np.float64), subsets=3,
                                           subset=n)) < TOL


def test_hex_paper_camera_full_size(orc, ltm):
    # the simulated plenoptic table at its size: 2048^2 px of 5 um, 53 x 61
    # lenslets, 100^3 at 1 mm, 2 x 2 angular samples, 200 samples per ray
    g = W.grid(100, 1.0)
    cam = W.hex_plenoptic_camera(2048, None, (2, 2), 200)
    x = W.flame(100, seed=5)
    plan = ltm.Plan(g, [cam])
    Ax = plan.project(_dev(x)).cpu().numpy()
    rng = np.random.default_rng(11)
    pix = np.unique(np.concatenate([rng.integers(0, 2048 * 2048, 300),
                                    np.array([0, 2047, 2048 * 2047, 2048 * 2048 - 1,
                                              1024 * 2048 + 1024])]))
    ref = orc.project_pixels(g, cam, x.astype(np.float64).reshape(-1), pix)
    e = rel_l2(Ax[pix], ref)
    print(f"hex 2048: sampled A {e:.2e}, lit fraction {np.mean(Ax > 0):.3f}", flush=True)
    assert np.count_nonzero(ref) > 100
    assert e < TOL
    y = W.uniform_random(2048 * 2048, seed=12)
    Aty = plan.backproject(_dev(y)).cpu().numpy()
    x64, y64 = x.astype(np.float64).reshape(-1), y.astype(np.float64)
    dot = abs(Ax.astype(np.float64) @ y64 - x64 @ Aty.astype(np.float64)) / (
        np.linalg.norm(Ax) * np.linalg.norm(y64))
    print(f"hex 2048: dot {dot:.2e}", flush=True)
    assert dot < 1e-9
