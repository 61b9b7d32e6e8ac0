"""The workload constants against the paper's camera tables (golden fixture
tests/golden/camera_tables.json), and the documented departures from them."""
import json
import os

import numpy as np

from paper_1812_03358_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "camera_tables.json")))


def test_single_lens_constants_match_table():
    t = GOLD["single_lens"]
    c = W.single_lens_camera()
    assert c["f_main"] == t["lens_focal_length"]
    assert c["r_main"] == t["lens_radius"]
    assert c["d_det"] == t["lens_to_detector_distance"]
    assert c["pixel_pitch"] == t["detector_pixel_pitch"]


def test_plenoptic_constants_match_table():
    t = GOLD["plenoptic"]
    c = W.plenoptic_camera()
    assert c["f_main"] == t["main_lens_focal_length"]
    assert c["r_main"] == t["main_lens_radius"]
    assert c["d_mla"] == t["lens_to_mla_distance"]
    assert c["d_mla_det"] == t["mla_to_detector_distance"]
    assert c["r_mla"] == t["microlens_radius"]
    # square grid, one focal length: the middle of the three the table lists
    assert c["f_mla"] == sorted(t["microlens_focal_lengths"])[1]
    # 16 pixels span one 0.2 mm lenslet (two lenslet radii)
    assert abs(16 * c["pixel_pitch"] - 2 * t["microlens_radius"]) < 1e-15


def test_cameras_are_placed_in_focus_on_the_volume_centre():
    c = W.plenoptic_camera()
    d = np.linalg.norm(c["lens_center"])
    assert abs(1 / d + 1 / c["d_mla"] - 1 / c["f_main"]) < 1e-15
    t = W.single_lens_camera()
    d = np.linalg.norm(t["lens_center"])
    assert abs(1 / d + 1 / t["d_det"] - 1 / t["f_main"]) < 1e-15


def test_poses_are_rotations():
    for phi in (0.0, 30.0, 60.0, 90.0, 217.0):
        a = np.array(W.azimuth_axes(phi)).reshape(3, 3)
        assert np.allclose(a @ a.T, np.eye(3), atol=1e-15)
        assert abs(np.linalg.det(a) - 1.0) < 1e-15


def test_batched_workload_mix():
    frames = W.config_batched()
    sizes = sorted(f["grid"]["nx"] for f in frames)
    assert sizes == sorted([96] * 12 + [128] * 12 + [160] * 12 + [192] * 12)
    for f in frames:
        n = f["grid"]["nx"]
        assert abs(n * f["grid"]["pitch"] - 160.0) < 1e-9
        assert [c["phi_deg"] for c in f["cameras"]] == [0.0, 30.0, 60.0, 90.0]
        assert all(c["samples"] == 2 * n for c in f["cameras"])


def test_noise_recipes():
    y = np.linspace(0, 2, 1000).astype(np.float32)
    yg = W.gaussian_noise(y, seed=11)
    sigma = 0.01 * np.linalg.norm(y) / np.sqrt(y.size)
    assert abs(np.std(yg - y) / sigma - 1) < 0.1
    yp = W.poisson_noise(y, seed=12)
    assert yp.dtype == np.float32 and yp.min() >= 0
    # counts are integers after scaling by peak / max
    counts = yp.astype(np.float64) * 1000 / 2.0
    assert np.allclose(counts, np.round(counts), atol=1e-3)


def test_weight_masks():
    m = W.bayer_green_mask(6, 4).reshape(4, 6)
    assert m.sum() == 12 and m[0, 1] == 1 and m[0, 0] == 0 and m[1, 0] == 1
    d = W.damaged_mask(100, 50).reshape(50, 100)
    assert (d == 0).sum() == 20 * 10 and d[5:15, 60:80].max() == 0 and d[0, 0] == 1


def test_three_camera_config():
    cfg = W.config_three_camera()
    kinds = [c["kind"] for c in cfg["cameras"]]
    assert kinds == [W.PLENOPTIC, W.SINGLE_LENS, W.SINGLE_LENS]
    assert [c["phi_deg"] for c in cfg["cameras"]] == [0.0, 30.0, -30.0]
    assert cfg["gains"][0] == 1.0
