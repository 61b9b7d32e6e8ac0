"""The C ABI on the host: the library loads without a GPU, exports every
function include/ltm.h declares, and validates descriptors before any
launch (error codes and messages)."""
import ctypes
import os
import re

import pytest

from paper_1812_03358_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1812_03358_amd import ltm
    return ltm


def header_functions():
    text = open(os.path.join(ROOT, "include", "ltm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ltm_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported(L):
    lib = L.lib()
    names = header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows every one of them
    assert set(names) <= set(L.declared_symbols())


def test_abi_version(L):
    assert L.lib().ltm_abi_version() == L.ABI_VERSION == 4


def _create(L, g, cams):
    gg = L.make_grid(g)
    cc = L.make_cameras(cams)
    h = ctypes.c_void_p()
    st = L.lib().ltm_plan_create(ctypes.byref(gg), cc, len(cams), ctypes.byref(h))
    msg = L.lib().ltm_last_error().decode()
    if st == 0:
        L.lib().ltm_plan_destroy(h)
    return st, msg


def test_valid_plan_and_sizes(L):
    g = W.grid(128, 1.25)
    cams = [W.plenoptic_camera(), W.single_lens_camera(64, (2, 2), 9, phi_deg=30.0)]
    gg, cc, h = L.make_grid(g), L.make_cameras(cams), ctypes.c_void_p()
    assert L.lib().ltm_plan_create(ctypes.byref(gg), cc, 2, ctypes.byref(h)) == 0
    nv, nm = ctypes.c_uint64(), ctypes.c_uint64()
    assert L.lib().ltm_plan_sizes(h, ctypes.byref(nv), ctypes.byref(nm)) == 0
    assert nv.value == 128 ** 3 and nm.value == 1024 * 1024 + 64 * 64
    b = ctypes.c_uint64()
    assert L.lib().ltm_plan_workspace_bytes(h, ctypes.byref(b)) == 0
    assert b.value >= 8 * 128 ** 3                      # FP64 adjoint accumulator
    # unbound plan refuses to launch
    st = L.lib().ltm_project(h, ctypes.c_void_p(8), ctypes.c_void_p(8), None)
    assert st == L.LTM_ERR_WORKSPACE
    t = L.Tiling()
    assert L.lib().ltm_plan_get_tiling(h, 1, 0, ctypes.byref(t)) == 0
    t.order = 128                                        # flags are bits 0..6
    assert L.lib().ltm_plan_set_tiling(h, 1, 0, ctypes.byref(t)) == L.LTM_ERR_INVALID
    t.order = 1
    t.splits = 1
    t.tile_u = t.tile_v = 16                             # 65536 pixels in one workgroup
    assert L.lib().ltm_plan_set_tiling(h, 1, 0, ctypes.byref(t)) == L.LTM_ERR_INVALID
    L.lib().ltm_plan_destroy(h)


@pytest.mark.parametrize("mutate,needle", [
    (lambda g, c: g.update(nx=1), "at least 2"),
    (lambda g, c: g.update(pitch=0.0), "pitch"),
    (lambda g, c: c.update(det_nu=1001), "multiple"),
    (lambda g, c: c.update(samples=0), "samples"),
    (lambda g, c: c.update(rays_u=9, rays_v=9), "rays"),
    (lambda g, c: c.update(f_mla=-3.0), "positive"),
    (lambda g, c: c.update(axes=[1, 0, 0, 0, 1, 0, 0, 0, -1]), "right-handed"),
    (lambda g, c: c.update(axes=[1, 0, 0, 0, 2, 0, 0, 0, 1]), "orthonormal"),
    (lambda g, c: c.update(kind=7), "kind"),
    (lambda g, c: c.update(det_nu=0), "empty"),
])
def test_invalid_descriptors_rejected(L, mutate, needle):
    g = W.grid(16, 1.0)
    c = W.plenoptic_camera(64, 4, (2, 2), 8)
    mutate(g, c)
    st, msg = _create(L, g, [c])
    assert st == L.LTM_ERR_INVALID
    assert needle in msg


def test_solver_requires_bound_plan(L):
    g = W.grid(8, 1.0)
    gg, cc, h = L.make_grid(g), L.make_cameras([W.single_lens_camera(8, (1, 1), 4)]), ctypes.c_void_p()
    assert L.lib().ltm_plan_create(ctypes.byref(gg), cc, 1, ctypes.byref(h)) == 0
    prm = L.SolverParams(1, 0, 0, 0, 0.0, 1.0, 0.0, 36.0, 1e-3, 100, 10)
    out = ctypes.c_void_p()
    st = L.lib().ltm_solver_create(h, ctypes.byref(prm), ctypes.c_void_p(256), None,
                                   ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(out))
    assert st == L.LTM_ERR_WORKSPACE
    # parameters are validated before anything else
    prm.rho_target = -1.0
    st = L.lib().ltm_solver_create(h, ctypes.byref(prm), ctypes.c_void_p(256), None,
                                   ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(out))
    assert st == L.LTM_ERR_INVALID and "rho_target" in L.lib().ltm_last_error().decode()
    L.lib().ltm_plan_destroy(h)


def test_solver_entry_points_reject_null(L):
    u, d = ctypes.c_uint32(), ctypes.c_double()
    assert L.lib().ltm_solver_solve(None, ctypes.byref(u), ctypes.byref(u), ctypes.byref(d),
                                    None) == L.LTM_ERR_INVALID
    assert L.lib().ltm_solver_reset_warm(None, ctypes.c_void_p(256), None, None, None,
                                         None) == L.LTM_ERR_INVALID


def test_brick_index_range_is_checked(L):
    # brick indices are FP32 sums of a grid coordinate times a brick stride:
    # a 1100-voxel axis with 16384-float bricks would round them
    g = W.grid((1100, 8, 8), 1.0)
    gg, cc, h = L.make_grid(g), L.make_cameras([W.single_lens_camera(64, (1, 1), 8)]), ctypes.c_void_p()
    assert L.lib().ltm_plan_create(ctypes.byref(gg), cc, 1, ctypes.byref(h)) == 0
    t = L.Tiling()
    assert L.lib().ltm_plan_get_tiling(h, 1, 0, ctypes.byref(t)) == 0
    assert (1100 + 2) * t.brick_floats < (1 << 24)      # the default respects it
    t.brick_floats = 16384
    assert L.lib().ltm_plan_set_tiling(h, 1, 0, ctypes.byref(t)) == L.LTM_ERR_INVALID
    assert "2^24" in L.lib().ltm_last_error().decode()
    L.lib().ltm_plan_destroy(h)


def test_noalloc_backproject_rejects_before_any_device_call(L):
    # the fixed accumulator holds 2^23 doubles: 204^3 = 8489664 voxels is one
    # plan too many, refused before the plan's binding is even looked at
    cam = [W.single_lens_camera(64, (1, 1), 8)]
    big = W.grid(204, 1.0)
    gg, cc, h = L.make_grid(big), L.make_cameras(cam), ctypes.c_void_p()
    assert L.lib().ltm_plan_create(ctypes.byref(gg), cc, 1, ctypes.byref(h)) == 0
    st = L.lib().ltm_backproject_noalloc(h, ctypes.c_void_p(256), ctypes.c_void_p(256), None)
    assert st == L.LTM_ERR_INVALID
    assert "8388608" in L.lib().ltm_last_error().decode()
    assert L.lib().ltm_backproject_noalloc(h, None, ctypes.c_void_p(256), None) == L.LTM_ERR_INVALID
    L.lib().ltm_plan_destroy(h)
    # 203^3 = 8365427 fits; the unbound plan is then refused
    ok = W.grid(203, 1.0)
    gg = L.make_grid(ok)
    assert L.lib().ltm_plan_create(ctypes.byref(gg), cc, 1, ctypes.byref(h)) == 0
    st = L.lib().ltm_backproject_noalloc(h, ctypes.c_void_p(256), ctypes.c_void_p(256), None)
    assert st == L.LTM_ERR_WORKSPACE
    L.lib().ltm_plan_destroy(h)


def test_autotune_candidates_and_occupancy_field(L):
    from paper_1812_03358_amd import autotune
    cams = [W.plenoptic_camera(1024, 64, (2, 2), 256), W.single_lens_camera(64, (8, 8), 64)]
    plan = L.Plan(W.grid(128, 1.25), cams, bind=False)
    for ci in range(2):
        for d in (0, 1):
            cands = autotune.candidates(plan, ci, d)
            assert len(cands) >= 8
            assert len({tuple(sorted(c.items())) for c in cands}) == len(cands)
            for c in cands:
                assert c["groups_per_cu"] == 0
                plan.set_tiling(d, ci, c, rebind=False)     # each one passes the checks
    # the occupancy cap: 0 or 2..8
    for cap, ok in ((0, True), (1, False), (2, True), (8, True), (9, False)):
        t = plan.get_tiling(1, 0)
        t.groups_per_cu = cap
        st = L.lib().ltm_plan_set_tiling(plan.handle, 1, 0, ctypes.byref(t))
        assert (st == 0) == ok, cap
    nb = ctypes.c_uint64()
    assert L.lib().ltm_autotune_workspace_bytes(plan.handle, ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 4 * 128 ** 3 + 8 * 128 ** 3      # two volumes and an accumulator
    ms = (ctypes.c_double * 8)()
    assert L.lib().ltm_autotune(plan.handle, None, ctypes.c_void_p(256), ctypes.c_void_p(256),
                                nb.value, None, 2, ms, None) == L.LTM_ERR_INVALID
    assert L.lib().ltm_autotune(plan.handle, ctypes.c_void_p(256), ctypes.c_void_p(256),
                                ctypes.c_void_p(256), nb.value, None, 0, ms, None) == L.LTM_ERR_INVALID
    assert L.lib().ltm_autotune(plan.handle, ctypes.c_void_p(256), ctypes.c_void_p(256),
                                ctypes.c_void_p(8), nb.value, None, 2, ms, None) == L.LTM_ERR_WORKSPACE


def test_tuned_table_parses():
    from paper_1812_03358_amd import autotune
    if not os.path.exists(autotune.TUNED_TABLE):
        pytest.skip("no tuned table committed")
    from paper_1812_03358_amd.tuned import make_table as M
    capped = {M.table_key("gfx950", f["grid"], c, d) for f in W.config_batched() for c in f["cameras"]
              for d in (0, 1)}
    rows = [l.rstrip("\n").split("\t") for l in open(autotune.TUNED_TABLE) if not l.startswith("#")]
    assert rows
    for key, tiling, times in rows:
        assert key.startswith("gfx950|")
        f = tiling.split()
        assert len(f) == 9 and all(v.isdigit() for v in f[:8]) and float(f[8]) > 0
        best, default = map(float, times.split())
        # a batch-capped entry may be slower alone than the default, but not
        # by much (slabs too deep for the capped brick would fall back to
        # global memory and run many times slower)
        assert 0 < best and (best <= default or (key in capped and best <= 1.25 * default))


def test_tuned_table_covers_the_batched_workload():
    """Every camera of the 48-frame workload has a table entry in both
    directions, and both keep the batch cap (bricks of at most 6144 floats,
    no occupancy padding), so the persistent sweeps run 5 workgroups per
    CU."""
    from paper_1812_03358_amd import autotune
    from paper_1812_03358_amd.tuned import make_table as M
    table = M.read_table(autotune.TUNED_TABLE)
    for f in W.config_batched():
        for c in f["cameras"]:
            for d in (0, 1):     # forward, adjoint
                t = table[M.table_key("gfx950", f["grid"], c, d)]
                assert t["brick_floats"] <= M.BATCH_BRICK_CAP and t["groups_per_cu"] == 0


def test_table_key_matches_the_library_hash():
    """The FNV-1a step against the published 64-bit test vectors (standard
    offset basis; the library seeds it with its own constant, which the
    table-coverage test checks through the library-written keys), and the
    key's readable fields."""
    from paper_1812_03358_amd.tuned import make_table as M
    assert M._fnv1a(b"a", 0xcbf29ce484222325) == 0xaf63dc4c8601ec8c
    assert M._fnv1a(b"foobar", 0xcbf29ce484222325) == 0x85944171f73967e8
    g = W.grid(96, 160.0 / 96)
    k = M.table_key("gfx950", g, W.plenoptic_camera(1024, 64, (2, 2), 192, 30.0), 1)
    assert k.startswith("gfx950|AT|kind1|grid96x96x96|det1024x1024|mla64x64|R2x2|S192|")


def test_binding_fails_loudly_without_library(L, monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        L.lib()


def test_hexagonal_camera_validation(L):
    import math
    g = W.grid(100, 1.0)
    ok = W.hex_plenoptic_camera()                        # the paper's 2048^2 camera
    assert _create(L, g, [ok])[0] == 0
    st, msg = _create(L, g, [W.hex_plenoptic_camera(rays=(3, 3))])
    assert st == L.LTM_ERR_INVALID and "<= 7" in msg
    bad = W.hex_plenoptic_camera()
    bad["f_hex"] = [2.8, -3.0, 3.2]
    st, msg = _create(L, g, [bad])
    assert st == L.LTM_ERR_INVALID and "focal" in msg
    # the reach rule: accepted exactly while the bound stays below 1.5 row spacings
    limit = 1.5 * math.sqrt(3) * W.PL_RMU

    def reach(c):
        e = c["d_mla_det"] / c["d_mla"]
        k = max(abs(1 + c["d_mla"] / c["d_mla_det"] - c["d_mla"] / f) for f in c["f_hex"])
        hd = 0.5 * c["pixel_pitch"] * math.hypot(c["det_nu"] - 1, c["det_nv"] - 1)
        return (e * hd + e * (c["r_main"] + k * c["r_mla"])) / (1 + e)

    for det in (1024, 2048, 2064, 2200, 3000):
        c = W.hex_plenoptic_camera(det)
        st, msg = _create(L, g, [c])
        assert (st == 0) == (reach(c) < limit), (det, msg)
        if st:
            assert "3 x 3" in msg
    assert reach(W.hex_plenoptic_camera(2048)) < limit < reach(W.hex_plenoptic_camera(3000))


def test_transport_operator_validation(L):
    g = W.grid(24, 1.0)
    ok = W.single_lens_camera(128, (4, 4), 8)
    h = ctypes.c_void_p()
    for basis in (0, 1):
        assert L.lib().ltm_xport_create(ctypes.byref(L.make_grid(g)), L.make_cameras([ok]), basis,
                                        ctypes.byref(h)) == 0
        b = (ctypes.c_uint32 * 4)()
        assert L.lib().ltm_xport_bands(h, b) == 0
        assert all(1 <= v <= 64 for v in b)
        n = ctypes.c_uint64()
        assert L.lib().ltm_xport_workspace_bytes(h, ctypes.byref(n)) == 0
        assert n.value >= 4 * 24 * 4 * 128 * 24                     # the filtering intermediate
        # unbound: refuses to launch
        assert L.lib().ltm_xport_project(h, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == \
            L.LTM_ERR_WORKSPACE
        L.lib().ltm_xport_destroy(h)
    def ws_of(cam, grid=g):
        assert L.lib().ltm_xport_create(ctypes.byref(L.make_grid(grid)), L.make_cameras([cam]), 1,
                                        ctypes.byref(h)) == 0, L.lib().ltm_last_error()
        n = ctypes.c_uint64()
        assert L.lib().ltm_xport_workspace_bytes(h, ctypes.byref(n)) == 0
        L.lib().ltm_xport_destroy(h)
        return n.value

    # posed: quarter turns, then the shear rotation of the rest
    ws0 = ws_of(W.single_lens_camera(128, (4, 4), 8))
    for phi in (20.0, -45.0, 50.0, 135.0, 180.0, -100.0):
        assert ws_of(W.single_lens_camera(128, (4, 4), 8, phi_deg=phi)) > ws0
    # a quarter turn alone adds one turned volume (24^3 floats, 256-byte aligned)
    assert ws_of(W.single_lens_camera(128, (4, 4), 8, phi_deg=90.0)) == ws0 + 4 * 24 ** 3
    # head-on square-array plenoptic: the factorized model, three intermediates
    pl = W.plenoptic_camera(64, 4, (3, 3), 8)
    assert L.lib().ltm_xport_create(ctypes.byref(L.make_grid(g)), L.make_cameras([pl]), 1,
                                    ctypes.byref(h)) == 0
    n = ctypes.c_uint64()
    assert L.lib().ltm_xport_workspace_bytes(h, ctypes.byref(n)) == 0
    cells = 9                                            # 3 x 3 cells, all centres inside the disc
    assert n.value >= 4 * (24 * 3 * 64 * 24 + 2 * cells * 64 * 64)
    b = (ctypes.c_uint32 * 4)()
    assert L.lib().ltm_xport_bands(h, b) == 0 and all(v >= 1 for v in b)
    L.lib().ltm_xport_destroy(h)
    # posed plenoptic: the rotated grid's volumes join the workspace
    for phi in (20.0, -45.0, 100.0, -170.0):
        pp = W.plenoptic_camera(64, 4, (3, 3), 8, phi_deg=phi)
        assert L.lib().ltm_xport_create(ctypes.byref(L.make_grid(g)), L.make_cameras([pp]), 1,
                                        ctypes.byref(h)) == 0
        m = ctypes.c_uint64()
        assert L.lib().ltm_xport_workspace_bytes(h, ctypes.byref(m)) == 0 and m.value > n.value
        L.lib().ltm_xport_destroy(h)
    import math
    a = math.radians(10.0)                               # a roll about the optical axis
    rolled = dict(ok, axes=[math.cos(a), math.sin(a), 0, -math.sin(a), math.cos(a), 0, 0, 0, 1])
    cases = [(rolled, L.LTM_ERR_UNSUPPORTED, "azimuth pose"),
             (W.hex_plenoptic_camera(64, (4, 4)), L.LTM_ERR_UNSUPPORTED, "square-array"),
             (dict(W.plenoptic_camera(64, 4, (2, 2), 8), det_nv=32), L.LTM_ERR_UNSUPPORTED,
              "square lenslets"),
             (W.single_lens_camera(128, (4, 4), 8, distance=10.0), L.LTM_ERR_INVALID, "in front")]
    for cam, status, needle in cases:
        st = L.lib().ltm_xport_create(ctypes.byref(L.make_grid(g)), L.make_cameras([cam]), 1,
                                      ctypes.byref(h))
        assert st == status and needle in L.lib().ltm_last_error().decode()
    assert L.lib().ltm_xport_create(ctypes.byref(L.make_grid(g)), L.make_cameras([ok]), 2,
                                    ctypes.byref(h)) == L.LTM_ERR_INVALID
