"""ltm_backproject_noalloc (the library's fixed FP64 accumulator in place of
the plan workspace's) against ltm_backproject and the FP64 oracle.

Two calls in a row through the C ABI, the second on a smaller volume, so a
stale accumulator left by the first call would show in the second.  The two
entry points run the same kernels; only the order of the FP64 atomic sums
differs, so they agree to FP32 output rounding, and each meets the oracle
bar of the parity tests (relative L2 <= 1e-5)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1812_03358_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = [
    # (grid dims, pitch, camera) -- the second is smaller than the first
    ((48, 40, 36), 4.0, lambda: W.plenoptic_camera(128, 8, (2, 2), 61, phi_deg=20.0)),
    ((20, 24, 18), 6.0, lambda: W.single_lens_camera(72, (2, 3), 29, phi_deg=-35.0)),
]


def test_noalloc_backproject_matches_workspace_entry_point(orc):
    from paper_1812_03358_amd import ltm

    stream = torch.cuda.current_stream()
    results = []
    for k, (dims, pitch, mk) in enumerate(CASES):
        g = W.grid(dims, pitch)
        cams = [mk()]
        print(f"noalloc case {k}: grid {dims}, camera kind {cams[0]['kind']}", flush=True)
        plan = ltm.Plan(g, cams)
        y = torch.from_numpy(W.uniform_random(plan.n_meas, seed=40 + k)).cuda()
        x_ref = plan.backproject(y)
        x_new = torch.full_like(x_ref, float("nan"))
        # called through the C ABI directly
        st = ltm.lib().ltm_backproject_noalloc(plan.handle, ctypes.c_void_p(y.data_ptr()),
                                               ctypes.c_void_p(x_new.data_ptr()),
                                               ctypes.c_void_p(stream.cuda_stream))
        assert st == ltm.LTM_OK, ltm.lib().ltm_last_error()
        torch.cuda.synchronize()
        a = x_new.cpu().numpy()
        b = x_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        e_pair = rel_l2(a, b)
        ref = orc.backproject(g, cams, y.cpu().numpy().astype(np.float64))
        e_new, e_old = rel_l2(a, ref), rel_l2(b, ref)
        print(f"  rel-L2 noalloc vs workspace {e_pair:.2e}, vs oracle {e_new:.2e} "
              f"(workspace entry point {e_old:.2e})", flush=True)
        assert e_pair <= 1e-7
        assert e_new <= 1e-5 and e_old <= 1e-5
        results.append(a)
    assert results[1].size < results[0].size


def test_noalloc_rejects_oversized_plan():
    from paper_1812_03358_amd import ltm

    g = W.grid(204, 1.0)
    plan = ltm.Plan(g, [W.single_lens_camera(32, (1, 1), 8)], bind=False)
    y = torch.zeros(plan.n_meas, device="cuda")
    x = torch.zeros(plan.n_voxels, device="cuda")
    with pytest.raises(ltm.LtmError) as e:
        plan.backproject_noalloc(y, x)
    assert e.value.status == ltm.LTM_ERR_INVALID
