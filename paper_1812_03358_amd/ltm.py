"""ctypes binding of libltm.so (include/ltm.h).

Argument marshalling only: every step of the camera operator, its adjoint
and the solver runs in the library's HIP kernels.  torch supplies device
memory (tensors) and streams.  Loading fails loudly when the library has not
been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libltm.so")

LTM_OK = 0
LTM_ERR_INVALID = 1
LTM_ERR_DEVICE = 2
LTM_ERR_NUMERIC = 3
LTM_ERR_WORKSPACE = 4
LTM_ERR_UNSUPPORTED = 5
FORWARD, ADJOINT = 0, 1
PSI_QUADRATIC, PSI_HYPERBOLA = 0, 1


class LtmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ltm status {status}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("nz", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("pitch_mm", ctypes.c_double)]


ABI_VERSION = 4


class Camera(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("det_nu", ctypes.c_uint32), ("det_nv", ctypes.c_uint32),
                ("mla_nu", ctypes.c_uint32), ("mla_nv", ctypes.c_uint32),
                ("rays_u", ctypes.c_uint32), ("rays_v", ctypes.c_uint32),
                ("samples", ctypes.c_uint32),
                ("pixel_pitch_mm", ctypes.c_double),
                ("f_main_mm", ctypes.c_double), ("r_main_mm", ctypes.c_double),
                ("d_det_mm", ctypes.c_double),
                ("d_mla_mm", ctypes.c_double), ("d_mla_det_mm", ctypes.c_double),
                ("f_mla_mm", ctypes.c_double), ("r_mla_mm", ctypes.c_double),
                ("axes", ctypes.c_double * 9), ("lens_center_mm", ctypes.c_double * 3),
                ("f_hex_mm", ctypes.c_double * 3)]


class Tiling(ctypes.Structure):
    _fields_ = [("tile_u", ctypes.c_uint32), ("tile_v", ctypes.c_uint32),
                ("block_u", ctypes.c_uint32), ("block_v", ctypes.c_uint32),
                ("order", ctypes.c_uint32), ("splits", ctypes.c_uint32),
                ("brick_floats", ctypes.c_uint32), ("groups_per_cu", ctypes.c_uint32),
                ("chunk_mm", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolverParams(ctypes.Structure):
    _fields_ = [("momentum", ctypes.c_uint32), ("gains", ctypes.c_uint32),
                ("psi_kind", ctypes.c_uint32), ("n_subsets", ctypes.c_uint32),
                ("beta", ctypes.c_double), ("delta", ctypes.c_double),
                ("nu", ctypes.c_double), ("c_r", ctypes.c_double),
                ("rho_target", ctypes.c_double), ("max_iter", ctypes.c_uint32),
                ("check_every", ctypes.c_uint32)]


class ConvDesc(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in
                ("ksize", "d", "h", "w", "c0", "c1", "cout", "upsample", "relu", "out_f32", "split",
                 "reserved")]


_lib = None

# name -> (restype, argtypes)
_VP, _U32, _U64, _D = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
_SIGS = {
    "ltm_abi_version": (ctypes.c_uint32, []),
    "ltm_last_error": (ctypes.c_char_p, []),
    "ltm_plan_create": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Camera), _U32,
                                       ctypes.POINTER(_VP)]),
    "ltm_plan_destroy": (None, [_VP]),
    "ltm_plan_sizes": (ctypes.c_int, [_VP, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "ltm_plan_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(_U64)]),
    "ltm_plan_bind_workspace": (ctypes.c_int, [_VP, _VP, _U64, _VP]),
    "ltm_plan_get_tiling": (ctypes.c_int, [_VP, _U32, _U32, ctypes.POINTER(Tiling)]),
    "ltm_plan_set_tiling": (ctypes.c_int, [_VP, _U32, _U32, ctypes.POINTER(Tiling)]),
    "ltm_plan_valid_rays": (ctypes.c_int, [_VP, _U32, ctypes.POINTER(_U64), _VP]),
    "ltm_plan_set_ray_subset": (ctypes.c_int, [_VP, _U32, _U32]),
    "ltm_project": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ltm_backproject": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ltm_backproject_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ltm_autotune_candidates": (ctypes.c_int, [_VP, _U32, _U32, _VP, _U32, ctypes.POINTER(_U32)]),
    "ltm_autotune_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(_U64)]),
    "ltm_autotune": (ctypes.c_int, [_VP, _VP, _VP, _VP, _U64, ctypes.c_char_p, _U32,
                                    ctypes.POINTER(_D), _VP]),
    "ltm_solver_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(_U64)]),
    "ltm_solver_create": (ctypes.c_int, [_VP, ctypes.POINTER(SolverParams), _VP, _VP, _VP, _U64,
                                         _VP, ctypes.POINTER(_VP)]),
    "ltm_solver_destroy": (None, [_VP]),
    "ltm_solver_reset": (ctypes.c_int, [_VP, _VP, _VP]),
    "ltm_solver_step": (ctypes.c_int, [_VP, _U32, _VP]),
    "ltm_solver_reset_warm": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                             ctypes.POINTER(_U32), _VP]),
    "ltm_solver_solve": (ctypes.c_int, [_VP, ctypes.POINTER(_U32), ctypes.POINTER(_U32),
                                        ctypes.POINTER(_D), _VP]),
    "ltm_solver_get_x": (ctypes.c_int, [_VP, _VP, _VP]),
    "ltm_solver_residual": (ctypes.c_int, [_VP, ctypes.POINTER(_D), ctypes.POINTER(_U32), _VP]),
    "ltm_solver_residual_x": (ctypes.c_int, [_VP, ctypes.POINTER(_D), _VP]),
    "ltm_solver_save": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_U32),
                                       _VP, _VP]),
    "ltm_solver_load": (ctypes.c_int, [_VP, _VP, _VP, _D, _U32, _VP, _VP]),
    "ltm_batch_create": (ctypes.c_int, [ctypes.POINTER(_VP), _U32, ctypes.POINTER(_VP)]),
    "ltm_batch_destroy": (None, [_VP]),
    "ltm_batch_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(_U64)]),
    "ltm_batch_bind": (ctypes.c_int, [_VP, _VP, _U64, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                      ctypes.POINTER(_VP), _VP]),
    "ltm_batch_project": (ctypes.c_int, [_VP, _VP]),
    "ltm_batch_backproject": (ctypes.c_int, [_VP, _VP]),
    "ltm_batch_sweep": (ctypes.c_int, [_VP, _VP]),
    "ltm_batch_graph_capture": (ctypes.c_int, [_VP, _VP]),
    "ltm_batch_graph_launch": (ctypes.c_int, [_VP, _VP]),
    "ltm_reg_grad_add": (ctypes.c_int, [ctypes.POINTER(Grid), _U32, _D, _D, _VP, _VP, _VP]),
}


_NN_SIGS = {
    "ltm_nn_packed_sizes": (ctypes.c_int, [_U32, _U32, _U32, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "ltm_nn_pack_weights": (ctypes.c_int, [_VP, _U32, _U32, _U32, _VP, _VP, _VP]),
    "ltm_nn_conv3d_forward": (ctypes.c_int, [ctypes.POINTER(ConvDesc), _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "ltm_nn_conv3d_dgrad": (ctypes.c_int, [ctypes.POINTER(ConvDesc), _VP, _VP, _VP, _VP, _VP]),
    "ltm_nn_conv3d_wgrad": (ctypes.c_int, [ctypes.POINTER(ConvDesc), _VP, _VP, _VP, _VP, _VP]),
    "ltm_nn_maxpool2": (ctypes.c_int, [_VP, _VP, _VP, _U32, _U32, _U32, _U32, _VP]),
    "ltm_nn_maxpool2_backward": (ctypes.c_int, [_VP, _VP, _VP, _U32, _U32, _U32, _U32, _VP]),
    "ltm_nn_upsample2_backward": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, _U32, _U32, _VP]),
    "ltm_nn_relu_backward": (ctypes.c_int, [_VP, _VP, _U32, _VP, _VP, _U64, _U32, _VP]),
    "ltm_nn_mse": (ctypes.c_int, [_VP, _VP, _VP, _VP, _U64, _VP]),
    "ltm_nn_adam": (ctypes.c_int, [_VP, _VP, _VP, _VP, _U64, _D, _D, _D, _D, _U32, _VP]),
    "ltm_nn_prep_input": (ctypes.c_int, [_VP, _VP, _VP, _U64, _VP]),
    "ltm_nn_add": (ctypes.c_int, [_VP, _VP, _U64, _VP]),
}
_SIGS.update(_NN_SIGS)

_XPORT_SIGS = {
    "ltm_xport_create": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Camera), _U32,
                                        ctypes.POINTER(_VP)]),
    "ltm_xport_destroy": (None, [_VP]),
    "ltm_xport_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(_U64)]),
    "ltm_xport_bind_workspace": (ctypes.c_int, [_VP, _VP, _U64, _VP]),
    "ltm_xport_project": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ltm_xport_backproject": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ltm_xport_bands": (ctypes.c_int, [_VP, ctypes.POINTER(_U32)]),
}
_SIGS.update(_XPORT_SIGS)
BASIS_DIRAC, BASIS_PILLBOX = 0, 1


def lib():
    """The loaded library; raises if libltm.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1812_03358_amd.build` (no CPU fallback exists)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        if h.ltm_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {h.ltm_abi_version()}, the binding "
                               f"expects {ABI_VERSION}: rebuild it")
        _lib = h
    return _lib


def declared_symbols():
    return list(_SIGS)


def _check(status: int):
    if status != LTM_OK:
        msg = lib().ltm_last_error()
        raise LtmError(status, msg.decode() if msg else "")


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor | None, dtype=torch.float32, numel: int | None = None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def make_grid(g: dict) -> Grid:
    return Grid(g["nx"], g["ny"], g["nz"], 0, g["pitch"])


def make_cameras(cams) -> ctypes.Array:
    arr = (Camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = Camera(c["kind"], c["det_nu"], c["det_nv"], c["mla_nu"], c["mla_nv"],
                        c["rays_u"], c["rays_v"], c["samples"], c["pixel_pitch"],
                        c["f_main"], c["r_main"], c["d_det"], c["d_mla"], c["d_mla_det"],
                        c["f_mla"], c["r_mla"], (ctypes.c_double * 9)(*c["axes"]),
                        (ctypes.c_double * 3)(*c["lens_center"]),
                        (ctypes.c_double * 3)(*c.get("f_hex", (0.0, 0.0, 0.0))))
    return arr


class Plan:
    """A camera operator A for one grid and a list of cameras."""

    def __init__(self, grid: dict, cameras, device="cuda", bind: bool = True, stream=None):
        self.grid = dict(grid)
        self.cameras = list(cameras)
        self._g = make_grid(grid)
        self._c = make_cameras(self.cameras)
        h = ctypes.c_void_p()
        _check(lib().ltm_plan_create(ctypes.byref(self._g), self._c, len(self.cameras),
                                     ctypes.byref(h)))
        self._h = h
        nv, nm = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().ltm_plan_sizes(h, ctypes.byref(nv), ctypes.byref(nm)))
        self.n_voxels, self.n_meas = nv.value, nm.value
        self.device = torch.device(device)
        self.workspace = None
        if bind:
            self.bind(stream)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ltm_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64()
        _check(lib().ltm_plan_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def bind(self, stream=None):
        nb = self.workspace_bytes()
        if self.workspace is None or self.workspace.numel() < nb:
            self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        _check(lib().ltm_plan_bind_workspace(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                             self.workspace.numel(), _stream(stream)))

    def get_tiling(self, direction: int, camera: int = 0) -> Tiling:
        t = Tiling()
        _check(lib().ltm_plan_get_tiling(self._h, direction, camera, ctypes.byref(t)))
        return t

    def set_tiling(self, direction: int, camera: int, tiling, stream=None, rebind=True):
        if isinstance(tiling, dict):
            t = self.get_tiling(direction, camera)
            for k, v in tiling.items():
                setattr(t, k, v)
            tiling = t
        _check(lib().ltm_plan_set_tiling(self._h, direction, camera, ctypes.byref(tiling)))
        if rebind:
            self.bind(stream)

    def set_ray_subset(self, n_subsets: int = 1, index: int = 0):
        """Restrict project/backproject to angular-sample subset `index` of
        `n_subsets` (mean over the subset); (1, 0) restores the full operator."""
        _check(lib().ltm_plan_set_ray_subset(self._h, n_subsets, index))

    def valid_rays(self, camera: int = 0, stream=None) -> int:
        n = ctypes.c_uint64()
        _check(lib().ltm_plan_valid_rays(self._h, camera, ctypes.byref(n), _stream(stream)))
        return n.value

    def valid_samples(self, stream=None) -> int:
        return sum(self.valid_rays(k, stream) * c["samples"] for k, c in enumerate(self.cameras))

    def project(self, x: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if y is None:
            y = torch.empty(self.n_meas, dtype=torch.float32, device=x.device)
        _check(lib().ltm_project(self._h, _ptr(x, numel=self.n_voxels),
                                 _ptr(y, numel=self.n_meas), _stream(stream)))
        return y

    def backproject(self, y: torch.Tensor, x: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if x is None:
            x = torch.empty(self.n_voxels, dtype=torch.float32, device=y.device)
        _check(lib().ltm_backproject(self._h, _ptr(y, numel=self.n_meas),
                                     _ptr(x, numel=self.n_voxels), _stream(stream)))
        return x

    def backproject_noalloc(self, y: torch.Tensor, x: torch.Tensor, stream=None) -> torch.Tensor:
        """A^T y through ltm_backproject_noalloc (the library's fixed
        accumulator instead of the workspace's); x must be given."""
        _check(lib().ltm_backproject_noalloc(self._h, _ptr(y, numel=self.n_meas),
                                             _ptr(x, numel=self.n_voxels), _stream(stream)))
        return x


class Solver:
    """Penalized NNLS (FISTA) on the GPU; see ltm_solver_* in include/ltm.h."""

    def __init__(self, plan: Plan, y: torch.Tensor, w: torch.Tensor | None = None, *,
                 beta=0.0, delta=1.0, nu=0.0, c_r=36.0, psi_kind=PSI_QUADRATIC,
                 momentum=True, gains=False, subsets=1, rho_target=0.0, max_iter=100,
                 check_every=10, stream=None):
        self.plan = plan
        self.y = y
        self.w = w
        b = ctypes.c_uint64()
        _check(lib().ltm_solver_workspace_bytes(plan.handle, ctypes.byref(b)))
        self.workspace = torch.empty(b.value, dtype=torch.uint8, device=y.device)
        self.params = SolverParams(int(momentum), int(gains), int(psi_kind), int(subsets),
                                   float(beta), float(delta), float(nu), float(c_r),
                                   float(rho_target), int(max_iter), int(check_every))
        h = ctypes.c_void_p()
        _check(lib().ltm_solver_create(plan.handle, ctypes.byref(self.params),
                                       _ptr(y, numel=plan.n_meas),
                                       _ptr(w, numel=plan.n_meas) if w is not None else None,
                                       ctypes.c_void_p(self.workspace.data_ptr()), b.value,
                                       _stream(stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ltm_solver_destroy(h)
            self._h = None

    def reset(self, x0: torch.Tensor | None = None, stream=None):
        _check(lib().ltm_solver_reset(self._h, _ptr(x0, numel=self.plan.n_voxels)
                                      if x0 is not None else None, _stream(stream)))

    def reset_warm(self, x0: torch.Tensor, stream=None):
        """Restart from a candidate start judged by the plain solver (see
        ltm_solver_reset_warm): returns (accepted, alpha, rho(alpha x0))."""
        a, r, ok = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint32()
        _check(lib().ltm_solver_reset_warm(self._h, _ptr(x0, numel=self.plan.n_voxels),
                                           ctypes.byref(a), ctypes.byref(r), ctypes.byref(ok),
                                           _stream(stream)))
        return bool(ok.value), a.value, r.value

    def step(self, n_iter: int = 1, stream=None):
        _check(lib().ltm_solver_step(self._h, int(n_iter), _stream(stream)))

    def solve(self, stream=None):
        """Iterate until the stop rule (rho_target, max_iter, check_every):
        returns (iterations, converged, rho of x)."""
        it, conv, rho = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_double()
        _check(lib().ltm_solver_solve(self._h, ctypes.byref(it), ctypes.byref(conv),
                                      ctypes.byref(rho), _stream(stream)))
        return it.value, bool(conv.value), rho.value

    def x(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.plan.n_voxels, dtype=torch.float32, device=self.y.device)
        _check(lib().ltm_solver_get_x(self._h, _ptr(out, numel=self.plan.n_voxels), _stream(stream)))
        return out

    def residual(self, stream=None):
        rho, it = ctypes.c_double(), ctypes.c_uint32()
        _check(lib().ltm_solver_residual(self._h, ctypes.byref(rho), ctypes.byref(it),
                                         _stream(stream)))
        return rho.value, it.value

    def save(self, stream=None):
        """Checkpoint: (x, z, t, iterations, gains)."""
        n = self.plan.n_voxels
        x = torch.empty(n, dtype=torch.float32, device=self.y.device)
        z = torch.empty_like(x)
        t, it = ctypes.c_double(), ctypes.c_uint32()
        gains = (ctypes.c_double * len(self.plan.cameras))()
        _check(lib().ltm_solver_save(self._h, _ptr(x), _ptr(z), ctypes.byref(t), ctypes.byref(it),
                                     ctypes.cast(gains, ctypes.c_void_p), _stream(stream)))
        return x, z, t.value, it.value, list(gains)

    def load(self, state, stream=None):
        x, z, t, it, gains = state
        g = (ctypes.c_double * len(gains))(*gains)
        _check(lib().ltm_solver_load(self._h, _ptr(x, numel=self.plan.n_voxels),
                                     _ptr(z, numel=self.plan.n_voxels), float(t), int(it),
                                     ctypes.cast(g, ctypes.c_void_p), _stream(stream)))

    def residual_x(self, stream=None) -> float:
        rho = ctypes.c_double()
        _check(lib().ltm_solver_residual_x(self._h, ctypes.byref(rho), _stream(stream)))
        return rho.value


class Batch:
    """One persistent sweep over several plans (see ltm_batch_* in ltm.h).

    x_in, y, x_out: lists of GPU tensors, one per plan."""

    def __init__(self, plans, x_in, y, x_out, stream=None):
        self.plans = list(plans)
        self.buffers = (list(x_in), list(y), list(x_out))
        arr = (_VP * len(self.plans))(*[p.handle for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().ltm_batch_create(arr, len(self.plans), ctypes.byref(h)))
        self._h = h
        b = ctypes.c_uint64()
        _check(lib().ltm_batch_workspace_bytes(h, ctypes.byref(b)))
        self.workspace = torch.empty(b.value, dtype=torch.uint8, device=y[0].device)
        for p, a, bb, c in zip(self.plans, x_in, y, x_out):
            _ptr(a, numel=p.n_voxels), _ptr(bb, numel=p.n_meas), _ptr(c, numel=p.n_voxels)
        mk = lambda ts: (_VP * len(ts))(*[t.data_ptr() for t in ts])
        _check(lib().ltm_batch_bind(h, ctypes.c_void_p(self.workspace.data_ptr()), b.value,
                                    mk(x_in), mk(y), mk(x_out), _stream(stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ltm_batch_destroy(h)
            self._h = None

    def project(self, stream=None):
        _check(lib().ltm_batch_project(self._h, _stream(stream)))

    def backproject(self, stream=None):
        _check(lib().ltm_batch_backproject(self._h, _stream(stream)))

    def sweep(self, stream=None):
        _check(lib().ltm_batch_sweep(self._h, _stream(stream)))

    def capture(self, stream):
        _check(lib().ltm_batch_graph_capture(self._h, _stream(stream)))

    def replay(self, stream=None):
        _check(lib().ltm_batch_graph_launch(self._h, _stream(stream)))


def reg_grad_add(grid: dict, z: torch.Tensor, g: torch.Tensor, beta: float, psi_kind: int,
                 delta: float, stream=None):
    gg = make_grid(grid)
    n = grid["nx"] * grid["ny"] * grid["nz"]
    _check(lib().ltm_reg_grad_add(ctypes.byref(gg), psi_kind, beta, delta, _ptr(z, numel=n),
                                  _ptr(g, numel=n), _stream(stream)))
    return g


class Transport:
    """The paper's L2-projected light-field transport (Dirac or pillbox
    angular basis) for one single-lens camera at an azimuth pose, or the
    factorized model of one square-array plenoptic camera at an azimuth pose;
    see ltm_xport_* in include/ltm.h.  Tables and the filtering intermediate live in a device
    workspace owned by this object."""

    def __init__(self, grid: dict, camera: dict, basis: int = BASIS_PILLBOX, device="cuda"):
        self.grid = dict(grid)
        self.camera = dict(camera)
        gg, cc = make_grid(grid), make_cameras([camera])
        h = ctypes.c_void_p()
        _check(lib().ltm_xport_create(ctypes.byref(gg), cc, int(basis), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_uint64()
        _check(lib().ltm_xport_workspace_bytes(h, ctypes.byref(n)))
        self.workspace = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=device)
        _check(lib().ltm_xport_bind_workspace(h, ctypes.c_void_p(self.workspace.data_ptr()),
                                              self.workspace.numel(), _stream(None)))
        self.n_voxels = grid["nx"] * grid["ny"] * grid["nz"]
        self.n_meas = camera["det_nu"] * camera["det_nv"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ltm_xport_destroy(h)
            self._h = None

    def bands(self):
        b = (ctypes.c_uint32 * 4)()
        _check(lib().ltm_xport_bands(self._h, b))
        return list(b)

    def project(self, x: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if y is None:
            y = torch.empty(self.n_meas, dtype=torch.float32, device=x.device)
        _check(lib().ltm_xport_project(self._h, _ptr(x, numel=self.n_voxels),
                                       _ptr(y, numel=self.n_meas), _stream(stream)))
        return y

    def backproject(self, y: torch.Tensor, x: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if x is None:
            x = torch.empty(self.n_voxels, dtype=torch.float32, device=y.device)
        _check(lib().ltm_xport_backproject(self._h, _ptr(y, numel=self.n_meas),
                                           _ptr(x, numel=self.n_voxels), _stream(stream)))
        return x
