"""ctypes binding of libelbm.so (include/elbm.h) -- argument marshalling only.

Every step of the method runs in the HIP library.  PyTorch supplies device memory
(the bound workspace and output tensors) and the HIP stream; it is imported before
the library is loaded so that both use the same HIP runtime.  There is no fallback:
if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libelbm.so")
# launch configurations measured for the benchmark workloads (elbm_tune cache format)
LAUNCH_CACHE = os.path.join(HERE, "launch_cache.txt")

STORE_F64, STORE_F32, STORE_F16S, STORE_BF16S = 0, 1, 2, 3
STORAGE = {"f64": STORE_F64, "f32": STORE_F32, "f16s": STORE_F16S, "bf16s": STORE_BF16S}
FACE_WALL, FACE_INLET, FACE_OUTFLOW = 1, 2, 3

STATUS = {0: "ELBM_OK", 1: "ELBM_EINVAL", 2: "ELBM_ESTATE", 3: "ELBM_ESMALL", 4: "ELBM_EDEVICE",
          5: "ELBM_EUNSTABLE", 6: "ELBM_ENOMEM"}

EXPORTS = [
    "elbm_create", "elbm_destroy", "elbm_status_string", "elbm_last_error", "elbm_set_face", "elbm_add_block",
    "elbm_set_solid", "elbm_set_force_uniform", "elbm_finalize", "elbm_level_box", "elbm_level_info",
    "elbm_node_class", "elbm_weights", "elbm_bind", "elbm_init_fields", "elbm_init_fields_static", "elbm_set_force_field", "elbm_advance",
    "elbm_read_moments", "elbm_read_populations", "elbm_sample_populations", "elbm_reduce", "elbm_check",
    "elbm_drag", "elbm_set_gamma_output", "elbm_brick_dims", "elbm_gamma_indicator", "elbm_transfer_state", "elbm_set_launch", "elbm_tune", "elbm_profile", "elbm_synchronize", "elbm_stream_copy",
    "elbm_state_bytes", "elbm_save_state", "elbm_load_state", "elbm_get_launch",
    "elbm_adjoint_bytes", "elbm_adjoint_bind", "elbm_adjoint_forward", "elbm_adjoint_backward",
    "elbm_adjoint_read", "elbm_adjoint_velocity", "elbm_adjoint_timing",
]

OBJECTIVES = {"drag": 0, "ke": 1}


class ElbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("storage", ctypes.c_int32), ("extent", ctypes.c_int64 * 3),
                ("periodic", ctypes.c_int32 * 3), ("nu0", ctypes.c_double), ("n_levels", ctypes.c_int32)]


_lib = None


def lib():
    """Load libelbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libelbm.so not built: run python -m paper_1608_06915_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        i32, i64 = ctypes.c_int, ctypes.c_int64
        sig = {
            "elbm_create": [ctypes.POINTER(_Desc), ctypes.POINTER(P)],
            "elbm_destroy": [P],
            "elbm_set_face": [P, i32, i32, dp],
            "elbm_add_block": [P, i32, i64p, i64p],
            "elbm_set_solid": [P, i32, i64p, i64p, P],
            "elbm_set_force_uniform": [P, dp],
            "elbm_finalize": [P, ctypes.POINTER(ctypes.c_size_t)],
            "elbm_level_box": [P, i32, i64p, i64p],
            "elbm_level_info": [P, i32, i64p, i64p, dp, i64p],
            "elbm_node_class": [P, i32, P],
            "elbm_weights": [P, i32, dp],
            "elbm_bind": [P, P, ctypes.c_size_t, P],
            "elbm_init_fields": [P, i32, dp, dp, dp],
            "elbm_init_fields_static": [P, i32, dp, dp, dp],
            "elbm_set_force_field": [P, i32, P],
            "elbm_advance": [P, i32],
            "elbm_read_moments": [P, i32, P, P, P],
            "elbm_read_populations": [P, i32, P],
            "elbm_sample_populations": [P, i32, i64, i64p, dp],
            "elbm_reduce": [P, dp, dp, i64p],
            "elbm_check": [P],
            "elbm_drag": [P, i32, dp, i64p, i32],
            "elbm_set_gamma_output": [P, i32],
            "elbm_brick_dims": [i32, i64p],
            "elbm_gamma_indicator": [P, i32, P, i64p],
            "elbm_transfer_state": [P, P],
            "elbm_set_launch": [P, i32, i32, i32, i32, i32, i32],
            "elbm_tune": [P, ctypes.c_char_p, i32],
            "elbm_get_launch": [P, P],
            "elbm_profile": [P, i32, dp, dp, i64p],
            "elbm_synchronize": [P],
            "elbm_stream_copy": [P, P, ctypes.c_size_t, i32, P],
            "elbm_state_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
            "elbm_save_state": [P, P],
            "elbm_load_state": [P, P],
            "elbm_adjoint_bytes": [P, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
            "elbm_adjoint_bind": [P, P, ctypes.c_size_t, i32, i32],
            "elbm_adjoint_forward": [P, i32, i32, i32, dp, dp],
            "elbm_adjoint_backward": [P],
            "elbm_adjoint_read": [P, i32, P, P],
            "elbm_adjoint_velocity": [P, i32, dp, dp, dp, dp],
            "elbm_adjoint_timing": [P, dp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        L.elbm_status_string.restype = ctypes.c_char_p
        L.elbm_status_string.argtypes = [ctypes.c_int]
        L.elbm_last_error.restype = ctypes.c_char_p
        L.elbm_last_error.argtypes = [P]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64(v: Sequence[int]) -> np.ndarray:
    a = np.zeros(3, dtype=np.int64)
    a[: len(v)] = v
    return a


def _f3(v) -> np.ndarray:
    a = np.zeros(3, dtype=np.float64)
    a[: len(v)] = v
    return a


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def stream_copy(dst: torch.Tensor, src: torch.Tensor, grid: int = 0, stream=None) -> None:
    """elbm_stream_copy: plain streaming copy of src into dst (device tensors of equal
    byte size, a multiple of 16), on `stream` (default: the current torch stream)."""
    nbytes = src.numel() * src.element_size()
    assert src.is_cuda and dst.is_cuda and dst.numel() * dst.element_size() == nbytes
    s = stream or torch.cuda.current_stream(src.device)
    rc = lib().elbm_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes, int(grid),
                                ctypes.c_void_p(s.cuda_stream))
    if rc:
        raise ElbmError(rc, "elbm_stream_copy")


class Lattice:
    """One refined lattice on the current HIP device.

    Methods mirror the C ABI (elbm_*); the workspace is a torch uint8 tensor and the
    stream the current torch stream at bind time."""

    def __init__(self, D: int, N, periodic, nu0: float, n_levels: int, storage="f32"):
        self.D, self.Q, self.L = D, (9 if D == 2 else 27), n_levels
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        d = _Desc()
        d.dim, d.storage, d.nu0, d.n_levels = D, self.storage, float(nu0), n_levels
        for a in range(3):
            d.extent[a] = int(N[a]) if a < D else 1
            d.periodic[a] = int(bool(periodic[a])) if a < D else 0
        h = ctypes.c_void_p()
        rc = lib().elbm_create(ctypes.byref(d), ctypes.byref(h))
        if rc:
            raise ElbmError(rc, "elbm_create failed")
        self._h = h
        self.workspace = None
        self.stream = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.elbm_destroy(h)
            self._h = None

    # -- plumbing
    def _ck(self, rc):
        if rc:
            raise ElbmError(rc, lib().elbm_last_error(self._h).decode())

    # -- description (elbm_set_face, elbm_add_block, elbm_set_solid, elbm_set_force_uniform)
    def set_face(self, face, kind, u=(0.0, 0.0, 0.0)):
        uu = _f3(u)
        self._ck(lib().elbm_set_face(self._h, face, kind, _dp(uu)))

    def add_block(self, level, lo, hi):
        a, b = _i64(lo), _i64(hi)
        self._ck(lib().elbm_add_block(self._h, level, _p64(a), _p64(b)))

    add_box = add_block

    def set_solid(self, level, lo, mask):
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        n = list(mask.shape[::-1]) + [1] * (3 - mask.ndim)
        a, b = _i64(lo), _i64(n)
        self._ck(lib().elbm_set_solid(self._h, level, _p64(a), _p64(b), mask.ctypes.data))

    def set_force_uniform(self, F):
        FF = _f3(F)
        self._ck(lib().elbm_set_force_uniform(self._h, _dp(FF)))

    def finalize(self):
        n = ctypes.c_size_t()
        self._ck(lib().elbm_finalize(self._h, ctypes.byref(n)))
        self.workspace_bytes = n.value
        return n.value

    # -- queries
    def level_box(self, level):
        lo, n = np.zeros(3, np.int64), np.zeros(3, np.int64)
        self._ck(lib().elbm_level_box(self._h, level, _p64(lo), _p64(n)))
        return lo, n

    def shape(self, level):
        _, n = self.level_box(level)
        return tuple(int(v) for v in n[: self.D][::-1])

    def level_info(self, level):
        nn, nf, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        b = ctypes.c_double()
        self._ck(lib().elbm_level_info(self._h, level, ctypes.byref(nn), ctypes.byref(nf), ctypes.byref(b),
                                       ctypes.byref(nb)))
        return nn.value, nf.value, b.value, nb.value

    def node_class(self, level):
        out = np.empty(self.shape(level), dtype=np.int32)
        self._ck(lib().elbm_node_class(self._h, level, out.ctypes.data))
        return out

    def weights(self, level):
        out = np.empty(self.shape(level))
        self._ck(lib().elbm_weights(self._h, level, _dp(out)))
        return out

    # -- device side
    def bind(self, device: Optional[torch.device] = None):
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)
        ptr = self.workspace.data_ptr()
        off = (-ptr) % 256
        self.stream = torch.cuda.current_stream(device)
        self._ck(lib().elbm_bind(self._h, ctypes.c_void_p(ptr + off), self.workspace_bytes,
                                 ctypes.c_void_p(self.stream.cuda_stream)))

    def init(self, level, rho, u, noise=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        self._ck(lib().elbm_init_fields(self._h, level, _dp(rho), _dp(u), None if nz is None else _dp(nz)))

    init_fields = init

    def init_static(self, level, rho, u, noise=None):
        """elbm_init_fields_static: the same initial state, staged through the library's
        static device buffer (no device allocation)."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        self._ck(lib().elbm_init_fields_static(self._h, level, _dp(rho), _dp(u), None if nz is None else _dp(nz)))

    def set_force_field(self, level, F: Optional[torch.Tensor]):
        if F is None:
            self._ck(lib().elbm_set_force_field(self._h, level, None))
            return
        assert F.dtype == torch.float64 and F.is_cuda and F.is_contiguous()
        assert F.numel() == self.D * int(np.prod(self.shape(level)))
        self._keep_force = F
        self._ck(lib().elbm_set_force_field(self._h, level, ctypes.c_void_p(F.data_ptr())))

    def advance(self, n=1):
        self._ck(lib().elbm_advance(self._h, int(n)))

    def synchronize(self):
        self._ck(lib().elbm_synchronize(self._h))

    def moments_device(self, level):
        """(rho, u) of a level as float64 device tensors over the level box (NaN at absent
        and solid nodes), left on the device; asynchronous on the bound stream."""
        sh = self.shape(level)
        dev = self.workspace.device
        rho = torch.empty(sh, dtype=torch.float64, device=dev)
        u = torch.empty((self.D,) + sh, dtype=torch.float64, device=dev)
        self._ck(lib().elbm_read_moments(self._h, level, ctypes.c_void_p(rho.data_ptr()),
                                         ctypes.c_void_p(u.data_ptr()), None))
        return rho, u

    def moments(self, level, gamma=False):
        sh = self.shape(level)
        dev = self.workspace.device
        rho = torch.empty(sh, dtype=torch.float64, device=dev)
        u = torch.empty((self.D,) + sh, dtype=torch.float64, device=dev)
        g = torch.empty(sh, dtype=torch.float64, device=dev) if gamma else None
        self._ck(lib().elbm_read_moments(self._h, level, ctypes.c_void_p(rho.data_ptr()),
                                         ctypes.c_void_p(u.data_ptr()),
                                         ctypes.c_void_p(g.data_ptr()) if gamma else None))
        self.synchronize()
        out = (rho.cpu().numpy(), u.cpu().numpy())
        return out + ((g.cpu().numpy(),) if gamma else ())

    def get_f(self, level):
        sh = (self.Q,) + self.shape(level)
        f = torch.empty(sh, dtype=torch.float64, device=self.workspace.device)
        self._ck(lib().elbm_read_populations(self._h, level, ctypes.c_void_p(f.data_ptr())))
        self.synchronize()
        return f.cpu().numpy()

    def sample_f(self, level, coords):
        c = np.zeros((len(coords), 3), dtype=np.int64)
        c[:, : np.asarray(coords).shape[1]] = coords
        out = np.empty((len(coords), self.Q))
        self._ck(lib().elbm_sample_populations(self._h, level, len(coords), _p64(c), _dp(out)))
        return out

    def reduce(self):
        m = ctypes.c_double()
        mom = np.zeros(3)
        bad = ctypes.c_int64()
        self._ck(lib().elbm_reduce(self._h, ctypes.byref(m), _dp(mom), ctypes.byref(bad)))
        return m.value, mom[: self.D], bad.value

    def check(self):
        rc = lib().elbm_check(self._h)
        if rc == 5:
            return False
        self._ck(rc)
        return True

    def drag(self, level, reset=False):
        F = np.zeros(3)
        st = ctypes.c_int64()
        self._ck(lib().elbm_drag(self._h, level, _dp(F), ctypes.byref(st), int(reset)))
        return F[: self.D], st.value

    def set_gamma_output(self, enable=True):
        self._ck(lib().elbm_set_gamma_output(self._h, int(enable)))

    def brick_dims(self):
        d = np.zeros(3, np.int64)
        st = lib().elbm_brick_dims(self.D, _p64(d))
        if st:
            raise ElbmError(st, "elbm_brick_dims")
        return d

    def gamma_indicator(self, level):
        """Per brick of the level, the largest |gamma - 2| over its fluid nodes (-1 where
        a brick has none), as an array over the brick grid, z/y, ..., x order."""
        grid = np.zeros(3, np.int64)
        self._ck(lib().elbm_gamma_indicator(self._h, level, None, _p64(grid)))
        out = torch.empty(int(grid.prod()), dtype=torch.float32, device=self.workspace.device)
        self._ck(lib().elbm_gamma_indicator(self._h, level, ctypes.c_void_p(out.data_ptr()), _p64(grid)))
        self.synchronize()
        return out.cpu().numpy().reshape(tuple(int(v) for v in grid[: self.D][::-1]))

    def transfer_from(self, src: "Lattice"):
        """Re-meshing: take over the current state of another bound lattice of the same
        domain, levels and parameters with other refinement blocks (coarse-step
        boundary)."""
        self._ck(lib().elbm_transfer_state(self._h, src._h))

    def set_launch(self, use_graph=1, wg_per_cu=0, xcd_remap=1, threads=256, occupancy=1, pipeline=0):
        self._ck(lib().elbm_set_launch(self._h, int(use_graph), int(wg_per_cu), int(xcd_remap), int(threads),
                                       int(occupancy), int(pipeline)))

    def get_launch(self):
        cfg = (ctypes.c_int32 * 6)()
        self._ck(lib().elbm_get_launch(self._h, cfg))
        return dict(zip(("use_graph", "wg_per_cu", "xcd_remap", "threads", "occupancy", "pipeline"), list(cfg)))

    def tune(self, cache_path=None, steps=3):
        self._ck(lib().elbm_tune(self._h, cache_path.encode() if cache_path else None, int(steps)))

    def use_cached_launch(self, cache_path=None) -> bool:
        """Apply the cached launch configuration for this workload shape (default cache:
        LAUNCH_CACHE).  Returns False, configuration unchanged, when the cache has none."""
        try:
            self.tune(cache_path or LAUNCH_CACHE, steps=1)
            return True
        except ElbmError as e:
            if e.status == 2 and "no cached launch configuration" in str(e):
                return False
            raise

    def profile(self, steps):
        tot, sc = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        self._ck(lib().elbm_profile(self._h, int(steps), ctypes.byref(tot), ctypes.byref(sc), ctypes.byref(n)))
        return tot.value, sc.value, n.value

    def state_bytes(self):
        n = ctypes.c_size_t()
        self._ck(lib().elbm_state_bytes(self._h, ctypes.byref(n)))
        return n.value

    def save_state(self, dst: torch.Tensor):
        assert dst.is_cuda and dst.numel() * dst.element_size() >= self.state_bytes()
        self._ck(lib().elbm_save_state(self._h, ctypes.c_void_p(dst.data_ptr())))

    def load_state(self, src: torch.Tensor):
        assert src.is_cuda and src.numel() * src.element_size() >= self.state_bytes()
        self._ck(lib().elbm_load_state(self._h, ctypes.c_void_p(src.data_ptr())))

    # -- discrete adjoint
    def adjoint_bind(self, n_max: int, K: int):
        """Allocate and bind the adjoint workspace for runs of up to n_max coarse steps,
        checkpointing every K."""
        n = ctypes.c_size_t()
        self._ck(lib().elbm_adjoint_bytes(self._h, int(n_max), int(K), ctypes.byref(n)))
        self.adjoint_workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=self.workspace.device)
        ptr = self.adjoint_workspace.data_ptr()
        self._ck(lib().elbm_adjoint_bind(self._h, ctypes.c_void_p(ptr + (-ptr) % 256), n.value, int(n_max), int(K)))

    def adjoint_forward(self, n: int, objective="drag", body_level=0, direction=(1.0, 0.0, 0.0)) -> float:
        J = ctypes.c_double()
        d = _f3(direction)
        self._ck(lib().elbm_adjoint_forward(self._h, int(n), OBJECTIVES[objective], int(body_level), _dp(d),
                                            ctypes.byref(J)))
        return J.value

    def adjoint_backward(self):
        self._ck(lib().elbm_adjoint_backward(self._h))

    def adjoint_read(self, level):
        """(dJ/df0 [Q, *box], dJ/dF [D, *box]) as float64 device tensors."""
        sh = self.shape(level)
        dev = self.workspace.device
        lam = torch.empty((self.Q,) + sh, dtype=torch.float64, device=dev)
        gF = torch.empty((self.D,) + sh, dtype=torch.float64, device=dev)
        self._ck(lib().elbm_adjoint_read(self._h, level, ctypes.c_void_p(lam.data_ptr()),
                                         ctypes.c_void_p(gF.data_ptr())))
        self.synchronize()
        return lam, gF

    def adjoint_velocity(self, level, rho, u, noise=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        out = np.zeros_like(u)
        self._ck(lib().elbm_adjoint_velocity(self._h, level, _dp(rho), _dp(u), None if nz is None else _dp(nz),
                                             _dp(out)))
        return out

    def adjoint_timing(self):
        """(forward with checkpoints, recomputation, reverse sweep, whole backward pass) in ms"""
        ms = np.zeros(4)
        self._ck(lib().elbm_adjoint_timing(self._h, _dp(ms)))
        return tuple(ms)


class ForceObjective(torch.autograd.Function):
    """J(F_0, ..., F_{L-1}) for per-level force fields F_l ([D, *box] float64 device
    tensors): loads the initial state, sets the fields, runs n coarse steps through
    elbm_adjoint_forward; backward runs elbm_adjoint_backward and returns dJ/dF_l."""

    @staticmethod
    def forward(ctx, lat, state, n, objective, body_level, direction, *forces):
        lat.load_state(state)
        for l, F in enumerate(forces):
            lat.set_force_field(l, F.detach().contiguous())
        J = lat.adjoint_forward(n, objective, body_level, direction)
        ctx.lat, ctx.nf = lat, len(forces)
        return torch.tensor(J, dtype=torch.float64, device=state.device)

    @staticmethod
    def backward(ctx, gJ):
        ctx.lat.adjoint_backward()
        grads = tuple(gJ * ctx.lat.adjoint_read(l)[1] for l in range(ctx.nf))
        return (None,) * 6 + grads


class VelocityObjective(torch.autograd.Function):
    """J(u0_0, ..., u0_{L-1}) for per-level initial velocity fields ([D, *box] float64
    tensors, initialised with rho0 and noise as elbm_init_fields); backward returns
    dJ/du0_l through elbm_adjoint_velocity."""

    @staticmethod
    def forward(ctx, lat, rho, noise, n, objective, body_level, direction, *u0):
        host = [u.detach().cpu().numpy() for u in u0]
        for l, u in enumerate(host):
            lat.init(l, rho[l], u, None if noise is None else noise[l])
        J = lat.adjoint_forward(n, objective, body_level, direction)
        ctx.lat, ctx.rho, ctx.noise, ctx.u0 = lat, rho, noise, host
        ctx.dev = [u.device for u in u0]
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        ctx.lat.adjoint_backward()
        grads = []
        for l, u in enumerate(ctx.u0):
            g = ctx.lat.adjoint_velocity(l, ctx.rho[l], u, None if ctx.noise is None else ctx.noise[l])
            grads.append(gJ.to(torch.float64).cpu() * torch.from_numpy(g).to(ctx.dev[l]))
        return (None,) * 7 + tuple(grads)
