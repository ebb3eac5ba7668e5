"""Plain FP64 CPU oracle for grid-refined KBC lattice Boltzmann (ctypes binding).

TEST INFRASTRUCTURE: the independent reference for the HIP library.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this package.
The arithmetic lives in ``elbm_oracle.c``; this module marshals arguments, apart from
``gamma_indicator``, a plain numpy reduction of the gamma field the C oracle returns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "elbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

FACE_WALL, FACE_INLET, FACE_OUTFLOW = 1, 2, 3


def compile_library(src: str, out: str, openmp: bool = False) -> str:
    """gcc, plain -O2, IEEE arithmetic; with openmp the node loops run on several
    threads (same arithmetic, same results: every parallel loop writes per-node values
    and every sum stays serial)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared"] + (["-fopenmp"] if openmp else []) + ["-o", tmp, src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the single-thread oracle and its OpenMP build."""
    for out, omp in ((_LIB, False), (_LIB_OMP, True)):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            compile_library(_SRC, out, omp)
    return _LIB


def _configure(L):
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    L.ora_create.restype = P
    L.ora_create.argtypes = [ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_int]
    L.ora_destroy.argtypes = [P]
    L.ora_error.restype = ctypes.c_char_p
    L.ora_error.argtypes = [P]
    for name, args in [
        ("ora_set_face", [P, ctypes.c_int, ctypes.c_int, dp]),
        ("ora_add_box", [P, ctypes.c_int, i64p, i64p]),
        ("ora_set_solid", [P, ctypes.c_int, i64p, i64p, ctypes.c_void_p]),
        ("ora_set_force_uniform", [P, dp]),
        ("ora_finalize", [P]),
        ("ora_level_box", [P, ctypes.c_int, i64p, i64p]),
        ("ora_level_info", [P, ctypes.c_int, i64p, i64p, dp]),
        ("ora_node_class", [P, ctypes.c_int, ctypes.c_void_p]),
        ("ora_weights", [P, ctypes.c_int, dp]),
        ("ora_init", [P, ctypes.c_int, dp, dp, dp]),
        ("ora_set_force_field", [P, ctypes.c_int, dp]),
        ("ora_set_f", [P, ctypes.c_int, dp]),
        ("ora_advance", [P, ctypes.c_int]),
        ("ora_get_f", [P, ctypes.c_int, dp]),
        ("ora_moments", [P, ctypes.c_int, dp, dp, dp]),
        ("ora_sample_f", [P, ctypes.c_int, ctypes.c_int64, i64p, dp]),
        ("ora_reduce", [P, dp, dp]),
        ("ora_drag", [P, ctypes.c_int, dp, i64p, ctypes.c_int]),
        ("ora_couple_states", [P, ctypes.c_int, dp, dp]),
        ("ora_transfer_state", [P, P]),
    ]:
        fn = getattr(L, name)
        fn.restype = ctypes.c_int
        fn.argtypes = args
    L.ora_feq.restype = None
    L.ora_feq.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
    L.ora_kbc.restype = ctypes.c_double
    L.ora_kbc.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp, dp]
    L.ora_beta.restype = ctypes.c_double
    L.ora_beta.argtypes = [ctypes.c_double]
    L.ora_threads.restype = ctypes.c_int
    L.ora_threads.argtypes = []
    L.ora_kbc_adj.restype = None
    L.ora_kbc_adj.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp, dp]
    for name, args in [
        ("ora_adjoint_run", [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]),
        ("ora_adjoint_state", [P, ctypes.c_int, dp]),
        ("ora_adjoint_force", [P, ctypes.c_int, dp]),
        ("ora_init_adjoint_u", [ctypes.c_int, ctypes.c_int64, dp, dp, dp, dp, dp]),
    ]:
        fn = getattr(L, name)
        fn.restype = ctypes.c_int
        fn.argtypes = args
    return L


def load_library(path: str):
    """A configured handle of an oracle library built from elbm_oracle.c (the OpenMP
    build, or a deliberately altered copy that a test uses to check a pin fails)."""
    return _configure(ctypes.CDLL(path))


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def lib_omp():
    """The OpenMP build (threads from OMP_NUM_THREADS, else every core)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
            build(force=True)
        _lib_omp = load_library(_LIB_OMP)
    return _lib_omp


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64(v):
    a = np.zeros(3, dtype=np.int64)
    a[: len(v)] = v
    return a


def _f3(v):
    a = np.zeros(3, dtype=np.float64)
    a[: len(v)] = v
    return a


def omp_threads() -> int:
    """Threads the OpenMP build's node loops run on."""
    return int(lib_omp().ora_threads())


def q_of(D: int) -> int:
    return 9 if D == 2 else 27


def beta(nu: float) -> float:
    return lib().ora_beta(float(nu))


def feq(D: int, rho: float, u) -> np.ndarray:
    out = np.empty(q_of(D))
    uu = _f3(u)
    lib().ora_feq(D, float(rho), _dp(uu), _dp(out))
    return out


def kbc(D: int, beta_: float, f, F=(0.0, 0.0, 0.0)):
    """One collision; returns (f_post, gamma, ds, dh)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    Q = q_of(D)
    out, ds, dh = np.empty(Q), np.empty(Q), np.empty(Q)
    FF = _f3(F)
    g = lib().ora_kbc(D, float(beta_), _dp(f), _dp(FF), _dp(out), _dp(ds), _dp(dh))
    return out, g, ds, dh


def kbc_adj(D: int, beta_: float, f, lo, F=(0.0, 0.0, 0.0)):
    """Reverse of one collision: (adjoint of f, adjoint of F) for the adjoint lo of f'."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    lf = np.empty(q_of(D))
    FF = _f3(F)
    lF = np.zeros(3)
    lib().ora_kbc_adj(D, float(beta_), _dp(f), _dp(FF), _dp(lo), _dp(lf), _dp(lF))
    return lf, lF[:D]


def init_adjoint_u(D, rho, u, noise, lam):
    """Gradient wrt the initial velocity through f = f^eq(rho, u)(1 + noise)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
    out = np.empty_like(u)
    lib().ora_init_adjoint_u(D, rho.size, _dp(rho), _dp(u), None if nz is None else _dp(nz), _dp(lam), _dp(out))
    return out


def gamma_indicator(gamma: np.ndarray, bdims) -> np.ndarray:
    """Under-resolution indicator per block of a level: resolved flow drives the
    stabiliser gamma of Eq. gamma_min_approx to its LBGK value 2, so |gamma - 2|
    measures under-resolution (Sec. IV, turbulent channel flow) and serves as the
    refinement criterion the conclusion (Sec. V) proposes.  `gamma` is a level's field
    (z/y, ..., x order, NaN at nodes without a value), `bdims` the block extent along
    x, y, z.  Blocks tile the field from its origin; the result holds, per block, the
    largest |gamma - 2| over its nodes with a value, -1 for a block without any."""
    D = gamma.ndim
    ext = [int(bdims[a]) for a in range(D)][::-1]  # block extent in array-axis order
    grid = [-(-gamma.shape[k] // ext[k]) for k in range(D)]
    out = np.full(grid, -1.0)
    for idx in np.ndindex(*grid):
        sl = tuple(slice(idx[k] * ext[k], (idx[k] + 1) * ext[k]) for k in range(D))
        block = gamma[sl]
        vals = np.abs(block[np.isfinite(block)] - 2.0)
        if vals.size:
            out[idx] = vals.max()
    return out


class OracleError(RuntimeError):
    pass


class Oracle:
    """The refined KBC hierarchy, run literally on the CPU in FP64."""

    def __init__(self, D, N, periodic, nu0, n_levels, library=None):
        """library: None (single thread), "omp" (the OpenMP build) or a handle from
        load_library."""
        self.D, self.Q, self.L = D, q_of(D), n_levels
        self._lib = lib() if library is None else lib_omp() if library == "omp" else library
        per = (ctypes.c_int * 3)(*[int(bool(p)) for p in list(periodic) + [0] * (3 - len(periodic))])
        NN = _i64(N)
        self._h = self._lib.ora_create(D, NN.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), per, float(nu0),
                                       n_levels)
        if not self._h:
            raise OracleError("ora_create failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ora_destroy(h)
            self._h = None

    def _ck(self, rc):
        if rc != 0:
            raise OracleError("oracle error %d: %s" % (rc, self._lib.ora_error(self._h).decode()))

    @staticmethod
    def _p64(a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def set_face(self, face, kind, u=(0.0, 0.0, 0.0)):
        uu = _f3(u)
        self._ck(self._lib.ora_set_face(self._h, face, kind, _dp(uu)))

    def add_box(self, level, lo, hi):
        a, b = _i64(lo), _i64(hi)
        self._ck(self._lib.ora_add_box(self._h, level, self._p64(a), self._p64(b)))

    def set_solid(self, level, lo, mask):
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        n = list(mask.shape[::-1]) + [1] * (3 - mask.ndim)
        a, b = _i64(lo), _i64(n)
        self._ck(self._lib.ora_set_solid(self._h, level, self._p64(a), self._p64(b), mask.ctypes.data))

    def set_force_uniform(self, F):
        FF = _f3(F)
        self._ck(self._lib.ora_set_force_uniform(self._h, _dp(FF)))

    def finalize(self):
        self._ck(self._lib.ora_finalize(self._h))

    def level_box(self, level):
        lo, n = np.zeros(3, np.int64), np.zeros(3, np.int64)
        self._ck(self._lib.ora_level_box(self._h, level, self._p64(lo), self._p64(n)))
        return lo, n

    def shape(self, level):
        """numpy shape of a dense level array (z, y, x) or (y, x)."""
        _, n = self.level_box(level)
        return tuple(int(v) for v in n[: self.D][::-1])

    def level_info(self, level):
        nn, nf = ctypes.c_int64(), ctypes.c_int64()
        b = ctypes.c_double()
        self._ck(self._lib.ora_level_info(self._h, level, ctypes.byref(nn), ctypes.byref(nf), ctypes.byref(b)))
        return nn.value, nf.value, b.value

    def node_class(self, level):
        out = np.empty(self.shape(level), dtype=np.int32)
        self._ck(self._lib.ora_node_class(self._h, level, out.ctypes.data))
        return out

    def weights(self, level):
        out = np.empty(self.shape(level))
        self._ck(self._lib.ora_weights(self._h, level, _dp(out)))
        return out

    def init(self, level, rho, u, noise=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        self._ck(self._lib.ora_init(self._h, level, _dp(rho), _dp(u), None if nz is None else _dp(nz)))

    def set_force_field(self, level, F):
        F = np.ascontiguousarray(F, dtype=np.float64)
        self._ck(self._lib.ora_set_force_field(self._h, level, _dp(F)))

    def set_f(self, level, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._ck(self._lib.ora_set_f(self._h, level, _dp(f)))

    def advance(self, n=1):
        self._ck(self._lib.ora_advance(self._h, int(n)))

    def get_f(self, level):
        out = np.empty((self.Q,) + self.shape(level))
        self._ck(self._lib.ora_get_f(self._h, level, _dp(out)))
        return out

    def moments(self, level):
        sh = self.shape(level)
        rho, u, g = np.empty(sh), np.empty((self.D,) + sh), np.empty(sh)
        self._ck(self._lib.ora_moments(self._h, level, _dp(rho), _dp(u), _dp(g)))
        return rho, u, g

    def sample_f(self, level, coords):
        c = np.zeros((len(coords), 3), dtype=np.int64)
        c[:, : np.asarray(coords).shape[1]] = coords
        out = np.empty((len(coords), self.Q))
        self._ck(self._lib.ora_sample_f(self._h, level, len(coords), self._p64(c), _dp(out)))
        return out

    def reduce(self):
        m = ctypes.c_double()
        mom = np.zeros(3)
        self._ck(self._lib.ora_reduce(self._h, ctypes.byref(m), _dp(mom)))
        return m.value, mom[: self.D]

    def adjoint(self, n, objective="drag", body_level=0, direction=(1.0, 0.0, 0.0)):
        """Run n coarse steps from the current state and the reverse sweep; returns J.
        objective: "drag" (mean momentum exchange along direction over every
        collision of body_level) or "ke" (final kinetic energy)."""
        J = ctypes.c_double()
        d = _f3(direction)
        self._ck(self._lib.ora_adjoint_run(self._h, int(n), 0 if objective == "drag" else 1, int(body_level), _dp(d),
                                       ctypes.byref(J)))
        return J.value

    def adjoint_state(self, level):
        out = np.empty((self.Q,) + self.shape(level))
        self._ck(self._lib.ora_adjoint_state(self._h, level, _dp(out)))
        return out

    def adjoint_force(self, level):
        out = np.empty((self.D,) + self.shape(level))
        self._ck(self._lib.ora_adjoint_force(self._h, level, _dp(out)))
        return out

    def drag(self, level, reset=False):
        F = np.zeros(3)
        st = ctypes.c_int64()
        self._ck(self._lib.ora_drag(self._h, level, _dp(F), ctypes.byref(st), int(reset)))
        return F[: self.D], st.value

    def couple_states(self, parent_level, g_parent, g_child):
        """Sec. III.C steps 3-4 alone on given post-stream states ([Q][box] of the two
        levels, NaN = missing); returns the coupled states."""
        gp = np.array(g_parent, dtype=np.float64, order="C", copy=True)
        gc = np.array(g_child, dtype=np.float64, order="C", copy=True)
        self._ck(self._lib.ora_couple_states(self._h, int(parent_level), _dp(gp), _dp(gc)))
        return gp, gc

    def transfer_from(self, src):
        """Re-meshing: take over the state of another oracle lattice of the same domain,
        levels and parameters with other refinement blocks (coarse-step boundary)."""
        self._ck(self._lib.ora_transfer_state(self._h, src._h))
