"""FP64 CPU oracle of the cascaded thermal LBM (Fei & Luo, arXiv:1801.04577).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code
with the GPU library and never imports it.

The arithmetic lives in ``clbm_oracle.c`` (literal dense matrices of Eq. (6),
(16), (17), numerical inverses, push streaming, Eq. (26)-(28) walls). This
module only marshals numpy arrays through ctypes.

Problem description: a plain dict with keys ``nx, ny, nu, alpha, g_beta, T0,
Fx, Fy, Q`` (floats), an optional source field ``Q_field`` ([ny][nx], added to
Q per node), optional rate overrides ``s_b, s_4, s_3, lambda_0,
lambda_2`` (None means the paper's default or rule) and ``sides``: four dicts
(order x-, x+, y-, y+) with ``kind`` ("periodic" or "wall"), ``u_wall`` and
the Robin data ``b1, b2, b3`` of ``b1 dT/dn + b2 T = b3`` (n outward).
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CLBM_ORACLE_LIB names another build of the same source (the mutation tests load
# copies with a planted mistake); the default is the library next to this file.
_LIBPATH = os.environ.get("CLBM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("nu", ctypes.c_double), ("alpha", ctypes.c_double),
        ("s_b", ctypes.c_double), ("s_4", ctypes.c_double), ("s_3", ctypes.c_double),
        ("lambda_0", ctypes.c_double), ("lambda_2", ctypes.c_double),
        ("g_beta", ctypes.c_double), ("T0", ctypes.c_double),
        ("Fx", ctypes.c_double), ("Fy", ctypes.c_double), ("Q", ctypes.c_double),
        ("viscous_heating", ctypes.c_int),
        ("kind", ctypes.c_int * 4), ("u_wall", ctypes.c_double * 4),
        ("b1", ctypes.c_double * 4), ("b2", ctypes.c_double * 4), ("b3", ctypes.c_double * 4),
        ("Q_field", ctypes.POINTER(ctypes.c_double)),
    ]


_D = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _build
        _build.build()
    L = ctypes.CDLL(_LIBPATH)
    P = ctypes.POINTER(_Params)
    vp = ctypes.c_void_p
    L.oracle_version.restype = ctypes.c_int
    L.oracle_rates.argtypes = [P, _D]
    for name in ("oracle_matrix_M", "oracle_matrix_MT", "oracle_matrix_Minv", "oracle_matrix_MTinv"):
        getattr(L, name).argtypes = [_D]
        getattr(L, name).restype = None
    for name in ("oracle_matrix_N", "oracle_matrix_NT"):
        getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_double, _D]
        getattr(L, name).restype = None
    L.oracle_equilibrium.argtypes = [ctypes.c_double] * 4 + [_D, _D]
    L.oracle_equilibrium.restype = None
    L.oracle_collide.argtypes = [P, _D, _D, _D, _D, _D]
    L.oracle_create.argtypes = [P, ctypes.POINTER(vp)]
    L.oracle_destroy.argtypes = [vp]
    L.oracle_destroy.restype = None
    L.oracle_init.argtypes = [vp, _D, _D, _D, _D]
    L.oracle_step.argtypes = [vp, ctypes.c_long, ctypes.c_int]
    L.oracle_step_count.argtypes = [vp]
    L.oracle_step_count.restype = ctypes.c_long
    L.oracle_macros.argtypes = [vp, _D, _D, _D, _D]
    L.oracle_get_state.argtypes = [vp, _D, _D]
    L.oracle_set_state.argtypes = [vp, _D, _D, ctypes.c_long]
    L.oracle_post_collision.argtypes = [vp, _D, _D, ctypes.c_int]
    L.oracle_wall_values.argtypes = [vp, ctypes.c_int, _D, _D]
    _lib = L
    return L


class OracleError(RuntimeError):
    pass


def _check(code, what):
    if code != 0:
        raise OracleError("%s failed with status %d" % (what, code))


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _nan_if_none(v):
    return float("nan") if v is None else float(v)


_KIND = {"periodic": 0, "wall": 1}


def make_params(prob):
    p = _Params()
    p.nx, p.ny = int(prob["nx"]), int(prob["ny"])
    p.nu, p.alpha = float(prob["nu"]), float(prob["alpha"])
    for k in ("s_b", "s_4", "s_3", "lambda_0", "lambda_2"):
        setattr(p, k, _nan_if_none(prob.get(k)))
    p.g_beta = float(prob.get("g_beta", 0.0))
    p.T0 = float(prob.get("T0", 0.0))
    p.Fx = float(prob.get("Fx", 0.0))
    p.Fy = float(prob.get("Fy", 0.0))
    p.Q = float(prob.get("Q", 0.0))
    p.viscous_heating = int(bool(prob.get("viscous_heating", False)))
    for s, side in enumerate(prob["sides"]):
        p.kind[s] = _KIND[side["kind"]]
        p.u_wall[s] = float(side.get("u_wall", 0.0))
        p.b1[s] = float(side.get("b1", 0.0))
        p.b2[s] = float(side.get("b2", 1.0))
        p.b3[s] = float(side.get("b3", 0.0))
    return p


def _source_field(prob):
    """The problem's per-node source field as a contiguous float64 [ny][nx] array, or None."""
    q = prob.get("Q_field")
    if q is None:
        return None
    q = np.ascontiguousarray(np.broadcast_to(np.asarray(q, dtype=np.float64),
                                             (int(prob["ny"]), int(prob["nx"]))))
    return q


def rates(prob):
    """(s_nu, s_b, s_3, s_4, lambda_0, lambda_1, lambda_2) the oracle uses."""
    out = np.zeros(7)
    _check(lib().oracle_rates(ctypes.byref(make_params(prob)), _ptr(out)), "oracle_rates")
    return out


def matrix_M():
    out = np.zeros(81)
    lib().oracle_matrix_M(_ptr(out))
    return out.reshape(9, 9)


def matrix_Minv():
    out = np.zeros(81)
    lib().oracle_matrix_Minv(_ptr(out))
    return out.reshape(9, 9)


def matrix_N(ux, uy):
    out = np.zeros(81)
    lib().oracle_matrix_N(float(ux), float(uy), _ptr(out))
    return out.reshape(9, 9)


def matrix_MT():
    out = np.zeros(25)
    lib().oracle_matrix_MT(_ptr(out))
    return out.reshape(5, 5)


def matrix_MTinv():
    out = np.zeros(25)
    lib().oracle_matrix_MTinv(_ptr(out))
    return out.reshape(5, 5)


def matrix_NT(ux, uy):
    out = np.zeros(25)
    lib().oracle_matrix_NT(float(ux), float(uy), _ptr(out))
    return out.reshape(5, 5)


def equilibrium(rho, ux, uy, T):
    f = np.zeros(9)
    g = np.zeros(5)
    lib().oracle_equilibrium(float(rho), float(ux), float(uy), float(T), _ptr(f), _ptr(g))
    return f, g


def collide(prob, f, g):
    """One node: returns (f_post, g_post, (rho, ux, uy, T))."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    fp = np.zeros(9)
    gp = np.zeros(5)
    m = np.zeros(4)
    _check(lib().oracle_collide(ctypes.byref(make_params(prob)), _ptr(f), _ptr(g), _ptr(fp),
                                _ptr(gp), _ptr(m)), "oracle_collide")
    return fp, gp, tuple(m)


def default_threads():
    """OMP_NUM_THREADS when set, else the host's cores (at most 16)."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, min(16, os.cpu_count() or 1))


class Sim:
    """A lattice advanced by the oracle. Fields are float64 arrays [ny][nx]."""

    def __init__(self, prob, rho=None, ux=None, uy=None, T=None, nthreads=None):
        self.prob = dict(prob)
        self.nx, self.ny = int(prob["nx"]), int(prob["ny"])
        self.nthreads = nthreads or default_threads()
        self._p = make_params(prob)
        # the source field stays referenced for the life of the simulation
        self._qfield = _source_field(prob)
        if self._qfield is not None:
            self._p.Q_field = _ptr(self._qfield)
        h = ctypes.c_void_p()
        _check(lib().oracle_create(ctypes.byref(self._p), ctypes.byref(h)), "oracle_create")
        self._h = h
        self.init(rho, ux, uy, T)

    def _field(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64),
                                                 (self.ny, self.nx)))
        return a

    def init(self, rho=None, ux=None, uy=None, T=None):
        fs = [self._field(a) for a in (rho, ux, uy, T)]
        self._keep = fs
        _check(lib().oracle_init(self._h, *[_ptr(a) for a in fs]), "oracle_init")

    def step(self, n=1):
        _check(lib().oracle_step(self._h, int(n), int(self.nthreads)), "oracle_step")

    @property
    def t(self):
        return lib().oracle_step_count(self._h)

    def macros(self):
        """(rho, ux, uy, T) at the current time, each [ny][nx]."""
        out = [np.zeros((self.ny, self.nx)) for _ in range(4)]
        _check(lib().oracle_macros(self._h, *[_ptr(a) for a in out]), "oracle_macros")
        return tuple(out)

    def state(self):
        f = np.zeros((self.ny, self.nx, 9))
        g = np.zeros((self.ny, self.nx, 5))
        _check(lib().oracle_get_state(self._h, _ptr(f), _ptr(g)), "oracle_get_state")
        return f, g

    def set_state(self, f, g, step=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.size == self.nx * self.ny * 9 and g.size == self.nx * self.ny * 5
        _check(lib().oracle_set_state(self._h, _ptr(f), _ptr(g), int(step)), "oracle_set_state")

    def post_collision(self):
        f = np.zeros((self.ny, self.nx, 9))
        g = np.zeros((self.ny, self.nx, 5))
        _check(lib().oracle_post_collision(self._h, _ptr(f), _ptr(g), int(self.nthreads)),
               "oracle_post_collision")
        return f, g

    def wall_values(self, side):
        n = self.ny if side < 2 else self.nx
        Tw = np.zeros(n)
        d = np.zeros(n)
        _check(lib().oracle_wall_values(self._h, int(side), _ptr(Tw), _ptr(d)), "oracle_wall_values")
        return Tw, d

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nan_to_default(x):
    return None if x is None or (isinstance(x, float) and math.isnan(x)) else x
