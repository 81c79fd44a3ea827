"""ctypes wrapper around the plain FP64 CPU oracle (dvm_oracle.cpp).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users. The oracle shares no code with the GPU
path; it is checked against the paper and the mathematics by the pins in the
test suite.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import quadrature

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dvm_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile the oracle with g++ -O3 -fopenmp into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
        lib.orc_create.restype = vp
        lib.orc_create.argtypes = [ctypes.c_int, ip, ctypes.POINTER(ctypes.c_uint8), ip, dp, dp,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int]
        lib.orc_destroy.argtypes = [vp]
        lib.orc_num_velocities.argtypes = [vp]
        lib.orc_set_initial.argtypes = [vp, dp, dp, dp]
        lib.orc_set_accommodation.restype = ctypes.c_int
        lib.orc_set_accommodation.argtypes = [vp, ctypes.c_double]
        lib.orc_set_shakhov.restype = ctypes.c_int
        lib.orc_set_shakhov.argtypes = [vp, ctypes.c_double]
        lib.orc_iterate.argtypes = [vp, ctypes.c_long, ctypes.c_double, ctypes.c_int, dp]
        lib.orc_get_moments.argtypes = [vp, dp, dp, dp, dp]
        lib.orc_get_phi.argtypes = [vp, dp]
        lib.orc_set_phi.argtypes = [vp, dp]
        lib.orc_get_flux.argtypes = [vp, dp, dp, dp]
        lib.orc_apply_advection.argtypes = [vp, ctypes.c_int, dp, dp]
        lib.orc_collision.argtypes = [vp, dp, dp]
        lib.orc_set_boundary_field.argtypes = [vp, dp]
        lib.orc_get_velocities.argtypes = [vp, dp, dp]
        lib.orc_iterations.restype = ctypes.c_long
        lib.orc_iterations.argtypes = [vp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


class OracleSolver:
    """One problem: mask (solid = 1, shape (N3, N2, N1) or (N2, N1), x1 fastest),
    1D velocity counts per axis, Kn, pressure jump J.

    If `grid` is None the half-range Gauss-Hermite grid of the oracle's own
    quadrature module is used; otherwise grid = [(nodes, weights), ...] per axis.
    stencil_rule 1 (default): first-order upwind stencil along an axis when
    either upstream image is solid; 0: only when the first one is.
    prandtl (with tau_feedback): Shakhov model with this Prandtl number.
    accommodation: Maxwell walls, the diffuse fraction alpha in (0, 1].
    """

    def __init__(self, solid, nv, kn, jump=1.0, lateral_periodic=False,
                 tau_feedback=False, threads=None, grid=None, stencil_rule=1, prandtl=None,
                 accommodation=1.0):
        lib = _load()
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        self.dim = solid.ndim
        if self.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.shape = solid.shape                      # (N2, N1) or (N3, N2, N1)
        self.n = list(reversed(solid.shape))          # [N1, N2(, N3)]
        self.N = int(solid.size)
        self.solid = solid
        if grid is None:
            grid = [quadrature.full_line_grid(int(m)) for m in nv]
        self.grid = [(np.asarray(x, float), np.asarray(w, float)) for x, w in grid]
        self.nv = [len(g[0]) for g in self.grid]
        nodes = np.concatenate([g[0] for g in self.grid]).astype(np.float64)
        weights = np.concatenate([g[1] for g in self.grid]).astype(np.float64)
        self.kn = float(kn)
        if threads is None:
            threads = os.cpu_count() or 1
        self.threads = int(threads)
        n_arr = (ctypes.c_int * 3)(*(self.n + [1] * (3 - self.dim)))
        nv_arr = (ctypes.c_int * 3)(*(self.nv + [1] * (3 - self.dim)))
        self._h = lib.orc_create(self.dim, n_arr,
                                 solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                 nv_arr, _dp(nodes), _dp(weights), self.kn, float(jump),
                                 int(bool(lateral_periodic)), int(bool(tau_feedback)),
                                 self.threads, int(stencil_rule))
        self._keep = (nodes, weights)
        self.K = lib.orc_num_velocities(self._h)
        if prandtl is not None and lib.orc_set_shakhov(self._h, float(prandtl)) != 0:
            raise ValueError("the Shakhov model needs tau_feedback and prandtl > 0")
        if accommodation != 1.0:
            if lib.orc_set_accommodation(self._h, float(accommodation)) != 0:
                raise ValueError("accommodation must be in (0, 1], and below 1 needs stencil_rule 1")
            self.set_initial()

    def close(self):
        if getattr(self, "_h", None):
            _load().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_initial(self, rho=None, u=None, tau=None):
        r = None if rho is None else np.ascontiguousarray(rho, np.float64).reshape(-1)
        uu = None if u is None else np.ascontiguousarray(u, np.float64).reshape(-1)
        t = None if tau is None else np.ascontiguousarray(tau, np.float64).reshape(-1)
        _load().orc_set_initial(self._h, _dp(r), _dp(uu), _dp(t))

    def iterate(self, iters, tol=0.0, stop_mode=0):
        st = np.zeros(5)
        rc = _load().orc_iterate(self._h, int(iters), float(tol), int(stop_mode), _dp(st))
        return {"converged": rc == 0, "iters": int(st[0]), "r": st[1], "err": st[2],
                "k": st[3], "Gp": st[4]}

    @property
    def iterations(self):
        return _load().orc_iterations(self._h)

    def moments(self):
        rho = np.zeros(self.N)
        u = np.zeros(self.dim * self.N)
        tau = np.zeros(self.N)
        q = np.zeros(self.dim * self.N)
        _load().orc_get_moments(self._h, _dp(rho), _dp(u), _dp(tau), _dp(q))
        return (rho.reshape(self.shape), u.reshape((self.dim,) + self.shape),
                tau.reshape(self.shape), q.reshape((self.dim,) + self.shape))

    def phi(self):
        p = np.zeros(2 * self.dim * self.N)
        _load().orc_get_phi(self._h, _dp(p))
        return p.reshape((self.dim, 2) + self.shape)

    def set_phi(self, phi):
        p = np.ascontiguousarray(phi, np.float64).reshape(-1)
        _load().orc_set_phi(self._h, _dp(p))

    def flux(self):
        gp = ctypes.c_double()
        kk = ctypes.c_double()
        sec = np.zeros(self.n[0])
        _load().orc_get_flux(self._h, ctypes.byref(gp), ctypes.byref(kk), _dp(sec))
        return gp.value, kk.value, sec

    def velocities(self):
        v = np.zeros(self.dim * self.K)
        w = np.zeros(self.K)
        _load().orc_get_velocities(self._h, _dp(v), _dp(w))
        return v.reshape(self.dim, self.K), w

    def apply_advection(self, k, field):
        f = np.ascontiguousarray(field, np.float64).reshape(-1)
        out = np.zeros(self.N)
        _load().orc_apply_advection(self._h, int(k), _dp(f), _dp(out))
        return out.reshape(self.shape)

    def collision(self, h):
        hh = np.ascontiguousarray(h, np.float64).reshape(-1)
        out = np.zeros(self.K)
        _load().orc_collision(self._h, _dp(hh), _dp(out))
        return out

    def set_boundary_field(self, f):
        ff = np.ascontiguousarray(f, np.float64).reshape(-1)
        _load().orc_set_boundary_field(self._h, _dp(ff))
