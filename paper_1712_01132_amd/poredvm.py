"""Thin Python binding of libporedvm (include/poredvm.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
libporedvm.so. PyTorch provides the device workspace (a uint8 tensor) and the
stream the library enqueues on. If the library is missing the binding raises;
there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libporedvm.so")

PDVM_OK, PDVM_NOT_CONVERGED = 0, 1
PDVM_E_INVAL, PDVM_E_NOMEM, PDVM_E_HIP = -1, -2, -3
PDVM_E_NONFINITE, PDVM_E_STATE, PDVM_E_UNSUPPORTED = -4, -5, -6
PDVM_FP64, PDVM_FP32 = 0, 1
PDVM_LATERAL_SPECULAR, PDVM_LATERAL_PERIODIC = 0, 1
PDVM_STOP_FIELD, PDVM_STOP_PAPER_ERR = 0, 1
SCHEDULES = {"auto": 0, "diagonals": 1, "rows": 2, "rows-agent": 3, "strips": 4, "queue": 5, "columns": 6}

_dp = ctypes.POINTER(ctypes.c_double)


class PdvmConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("solid", ctypes.POINTER(ctypes.c_uint8)),
        ("nv", ctypes.c_int32 * 3),
        ("vnode", _dp * 3),
        ("vweight", _dp * 3),
        ("kn", ctypes.c_double),
        ("jump", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("lateral_bc", ctypes.c_int32),
        ("tau_feedback", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("tile", ctypes.c_int32 * 3),
        ("stencil_rule", ctypes.c_int32),
        ("sweep_schedule", ctypes.c_int32),
        ("prandtl", ctypes.c_double),
        ("specular_fraction", ctypes.c_double),
    ]


class PdvmStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int64),
        ("total_iters", ctypes.c_int64),
        ("r", ctypes.c_double),
        ("err", ctypes.c_double),
        ("k", ctypes.c_double),
        ("gp", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("converged", ctypes.c_int32),
    ]


class PdvmTiming(ctypes.Structure):
    _fields_ = [
        ("sweep_ms_per_launch", ctypes.c_double),
        ("moments_ms_per_launch", ctypes.c_double),
        ("reduce_ms_per_launch", ctypes.c_double),
        ("sweep_ms_per_iter", ctypes.c_double),
        ("moments_ms_per_iter", ctypes.c_double),
        ("iter_ms", ctypes.c_double),
        ("sweep_launches_per_iter", ctypes.c_int32),
        ("sweep_bytes_per_iter", ctypes.c_double),
        ("moments_bytes_per_iter", ctypes.c_double),
        ("fluid_cells", ctypes.c_double),
        ("velocities", ctypes.c_double),
    ]


# every symbol include/poredvm.h declares
EXPORTED = [
    "pdvm_halfrange_gh", "pdvm_workspace_bytes", "pdvm_create", "pdvm_set_initial",
    "pdvm_iterate", "pdvm_get_moments", "pdvm_get_flux", "pdvm_get_state",
    "pdvm_set_state", "pdvm_time_kernels", "pdvm_destroy", "pdvm_last_error",
    "pdvm_batch_create", "pdvm_batch_size", "pdvm_batch_set_initial", "pdvm_batch_iterate",
    "pdvm_batch_get_moments", "pdvm_batch_get_flux", "pdvm_sweep_schedule", "pdvm_set_wait_limit",
    "pdvm_iterate_noalloc",
]

_lib = None


class PdvmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("poredvm error %d: %s" % (code, msg))
        self.code = code


def load():
    """Load libporedvm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libporedvm.so is not built (run __graft_entry__.build() or "
                           "python paper_1712_01132_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.pdvm_halfrange_gh.argtypes = [ctypes.c_int32, _dp, _dp]
    lib.pdvm_workspace_bytes.restype = ctypes.c_size_t
    lib.pdvm_workspace_bytes.argtypes = [ctypes.POINTER(PdvmConfig)]
    lib.pdvm_create.argtypes = [ctypes.POINTER(PdvmConfig), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.pdvm_set_initial.argtypes = [vp, _dp, _dp]
    lib.pdvm_iterate.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(PdvmStats)]
    lib.pdvm_iterate_noalloc.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                         ctypes.POINTER(PdvmStats)]
    lib.pdvm_get_moments.argtypes = [vp, _dp, _dp, _dp, _dp]
    lib.pdvm_get_flux.argtypes = [vp, _dp, _dp, _dp]
    lib.pdvm_get_state.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.pdvm_set_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.pdvm_time_kernels.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(PdvmTiming)]
    lib.pdvm_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(PdvmConfig), vp, ctypes.POINTER(vp)]
    lib.pdvm_batch_size.restype = ctypes.c_int32
    lib.pdvm_batch_size.argtypes = [vp]
    lib.pdvm_batch_set_initial.argtypes = [vp, ctypes.c_int32, _dp, _dp]
    lib.pdvm_batch_iterate.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                       ctypes.POINTER(PdvmStats)]
    lib.pdvm_batch_get_moments.argtypes = [vp, ctypes.c_int32, _dp, _dp, _dp, _dp]
    lib.pdvm_sweep_schedule.restype = ctypes.c_int32
    lib.pdvm_sweep_schedule.argtypes = [vp]
    lib.pdvm_batch_get_flux.argtypes = [vp, ctypes.c_int32, _dp, _dp, _dp]
    lib.pdvm_set_wait_limit.argtypes = [vp, ctypes.c_double]
    lib.pdvm_destroy.argtypes = [vp]
    lib.pdvm_last_error.restype = ctypes.c_char_p
    lib.pdvm_last_error.argtypes = [vp]
    _lib = lib
    return lib


def _err(handle=None):
    return load().pdvm_last_error(handle).decode(errors="replace")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def velocity_grid(n_total):
    """Half-range Gauss-Hermite 1D grid of n_total nodes (nodes, weights)."""
    x = np.zeros(n_total)
    w = np.zeros(n_total)
    rc = load().pdvm_halfrange_gh(int(n_total), _ptr(x), _ptr(w))
    if rc != PDVM_OK:
        raise PdvmError(rc, _err())
    return x, w


def make_config(solid, nv, kn, jump=1.0, precision="fp64", lateral="specular",
                tau_feedback=False, tile=None, check_every=16, grid=None, stencil_rule=1, schedule="auto",
                prandtl=None, accommodation=1.0):
    """Build a PdvmConfig; returns (config, keepalive) -- keep both alive.
    prandtl (with tau_feedback): Shakhov model with this Prandtl number.
    accommodation: Maxwell walls, the diffuse fraction alpha in (0, 1]."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    dim = solid.ndim
    if dim not in (2, 3):
        raise ValueError("the mask must be 2D or 3D")
    n = list(reversed(solid.shape))
    if grid is None:
        grid = [velocity_grid(int(m)) for m in nv]
    grid = [(np.ascontiguousarray(x, np.float64), np.ascontiguousarray(w, np.float64)) for x, w in grid]
    cfg = PdvmConfig()
    cfg.dim = dim
    for a in range(3):
        cfg.n[a] = n[a] if a < dim else 1
        cfg.nv[a] = len(grid[a][0]) if a < dim else 1
        cfg.tile[a] = int(tile[a]) if (tile is not None and a < dim) else 0
    cfg.solid = solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    for a in range(dim):
        cfg.vnode[a] = _ptr(grid[a][0])
        cfg.vweight[a] = _ptr(grid[a][1])
    cfg.kn = float(kn)
    cfg.jump = float(jump)
    cfg.precision = {"fp64": PDVM_FP64, "fp32": PDVM_FP32}[precision]
    cfg.lateral_bc = {"specular": PDVM_LATERAL_SPECULAR, "periodic": PDVM_LATERAL_PERIODIC}[lateral]
    cfg.tau_feedback = int(bool(tau_feedback))
    cfg.check_every = int(check_every)
    cfg.stencil_rule = int(stencil_rule)
    cfg.sweep_schedule = SCHEDULES[schedule]
    cfg.prandtl = 0.0 if prandtl is None else float(prandtl)
    cfg.specular_fraction = 1.0 - float(accommodation)
    return cfg, (solid, grid)


class Solver:
    """One porous-media problem on the current GPU.

    solid: uint8 mask (1 = solid), shape (N2, N1) or (N3, N2, N1), x1 fastest.
    nv: 1D velocity counts per axis; kn: Knudsen number (L = N1 voxels).
    tau_feedback: keep the temperature term of the source (2D: with the second
    reduced function psi); prandtl (with tau_feedback): Shakhov model;
    accommodation: Maxwell walls, the diffuse fraction alpha in (0, 1].
    """

    def __init__(self, solid, nv, kn, jump=1.0, precision="fp64", lateral="specular",
                 tau_feedback=False, tile=None, check_every=16, grid=None, device=None,
                 stencil_rule=1, schedule="auto", prandtl=None, accommodation=1.0):
        import torch

        lib = load()
        self.shape = np.asarray(solid).shape
        self.dim = len(self.shape)
        self.N = int(np.prod(self.shape))
        self.cfg, self._keep = make_config(solid, nv, kn, jump, precision, lateral,
                                           tau_feedback, tile, check_every, grid, stencil_rule, schedule,
                                           prandtl, accommodation)
        nbytes = lib.pdvm_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise PdvmError(PDVM_E_INVAL, _err())
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        h = ctypes.c_void_p()
        rc = lib.pdvm_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                             nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != PDVM_OK:
            raise PdvmError(rc, _err())
        self._h = h
        self.workspace_bytes = nbytes

    def _check(self, rc, ok=(PDVM_OK,)):
        if rc not in ok:
            raise PdvmError(rc, _err(self._h))
        return rc

    def close(self):
        if getattr(self, "_h", None):
            load().pdvm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_initial(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, np.float64).reshape(-1)
        uu = None if u is None else np.ascontiguousarray(u, np.float64).reshape(-1)
        self._check(load().pdvm_set_initial(self._h, _ptr(r), _ptr(uu)))

    def iterate(self, max_iters, tol=0.0, stop_mode="field"):
        st = PdvmStats()
        mode = {"field": PDVM_STOP_FIELD, "paper": PDVM_STOP_PAPER_ERR}[stop_mode]
        rc = self._check(load().pdvm_iterate(self._h, int(max_iters), float(tol), mode, ctypes.byref(st)),
                         ok=(PDVM_OK, PDVM_NOT_CONVERGED))
        return {"converged": rc == PDVM_OK, "iters": st.iters, "total_iters": st.total_iters,
                "r": st.r, "err": st.err, "k": st.k, "Gp": st.gp, "seconds": st.seconds}

    def iterate_noalloc(self, max_iters, tol=0.0, stop_mode="field"):
        """iterate() through pdvm_iterate_noalloc: no allocation, the kernels'
        scratch in the library's static per-GPU array."""
        st = PdvmStats()
        mode = {"field": PDVM_STOP_FIELD, "paper": PDVM_STOP_PAPER_ERR}[stop_mode]
        rc = self._check(load().pdvm_iterate_noalloc(self._h, int(max_iters), float(tol), mode, ctypes.byref(st)),
                         ok=(PDVM_OK, PDVM_NOT_CONVERGED))
        return {"converged": rc == PDVM_OK, "iters": st.iters, "total_iters": st.total_iters,
                "r": st.r, "err": st.err, "k": st.k, "Gp": st.gp, "seconds": st.seconds}

    def moments(self, diagnostics=True):
        rho = np.zeros(self.N)
        u = np.zeros(self.dim * self.N)
        tau = np.zeros(self.N) if diagnostics else None
        q = np.zeros(self.dim * self.N) if diagnostics else None
        self._check(load().pdvm_get_moments(self._h, _ptr(rho), _ptr(u), _ptr(tau), _ptr(q)))
        out = [rho.reshape(self.shape), u.reshape((self.dim,) + self.shape)]
        if diagnostics:
            out += [tau.reshape(self.shape), q.reshape((self.dim,) + self.shape)]
        return tuple(out)

    def flux(self):
        gp = ctypes.c_double()
        k = ctypes.c_double()
        sec = np.zeros(self.shape[-1])
        self._check(load().pdvm_get_flux(self._h, ctypes.byref(gp), ctypes.byref(k), _ptr(sec)))
        return gp.value, k.value, sec

    def get_state(self):
        n = ctypes.c_size_t(0)
        self._check(load().pdvm_get_state(self._h, None, ctypes.byref(n)))
        buf = (ctypes.c_char * n.value)()
        self._check(load().pdvm_get_state(self._h, buf, ctypes.byref(n)))
        return bytes(buf)

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(load().pdvm_set_state(self._h, buf, len(blob)))

    def time_kernels(self, iters=5):
        t = PdvmTiming()
        self._check(load().pdvm_time_kernels(self._h, int(iters), ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in PdvmTiming._fields_}

    @property
    def schedule(self):
        """"diagonals", "rows" (agent-scope), "rows-xcd" (XCD-local row pipeline), "strips" or
        "queue" (per-XCD tile queues)."""
        return {0: "diagonals", 1: "rows", 2: "rows-xcd", 3: "strips", 4: "queue", 5: "columns"}[load().pdvm_sweep_schedule(self._h)]

    def set_wait_limit(self, seconds):
        """Bound on each row-pipeline wait for the upstream row (default 2 s)."""
        self._check(load().pdvm_set_wait_limit(self._h, float(seconds)))


class Batch:
    """Many problems iterated together on the current GPU (one graph replay per
    iteration covers all of them; converged problems retire).

    problems: list of (solid mask, kn) pairs -- masks of any size, same dim.
    All problems share nv, precision, stencil rule and tau feedback.
    """

    def __init__(self, problems, nv, precision="fp32", jump=1.0, lateral="specular",
                 tile=None, check_every=16, grid=None, stencil_rule=1, device=None, schedule="auto"):
        import torch

        lib = load()
        if grid is None:
            grid = [velocity_grid(int(m)) for m in nv]
        self.shapes = [np.asarray(m).shape for m, _ in problems]
        self.kns = [float(k) for _, k in problems]
        cfgs = (PdvmConfig * len(problems))()
        self._keep = []
        for i, (m, kn) in enumerate(problems):
            c, keep = make_config(m, nv, kn, jump, precision, lateral, False, tile, check_every,
                                  grid, stencil_rule, schedule)
            cfgs[i] = c
            self._keep.append(keep)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        rc = lib.pdvm_batch_create(len(problems), cfgs, ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h))
        if rc != PDVM_OK:
            raise PdvmError(rc, _err())
        self._h = h
        self.n = len(problems)

    def _check(self, rc, ok=(PDVM_OK,)):
        if rc not in ok:
            raise PdvmError(rc, _err(self._h))
        return rc

    def close(self):
        if getattr(self, "_h", None):
            load().pdvm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_initial(self, i, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, np.float64).reshape(-1)
        uu = None if u is None else np.ascontiguousarray(u, np.float64).reshape(-1)
        self._check(load().pdvm_batch_set_initial(self._h, int(i), _ptr(r), _ptr(uu)))

    def iterate(self, max_iters, tol=0.0, stop_mode="field"):
        st = (PdvmStats * self.n)()
        mode = {"field": PDVM_STOP_FIELD, "paper": PDVM_STOP_PAPER_ERR}[stop_mode]
        self._check(load().pdvm_batch_iterate(self._h, int(max_iters), float(tol), mode, st),
                    ok=(PDVM_OK, PDVM_NOT_CONVERGED))
        return [{"converged": bool(x.converged), "iters": x.iters, "total_iters": x.total_iters,
                 "r": x.r, "err": x.err, "k": x.k, "Gp": x.gp, "seconds": x.seconds} for x in st]

    def moments(self, i, diagnostics=False):
        shape = self.shapes[i]
        N = int(np.prod(shape))
        dim = len(shape)
        rho = np.zeros(N)
        u = np.zeros(dim * N)
        tau = np.zeros(N) if diagnostics else None
        q = np.zeros(dim * N) if diagnostics else None
        self._check(load().pdvm_batch_get_moments(self._h, int(i), _ptr(rho), _ptr(u), _ptr(tau), _ptr(q)))
        out = [rho.reshape(shape), u.reshape((dim,) + shape)]
        if diagnostics:
            out += [tau.reshape(shape), q.reshape((dim,) + shape)]
        return tuple(out)

    @property
    def schedule(self):
        return {0: "diagonals", 1: "rows", 2: "rows-xcd", 3: "strips", 4: "queue", 5: "columns"}[load().pdvm_sweep_schedule(self._h)]

    def flux(self, i):
        gp = ctypes.c_double()
        k = ctypes.c_double()
        sec = np.zeros(self.shapes[i][-1])
        self._check(load().pdvm_batch_get_flux(self._h, int(i), ctypes.byref(gp), ctypes.byref(k), _ptr(sec)))
        return gp.value, k.value, sec

    def time_kernels(self, iters=5):
        t = PdvmTiming()
        self._check(load().pdvm_time_kernels(self._h, int(iters), ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in PdvmTiming._fields_}
