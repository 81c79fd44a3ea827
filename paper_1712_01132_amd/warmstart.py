"""Thin Python binding of the warm-start network (include/poredvm_unet.h).

The network maps a solid mask and Kn to initial density and velocity fields
for the iteration. Every layer, the loss, the backward pass and Adam run in
the library's HIP kernels (bf16 matrix-core convolutions); this module only
marshals arguments, draws the seeded initial weights and stores trained
weights as a plain .npz file.
"""
import ctypes
import os

import numpy as np

from . import poredvm

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(_HERE, "weights", "warmstart_unet.npz")

EXPORTED = [
    "pdvm_unet_num_params", "pdvm_unet_create", "pdvm_unet_set_params", "pdvm_unet_get_params",
    "pdvm_unet_set_sample", "pdvm_unet_train_step", "pdvm_unet_get_grads", "pdvm_unet_forward",
    "pdvm_unet_predict", "pdvm_unet_time", "pdvm_unet_destroy", "pdvm_unet_last_error",
]

# (name, Cout, taps, Cin) in parameter order; mirrors the layer table of the library
LAYERS = [
    ("enc1a", 32, 9, 8), ("enc1b", 32, 9, 32), ("enc2a", 64, 9, 32), ("enc2b", 64, 9, 64),
    ("enc3a", 128, 9, 64), ("enc3b", 128, 9, 128), ("bott_a", 256, 9, 128), ("bott_b", 256, 9, 256),
    ("dec3a", 128, 9, 384), ("dec3b", 128, 9, 128), ("dec2a", 64, 9, 192), ("dec2b", 64, 9, 64),
    ("dec1a", 32, 9, 96), ("dec1b", 32, 9, 32), ("head", 3, 1, 32),
]


class PdvmUnetTiming(ctypes.Structure):
    _fields_ = [("forward_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("forward_flop", ctypes.c_double), ("step_flop", ctypes.c_double),
                ("mfma_ms_per_step", ctypes.c_double)]


_bound = False


def _lib():
    global _bound
    lib = poredvm.load()
    if _bound:
        return lib
    vp = ctypes.c_void_p
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    lib.pdvm_unet_num_params.restype = ctypes.c_int64
    lib.pdvm_unet_num_params.argtypes = []
    lib.pdvm_unet_create.argtypes = [ctypes.c_int32] * 4 + [vp, ctypes.POINTER(vp)]
    lib.pdvm_unet_set_params.argtypes = [vp, fp, ctypes.c_int64]
    lib.pdvm_unet_get_params.argtypes = [vp, fp, ctypes.c_int64]
    lib.pdvm_unet_get_grads.argtypes = [vp, fp, ctypes.c_int64]
    lib.pdvm_unet_set_sample.argtypes = [vp, ctypes.c_int32, u8, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.pdvm_unet_train_step.argtypes = [vp, ip, ctypes.c_int32, ctypes.c_float, ctypes.c_int32, dp]
    lib.pdvm_unet_forward.argtypes = [vp, ip, ctypes.c_int32, fp]
    lib.pdvm_unet_predict.argtypes = [vp, u8, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.pdvm_unet_time.argtypes = [vp, ip, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(PdvmUnetTiming)]
    lib.pdvm_unet_destroy.restype = None
    lib.pdvm_unet_destroy.argtypes = [vp]
    lib.pdvm_unet_last_error.restype = ctypes.c_char_p
    lib.pdvm_unet_last_error.argtypes = [vp]
    _bound = True
    return lib


def num_params():
    return int(_lib().pdvm_unet_num_params())


def init_params(seed):
    """He-normal weights (numpy PCG64, seeded), zero biases; the six zero
    input channels of the first layer get zero weights."""
    rng = np.random.default_rng(seed)
    out = []
    for name, cout, taps, cin in LAYERS:
        w = rng.standard_normal((cout, taps, cin)) * np.sqrt(2.0 / (taps * cin))
        if name == "enc1a":
            w[:, :, 2:] = 0.0
        if name == "head":
            w *= 0.1
        out += [w.ravel(), np.zeros(cout)]
    p = np.concatenate(out).astype(np.float32)
    return p


def split_params(p):
    """Parameter vector -> list of (weights [Cout][taps][Cin], bias [Cout])."""
    out, o = [], 0
    for _, cout, taps, cin in LAYERS:
        n = cout * taps * cin
        out.append((p[o:o + n].reshape(cout, taps, cin), p[o + n:o + n + cout]))
        o += n + cout
    assert o == len(p)
    return out


def _f(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Net:
    """A network instance for n2 x n1 images (multiples of 8)."""

    def __init__(self, n1, n2, batch_max=8, dataset_max=0, stream=None):
        import torch
        lib = _lib()
        self.n1, self.n2 = int(n1), int(n2)
        self._stream = stream or torch.cuda.Stream()
        h = ctypes.c_void_p()
        rc = lib.pdvm_unet_create(self.n1, self.n2, int(batch_max), int(dataset_max),
                                  ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise poredvm.PdvmError(rc, lib.pdvm_unet_last_error(None).decode())
        self._h = h
        self.np = num_params()

    def _check(self, rc):
        if rc != 0:
            raise poredvm.PdvmError(rc, _lib().pdvm_unet_last_error(self._h).decode())

    def close(self):
        if self._h:
            _lib().pdvm_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(_lib().pdvm_unet_set_params(self._h, _f(p), len(p)))

    def params(self):
        p = np.zeros(self.np, np.float32)
        self._check(_lib().pdvm_unet_get_params(self._h, _f(p), len(p)))
        return p

    def grads(self):
        g = np.zeros(self.np, np.float32)
        self._check(_lib().pdvm_unet_get_grads(self._h, _f(g), len(g)))
        return g

    def set_sample(self, slot, solid, kn, rho, u, jump=1.0):
        s = np.ascontiguousarray(solid, dtype=np.uint8)
        r = np.ascontiguousarray(rho, dtype=np.float64)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        assert s.shape == (self.n2, self.n1) and r.shape == s.shape and uu.shape == (2,) + s.shape
        self._check(_lib().pdvm_unet_set_sample(self._h, int(slot), s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                                float(kn), float(jump), _d(r), _d(uu)))

    def train_step(self, slots, lr=1e-3, update=True):
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        loss = ctypes.c_double()
        self._check(_lib().pdvm_unet_train_step(self._h, sl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                len(sl), float(lr), int(bool(update)), ctypes.byref(loss)))
        return loss.value

    def forward(self, slots):
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        out = np.zeros((len(sl), self.n2, self.n1, 4), np.float32)
        self._check(_lib().pdvm_unet_forward(self._h, sl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             len(sl), _f(out)))
        return out

    def predict(self, solid, kn, jump=1.0):
        """Warm-start fields (rho, u) for one mask of this instance's size."""
        s = np.ascontiguousarray(solid, dtype=np.uint8)
        assert s.shape == (self.n2, self.n1)
        rho = np.zeros(s.shape)
        u = np.zeros((2,) + s.shape)
        self._check(_lib().pdvm_unet_predict(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                             float(kn), float(jump), _d(rho), _d(u)))
        return rho, u

    def time(self, slots, reps=5):
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        t = PdvmUnetTiming()
        self._check(_lib().pdvm_unet_time(self._h, sl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          len(sl), int(reps), ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in PdvmUnetTiming._fields_}


def weight_mask():
    """True at the convolution weights of the parameter vector, False at the biases."""
    out = []
    for _, cout, taps, cin in LAYERS:
        out += [np.ones(cout * taps * cin, bool), np.zeros(cout, bool)]
    return np.concatenate(out)


def bf16_weights(p):
    """The parameter vector with its convolution weights rounded to bfloat16
    (nearest, ties to even), the values the network computes with; biases are
    FP32 in the network and stay exact."""
    p = np.array(p, np.float32)
    u = p.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    w = weight_mask()
    p[w] = r[w]
    return p


def save_weights(p, path=WEIGHTS_PATH, **meta):
    """Store trained parameters (weights as their bfloat16 values, which loses
    nothing the network uses) in a compressed .npz with JSON metadata."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez_compressed(path, params=bf16_weights(p), **{k: np.asarray(v) for k, v in meta.items()})


def load_weights(path=WEIGHTS_PATH):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), {k: z[k] for k in z.files if k != "params"}


def ramp_start(mask, jump=1.0):
    """The pressure ramp that the jump condition imposes on average (Eq.
    periodic_BC): rho = jump (1/2 - x1) at the fluid nodes (x1 at the node,
    L = 1), u = 0. It needs no training and already removes the slowest part
    of the start-up from rest, so it is the baseline a learned start has to
    beat."""
    mask = np.asarray(mask)
    n1 = mask.shape[-1]
    x1 = (np.arange(n1) + 0.5) / n1
    rho = np.broadcast_to(jump * (0.5 - x1), mask.shape).copy()
    rho[mask != 0] = 0.0
    return rho, np.zeros((mask.ndim,) + mask.shape)


def judged_start(mask, nv, kn, start, trial=50, precision="fp32", jump=1.0, tile=None, grid=None, fallback="ramp"):
    """The iteration judges a guessed start: `trial` iterations from the start
    fields (rho, u) and `trial` iterations from the fallback (the pressure
    ramp of `ramp_start`, or rest with fallback=None), each in its own solver.
    The one whose velocity field still changes less per iteration
    (r * max|u|, the absolute change at the last trial iteration) goes on and
    is returned; the other is closed. Returns (solver, used_start, change_start,
    change_fallback)."""
    kw = dict(precision=precision, jump=jump, tile=tile)
    if grid is not None:
        kw["grid"] = grid

    def run(init):
        s = poredvm.Solver(mask, nv, kn, **kw)
        if init is not None:
            s.set_initial(*init)
        r = s.iterate(trial)["r"]
        _, u = s.moments(diagnostics=False)
        return s, r * float(np.abs(u).max())

    a, da = run(start)
    b, db = run(ramp_start(mask, jump) if fallback == "ramp" else None)
    if da < db:
        b.close()
        return a, True, da, db
    a.close()
    return b, False, da, db
