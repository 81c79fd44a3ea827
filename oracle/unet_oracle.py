"""CPU reference of the warm-start network: test infrastructure only.

Only tests/, the smoke check and the benchmark's CPU baseline use this
module; the product never imports it. It shares no code with the library.

Plain PyTorch CPU operations in float64 implement the network contract of the
library: input features, target normalisation, the U-Net (4 levels, 32/64/128/256
channels, two 3x3 convolutions with ReLU per level, 2x2 max pooling, nearest
upsampling with skip concatenation, 1x1 head), the masked squared-error loss,
its gradients and one Adam step.

Padding is circular along x1 (the periodic flow axis, the last tensor axis)
and zero along x2. The library computes with bfloat16 operands and FP32
accumulation. With `bf16=True` this reference rounds to bfloat16 (nearest,
ties to even) at the same places: the network input, every weight, every
stored activation, and the gradient at every convolution output. It keeps
every sum exact in float64, so only accumulation order separates the two
sides.
"""
import math

import numpy as np
import torch
import torch.nn.functional as F

# (Cout, taps, Cin) per layer, in parameter order
ARCH = [(32, 9, 8), (32, 9, 32), (64, 9, 32), (64, 9, 64), (128, 9, 64), (128, 9, 128),
        (256, 9, 128), (256, 9, 256), (128, 9, 384), (128, 9, 128), (64, 9, 192), (64, 9, 64),
        (32, 9, 96), (32, 9, 32), (3, 1, 32)]
U_SCALE, KN_KNEE, REF_LEN = 10.0, 10.0, 256.0


def num_params():
    return sum(c * t * i + c for c, t, i in ARCH)


def bf16_round(x):
    """Nearest bfloat16 value (8 significant bits, ties to even) of float64
    values, returned as float64."""
    x = torch.as_tensor(x, dtype=torch.float64)
    m, e = torch.frexp(x)                  # x = m 2^e, 0.5 <= |m| < 1
    q = torch.round(torch.ldexp(m, torch.full_like(e, 8)))  # 8 significant bits, half to even
    return torch.ldexp(q, e - 8)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; rounds the incoming gradient to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return bf16_round(g)


class _RoundValue(torch.autograd.Function):
    """Rounds the value to bfloat16; passes the gradient through."""

    @staticmethod
    def forward(ctx, x):
        return bf16_round(x)

    @staticmethod
    def backward(ctx, g):
        return g


def unpack(params):
    """Logical parameter vector -> [(weight [Cout, Cin, kh, kw], bias [Cout])] in float64."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    out, o = [], 0
    for cout, taps, cin in ARCH:
        n = cout * taps * cin
        w = p[o:o + n].reshape(cout, taps, cin)
        k = 3 if taps == 9 else 1
        w = w.reshape(cout, k, k, cin).permute(0, 3, 1, 2).contiguous()
        out.append((w, p[o + n:o + n + cout].clone()))
        o += n + cout
    return out


def conv(x, w, b):
    """Convolution (cross-correlation) with 'same' output size: circular
    padding along the last axis (x1), zero padding along x2."""
    k = w.shape[-1]
    if k == 3:
        x = F.pad(x, (1, 1, 0, 0), mode="circular")
        x = F.pad(x, (0, 0, 1, 1))
    return F.conv2d(x, w, b)


def make_input(solids, kns, bf16=True):
    """[B, 8, n2, n1]: solid (0/1), f = ln(Kn n1 / 256) / 3, six zero channels."""
    solids = [np.asarray(s) for s in solids]
    n2, n1 = solids[0].shape
    x = torch.zeros((len(solids), 8, n2, n1), dtype=torch.float64)
    for b, (s, kn) in enumerate(zip(solids, kns)):
        x[b, 0] = torch.as_tensor((s != 0).astype(np.float64))
        x[b, 1] = float(np.float32(math.log(kn * n1 / REF_LEN) / 3.0))
    return bf16_round(x) if bf16 else x


def _sigma(kn256):
    a = KN_KNEE * kn256
    return a / (1.0 + a)


def make_targets(solid, rho, u, kn, jump=1.0):
    """Normalised targets [3, n2, n1] and the sample weight 1 / (3 n_fluid):
    t0 = (rho + J (x1 - 1/2) - its fluid mean) N1 / (256 J); t_j = U sigma u_j N1 / (256 J)."""
    solid = np.asarray(solid) != 0
    n2, n1 = solid.shape
    x1 = (np.arange(n1) + 0.5) / n1
    pr = np.asarray(rho, np.float64) + jump * (x1[None, :] - 0.5)
    fluid = ~solid
    mean = pr[fluid].mean()
    g = n1 / (REF_LEN * jump)
    us = U_SCALE * _sigma(kn * n1 / REF_LEN) * g
    t = np.zeros((3, n2, n1))
    t[0][fluid] = (pr[fluid] - mean) * g
    t[1][fluid] = np.asarray(u)[0][fluid] * us
    t[2][fluid] = np.asarray(u)[1][fluid] * us
    return t, 1.0 / (3.0 * fluid.sum())


def fields_from_output(out, solid, kn, jump=1.0):
    """Inverse of the target normalisation (fluid mean density 0): out [3, n2, n1]."""
    solid = np.asarray(solid) != 0
    n2, n1 = solid.shape
    x1 = (np.arange(n1) + 0.5) / n1
    g = n1 / (REF_LEN * jump)
    us = U_SCALE * _sigma(kn * n1 / REF_LEN) * g
    rho = np.where(solid, 0.0, np.asarray(out[0]) / g - jump * (x1[None, :] - 0.5))
    u = np.stack([np.where(solid, 0.0, np.asarray(out[j]) / us) for j in (1, 2)])
    return rho, u


def _net(layers, x, bf16):
    rv = _RoundValue.apply if bf16 else (lambda t: t)
    rg = _RoundGrad.apply if bf16 else (lambda t: t)

    def block(t, i):
        w, b = layers[i]
        return rv(F.relu(rg(conv(t, rv(w), b))))

    e1 = block(block(x, 0), 1)
    e2 = block(block(F.max_pool2d(e1, 2), 2), 3)
    e3 = block(block(F.max_pool2d(e2, 2), 4), 5)
    bt = block(block(F.max_pool2d(e3, 2), 6), 7)

    def up(t):
        return F.interpolate(t, scale_factor=2, mode="nearest")

    d3 = block(block(torch.cat([up(bt), e3], 1), 8), 9)
    d2 = block(block(torch.cat([up(d3), e2], 1), 10), 11)
    d1 = block(block(torch.cat([up(d2), e1], 1), 12), 13)
    w, b = layers[14]
    return rg(conv(d1, rv(w), b))


def forward(params, x, bf16=True):
    """U-Net output [B, 3, n2, n1] (float64) for the input x of make_input."""
    with torch.no_grad():
        return _net(unpack(params), x, bf16)


def loss_fn(pred, targets, solids, wsamp):
    """mean over the batch of wsamp_b * sum over fluid voxels and outputs of (pred - target)^2."""
    B = pred.shape[0]
    total = 0.0
    for b in range(B):
        fluid = torch.as_tensor(np.asarray(solids[b]) == 0)
        d = (pred[b] - torch.as_tensor(targets[b])) * fluid
        total = total + wsamp[b] * (d * d).sum()
    return total / B


def loss_and_grads(params, solids, kns, targets, wsamp, bf16=True):
    """Loss and its gradient with respect to the logical parameter vector."""
    layers = unpack(params)
    leaves = []
    for w, b in layers:
        w.requires_grad_(True)
        b.requires_grad_(True)
        leaves += [w, b]
    x = make_input(solids, kns, bf16)
    pred = _net(layers, x, bf16)
    loss = loss_fn(pred, targets, solids, wsamp)
    loss.backward()
    g = []
    for (cout, taps, cin), (w, b) in zip(ARCH, layers):
        k = 3 if taps == 9 else 1
        gw = w.grad.permute(0, 2, 3, 1).reshape(cout, taps * cin)
        g += [gw.reshape(-1), b.grad]
    return float(loss.detach()), torch.cat(g).numpy()


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments), float64; returns (params, m, v)."""
    p = np.asarray(params, np.float64)
    g = np.asarray(grads, np.float64)
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
