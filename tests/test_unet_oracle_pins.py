"""Pins of the CPU reference of the warm-start network (oracle/unet_oracle.py)
against facts it does not compute itself: bfloat16 rounding of hand-derived
values, brute-force convolution loops, exact shift equivariance along the
periodic axis, finite differences of the loss, closed forms of the target
normalisation, the loss and the first Adam step."""
import numpy as np
import pytest
import torch

from oracle import unet_oracle as U


def test_bf16_rounding_known_values():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even significand (1).
    # 1 + 3 2^-8 lies halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even).
    vals = [1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -(1 + 2 ** -8 + 2 ** -20), 3.0, 0.0,
            2.0 ** -130, 1.9921875, 1.99609375, 1.998046875]
    # 1.9921875 = 1 + 127/128 is exact; 2 - 2^-8 is the tie between it (odd) and 2 (even)
    want = [1.0, 1 + 2 ** -6, 1 + 2 ** -7, -(1 + 2 ** -7), 3.0, 0.0, 2.0 ** -130, 1.9921875, 2.0, 2.0]
    got = U.bf16_round(torch.tensor(vals, dtype=torch.float64)).tolist()
    assert got == want


def _conv_loops(x, w, b):
    """out[o, y, x] = b[o] + sum_{c, ky, kx} in[c, y + ky - k/2, (x + kx - k/2) mod W] w[o, c, ky, kx];
    rows outside 0..H-1 read 0."""
    C, H, W = x.shape
    O, _, k, _ = w.shape
    h = k // 2
    out = np.zeros((O, H, W))
    for o in range(O):
        for yy in range(H):
            for xx in range(W):
                s = b[o]
                for c in range(C):
                    for ky in range(k):
                        for kx in range(k):
                            y2 = yy + ky - h
                            if 0 <= y2 < H:
                                s += x[c, y2, (xx + kx - h) % W] * w[o, c, ky, kx]
                out[o, yy, xx] = s
    return out


@pytest.mark.parametrize("k", [3, 1])
def test_conv_matches_brute_force_loops(k):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 5, 6))
    w = rng.standard_normal((4, 3, k, k))
    b = rng.standard_normal(4)
    got = U.conv(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b))[0].numpy()
    np.testing.assert_allclose(got, _conv_loops(x, w, b), rtol=0, atol=1e-12)


def _random_case(seed, n=16, B=2):
    rng = np.random.default_rng(seed)
    solids = [(rng.random((n, n)) < 0.3).astype(np.uint8) for _ in range(B)]
    kns = [float(np.exp(rng.uniform(np.log(0.05), np.log(20)))) for _ in range(B)]
    p = rng.standard_normal(U.num_params()) * 0.05
    return rng, solids, kns, p


def test_network_is_exactly_shift_equivariant_along_x1_only():
    _, solids, kns, p = _random_case(1)
    x = U.make_input(solids, kns, bf16=False)
    y = U.forward(p, x, bf16=False)
    ys = U.forward(p, torch.roll(x, 8, dims=3), bf16=False)
    assert torch.equal(ys, torch.roll(y, 8, dims=3))  # circular padding along x1
    yv = U.forward(p, torch.roll(x, 8, dims=2), bf16=False)
    assert not torch.allclose(yv, torch.roll(y, 8, dims=2))  # zero padding along x2


def test_loss_gradient_matches_finite_differences():
    rng, solids, kns, p = _random_case(2, n=8)
    targets, ws = [], []
    for s, kn in zip(solids, kns):
        t, w = U.make_targets(s, rng.standard_normal(s.shape), rng.standard_normal((2,) + s.shape) * 0.1, kn)
        targets.append(t)
        ws.append(w)
    _, g = U.loss_and_grads(p, solids, kns, targets, ws, bf16=False)
    x = U.make_input(solids, kns, bf16=False)

    def loss_at(q):
        return float(U.loss_fn(U.forward(q, x, bf16=False), targets, solids, ws))

    # one weight and one bias of every layer, at positions that a transposed
    # layout would confuse
    idx, o = [], 0
    for cout, taps, cin in U.ARCH:
        n = cout * taps * cin
        idx += [o + (cout - 1) * taps * cin + (taps // 2) * cin + 1, o + n + cout - 1]
        o += n + cout
    for i in idx:
        h = 1e-5
        qp, qm = p.copy(), p.copy()
        qp[i] += h
        qm[i] -= h
        fd = (loss_at(qp) - loss_at(qm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_targets_closed_form_and_round_trip():
    n = 16
    solid = np.zeros((n, 2 * n), np.uint8)
    solid[3:6, 4:9] = 1
    x1 = (np.arange(2 * n) + 0.5) / (2 * n)
    J, kn, c = 2.0, 0.7, 0.3
    rho = np.broadcast_to(-J * (x1 - 0.5) + c, solid.shape)
    u = np.stack([np.full(solid.shape, 0.02), np.full(solid.shape, -0.01)])
    t, w = U.make_targets(solid, rho, u, kn, J)
    g = 2 * n / (256.0 * J)
    K = kn * 2 * n / 256.0
    sig = 10 * K / (1 + 10 * K)
    fl = solid == 0
    assert np.allclose(t[0][fl], 0.0, atol=1e-15)
    assert np.allclose(t[1][fl], 10 * sig * 0.02 * g) and np.allclose(t[2][fl], -10 * sig * 0.01 * g)
    assert np.all(t[:, ~fl] == 0) and w == 1.0 / (3 * fl.sum())
    r2, u2 = U.fields_from_output(t, solid, kn, J)
    assert np.allclose(r2[fl], (rho - c)[fl], atol=1e-14) and np.allclose(u2[:, fl], u[:, fl], atol=1e-15)


def test_loss_closed_form():
    rng, solids, kns, _ = _random_case(3)
    pred = torch.zeros((2, 3) + solids[0].shape, dtype=torch.float64)
    targets = [np.full((3,) + s.shape, -1.0) for s in solids]
    ws = [1.0 / (3 * (s == 0).sum()) for s in solids]
    assert abs(float(U.loss_fn(pred, targets, solids, ws)) - 1.0) < 1e-14


def test_first_adam_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    p = np.array([1.0, 1.0, 1.0])
    q, m, v = U.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # after one step the bias-corrected moments are g and g^2
    np.testing.assert_allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-13)
