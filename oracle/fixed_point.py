"""Direct solve of the discretised fixed point on tiny grids (bordered LU).

TEST INFRASTRUCTURE ONLY. An independent check of the iterative oracle: it
assembles, from the paper's definitions and in its own code, the linear system
that a converged iteration satisfies, and solves it with a sparse direct LU
(scipy's SuperLU). It shares no code with the C++ oracle or the GPU path.

At convergence every lagged quantity equals its current value, so for each
fluid node x and discrete velocity v_k (Sec. 2.3, Eq. Discretised_linearised_
Boltzmann_equations; boundary values from Sec. 2.1):

    den h(x,k) - nu [rho(x) + 2 u(x).v_k] - sum_j a_j (c1 Y1_j + c2 Y2_j) = 0,

with a_j = |v_jk|/dx, (c1, c2) = (2, -1/2) and den = nu + sum 1.5 a_j for the
second-order stencil, (c1) = (1) and a_j in place of 1.5 a_j for the first-order
one (used when an upstream image is solid, see `stencil_rule`). Y are upstream values:
the unknown h at a fluid node inside the domain; h at the periodic / mirror
image plus the pressure jump at a ghost node; the wall density
Phi_j^-s(x_f)/D_j (+ jump) at a solid node, with Phi_j^+-(x) =
sum_{+-v_j>0} W |v_j| h(x, .) (Eq. wall_density).

Constants are in the null space (a uniform shift of h is an exact solution of
the homogeneous system), and the right-hand side built from the jump need not
be in the range. The iteration then converges to h* + l delta (a uniform drift
of delta per iteration). Writing h^(l+1) = h* + (l+1) delta for the values the
sweep takes from the current iteration and h* + l delta for the lagged ones
gives M h* + delta m = b, where m = den - (sum of the coefficients on current
fluid upstream values). The gauge g^T h* = mean over fluid nodes of rho = 0
closes the system:

    [[M, m], [g^T, 0]] [h*; delta] = [b; 0].
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import quadrature


def _velocity_table(grid, dim):
    # tensor product, k = a + n1 (b + n2 c); same role as the paper's v^(k), W_k
    xs = [np.asarray(g[0], float) for g in grid]
    ws = [np.asarray(g[1], float) for g in grid]
    while len(xs) < 3:
        xs.append(np.zeros(1))
        ws.append(np.ones(1))
    n = [len(x) for x in xs]
    K = n[0] * n[1] * n[2]
    v = np.zeros((3, K))
    W = np.zeros(K)
    mirror = np.zeros((3, K), int)
    for c in range(n[2]):
        for b in range(n[1]):
            for a in range(n[0]):
                k = a + n[0] * (b + n[1] * c)
                v[:, k] = (xs[0][a], xs[1][b], xs[2][c])
                W[k] = ws[0][a] * ws[1][b] * ws[2][c]
                mirror[0, k] = (n[0] - 1 - a) + n[0] * (b + n[1] * c)
                mirror[1, k] = a + n[0] * ((n[1] - 1 - b) + n[1] * c)
                mirror[2, k] = a + n[0] * (b + n[1] * (n[2] - 1 - c))
    return v[:dim], W, mirror[:dim]


def solve_fixed_point(solid, nv, kn, jump=1.0, lateral_periodic=False, grid=None, stencil_rule=1):
    """Return dict with rho (gauge mean 0 over fluid), u (dim, ...), delta, h.

    solid: (N2, N1) or (N3, N2, N1) uint8 mask, 1 = solid. stencil_rule 1: the
    first-order stencil is used when either upstream image is solid; 0: only
    when the first one is (a solid second image then enters the second-order
    stencil with its wall value)."""
    solid = np.asarray(solid, np.uint8)
    dim = solid.ndim
    shape = solid.shape
    n = list(reversed(shape)) + [1] * (3 - dim)   # [N1, N2, N3]
    if grid is None:
        grid = [quadrature.full_line_grid(int(m)) for m in nv]
    v, W, mirror = _velocity_table(grid, dim)
    K = len(W)
    D = np.array([np.sum(W * v[j] * (v[j] > 0)) for j in range(dim)])
    nu = 0.0 if np.isinf(kn) else np.sqrt(np.pi) / (2.0 * kn)
    inv_dx = float(n[0])
    flat = solid.reshape(-1)

    def cell(x):
        return x[0] + n[0] * (x[1] + n[1] * x[2])

    fluid_cells = [c for c in range(flat.size) if not flat[c]]
    fidx = -np.ones(flat.size, int)
    for i, c in enumerate(fluid_cells):
        fidx[c] = i
    nf = len(fluid_cells)
    nun = nf * K

    def unk(c, k):
        return fidx[c] * K + k

    def image(j, cj):
        """(real coordinate, mirrored?, jump multiple) of an outside coordinate."""
        if j == 0:
            return (cj + n[0], False, 1) if cj < 0 else (cj - n[0], False, -1)
        if lateral_periodic:
            return cj % n[j], False, 0
        return (-cj - 1 if cj < 0 else 2 * n[j] - 1 - cj), True, 0

    def resolve(y, j):
        """Real node, mirrored flag and jump multiple of global node y."""
        yr = list(y)
        if 0 <= y[j] < n[j]:
            return yr, False, 0, False
        r, mir, jm = image(j, y[j])
        yr[j] = r
        return yr, mir, jm, True

    rows, cols, vals = [], [], []
    b = np.zeros(nun + 1)
    mcol = np.zeros(nun)

    def add(r, c, val):
        rows.append(r)
        cols.append(c)
        vals.append(val)

    for c in fluid_cells:
        x = [c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]
        for k in range(K):
            r = unk(c, k)
            den = nu
            cur = 0.0
            # source nu [rho + 2 u.v_k] in terms of h(x, .)
            for kk in range(K):
                coef = W[kk] * (1.0 + 2.0 * sum(v[j, kk] * v[j, k] for j in range(dim)))
                add(r, unk(c, kk), -nu * coef)
            for j in range(dim):
                s = 1 if v[j, k] > 0 else -1
                a = abs(v[j, k]) * inv_dx

                def upstream(m, weight):
                    """Add weight * Y_m (moved to the left side); returns
                    (is_solid, is_current_fluid)."""
                    y = list(x)
                    y[j] -= m * s
                    yr, mir, jm, ghost = resolve(y, j)
                    cy = cell(yr)
                    if flat[cy]:
                        f = list(y)
                        f[j] += s
                        fr, fmir, fjm, _ = resolve(f, j)
                        cf = cell(fr)
                        want_pos = (s < 0) != fmir   # incoming half at the wall
                        for kk in range(K):
                            if (v[j, kk] > 0) == want_pos:
                                add(r, unk(cf, kk), -weight * W[kk] * abs(v[j, kk]) / D[j])
                        b[r] += weight * fjm * jump
                        return True, False
                    kk = mirror[j, k] if mir else k
                    add(r, unk(cy, kk), -weight)
                    b[r] += weight * jm * jump
                    return False, not ghost

                # the upstream images decide the order
                y = list(x)
                y[j] -= s
                yr, _, _, _ = resolve(y, j)
                y1_solid = bool(flat[cell(yr)])
                y2_solid = False
                if not y1_solid:
                    y = list(x)
                    y[j] -= 2 * s
                    yr, _, _, _ = resolve(y, j)
                    y2_solid = bool(flat[cell(yr)])
                if y1_solid or (stencil_rule == 1 and y2_solid):
                    den += a
                    _, c1cur = upstream(1, a)
                    cur += a if c1cur else 0.0
                else:
                    den += 1.5 * a
                    _, c1cur = upstream(1, 2.0 * a)
                    _, c2cur = upstream(2, -0.5 * a)
                    cur += (2.0 * a if c1cur else 0.0) + (-0.5 * a if c2cur else 0.0)
            add(r, r, den)
            mcol[r] = den - cur
    # drift column and gauge row
    for r in range(nun):
        if mcol[r] != 0.0:
            add(r, nun, mcol[r])
    for c in fluid_cells:
        for k in range(K):
            add(nun, unk(c, k), W[k] / nf)
    A = sp.csc_matrix((vals, (rows, cols)), shape=(nun + 1, nun + 1))
    sol = spla.spsolve(A, b)
    h = sol[:nun].reshape(nf, K)
    delta = sol[nun]
    rho = np.zeros(flat.size)
    u = np.zeros((dim, flat.size))
    for i, c in enumerate(fluid_cells):
        rho[c] = np.dot(W, h[i])
        for j in range(dim):
            u[j, c] = np.dot(W * v[j], h[i])
    return {"rho": rho.reshape(shape), "u": u.reshape((dim,) + shape), "delta": delta,
            "h": h, "fluid_cells": np.array(fluid_cells)}
