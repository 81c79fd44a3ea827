"""Half-range Gauss-Hermite velocity grids, computed in high precision.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

The paper builds its Cartesian velocity grid from half-range Gauss-Hermite
quadrature (Sec. 2.2, citing Gautschi's ORTHPOL). The rule for the weight
exp(-x^2) on [0, inf) is defined here the plain way:

  1. the moments mu_m = int_0^inf x^m exp(-x^2) dx = Gamma((m+1)/2) / 2;
  2. the recurrence coefficients of the monic orthogonal polynomials from those
     moments by the Chebyshev algorithm (Gautschi, "Orthogonal polynomials:
     computation and approximation", Sec. 2.1.7);
  3. nodes and weights from the Jacobi matrix (Golub-Welsch): nodes are its
     eigenvalues, weights mu_0 times the squared first eigenvector components.

Everything runs in mpmath at 150 significant digits and is rounded to float64
at the end. The full-line 1D grid mirrors the half-range nodes to both signs and
normalises the weights by sqrt(pi), so that the 1D weights sum to one and absorb
the equilibrium factor exp(-x^2)/sqrt(pi) (Sec. 2.1, Eq. perturbed_quantities).
"""
from functools import lru_cache

import mpmath
import numpy as np

_DPS = 150


def _moments(count):
    return [mpmath.gamma(mpmath.mpf(m + 1) / 2) / 2 for m in range(count)]


def _chebyshev(n):
    """Recurrence coefficients alpha_0..alpha_{n-1}, beta_0..beta_{n-1}."""
    mu = _moments(2 * n)
    sig_prev = [mpmath.mpf(0)] * (2 * n)  # sigma_{k-2}
    sig = list(mu)                       # sigma_{k-1}
    alpha = [mu[1] / mu[0]]
    beta = [mu[0]]
    for k in range(1, n):
        new = [mpmath.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            new[l] = sig[l + 1] - alpha[k - 1] * sig[l] - beta[k - 1] * sig_prev[l]
        alpha.append(new[k + 1] / new[k] - sig[k] / sig[k - 1])
        beta.append(new[k] / sig[k - 1])
        sig_prev, sig = sig, new
    return alpha, beta


@lru_cache(maxsize=None)
def halfrange_gh_mp(n):
    """n-point half-range Gauss-Hermite rule as mpmath numbers (nodes ascending)."""
    if n < 1:
        raise ValueError("need at least one node")
    with mpmath.workdps(_DPS):
        alpha, beta = _chebyshev(n)
        jac = mpmath.matrix(n, n)
        for i in range(n):
            jac[i, i] = alpha[i]
            if i + 1 < n:
                off = mpmath.sqrt(beta[i + 1])
                jac[i, i + 1] = off
                jac[i + 1, i] = off
        evals, evecs = mpmath.eigsy(jac)
        pairs = sorted((evals[i], beta[0] * evecs[0, i] ** 2) for i in range(n))
        return tuple(p[0] for p in pairs), tuple(p[1] for p in pairs)


def halfrange_gh(n):
    """float64 nodes and (unnormalised) weights of the n-point half-range rule."""
    x, w = halfrange_gh_mp(n)
    return np.array([float(v) for v in x]), np.array([float(v) for v in w])


def full_line_grid(n_total):
    """1D grid of n_total (even) nodes: the n_total/2-point half-range rule
    mirrored to both signs, weights normalised so that they sum to one.

    Returns (nodes ascending, weights)."""
    if n_total < 2 or n_total % 2:
        raise ValueError("the 1D velocity count must be even and >= 2")
    x, w = halfrange_gh_mp(n_total // 2)
    with mpmath.workdps(_DPS):
        sp = mpmath.sqrt(mpmath.pi)
        nodes = [-v for v in reversed(x)] + list(x)
        weights = [v / sp for v in reversed(w)] + [v / sp for v in w]
    return (np.array([float(v) for v in nodes]),
            np.array([float(v) for v in weights]))
