"""Seeded synthetic porous geometries (solid masks) for the pore-scale solver.

This module only draws and rasterises shapes; it holds none of the solver's
arithmetic, and both the GPU path and the CPU oracle take its masks as input.

Masks are uint8 arrays, 1 = solid, shaped (N2, N1) in 2D and (N3, N2, N1) in 3D,
so that x1 (the flow axis) is the fastest index. Cell (i, j[, l]) has its node
at the voxel centre. Random shapes are placed with numpy's PCG64 generator.

Percolation: the medium is periodic along x1 (pressure-jump periodic inlet and
outlet) and mirrored at the lateral faces, so a pore component carries flow only
if it winds around x1. Components that do not are filled with solid by
`fill_nonpercolating`; they would add undetermined constant modes to the
density field (Sec. 2.1 sets one density level per connected gas volume only
through the initial state).
"""
import numpy as np
from scipy import ndimage


def centred_disc(n=64, radius=None):
    """Periodic unit cell n x n with one solid disc at the centre.
    Solid iff (i + 1/2 - n/2)^2 + (j + 1/2 - n/2)^2 <= r^2, r = n/4 by default."""
    r = n / 4.0 if radius is None else float(radius)
    c = np.arange(n) + 0.5 - n / 2.0
    d2 = c[None, :] ** 2 + c[:, None] ** 2
    return (d2 <= r * r).astype(np.uint8)


def plane_channel(n1, n2):
    """Plane channel: solid rows j = 0 and j = n2-1, fluid between."""
    m = np.zeros((n2, n1), np.uint8)
    m[0, :] = 1
    m[-1, :] = 1
    return m


def sierpinski_carpet(level=3, size=540):
    """Level-`level` Sierpinski carpet rasterised on size x size pixels; the
    removed squares are solid (porosity (8/9)^level)."""
    m = np.zeros((size, size), np.uint8)
    idx = (np.arange(size) + 0.5) / size
    for lev in range(1, level + 1):
        cells = 3 ** lev
        d = np.floor(idx * cells).astype(int) % 3
        m |= ((d[:, None] == 1) & (d[None, :] == 1)).astype(np.uint8)
    return m


def cubic_sphere_quadrant(n1=200, n2=100, n3=100, porosity=0.75):
    """Quadrant of a simple-cubic sphere unit cell: x1 spans the whole period
    (n1 = one cell length), x2 and x3 one half each (the symmetry planes are the
    specular lateral faces). The sphere sits at the cell centre; its radius is
    set so that the solid fraction is 1 - porosity."""
    i = np.arange(n1) + 0.5 - n1 / 2.0
    j = np.arange(n2) + 0.5
    k = np.arange(n3) + 0.5
    d2 = i[None, None, :] ** 2 + j[None, :, None] ** 2 + k[:, None, None] ** 2
    target = (1.0 - porosity) * d2.size
    s = np.sort(d2.ravel())
    r2 = s[int(round(target)) - 1]
    return (d2 <= r2).astype(np.uint8)


def _label_periodic_x1(fluid, structure):
    """Label fluid components with x1 (last axis) periodic: returns labels on the
    domain and, for each label, whether it winds around x1."""
    n1 = fluid.shape[-1]
    doubled = np.concatenate([fluid, fluid], axis=-1)
    lab, nlab = ndimage.label(doubled, structure=structure)
    # union the labels across the seam x1 = 2 n1 - 1 -> 0 of the doubled domain
    parent = np.arange(nlab + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    left = lab[..., 0].ravel()
    right = lab[..., -1].ravel()
    for a, b in zip(left, right):
        if a and b:
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[ra] = rb
    roots = np.array([find(a) for a in range(nlab + 1)])
    lab = roots[lab]
    # a component winds around x1 iff its two copies in the doubled periodic
    # domain are one component
    first = lab[..., :n1]
    second = lab[..., n1:]
    winds = set(np.unique(first[(first > 0) & (first == second)]).tolist())
    return first, winds


def fill_nonpercolating(solid):
    """Fill every pore component that does not wind around x1 with solid.
    4-connectivity in 2D, 6-connectivity in 3D."""
    solid = np.asarray(solid, np.uint8)
    fluid = solid == 0
    structure = ndimage.generate_binary_structure(solid.ndim, 1)
    lab, winds = _label_periodic_x1(fluid, structure)
    keep = np.isin(lab, list(winds)) if winds else np.zeros_like(fluid)
    return np.where(keep, 0, 1).astype(np.uint8)


def percolates(solid):
    """True if at least one pore component winds around x1."""
    solid = np.asarray(solid, np.uint8)
    structure = ndimage.generate_binary_structure(solid.ndim, 1)
    _, winds = _label_periodic_x1(solid == 0, structure)
    return len(winds) > 0


def porosity(solid):
    return float(1.0 - np.asarray(solid).mean())


def _stamp_disc(solid, ci, cj, r):
    n2, n1 = solid.shape
    j0, j1 = max(0, int(np.floor(cj - r))), min(n2, int(np.ceil(cj + r)) + 1)
    ii = np.arange(int(np.floor(ci - r)), int(np.ceil(ci + r)) + 1)
    jj = np.arange(j0, j1)
    dx = ii + 0.5 - ci
    dy = jj + 0.5 - cj
    hit = dx[None, :] ** 2 + dy[:, None] ** 2 <= r * r
    cols = np.mod(ii, n1)  # periodic along x1, clipped along x2
    for a, j in enumerate(jj):
        solid[j, cols[hit[a]]] = 1


def _stamp_sphere(solid, ci, cj, ck, r):
    n3, n2, n1 = solid.shape
    ii = np.arange(int(np.floor(ci - r)), int(np.ceil(ci + r)) + 1)
    jj = np.arange(max(0, int(np.floor(cj - r))), min(n2, int(np.ceil(cj + r)) + 1))
    kk = np.arange(max(0, int(np.floor(ck - r))), min(n3, int(np.ceil(ck + r)) + 1))
    dx = ii + 0.5 - ci
    dy = jj + 0.5 - cj
    dz = kk + 0.5 - ck
    hit = dx[None, None, :] ** 2 + dy[None, :, None] ** 2 + dz[:, None, None] ** 2 <= r * r
    cols = np.mod(ii, n1)
    for c, k in enumerate(kk):
        for b, j in enumerate(jj):
            solid[k, j, cols[hit[c, b]]] = 1


def random_discs(n1, n2, target_porosity, rmin=4.0, rmax=20.0, seed=0, max_shapes=100000):
    """Boolean model of overlapping discs: centres uniform in the box, radii
    uniform in [rmin, rmax], periodic along x1 and clipped along x2. Discs are
    added one at a time until the porosity after removing non-percolating pores
    is at or below the target (checked every few discs, then refined)."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((n2, n1), np.uint8)
    placed = []
    while len(placed) < max_shapes:
        ci, cj = rng.uniform(0, n1), rng.uniform(0, n2)
        r = rng.uniform(rmin, rmax)
        _stamp_disc(solid, ci, cj, r)
        placed.append((ci, cj, r))
        if porosity(solid) <= target_porosity + 0.02:
            filled = fill_nonpercolating(solid)
            if porosity(filled) <= target_porosity:
                if percolates(filled):
                    return filled
                # lost percolation: restart from a fresh draw sequence
                solid[:] = 0
                placed.clear()
    raise RuntimeError("could not reach the target porosity")


def random_spheres(n1, n2, n3, target_porosity, rmin=4.0, rmax=10.0, seed=0, max_shapes=200000):
    """3D Boolean model of overlapping spheres, periodic along x1 and clipped
    along x2, x3, with the same stopping rule as `random_discs`
    (6-connected percolation)."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((n3, n2, n1), np.uint8)
    count = 0
    while count < max_shapes:
        ci, cj, ck = rng.uniform(0, n1), rng.uniform(0, n2), rng.uniform(0, n3)
        r = rng.uniform(rmin, rmax)
        _stamp_sphere(solid, ci, cj, ck, r)
        count += 1
        if porosity(solid) <= target_porosity + 0.02:
            filled = fill_nonpercolating(solid)
            if porosity(filled) <= target_porosity:
                if percolates(filled):
                    return filled
                solid[:] = 0
                count = 0
    raise RuntimeError("could not reach the target porosity")


# --- the workloads used by the tests and the benchmark -------------------------

def workload_unit_cell():
    """64 x 64 periodic unit cell with one centred disc of radius 0.25 L."""
    return centred_disc(64)


def workload_rock2d(seed=1, n=512, target_porosity=0.40):
    """512 x 512 overlapping random discs, radii U(4, 20) px, porosity 0.4,
    pore space connected (percolating along x1)."""
    return random_discs(n, n, target_porosity, 4.0, 20.0, seed)


def workload_pack3d(seed=7, n=96, target_porosity=0.35):
    """96^3 overlapping random spheres, radii U(4, 10) voxels, porosity 0.35."""
    return random_spheres(n, n, n, target_porosity, 4.0, 10.0, seed)


def workload_batch(count=64, seed0=1000, smin=128, smax=384):
    """Mixed-size batch: square sides U{smin..smax}, porosity U(0.3, 0.6),
    discs r ~ U(4, 20), Kn log-uniform in [0.05, 20] (L = the side).
    Returns a list of (mask, kn)."""
    out = []
    for b in range(count):
        rng = np.random.default_rng(seed0 + b)
        s = int(rng.integers(smin, smax + 1))
        eps = float(rng.uniform(0.3, 0.6))
        kn = float(np.exp(rng.uniform(np.log(0.05), np.log(20.0))))
        out.append((random_discs(s, s, eps, 4.0, 20.0, seed0 + b), kn))
    return out


def workload_warmstart(seed, n=256):
    """One sample of the warm-start data set: n x n discs r ~ U(4, 20),
    porosity U(0.3, 0.6), Kn log-uniform in [0.05, 20] (L = n voxels).
    Training seeds are 10000..11999, held-out seeds 20000..20199.
    Returns (mask, kn)."""
    rng = np.random.default_rng(seed)
    eps = float(rng.uniform(0.3, 0.6))
    kn = float(np.exp(rng.uniform(np.log(0.05), np.log(20.0))))
    return random_discs(n, n, eps, 4.0, 20.0, seed), kn
