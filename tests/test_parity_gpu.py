"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Both sides get the same seeded inputs: the mask from the geometry generators
and the velocity grid from the oracle's own quadrature. FP64 results must
agree within 1e-10 relative on the moments and the permeability; the FP32 path
(FP32 sweep and storage, FP64 moments and reductions) within 1e-5.
"""
import math

import numpy as np
import pytest

from oracle import quadrature
from oracle.oracle import OracleSolver
from paper_1712_01132_amd import geometry, poredvm

pytestmark = pytest.mark.gpu

RTOL64 = 1e-10
RTOL32 = 1e-5


def rel(a, b):
    scale = float(np.max(np.abs(b)))
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / (scale if scale > 0 else 1.0)


def pair(mask, nv, kn, precision="fp64", lateral="specular", tile=None, jump=1.0, tau=False, threads=16,
         rule=1, schedule="auto", prandtl=None, alpha=1.0):
    o = OracleSolver(mask, nv, kn, jump=jump, lateral_periodic=(lateral == "periodic"),
                     tau_feedback=tau, threads=threads, stencil_rule=rule, prandtl=prandtl, accommodation=alpha)
    s = poredvm.Solver(mask, nv, kn, jump=jump, precision=precision, lateral=lateral,
                       tau_feedback=tau, tile=tile, grid=o.grid, stencil_rule=rule, schedule=schedule,
                       prandtl=prandtl, accommodation=alpha)
    return o, s


def compare(o, s, rtol, diagnostics=True):
    ro, uo, to, qo = o.moments()
    out = s.moments(diagnostics=diagnostics)
    rg, ug = out[0], out[1]
    scale = max(np.abs(uo).max(), np.abs(ro).max())
    assert np.max(np.abs(ug - uo)) <= rtol * np.abs(uo).max(), rel(ug, uo)
    assert np.max(np.abs(rg - ro)) <= rtol * scale, rel(rg, ro)
    if diagnostics:
        tg, qg = out[2], out[3]
        assert np.max(np.abs(tg - to)) <= rtol * max(np.abs(to).max(), scale), rel(tg, to)
        assert np.max(np.abs(qg - qo)) <= rtol * max(np.abs(qo).max(), scale), rel(qg, qo)
    go, ko, so = o.flux()
    gg, kg, sg = s.flux()
    assert abs(kg - ko) <= rtol * abs(ko)
    assert np.max(np.abs(sg - so)) <= rtol * np.abs(so).max()


def random_mask(shape, frac, seed):
    rng = np.random.default_rng(seed)
    while True:
        m = geometry.fill_nonpercolating((rng.random(shape) < frac).astype(np.uint8))
        if geometry.percolates(m) and m.sum() > 0:
            return m


def test_unit_cell_fp64_converges_like_oracle():
    m = geometry.workload_unit_cell()
    o, s = pair(m, [16, 16], 1.0)
    a = o.iterate(2000, 1e-8)
    b = s.iterate(2000, 1e-8)
    assert a["converged"] and b["converged"]
    assert a["iters"] == b["iters"]
    assert abs(a["r"] - b["r"]) <= 1e-6 * a["r"]
    assert abs(a["k"] - b["k"]) <= RTOL64 * abs(a["k"])
    compare(o, s, RTOL64)


@pytest.mark.parametrize("shape,nv,kn,tile,lateral,rule", [
    ((29, 37), [6, 8], 0.3, (8, 5), "specular", 1),
    ((29, 37), [6, 8], 0.3, (8, 5), "specular", 0),
    ((16, 20), [4, 4], 2.0, (16, 16), "periodic", 1),
    ((21, 70), [4, 4], 0.9, (32, 7), "specular", 1),
    ((9, 11, 13), [4, 4, 6], 0.7, (4, 4, 3), "specular", 1),
    ((9, 11, 13), [4, 4, 6], 0.7, (16, 4, 3), "specular", 0),
    ((8, 8, 8), [4, 4, 4], 1.5, (3, 5, 8), "periodic", 1),
])
def test_ragged_tiles_fp64_match_oracle(shape, nv, kn, tile, lateral, rule):
    m = random_mask(shape, 0.3, sum(shape))
    o, s = pair(m, nv, kn, lateral=lateral, tile=tile, rule=rule)
    for iters in (1, 7):
        o.iterate(iters)
        s.iterate(iters)
        compare(o, s, RTOL64)


@pytest.mark.parametrize("tile,rule", [((4, 4, 4), 1), ((4, 3, 5), 1), ((4, 4, 2), 0), ((8, 8, 3), 1)])
def test_ragged_tiles_3d_fp32_match_oracle(tile, rule):
    """3D FP32: with 4 x 4 tiles the sweep keeps the two upstream planes in
    registers; ragged tiles along every axis and both stencil rules."""
    m = random_mask((9, 11, 13), 0.25, 17)
    o, s = pair(m, [4, 4, 6], 0.7, precision="fp32", tile=tile, rule=rule)
    for iters in (1, 7):
        o.iterate(iters)
        s.iterate(iters)
        compare(o, s, RTOL32)


@pytest.mark.parametrize("shape,nv,tile,precision,lateral,rule", [
    ((29, 37), [6, 8], (8, 8), "fp64", "specular", 1),
    ((29, 37), [6, 8], (8, 5), "fp64", "specular", 0),
    ((33, 26), [8, 8], (3, 8), "fp32", "periodic", 1),
    ((17, 40), [4, 4], (4, 4), "fp64", "specular", 1),
    ((40, 9), [4, 6], (1, 4), "fp64", "specular", 1),
    ((64, 64), [24, 24], (8, 8), "fp32", "specular", 1),
    ((72, 56), [32, 32], (8, 8), "fp64", "specular", 1),
    ((40, 33), [16, 32], (8, 5), "fp32", "periodic", 0),
    ((70, 24), [8, 8], (4, 4), "fp64", "specular", 1),
    ((45, 30), [6, 6], (4, 4), "fp32", "periodic", 1),
    ((37, 29), [24, 24], (4, 4), "fp64", "specular", 1),
    ((50, 44), [16, 32], (4, 4), "fp32", "periodic", 0),
])
def test_row_pipeline_equals_tile_diagonals_bitwise(shape, nv, tile, precision, lateral, rule):
    """The one-launch row pipeline and the per-diagonal launches run the same
    arithmetic on the same values: every iterate is bitwise identical. Wide
    velocity grids give several chains per octant; narrow and ragged tiles
    exercise the register-carried left halo; more tile rows than one band
    holds, partial last bands and one- or two-voxel top rows exercise the LDS
    ring and the hand-over between bands; 4x4 tiles with several 64-velocity
    groups per octant, one of them partly empty, give several chains per
    band."""
    m = random_mask(shape, 0.3, sum(shape) + 7)
    out = []
    for sched in ("rows", "diagonals"):
        s = poredvm.Solver(m, nv, 0.6, precision=precision, lateral=lateral, tile=tile, stencil_rule=rule,
                           schedule=sched)
        r = s.iterate(12)
        out.append((s.moments(diagnostics=False), r["k"], r["r"]))
        s.close()
    (a, ka, ra), (b, kb, rb) = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and ka == kb and ra == rb


def test_row_pipeline_protocols():
    """Every tile row (and every band of strips) is padded to a multiple of 8
    blocks, so under round-robin placement each velocity chain runs on one XCD
    whatever the velocity grid: the creation probe confirms it and the
    automatic choice is the XCD-local row pipeline; STRIPS the strip pipeline.
    ROWS_AGENT forces the agent-scope protocol; all give the same iterates."""
    m = random_mask((40, 48), 0.3, 5)
    for nv in ([32, 32], [6, 8], [24, 24]):
        res = []
        for sched, want in (("auto", "rows-xcd"), ("strips", "strips"), ("rows-agent", "rows"),
                            ("diagonals", "diagonals")):
            s = poredvm.Solver(m, nv, 0.6, schedule=sched)
            assert s.schedule == want, (nv, sched, s.schedule)
            s.iterate(5)
            res.append(s.moments(diagnostics=False)[1])
            s.close()
        assert all(np.array_equal(res[0], r) for r in res[1:])


@pytest.mark.parametrize("shape,nv,precision,lateral,rule", [
    ((29, 37), [6, 8], "fp64", "specular", 1),     # one 64-velocity group: the pair's second is empty
    ((37, 29), [32, 32], "fp64", "specular", 1),   # four groups per octant, two pairs
    ((70, 24), [24, 24], "fp32", "specular", 1),   # three groups (the last partial); partial band and strip
    ((45, 7), [8, 8], "fp64", "specular", 0),      # fewer columns than one staging chunk
    ((9, 40), [16, 16], "fp32", "periodic", 1),    # three strips, the last one row high
    ((130, 33), [8, 8], "fp64", "specular", 0),    # many bands: hand-over through h between bands
    ((2, 2), [2, 2], "fp64", "specular", 1),       # the minimal domain
    ((5, 3), [4, 4], "fp32", "periodic", 0),
])
def test_strips_equal_tile_diagonals_bitwise(shape, nv, precision, lateral, rule):
    """The strip pipeline runs the same arithmetic on the same records as the
    tile diagonals: every iterate is bitwise identical."""
    m = random_mask(shape, 0.3, sum(shape) + 13)
    out = []
    for sched in ("strips", "diagonals"):
        s = poredvm.Solver(m, nv, 0.6, precision=precision, lateral=lateral, stencil_rule=rule, schedule=sched)
        assert s.schedule == sched
        r = s.iterate(12)
        out.append((s.moments(diagnostics=False), r["k"], r["r"]))
        s.close()
    (a, ka, ra), (b, kb, rb) = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and ka == kb and ra == rb


@pytest.mark.parametrize("shape_id", [0, 1, 2, 3])
def test_every_strip_shape_equals_tile_diagonals_bitwise(shape_id, monkeypatch):
    """Each compiled strip shape (4 or 2 rows per strip, 2 or 1 velocity groups
    per wavefront), chosen through the tuning override, on masks with several
    bands, partial strips and an odd group count."""
    monkeypatch.setenv("PDVM_STRIP_SHAPE", str(shape_id))
    for shape, nv, precision in (((67, 41), [24, 24], "fp64"), ((33, 50), [16, 16], "fp32")):
        m = random_mask(shape, 0.3, sum(shape) + shape_id)
        out = []
        for sched in ("strips", "diagonals"):
            s = poredvm.Solver(m, nv, 0.8, precision=precision, schedule=sched)
            s.iterate(7)
            out.append(s.moments(diagnostics=False))
            s.close()
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])

def test_minimal_domain_and_grid():
    m = np.zeros((2, 2), np.uint8)
    o, s = pair(m, [2, 2], 0.5)
    o.iterate(5)
    s.iterate(5)
    compare(o, s, RTOL64)


def test_free_molecular_channel_closed_form_on_gpu():
    n1, n2, nv = 8, 10, 8
    m = geometry.plane_channel(n1, n2)
    s = poredvm.Solver(m, [nv, nv], math.inf)
    r = s.iterate(100000, 1e-14)
    assert r["converged"]
    _, u = s.moments(diagnostics=False)
    x, w = poredvm.velocity_grid(nv)
    A = 0.5 * np.sum(w[x > 0] / x[x > 0])
    u1 = (n2 - 1) / n1 * A
    assert np.max(np.abs(u[0][m == 0] - u1)) <= 1e-12 * u1


def test_tile_shape_does_not_change_results_bitwise():
    m = random_mask((40, 48), 0.35, 3)
    res = []
    for tile in [(16, 16), (8, 4), (32, 40), (5, 7)]:
        s = poredvm.Solver(m, [8, 8], 0.5, tile=tile)
        s.iterate(6)
        res.append(s.moments(diagnostics=False))
        s.close()
    for r in res[1:]:
        assert np.array_equal(r[0], res[0][0]) and np.array_equal(r[1], res[0][1])


def test_repeat_runs_are_bitwise_identical():
    m = random_mask((33, 31), 0.3, 4)
    outs = []
    for _ in range(2):
        s = poredvm.Solver(m, [8, 8], 0.8, precision="fp32")
        s.iterate(9)
        outs.append(s.moments(diagnostics=False))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_checkpoint_resume_is_bitwise():
    m = random_mask((24, 30), 0.3, 5)
    a = poredvm.Solver(m, [6, 6], 0.4)
    a.iterate(250)                    # crosses iteration 100 and 200 (k history)
    blob = a.get_state()
    a.iterate(120)
    b = poredvm.Solver(m, [6, 6], 0.4)
    b.set_state(blob)
    rb = b.iterate(120)
    ra_m = a.moments()
    rb_m = b.moments()
    for x, y in zip(ra_m, rb_m):
        assert np.array_equal(x, y)
    assert rb["total_iters"] == 370
    with pytest.raises(poredvm.PdvmError):
        c = poredvm.Solver(m, [8, 8], 0.4)
        c.set_state(blob)


def test_fp32_checkpoint_continues_in_fp64():
    """An FP32 phase handed to an FP64 solver through the checkpoint: the FP64
    continuation tracks the FP64 oracle to the FP32 tolerance, and the handover
    itself loses nothing (FP32 -> FP64 is exact)."""
    m = random_mask((24, 32), 0.3, 8)
    o, s32 = pair(m, [8, 8], 0.5, precision="fp32")
    s32.iterate(150)
    blob = s32.get_state()
    s64 = poredvm.Solver(m, [8, 8], 0.5, precision="fp64", grid=o.grid)
    s64.set_state(blob)
    r32, u32 = s32.moments(diagnostics=False)
    r64, u64 = s64.moments(diagnostics=False)
    assert np.array_equal(r32, r64) and np.array_equal(u32, u64)
    back = s64.get_state()
    s32b = poredvm.Solver(m, [8, 8], 0.5, precision="fp32", grid=o.grid)
    s32b.set_state(back)  # and back: FP64 values that came from FP32 round to themselves
    s32.iterate(10)
    s32b.iterate(10)
    for x, y in zip(s32.moments(diagnostics=False), s32b.moments(diagnostics=False)):
        assert np.array_equal(x, y)
    st = s64.iterate(250)
    assert st["total_iters"] == 400
    o.iterate(400)
    compare(o, s64, RTOL32, diagnostics=False)


def test_warm_start_matches_oracle():
    m = random_mask((20, 24), 0.3, 6)
    fl = m == 0
    rng = np.random.default_rng(1)
    rho = rng.normal(size=m.shape) * fl
    u = rng.normal(size=(2,) + m.shape) * fl * 0.1
    o, s = pair(m, [8, 8], 0.6)
    o.set_initial(rho, u)
    s.set_initial(rho, u)
    compare(o, s, RTOL64, diagnostics=False)
    o.iterate(5)
    s.iterate(5)
    compare(o, s, RTOL64)


def test_tau_feedback_3d_matches_oracle():
    m = random_mask((8, 9, 10), 0.25, 7)
    o, s = pair(m, [4, 4, 4], 0.9, tau=True)
    o.iterate(8)
    s.iterate(8)
    compare(o, s, RTOL64)


@pytest.mark.parametrize("shape,nv,kn,tile,schedule,precision,lateral,rule", [
    ((37, 29), [8, 8], 0.7, (4, 4), "rows", "fp64", "specular", 1),
    ((37, 29), [8, 8], 0.7, (8, 8), "diagonals", "fp64", "specular", 1),
    ((33, 26), [24, 24], 0.3, (8, 8), "rows", "fp64", "periodic", 1),
    ((33, 26), [24, 24], 0.3, (4, 4), "diagonals", "fp64", "specular", 0),
    ((29, 40), [6, 10], 2.0, (4, 4), "rows", "fp64", "specular", 0),
    ((45, 40), [16, 16], 1.5, (4, 4), "rows", "fp32", "specular", 1),
])
def test_tau_feedback_2d_matches_oracle(shape, nv, kn, tile, schedule, precision, lateral, rule):
    """2D with the temperature fed back: each velocity slot of an octant has a
    psi slot after the octant's last velocity (Ko = 288 with the 24 x 24 grid:
    psi starts inside a 64-velocity group and the last group is partial).
    Random geometries: the GPU runs the oracle's iteration, lag included."""
    m = random_mask(shape, 0.3, sum(shape) + 11)
    o, s = pair(m, nv, kn, precision=precision, lateral=lateral, tile=tile, tau=True, rule=rule,
                schedule=schedule)
    assert s.schedule.startswith(schedule)
    o.iterate(12)
    s.iterate(12)
    compare(o, s, RTOL64 if precision == "fp64" else RTOL32)


@pytest.mark.parametrize("nv,tile,pr,alpha,precision", [
    ([24, 24], (4, 4), None, 1.0, "fp64"),
    ([8, 8], (8, 8), None, 1.0, "fp64"),
    ([24, 24], (4, 4), 2.0 / 3.0, 1.0, "fp64"),
    ([10, 8], (8, 8), 0.5, 0.6, "fp32"),
    ([24, 24], (4, 4), None, 0.7, "fp64"),
    ([8, 8], (8, 5), 2.0 / 3.0, 0.5, "fp64"),
])
def test_tau_feedback_2d_row_pipeline_equals_tile_diagonals_bitwise(nv, tile, pr, alpha, precision):
    """tau fed back (psi), with the Shakhov model and Maxwell walls: the row
    pipeline and the tile diagonals give bitwise identical iterates."""
    m = random_mask((41, 35), 0.3, 21)
    out = []
    for sched in ("rows", "diagonals"):
        s = poredvm.Solver(m, nv, 0.4, tau_feedback=True, tile=tile, schedule=sched, prandtl=pr,
                           accommodation=alpha, precision=precision)
        s.iterate(9)
        out.append(s.moments())
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,nv,kn,tile,precision,pr", [
    ((8, 9, 10), [4, 4, 4], 0.9, None, "fp64", 2.0 / 3.0),
    ((7, 10, 12), [6, 6, 6], 0.3, (8, 8, 4), "fp64", 0.4),
    ((9, 8, 11), [8, 8, 8], 1.7, (4, 4, 3), "fp32", 2.0 / 3.0),
    ((37, 29), [8, 8], 0.7, (4, 4), "fp64", 2.0 / 3.0),
    ((33, 26), [24, 24], 0.3, (8, 8), "fp64", 0.5),
    ((45, 40), [16, 16], 1.5, (4, 4), "fp32", 2.0 / 3.0),
])
def test_shakhov_matches_oracle(shape, nv, kn, tile, precision, pr):
    """Shakhov model (heat flux fed back) on random geometries, 3D and 2D
    (with psi); 2D takes the row pipeline."""
    m = random_mask(shape, 0.25, sum(shape) + 5)
    o, s = pair(m, nv, kn, precision=precision, tile=tile, tau=True, prandtl=pr)
    assert s.schedule == "queue" if len(shape) == 3 else s.schedule.startswith("rows")
    o.iterate(10)
    s.iterate(10)
    compare(o, s, RTOL64 if precision == "fp64" else RTOL32)
    # the heat-flux term changes the iterate (it is not a no-op)
    b = poredvm.Solver(m, nv, kn, precision=precision, tile=tile, tau_feedback=True, grid=o.grid)
    b.iterate(10)
    assert np.abs(b.moments()[3] - s.moments()[3]).max() > 1e-6 * np.abs(s.moments()[3]).max()
    b.close()


def test_shakhov_checkpoint_resume_is_bitwise():
    m = random_mask((30, 28), 0.3, 17)
    s = poredvm.Solver(m, [8, 8], 0.5, tau_feedback=True, prandtl=2.0 / 3.0)
    s.iterate(7)
    st = s.get_state()
    s.iterate(6)
    a = s.moments()
    t = poredvm.Solver(m, [8, 8], 0.5, tau_feedback=True, prandtl=2.0 / 3.0)
    t.set_state(st)
    t.iterate(6)
    for x, y in zip(a, t.moments()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("shape,nv,kn,tile,precision,lateral,alpha,tau,pr", [
    ((37, 29), [8, 8], 0.7, (4, 4), "fp64", "specular", 0.5, False, None),
    ((33, 26), [24, 24], 0.3, (8, 8), "fp64", "periodic", 0.8, False, None),
    ((37, 29), [8, 8], 0.7, (8, 8), "fp64", "specular", 0.6, True, None),
    ((37, 29), [8, 8], 0.7, (4, 4), "fp64", "specular", 0.6, True, 2.0 / 3.0),
    ((45, 40), [16, 16], 1.5, (4, 4), "fp32", "specular", 0.3, False, None),
    ((8, 9, 10), [4, 4, 4], 0.9, None, "fp64", "specular", 0.5, False, None),
    ((7, 10, 12), [6, 6, 6], 0.4, (4, 4, 3), "fp64", "periodic", 0.7, True, 0.5),
])
def test_maxwell_walls_match_oracle(shape, nv, kn, tile, precision, lateral, alpha, tau, pr):
    """Maxwell walls (alpha < 1), alone and with tau fed back (psi) and the
    Shakhov model, 2D and 3D, on random geometries."""
    m = random_mask(shape, 0.25, sum(shape) + 3)
    o, s = pair(m, nv, kn, precision=precision, lateral=lateral, tile=tile, tau=tau, prandtl=pr, alpha=alpha)
    assert s.schedule == "queue" if len(shape) == 3 else s.schedule.startswith("rows")
    o.iterate(10)
    s.iterate(10)
    compare(o, s, RTOL64 if precision == "fp64" else RTOL32)


def test_maxwell_free_molecular_channel_closed_form_on_gpu():
    """The closed form of the free-molecular channel with Maxwell walls:
    u1 = J dx A [(N2 - 1) + 2 ((1 - alpha)/alpha)(N2 - 2)], A = sum_{v2>0} W v1^2/v2."""
    n1, n2, nv, alpha = 8, 10, 8, 0.5
    m = geometry.plane_channel(n1, n2)
    s = poredvm.Solver(m, [nv, nv], math.inf, accommodation=alpha)
    r = s.iterate(100000, 1e-14)
    assert r["converged"]
    x, w = poredvm.velocity_grid(nv)
    A = 0.5 * np.sum(w[x > 0] / x[x > 0])
    u1 = A / n1 * ((n2 - 1) + 2 * (1 - alpha) / alpha * (n2 - 2))
    u = s.moments(diagnostics=False)[1]
    assert np.max(np.abs(u[0][m == 0] - u1)) <= 1e-10 * u1


@pytest.mark.parametrize("nv,tile,precision", [([24, 24], (4, 4), "fp64"), ([8, 8], (8, 8), "fp32")])
def test_maxwell_row_pipeline_equals_tile_diagonals_bitwise(nv, tile, precision):
    m = random_mask((43, 37), 0.3, 23)
    out = []
    for sched in ("rows", "diagonals"):
        s = poredvm.Solver(m, nv, 0.4, tile=tile, schedule=sched, accommodation=0.65, precision=precision)
        s.iterate(9)
        out.append(s.moments())
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_maxwell_checkpoint_resume_is_bitwise():
    m = random_mask((30, 28), 0.3, 19)
    s = poredvm.Solver(m, [8, 8], 0.5, accommodation=0.6)
    s.iterate(7)
    st = s.get_state()
    s.iterate(6)
    a = s.moments()
    t = poredvm.Solver(m, [8, 8], 0.5, accommodation=0.6)
    t.set_state(st)
    t.iterate(6)
    for x, y in zip(a, t.moments()):
        assert np.array_equal(x, y)


def test_paper_stop_mode_matches_oracle():
    m = random_mask((16, 16), 0.3, 8)
    o, s = pair(m, [6, 6], 1.0)
    a = o.iterate(5000, 1e-9, stop_mode=1)
    b = s.iterate(5000, 1e-9, stop_mode="paper")
    assert a["converged"] and b["converged"] and a["iters"] == b["iters"]
    assert a["iters"] % 100 == 0
    assert abs(a["err"] - b["err"]) <= 1e-6 * a["err"] + 1e-18


def test_zero_driving_force_on_gpu():
    m = random_mask((18, 14), 0.3, 9)
    s = poredvm.Solver(m, [6, 6], 0.5, jump=0.0)
    rng = np.random.default_rng(3)
    fl = m == 0
    s.set_initial(rng.normal(size=m.shape) * fl, rng.normal(size=(2,) + m.shape) * fl)
    s.iterate(3000)
    rho, u = s.moments(diagnostics=False)
    assert np.abs(u).max() <= 1e-12
    assert np.ptp(rho[fl]) <= 1e-11


def test_nonfinite_iterate_keeps_last_good_state():
    m = random_mask((12, 12), 0.3, 10)
    s = poredvm.Solver(m, [4, 4], 1.0)
    rho = np.zeros(m.shape)
    rho[m == 0] = 0.5
    rho[np.argwhere(m == 0)[0][0], np.argwhere(m == 0)[0][1]] = np.nan
    s.set_initial(rho, None)
    before = s.moments(diagnostics=False)
    with pytest.raises(poredvm.PdvmError) as e:
        s.iterate(10)
    assert e.value.code == poredvm.PDVM_E_NONFINITE
    after = s.moments(diagnostics=False)
    assert np.array_equal(np.isnan(before[0]), np.isnan(after[0]))
    np.testing.assert_array_equal(np.nan_to_num(before[0]), np.nan_to_num(after[0]))


def test_fp32_unit_cell_within_tolerance():
    m = geometry.workload_unit_cell()
    o, s = pair(m, [16, 16], 1.0, precision="fp32")
    a = o.iterate(2000, 1e-8)
    b = s.iterate(2000, 1e-6)
    assert b["converged"]
    _, uo, _, _ = o.moments()
    _, ug = s.moments(diagnostics=False)
    assert rel(ug, uo) <= RTOL32
    assert abs(b["k"] - a["k"]) <= RTOL32 * abs(a["k"])


@pytest.mark.parametrize("kn", [0.1, 1.0, 10.0])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rock2d_full_size_two_iterations(precision, kn):
    """The 2D rock at full size (512^2 voxels, 32 x 32 velocities) at each of
    its three Knudsen numbers, in the benchmark's launch configuration."""
    m = geometry.workload_rock2d(seed=1)
    o, s = pair(m, [32, 32], kn, precision=precision)
    o.iterate(2)
    s.iterate(2)
    compare(o, s, RTOL64 if precision == "fp64" else RTOL32, diagnostics=False)


def test_pack3d_full_size_three_iterations_fp32():
    """The 3D pack at full size (96^3 voxels, 16^3 velocities, Kn = 0.5), FP32.
    From the second iteration on the source, the wall densities and the
    lagged mirror and wrap values are nonzero, so all of them are compared."""
    m = geometry.workload_pack3d(seed=7)
    o, s = pair(m, [16, 16, 16], 0.5, precision="fp32")
    for _ in range(3):
        o.iterate(1)
        s.iterate(1)
        compare(o, s, RTOL32, diagnostics=False)


_BATCH64 = None


def _batch64():
    global _BATCH64
    if _BATCH64 is None:
        _BATCH64 = geometry.workload_batch(64)
    return _BATCH64


def test_batch64_full_size_against_oracle_fp32():
    """The 64-problem batch (sides 128 to 384, porosity 0.3 to 0.6, Kn 0.05 to
    20, 24 x 24 velocities, FP32) through the batch calls, in the benchmark's
    launch configuration; after 3 iterations the largest and the smallest
    problem and those with the smallest and the largest Kn are compared with
    the oracle element by element."""
    probs = _batch64()
    sides = [m.shape[0] for m, _ in probs]
    kns = [kn for _, kn in probs]
    pick = sorted({int(np.argmax(sides)), int(np.argmin(sides)), int(np.argmin(kns)), int(np.argmax(kns))})
    assert len(pick) == 4
    grid = [quadrature.full_line_grid(24)] * 2  # the oracle's own quadrature on both sides
    b = poredvm.Batch(probs, [24, 24], precision="fp32", grid=grid)
    res = b.iterate(3)
    assert all(r["iters"] == 3 for r in res)
    for i in pick:
        m, kn = probs[i]
        o = OracleSolver(m, [24, 24], kn, threads=16, grid=grid)
        o.iterate(3)
        ro, uo, _, _ = o.moments()
        rg, ug = b.moments(i)
        scale = max(np.abs(uo).max(), np.abs(ro).max())
        assert np.max(np.abs(ug - uo)) <= RTOL32 * np.abs(uo).max(), (i, rel(ug, uo))
        assert np.max(np.abs(rg - ro)) <= RTOL32 * scale, (i, rel(rg, ro))
        _, ko, so = o.flux()
        _, kg, sg = b.flux(i)
        assert abs(kg - ko) <= RTOL32 * abs(ko), i
        assert np.max(np.abs(sg - so)) <= RTOL32 * np.abs(so).max(), i
        o.close()
