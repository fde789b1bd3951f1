"""GPU parity of the C^2 gridded medium (FGA_MEDIUM_GRID with smooth = 1: c is
the periodic cubic B-spline through the node values, grad c and the Hessian
its exact derivatives) against the oracle on the same seeded inputs:

  - the spline coefficients the table build writes (a recursive filter on the
    GPU, a cyclic tridiagonal solve in the oracle);
  - beam states after RK4 evolution (eq:char_plus, eq:char_minus, eq:DzDt,
    eq:amp_P, eq:amp_SV, eq:amp_SH) with beams clustered (the stencils come
    from the workgroup's LDS block) and scattered over several periods (the
    stencils come from global memory), with c_S from a ratio or a field;
  - the two-way decomposition, which divides the velocity data by c_b at
    the quadrature points (eq:psi);
  - point-source beams and the seismograms of evolved beams (eq:FGA).

Bar: relative L2 <= 1e-10 (S: 1e-12 absolute), integers exact.
"""
import math

import numpy as np
import pytest

import fga_inputs as fi
import oracle as om
from test_gpu_parity import (RTOL, SRC_M, compare_states, fga, oracle_to_dict, rel_l2, say, small_c2,
                             two_way_velocity)

pytestmark = pytest.mark.gpu

TP = 2 * math.pi


def mesh(n):
    return fi.Mesh3(tuple(n), (0.0, 0.0, 0.0), tuple(1.0 / k for k in n))


def fields(n, seed):
    m = mesh(n)
    Z, Y, X = np.meshgrid(m.axis(2), m.axis(1), m.axis(0), indexing="ij")
    g = np.random.default_rng(seed)
    cp = 1.7 * (1.0 + 0.15 * np.sin(TP * X) * np.cos(TP * Z) + 0.08 * np.cos(TP * (Y + X)))
    cp += 0.01 * g.standard_normal(cp.shape)
    cs = 0.6 * cp + 0.03 * np.cos(TP * Y) * np.sin(TP * Z)
    return m, cp, cs


def media(n, two, seed=21):
    m = fga()
    ms, cp, cs = fields(n, seed)
    if two:
        return (om.grid(cp, ms, cs_nodes=cs, smooth=True), m.Medium.grid(cp, ms, cs_nodes=cs, smooth=True))
    return om.grid(cp, ms, cs_ratio=0.58, smooth=True), m.Medium.grid(cp, ms, cs_ratio=0.58, smooth=True)


@pytest.mark.parametrize("n,two", [((12, 10, 14), False), ((7, 9, 8), True), ((64, 64, 64), True)])
def test_spline_coefficients_parity(n, two):
    say("spline coefficients", n, two)
    mo, mg = media(n, two)
    N = n[0] * n[1] * n[2]
    nf = 2 if two else 1
    table = mg._keep[0].cpu().numpy()
    assert table.size == 17 * N * nf
    coef = table[16 * N * nf:].reshape(nf, n[2], n[1], n[0])
    ref = mo._keep[-1]
    assert np.abs(coef - ref).max() <= 1e-13 * np.abs(ref).max()


def random_beams(nb, lo, hi, seed):
    g = np.random.default_rng(seed)
    ob = np.zeros(nb, dtype=om.BEAM_DTYPE)
    ob["Q"] = lo + (hi - lo) * g.random((nb, 3))
    d = g.standard_normal((nb, 3))
    ob["P"] = d / np.linalg.norm(d, axis=1)[:, None] * (0.8 + g.random(nb))[:, None]
    for i in range(3):
        ob["ZQ"][:, i, i] = 1.0
        ob["ZP"][:, i, i] = -1j
    ob["branch"] = g.integers(0, 3, nb)
    ob["a"][:, 0] = 1.0 + 0.5j
    ob["a"][:, 1] = np.where(ob["branch"] == 0, 0.0, 0.3j)
    ob["w"] = g.standard_normal(nb) + 1j * g.standard_normal(nb)
    e = g.standard_normal((nb, 3))
    ob["e"] = e / np.linalg.norm(e, axis=1)[:, None]
    ob["sigma"] = np.where(g.random(nb) < 0.5, 1, -1)
    ob["alive"] = 1
    ob["lineage"] = np.arange(nb)
    om.reframe(ob)
    return ob


@pytest.mark.parametrize("layout", ["clustered", "scattered"])
@pytest.mark.parametrize("two", [False, True])
def test_smooth_evolve_parity(layout, two):
    """700 beams (several workgroups and a ragged tail), all three branches,
    both signs of sigma; 120 RK4 steps in launches of 37."""
    m = fga()
    say("smooth evolve", layout, two)
    mo, mg = media((32, 28, 36), two)
    lo, hi = (0.42, 0.58) if layout == "clustered" else (-1.3, 2.2)
    ob = random_beams(700, lo, hi, 5 if two else 6)
    bs = m.BeamSet(len(ob) + 9)
    bs.load(oracle_to_dict(ob))
    m.fga_evolve(mg, bs, 2e-3, 120, chunk=37)
    om.evolve(mo, ob, 2e-3, 120)
    compare_states(bs.export(), ob)


def smooth_work(**kw):
    w = small_c2(**kw)
    w.medium_smooth = True
    return w


def test_smooth_decompose_two_way_parity():
    m = fga()
    say("smooth two-way decomposition")
    w = smooth_work(nq=4, np_=3, ny=16, nmed=16)
    w.cull_abs = 0.0
    g = two_way_velocity(w)
    ob = om.decompose_two_way(w, g)
    bs = m.fga_decompose(m.medium_for(w), m.mesh_for(w, one_way=False), w.f, g=g)
    gexp = bs.export()
    assert bs.count == len(ob) == 6 * w.qmesh.count * w.pmesh.count
    assert np.array_equal(gexp["lineage"], ob["lineage"])
    assert np.array_equal(gexp["sigma"], ob["sigma"])
    assert rel_l2(gexp["w"], ob["w"]) <= RTOL
    compare_states(gexp, ob)
    # the trilinear medium gives other weights: the test sees the cubic one
    w.medium_smooth = False
    assert rel_l2(om.decompose_two_way(w, g)["w"], ob["w"]) > 1e-6


def test_smooth_point_source_parity():
    m = fga()
    say("smooth point source")
    w = smooth_work(nmed=16)
    mo, mg = om.medium_for(w), m.medium_for(w)
    kw = dict(nq=5, ndir=40, nshell=3, ricker=True, rho0=1.0)
    x0 = [0.43, 0.52, 0.61]
    ob = om.point_source_beams(mo, om.point_source(1.0 / 32, x0, SRC_M, **kw))
    bs = m.fga_decompose_point_source(mg, m.point_source(1.0 / 32, x0, SRC_M, **kw))
    g = bs.export()
    assert np.array_equal(g["lineage"], ob["lineage"])
    for k in ("branch", "sigma", "layer"):
        assert np.array_equal(g[k], ob[k]), k
    assert rel_l2(g["Q"], ob["Q"]) <= 1e-14
    assert rel_l2(g["w"], ob["w"]) <= RTOL
    assert np.array_equal(g["e"], ob["e"])


def test_smooth_seismogram_parity():
    """Decomposed packet beams evolved in the C^2 medium with receivers
    sampled every 5 steps: the same seismograms as the oracle's evolve +
    Gaussian sums."""
    m = fga()
    say("smooth seismograms")
    w = smooth_work(nq=4, np_=2, ny=16, nmed=24)
    ob = om.decompose(w)
    mo, mg = om.medium_for(w), m.medium_for(w)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    rec = fi.uniform_points(9, fi.rng(2, 91), 0.3, 0.7)
    nsteps, dt, stride = 40, 2e-3, 5
    seis, _ = m.fga_evolve(mg, bs, dt, nsteps, receivers=rec, eps=w.eps, tau=w.tau, stride=stride)
    ref = np.zeros((len(rec), nsteps // stride, 3), dtype=np.complex128)
    for k in range(nsteps // stride):
        om.evolve(mo, ob, dt, stride)
        ref[:, k, :], _ = om.sum_points(ob, rec, w.eps, w.tau)
    assert np.abs(ref).max() > 0
    assert rel_l2(m.to_complex(seis), ref) <= RTOL


def test_smooth_evolve_tiny_grid():
    """A 3 x 4 x 5 node grid: the 4-node stencils wrap onto the same nodes
    (periodic images), in the LDS block and in global memory alike."""
    m = fga()
    say("smooth evolve, tiny grid")
    mo, mg = media((3, 4, 5), True)
    ob = random_beams(300, -0.5, 1.5, 8)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    m.fga_evolve(mg, bs, 2e-3, 60, chunk=25)
    om.evolve(mo, ob, 2e-3, 60)
    compare_states(bs.export(), ob)
