"""GPU parity of merged S beams (merge_s = 1 in fga_mesh, fga_point_source and
fga_point_force): one S beam per (q, p, direction) carrying the SH and SV
weights, against the oracle's decomposition followed by its merge of each
SH/SV pair (oracle.merge_s_beams, pinned against the pair's field).

  - decomposition, one- and two-way and with a cull that leaves single
    members: the same lineage set (exact), branches, states and weights;
  - point moment-tensor source and point force: the same;
  - seismograms of the merged set after evolution in a smooth gridded medium
    equal those of the unmerged oracle beams (the pair's field), with 2/3 of
    the beams;
  - merged beams through flat and spherical interfaces (children made) give
    the oracle's seismograms of the same merged beams.

Bar: relative L2 <= 1e-10, integers exact.
"""
import math

import numpy as np
import pytest

import fga_inputs as fi
import oracle as om
from test_gpu_parity import (RTOL, SRC_M, compare_states, fga, layered_case, oracle_to_dict, rel_l2, say,
                             small_c2, two_way_velocity)

pytestmark = pytest.mark.gpu


def check_beams(g, mb):
    assert np.array_equal(g["lineage"], mb["lineage"])
    for k in ("branch", "sigma", "layer"):
        assert np.array_equal(g[k], mb[k]), k
    assert rel_l2(g["w"], mb["w"]) <= RTOL
    assert np.array_equal(g["e"], mb["e"])
    compare_states(g, mb)


@pytest.mark.parametrize("mode", ["one_way", "two_way", "cull"])
def test_decompose_merge_parity(mode):
    m = fga()
    say("merged decomposition", mode)
    w = small_c2(nq=4, np_=3, ny=16, nmed=16)
    nqp = w.qmesh.count * w.pmesh.count
    w.cull_abs = 0.0
    g = None
    if mode == "two_way":
        g = two_way_velocity(w)
        ob = om.decompose_two_way(w, g)
    else:
        if mode == "cull":
            full = om.decompose(w)
            v = np.sort(np.abs(full["w"]))
            k = int(0.55 * len(v))
            while v[k + 1] <= v[k] * (1 + 1e-8):      # a gap between two distinct values
                k += 1
            w.cull_abs = 0.5 * float(v[k] + v[k + 1]) / (
                w.qmesh.cell_volume * w.pmesh.cell_volume * (2 * math.pi * w.eps) ** -4.5)
        ob = om.decompose(w)
    mb = om.merge_s_beams(ob, nqp)
    if mode == "cull":
        # the kept sets must not depend on a psi within rounding of the threshold
        norm = w.qmesh.cell_volume * w.pmesh.cell_volume * (2 * math.pi * w.eps) ** -4.5
        full_abs = np.abs(full["w"]) / norm
        assert np.min(np.abs(full_abs - w.cull_abs)) > 1e-9 * w.cull_abs
    bs = m.fga_decompose(m.medium_for(w), m.mesh_for(w, one_way=g is None, merge_s=True), w.f, g=g)
    gexp = bs.export()
    assert bs.count == len(mb) < len(ob)
    check_beams(gexp, mb)


@pytest.mark.parametrize("kind", ["moment_tensor", "force"])
def test_source_merge_parity(kind):
    m = fga()
    say("merged source", kind)
    w = small_c2(nmed=16)
    mo, mg = om.medium_for(w), m.medium_for(w)
    if kind == "moment_tensor":
        eps, x0 = 1.0 / 32, [0.43, 0.52, 0.61]
        kw = dict(nq=5, ndir=40, nshell=3, ricker=True, rho0=1.0)
        ob = om.point_source_beams(mo, om.point_source(eps, x0, SRC_M, **kw))
        bs = m.fga_decompose_point_source(mg, m.point_source(eps, x0, SRC_M, merge_s=True, **kw))
    else:
        eps, x0 = 1.0 / 64, [0.43, 0.52, 0.61]
        kw = dict(nq=5, qhalf=0.3, ndir=24, nshell=3, omega=64.0, t0=0.01, width=0.05, t_ref=-0.01,
                  shell_lo=0.3, shell_hi=1.7)
        ob = om.point_force_beams(mo, om.point_force(eps, x0, [1.0, 1.0, 1.0], **kw))
        bs = m.fga_decompose_point_force(mg, m.point_force(eps, x0, [1.0, 1.0, 1.0], merge_s=True, **kw))
    nqp = kw["nq"] ** 3 * kw["ndir"] * kw["nshell"]
    mb = om.merge_s_beams(ob, nqp)
    g = bs.export()
    assert bs.count == len(mb) < len(ob)
    check_beams(g, mb)


def test_merged_seismograms_equal_the_pairs():
    """The merged set, evolved in the smooth gridded medium with receivers
    sampled every 5 steps, gives the seismograms of the unmerged oracle
    beams."""
    m = fga()
    say("merged seismograms")
    w = small_c2(nq=4, np_=2, ny=16, nmed=24)
    ob = om.decompose(w)
    mo, mg = om.medium_for(w), m.medium_for(w)
    bs = m.fga_decompose(mg, m.mesh_for(w, merge_s=True), w.f)
    assert 3 * bs.count == 2 * len(ob)
    rec = fi.uniform_points(9, fi.rng(2, 91), 0.3, 0.7)
    nsteps, dt, stride = 40, 2e-3, 5
    seis, _ = m.fga_evolve(mg, bs, dt, nsteps, receivers=rec, eps=w.eps, tau=w.tau, stride=stride)
    ref = np.zeros((len(rec), nsteps // stride, 3), dtype=np.complex128)
    for k in range(nsteps // stride):
        om.evolve(mo, ob, dt, stride)
        ref[:, k, :], _ = om.sum_points(ob, rec, w.eps, w.tau)
    assert rel_l2(m.to_complex(seis), ref) <= RTOL


@pytest.mark.parametrize("name", ["flat", "sphere"])
def test_merged_beams_through_interfaces(name):
    m = fga()
    say("merged beams through interfaces", name)
    w, ob, med_o, med_g = layered_case(name)
    mb = om.merge_s_beams(ob, w.qmesh.count * w.pmesh.count)
    rec = fi.uniform_points(9, np.random.default_rng(9), 0.2, 0.8)
    nsteps, dt, tau, stride = 30, 0.005, 25.0, 3
    bs = m.BeamSet(8 * len(mb))
    bs.load(oracle_to_dict(mb))
    seis, st = m.fga_evolve(med_g, bs, dt, nsteps, receivers=rec, eps=w.eps, tau=tau, stride=stride)
    ref = np.zeros((len(rec), nsteps // stride, 3), dtype=np.complex128)
    cnt = 0
    cur = mb.copy()
    for s in range(nsteps // stride):
        cur, _ = om.evolve_layered(med_o, cur, dt, stride, gmax=3, child_cut=1e-3)
        cur = cur[cur["alive"] == 1].copy()
        u, c = om.sum_points(cur, rec, w.eps, tau)
        ref[:, s, :] = u
        cnt += c
    assert st["spawned"] > 0
    assert st["evals"] == cnt
    assert rel_l2(m.to_complex(seis), ref) <= RTOL
