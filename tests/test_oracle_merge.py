"""Pins of the oracle's merge of SH/SV beam pairs (oracle.merge_s_beams).

The SH and SV beams of one (q, p, direction) share their ray, and the S
amplitude equations and the interface split are linear in the amplitude,
so one beam on the common ray with amplitude w_SH a_SH + w_SV a_SV gives
the same field (eq:FGA) as the pair.  The pins check this against the
already pinned evolution and summation:

  - the merged set is the P beams plus one beam per (q, p, direction) with
    an S member, and every pair shares its ray exactly;
  - evolved in a smooth gridded medium, with one- and two-way data and with
    a cull that leaves single members, the merged set sums to the pair's
    field at receivers (1e-13 relative);
  - through flat and spherical interfaces (children made, no child cutoff)
    the same holds;
  - a mistake in the merge (the SV weight dropped, or applied to the wrong
    component) breaks the equality.
"""
import numpy as np
import pytest

import fga_inputs as fi
import oracle as om


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def work():
    return fi.smooth_medium_packet(nq=4, np_=3, ny=16, nmed=16, nout=0, nrec=0)


def field(beams, x, w):
    u, _ = om.sum_points(beams, x, w.eps, w.tau)
    return u


@pytest.mark.parametrize("mode", ["one_way", "two_way", "cull"])
def test_merged_beams_sum_to_the_pairs_field(mode):
    w = work()
    nqp = w.qmesh.count * w.pmesh.count
    if mode == "two_way":
        d = fi.unit_vector(fi.rng(2, 77))
        g = 2.0 * fi.gaussian_plane_wave(w.ymesh, w.eps, (0.45, 0.5, 0.55), 0.12, (1.0, 0.5, 0.0), d)
        ob = om.decompose_two_way(w, g)
    else:
        if mode == "cull":
            full = om.decompose(w)
            w.cull_abs = float(np.quantile(np.abs(full["w"]), 0.55)) / (
                w.qmesh.cell_volume * w.pmesh.cell_volume * (2 * np.pi * w.eps) ** -4.5)
        ob = om.decompose(w)
    mb = om.merge_s_beams(ob, nqp)
    nP = int(np.sum(ob["branch"] == 0))
    keys = set(ob["lineage"][ob["branch"] == 1].tolist()) | set((ob["lineage"][ob["branch"] == 2] - 2 * nqp).tolist())
    assert len(mb) == nP + len(keys)
    assert set(mb["lineage"][mb["branch"] == 1].tolist()) == keys
    if mode == "cull":
        sh = set(ob["lineage"][ob["branch"] == 1].tolist())
        sv = set((ob["lineage"][ob["branch"] == 2] - 2 * nqp).tolist())
        assert sh ^ sv                      # single members exist
    med = om.medium_for(w)
    x = fi.uniform_points(40, fi.rng(2, 5), 0.25, 0.75)
    for k in range(3):
        om.evolve(med, ob, 2e-3, 20)
        om.evolve(med, mb, 2e-3, 20)
        ref = field(ob, x, w)
        assert rel(field(mb, x, w), ref) < 1e-13, k


@pytest.mark.parametrize("geo", [0, 1])
def test_merged_beams_through_interfaces(geo):
    w = fi.homogeneous_packet(nq=4, np_=2, ny=16, nout=0)
    nqp = w.qmesh.count * w.pmesh.count
    ob = om.decompose(w)
    if geo == 0:
        med = om.layered(0, [0.42, 0.58], [1.7, 2.2, 1.9], [1.0, 1.3, 1.1], [1.0, 1.35, 1.2])
        lev, bounds = ob["Q"][:, 2], [0.42, 0.58]
        ob["layer"] = (lev > bounds[0]).astype(int) + (lev > bounds[1]).astype(int)
    else:
        med = om.layered(1, [0.95, 0.8], [1.7, 2.1, 2.4], [1.0, 1.2, 1.4], [1.0, 1.25, 1.5])
        r = np.linalg.norm(ob["Q"], axis=1)
        ob["layer"] = (r < 0.95).astype(int) + (r < 0.8).astype(int)
    mb = om.merge_s_beams(ob, nqp)
    x = fi.uniform_points(30, fi.rng(1, 9), 0.2, 0.8)
    a, _ = om.evolve_layered(med, ob, 0.005, 50, gmax=3, child_cut=0.0)
    b, _ = om.evolve_layered(med, mb, 0.005, 50, gmax=3, child_cut=0.0)
    assert np.sum(a["gen"] > 0) > 0                       # children were made
    ua = field(a[a["alive"] == 1], x, w)
    ub = field(b[b["alive"] == 1], x, w)
    assert rel(ub, ua) < 1e-12


def test_planted_merge_mistakes_are_seen():
    w = work()
    nqp = w.qmesh.count * w.pmesh.count
    ob = om.decompose(w)
    x = fi.uniform_points(40, fi.rng(2, 5), 0.25, 0.75)
    med = om.medium_for(w)
    mb = om.merge_s_beams(ob, nqp)
    om.evolve(med, ob, 2e-3, 20)
    ref = field(ob, x, w)
    for plant in ("drop_sv", "swap"):
        bad = mb.copy()
        s = bad["branch"] == 1
        if plant == "drop_sv":
            bad["a"][s, 0] = 0.0
        else:
            bad["a"][s] = bad["a"][s][:, ::-1]
        om.evolve(med, bad, 2e-3, 20)
        assert rel(field(bad, x, w), ref) > 1e-3, plant
