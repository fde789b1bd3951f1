"""Pins of the oracle's frame-free S polarisation (oracle.evolve(...,
s_vector=True)): the S amplitude carried as the physical vector
A = a_SV N_SV + a_SH N_SH, advanced by dA/dt = s A - (A . dPhat/dt) Phat
(what eq:amp_SV / eq:amp_SH give for the sum once the frame's rotation is
differentiated out) and returned to the beam's frame at the end:

  - in a medium that bends the rays it agrees with the framed evolution
    (itself pinned) to RK4 truncation: the difference falls as dt^4;
  - its physical polarisation does not depend on the reference axis the
    beam started with (the framed form needs the axis; this one does not);
  - P beams step exactly as in the framed evolution.
"""
import math

import numpy as np

import fga_inputs as fi
import oracle as om


def steep_medium():
    n = 16
    mesh = fi.node_grid(n)
    ax = mesh.axis(0)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    cp = 1.7 * (1.0 + 0.25 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z) + 0.1 * np.cos(2 * np.pi * Y))
    return om.grid(cp, mesh, cs_ratio=0.6, smooth=True)


def s_beams(nb=40, seed=11, axis=None):
    g = np.random.default_rng(seed)
    ob = np.zeros(nb, dtype=om.BEAM_DTYPE)
    ob["Q"] = g.random((nb, 3))
    d = g.standard_normal((nb, 3))
    ob["P"] = d / np.linalg.norm(d, axis=1)[:, None] * 1.3
    for i in range(3):
        ob["ZQ"][:, i, i] = 1.0
        ob["ZP"][:, i, i] = -1j
    ob["a"][:, 0] = 1.0 + 0.4j
    ob["a"][:, 1] = -0.3 + 0.8j
    ob["w"] = 1.0
    ob["branch"] = np.where(np.arange(nb) % 2 == 0, 1, 2)
    ob["sigma"] = np.where(np.arange(nb) % 3 == 0, -1, 1)
    ob["alive"] = 1
    ob["lineage"] = np.arange(nb)
    for i in range(nb):
        if axis is None:
            P = ob["P"][i]
            ob["e"][i] = [1.0, 0, 0] if abs(P[2]) / np.linalg.norm(P) > math.cos(math.radians(20)) else [0, 0, 1.0]
        else:
            ob["e"][i] = axis
    return ob


def run(med, ob, T, n, s_vector):
    b = ob.copy()
    om.evolve(med, b, T / n, n, s_vector=s_vector)
    return b, om.amplitude_vectors(b)


def test_agrees_with_framed_evolution_to_rk4_order():
    med = steep_medium()
    ob = s_beams()
    T = 0.4
    errs = []
    for n in (50, 100):
        bf, Af = run(med, ob, T, n, False)
        bv, Av = run(med, ob, T, n, True)
        assert np.array_equal(bf["Q"], bv["Q"]) and np.array_equal(bf["P"], bv["P"])
        errs.append(np.linalg.norm(Av - Af) / np.linalg.norm(Af))
    # the rays bend: the polarisation turns by O(1) over T, so dropping the transport
    # term would differ at O(1); RK4 truncation falls 16x per halving
    assert errs[1] < 1e-8, errs
    assert 10.0 < errs[0] / errs[1] < 24.0, errs


def test_independent_of_the_starting_axis():
    med = steep_medium()
    ob = s_beams(axis=[0.0, 0.0, 1.0])
    # keep beams not too close to either axis so both frames are valid
    P = ob["P"] / np.linalg.norm(ob["P"], axis=1)[:, None]
    ok = (np.abs(P[:, 2]) < 0.9) & (np.abs(P[:, 0]) < 0.9)
    ob = om.take_beams(ob, np.nonzero(ok)[0])
    ob2 = ob.copy()
    A0 = om.amplitude_vectors(ob)
    ob2["e"] = [1.0, 0.0, 0.0]
    # the same physical polarisation in the other frame
    for i in range(len(ob2)):
        Pp = ob2["P"][i]
        nsh = np.cross(ob2["e"][i], Pp); nsh /= np.linalg.norm(nsh)
        nsv = np.cross(Pp / np.linalg.norm(Pp), nsh)
        ob2["a"][i] = [A0[i] @ nsv, A0[i] @ nsh]
    assert np.abs(om.amplitude_vectors(ob2) - A0).max() < 1e-14
    _, A = run(med, ob, 0.4, 60, True)
    _, B = run(med, ob2, 0.4, 60, True)
    assert np.abs(A - B).max() < 1e-12 * np.abs(A).max()
    # the framed form depends on the axis at truncation level only as well, but not to rounding
    _, Af = run(med, ob, 0.4, 60, False)
    _, Bf = run(med, ob2, 0.4, 60, False)
    assert np.abs(Af - Bf).max() > 1e3 * np.abs(A - B).max()


def test_p_beams_step_as_in_the_framed_evolution():
    med = steep_medium()
    ob = s_beams()
    ob["branch"] = 0
    ob["a"][:, 1] = 0.0
    bf, _ = run(med, ob, 0.2, 30, False)
    bv, _ = run(med, ob, 0.2, 30, True)
    for k in ("Q", "P", "ZQ", "ZP", "a", "S"):
        assert np.array_equal(bf[k], bv[k]), k


def test_layered_media_with_curved_rays():
    """In layered media with a gradient layer and an anomaly, the frame-free
    regular steps of S beams give the same children (the ray does not depend
    on the amplitude) and polarisations within RK4 truncation of the framed
    run, falling with the step."""
    import fga_inputs as fi2
    from test_oracle_interfaces import one_beam
    med = om.layered(0, [0.5], [1.7, 2.2], [1.0, 1.25], [1.0, 1.3], grad=[0.4, -0.3],
                     anomaly={1: (0.2, 30.0, (0.3, 0.0, 0.6), (1.0, 0.0, 1.0))})
    g = np.random.default_rng(4)
    beams = []
    for k in range(12):
        q = np.array([0.2, 0.3, 0.3]) + 0.1 * g.random(3)
        p = g.standard_normal(3)
        p[2] = abs(p[2]) + 0.5
        b = one_beam(q, p / np.linalg.norm(p) * 1.3, 2)
        b["lineage"] = k
        beams.append(b)
    ob = np.concatenate(beams)
    errs = []
    for n in (60, 120):
        a, _ = om.evolve_layered(med, ob.copy(), 0.6 / n, n, child_cut=0.0)
        v, _ = om.evolve_layered(med, ob.copy(), 0.6 / n, n, child_cut=0.0, s_vector=True)
        a, v = a[a["alive"] == 1], v[v["alive"] == 1]
        assert np.array_equal(a["lineage"], v["lineage"]) and np.array_equal(a["Q"], v["Q"])
        assert np.sum(a["gen"] > 0) > 0
        A, V = om.amplitude_vectors(a), om.amplitude_vectors(v)
        errs.append(np.linalg.norm(A - V) / np.linalg.norm(A))
    assert 0 < errs[1] < 1e-7, errs
    assert errs[0] / errs[1] > 8.0, errs
