"""Pins of the oracle's Gaussian layer anomaly (the low-velocity region of the
crosswell model, Sec. 4 eq:true_c): c_b multiplied by
1 - amp exp(-beta sum_d w_d (x_d - x0_d)^2) inside one layer.

  - the gradient and the Hessian are the derivatives of the returned speed
    (central differences), alone and on top of a linear-gradient layer;
  - at the centre the speed is c (1 - amp), and it does not change along an
    axis of weight 0 (the model's invariant direction);
  - a ray through the anomaly keeps its Hamiltonian c(Q)|P| (eq:char_plus);
  - across an interface with the anomaly on either side, the children's dzQ
    and dzP (the derived map, curved rays, the secant crossing) equal central
    differences of the child's Q and P over neighbouring initial (q, p).
"""
import numpy as np
import pytest

import oracle as om
from test_oracle_interfaces import child_of, one_beam

ANOM = (0.3, 40.0, (0.45, 0.0, 0.42), (1.0, 0.0, 1.0))


def med(grad=None, layer=0, anom=ANOM, surface=0.0):
    return om.layered(0, [0.5], [1.7, 2.2], [1.0, 1.25], [1.0, 1.3], grad=grad, anomaly={layer: anom},
                      surface=surface)


@pytest.mark.parametrize("grad", [None, [0.4, -0.3]])
def test_derivatives_are_those_of_the_speed(grad):
    m = med(grad)
    pts = np.random.default_rng(3).random((40, 3)) * np.array([0.8, 0.8, 0.45]) + np.array([0.05, 0.1, 0.02])
    for sp in (0, 1):
        c, g, H = om.speed(m, sp, pts)
        h = 1e-5
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            cp_, gp, _ = om.speed(m, sp, pts + e)
            cm, gm, _ = om.speed(m, sp, pts - e)
            assert np.abs((cp_ - cm) / (2 * h) - g[:, i]).max() < 1e-7
            assert np.abs((gp - gm) / (2 * h) - H[:, :, i]).max() < 1e-5
        assert np.abs(H - np.transpose(H, (0, 2, 1))).max() < 1e-13 * np.abs(H).max()


def test_centre_value_and_invariant_axis():
    m = med()
    x0 = np.array(ANOM[2])
    c, g, _ = om.speed(m, 0, x0[None, :])
    assert abs(c[0] - 1.7 * (1 - ANOM[0])) < 1e-15 and np.abs(g).max() < 1e-15
    pts = np.random.default_rng(5).random((20, 3)) * 0.45
    a = om.speed(m, 0, pts)
    b = om.speed(m, 0, pts + np.array([0.0, 0.37, 0.0]))
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    # outside its layer the anomaly does not act
    m2 = med(layer=1)
    c1, _, _ = om.speed(m2, 0, x0[None, :])
    assert c1[0] == 1.7


def test_ray_keeps_its_hamiltonian():
    m = med()
    b = one_beam(np.array([0.2, 0.3, 0.3]), np.array([1.0, 0.2, 0.25]), 0)
    c0, _, _ = om.speed(m, 0, b["Q"])
    H0 = c0[0] * np.linalg.norm(b["P"][0])
    out, _ = om.evolve_layered(m, b, 2e-3, 150)
    live = out[out["alive"] == 1]
    assert len(live) == 1 and live["layer"][0] == 0 and live["Q"][0][0] > 0.45   # passed the centre
    c1, _, _ = om.speed(m, 0, live["Q"])
    H1 = c1[0] * np.linalg.norm(live["P"][0])
    assert abs(H1 - H0) < 1e-10 * H0
    # the ray bends: the direction of P has turned
    p0 = b["P"][0] / np.linalg.norm(b["P"][0])
    p1 = live["P"][0] / np.linalg.norm(live["P"][0])
    assert np.arccos(np.clip(p0 @ p1, -1, 1)) > 0.05


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("branch,k", [(0, 2), (0, 0), (2, 3)])
def test_interface_jacobian_fd_with_anomaly(side, branch, k):
    """The anomaly on the incident side (side 0) or the far side (side 1) of
    the interface z = 0.5, centred near the crossing point."""
    anom = (0.25, 30.0, (0.3, 0.0, 0.5), (1.0, 0.0, 1.0))
    m = med(layer=side, anom=anom)
    q0 = np.array([0.3, 0.4, 0.47])
    p0 = np.array([0.35, -0.2, 1.0])
    p0 = p0 / np.linalg.norm(p0) * 1.3
    nsteps, dt = 6, 0.01
    out, _ = om.evolve_layered(m, one_beam(q0, p0, branch), dt, nsteps)
    lin = om.child_lineage(5, 0, k)
    c = child_of(out, lin)
    h = 1e-5
    D = {}
    for m_ in range(3):
        for which in ("q", "p"):
            res = []
            for s in (1, -1):
                q, p = q0.copy(), p0.copy()
                (q if which == "q" else p)[m_] += s * h
                o, _ = om.evolve_layered(m, one_beam(q, p, branch), dt, nsteps)
                res.append(child_of(o, lin))
            D[which, m_] = ((res[0]["Q"] - res[1]["Q"]) / (2 * h), (res[0]["P"] - res[1]["P"]) / (2 * h))
    dQq = np.array([D["q", i][0] for i in range(3)])
    dPq = np.array([D["q", i][1] for i in range(3)])
    dQp = np.array([D["p", i][0] for i in range(3)])
    dPp = np.array([D["p", i][1] for i in range(3)])
    tol = 1e-6
    assert np.abs(c["ZQ"].real - dQq).max() <= tol
    assert np.abs(-c["ZQ"].imag - dQp).max() <= tol
    assert np.abs(c["ZP"].real - dPq).max() <= tol
    assert np.abs(-c["ZP"].imag - dPp).max() <= tol
