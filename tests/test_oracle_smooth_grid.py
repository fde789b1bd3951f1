"""Pins of the oracle's C^2 gridded medium: c is the periodic cubic B-spline
through the node values, and its gradient and Hessian are the exact
derivatives of that spline (the smooth-medium assumption of Sec. 2, under
which the ray and variational equations, eq:char_plus and eq:DzDt, need
c, grad c and its Hessian; the paper states no interpolation):

  - the spline takes the node values exactly, for arbitrary (rough) node
    data on small and non-cubic grids, which pins the periodic tridiagonal
    solve of the coefficients along each axis;
  - on a smooth periodic field it converges at the orders of cubic spline
    interpolation: h^4 for c, h^3 for grad c, h^2 for the Hessian;
  - grad c and the Hessian are the derivatives of the c it returns (central
    differences of the oracle's own c and grad c), which trilinear
    interpolation of separately differenced fields does not give;
  - c, grad c and the Hessian are continuous across cell faces (C^2), and
    the medium is periodic with the grid's period;
  - c_S follows cs_ratio or a second node field.
"""
import math

import numpy as np

import fga_inputs as fi
import oracle as om

TP = 2 * math.pi


def field(x, y, z):
    return 1.0 + 0.1 * np.sin(TP * x) * np.cos(TP * y) + 0.05 * np.sin(TP * (z + x))


def exact(pts):
    x, y, z = pts.T
    c = field(x, y, z)
    g = np.stack([0.1 * TP * np.cos(TP * x) * np.cos(TP * y) + 0.05 * TP * np.cos(TP * (z + x)),
                  -0.1 * TP * np.sin(TP * x) * np.sin(TP * y),
                  0.05 * TP * np.cos(TP * (z + x))], axis=1)
    s = -TP * TP
    hxx = 0.1 * s * np.sin(TP * x) * np.cos(TP * y) + 0.05 * s * np.sin(TP * (z + x))
    hyy = 0.1 * s * np.sin(TP * x) * np.cos(TP * y)
    hzz = 0.05 * s * np.sin(TP * (z + x))
    hxy = -0.1 * TP * TP * np.cos(TP * x) * np.sin(TP * y)
    hxz = 0.05 * s * np.sin(TP * (z + x))
    hyz = np.zeros_like(x)
    H = np.stack([hxx, hxy, hxz, hxy, hyy, hyz, hxz, hyz, hzz], axis=1).reshape(-1, 3, 3)
    return c, g, H


def mesh(n, lo=(0.0, 0.0, 0.0), period=(1.0, 1.0, 1.0)):
    return fi.Mesh3(tuple(n), tuple(lo), tuple(p / k for p, k in zip(period, n)))


def nodes_of(f, m):
    Z, Y, X = np.meshgrid(m.axis(2), m.axis(1), m.axis(0), indexing="ij")
    return f(X, Y, Z)


def test_interpolates_rough_node_values():
    g = np.random.default_rng(41)
    for n in ((1, 3, 4), (2, 5, 3), (6, 4, 7), (9, 8, 5)):
        m = mesh(n, lo=(-0.3, 0.2, 0.1), period=(0.7, 1.3, 1.1))
        f = 1.0 + 0.4 * g.random((n[2], n[1], n[0]))
        med = om.grid(f, m, cs_ratio=0.5, smooth=True)
        c, _, _ = om.speed(med, 0, m.points())
        assert np.abs(c - f.ravel()).max() < 1e-13, n


def test_converges_at_cubic_spline_orders():
    pts = np.random.default_rng(7).random((200, 3)) * 2.0 - 0.5   # includes periodic images
    errs = []
    for n in ((16, 20, 24), (32, 40, 48)):
        m = mesh(n)
        med = om.grid(nodes_of(field, m), m, cs_ratio=0.5, smooth=True)
        c, g, H = om.speed(med, 0, pts)
        ce, ge, He = exact(np.mod(pts, 1.0))
        errs.append((np.abs(c - ce).max(), np.abs(g - ge).max(), np.abs(H - He).max()))
    assert errs[1][0] < 2e-6 and errs[1][1] < 2e-4 and errs[1][2] < 2e-2, errs
    for k, order in enumerate((4, 3, 2)):
        r = errs[0][k] / errs[1][k]
        assert 0.75 * 2 ** order < r < 1.3 * 2 ** order, (k, errs)


def test_derivatives_are_those_of_the_value():
    """Central differences of the returned c give the returned grad c, and of
    grad c the Hessian, on rough node data (so no smoothness of the data can
    hide a wrong derivative weight)."""
    n = (7, 6, 5)
    m = mesh(n, lo=(0.1, -0.2, 0.3), period=(1.0, 0.8, 1.2))
    f = 1.0 + 0.3 * np.random.default_rng(3).random((n[2], n[1], n[0]))
    med = om.grid(f, m, cs_ratio=0.5, smooth=True)
    pts = np.random.default_rng(5).random((60, 3)) * 1.5
    c, g, H = om.speed(med, 0, pts)
    d = 1e-5
    for i in range(3):
        e = np.zeros(3)
        e[i] = d
        cp, gp, _ = om.speed(med, 0, pts + e)
        cm, gm, _ = om.speed(med, 0, pts - e)
        assert np.abs((cp - cm) / (2 * d) - g[:, i]).max() < 1e-6 * np.abs(g).max()
        assert np.abs((gp - gm) / (2 * d) - H[:, :, i]).max() < 1e-5 * np.abs(H).max()
    assert np.abs(H - np.transpose(H, (0, 2, 1))).max() == 0.0


def test_c2_across_faces_and_periodic():
    n = (6, 5, 7)
    m = mesh(n, lo=(0.0, 0.1, -0.2), period=(1.0, 1.0, 0.9))
    f = 1.0 + 0.3 * np.random.default_rng(9).random((n[2], n[1], n[0]))
    med = om.grid(f, m, cs_ratio=0.5, smooth=True)
    g = np.random.default_rng(10)
    base = g.random((30, 3)) * np.array([1.0, 1.0, 0.9]) + np.array([0.0, 0.1, -0.2])
    for ax in range(3):
        on = base.copy()
        k = np.floor((on[:, ax] - m.lo[ax]) / m.h[ax])
        on[:, ax] = m.lo[ax] + k * m.h[ax]
        e = np.zeros(3)
        e[ax] = 1e-9 * m.h[ax]
        a = om.speed(med, 0, on - e)
        b = om.speed(med, 0, on + e)
        for u, v, tol in zip(a, b, (1e-9, 1e-6, 1e-4)):
            assert np.abs(u - v).max() < tol * max(1.0, np.abs(u).max()), ax
    shift = np.array([1.0, 1.0, 0.9]) * np.array([[2, -1, 3]])
    for u, v in zip(om.speed(med, 0, base), om.speed(med, 0, base + shift)):
        assert np.allclose(u, v, rtol=1e-12, atol=1e-12)


def test_shear_speed_field():
    m = mesh((8, 8, 8))
    cp = nodes_of(field, m)
    cs = 0.5 + 0.2 * nodes_of(lambda x, y, z: np.cos(TP * y) * np.sin(TP * z), m)
    pts = np.random.default_rng(11).random((40, 3))
    one = om.grid(cp, m, cs_ratio=0.55, smooth=True)
    for u, v in zip(om.speed(one, 1, pts), om.speed(one, 0, pts)):
        assert np.allclose(u, 0.55 * v, rtol=1e-15, atol=0)
    two = om.grid(cp, m, cs_nodes=cs, smooth=True)
    c, _, _ = om.speed(two, 1, m.points())
    assert np.abs(c - cs.ravel()).max() < 1e-13
    c0, _, _ = om.speed(two, 0, m.points())
    assert np.abs(c0 - cp.ravel()).max() < 1e-13
