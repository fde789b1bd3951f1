"""Pins of the oracle's point moment-tensor source (decomposition of
u(0) = 0, u_t(0) = -(1/rho0) M grad delta(x - x0); Sec. 2.1 eq:psi with
eq:alpha^k at f = 0):

  - each beam's weight from the closed-form FBI[g / c_b] equals the two-way
    weight of the packet decomposition (itself pinned by the u(0) = f and
    u_t(0) = g tests) applied to a direct quadrature of the FBI of the same
    source smoothed by a narrow Gaussian, to O(sigma^2) (homogeneous and
    linear-gradient media, so both the kernel-derivative and the speed-
    gradient terms are checked);
  - Gauss-Legendre shells reproduce numpy's nodes and integrate polynomials
    exactly; the p measure integrates the shell volume exactly;
  - Fibonacci directions are unit vectors in equal-area z bands;
  - the Ricker weight peaks at omega0 with value 1.
"""
import math

import numpy as np
import pytest

import fga_inputs as fi
import oracle as om

M6 = [1.0, 0.5, -0.3, 0.2, 0.1, -0.4]


def sym(M):
    return np.array([[M[0], M[3], M[4]], [M[3], M[1], M[5]], [M[4], M[5], M[2]]])


def test_gauss_legendre_against_numpy_and_polynomials():
    for n in (1, 3, 6, 11):
        x, w = om.gauss_legendre(n, 0.3, 2.0)
        X, W = np.polynomial.legendre.leggauss(n)
        assert np.allclose(np.sort(x), np.sort(1.15 + 0.85 * X), atol=1e-14)
        assert np.allclose(w[np.argsort(x)], (0.85 * W)[np.argsort(X)], atol=1e-14)
        for k in range(2 * n):
            exact = (2.0 ** (k + 1) - 0.3 ** (k + 1)) / (k + 1)
            assert abs(np.sum(w * x ** k) - exact) <= 1e-13 * max(1.0, exact)


def test_shell_measure_integrates_volume():
    """sum over shells and directions of |p|^2 w 4 pi / ndir = shell volume."""
    x, w = om.gauss_legendre(4, 0.5, 1.7)
    ndir = 50
    vol = sum(x[s] ** 2 * w[s] * 4 * math.pi / ndir for s in range(4)) * ndir
    assert abs(vol - 4 * math.pi / 3 * (1.7 ** 3 - 0.5 ** 3)) <= 1e-12


def test_fibonacci_directions():
    n = 400
    d = om.fibonacci_dirs(n)
    assert np.abs(np.linalg.norm(d, axis=1) - 1).max() <= 1e-15
    assert abs(d[:, 2].sum()) <= 1e-12                     # symmetric in z
    # equal-area: each of 8 z-bands of equal height holds n/8 points
    counts = np.histogram(d[:, 2], bins=8, range=(-1, 1))[0]
    assert np.all(np.abs(counts - n / 8) <= 1)


def test_ricker_peak():
    w0 = 3.7
    vals = [om.ricker(w, w0) for w in np.linspace(0.1, 10, 991)]
    k = int(np.argmax(vals))
    assert abs(np.linspace(0.1, 10, 991)[k] - w0) <= 0.011
    assert abs(om.ricker(w0, w0) - 1.0) <= 1e-15


def smoothed_source_fbi(med, cb_fn, x0, M, rho0, sigma, q, p, eps, h):
    """FBI of g_sigma / c_b by direct quadrature, g_sigma = -(1/rho0) M grad G_sigma(y - x0)."""
    n = int(round(12 * sigma / h))
    mesh = fi.Mesh3((n, n, n), tuple(np.asarray(x0) - 6 * sigma + 0.5 * h), (h, h, h))
    Y = mesh.points().reshape(n, n, n, 3)   # [z][y][x][3]
    d = Y - np.asarray(x0)
    r2 = np.sum(d * d, axis=-1)
    Gs = np.exp(-r2 / (2 * sigma ** 2)) / (2 * math.pi * sigma ** 2) ** 1.5
    grad = -d / sigma ** 2 * Gs[..., None]
    g = -(1.0 / rho0) * np.einsum("ij,zyxj->zyxi", sym(M), grad)
    c = cb_fn(Y)
    f = np.moveaxis(g / c[..., None], -1, 0).astype(np.complex128)
    return om.fbi(f, mesh, q[None, :], p[None, :], eps)[0]


def two_way_psi(b, G, eps):
    """psi of the two-way decomposition (f = 0, FBI[g/c_b] = G) for the branch
    and direction of beam b at its (q, p): the oracle's own weight, pinned by
    tests/test_oracle_twoway.py, on a one-point mesh of unit cell measure."""
    br = int(b["branch"])
    qm = fi.Mesh3((1, 1, 1), tuple(b["Q"]), (1.0, 1.0, 1.0))
    pm = fi.Mesh3((1, 1, 1), tuple(b["P"]), (1.0, 1.0, 1.0))
    Gt = np.zeros((1, 2, 3), dtype=np.complex128)
    Gt[0, 0 if br == 0 else 1] = G
    bb = om.make_beams(qm, pm, np.zeros((1, 3), dtype=np.complex128), eps, np.array([0]), np.array([0]),
                       one_way=False, Gt=Gt, branch_mask=1 << br)
    sel = bb[bb["sigma"] == b["sigma"]]
    return sel["w"][0] * (2 * math.pi * eps) ** 4.5


@pytest.mark.parametrize("medium_kind", ["homogeneous", "linear"])
def test_closed_form_against_smoothed_quadrature(medium_kind):
    eps = 1.0 / 16
    x0 = np.array([0.5, 0.45, 0.52])
    rho0 = 1.3
    if medium_kind == "homogeneous":
        med = om.homogeneous(math.sqrt(3.0), 1.0, 1.3)
        grad = np.zeros(3)
    else:
        grad = np.array([0.3, -0.2, 0.25])
        med = om.linear(math.sqrt(3.0), 1.0, grad)

    def cb(Y, c0=1.0):
        return c0 * (1.0 + Y @ grad)

    src = om.point_source(eps, x0, M6, nq=3, qhalf=0.12, ndir=6, nshell=2, ricker=False, rho0=rho0)
    beams = om.point_source_beams(med, src)
    nq, ndir, nshell = 3, 6, 2
    Nq, Np = nq ** 3, ndir * nshell
    hq = 2 * 0.12 / nq
    dq = hq ** 3
    norm = (2 * math.pi * eps) ** -4.5
    # S beams (branch 1, SH) and P beams (branch 0) at a few (q, p)
    for lin in (5, Nq * 3 + 13, (2 * Np + 7) * Nq + 20):   # P "+", P "+" other p, SH "+"
        b = beams[beams["lineage"] == lin][0]
        br = int(b["branch"])
        cP = math.sqrt(3.0) * (1.0 + x0 @ grad)
        c0 = math.sqrt(3.0) if br == 0 else 1.0
        xs, ws = om.gauss_legendre(nshell, 0.2 * cP / (c0 * (1 + x0 @ grad)), 2.5 * cP / (c0 * (1 + x0 @ grad)))
        ip = (lin // Nq) % Np
        sh = ip // ndir
        np_ = xs[sh]
        dp = np_ ** 2 * ws[sh] * 4 * math.pi / ndir
        got = b["w"] / (dq * dp * norm)                        # psi of the closed form
        p = b["P"]
        refs = []
        for sigma in (0.006, 0.003):
            G = smoothed_source_fbi(med, lambda Y: cb(Y, c0), x0, M6, rho0, sigma, b["Q"], p, eps, sigma / 6)
            refs.append(two_way_psi(b, G, eps))
        e0, e1 = abs(got - refs[0]), abs(got - refs[1])
        assert 3.0 < e0 / e1 < 5.0               # O(sigma^2) approach to the closed form
        extrap = (4.0 * refs[1] - refs[0]) / 3.0  # Richardson: the sigma^2 term removed
        assert abs(got - extrap) <= 1e-3 * abs(got)
