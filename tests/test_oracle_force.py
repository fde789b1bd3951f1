"""Pins of the point-force source (the accuracy experiment of Sec. 2.3,
eq:ex_homo) and of its closed-form solution (eq:ex_anal):

  - the oracle's beam weight, a Gaussian integral over the source time s
    done in closed form, equals the Gauss-Legendre quadrature in s of the
    impulsive two-way weights (eq:psi, eq:alpha^k with f = 0, pinned in
    test_oracle_twoway.py) of U(.; s), each launched from the point its
    beam centre passes at time s;
  - the closed-form displacement satisfies the elastic wave equation away
    from the source (fourth-order finite differences in x and t) and carries
    the source's strength: the traction over a small sphere around x0
    balances the applied force d F(t).
"""
import math

import numpy as np

import fga_inputs as fi
import oracle as om
import point_force_exact as pfe

CP, CS, RHO = math.sqrt(3.0), 1.0, 1.0
OMEGA, T0, WIDTH = 64.0, 0.01, 0.05
X0, D = (0.5, 0.5, 0.5), (1.0, -0.5, 0.7)


def test_force_weight_is_time_integral_of_impulse_weights():
    eps, t_ref = 1.0 / 64, -0.004
    med = om.homogeneous(CP, CS, RHO)
    src = om.point_force(eps, X0, D, nq=5, qhalf=0.3, ndir=12, nshell=3, omega=OMEGA, t0=T0, width=WIDTH,
                         t_ref=t_ref, shell_lo=0.4, shell_hi=1.6)
    beams = om.point_force_beams(med, src)
    nq, Nq, Np = 5, 125, 36
    hq = 0.6 / nq
    g = np.random.default_rng(6)
    sv, sw = np.polynomial.legendre.leggauss(400)
    lo, hi = -T0 - 8 * WIDTH, -T0 + 8 * WIDTH
    s = 0.5 * (lo + hi) + 0.5 * (hi - lo) * sv
    ws = 0.5 * (hi - lo) * sw
    checked = 0
    for k in g.choice(len(beams), size=40, replace=False):
        b = beams[k]
        br, sg = int(b["branch"]), int(b["sigma"])
        c = CP if br == 0 else CS
        p = b["P"]
        ph = p / np.linalg.norm(p)
        lin = int(b["lineage"])
        ip = (lin // Nq) % Np
        xs, wsh = om.gauss_legendre(3, 0.4 * CP / c, 1.6 * CP / c)
        dp = np.linalg.norm(p) ** 2 * wsh[ip // 12] * 4 * math.pi / 12
        psi_closed = b["w"] / (hq ** 3 * dp * (2 * math.pi * eps) ** -4.5)
        # impulse weights of U(.; s_j) at the points q' + sigma c (s_j - t_ref) p/|p|
        qs = b["Q"][None, :] + sg * c * (s - t_ref)[:, None] * ph[None, :]
        Dv = np.asarray(X0)[None, :] - qs
        K = np.exp(-1j * (Dv @ p) / eps - np.sum(Dv * Dv, axis=1) / (2 * eps))   # FBI of delta(. - x0)
        Fs = pfe.source_time_function(s, OMEGA, T0, WIDTH)
        G = (Fs * K / (RHO * c))[:, None] * np.asarray(D)[None, :]
        Gt = np.zeros((len(s), 2, 3), dtype=np.complex128)
        Gt[:, 0 if br == 0 else 1] = G
        qm = fi.Mesh3((1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
        psi_s = np.empty(len(s), dtype=np.complex128)
        for j in range(len(s)):
            qm.lo = tuple(qs[j])
            pm = fi.Mesh3((1, 1, 1), tuple(p), (1.0, 1.0, 1.0))
            bb = om.make_beams(qm, pm, np.zeros((1, 3), dtype=np.complex128), eps, np.array([0]), np.array([0]),
                               one_way=False, Gt=Gt[j:j + 1], branch_mask=1 << br)
            psi_s[j] = bb[bb["sigma"] == sg]["w"][0] * (2 * math.pi * eps) ** 4.5
        quad = np.sum(ws * psi_s)
        scale = max(abs(quad), 1e-30)
        if abs(quad) < 1e-12 * np.abs(beams["w"]).max() / (hq ** 3 * dp * (2 * math.pi * eps) ** -4.5):
            continue
        assert abs(psi_closed - quad) <= 1e-9 * scale, (k, psi_closed, quad)
        checked += 1
    assert checked >= 20


def fd4(f, h):
    """Fourth-order central second derivative of f(shift) at 0."""
    return (-f(2 * h) + 16 * f(h) - 30 * f(0.0) + 16 * f(-h) - f(-2 * h)) / (12 * h * h)


def d1(f, y, k, h):
    """Fourth-order central first derivative of f (points -> values) along axis k."""
    e = np.eye(3)[k] * h
    return (-f(y + 2 * e) + 8 * f(y + e) - 8 * f(y - e) + f(y - 2 * e)) / (12 * h)


def test_exact_solution_satisfies_wave_equation():
    """rho u_tt = (lambda + mu) grad div u + mu Lap u at points 0.01..0.3
    from the source, with lambda = rho (c_P^2 - 2 c_S^2), mu = rho c_S^2;
    the residual is below 1e-5 of the terms (fourth-order differences)."""
    lam, mu = RHO * (CP * CP - 2 * CS * CS), RHO * CS * CS
    g = np.random.default_rng(2)
    dirs = g.standard_normal((24, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    r = np.geomspace(0.01, 0.3, 24)
    x = np.asarray(X0) + r[:, None] * dirs
    t, h, ht = 0.12, 1e-4, 1e-4

    def u(y, tt=t):
        return pfe.displacement(y, tt, X0, D, CP, CS, RHO, OMEGA, T0, WIDTH, nodes=128)

    utt = fd4(lambda e: u(x, t + e), ht)
    lap = sum(fd4(lambda e, k=k: u(x + e * np.eye(3)[k]), h) for k in range(3))

    def div(y):
        return sum(d1(lambda z, k=k: u(z)[:, k], y, k, h) for k in range(3))

    gd = np.stack([d1(div, x, i, h) for i in range(3)], axis=1)
    res = RHO * utt - (lam + mu) * gd - mu * lap
    scale = np.linalg.norm(RHO * utt, axis=1) + np.linalg.norm(mu * lap, axis=1)
    assert np.max(np.linalg.norm(res, axis=1) / scale) < 1e-5


def test_exact_solution_carries_the_source_strength():
    """The traction sigma.n integrated over a sphere of radius 2e-4 around x0
    balances the force: int sigma.n dS = -d F(t) (the enclosed inertia is
    O((k r)^2) smaller), at three times."""
    lam, mu = RHO * (CP * CP - 2 * CS * CS), RHO * CS * CS
    r0, h = 2e-4, 1e-6
    n = om.fibonacci_dirs(2000)       # equal-area points on the unit sphere
    x = np.asarray(X0) + r0 * n
    for t in (-0.01, 0.0, 0.02):
        def u(y):
            return pfe.displacement(y, t, X0, D, CP, CS, RHO, OMEGA, T0, WIDTH, nodes=64)

        J = np.stack([d1(u, x, k, h) for k in range(3)], axis=2)     # J[:, i, k] = d u_i / d x_k
        divu = J[:, 0, 0] + J[:, 1, 1] + J[:, 2, 2]
        sig = lam * divu[:, None, None] * np.eye(3)[None] + mu * (J + np.transpose(J, (0, 2, 1)))
        trac = np.einsum("pik,pk->pi", sig, n)
        total = trac.mean(axis=0) * 4 * math.pi * r0 * r0
        f = np.asarray(D) * pfe.source_time_function(t, OMEGA, T0, WIDTH)
        assert np.linalg.norm(total + f) <= 2e-3 * np.linalg.norm(f), (t, total, f)
