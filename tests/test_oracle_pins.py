"""Pins of the CPU oracle against what the method and the mathematics fix.

Each test checks an oracle function against something other than itself:
closed-form solutions, invariants of the Hamiltonian flow, finite-difference
Jacobians, brute force, or convergence of a discretisation.  The paper
passages each one follows are named in the test docstrings.
"""
import math

import numpy as np
import pytest

import fga_inputs as fi
import oracle as om

A0 = 2.0 ** 1.5


def one_beam(q, p, branch=0, sigma=1, e=None):
    b = np.zeros(1, dtype=om.BEAM_DTYPE)
    b["Q"][0] = q
    b["P"][0] = p
    for i in range(3):
        b["ZQ"][0, i, i] = 1.0
        b["ZP"][0, i, i] = -1j
    if branch == 0:
        b["a"][0] = (A0, 0)
    elif branch == 1:
        b["a"][0] = (0, A0)
    else:
        b["a"][0] = (A0, 0)
    b["w"][0] = 1.0
    if e is None:
        e = [0.0, 0.0, 1.0]
    b["e"][0] = e
    b["branch"][0] = branch
    b["sigma"][0] = sigma
    b["alive"][0] = 1
    return b


BUMP = dict(cp=math.sqrt(3.0), cs=1.0, x0=(0.55, 0.45, 0.5), amp=0.3, s=0.2)


def bump():
    return om.bump(BUMP["cp"], BUMP["cs"], BUMP["x0"], BUMP["amp"], BUMP["s"])


# ---------------------------------------------------------------------------
# P1: FBI quadrature against the closed form for Gaussian-enveloped plane waves
# ---------------------------------------------------------------------------

def fbi_closed_form_1d(q, p, eps, c, w, k0):
    """int exp(-(y-c)^2/(2w^2) + i k0 y/eps - i p (y-q)/eps - (y-q)^2/(2 eps)) dy
    over the real line: exponent -A y^2 + B y + C0."""
    A = 1.0 / (2 * w * w) + 1.0 / (2 * eps)
    B = c / (w * w) + 1j * (k0 - p) / eps + q / eps
    C0 = -c * c / (2 * w * w) + 1j * p * q / eps - q * q / (2 * eps)
    return np.sqrt(np.pi / A) * np.exp(B * B / (4 * A) + C0)


def test_fbi_matches_closed_form():
    """eq:psi: the FBI weight of f = A(y) d exp(i k0.y/eps) is a product of
    three Gaussian integrals; the oracle's quadrature must reproduce it."""
    eps, w, c, k0 = 1.0 / 32, 0.1, (0.5, 0.5, 0.5), (1.0, 0.0, 0.0)
    d = fi.unit_vector(fi.rng(99, 1))
    ymesh = fi.cell_centred(96, -0.3, 1.3)
    f = fi.gaussian_plane_wave(ymesh, eps, c, w, k0, d)
    g = np.random.default_rng(5)
    q = 0.5 + 0.3 * (g.random((6, 3)) - 0.5)
    p = np.array(k0) + 0.6 * (g.random((6, 3)) - 0.5)
    F = om.fbi(f, ymesh, q, p, eps)
    for i in range(6):
        s = np.prod([fbi_closed_form_1d(q[i, k], p[i, k], eps, c[k], w, k0[k]) for k in range(3)])
        ref = d * s
        assert np.max(np.abs(F[i] - ref)) <= 1e-11 * np.max(np.abs(ref)) + 1e-300


# ---------------------------------------------------------------------------
# P2: homogeneous medium, closed-form straight rays and amplitudes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("branch", [0, 1, 2])
@pytest.mark.parametrize("sigma", [1, -1])
def test_homogeneous_closed_form(branch, sigma):
    """eq:char_plus/minus, eq:DzDt, eq:amp_P/SV/SH in a constant medium:
    Q = q + sigma c t p/|p|, P = p, dzQ = I - i sigma (c t/|p|)(I - pp^T/|p|^2),
    dzP = -i I, a = 2^{3/2}(1 - i sigma c t/(2|p|)) times the initial unit
    polarisation, S = 0.  All are linear in t, so RK4 is exact to rounding."""
    cp, cs = math.sqrt(3.0), 1.0
    med = om.homogeneous(cp, cs)
    q = np.array([0.3, 0.6, 0.45])
    p = np.array([1.1, -0.2, 0.35])
    b = one_beam(q, p, branch, sigma, e=[0, 0, 1])
    c = cp if branch == 0 else cs
    dt, n = 0.005, 100
    for step in range(1, n + 1):
        om.evolve(med, b, dt, 1)
        t = step * dt
        np_ = np.linalg.norm(p)
        ph = p / np_
        Qr = q + sigma * c * t * ph
        ZQr = np.eye(3) - 1j * sigma * (c * t / np_) * (np.eye(3) - np.outer(ph, ph))
        ar = A0 * (1 - 1j * sigma * c * t / (2 * np_))
        assert np.allclose(b["Q"][0], Qr, rtol=0, atol=1e-13)
        assert np.allclose(b["P"][0], p, rtol=0, atol=1e-13)
        assert np.allclose(b["ZQ"][0], ZQr, rtol=0, atol=1e-12)
        assert np.allclose(b["ZP"][0], -1j * np.eye(3), rtol=0, atol=1e-12)
        a_expect = [ar, 0] if branch in (0, 2) else [0, ar]
        assert np.allclose(b["a"][0], a_expect, rtol=0, atol=1e-12)
        assert abs(b["S"][0]) < 1e-13


# ---------------------------------------------------------------------------
# P4: Hamiltonian conservation and RK4 order
# ---------------------------------------------------------------------------

def H_of(med, b):
    sp = 0 if b["branch"][0] == 0 else 1
    c, _, _ = om.speed(med, sp, b["Q"])
    return c[0] * np.linalg.norm(b["P"][0])


@pytest.mark.parametrize("branch,sigma", [(0, 1), (1, -1), (2, 1)])
def test_hamiltonian_conserved_fourth_order(branch, sigma):
    """H = c(Q)|P| is constant along both flows (Sec. 2.2, remark after
    eq:char_minus); the RK4 drift must fall at least ~16x when dt halves
    (fourth order or better)."""
    med = bump()
    q, p = np.array([0.3, 0.4, 0.5]), np.array([1.0, 0.3, -0.1])
    errs = []
    for n in (25, 50, 100):
        b = one_beam(q, p, branch, sigma)
        H0 = H_of(med, b)
        om.evolve(med, b, 0.4 / n, n)
        errs.append(abs(H_of(med, b) - H0) / H0)
    assert errs[-1] < 1e-8
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 12 and r2 > 12, (errs, r1, r2)


# ---------------------------------------------------------------------------
# P5: symplecticity of the Jacobian, |det Z| >= 2^{3/2}, Z^{-1} dzQ symmetric
# ---------------------------------------------------------------------------

def jacobian(b):
    """Standard Jacobian d(Q,P)/d(q,p) from the oracle's dzQ, dzP, whose
    entries are (dzQ)[m][j] = d Q_j/d q_m - i d Q_j/d p_m."""
    ZQ, ZP = b["ZQ"][0], b["ZP"][0]
    Aq = ZQ.real.T         # dQ/dq
    Bp = -ZQ.imag.T        # dQ/dp
    Cq = ZP.real.T         # dP/dq
    Dp = -ZP.imag.T        # dP/dp
    return np.block([[Aq, Bp], [Cq, Dp]])


@pytest.mark.parametrize("branch,sigma", [(0, 1), (2, -1)])
def test_symplectic_and_Z_bounds(branch, sigma):
    """App. A: the flow map is canonical (eq:symplectic, eq:p1-p4), so
    J^T Omega J = Omega, Z Z^* - 2I is positive semidefinite (|det Z| >= 2^{3/2})
    and Z^{-1} dzQ is symmetric (the argument that m_{SH->SV} = 0)."""
    med = bump()
    b = one_beam(np.array([0.35, 0.5, 0.42]), np.array([0.9, -0.4, 0.2]), branch, sigma)
    Om = np.block([[np.zeros((3, 3)), np.eye(3)], [-np.eye(3), np.zeros((3, 3))]])
    for _ in range(8):
        om.evolve(med, b, 0.005, 20)
        J = jacobian(b)
        # RK4 is not a symplectic integrator: the defect is its O(dt^4) error
        assert np.max(np.abs(J.T @ Om @ J - Om)) < 2e-8
        Z = b["ZQ"][0] + 1j * b["ZP"][0]
        ev = np.linalg.eigvalsh(Z @ Z.conj().T - 2 * np.eye(3))
        assert ev.min() > -1e-9
        assert abs(np.linalg.det(Z)) >= 2 ** 1.5 * (1 - 1e-9)
        M = np.linalg.solve(Z, b["ZQ"][0])
        assert np.max(np.abs(M - M.T)) < 1e-9


# ---------------------------------------------------------------------------
# P6: amplitude identity and S-polarisation frame independence
# ---------------------------------------------------------------------------

def test_p_amplitude_identity():
    """eq:amp_P integrates exactly to a(t) = 2^{3/2} c(Q_t)/c(q) sqrt(det Z_t/8):
    sigma grad c.P/|P| = d/dt log c(Q) and tr(Z^{-1} dZ/dt) = d/dt log det Z."""
    for sigma in (1, -1):
        med = bump()
        q, p = np.array([0.3, 0.5, 0.5]), np.array([1.0, 0.2, 0.1])
        c0 = om.speed(med, 0, q)[0][0]
        errs = []
        for n in (60, 120):
            b = one_beam(q, p, 0, sigma)
            root_prev = math.sqrt(8.0) + 0j
            worst = 0.0
            for _ in range(n):
                om.evolve(med, b, 0.3 / n, 1)
                Z = b["ZQ"][0] + 1j * b["ZP"][0]
                r = np.sqrt(np.linalg.det(Z) + 0j)
                if abs(r - root_prev) > abs(-r - root_prev):
                    r = -r
                root_prev = r
                c = om.speed(med, 0, b["Q"][0])[0][0]
                expect = A0 * (c / c0) * r / math.sqrt(8.0)
                worst = max(worst, abs(b["a"][0][0] - expect) / abs(expect))
            errs.append(worst)
        # the identity holds for the exact flow; RK4 meets it to O(dt^4)
        assert errs[0] < 1e-8 and errs[0] / errs[1] > 12, errs


def test_s_polarisation_frame_independent():
    """eq:amp_SV/eq:amp_SH: the coupling term makes a_SV N_SV + a_SH N_SH
    independent of which perpendicular frame is used; the physical vector
    stays orthogonal to P and its norm follows the scalar factor of the P
    identity with c = c_S."""
    med = bump()
    q, p = np.array([0.3, 0.5, 0.48]), np.array([1.0, 0.25, 0.3])
    outs = []
    for e in ([0, 0, 1], [0, 1, 0], [1 / math.sqrt(2), 0, 1 / math.sqrt(2)]):
        b = one_beam(q, p, 2, 1, e=e)
        # common initial physical polarisation: the SV direction of frame e_z
        nsh = np.cross([0, 0, 1], p); nsh /= np.linalg.norm(nsh)
        nsv = np.cross(p / np.linalg.norm(p), nsh)
        fsh = np.cross(e, p); fsh /= np.linalg.norm(fsh)
        fsv = np.cross(p / np.linalg.norm(p), fsh)
        b["a"][0] = (A0 * np.dot(nsv, fsv), A0 * np.dot(nsv, fsh))
        om.evolve(med, b, 0.004, 100)
        outs.append((b.copy(), om.amplitude_vectors(b)[0]))
    A_ref = outs[0][1]
    for bb, A in outs[1:]:
        assert np.max(np.abs(A - A_ref)) < 1e-9 * np.linalg.norm(A_ref)
    b = outs[0][0]
    Ph = b["P"][0] / np.linalg.norm(b["P"][0])
    assert abs(np.dot(A_ref, Ph)) < 1e-12 * np.linalg.norm(A_ref)
    Z = b["ZQ"][0] + 1j * b["ZP"][0]
    c0 = om.speed(med, 1, q)[0][0]
    c = om.speed(med, 1, b["Q"][0])[0][0]
    scal = A0 * (c / c0) * abs(np.sqrt(np.linalg.det(Z) + 0j)) / math.sqrt(8.0)
    assert abs(np.linalg.norm(A_ref) - scal) < 1e-9 * scal


def test_reframe_keeps_polarisation():
    """Changing the reference axis rotates (a_SV, a_SH) but leaves the
    physical polarisation unchanged."""
    b = one_beam(np.zeros(3), np.array([0.05, 0.02, 1.0]), 2, 1, e=[0, 0, 1])
    b["a"][0] = (1.0 + 0.5j, -0.3 + 0.2j)
    A_before = om.amplitude_vectors(b)[0]
    om.reframe(b)
    assert list(b["e"][0]) == [1.0, 0.0, 0.0]
    A_after = om.amplitude_vectors(b)[0]
    assert np.max(np.abs(A_after - A_before)) < 1e-14


# ---------------------------------------------------------------------------
# P7: finite-difference Jacobian pins the variational equations and layout
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [1, -1])
def test_variational_matches_finite_differences(sigma):
    """eq:DzDt with eq:op_zZ_app: Re dzQ[m][j] = dQ_j/dq_m,
    -Im dzQ[m][j] = dQ_j/dp_m, and likewise for dzP, checked against central
    differences of neighbouring trajectories."""
    med = bump()
    q, p = np.array([0.32, 0.47, 0.55]), np.array([0.95, 0.3, -0.2])
    dt, n = 0.005, 80
    b = one_beam(q, p, 0, sigma)
    om.evolve(med, b, dt, n)
    h = 1e-5
    for m in range(3):
        for which in ("q", "p"):
            e = np.zeros(3); e[m] = h
            bp = one_beam(q + e, p, 0, sigma) if which == "q" else one_beam(q, p + e, 0, sigma)
            bm = one_beam(q - e, p, 0, sigma) if which == "q" else one_beam(q, p - e, 0, sigma)
            om.evolve(med, bp, dt, n)
            om.evolve(med, bm, dt, n)
            dQ = (bp["Q"][0] - bm["Q"][0]) / (2 * h)
            dP = (bp["P"][0] - bm["P"][0]) / (2 * h)
            if which == "q":
                eQ, eP = b["ZQ"][0][m].real, b["ZP"][0][m].real
            else:
                eQ, eP = -b["ZQ"][0][m].imag, -b["ZP"][0][m].imag
            assert np.max(np.abs(dQ - eQ)) < 1e-6
            assert np.max(np.abs(dP - eP)) < 1e-6


def test_minus_flow_reverses_plus_flow():
    """eq:char_minus is eq:char_plus with the right-hand side negated, so
    running "+" for time T then "-" for time T returns (Q, P), the
    Jacobians and a_P to their initial values (up to RK4 error)."""
    med = bump()
    q, p = np.array([0.4, 0.5, 0.45]), np.array([1.0, -0.3, 0.2])
    b = one_beam(q, p, 0, 1)
    om.evolve(med, b, 0.004, 100)
    b["sigma"][0] = -1
    om.evolve(med, b, 0.004, 100)
    assert np.max(np.abs(b["Q"][0] - q)) < 1e-9
    assert np.max(np.abs(b["P"][0] - p)) < 1e-9
    assert np.max(np.abs(b["ZQ"][0] - np.eye(3))) < 1e-8
    assert np.max(np.abs(b["ZP"][0] + 1j * np.eye(3))) < 1e-8
    assert abs(b["a"][0][0] - A0) < 1e-8


# ---------------------------------------------------------------------------
# P3: t = 0 recovery (decomposition + summation reproduce the initial data)
# ---------------------------------------------------------------------------

def sum_1d(x, qs, ps, hq, hp, eps, c, w, k0):
    """sum_{q,p} hq hp F(q,p) exp(i p (x-q)/eps - (x-q)^2/(2 eps)) in one
    dimension, F the closed-form 1-D FBI transform."""
    Q, Pm = np.meshgrid(qs, ps, indexing="ij")
    F = fbi_closed_form_1d(Q, Pm, eps, c, w, k0)
    out = []
    for xv in np.atleast_1d(x):
        out.append(np.sum(hq * hp * F * np.exp(1j * Pm * (xv - Q) / eps - (xv - Q) ** 2 / (2 * eps))))
    return np.array(out)


def test_recovery_normalisation_1d_fine_mesh():
    """eq:FGA with eq:psi, eq:alpha^k read with 1/(2kc|p|): on a resolved mesh
    the per-axis factor 2^{1/2}(2 pi eps)^{-3/2} sum_{q,p} F G returns the
    1-D data.  (With the printed |p|^3 the result would be off by |p|^-2.)"""
    eps, w, c, k0 = 1.0 / 64, 0.1, 0.5, 1.0
    hq = math.sqrt(eps) / 3
    qs = np.arange(-0.6, 1.6, hq)
    sp = fi.packet_momentum_spread(eps, w)
    hp = 2 * math.pi * eps / 4.0
    ps = k0 + np.arange(-7 * sp, 7 * sp, hp)
    x = np.linspace(0.35, 0.65, 7)
    got = math.sqrt(2.0) * (2 * math.pi * eps) ** -1.5 * sum_1d(x, qs, ps, hq, hp, eps, c, w, k0)
    ref = np.exp(-(x - c) ** 2 / (2 * w * w) + 1j * k0 * x / eps)
    assert np.max(np.abs(got - ref)) < 1e-8


def test_recovery_3d_equals_product_of_1d_sums():
    """With all three branches the projections sum to the identity
    (P/|P|, N_SH, N_SV orthonormal) and the box window is separable, so the
    oracle's 3-D beam sum at t = 0 must equal d times the product of the
    three 1-D sums of the previous test, times 2^{3/2}(2 pi eps)^{-9/2}."""
    eps, w, c, k0 = 1.0 / 16, 0.15, (0.5, 0.5, 0.5), (2.0, 0.0, 0.0)
    d = fi.unit_vector(fi.rng(98, 1))
    qmesh = fi.cell_centred(5, 0.1, 0.9)
    pmesh = fi.p_mesh_around(k0, eps, w, 4)
    iq, ip = np.meshgrid(np.arange(qmesh.count), np.arange(pmesh.count), indexing="xy")
    iq, ip = iq.ravel(), ip.ravel()
    qs, ps = qmesh.points()[iq], pmesh.points()[ip]
    Ft = np.empty((len(iq), 3), dtype=np.complex128)
    for i in range(len(iq)):
        s = np.prod([fbi_closed_form_1d(qs[i, k], ps[i, k], eps, c[k], w, k0[k]) for k in range(3)])
        Ft[i] = d * s
    beams = om.make_beams(qmesh, pmesh, Ft, eps, iq, ip, one_way=True)
    assert len(beams) == 3 * len(iq)
    x = 0.5 + 0.3 * (np.random.default_rng(3).random((12, 3)) - 0.5)
    tau = 3.0
    u, cnt = om.sum_points(beams, x, eps, tau)
    R = math.sqrt(2 * tau * eps)
    ref = np.empty_like(u)
    for i in range(len(x)):
        fac = 1.0 + 0j
        for k in range(3):
            qa, pa = qmesh.axis(k), pmesh.axis(k)
            qa = qa[np.abs(x[i, k] - qa) <= R]
            fac *= sum_1d(x[i, k], qa, pa, qmesh.h[k], pmesh.h[k], eps, c[k], w, k0[k])[0]
        ref[i] = d * fac * A0 * (2 * math.pi * eps) ** -4.5
    assert np.max(np.abs(u - ref)) < 1e-11 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# Summation window and brute force
# ---------------------------------------------------------------------------

def test_window_truncation_bound_and_count():
    """eq:FGA with the box window: dropping beams outside max|x-Q| <= sqrt(2 tau
    eps) changes each term by at most exp(-tau) relative; the number of terms
    counted equals the brute-force count of (beam, point) pairs in window."""
    w = fi.smooth_medium_packet(nq=4, np_=2, ny=16, nrec=0, nout=0, nmed=8)
    beams = om.decompose(w)
    om.evolve(om.homogeneous(w.cp0, w.cs0), beams, 0.01, 5)
    x = fi.uniform_points(40, np.random.default_rng(1))
    tau = 4.0
    u_w, cnt = om.sum_points(beams, x, w.eps, tau)
    u_all, cnt_all = om.sum_points(beams, x, w.eps, 1e9)
    assert cnt_all == len(beams) * len(x)
    R = math.sqrt(2 * tau * w.eps)
    inwin = np.all(np.abs(x[:, None, :] - beams["Q"][None, :, :]) <= R, axis=2)
    assert cnt == int(inwin.sum())
    bound = np.abs(beams["w"]).sum() * np.abs(om.amplitude_vectors(beams)).max() * math.exp(-tau)
    assert np.max(np.abs(u_w - u_all)) <= bound


# ---------------------------------------------------------------------------
# Gridded medium: trilinear interpolation of central-difference fields
# ---------------------------------------------------------------------------

def test_grid_medium_second_order():
    """The gridded-medium reading (periodic node values, central differences,
    trilinear interpolation) converges at second order to the analytic
    speed, gradient and Hessian of a smooth periodic field."""
    tp = 2 * math.pi

    def field(x, y, z):
        return 1.5 + 0.1 * np.sin(tp * x) * np.cos(tp * y) + 0.05 * np.sin(tp * (z + x))

    def exact(pts):
        x, y, z = pts.T
        c = field(x, y, z)
        g = np.stack([0.1 * tp * np.cos(tp * x) * np.cos(tp * y) + 0.05 * tp * np.cos(tp * (z + x)),
                      -0.1 * tp * np.sin(tp * x) * np.sin(tp * y),
                      0.05 * tp * np.cos(tp * (z + x))], axis=1)
        s = -tp * tp
        hxx = 0.1 * s * np.sin(tp * x) * np.cos(tp * y) + 0.05 * s * np.sin(tp * (z + x))
        hyy = 0.1 * s * np.sin(tp * x) * np.cos(tp * y)
        hzz = 0.05 * s * np.sin(tp * (z + x))
        hxy = -0.1 * tp * tp * np.cos(tp * x) * np.sin(tp * y)
        hxz = 0.05 * s * np.sin(tp * (z + x))
        hyz = np.zeros_like(x)
        H = np.stack([hxx, hxy, hxz, hxy, hyy, hyz, hxz, hyz, hzz], axis=1).reshape(-1, 3, 3)
        return c, g, H

    pts = np.random.default_rng(7).random((200, 3)) * 2.0 - 0.5   # includes periodic images
    errs = []
    for n in (16, 32, 64):
        mesh = fi.node_grid(n)
        ax = mesh.axis(0)
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
        med = om.grid(field(X, Y, Z), mesh, cs_ratio=0.5)
        c, g, H = om.speed(med, 0, pts)
        ce, ge, He = exact(np.mod(pts, 1.0))
        errs.append((np.abs(c - ce).max(), np.abs(g - ge).max(), np.abs(H - He).max()))
        cs, _, _ = om.speed(med, 1, pts)
        assert np.allclose(cs, 0.5 * c, rtol=1e-15, atol=0)
    for k in range(3):
        r = errs[1][k] / errs[2][k]
        assert 3.0 < r < 5.5, (k, errs)


# ---------------------------------------------------------------------------
# Station coordinates of the Earth examples (radius, longitude, latitude)
# ---------------------------------------------------------------------------

def test_spherical_station_coordinates():
    """The axes land where the coordinates name them, the radius is the
    distance from the centre, and the longitude and latitude are recovered
    by arctan2 and arcsin of the Cartesian point."""
    axes = om.spherical_to_cartesian([[1, 0, 0], [1, math.pi / 2, 0], [1, 0, math.pi / 2], [2, math.pi, 0],
                                      [3, -math.pi / 2, -math.pi / 2]])
    assert np.allclose(axes, [[1, 0, 0], [0, 1, 0], [0, 0, 1], [-2, 0, 0], [0, 0, -3]], atol=1e-15)
    g = np.random.default_rng(8)
    rtp = np.stack([g.uniform(0.2, 2.0, 50), g.uniform(-math.pi, math.pi, 50), g.uniform(-1.5, 1.5, 50)], axis=1)
    x = om.spherical_to_cartesian(rtp)
    assert np.allclose(np.linalg.norm(x, axis=1), rtp[:, 0], rtol=1e-14)
    assert np.allclose(np.arctan2(x[:, 1], x[:, 0]), rtp[:, 1], atol=1e-13)
    assert np.allclose(np.arcsin(x[:, 2] / rtp[:, 0]), rtp[:, 2], atol=1e-13)
