"""Pins of the oracle's interface step (Sec. 3.1: eq:p:int, eq:Yilmaz,
eq:Inter_DzQDzP) against what physics and the mathematics fix, independently
of how the oracle sets the problem up:

  - the outgoing plane waves satisfy continuity of displacement and traction,
    re-evaluated here in global coordinates from the 3-D stress tensor;
  - energy flux through the interface balances (pre-critical incidence);
  - no contrast gives pure transmission; normal incidence gives the
    impedance formulas;
  - Snell: frequency H and tangential momentum are preserved;
  - the printed Zoeppritz matrix (with its last right-hand-side entry read as
    sin 2 theta_r) gives the same coefficient magnitudes after conversion
    from potential to displacement normalisation;
  - the mapped (dzQ, dzP) equal finite-difference Jacobians of neighbouring
    rays that cross the interface, and stay symplectic.
"""
import math

import numpy as np
import pytest

import oracle as om

A0 = 2.0 ** 1.5


def medium(geometry=0, bounds=(0.5,), cp=(1.7, 2.2), cs=(1.0, 1.25), rho=(1.0, 1.3), grad=None):
    return om.layered(geometry, list(bounds), list(cp), list(cs), list(rho), grad=grad)


def lame(cp, cs, rho):
    return rho * (cp * cp - 2 * cs * cs), rho * cs * cs


def traction(P, A, lam, mu, n):
    """sigma.n of the plane wave A exp(i P.x/eps), the common factor i/eps dropped."""
    div = np.dot(P, A)
    grad = np.outer(P, A)   # d_i u_j -> P_i A_j
    sig = lam * div * np.eye(3) + mu * (grad + grad.T)
    return sig @ n


def incident(sp, theta, phi=0.3, pol=None):
    """Unit momentum at angle theta to +z (azimuth phi) and an amplitude vector."""
    P = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
    if sp == 0:
        return P, (1.0 + 0.5j) * P
    # S: a polarisation orthogonal to P
    a = np.cross(P, [0.3, -0.7, 0.2])
    a /= np.linalg.norm(a)
    b = np.cross(P, a)
    if pol is None:
        pol = (0.8 - 0.2j, 0.6 + 0.3j)
    return P, pol[0] * a + pol[1] * b


def check_boundary(med_args, sp, P, A, normal=(0, 0, 1.0)):
    cp, cs, rho = med_args["cp"], med_args["cs"], med_args["rho"]
    med = medium(**med_args)
    n = np.asarray(normal, dtype=float)
    md = om.interface_modes(med, 0, 1, n, sp, P, A)
    lam = [lame(cp[i], cs[i], rho[i])[0] for i in range(2)]
    mu = [lame(cp[i], cs[i], rho[i])[1] for i in range(2)]
    u1 = A.astype(complex).copy()
    t1 = traction(P, A, lam[0], mu[0], n)
    u2 = np.zeros(3, complex)
    t2 = np.zeros(3, complex)
    for m in md:
        assert m["exists"]
        if m["side"] == 0:
            u1 += m["A"]
            t1 += traction(m["P"], m["A"], lam[0], mu[0], n)
        else:
            u2 += m["A"]
            t2 += traction(m["P"], m["A"], lam[1], mu[1], n)
    scale = np.linalg.norm(A) * (1 + np.linalg.norm(P) * max(lam + mu))
    assert np.linalg.norm(u1 - u2) <= 1e-13 * scale
    assert np.linalg.norm(t1 - t2) <= 1e-13 * scale
    return md


MEDIA = [dict(cp=(1.7, 2.2), cs=(1.0, 1.25), rho=(1.0, 1.3)),
         dict(cp=(2.2, 1.7), cs=(1.25, 1.0), rho=(1.3, 1.0)),
         dict(cp=(1.7, 1.9), cs=(1.0, 0.9), rho=(1.0, 1.15))]


@pytest.mark.parametrize("mi", range(len(MEDIA)))
@pytest.mark.parametrize("sp", [0, 1])
def test_boundary_conditions_and_energy(mi, sp):
    """Pre-critical incidence: the four outgoing plane waves with the incident
    one satisfy u and sigma.n continuity; the normal energy flux
    rho c cos(angle) |A|^2 balances; H and the tangential momentum are kept."""
    args = MEDIA[mi]
    cp, cs, rho = args["cp"], args["cs"], args["rho"]
    c_in = cp[0] if sp == 0 else cs[0]
    for theta in (0.05, 0.25, 0.45):
        P, A = incident(sp, theta)
        # pre-critical for every mode in these media at these angles
        md = check_boundary(args, sp, P, A)
        H = c_in * np.linalg.norm(P)
        flux_in = rho[0] * c_in * abs(P[2]) / np.linalg.norm(P) * np.vdot(A, A).real
        flux_out = 0.0
        for m in md:
            side = m["side"]
            c = (cp if m["sp"] == 0 else cs)[side]
            Pm = m["P"]
            assert abs(c * np.linalg.norm(Pm) - H) <= 1e-14 * H
            assert np.allclose(Pm[:2], P[:2], rtol=0, atol=1e-15)
            assert (Pm[2] > 0) == (side == 1)
            flux_out += rho[side] * c * abs(Pm[2]) / np.linalg.norm(Pm) * np.vdot(m["A"], m["A"]).real
            # polarisation: P modes along P, S modes orthogonal to it
            if m["sp"] == 0:
                assert np.linalg.norm(np.cross(Pm, m["A"])) <= 1e-13 * np.linalg.norm(Pm) * (1 + abs(m["A"]).max())
            else:
                assert abs(np.dot(Pm, m["A"])) <= 1e-13 * np.linalg.norm(Pm) * (1 + abs(m["A"]).max())
        assert abs(flux_out - flux_in) <= 1e-12 * flux_in


@pytest.mark.parametrize("sp", [0, 1])
def test_no_contrast_is_transparent(sp):
    args = dict(cp=(1.7, 1.7), cs=(1.0, 1.0), rho=(1.1, 1.1))
    P, A = incident(sp, 0.4)
    md = check_boundary(args, sp, P, A)
    for k, m in enumerate(md):
        if k == 2 + sp:
            assert np.allclose(m["A"], A, atol=1e-14)
            assert np.allclose(m["P"], P, atol=1e-15)
        else:
            assert np.linalg.norm(m["A"]) <= 1e-14


def test_normal_incidence_impedances():
    args = MEDIA[0]
    cp, cs, rho = args["cp"], args["cs"], args["rho"]
    med = medium(**args)
    z = np.array([0, 0, 1.0])
    # P: displacement along P for each mode, so the reflected one points down
    md = om.interface_modes(med, 0, 1, z, 0, z, z.astype(complex))
    Z1, Z2 = rho[0] * cp[0], rho[1] * cp[1]
    assert abs(-md[0]["A"][2] - (Z2 - Z1) / (Z1 + Z2)) <= 1e-15
    assert abs(md[2]["A"][2] - 2 * Z1 / (Z1 + Z2)) <= 1e-15
    assert np.linalg.norm(md[1]["A"]) <= 1e-15 and np.linalg.norm(md[3]["A"]) <= 1e-15
    # S polarised along x: no sign flip of the transverse displacement
    x = np.array([1.0 + 0j, 0, 0])
    md = om.interface_modes(med, 0, 1, z, 1, z, x)
    Z1, Z2 = rho[0] * cs[0], rho[1] * cs[1]
    assert abs(md[1]["A"][0] - (Z1 - Z2) / (Z1 + Z2)) <= 1e-15
    assert abs(md[3]["A"][0] - 2 * Z1 / (Z1 + Z2)) <= 1e-15
    assert np.linalg.norm(md[0]["A"]) <= 1e-15 and np.linalg.norm(md[2]["A"]) <= 1e-15


def printed_zoeppritz(theta_i, cp, cs, rho):
    """The P-incidence system as printed (potential normalisation), with the
    last right-hand-side entry read as sin(2 theta_r)."""
    a1, a2 = cp
    b1, b2 = cs
    p = math.sin(theta_i) / a1
    th_r = theta_i
    ph_r = math.asin(p * b1)
    th_t = math.asin(p * a2)
    ph_t = math.asin(p * b2)
    r = rho[1] / rho[0]
    M = np.array([
        [math.cos(th_r), a1 / b1 * math.sin(ph_r), a1 / a2 * math.cos(th_t), -a1 / b2 * math.sin(ph_t)],
        [-math.sin(th_r), a1 / b1 * math.cos(ph_r), a1 / a2 * math.sin(th_t), a1 / b2 * math.cos(ph_t)],
        [-math.cos(2 * ph_r), -math.sin(2 * ph_r), r * math.cos(2 * ph_t), -r * math.sin(2 * ph_t)],
        [math.sin(2 * th_r), -(a1 / b1) ** 2 * math.cos(2 * ph_r), r * (a1 * b2) ** 2 / (a2 * b1) ** 2 * math.sin(2 * th_t),
         r * a1 ** 2 / b1 ** 2 * math.cos(2 * ph_t)]])
    rhs = np.array([math.cos(th_r), math.sin(th_r), math.cos(2 * ph_r), math.sin(2 * th_r)])
    return np.linalg.solve(M, rhs)


@pytest.mark.parametrize("theta", [0.1, 0.3, 0.5])
def test_printed_zoeppritz_magnitudes(theta):
    """|coefficients| of the printed system, converted by c_in / c_out from
    potential to displacement amplitude, equal the oracle's |A_out| / |A_in|."""
    args = MEDIA[2]
    cp, cs, rho = args["cp"], args["cs"], args["rho"]
    x = printed_zoeppritz(theta, cp, cs, rho)
    P, A = incident(0, theta, phi=0.0)
    md = om.interface_modes(medium(**args), 0, 1, np.array([0, 0, 1.0]), 0, P, A)
    ain = np.linalg.norm(A)
    speeds = [cp[0], cs[0], cp[1], cs[1]]
    for k in range(4):
        got = np.linalg.norm(md[k]["A"]) / ain
        want = abs(x[k]) * cp[0] / speeds[k]
        assert abs(got - want) <= 1e-12 * max(1.0, want), (k, got, want)


def test_post_critical_drops_evanescent_mode():
    """Past the P critical angle into a faster layer no transmitted P beam is
    made; the surviving coefficients turn complex and still satisfy the
    boundary conditions with the evanescent wave included (checked through
    the energy balance: the evanescent wave carries no normal flux)."""
    args = MEDIA[0]
    cp, cs, rho = args["cp"], args["cs"], args["rho"]
    theta = math.asin(cp[0] / cp[1]) + 0.1
    P, A = incident(0, theta)
    md = om.interface_modes(medium(**args), 0, 1, np.array([0, 0, 1.0]), 0, P, A)
    assert not md[2]["exists"] and md[0]["exists"] and md[1]["exists"] and md[3]["exists"]
    flux_in = rho[0] * cp[0] * abs(P[2]) * np.vdot(A, A).real
    flux = 0.0
    for k in (0, 1, 3):
        m = md[k]
        c = (cp if m["sp"] == 0 else cs)[m["side"]]
        flux += rho[m["side"]] * c * abs(m["P"][2]) / np.linalg.norm(m["P"]) * np.vdot(m["A"], m["A"]).real
    assert abs(flux - flux_in) <= 1e-12 * flux_in
    assert abs(np.angle(md[0]["A"][2])) > 1e-3   # a phase shift appears


@pytest.mark.parametrize("sp,theta", [(0, 0.0), (0, 0.4), (0, 1.2), (1, 0.3), (1, 0.5), (1, 0.9)])
def test_free_surface_is_traction_free(sp, theta):
    """At a traction-free surface the incident plus reflected plane waves
    exert no traction (re-evaluated from the 3-D stress tensor, before the
    critical angle, where every reflected wave propagates); no wave is
    transmitted; the reflected energy flux equals the incident one (past the
    critical angle the evanescent P carries none); normal P incidence
    reflects P alone with the same displacement (the surface doubles it)."""
    cp, cs, rho = 1.7, 1.0, 1.3
    med = om.layered(0, [], [cp], [cs], [rho], surface=0.8)
    lam, mu = lame(cp, cs, rho)
    P, A = incident(sp, theta)
    P = P * (1.0 / (cp if sp == 0 else cs))
    n = np.array([0, 0, 1.0])
    md = om.free_surface_modes(med, 0, n, sp, P, A)
    assert not md[2]["exists"] and not md[3]["exists"]
    c_in = cp if sp == 0 else cs
    flux_in = rho * c_in * abs(P[2]) / np.linalg.norm(P) * np.vdot(A, A).real
    flux = sum(rho * (cp if m["sp"] == 0 else cs) * abs(m["P"][2]) / np.linalg.norm(m["P"]) * np.vdot(m["A"], m["A"]).real
               for m in md[:2] if m["exists"])
    assert abs(flux - flux_in) <= 1e-12 * flux_in     # past the critical angle the evanescent P carries none
    if all(m["exists"] for m in md[:2]):
        t = traction(P, A, lam, mu, n)
        for m in md[:2]:
            t = t + traction(m["P"], m["A"], lam, mu, n)
        scale = np.linalg.norm(A) * np.linalg.norm(P) * (lam + 2 * mu)
        assert np.linalg.norm(t) <= 1e-13 * scale
    if sp == 0 and theta == 0.0:
        assert np.linalg.norm(md[1]["A"]) <= 1e-14
        assert abs(abs(md[0]["A"][2]) - abs(A[2])) <= 1e-14 * abs(A[2])
        assert abs((A[2] + md[0]["A"][2]) - 2 * A[2]) <= 1e-14 * abs(A[2])


def one_beam(q, p, branch, sigma=1, layer=0):
    b = np.zeros(1, dtype=om.BEAM_DTYPE)
    b["Q"][0] = q
    b["P"][0] = p
    for i in range(3):
        b["ZQ"][0, i, i] = 1.0
        b["ZP"][0, i, i] = -1j
    b["a"][0] = (A0, 0.3j) if branch else (A0, 0)
    b["w"][0] = 1.0
    b["e"][0] = [0.0, 0.0, 1.0] if abs(p[2]) / np.linalg.norm(p) <= math.cos(math.radians(20)) else [1.0, 0, 0]
    b["branch"][0] = branch
    b["sigma"][0] = sigma
    b["layer"][0] = layer
    b["alive"][0] = 1
    b["lineage"][0] = 5
    return b


def child_of(out, lineage):
    sel = out[out["lineage"] == lineage]
    assert len(sel) == 1
    return sel[0]


@pytest.mark.parametrize("grad", [False, True])
@pytest.mark.parametrize("geometry", [0, 1])
@pytest.mark.parametrize("branch,k", [(0, 2), (0, 0), (0, 3), (2, 3), (2, 1)])
def test_interface_jacobian_fd(geometry, branch, k, grad):
    """dzQ and dzP of a child (mapped by eq:Inter_DzQDzP with F and W = F^-T,
    plus the curvature term of a spherical interface) against central
    differences of the child's Q and P over neighbouring initial (q, p), all
    crossing in the same step: d/dq = Re dz, d/dp = -Im dz, within 1e-6 on
    the plane and on the sphere, several steps after the crossing; the
    symplectic identities hold after the map.  With grad, both layers have
    linear speeds (c = c_i (1 + g_i v), v = z or |x|): curved rays, the
    crossing found by secant iterations and the gradient terms of the map."""
    if geometry == 0:
        med = medium(0, (0.5,), grad=[0.3, -0.4] if grad else None)
        q0 = np.array([0.3, 0.4, 0.47])
        p0 = np.array([0.35, -0.2, 1.0])
        nsteps, dt = 6, 0.01
        layer = 0
    else:
        med = medium(1, (0.6,), grad=[0.25, 0.35] if grad else None)
        q0 = np.array([0.05, 0.1, 0.66])
        p0 = np.array([0.2, 0.35, -1.0])
        nsteps, dt = 10, 0.01
        layer = 0
    p0 = p0 / np.linalg.norm(p0) * 1.3
    out, _ = om.evolve_layered(med, one_beam(q0, p0, branch, layer=layer), dt, nsteps)
    lin = om.child_lineage(5, 0, k)
    c = child_of(out, lin)
    assert c["gen"] == 1
    h = 1e-5
    dQq = np.zeros((3, 3)); dQp = np.zeros((3, 3)); dPq = np.zeros((3, 3)); dPp = np.zeros((3, 3))
    for m in range(3):
        for which in ("q", "p"):
            res = []
            for s in (1, -1):
                q, p = q0.copy(), p0.copy()
                if which == "q":
                    q[m] += s * h
                else:
                    p[m] += s * h
                o, _ = om.evolve_layered(med, one_beam(q, p, branch, layer=layer), dt, nsteps)
                res.append(child_of(o, lin))
            dq = (res[0]["Q"] - res[1]["Q"]) / (2 * h)
            dp = (res[0]["P"] - res[1]["P"]) / (2 * h)
            if which == "q":
                dQq[m], dPq[m] = dq, dp
            else:
                dQp[m], dPp[m] = dq, dp
    tol = 1e-6
    assert np.abs(c["ZQ"].real - dQq).max() <= tol
    assert np.abs(-c["ZQ"].imag - dQp).max() <= tol
    assert np.abs(c["ZP"].real - dPq).max() <= tol
    assert np.abs(-c["ZP"].imag - dPp).max() <= tol
    # symplectic structure after the map (P5 / P8); in gradient layers RK4,
    # which is not a symplectic scheme, leaves its truncation error in it
    ZQ, ZP = c["ZQ"], c["ZP"]
    stol = 1e-8 if grad else 1e-12
    assert np.abs(ZQ @ ZP.T - ZP @ ZQ.T).max() <= stol
    Z = ZQ + 1j * ZP
    S = np.linalg.solve(Z, ZQ)
    assert np.abs(S - S.T).max() <= stol


@pytest.mark.parametrize("geometry", [0, 1])
@pytest.mark.parametrize("branch,k", [(0, 0), (0, 1), (2, 1), (2, 0)])
def test_free_surface_jacobian_fd(geometry, branch, k):
    """Children reflected at a free surface (plane z = 0.5 or sphere |x| =
    0.6 around a gradient layer): dzQ, dzP equal finite differences of
    neighbouring rays (1e-6), as at an interface."""
    if geometry == 0:
        med = om.layered(0, [], [1.7], [1.0], [1.0], grad=[0.3], surface=0.5)
        q0 = np.array([0.3, 0.4, 0.47])
        p0 = np.array([0.35, -0.2, 1.0])
        nsteps, dt = 6, 0.01
    else:
        med = om.layered(1, [], [1.7], [1.0], [1.0], surface=0.6)
        q0 = np.array([0.05, 0.1, 0.55])
        p0 = np.array([0.2, 0.35, 1.0])
        nsteps, dt = 10, 0.01
    p0 = p0 / np.linalg.norm(p0) * 1.3
    out, _ = om.evolve_layered(med, one_beam(q0, p0, branch), dt, nsteps)
    lin = om.child_lineage(5, 0, k)
    c = child_of(out, lin)
    assert c["gen"] == 1 and c["layer"] == 0
    h = 1e-5
    d = {}
    for m in range(3):
        for which in ("q", "p"):
            res = []
            for sgn in (1, -1):
                q, p = q0.copy(), p0.copy()
                (q if which == "q" else p)[m] += sgn * h
                o, _ = om.evolve_layered(med, one_beam(q, p, branch), dt, nsteps)
                res.append(child_of(o, lin))
            d[(which, m)] = ((res[0]["Q"] - res[1]["Q"]) / (2 * h), (res[0]["P"] - res[1]["P"]) / (2 * h))
    dQq = np.array([d[("q", m)][0] for m in range(3)])
    dPq = np.array([d[("q", m)][1] for m in range(3)])
    dQp = np.array([d[("p", m)][0] for m in range(3)])
    dPp = np.array([d[("p", m)][1] for m in range(3)])
    assert np.abs(c["ZQ"].real - dQq).max() <= 1e-6
    assert np.abs(-c["ZQ"].imag - dQp).max() <= 1e-6
    assert np.abs(c["ZP"].real - dPq).max() <= 1e-6
    assert np.abs(-c["ZP"].imag - dPp).max() <= 1e-6


def test_sphere_curvature_term_is_needed():
    """On a sphere the flat map alone (curvature 0) misses the turning of the
    normal: at the crossing its dzP differs from the map with the curvature
    term by O(|mu| |dzQ| / R), far beyond the 1e-6 of the finite-difference
    pin above; on a plane the two coincide."""
    Pin = np.array([0.2, 0.35, -1.0])
    Pin = Pin / np.linalg.norm(Pin) * 1.3
    x = np.array([0.05, 0.1, 0.0])
    x[2] = math.sqrt(0.6 ** 2 - x[0] ** 2 - x[1] ** 2)
    n = x / 0.6                      # outward motion into the outer layer (curvature +1/R)
    n = -n if np.dot(Pin, n) < 0 else n
    kc = (1.0 if np.dot(n, x) > 0 else -1.0) / 0.6
    c_in, c_out = 1.7, 2.2
    pt = Pin - np.dot(Pin, n) * n
    pno = math.sqrt((c_in / c_out) ** 2 * np.dot(Pin, Pin) - np.dot(pt, pt))
    Pout = pt + pno * n
    ZQ = np.eye(3, dtype=np.complex128)
    ZP = -1j * np.eye(3, dtype=np.complex128)
    _, zp_flat = om.interface_jacobians(n, Pin, Pout, c_in, c_out, ZQ, ZP)
    _, zp_curv = om.interface_jacobians(n, Pin, Pout, c_in, c_out, ZQ, ZP, kcurv=kc)
    assert np.abs(zp_curv - zp_flat).max() > 1e-2
    _, zp_plane = om.interface_jacobians(n, Pin, Pout, c_in, c_out, ZQ, ZP, kcurv=0.0)
    assert np.array_equal(zp_plane, zp_flat)


def test_modes_take_the_local_speeds():
    """In linear-gradient layers the boundary problem at a crossing point x
    is that of constant layers with the speeds each layer has at x."""
    grad = [0.3, -0.4]
    x = np.array([0.2, 0.7, 0.5])
    med = medium(0, (0.5,), grad=grad)
    cp, cs = (1.7, 2.2), (1.0, 1.25)
    loc = medium(0, (0.5,), cp=[c * (1 + g * x[2]) for c, g in zip(cp, grad)],
                 cs=[c * (1 + g * x[2]) for c, g in zip(cs, grad)])
    P = np.array([0.3, -0.2, 1.1])
    A = (P / np.linalg.norm(P)).astype(np.complex128)
    a = om.interface_modes(med, 0, 1, np.array([0, 0, 1.0]), 0, P, A, x=x)
    b = om.interface_modes(loc, 0, 1, np.array([0, 0, 1.0]), 0, P, A)
    for k in range(4):
        assert a[k]["exists"] == b[k]["exists"]
        assert np.allclose(a[k]["P"], b[k]["P"], rtol=0, atol=1e-14)
        assert np.allclose(a[k]["A"], b[k]["A"], rtol=0, atol=1e-14)


def test_gradient_layer_ray_keeps_frequency():
    """Inside a linear-gradient layer the ray bends and H = c(Q)|P| stays
    fixed (to the RK4 error), on a plane and on a sphere."""
    for geometry, bounds, grad, q0, p0 in ((0, (0.9,), [0.5, 0.0], [0.3, 0.4, 0.1], [0.8, 0.1, 1.0]),
                                           (1, (0.2,), [0.4, 0.0], [0.1, 0.5, 0.3], [1.0, -0.3, 0.2])):
        med = medium(geometry, bounds, grad=grad)
        b = one_beam(np.array(q0), np.array(p0), 0)
        H0 = om.speed(med, 0, b["Q"])[0][0] * np.linalg.norm(b["P"][0])
        out, _ = om.evolve_layered(med, b, 0.005, 60)
        c = out[0]
        assert c["layer"] == 0 and c["alive"] == 1
        H1 = om.speed(med, 0, c["Q"][None])[0][0] * np.linalg.norm(c["P"])
        assert abs(H1 - H0) <= 1e-9 * H0
        assert np.linalg.norm(np.cross(c["P"], b["P"][0])) > 1e-3      # the ray has turned


def test_generation_cap_and_lineage():
    """A beam bouncing in a slab splits at every hit until the generation cap;
    lineage numbers are unique and encode the generation."""
    med = om.layered(0, [0.3, 0.7], [1.7, 2.3, 1.7], [1.0, 1.3, 1.0], [1.0, 1.4, 1.0])
    b = one_beam([0.5, 0.5, 0.5], np.array([0.2, 0.1, 1.0]), 0, layer=1)
    out, ncap = om.evolve_layered(med, b, 0.01, 200, gmax=2)
    assert len(np.unique(out["lineage"])) == len(out)
    assert ncap > 0
    assert out["gen"].max() == 2
    assert np.all((out["lineage"] >> 58) == out["gen"])
    alive = out[out["alive"] == 1]
    assert np.all(alive["gen"] <= 2)
    # every live beam sits in the layer its centre is in
    for bb in alive:
        z = bb["Q"][2]
        L = 0 if z < 0.3 else (1 if z < 0.7 else 2)
        assert bb["layer"] == L or abs(z - 0.3) < 1e-12 or abs(z - 0.7) < 1e-12
