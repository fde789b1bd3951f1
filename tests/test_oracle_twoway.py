"""Pins of the oracle's two-way decomposition weight (Sec. 2.1, eq:psi with
eq:alpha^k read with prefactor 1/(2 k c |p|)):

    psi_{b,+-} = (1/2) FBI[f].n_b +- (i eps / (2|p|)) FBI[g / c_b].n_b.

Neither coefficient is checked by retyping it.  They are fixed by what the
initial-value problem eq:ini demands of the summation formula eq:FGA:

  - at t = 0 the sum over both directions returns u(0) = f (the g-terms cancel
    between the two directions, the 1/2 on f does not);
  - its time derivative at t = 0, taken by central differences of RK4 steps
    of +-dt, returns u_t(0) = g (this fixes the g-coefficient's size, sign and
    power of |p|);
  - for a pure-P field f with g = -i c_P |D| f (a wave travelling along +p)
    the "-" weights vanish and the "+" weights equal the one-way weights
    FBI[f].n_b, up to the asymptotic error of the method.

Each test also plants a known mistake in the oracle (the g-term doubled, its
sign flipped, |p|^3 for |p|, the 1/2 dropped) and checks that the same
criterion then fails, so the pins are known to catch those readings.
"""
import math

import numpy as np
import pytest

import fga_inputs as fi
import oracle as om
from test_oracle_pins import fbi_closed_form_1d

CP, CS = math.sqrt(3.0), 1.0
WIDTH, CENTRE, K0 = 0.12, (0.5, 0.5, 0.5), (2.0, 0.0, 0.0)   # |k0| = 2: a |p| power shows


@pytest.fixture
def planted():
    """Yields a setter for the planted mistake; always removes it afterwards."""
    yield om.plant_two_way_error
    om.plant_two_way_error(0)


def packet_fbi(qs, ps, eps, d):
    """Closed-form FBI of d exp(-|y-c|^2/(2 w^2) + i k0.y/eps) at the pairs (qs, ps)."""
    s = np.ones(len(qs), dtype=np.complex128)
    for k in range(3):
        s *= fbi_closed_form_1d(qs[:, k], ps[:, k], eps, CENTRE[k], WIDTH, K0[k])
    return s[:, None] * np.asarray(d)[None, :]


def packet(x, eps, d):
    r2 = np.sum((x - np.asarray(CENTRE)) ** 2, axis=1)
    return (np.exp(-r2 / (2 * WIDTH ** 2) + 1j * (x @ np.asarray(K0)) / eps))[:, None] * np.asarray(d)[None, :]


def two_way_case(eps=1.0 / 16, nq=8, np_=5):
    """Beams of displacement f and velocity g, both Gaussian packets with
    seeded polarisations, in the homogeneous medium (FBI[g/c_b] = FBI[g]/c_b)."""
    df = fi.unit_vector(fi.rng(97, 1))
    dg = 3.0 * fi.unit_vector(fi.rng(97, 2))
    qmesh = fi.cell_centred(nq, 0.0, 1.0)
    pmesh = fi.p_mesh_around(K0, eps, WIDTH, np_)
    iq, ip = np.meshgrid(np.arange(qmesh.count), np.arange(pmesh.count), indexing="xy")
    iq, ip = iq.ravel(), ip.ravel()
    qs, ps = qmesh.points()[iq], pmesh.points()[ip]
    Ft = packet_fbi(qs, ps, eps, df)
    Gg = packet_fbi(qs, ps, eps, dg)
    Gt = np.stack([Gg / CP, Gg / CS], axis=1)
    x = np.asarray(CENTRE) + 0.12 * (np.random.default_rng(5).random((40, 3)) - 0.5)

    def beams(one_way=False):
        return om.make_beams(qmesh, pmesh, Ft, eps, iq, ip, one_way=one_way, Gt=None if one_way else Gt)

    return beams, x, packet(x, eps, df), packet(x, eps, dg), eps


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def u_and_ut(beams, x, eps, dt=1e-3, tau=12.0):
    """u(0) and the central difference (u(dt) - u(-dt)) / (2 dt) of the FGA sum."""
    med = om.homogeneous(CP, CS)
    u0, _ = om.sum_points(beams, x, eps, tau)
    bp, bm = beams.copy(), beams.copy()
    om.evolve(med, bp, dt, 1)
    om.evolve(med, bm, -dt, 1)
    up, _ = om.sum_points(bp, x, eps, tau)
    um, _ = om.sum_points(bm, x, eps, tau)
    return u0, (up - um) / (2 * dt)


def test_two_way_sum_at_t0_returns_f(planted):
    """u(0) = f: the two-way beams at t = 0 sum to the one-way sum (the g-terms
    of the two directions cancel exactly) and to f within the discretisation
    error of the mesh (1.5 % at eps = 1/16 with these meshes)."""
    beams, x, f, g, eps = two_way_case()
    two, one = beams(), beams(one_way=True)
    assert len(two) == 2 * len(one)
    u2, _ = om.sum_points(two, x, eps, 12.0)
    u1, _ = om.sum_points(one, x, eps, 12.0)
    del two, one
    assert rel(u2, u1) <= 1e-12
    assert rel(u2, f) <= 0.03
    planted(4)                                       # 1/2 on f dropped
    u2bad, _ = om.sum_points(beams(), x, eps, 12.0)
    assert rel(u2bad, f) > 0.5


def test_two_way_time_derivative_returns_g(planted):
    """u_t(0) = g: the central difference of RK4 steps of +-1e-3 returns the
    initial velocity within 3 % (1.5 % measured at eps = 1/16; 0.2 % at
    eps = 1/32 with a 10^3 x 6^3 mesh).  The planted mistakes give 72-200 %."""
    beams, x, f, g, eps = two_way_case()
    u0, ut = u_and_ut(beams(), x, eps)
    assert rel(u0, f) <= 0.03
    assert rel(ut, g) <= 0.03
    for kind in (1, 2, 3):       # g-term doubled; g-term sign flipped; |p|^3 for |p|
        planted(kind)
        _, ut_bad = u_and_ut(beams(), x, eps)
        assert rel(ut_bad, g) > 0.5, kind
    planted(0)


def pure_p_case(eps=1.0 / 16, ny=64):
    """Pure-P displacement f_P (Fourier projection xi xi^T/|xi|^2 of a
    Gaussian packet on a periodic box) and g = -i c_P |D| f_P, a P wave
    travelling along its wave vector; homogeneous medium."""
    d = fi.unit_vector(fi.rng(96, 1))
    ym = fi.Mesh3((ny,) * 3, (-0.5,) * 3, (2.0 / ny,) * 3)
    f = fi.gaussian_plane_wave(ym, eps, CENTRE, WIDTH, K0, d)
    xi = 2 * math.pi * np.fft.fftfreq(ny, d=2.0 / ny)
    KZ, KY, KX = np.meshgrid(xi, xi, xi, indexing="ij")
    K = np.stack([KX, KY, KZ])
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    fh = np.fft.fftn(f, axes=(1, 2, 3))
    fPh = K * (np.einsum("izyx,izyx->zyx", K, fh) / np.where(kk > 0, kk ** 2, 1.0))[None]
    fP = np.fft.ifftn(fPh, axes=(1, 2, 3))
    g = np.fft.ifftn(-1j * CP * kk[None] * fPh, axes=(1, 2, 3))
    w = fi.homogeneous_packet(eps=eps, nq=6, np_=4, ny=ny, nout=0)
    w.ymesh, w.f = ym, fP
    w.qmesh = fi.cell_centred(5, 0.25, 0.75)
    w.pmesh = fi.p_mesh_around(K0, eps, WIDTH, 4)
    return w, g


def test_pure_p_wave_has_no_minus_beams(planted):
    """For g = -i c_P |D| f_P the P beams' "-" weights are small against the
    "+" weights and the "+" weights equal the one-way weights FBI[f].n_P
    (3.6 % at eps = 1/16; measured 3.0 % at 1/32 and 2.3 % at 1/64: the
    mismatch FBI[|D| f] - (|p|/eps) FBI[f] is a finite-eps effect).  The
    planted mistakes give 34-2800 %."""
    w, g = pure_p_case()

    def ratios(two, one):
        plus, minus = two[two["sigma"] == 1], two[two["sigma"] == -1]
        assert np.array_equal(plus["lineage"], one["lineage"])
        return (np.linalg.norm(minus["w"]) / np.linalg.norm(plus["w"]),
                np.linalg.norm(plus["w"] - one["w"]) / np.linalg.norm(one["w"]))

    one = om.decompose(w, branch_mask=1)
    r_minus, r_plus = ratios(om.decompose_two_way(w, g, branch_mask=1), one)
    assert r_minus <= 0.05 and r_plus <= 0.05
    # the same weights from the FBI values, with each mistake planted
    iq, ip = np.meshgrid(np.arange(w.qmesh.count), np.arange(w.pmesh.count), indexing="xy")
    iq, ip = iq.ravel(), ip.ravel()
    qs, ps = w.qmesh.points()[iq], w.pmesh.points()[ip]
    Ft = om.fbi(w.f, w.ymesh, qs, ps, w.eps)
    G = om.fbi(g, w.ymesh, qs, ps, w.eps)
    Gt = np.stack([G / CP, G / CS], axis=1)
    for kind in (1, 2, 3, 4):
        planted(kind)
        two = om.make_beams(w.qmesh, w.pmesh, Ft, w.eps, iq, ip, one_way=False, Gt=Gt, branch_mask=1)
        bad = ratios(two, one)
        assert max(bad) > 0.3, (kind, bad)
    planted(0)
