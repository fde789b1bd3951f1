"""Pins of the reference solver of the radially symmetric waveguide check
(tests/radial_fd.py; Sec. 3.2, eq:we_radially_symmetric):

  - in a homogeneous medium it reproduces the closed-form radial solution
    (r psi solves the 1-D wave equation, extended oddly through r = 0;
    u = d_r psi), to second order in the grid spacing;
  - across interfaces it converges under refinement and conserves the
    elastic energy;
  - at an interface far from the centre a pulse is reflected with the
    displacement coefficient of normal incidence, (rho1 c1 - rho2 c2) /
    (rho1 c1 + rho2 c2), which the elastic conditions (continuity of u and
    of s_rr) give and the velocity-only conditions of the scalar form would
    not.
"""
import math

import numpy as np

import radial_fd as rf

SIG, ELL = 0.022, 0.049      # shell half-width and wavelength of phi0 (ratio as in the paper)


def phi0(r):
    return np.exp(-r * r / (2 * SIG * SIG)) * np.cos(2 * math.pi * r / ELL)


def dphi0(r):
    e = np.exp(-r * r / (2 * SIG * SIG))
    return -(r / SIG ** 2) * e * np.cos(2 * math.pi * r / ELL) - (2 * math.pi / ELL) * e * np.sin(2 * math.pi * r / ELL)


def exact_homogeneous(t, r, r0, c):
    """u = d_r psi, r psi = (G(r - ct) + G(r + ct))/2, G(s) = s phi0(s - r0) odd in s."""
    def G(s):
        return np.sign(s) * np.abs(s) * phi0(np.abs(s) - r0)

    def dG(s):
        a = np.abs(s)
        return phi0(a - r0) + a * dphi0(a - r0)

    rp = 0.5 * (G(r - c * t) + G(r + c * t))
    drp = 0.5 * (dG(r - c * t) + dG(r + c * t))
    return drp / r - rp / r ** 2


def test_homogeneous_closed_form():
    r0, c = 0.3, math.sqrt(3.0)
    stations = np.array([0.12, 0.35, 0.5])
    times = np.linspace(0.0, 0.16, 9)
    errs = []
    for h in (ELL / 40, ELL / 80):
        got, dt = rf.solve([], [c], [1.0], [1.0], lambda r: dphi0(r - r0), 1.0, 0.16, h, times, stations)
        ref = np.array([exact_homogeneous(t, stations, r0, c) for t in times])
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[1] < 5e-3                   # measured 1.2e-2, 3.1e-3, 7.2e-4 at h = l/40, l/80, l/160
    assert errs[0] / errs[1] > 3.0          # second order


def layered():
    return [0.45, 0.38], [1.9, 1.8, 1.7], [1.1, 1.05, 1.0], [1.3, 1.15, 1.0]


def test_layers_converge_and_conserve_energy():
    radii, cp, cs, rho = layered()
    r0 = 0.3
    stations = np.array([0.34, 0.42, 0.5])
    times = np.linspace(0.0, 0.18, 10)
    sols = [rf.solve(radii, cp, cs, rho, lambda r: dphi0(r - r0), 1.0, 0.18, h, times, stations)[0]
            for h in (ELL / 20, ELL / 40, ELL / 80)]
    d1 = np.linalg.norm(sols[1] - sols[0])
    d2 = np.linalg.norm(sols[2] - sols[1])
    assert d1 / d2 > 1.8                     # at least first order at the interfaces
    assert d2 < 0.02 * np.linalg.norm(sols[2])
    # energy at t = 0, 0.06, 0.12 from the nodal field and a central difference in time
    h, e = ELL / 60, 2e-4
    n = int(math.ceil(1.0 / h))
    r = np.arange(n + 1) * h
    tt = np.arange(0, 601) * e                       # 0 .. 0.12
    a, _ = rf.solve(radii, cp, cs, rho, lambda rr: dphi0(rr - r0), 1.0, tt[-1], h, tt, r[1:-1])
    E = []
    for k in (1, 300, 599):
        uu = np.concatenate([[0.0], a[k], [0.0]])
        ut = np.concatenate([[0.0], (a[k + 1] - a[k - 1]) / (2 * e), [0.0]])
        E.append(rf.energy(radii, cp, cs, rho, uu, ut, h))
    assert max(abs(x - E[0]) for x in E) < 1e-2 * E[0], E


def test_normal_incidence_reflection_coefficient():
    """A pulse far from the centre (r0 = 3, so that 1/(k r) is small) runs
    outward into an interface at r = 3.2; the reflected pulse, measured at
    r = 3.1 after it has passed back, has the displacement amplitude ratio
    (rho1 c1 - rho2 c2)/(rho1 c1 + rho2 c2) of the incident pulse (within
    1 %)."""
    radii = [3.2]
    cp, cs, rho = [2.0, 1.6], [1.1, 1.0], [1.5, 1.0]     # shell 0 outside r = 3.2
    r0, st = 3.0, 3.1
    c1, c2 = cp[1], cp[0]
    z1, z2 = rho[1] * c1, rho[0] * c2
    # incident pulse passes r = 3.1 at t = 0.1/c1 (the outgoing half of the data), the reflection at 0.3/c1
    times = np.arange(0, 901) * (0.45 / c1 / 900)
    got, _ = rf.solve(radii, cp, cs, rho, lambda r: dphi0(r - r0) * (r > 2.5), 4.0, times[-1], ELL / 60, times, [st])
    tr = got[:, 0]
    inc = np.abs(tr[(times > 0.05 / c1) & (times < 0.15 / c1)]).max()
    ref = np.abs(tr[(times > 0.25 / c1) & (times < 0.4 / c1)]).max()
    # the outgoing wave decays as 1/r from 3.1 to 3.2 and the reflected one, an ingoing spherical wave
    # about the same centre, grows as 1/r back to 3.1: the spreading cancels
    R = abs(z1 - z2) / (z1 + z2)
    assert abs(ref / inc - R) < 0.01 * R, (ref / inc, R)
    assert abs(ref / inc - abs(c2 - c1) / (c1 + c2)) > 0.5 * R      # not the velocity-only coefficient
