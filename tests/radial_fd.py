"""Reference solution of the radially symmetric waveguide check (Sec. 3.2,
the P-wave example in a 1-D layered Earth model, eq:we_radially_symmetric):
the radial displacement u(t, r) of a radially symmetric elastic field
u = u(t, r) x/|x| in concentric homogeneous shells, by second-order finite
differences on a staggered radial grid.

Equations (isotropic, per shell lambda, mu, rho):
  rho u_tt = d_r s_rr + (2/r)(s_rr - s_tt),
  s_rr = (lambda + 2 mu) u_r + 2 lambda u/r,   s_tt = lambda u_r + 2 (lambda + mu) u/r,
which inside a shell is u_tt = c_P^2 (u_rr + 2 u_r/r - 2 u/r^2), the radial
derivative of eq:we_radially_symmetric for u = d_r psi; across an interface
u and s_rr are continuous (the elastic boundary conditions, which the
scalar form does not state).  u = 0 at r = 0.

Grid: u at r_j = j h (j = 0..n), s_rr at r_{j+1/2}; the material at a
half node is that of its midpoint, at a node the average of the two
adjacent half nodes (harmonic for the stiffness, arithmetic for the
density).  Leapfrog in time.  Test helper: the tests check it against the
closed-form solution in a homogeneous medium and for convergence and energy
conservation across interfaces before the GPU check uses it.
"""
import math

import numpy as np


def layer_of(r, radii):
    """Shell index of radius r: 0 outermost, radii descending (as the library's spherical layers)."""
    k = np.zeros_like(np.asarray(r, dtype=np.float64), dtype=np.int64)
    for b in radii:
        k += (np.asarray(r) < b).astype(np.int64)
    return k


def solve(radii, cp, cs, rho, u0, rmax, T, h, times, stations, cfl=0.4):
    """u(t, r_station) at the given times, u(0) = u0(r), u_t(0) = 0.

    radii: interface radii, descending; cp, cs, rho: per shell (0 outermost).
    Returns an array [len(times)][len(stations)] (linear interpolation in r)
    and the time step; times must be a uniform grid k * delta from 0, and
    the step is delta divided by the smallest integer that keeps the
    Courant number at most cfl."""
    cp, cs, rho = (np.asarray(v, dtype=np.float64) for v in (cp, cs, rho))
    n = int(math.ceil(rmax / h))
    r = np.arange(n + 1) * h
    rh = (np.arange(n) + 0.5) * h
    Lh = layer_of(rh, radii)
    lam_h = rho[Lh] * (cp[Lh] ** 2 - 2 * cs[Lh] ** 2)
    mu_h = rho[Lh] * cs[Lh] ** 2
    M_h = lam_h + 2 * mu_h
    # nodes: average of the neighbouring half nodes
    rho_h = rho[Lh]
    rho_n = np.empty(n + 1)
    rho_n[1:-1] = 0.5 * (rho_h[:-1] + rho_h[1:])
    rho_n[0], rho_n[-1] = rho_h[0], rho_h[-1]
    lam_n = np.empty(n + 1)
    mu_n = np.empty(n + 1)
    lam_n[1:-1] = 2.0 / (1.0 / lam_h[:-1] + 1.0 / lam_h[1:]) if np.all(lam_h > 0) else 0.5 * (lam_h[:-1] + lam_h[1:])
    mu_n[1:-1] = 2.0 / (1.0 / mu_h[:-1] + 1.0 / mu_h[1:])
    lam_n[0], lam_n[-1], mu_n[0], mu_n[-1] = lam_h[0], lam_h[-1], mu_h[0], mu_h[-1]
    # times: a uniform grid k * delta starting at 0; the step divides delta
    times = np.asarray(times, dtype=np.float64)
    delta = times[1] - times[0] if len(times) > 1 else max(times[0], h)
    if abs(times[0]) > 1e-12 or np.max(np.abs(np.diff(times) - delta)) > 1e-9 * max(delta, 1.0):
        raise ValueError("times must be a uniform grid starting at 0")
    nsub = max(1, int(math.ceil(delta / (cfl * h / cp.max()))))
    dt = delta / nsub
    nsteps_total = nsub * (len(times) - 1)
    want = {k * nsub: k for k in range(len(times))}
    out = np.zeros((len(times), len(stations)))
    u = u0(r).astype(np.float64)
    u[0] = 0.0

    def accel(u):
        ur_h = (u[1:] - u[:-1]) / h
        um_h = 0.5 * (u[1:] + u[:-1])
        srr_h = M_h * ur_h + 2 * lam_h * um_h / rh
        a = np.zeros_like(u)
        # node j: d_r s_rr from the half nodes, (2/r)(s_rr - s_tt) = (4 mu / r)(u_r - u/r) at the node
        ur_n = (u[2:] - u[:-2]) / (2 * h)
        rn = r[1:-1]
        a[1:-1] = ((srr_h[1:] - srr_h[:-1]) / h + 4 * mu_n[1:-1] * (ur_n - u[1:-1] / rn) / rn) / rho_n[1:-1]
        return a

    # first step from u_t = 0: u^1 = u^0 + dt^2/2 a(u^0)
    u_prev = u.copy()
    u = u + 0.5 * dt * dt * accel(u)
    u[0] = 0.0
    u[-1] = 0.0

    def sample(uu):
        return np.interp(stations, r, uu)

    if 0 in want:
        out[want[0]] = sample(u_prev)
    if 1 in want:
        out[want[1]] = sample(u)
    for s in range(2, nsteps_total + 1):
        u_next = 2 * u - u_prev + dt * dt * accel(u)
        u_next[0] = 0.0
        u_next[-1] = 0.0
        u_prev, u = u, u_next
        if s in want:
            out[want[s]] = sample(u)
    return out, dt


def energy(radii, cp, cs, rho, u, ut, h):
    """Elastic energy 4 pi int (rho ut^2 / 2 + W) r^2 dr of a radial field on the node grid."""
    cp, cs, rho = (np.asarray(v, dtype=np.float64) for v in (cp, cs, rho))
    n = len(u) - 1
    rh = (np.arange(n) + 0.5) * h
    L = layer_of(rh, radii)
    lam = rho[L] * (cp[L] ** 2 - 2 * cs[L] ** 2)
    mu = rho[L] * cs[L] ** 2
    ur = (u[1:] - u[:-1]) / h
    um = 0.5 * (u[1:] + u[:-1])
    ut_h = 0.5 * (ut[1:] + ut[:-1])
    # strains: e_rr = u_r, e_tt = e_pp = u/r
    err, ett = ur, um / rh
    W = 0.5 * lam * (err + 2 * ett) ** 2 + mu * (err ** 2 + 2 * ett ** 2)
    return 4 * math.pi * np.sum((0.5 * rho[L] * ut_h ** 2 + W) * rh ** 2) * h
