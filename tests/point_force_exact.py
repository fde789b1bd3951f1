"""Closed-form displacement of a point force in a homogeneous isotropic
elastic whole space (the accuracy experiment of Sec. 2.3, eq:ex_homo and its
solution eq:ex_anal): for rho u_tt = (lambda + mu) grad div u + mu Lap u +
d F(t) delta(x - x0),

  u_i = r_i r_j d_j F(t - r/c_P) / (4 pi rho c_P^2 r^3)
      + (r^2 delta_ij - r_i r_j) d_j F(t - r/c_S) / (4 pi rho c_S^2 r^3)
      + (3 r_i r_j - r^2 delta_ij) d_j / (4 pi rho r^5) int_{r/c_P}^{r/c_S} s F(t - s) ds,

r = x - x0.  The near-field integral is evaluated by Gauss-Legendre
quadrature (its integrand is smooth on a finite interval).  Test helper:
the tests check this formula against the wave equation and the source
strength before the GPU accuracy test uses it.
"""
import math

import numpy as np


def source_time_function(t, omega, t0, width):
    """F(t) = cos(omega (t + t0)) exp(-(t + t0)^2 / width^2)."""
    v = np.asarray(t) + t0
    return np.cos(omega * v) * np.exp(-v * v / (width * width))


def displacement(x, t, x0, d, cp, cs, rho, omega, t0, width, nodes=96):
    """u(t, x) at points x (n, 3); returns (n, 3) real."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    rv = x - np.asarray(x0)[None, :]
    r = np.linalg.norm(rv, axis=1)
    d = np.asarray(d, dtype=np.float64)
    rd = rv @ d                                   # r_j d_j
    F = lambda tt: source_time_function(tt, omega, t0, width)
    a, b = r / cp, r / cs
    gx, gw = np.polynomial.legendre.leggauss(nodes)
    s = 0.5 * (a + b)[:, None] + 0.5 * (b - a)[:, None] * gx[None, :]
    near = 0.5 * (b - a) * np.sum(gw[None, :] * s * F(t - s), axis=1)
    k = 1.0 / (4.0 * math.pi * rho)
    term_p = k * F(t - a) / (cp * cp * r ** 3)
    term_s = k * F(t - b) / (cs * cs * r ** 3)
    term_n = k * near / r ** 5
    u = (rv * (rd * term_p)[:, None]
         + (r * r)[:, None] * d[None, :] * term_s[:, None] - rv * (rd * term_s)[:, None]
         + 3.0 * rv * (rd * term_n)[:, None] - (r * r)[:, None] * d[None, :] * term_n[:, None])
    return u
