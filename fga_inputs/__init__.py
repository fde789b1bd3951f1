"""Seeded synthetic inputs for the FGA workloads.

This module only draws and lays out input data: velocity-model node values,
initial displacement fields on a quadrature grid, phase-space mesh
descriptors, receiver positions and request streams.  It holds none of the
method's arithmetic (no FBI projection, no ray or amplitude equations, no
Gaussian summation) and is the only code shared by the CPU oracle tests and
the GPU path.

Conventions
-----------
* A uniform axis-aligned point set ("mesh") is described by ``(n, lo, h)``
  per axis: points ``lo[d] + i*h[d]`` for ``i = 0..n[d]-1``.  Cell-centred
  meshes of a box ``[a, b]`` use ``lo = a + h/2``.
* 3-D arrays are stored ``[z][y][x]`` (x fastest); vector fields are
  ``[component][z][y][x]``.
* Every random draw uses ``numpy.random.default_rng(1000*family + purpose)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SQRT3 = math.sqrt(3.0)


def rng(family: int, purpose: int) -> np.random.Generator:
    """Seeded generator for input ``purpose`` of the seed family ``family`` (one per workload)."""
    return np.random.default_rng(1000 * family + purpose)


@dataclass
class Mesh3:
    """Uniform point set ``lo + i*h`` on each axis (i = 0..n-1)."""
    n: tuple
    lo: tuple
    h: tuple

    @property
    def count(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def cell_volume(self) -> float:
        return float(self.h[0] * self.h[1] * self.h[2])

    def axis(self, d: int) -> np.ndarray:
        return self.lo[d] + self.h[d] * np.arange(self.n[d], dtype=np.float64)

    def points(self) -> np.ndarray:
        """All points, shape (count, 3), x index fastest."""
        z, y, x = np.meshgrid(self.axis(2), self.axis(1), self.axis(0), indexing="ij")
        return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def cell_centred(n: int, a: float, b: float) -> Mesh3:
    """n^3 cell-centred points on the cube [a, b]^3."""
    h = (b - a) / n
    return Mesh3((n, n, n), (a + 0.5 * h,) * 3, (h,) * 3)


def box_mesh(n: int, centre, half_width: float) -> Mesh3:
    """n^3 cell-centred points on the box centre +- half_width (per axis)."""
    h = 2.0 * half_width / n
    lo = tuple(float(c) - half_width + 0.5 * h for c in centre)
    return Mesh3((n, n, n), lo, (h,) * 3)


def packet_momentum_spread(eps: float, width: float) -> float:
    """Standard deviation, per axis, of |FBI transform| of a Gaussian-enveloped
    plane wave of envelope std ``width`` in the momentum variable p.  Used
    only to place the p-mesh (the paper leaves mesh placement to the user)."""
    return eps * math.sqrt(1.0 / width ** 2 + 1.0 / eps)


def p_mesh_around(k0, eps: float, width: float, n: int, nsig: float = 3.0) -> Mesh3:
    """Cell-centred p-mesh spanning k0 +- nsig*sigma_p per axis."""
    sp = packet_momentum_spread(eps, width)
    return box_mesh(n, k0, nsig * sp)


def unit_vector(g: np.random.Generator) -> np.ndarray:
    v = g.standard_normal(3)
    return v / np.linalg.norm(v)


def gaussian_plane_wave(ymesh: Mesh3, eps: float, centre, width: float, k0, d) -> np.ndarray:
    """f(y) = exp(-|y-centre|^2/(2 width^2)) * d * exp(i k0.y/eps) on ymesh.

    Returns complex128 array [3][z][y][x]."""
    x = ymesh.axis(0)[None, None, :]
    y = ymesh.axis(1)[None, :, None]
    z = ymesh.axis(2)[:, None, None]
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    phase = (k0[0] * x + k0[1] * y + k0[2] * z) / eps
    s = np.exp(-r2 / (2.0 * width ** 2)) * np.exp(1j * phase)
    d = np.asarray(d, dtype=np.complex128)
    return np.ascontiguousarray(d[:, None, None, None] * s[None])


def gaussian_random_field(n: int, corr_len: float, std: float, clip: float,
                          g: np.random.Generator) -> np.ndarray:
    """Periodic Gaussian random field on the n^3 node grid of [0,1)^3.

    White noise filtered in Fourier space so that the covariance is
    proportional to exp(-r^2/(2 corr_len^2)); rescaled to the given standard
    deviation and clipped to [-clip, clip].  Array order [z][y][x]."""
    noise = g.standard_normal((n, n, n))
    xi = 2.0 * math.pi * np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(xi, xi, xi, indexing="ij")
    filt = np.exp(-(corr_len ** 2) * (kx ** 2 + ky ** 2 + kz ** 2) / 4.0)
    f = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    f = f - f.mean()
    f = f * (std / f.std())
    return np.clip(f, -clip, clip)


def node_grid(n: int) -> Mesh3:
    """n^3 node grid of the periodic unit cube: nodes i/n."""
    return Mesh3((n, n, n), (0.0, 0.0, 0.0), (1.0 / n,) * 3)


def uniform_points(count: int, g: np.random.Generator, lo=0.0, hi=1.0) -> np.ndarray:
    return lo + (hi - lo) * g.random((count, 3))


# ---------------------------------------------------------------------------
# Workload descriptions.  Each is a plain dictionary of sizes and seeds; the
# arrays are produced on demand by ``make_workload``.
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    eps: float
    cp0: float
    cs0: float
    qmesh: Mesh3
    pmesh: Mesh3
    ymesh: Mesh3
    f: np.ndarray                  # complex128 [3][z][y][x] initial displacement
    dt: float
    nsteps: int
    out_grid: Mesh3 | None
    receivers: np.ndarray | None   # (n_r, 3)
    medium_nodes: np.ndarray | None = None   # c_p node values [z][y][x] (grid media)
    medium_grid: Mesh3 | None = None
    cs_ratio: float = 1.0 / SQRT3
    medium_smooth: bool = False    # grid media: cubic B-spline of the nodes instead of trilinear
    branches: tuple = (0, 1, 2)    # P, SH, SV
    tau: float = 25.0
    cull_abs: float = 0.0          # |psi| threshold below which a beam is not created
    extra: dict = field(default_factory=dict)


def homogeneous_packet(name="c1", eps=1.0 / 32, nq=8, np_=4, ny=64, nsteps=100,
                       dt=0.005, nout=32, family=1, tau=25.0) -> Workload:
    """Plain FGA in a homogeneous medium (cp = sqrt(3), cs = 1): a Gaussian
    plane-wave packet of width 0.1 centred at (0.5,0.5,0.5) travelling along
    x, one-way data, q nq^3 on [0,1]^3, p np^3 around k0 = (1,0,0)."""
    width, centre, k0 = 0.1, (0.5, 0.5, 0.5), (1.0, 0.0, 0.0)
    d = unit_vector(rng(family, 1))
    ymesh = cell_centred(ny, 0.0, 1.0)
    return Workload(
        name=name, eps=eps, cp0=SQRT3, cs0=1.0,
        qmesh=cell_centred(nq, 0.0, 1.0),
        pmesh=p_mesh_around(k0, eps, width, np_),
        ymesh=ymesh,
        f=gaussian_plane_wave(ymesh, eps, centre, width, k0, d),
        dt=dt, nsteps=nsteps,
        out_grid=cell_centred(nout, 0.0, 1.0) if nout else None,
        receivers=None, tau=tau,
        extra={"width": width, "centre": centre, "k0": k0, "d": d},
    )


def smooth_medium_packet(name="c2", eps=1.0 / 128, nq=32, np_=8, ny=128, nmed=128,
                         nsteps=1000, dt=1e-3, nout=128, nrec=256, family=2,
                         tau=25.0, cull_rel=1e-10) -> Workload:
    """Smooth heterogeneous medium cp = sqrt(3)(1 + 0.2 g), cs = cp/sqrt(3),
    g a periodic Gaussian random field (correlation length 0.2, std 1/3,
    clipped to |g| <= 1) on an nmed^3 node grid; Gaussian plane-wave packet
    initial data; receivers uniform in [0,1]^3."""
    width, centre, k0 = 0.1, (0.5, 0.5, 0.5), (1.0, 0.0, 0.0)
    gfield = gaussian_random_field(nmed, 0.2, 1.0 / 3.0, 1.0, rng(family, 1))
    cp_nodes = SQRT3 * (1.0 + 0.2 * gfield)
    d = unit_vector(rng(family, 3))
    ymesh = cell_centred(ny, 0.0, 1.0)
    rec = uniform_points(nrec, rng(family, 2)) if nrec else None
    # Peak |psi| of this data is bounded by the y-integral of |f|, which is at
    # most (2 pi width^2)^{3/2}; beams below cull_rel times that are not made.
    peak = (2.0 * math.pi * width ** 2) ** 1.5
    return Workload(
        name=name, eps=eps, cp0=SQRT3, cs0=1.0,
        qmesh=cell_centred(nq, 0.0, 1.0),
        pmesh=p_mesh_around(k0, eps, width, np_),
        ymesh=ymesh,
        f=gaussian_plane_wave(ymesh, eps, centre, width, k0, d),
        dt=dt, nsteps=nsteps,
        out_grid=cell_centred(nout, 0.0, 1.0) if nout else None,
        receivers=rec, medium_nodes=cp_nodes, medium_grid=node_grid(nmed),
        tau=tau, cull_abs=cull_rel * peak,
        extra={"width": width, "centre": centre, "k0": k0, "d": d},
    )


def mixed_waves(eps=1.0 / 512, nq=50, np_=8, ny=256, nsteps=250, dt=1e-3, nout=256, tau=16.0, waves=4):
    """The smooth random medium and packet form of the smooth-medium workload at eps = 1/512,
    q nq^3 x p np_^3 x 3 branches, evolved to T = nsteps dt and summed on an
    nout^3 grid of [0,1]^3.  The q mesh is cut into `waves` slabs along z
    (sizes differing by at most one plane), each decomposed, evolved and summed
    on its own.  Returns (workload, list of the slabs' q meshes)."""
    w = smooth_medium_packet(name="c4", eps=eps, nq=nq, np_=np_, ny=ny, nsteps=nsteps, dt=dt, nout=nout, nrec=0,
                             family=2, tau=tau)
    q = w.qmesh
    cuts = [round(k * q.n[2] / waves) for k in range(waves + 1)]
    slabs = [Mesh3((q.n[0], q.n[1], cuts[k + 1] - cuts[k]), (q.lo[0], q.lo[1], q.lo[2] + cuts[k] * q.h[2]), q.h)
             for k in range(waves) if cuts[k + 1] > cuts[k]]
    return w, slabs


def radial_shell(ymesh: Mesh3, r0: float, sigma: float, ell: float) -> np.ndarray:
    """u = grad phi0(|y| - r0), phi0(s) = exp(-s^2/(2 sigma^2)) cos(2 pi s/ell): a
    radially symmetric shell of P-wave displacement (the waveguide example's
    initial data).  Returns complex128 [3][z][y][x] (real values)."""
    x = ymesh.axis(0)[None, None, :]
    y = ymesh.axis(1)[None, :, None]
    z = ymesh.axis(2)[:, None, None]
    r = np.sqrt(x * x + y * y + z * z)
    s = r - r0
    e = np.exp(-s * s / (2 * sigma * sigma))
    dphi = -(s / sigma ** 2) * e * np.cos(2 * math.pi * s / ell) - (2 * math.pi / ell) * e * np.sin(2 * math.pi * s / ell)
    rr = np.where(r > 0, r, 1.0)
    out = np.stack([dphi * x / rr, dphi * y / rr, dphi * z / rr]).astype(np.complex128)
    return np.ascontiguousarray(out)


# ---------------------------------------------------------------------------
# tomography-style request sweep (serving)
# ---------------------------------------------------------------------------

# eps -> (q points per axis, Fibonacci directions, |p| shells) of a point-source request
SWEEP_MESHES = {1.0 / 32: (5, 64, 3), 1.0 / 64: (6, 120, 4), 1.0 / 128: (8, 200, 4)}


def sweep_model(j: int, nmed: int = 128) -> np.ndarray:
    """c_P node values of resident model j (0..3): the smooth random medium
    recipe (correlation length 0.2, std 1/3, clipped) with its own seed."""
    g = gaussian_random_field(nmed, 0.2, 1.0 / 3.0, 1.0, rng(5, 1 + j))
    return SQRT3 * (1.0 + 0.2 * g)


def moment_tensor(g: np.random.Generator) -> list:
    """Symmetric moment tensor with N(0,1) entries, Frobenius-normalised;
    returned as (xx, yy, zz, xy, xz, yz)."""
    a = g.standard_normal((3, 3))
    m = 0.5 * (a + a.T)
    m /= np.linalg.norm(m)
    return [m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[0, 2], m[1, 2]]


def sweep_request(i: int, nmodels: int = 4, nsteps: int = 250, dt: float = 2e-3, tau: float = 25.0) -> dict:
    """Request i of the sweep: model index, a point moment-tensor source at
    a uniform position in [0.25, 0.75]^3 with a random moment tensor and a
    Ricker wavelet, eps from SWEEP_MESHES, 128..1024 receivers uniform in
    [0,1]^3."""
    g = rng(5, 100 + i)
    model = int(g.integers(0, nmodels))
    x0 = g.uniform(0.25, 0.75, 3)
    M = moment_tensor(g)
    eps = list(SWEEP_MESHES)[int(g.integers(0, len(SWEEP_MESHES)))]
    nq, ndir, nshell = SWEEP_MESHES[eps]
    nrec = int(g.integers(128, 1025))
    return {
        "model": model, "eps": eps, "nsteps": nsteps, "dt": dt, "tau": tau,
        "x0": x0, "M": M, "nq": nq, "ndir": ndir, "nshell": nshell,
        "receivers": uniform_points(nrec, g),
    }


# The tomography sweep at its stated sizes: eps from {1/64, 1/128, 1/256,
# 1/512}; the point-source meshes (q 8^3 x directions x shells x 3 branches x
# 2 directions) give about 1e5, 8e5, 6.4e6 and 5.1e7 candidate beams; 2000
# samples over T = 1.
SWEEP5_MESHES = {1.0 / 64: (8, 16, 2), 1.0 / 128: (8, 65, 4), 1.0 / 256: (8, 520, 4), 1.0 / 512: (8, 4167, 4)}


def sweep5_request(i: int, nmodels: int = 4, nsteps: int = 2000, T: float = 1.0, tau: float = 25.0,
                   eps_index: int = None) -> dict:
    """Request i of the sweep at its stated sizes: model index, a point
    moment-tensor source (Ricker) at a uniform position in [0.25, 0.75]^3
    with a random moment tensor, eps drawn uniformly from SWEEP5_MESHES (or
    the given index), 128..1024 receivers uniform in [0,1]^3, nsteps samples."""
    g = rng(5, 400 + i)
    model = int(g.integers(0, nmodels))
    x0 = g.uniform(0.25, 0.75, 3)
    M = moment_tensor(g)
    k = int(g.integers(0, len(SWEEP5_MESHES)))
    eps = list(SWEEP5_MESHES)[k if eps_index is None else eps_index]
    nq, ndir, nshell = SWEEP5_MESHES[eps]
    nrec = int(g.integers(128, 1025))
    return {
        "model": model, "eps": eps, "nsteps": nsteps, "dt": T / nsteps, "tau": tau,
        "x0": x0, "M": M, "nq": nq, "ndir": ndir, "nshell": nshell,
        "receivers": uniform_points(nrec, g),
    }


# ---------------------------------------------------------------------------
# layered spherical Earth-like model with a point source
# ---------------------------------------------------------------------------

def fibonacci_sphere(n: int, g: np.random.Generator) -> np.ndarray:
    """n points of a Fibonacci lattice on the unit sphere, randomly rotated;
    returned in Cartesian coordinates."""
    i = np.arange(n)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = i * math.pi * (3.0 - math.sqrt(5.0))
    pts = np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)
    q, _ = np.linalg.qr(g.standard_normal((3, 3)))
    return pts @ q.T


def layered_earth(family: int = 3, eps: float = 1.0 / 256, nq: int = 8, ndir: int = 1600, nshell: int = 4,
                  nsteps: int = 2000, T: float = 1.5, nrec: int = 512) -> dict:
    """Unit sphere with 4 layers: 3 interface radii in (0.3, 0.95) at least
    0.1 apart; the top layer has c_P = sqrt(3), c_S = 1, rho = 1 and each
    deeper layer multiplies each of them by U[1.05, 1.20]; a point
    moment-tensor source with a Ricker wavelet at radius U[0.6, 0.9] in a
    random direction; receivers on a Fibonacci lattice of the surface r = 1,
    given in spherical coordinates (r, longitude, latitude) as the Earth
    examples give stations ("receivers_rtp")."""
    g = rng(family, 1)
    while True:
        radii = np.sort(g.uniform(0.3, 0.95, 3))[::-1]
        if np.all(-np.diff(radii) >= 0.1):
            break
    cp, cs, rho = [SQRT3], [1.0], [1.0]
    for _ in range(3):
        cp.append(cp[-1] * g.uniform(1.05, 1.20))
        cs.append(cs[-1] * g.uniform(1.05, 1.20))
        rho.append(rho[-1] * g.uniform(1.05, 1.20))
    gs = rng(family, 2)
    d = unit_vector(gs)
    x0 = d * gs.uniform(0.6, 0.9)
    M = moment_tensor(gs)
    pts = fibonacci_sphere(nrec, rng(family, 3))
    theta = np.arctan2(pts[:, 1], pts[:, 0])
    phi = np.arcsin(np.clip(pts[:, 2], -1.0, 1.0))
    rtp = np.stack([np.ones(nrec), theta, phi], axis=1)
    return {"bounds": list(radii), "cp": cp, "cs": cs, "rho": rho, "x0": x0, "M": M, "eps": eps, "nq": nq,
            "ndir": ndir, "nshell": nshell, "nsteps": nsteps, "dt": T / nsteps, "receivers_rtp": rtp, "tau": 25.0}


def crosswell(source: int = 8, eps: float = 1.0 / 128, nq: int = 8, ndir: int = 1600, nshell: int = 4,
              nsteps: int = 2000, T: float = 2.0, true_model: bool = True) -> dict:
    """The crosswell model of the tomography example (Sec. 4, eq:true_c; with
    true_model=False the initial model eq:ini_c), nondimensional: lengths in
    100 m, speeds in 1000 m/s (times in 0.1 s).  Three flat layers below a
    traction-free surface: depth 0-100 m c_P = 1.8, 100-200 m c_P = 2.0 with
    the Gaussian low-velocity region 1 - 0.1 exp(-(22.2)((x - 0.75)^2 + (z -
    z_c)^2)) (beta = 1/450 m^-2, centre x 75 m, depth 150 m, invariant in y),
    below 200 m c_P = 2.2; c_S = c_P/sqrt(3) throughout; density 1 (the paper
    gives none).  Depth d maps to z = 3 - d/100 (z up; the surface at z = 3,
    the interfaces at z = 2 and 1, layer 0 the deepest).  16 sources at x = 0
    spaced 16 m in depth from 8 m, 32 receivers at x = 1.5 spaced 8 m from
    4 m (the figure's positions are not given in the text); `source` picks
    one (8: the ninth from the top).  The source is an explosion (moment
    tensor I) with a Ricker wavelet; eps = 1/128 is about 400 Hz at 2000 m/s
    (the text names no frequency)."""
    depth_src = 0.08 + 0.16 * np.arange(16)
    depth_rec = 0.04 + 0.08 * np.arange(32)
    anomaly = {1: (0.1, 1.0e4 / 450.0, (0.75, 0.0, 1.5), (1.0, 0.0, 1.0))} if true_model else None
    cp = [2.2, 2.0, 1.8]
    return {"bounds": [1.0, 2.0], "cp": cp, "cs": [c / SQRT3 for c in cp], "rho": [1.0, 1.0, 1.0],
            "anomaly": anomaly, "surface": 3.0,
            "x0": np.array([0.0, 0.0, 3.0 - depth_src[source]]), "M": [1.0, 1.0, 1.0, 0.0, 0.0, 0.0],
            "eps": eps, "nq": nq, "ndir": ndir, "nshell": nshell, "nsteps": nsteps, "dt": T / nsteps,
            "receivers": np.stack([np.full(32, 1.5), np.zeros(32), 3.0 - depth_rec], axis=1), "tau": 25.0,
            "sources": np.stack([np.zeros(16), np.zeros(16), 3.0 - depth_src], axis=1)}
