"""CPU oracle for the FGA hot path -- TEST INFRASTRUCTURE ONLY.

Plain FP64 implementation (C99 + OpenMP in ``fga_oracle.c``, driven from
here through ctypes) of the frozen Gaussian approximation of the 3-D elastic
wave equation: FBI decomposition (eq:psi, eq:alpha^k), RK4 of the ray,
variational and amplitude ODEs (eq:char_plus/minus, eq:DzDt, eq:amp_P/SV/SH),
the interface map (eq:p:int, eq:Yilmaz, eq:Inter_DzQDzP) and the windowed
Gaussian summation (eq:FGA).  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it; the GPU library never does, and it
shares no code with the GPU library.

Beams are numpy structured arrays (``BEAM_DTYPE``) mirroring ``om_beam``.
Beam numbering ("lineage") follows the canonical enumeration
    lineage = ((branch*2 + dir)*Np + ip)*Nq + iq,
branch 0/1/2 = P/SH/SV, dir 0/1 = "+"/"-", ip and iq the row-major mesh
indices with x fastest.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fga_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = "%s.%d.tmp" % (_LIB_PATH, os.getpid())   # one per process: parallel test workers
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


BEAM_DTYPE = np.dtype([
    ("Q", "f8", 3), ("P", "f8", 3),
    ("ZQ", "c16", (3, 3)), ("ZP", "c16", (3, 3)),
    ("a", "c16", 2), ("S", "f8"), ("w", "c16"), ("e", "f8", 3),
    ("branch", "i4"), ("sigma", "i4"), ("layer", "i4"), ("gen", "i4"), ("alive", "i4"),
    ("lineage", "i8"),
], align=True)


class Medium(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("geometry", C.c_int),
        ("cp", C.c_double), ("cs", C.c_double), ("rho", C.c_double),
        ("n", C.c_int * 3), ("lo", C.c_double * 3), ("h", C.c_double * 3),
        ("tab", C.POINTER(C.c_double)), ("cs_ratio", C.c_double), ("two_fields", C.c_int),
        ("smooth", C.c_int), ("coef", C.POINTER(C.c_double)),
        ("x0", C.c_double * 3), ("amp", C.c_double), ("s", C.c_double), ("g", C.c_double * 3),
        ("nlayer", C.c_int), ("bound", C.c_double * 8),
        ("cpl", C.c_double * 8), ("csl", C.c_double * 8), ("rhol", C.c_double * 8), ("gradl", C.c_double * 8),
        ("anom_amp", C.c_double * 8), ("anom_beta", C.c_double * 8), ("anom_x", (C.c_double * 3) * 8),
        ("anom_w", (C.c_double * 3) * 8),
        ("surface", C.c_double),
    ]


HOMOGENEOUS, GRID, BUMP, LINEAR, LAYERED = 0, 1, 2, 3, 4


class PointForce(C.Structure):
    _fields_ = [("eps", C.c_double), ("x0", C.c_double * 3), ("d", C.c_double * 3), ("rho0", C.c_double),
                ("nq", C.c_int), ("qhalf", C.c_double), ("ndir", C.c_int), ("nshell", C.c_int),
                ("shell_lo", C.c_double), ("shell_hi", C.c_double), ("omega", C.c_double), ("t0", C.c_double),
                ("width", C.c_double), ("t_ref", C.c_double), ("branch_mask", C.c_int), ("cull_abs", C.c_double)]


class PointSource(C.Structure):
    _fields_ = [("eps", C.c_double), ("x0", C.c_double * 3), ("M", C.c_double * 6), ("rho0", C.c_double),
                ("nq", C.c_int), ("qhalf", C.c_double), ("ndir", C.c_int), ("nshell", C.c_int),
                ("shell_lo", C.c_double), ("shell_hi", C.c_double), ("ricker", C.c_int), ("branch_mask", C.c_int),
                ("cull_abs", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        L.om_beam_size.restype = C.c_size_t
        L.om_sum_points.restype = C.c_int64
        L.om_sum_points.argtypes = [vp, C.c_int64, vp, C.c_int64, C.c_double, C.c_double, vp]
        L.om_evolve.argtypes = [vp, vp, C.c_int64, C.c_double, C.c_int]
        L.om_evolve_svec.argtypes = [vp, vp, C.c_int64, C.c_double, C.c_int]
        L.om_fbi_many.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, C.c_double, vp]
        L.om_make_beams_many.restype = C.c_int64
        L.om_make_beams_many.argtypes = [vp, vp, vp, vp, C.c_int64, vp, vp, C.c_int64, C.c_int64, C.c_int,
                                         C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, vp]
        L.om_make_beams.restype = C.c_int
        L.om_make_beams.argtypes = [vp, vp, vp, vp, C.c_int, C.c_double, C.c_double, C.c_double,
                                    C.c_int, C.c_double, C.c_int64, C.c_int64, vp]
        L.om_grid_fields.argtypes = [vp, vp, vp, vp]
        L.om_grid_spline_coefficients.argtypes = [vp, vp, vp]
        L.om_speed_many.argtypes = [vp, C.c_int, vp, C.c_int64, vp]
        L.om_rhs_beam.argtypes = [vp, vp, vp]
        L.om_amplitude_vectors.argtypes = [vp, C.c_int64, vp]
        L.om_reframe_many.argtypes = [vp, C.c_int64]
        L.om_rk4_step.argtypes = [vp, vp, C.c_double]
        L.om_evolve_layered.restype = C.c_int64
        L.om_evolve_layered.argtypes = [vp, vp, C.c_int64, C.c_int64, C.c_double, C.c_int, C.c_int, C.c_double,
                                        vp, C.c_int]
        L.om_interface_modes.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_int, vp, vp, vp]
        L.om_free_surface_modes.argtypes = [vp, C.c_int, vp, vp, C.c_int, vp, vp, vp]
        L.om_interface_jacobians.argtypes = [vp, vp, vp, C.c_double, C.c_double, vp, vp, C.c_double, vp, vp]
        L.om_child_lineage.restype = C.c_int64
        L.om_child_lineage.argtypes = [C.c_int64, C.c_int, C.c_int]
        L.om_layer_exit.restype = C.c_int
        L.om_layer_exit.argtypes = [vp, C.c_int, vp, vp, vp]
        L.om_point_source_beams.restype = C.c_int64
        L.om_point_source_beams.argtypes = [vp, vp, vp]
        L.om_point_source_size.restype = C.c_size_t
        L.om_point_force_beams.restype = C.c_int64
        L.om_point_force_beams.argtypes = [vp, vp, vp]
        L.om_point_force_size.restype = C.c_size_t
        if L.om_point_force_size() != C.sizeof(PointForce):
            raise RuntimeError("oracle point-force layout mismatch")
        L.om_fibonacci_dirs.argtypes = [C.c_int, vp]
        L.om_gauss_legendre.argtypes = [C.c_int, C.c_double, C.c_double, vp, vp]
        L.om_ricker.restype = C.c_double
        L.om_ricker.argtypes = [C.c_double, C.c_double]
        if L.om_point_source_size() != C.sizeof(PointSource):
            raise RuntimeError("oracle point-source layout mismatch")
        L.om_medium_size.restype = C.c_size_t
        if L.om_medium_size() != C.sizeof(Medium):
            raise RuntimeError("oracle medium layout mismatch")
        if L.om_beam_size() != BEAM_DTYPE.itemsize:
            raise RuntimeError("oracle beam layout mismatch: C %d vs numpy %d"
                               % (L.om_beam_size(), BEAM_DTYPE.itemsize))
        _lib = L
    return _lib


def take_beams(b: np.ndarray, index) -> np.ndarray:
    """b[index] for a beam array, copied as raw records (numpy's per-field
    gather of this structured type is two orders of magnitude slower)."""
    raw = np.ascontiguousarray(b).view(np.dtype((np.void, BEAM_DTYPE.itemsize)))
    return raw[np.asarray(index)].view(BEAM_DTYPE)


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# media
# ---------------------------------------------------------------------------

class OracleMedium:
    """Owns an ``om_medium`` plus any derived node tables."""

    def __init__(self, m: Medium, keep=()):
        self.m = m
        self._keep = list(keep)

    @property
    def ref(self):
        return C.byref(self.m)


def homogeneous(cp: float, cs: float, rho: float = 1.0) -> OracleMedium:
    m = Medium()
    m.kind, m.cp, m.cs, m.rho = HOMOGENEOUS, cp, cs, rho
    return OracleMedium(m)


def bump(cp: float, cs: float, x0, amp: float, s: float) -> OracleMedium:
    m = Medium()
    m.kind, m.cp, m.cs = BUMP, cp, cs
    m.x0[:] = list(x0)
    m.amp, m.s = amp, s
    return OracleMedium(m)


def linear(cp: float, cs: float, g) -> OracleMedium:
    m = Medium()
    m.kind, m.cp, m.cs = LINEAR, cp, cs
    m.g[:] = list(g)
    return OracleMedium(m)


def grid(cp_nodes: np.ndarray, mesh, cs_ratio: float = None, cs_nodes: np.ndarray = None,
         smooth: bool = False) -> OracleMedium:
    """Periodic node-grid medium; nodes mesh.lo + i*mesh.h, arrays [z][y][x].
    smooth=False: trilinear interpolation of node values of c, grad c and
    its Hessian (grad c and H by finite differences on the nodes);
    smooth=True: c is the periodic cubic B-spline through the node values
    (C^2, grad c and H its exact derivatives)."""
    lib_ = lib()
    n = np.array(mesh.n, dtype=np.int32)
    h = np.array(mesh.h, dtype=np.float64)
    fields = [np.ascontiguousarray(cp_nodes, dtype=np.float64)]
    if cs_nodes is not None:
        fields.append(np.ascontiguousarray(cs_nodes, dtype=np.float64))
    tab = np.empty((len(fields),) + tuple(int(v) for v in mesh.n[::-1]) + (10,), dtype=np.float64)
    for i, f in enumerate(fields):
        lib_.om_grid_fields(_p(f), _p(n), _p(h), _p(tab[i]))
    m = Medium()
    m.kind = GRID
    m.n[:] = [int(v) for v in mesh.n]
    m.lo[:] = [float(v) for v in mesh.lo]
    m.h[:] = [float(v) for v in mesh.h]
    m.tab = tab.ctypes.data_as(C.POINTER(C.c_double))
    m.two_fields = 1 if cs_nodes is not None else 0
    m.cs_ratio = 0.0 if cs_ratio is None else cs_ratio
    keep = [tab, n, h]
    if smooth:
        coef = np.empty((len(fields),) + tuple(int(v) for v in mesh.n[::-1]), dtype=np.float64)
        for i, f in enumerate(fields):
            lib_.om_grid_spline_coefficients(_p(f), _p(n), _p(coef[i]))
        m.smooth = 1
        m.coef = coef.ctypes.data_as(C.POINTER(C.c_double))
        keep.append(coef)
    return OracleMedium(m, keep=keep)


def layered(geometry: int, bounds, cp, cs, rho, grad=None, surface=0.0, anomaly=None) -> OracleMedium:
    """Flat (geometry 0) or spherical (1) layers; grad: relative gradient per
    layer, c_b(x) = c_b,i (1 + grad[i] v(x)) with v = z or |x| (None: constant);
    surface > 0: a traction-free surface at z = surface above the last layer
    (flat) or |x| = surface around layer 0 (spherical); anomaly: {layer:
    (amp, beta, centre (3), axis weights (3))}, c_b multiplied by
    1 - amp exp(-beta sum_d w_d (x_d - centre_d)^2) in that layer."""
    m = Medium()
    m.kind, m.geometry = LAYERED, geometry
    m.nlayer = len(cp)
    m.bound[:len(bounds)] = list(bounds)
    m.cpl[:len(cp)] = list(cp)
    m.csl[:len(cs)] = list(cs)
    m.rhol[:len(rho)] = list(rho)
    if grad is not None:
        m.gradl[:len(grad)] = list(grad)
    for L, (amp, beta, x0, wts) in (anomaly or {}).items():
        m.anom_amp[L], m.anom_beta[L] = float(amp), float(beta)
        m.anom_x[L][:] = [float(v) for v in x0]
        m.anom_w[L][:] = [float(v) for v in wts]
    m.surface = float(surface)
    m.cp, m.cs, m.rho = cp[0], cs[0], rho[0]
    return OracleMedium(m)


def speed(med: OracleMedium, sp: int, x: np.ndarray):
    """c, grad c, Hessian of wave type sp at points x (n,3)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.empty((x.shape[0], 13))
    lib().om_speed_many(med.ref, sp, _p(x), x.shape[0], _p(out))
    return out[:, 0], out[:, 1:4], out[:, 4:].reshape(-1, 3, 3)


# ---------------------------------------------------------------------------
# decomposition
# ---------------------------------------------------------------------------

def fbi(f: np.ndarray, ymesh, q: np.ndarray, p: np.ndarray, eps: float) -> np.ndarray:
    """FBI transform (eq:psi integrand without alpha's prefactor) of the
    vector field f [3][z][y][x] at the (q, p) pairs (n,3), by quadrature on
    ymesh.  Returns complex (n,3)."""
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1, 3)
    f = np.ascontiguousarray(f, dtype=np.complex128)
    yn = np.array(ymesh.n, dtype=np.int32)
    ylo = np.array(ymesh.lo, dtype=np.float64)
    yh = np.array(ymesh.h, dtype=np.float64)
    out = np.empty((q.shape[0], 3), dtype=np.complex128)
    lib().om_fbi_many(_p(f), _p(yn), _p(ylo), _p(yh), _p(q), _p(p), q.shape[0], eps, _p(out))
    return out


def make_beams(qmesh, pmesh, Ft: np.ndarray, eps: float, iq: np.ndarray, ip: np.ndarray,
               one_way: bool = True, Gt: np.ndarray = None, branch_mask: int = 7,
               cull_abs: float = 0.0) -> np.ndarray:
    """Beams of the mesh points (qmesh[iq], pmesh[ip]) from their FBI values
    Ft (n,3) (and Gt (n,2,3) = FBI[g/c_P], FBI[g/c_S] when g != 0).
    Returned sorted by lineage."""
    lib_ = lib()
    iq = np.ascontiguousarray(iq, dtype=np.int64)
    ip = np.ascontiguousarray(ip, dtype=np.int64)
    qs = np.ascontiguousarray(qmesh.points()[iq])
    ps = np.ascontiguousarray(pmesh.points()[ip])
    nq, npm = qmesh.count, pmesh.count
    dq, dp = qmesh.cell_volume, pmesh.cell_volume
    F = np.ascontiguousarray(Ft, dtype=np.complex128).reshape(-1, 3)
    G = None if Gt is None else np.ascontiguousarray(Gt, dtype=np.complex128).reshape(-1, 2, 3)
    out = np.zeros(6 * len(iq), dtype=BEAM_DTYPE)
    k = lib_.om_make_beams_many(_p(qs), _p(ps), _p(F), None if G is None else _p(G), len(iq), _p(iq), _p(ip),
                                nq, npm, 1 if one_way else 0, eps, dq, dp, branch_mask, cull_abs, _p(out))
    out = out[:k]
    return take_beams(out, np.argsort(out["lineage"], kind="stable"))


def merge_s_beams(beams: np.ndarray, nqp: int) -> np.ndarray:
    """One S beam per (q, p, direction) in place of the SH and SV pair.

    The SH and SV beams of one (q, p, direction) start from the same data and
    both move with c_S, so their rays (Q, P, dzQ, dzP, S, frame axis e) are the
    same at every time (eq:char_plus, eq:char_minus, eq:DzDt), and the S
    amplitude equations (eq:amp_SV, eq:amp_SH) are linear in (a_SV, a_SH).
    The pair's contribution w_SH A_SH + w_SV A_SV to eq:FGA is therefore that
    of one beam on the common ray with weight 1 and amplitude
    w_SH a_SH + w_SV a_SV.  nqp = Nq Np: an SV beam's lineage is that of its
    SH partner plus 2 nqp (lineage ((b 2 + dir) Np + ip) Nq + iq); a beam
    whose partner is missing (culled) keeps only its own term.  The merged
    beam has the SH lineage and branch 1.  Returned sorted by lineage."""
    b = np.ascontiguousarray(beams)
    pb = b[b["branch"] == 0]
    sh, sv = b[b["branch"] == 1], b[b["branch"] == 2]
    key_sv = sv["lineage"] - 2 * nqp
    keys = np.union1d(sh["lineage"], key_sv)
    out = np.zeros(len(keys), dtype=BEAM_DTYPE)
    out["a"] = 0.0
    ray = ("Q", "P", "ZQ", "ZP", "S", "e", "sigma", "layer", "gen", "alive")
    for src, key in ((sh, sh["lineage"]), (sv, key_sv)):
        at = np.searchsorted(keys, key)
        for f in ray:
            out[f][at] = src[f]
        out["a"][at] += src["w"][:, None] * src["a"]
    # the two members of a pair share the ray exactly
    both_sh = np.isin(sh["lineage"], key_sv)
    both_sv = np.isin(key_sv, sh["lineage"])
    a_, b_ = sh[both_sh], sv[both_sv][np.argsort(key_sv[both_sv], kind="stable")]
    a_ = a_[np.argsort(a_["lineage"], kind="stable")]
    for f in ("Q", "P", "ZQ", "ZP", "S", "e", "sigma"):
        if not np.array_equal(a_[f], b_[f]):
            raise ValueError("SH and SV beams of one (q, p, direction) differ in " + f)
    out["lineage"] = keys
    out["branch"] = 1
    out["w"] = 1.0
    m = np.concatenate([pb, out])
    return take_beams(m, np.argsort(m["lineage"], kind="stable"))


def decompose(work, one_way: bool = True, iq=None, ip=None, branch_mask: int = 7) -> np.ndarray:
    """Step 1 of the method (Sec. 2.2 algorithm): FBI weights and initial
    beams for all mesh points, or for the listed (iq, ip) pairs."""
    if iq is None:
        iq_all, ip_all = np.meshgrid(np.arange(work.qmesh.count), np.arange(work.pmesh.count), indexing="xy")
        iq, ip = iq_all.ravel(), ip_all.ravel()
    iq = np.asarray(iq, dtype=np.int64)
    ip = np.asarray(ip, dtype=np.int64)
    Ft = fbi(work.f, work.ymesh, work.qmesh.points()[iq], work.pmesh.points()[ip], work.eps)
    return make_beams(work.qmesh, work.pmesh, Ft, work.eps, iq, ip, one_way=one_way,
                      branch_mask=branch_mask, cull_abs=work.cull_abs)


def decompose_two_way(work, g: np.ndarray, iq=None, ip=None, branch_mask: int = 7) -> np.ndarray:
    """Step 1 with both directions (eq:psi, eq:alpha^k): initial displacement
    work.f and velocity g (complex [3][z][y][x] on work.ymesh); the speeds
    c_P, c_S at the quadrature points come from the work's medium."""
    if iq is None:
        iq_all, ip_all = np.meshgrid(np.arange(work.qmesh.count), np.arange(work.pmesh.count), indexing="xy")
        iq, ip = iq_all.ravel(), ip_all.ravel()
    iq = np.asarray(iq, dtype=np.int64)
    ip = np.asarray(ip, dtype=np.int64)
    qs, ps = work.qmesh.points()[iq], work.pmesh.points()[ip]
    Ft = fbi(work.f, work.ymesh, qs, ps, work.eps)
    med = medium_for(work)
    y = work.ymesh.points()
    n = tuple(int(v) for v in work.ymesh.n[::-1])
    Gt = np.empty((len(iq), 2, 3), dtype=np.complex128)
    for sp in (0, 1):
        c = speed(med, sp, y)[0].reshape(n)
        Gt[:, sp] = fbi(np.asarray(g) / c[None], work.ymesh, qs, ps, work.eps)
    return make_beams(work.qmesh, work.pmesh, Ft, work.eps, iq, ip, one_way=False, Gt=Gt,
                      branch_mask=branch_mask, cull_abs=work.cull_abs)


def plant_two_way_error(kind: int) -> None:
    """Plant a known mistake in the two-way weight (see om_plant_twoway_error
    in fga_oracle.c; 0 removes it).  Only the pins of that weight call this."""
    C.c_int.in_dll(lib(), "om_plant_twoway_error").value = int(kind)


# ---------------------------------------------------------------------------
# evolution and reconstruction
# ---------------------------------------------------------------------------

def evolve(med: OracleMedium, beams: np.ndarray, dt: float, nsteps: int, s_vector: bool = False) -> None:
    """Advance beams in place by nsteps classic RK4 steps.  s_vector: S
    amplitudes advanced as the frame-free polarisation vector (parallel
    transport along the ray) and returned to the beam's frame at the end."""
    assert beams.dtype == BEAM_DTYPE and beams.flags.c_contiguous
    f = lib().om_evolve_svec if s_vector else lib().om_evolve
    f(med.ref, _p(beams), beams.shape[0], dt, nsteps)


def evolve_layered(med: OracleMedium, beams: np.ndarray, dt: float, nsteps: int, gmax: int = 3,
                   child_cut: float = 1e-3, capacity: int = None, s_vector: bool = False):
    """Advance beams by nsteps RK4 steps in a layered medium, splitting beams
    at interfaces.  Returns (beam array holding parents and children; retired
    beams have alive = 0, number of beams retired at the generation cap).
    s_vector: where some layer curves the rays, S beams take their regular
    steps with the frame-free amplitude."""
    n = beams.shape[0]
    cap = capacity if capacity is not None else max(16, 8 * n)
    buf = np.zeros(cap, dtype=BEAM_DTYPE)
    buf[:n] = beams
    ncap = C.c_int64(0)
    m = lib().om_evolve_layered(med.ref, _p(buf), n, cap, dt, nsteps, gmax, child_cut, C.byref(ncap),
                                1 if s_vector else 0)
    if m < 0:
        raise RuntimeError("beam capacity %d exceeded" % cap)
    return buf[:m].copy(), int(ncap.value)


# interface mode record, as filled by om_interface_modes
MODE_DTYPE = np.dtype([("exists", np.int32), ("sp", np.int32), ("side", np.int32), ("P", np.float64, 3),
                       ("A", np.complex128, 3)], align=True)


def interface_modes(med: OracleMedium, layer: int, new_layer: int, normal, sp_in: int, P, A, x=(0.0, 0.0, 0.0)):
    """Snell / elastic boundary problem at the interface point x: returns the
    4 outgoing modes (P reflected, S reflected, P transmitted, S transmitted)."""
    out = np.zeros(4, dtype=MODE_DTYPE)
    n = np.ascontiguousarray(normal, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.complex128)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    lib().om_interface_modes(med.ref, layer, new_layer, _p(xx), _p(n), sp_in, _p(P), _p(A), _p(out))
    return out


def free_surface_modes(med: OracleMedium, layer: int, normal, sp_in: int, P, A, x=(0.0, 0.0, 0.0)):
    """Reflected modes (P, S; the transmitted two do not exist) of a plane
    wave at a traction-free surface with outward normal `normal` at x."""
    out = np.zeros(4, dtype=MODE_DTYPE)
    n = np.ascontiguousarray(normal, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.complex128)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    lib().om_free_surface_modes(med.ref, layer, _p(xx), _p(n), sp_in, _p(P), _p(A), _p(out))
    return out


def interface_jacobians(normal, Pin, Pout, c_in, c_out, ZQ, ZP, grad_in=(0, 0, 0), grad_out=(0, 0, 0), kcurv=0.0):
    """Map (dzQ, dzP) across an interface to one outgoing mode (kcurv: the
    signed curvature s/R of a spherical interface, 0 for a flat one)."""
    ZQ = np.array(ZQ, dtype=np.complex128, order="C")
    ZP = np.array(ZP, dtype=np.complex128, order="C")
    args = [np.ascontiguousarray(v, dtype=np.float64) for v in (normal, Pin, Pout)]
    g = [np.ascontiguousarray(v, dtype=np.float64) for v in (grad_in, grad_out)]
    lib().om_interface_jacobians(_p(args[0]), _p(args[1]), _p(args[2]), c_in, c_out, _p(g[0]), _p(g[1]),
                                 float(kcurv), _p(ZQ), _p(ZP))
    return ZQ, ZP


def point_source(eps, x0, M, nq, qhalf=None, ndir=64, nshell=4, shell_lo=0.2, shell_hi=2.5, ricker=True,
                 rho0=0.0, branch_mask=7, cull_abs=0.0) -> PointSource:
    """Parameters of a point moment-tensor source (M = xx, yy, zz, xy, xz, yz)."""
    src = PointSource()
    src.eps = eps
    src.x0[:] = list(x0)
    src.M[:] = list(M)
    src.rho0 = rho0
    src.nq = nq
    src.qhalf = 4.0 * eps ** 0.5 if qhalf is None else qhalf
    src.ndir, src.nshell = ndir, nshell
    src.shell_lo, src.shell_hi = shell_lo, shell_hi
    src.ricker = 1 if ricker else 0
    src.branch_mask = branch_mask
    src.cull_abs = cull_abs
    return src


def point_source_candidates(src: PointSource) -> int:
    return src.nq ** 3 * src.ndir * src.nshell * bin(src.branch_mask & 7).count("1") * 2


def point_source_beams(med: OracleMedium, src: PointSource) -> np.ndarray:
    """Beams of a point moment-tensor source (closed-form weights), lineage order."""
    out = np.zeros(point_source_candidates(src), dtype=BEAM_DTYPE)
    n = lib().om_point_source_beams(med.ref, C.byref(src), _p(out))
    return out[:n].copy()


def point_force(eps, x0, d, nq, qhalf, ndir, nshell, omega, t0, width, t_ref, shell_lo=0.2, shell_hi=2.5,
                rho0=0.0, branch_mask=7, cull_abs=0.0) -> PointForce:
    """Parameters of a point force d F(t), F(t) = cos(omega (t + t0)) exp(-(t + t0)^2/width^2),
    whose beams are launched at t_ref."""
    src = PointForce()
    src.eps = eps
    src.x0[:] = list(x0)
    src.d[:] = list(d)
    src.rho0 = rho0
    src.nq, src.qhalf, src.ndir, src.nshell = nq, qhalf, ndir, nshell
    src.shell_lo, src.shell_hi = shell_lo, shell_hi
    src.omega, src.t0, src.width, src.t_ref = omega, t0, width, t_ref
    src.branch_mask = branch_mask
    src.cull_abs = cull_abs
    return src


def point_force_beams(med: OracleMedium, src: PointForce) -> np.ndarray:
    """Beams of a point force with its time function folded in (Duhamel), lineage order."""
    ncand = src.nq ** 3 * src.ndir * src.nshell * bin(src.branch_mask & 7).count("1") * 2
    out = np.zeros(ncand, dtype=BEAM_DTYPE)
    n = lib().om_point_force_beams(med.ref, C.byref(src), _p(out))
    return out[:n].copy()


def fibonacci_dirs(n: int) -> np.ndarray:
    d = np.zeros((n, 3))
    lib().om_fibonacci_dirs(n, _p(d))
    return d


def gauss_legendre(n: int, a: float, b: float):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().om_gauss_legendre(n, a, b, _p(x), _p(w))
    return x, w


def ricker(w: float, w0: float) -> float:
    return lib().om_ricker(w, w0)


def child_lineage(parent: int, gen: int, k: int) -> int:
    return int(lib().om_child_lineage(parent, gen, k))


def rhs(med: OracleMedium, beam: np.ndarray) -> np.ndarray:
    """Time derivative of one beam's state (fields Q, P, ZQ, ZP, a, S)."""
    b = np.ascontiguousarray(beam.reshape(1))
    d = np.zeros(1, dtype=BEAM_DTYPE)
    lib().om_rhs_beam(med.ref, _p(b), _p(d))
    return d[0]


def amplitude_vectors(beams: np.ndarray) -> np.ndarray:
    """Physical amplitude vectors A (n,3) complex."""
    b = np.ascontiguousarray(beams)
    A = np.empty((b.shape[0], 3), dtype=np.complex128)
    lib().om_amplitude_vectors(_p(b), b.shape[0], _p(A))
    return A


def reframe(beams: np.ndarray) -> None:
    lib().om_reframe_many(_p(beams), beams.shape[0])


def spherical_to_cartesian(rtp: np.ndarray) -> np.ndarray:
    """Stations given as (r, theta, phi), theta the longitude and phi the
    latitude (the coordinates of the Earth examples, opening of Sec. 3):
    x = (r cos theta cos phi, r sin theta cos phi, r sin phi)."""
    rtp = np.asarray(rtp, dtype=np.float64).reshape(-1, 3)
    r, th, ph = rtp[:, 0], rtp[:, 1], rtp[:, 2]
    return np.stack([r * np.cos(th) * np.cos(ph), r * np.sin(th) * np.cos(ph), r * np.sin(ph)], axis=1)


def sum_points(beams: np.ndarray, x: np.ndarray, eps: float, tau: float):
    """Windowed Gaussian summation (eq:FGA) at points x (n,3).
    Returns (u (n,3) complex, number of in-window beam-point terms)."""
    b = np.ascontiguousarray(beams)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.empty((x.shape[0], 3), dtype=np.complex128)
    cnt = lib().om_sum_points(_p(b), b.shape[0], _p(x), x.shape[0], eps, tau, _p(out))
    return out, int(cnt)


def medium_for(work) -> OracleMedium:
    if work.medium_nodes is None:
        return homogeneous(work.cp0, work.cs0)
    return grid(work.medium_nodes, work.medium_grid, cs_ratio=work.cs_ratio, smooth=work.medium_smooth)
