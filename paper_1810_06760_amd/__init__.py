"""Python binding of the gfx950 FGA library (libfga.so).

Thin ctypes marshalling over the C ABI declared in include/fga.h: every step
of the method runs in the library's HIP kernels; PyTorch only provides
device memory and the current stream.  Importing this module does not need a
GPU, but every call does, and a missing or unbuilt library raises at once
(there is no CPU fallback).

The functions keep the C names: fga_medium_grid_build, fga_decompose,
fga_evolve, fga_reconstruct_points, fga_reconstruct_grid.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfga.so")
_lib = None

# plane indices (include/fga.h)
FGA_Q, FGA_P = 0, 3
FGA_ZQ_RE, FGA_ZQ_IM, FGA_ZP_RE, FGA_ZP_IM = 6, 15, 24, 33
FGA_A0_RE, FGA_A0_IM, FGA_A1_RE, FGA_A1_IM = 42, 43, 44, 45
FGA_S, FGA_W_RE, FGA_W_IM, FGA_E = 46, 47, 48, 49
FGA_NF64 = 52
FGA_BRANCH, FGA_SIGMA, FGA_LAYER, FGA_GEN, FGA_FLAGS, FGA_NI32 = 0, 1, 2, 3, 4, 5
FGA_FLAG_ALIVE, FGA_FLAG_QUARANTINED = 1, 2
FGA_MEDIUM_HOMOGENEOUS, FGA_MEDIUM_GRID, FGA_MEDIUM_LAYERED = 0, 1, 2
FGA_FP64, FGA_FP32, FGA_BF16X3, FGA_FP16X3, FGA_FP16X2, FGA_FP32_ACC32 = 0, 1, 2, 3, 4, 5
FGA_COORDS_CARTESIAN, FGA_COORDS_SPHERICAL = 0, 1
FGA_GRID_NODE_DOUBLES = 16
STATUS = {0: "FGA_OK", 1: "FGA_EINVAL", 2: "FGA_ENOMEM", 3: "FGA_EDEVICE", 4: "FGA_ENUMERIC",
          5: "FGA_ECAPACITY", 6: "FGA_EUNSUPPORTED"}

EXPORTED = ["fga_last_error", "fga_version", "fga_medium_grid_table_bytes", "fga_medium_grid_build",
            "fga_decompose_workspace_bytes", "fga_decompose_candidates", "fga_decompose",
            "fga_evolve_workspace_bytes", "fga_evolve", "fga_reconstruct_points_workspace_bytes",
            "fga_reconstruct_points", "fga_reconstruct_points_noalloc_max_bytes", "fga_reconstruct_points_noalloc",
            "fga_reconstruct_grid_workspace_bytes", "fga_reconstruct_grid",
            "fga_reconstruct_grid_add",
            "fga_profile_enable", "fga_profile_read", "fga_server_footprint", "fga_server_create",
            "fga_server_submit", "fga_server_poll", "fga_server_status", "fga_server_destroy",
            "fga_point_source_candidates", "fga_decompose_point_source_workspace_bytes",
            "fga_decompose_point_source", "fga_point_force_candidates", "fga_decompose_point_force_workspace_bytes",
            "fga_decompose_point_force", "fga_beams_info", "fga_beams_export", "fga_beams_import"]
FGA_K_INTEGRATE, FGA_K_SUM_POINTS, FGA_K_GRID_TILE, FGA_K_FBI_GEMM = 0, 1, 2, 3
KERNEL_NAMES = {0: "integrate", 1: "sum_points", 2: "grid_tile", 3: "fbi_gemm"}


class FgaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Beams(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("f64", C.c_void_p), ("i32", C.c_void_p),
                ("lineage", C.c_void_p)]


class MediumC(C.Structure):
    _fields_ = [("kind", C.c_int), ("cp", C.c_double), ("cs", C.c_double), ("rho", C.c_double),
                ("n", C.c_int * 3), ("lo", C.c_double * 3), ("h", C.c_double * 3), ("table", C.c_void_p),
                ("two_fields", C.c_int), ("cs_ratio", C.c_double), ("geometry", C.c_int), ("nlayer", C.c_int),
                ("bound", C.c_double * 8), ("cpl", C.c_double * 8), ("csl", C.c_double * 8),
                ("rhol", C.c_double * 8), ("gradl", C.c_double * 8),
                ("anom_amp", C.c_double * 8), ("anom_beta", C.c_double * 8), ("anom_x", (C.c_double * 3) * 8),
                ("anom_w", (C.c_double * 3) * 8),
                ("surface", C.c_double), ("smooth", C.c_int)]


class MeshC(C.Structure):
    _fields_ = [("eps", C.c_double),
                ("nq", C.c_int * 3), ("qlo", C.c_double * 3), ("qh", C.c_double * 3),
                ("np", C.c_int * 3), ("plo", C.c_double * 3), ("ph", C.c_double * 3),
                ("ny", C.c_int * 3), ("ylo", C.c_double * 3), ("yh", C.c_double * 3),
                ("branch_mask", C.c_int), ("one_way", C.c_int), ("cull_abs", C.c_double), ("merge_s", C.c_int)]


class ReceiversC(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyz", C.c_void_p), ("stride", C.c_int), ("eps", C.c_double),
                ("tau", C.c_double), ("precision", C.c_int), ("coords", C.c_int)]


class EvolveOptsC(C.Structure):
    _fields_ = [("chunk", C.c_int), ("cutoff_abs", C.c_double), ("compact", C.c_int), ("batch", C.c_int64),
                ("resort", C.c_int), ("gen_max", C.c_int), ("child_cut", C.c_double), ("s_vector", C.c_int)]


class EvolveStatsC(C.Structure):
    _fields_ = [("beam_steps", C.c_int64), ("evals", C.c_int64), ("culled", C.c_int64),
                ("quarantined", C.c_int64), ("crossings", C.c_int64), ("spawned", C.c_int64), ("capped", C.c_int64)]


class PointSourceC(C.Structure):
    _fields_ = [("eps", C.c_double), ("x0", C.c_double * 3), ("M", C.c_double * 6), ("rho0", C.c_double),
                ("nq", C.c_int), ("qhalf", C.c_double), ("ndir", C.c_int), ("nshell", C.c_int),
                ("shell_lo", C.c_double), ("shell_hi", C.c_double), ("ricker", C.c_int), ("branch_mask", C.c_int),
                ("cull_abs", C.c_double), ("merge_s", C.c_int)]


class PointForceC(C.Structure):
    _fields_ = [("eps", C.c_double), ("x0", C.c_double * 3), ("d", C.c_double * 3), ("rho0", C.c_double),
                ("nq", C.c_int), ("qhalf", C.c_double), ("ndir", C.c_int), ("nshell", C.c_int),
                ("shell_lo", C.c_double), ("shell_hi", C.c_double), ("omega", C.c_double), ("t0", C.c_double),
                ("width", C.c_double), ("t_ref", C.c_double), ("branch_mask", C.c_int), ("cull_abs", C.c_double),
                ("merge_s", C.c_int)]


class RequestC(C.Structure):
    _fields_ = [("medium", MediumC), ("mesh", MeshC), ("f", C.c_void_p), ("n_receivers", C.c_int64),
                ("receivers", C.c_void_p), ("tau", C.c_double), ("dt", C.c_double), ("nsteps", C.c_int),
                ("stride", C.c_int), ("seis_out", C.c_void_p), ("precision", C.c_int), ("point_source", C.c_int),
                ("source", PointSourceC), ("receiver_coords", C.c_int)]


class CompletionC(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("footprint", C.c_size_t), ("beams", C.c_int64), ("beam_steps", C.c_int64),
                ("evals", C.c_int64)]


def lib():
    """Load libfga.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfga.so is not built (run python -m paper_1810_06760_amd.build); "
                               "there is no CPU fallback")
        # torch first: the library then binds to the HIP runtime torch has loaded,
        # so device memory and streams from torch are valid in it
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i64, sz, st = C.c_void_p, C.c_int64, C.c_size_t, C.c_int
        L.fga_last_error.restype = C.c_char_p
        L.fga_version.restype = C.c_char_p
        L.fga_medium_grid_table_bytes.restype = sz
        L.fga_medium_grid_table_bytes.argtypes = [vp, C.c_int]
        L.fga_medium_grid_build.restype = st
        L.fga_medium_grid_build.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fga_decompose_workspace_bytes.restype = sz
        L.fga_decompose_workspace_bytes.argtypes = [vp, C.c_int]
        L.fga_decompose_candidates.restype = i64
        L.fga_decompose_candidates.argtypes = [vp]
        L.fga_decompose.restype = st
        L.fga_decompose.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
        L.fga_evolve_workspace_bytes.restype = sz
        L.fga_evolve_workspace_bytes.argtypes = [vp, C.c_int, vp, vp]
        L.fga_evolve.restype = st
        L.fga_evolve.argtypes = [vp, vp, C.c_double, C.c_int, vp, vp, vp, vp, sz, vp, vp]
        L.fga_reconstruct_points_workspace_bytes.restype = sz
        L.fga_reconstruct_points_workspace_bytes.argtypes = [vp, i64]
        L.fga_reconstruct_points.restype = st
        L.fga_reconstruct_points.argtypes = [vp, C.c_double, C.c_double, i64, vp, C.c_int, vp, vp, sz, vp, vp]
        L.fga_reconstruct_points_noalloc_max_bytes.restype = sz
        L.fga_reconstruct_points_noalloc_max_bytes.argtypes = []
        L.fga_reconstruct_points_noalloc.restype = st
        L.fga_reconstruct_points_noalloc.argtypes = [vp, C.c_double, C.c_double, i64, vp, C.c_int, vp, vp, vp]
        L.fga_reconstruct_grid_workspace_bytes.restype = sz
        L.fga_reconstruct_grid_workspace_bytes.argtypes = [vp, vp, C.c_double, C.c_double, vp]
        L.fga_reconstruct_grid.restype = st
        L.fga_reconstruct_grid.argtypes = [vp, C.c_double, C.c_double, vp, vp, vp, C.c_int, vp, vp, sz, vp, vp]
        L.fga_reconstruct_grid_add.restype = st
        L.fga_reconstruct_grid_add.argtypes = L.fga_reconstruct_grid.argtypes
        L.fga_beams_info.restype = st
        L.fga_beams_info.argtypes = [vp, vp, vp, sz, vp]
        L.fga_beams_export.restype = st
        L.fga_beams_export.argtypes = [vp, vp, vp, vp, vp]
        L.fga_beams_import.restype = st
        L.fga_beams_import.argtypes = [vp, i64, vp, vp, vp, vp]
        L.fga_profile_enable.restype = st
        L.fga_profile_enable.argtypes = [C.c_int]
        L.fga_profile_read.restype = st
        L.fga_profile_read.argtypes = [C.c_int, vp, vp, C.c_int]
        L.fga_point_source_candidates.restype = i64
        L.fga_point_source_candidates.argtypes = [vp]
        L.fga_decompose_point_source_workspace_bytes.restype = sz
        L.fga_decompose_point_source_workspace_bytes.argtypes = [vp]
        L.fga_decompose_point_source.restype = st
        L.fga_decompose_point_source.argtypes = [vp, vp, vp, vp, sz, vp]
        L.fga_point_force_candidates.restype = i64
        L.fga_point_force_candidates.argtypes = [vp]
        L.fga_decompose_point_force_workspace_bytes.restype = sz
        L.fga_decompose_point_force_workspace_bytes.argtypes = [vp]
        L.fga_decompose_point_force.restype = st
        L.fga_decompose_point_force.argtypes = [vp, vp, vp, vp, sz, vp]
        L.fga_server_footprint.restype = sz
        L.fga_server_footprint.argtypes = [vp]
        L.fga_server_create.restype = st
        L.fga_server_create.argtypes = [sz, C.c_int, vp]
        L.fga_server_submit.restype = st
        L.fga_server_submit.argtypes = [vp, vp, vp]
        L.fga_server_poll.restype = st
        L.fga_server_poll.argtypes = [vp, vp, C.c_int, vp, C.c_int]
        L.fga_server_status.restype = st
        L.fga_server_status.argtypes = [vp, vp, vp, vp, vp]
        L.fga_server_destroy.restype = st
        L.fga_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise FgaError(status, lib().fga_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the FGA library needs a ROCm GPU; none is visible")
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _workspace(nbytes, ws=None):
    """A byte tensor of at least nbytes: ws itself if it is large enough."""
    if ws is not None and ws.numel() >= nbytes:
        return ws
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def _dev(a, dtype=None):
    """numpy / torch array -> contiguous CUDA tensor."""
    torch = _torch()
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a))
    a = a.to(device="cuda")
    if dtype is not None:
        a = a.to(dtype)
    return a.contiguous()


def _complex_dev(a):
    """complex array -> CUDA float64 tensor of interleaved (re, im)."""
    torch = _torch()
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.complex128)
        return torch.from_numpy(a.view(np.float64).copy()).to("cuda")
    if a.dtype == torch.float64 and a.is_cuda and a.is_contiguous():
        return a  # already interleaved (re, im) on the device
    return torch.view_as_real(a.to(torch.complex128).contiguous()).reshape(-1).to("cuda").contiguous()


# ---------------------------------------------------------------------------
# beams
# ---------------------------------------------------------------------------

class BeamsStatsC(C.Structure):
    _fields_ = [("count", C.c_int64), ("alive", C.c_int64), ("quarantined", C.c_int64),
                ("by_branch", C.c_int64 * 3), ("children", C.c_int64)]


FGA_BEAMS_INFO_WORKSPACE = 64


class BeamSet:
    """Structure-of-arrays beam planes in device memory (caller-owned)."""

    def __init__(self, capacity: int):
        torch = _torch()
        self.capacity = int(capacity)
        self.f64 = torch.zeros((FGA_NF64, max(self.capacity, 1)), dtype=torch.float64, device="cuda")
        self.i32 = torch.zeros((FGA_NI32, max(self.capacity, 1)), dtype=torch.int32, device="cuda")
        self.lineage = torch.zeros(max(self.capacity, 1), dtype=torch.int64, device="cuda")
        self.c = Beams(self.capacity, 0, self.f64.data_ptr(), self.i32.data_ptr(), self.lineage.data_ptr())

    @property
    def count(self) -> int:
        return int(self.c.count)

    def info(self) -> dict:
        """fga_beams_info: counts over the beams [0, count)."""
        torch = _torch()
        ws = torch.empty(FGA_BEAMS_INFO_WORKSPACE // 8, dtype=torch.float64, device="cuda")
        out = BeamsStatsC()
        _check(lib().fga_beams_info(C.byref(self.c), C.byref(out), ws.data_ptr(), FGA_BEAMS_INFO_WORKSPACE,
                                    _stream()))
        return {"count": out.count, "alive": out.alive, "quarantined": out.quarantined,
                "by_branch": list(out.by_branch), "children": out.children}

    def export(self, index=None) -> dict:
        """Host copy of the live beams (fga_beams_export; or of the slots in
        `index`, a device int64 tensor): dict of numpy arrays."""
        if index is None:
            n = self.count
            F = np.empty((FGA_NF64, n))
            I = np.empty((FGA_NI32, n), dtype=np.int32)
            lin = np.empty(n, dtype=np.int64)
            _check(lib().fga_beams_export(C.byref(self.c), F.ctypes.data, I.ctypes.data, lin.ctypes.data,
                                          _stream()))
        else:
            n = int(index.numel())
            F = self.f64[:, index].cpu().numpy()
            I = self.i32[:, index].cpu().numpy()
            lin = self.lineage[index].cpu().numpy().copy()
        ZQ = (F[FGA_ZQ_RE:FGA_ZQ_RE + 9] + 1j * F[FGA_ZQ_IM:FGA_ZQ_IM + 9]).T.reshape(n, 3, 3)
        ZP = (F[FGA_ZP_RE:FGA_ZP_RE + 9] + 1j * F[FGA_ZP_IM:FGA_ZP_IM + 9]).T.reshape(n, 3, 3)
        a = np.stack([F[FGA_A0_RE] + 1j * F[FGA_A0_IM], F[FGA_A1_RE] + 1j * F[FGA_A1_IM]], axis=1)
        return {
            "Q": F[FGA_Q:FGA_Q + 3].T.copy(), "P": F[FGA_P:FGA_P + 3].T.copy(), "ZQ": ZQ, "ZP": ZP, "a": a,
            "S": F[FGA_S].copy(), "w": F[FGA_W_RE] + 1j * F[FGA_W_IM], "e": F[FGA_E:FGA_E + 3].T.copy(),
            "branch": I[FGA_BRANCH].copy(), "sigma": I[FGA_SIGMA].copy(), "layer": I[FGA_LAYER].copy(),
            "gen": I[FGA_GEN].copy(), "flags": I[FGA_FLAGS].copy(),
            "lineage": lin,
        }

    def load(self, d: dict) -> None:
        """Set the live beams from host arrays (same keys as export();
        fga_beams_import)."""
        n = len(d["Q"])
        if n > self.capacity:
            raise ValueError("capacity %d < %d beams" % (self.capacity, n))
        F = np.zeros((FGA_NF64, n))
        F[FGA_Q:FGA_Q + 3] = np.asarray(d["Q"]).T
        F[FGA_P:FGA_P + 3] = np.asarray(d["P"]).T
        ZQ = np.asarray(d["ZQ"]).reshape(n, 9).T
        ZP = np.asarray(d["ZP"]).reshape(n, 9).T
        F[FGA_ZQ_RE:FGA_ZQ_RE + 9], F[FGA_ZQ_IM:FGA_ZQ_IM + 9] = ZQ.real, ZQ.imag
        F[FGA_ZP_RE:FGA_ZP_RE + 9], F[FGA_ZP_IM:FGA_ZP_IM + 9] = ZP.real, ZP.imag
        a = np.asarray(d["a"])
        F[FGA_A0_RE], F[FGA_A0_IM], F[FGA_A1_RE], F[FGA_A1_IM] = a[:, 0].real, a[:, 0].imag, a[:, 1].real, a[:, 1].imag
        F[FGA_S] = d["S"]
        F[FGA_W_RE], F[FGA_W_IM] = np.real(d["w"]), np.imag(d["w"])
        F[FGA_E:FGA_E + 3] = np.asarray(d["e"]).T
        I = np.zeros((FGA_NI32, n), dtype=np.int32)
        I[FGA_BRANCH], I[FGA_SIGMA] = d["branch"], d["sigma"]
        I[FGA_LAYER] = d.get("layer", 0)
        I[FGA_GEN] = d.get("gen", 0)
        I[FGA_FLAGS] = d.get("flags", FGA_FLAG_ALIVE)
        lin = np.ascontiguousarray(d["lineage"], dtype=np.int64)
        _check(lib().fga_beams_import(C.byref(self.c), n, F.ctypes.data, I.ctypes.data, lin.ctypes.data,
                                      _stream()))


# ---------------------------------------------------------------------------
# media
# ---------------------------------------------------------------------------

class Medium:
    """A medium description plus the device tables it references."""

    def __init__(self, c: MediumC, keep=()):
        self.c = c
        self._keep = list(keep)

    @staticmethod
    def homogeneous(cp: float, cs: float, rho: float = 1.0) -> "Medium":
        m = MediumC()
        m.kind, m.cp, m.cs, m.rho = FGA_MEDIUM_HOMOGENEOUS, cp, cs, rho
        return Medium(m)

    @staticmethod
    def grid(cp_nodes, mesh, cs_ratio: float = None, cs_nodes=None, smooth: bool = False) -> "Medium":
        """Periodic node grid (nodes mesh.lo + i*mesh.h), arrays [z][y][x];
        smooth: c is the cubic B-spline through the node values (C^2) instead
        of the trilinear interpolation of central-difference node fields."""
        torch = _torch()
        n = (C.c_int * 3)(*[int(v) for v in mesh.n])
        h = (C.c_double * 3)(*[float(v) for v in mesh.h])
        cp = _dev(cp_nodes, torch.float64)
        cs = _dev(cs_nodes, torch.float64) if cs_nodes is not None else None
        nbytes = lib().fga_medium_grid_table_bytes(n, 1 if cs is not None else 0)
        table = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
        fga_medium_grid_build(n, h, cp, cs, table)
        # complete before any other stream (a server slot) reads the table
        torch.cuda.synchronize()
        m = MediumC()
        m.kind = FGA_MEDIUM_GRID
        m.n[:] = list(n)
        m.lo[:] = [float(v) for v in mesh.lo]
        m.h[:] = list(h)
        m.table = table.data_ptr()
        m.two_fields = 1 if cs is not None else 0
        m.cs_ratio = 0.0 if cs_ratio is None else float(cs_ratio)
        m.smooth = 1 if smooth else 0
        return Medium(m, keep=[table, cp, cs])

    @staticmethod
    def layered(geometry: int, bounds, cp, cs, rho, grad=None, surface=0.0, anomaly=None) -> "Medium":
        """Flat (geometry 0) or spherical (1) layers; grad: relative gradient
        per layer, c_b(x) = c_b,l (1 + grad[l] v(x)), v = z or |x| (None: constant);
        surface > 0: a traction-free surface at z = surface above the last layer
        (flat) or |x| = surface around layer 0 (spherical); anomaly: {layer:
        (amp, beta, centre (3), axis weights (3))}, the layer's speeds times
        1 - amp exp(-beta sum_d w_d (x_d - centre_d)^2)."""
        m = MediumC()
        m.kind, m.geometry, m.nlayer = FGA_MEDIUM_LAYERED, geometry, len(cp)
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
        return Medium(m)


def medium_for(work) -> Medium:
    if work.medium_nodes is None:
        return Medium.homogeneous(work.cp0, work.cs0)
    return Medium.grid(work.medium_nodes, work.medium_grid, cs_ratio=work.cs_ratio, smooth=work.medium_smooth)


# ---------------------------------------------------------------------------
# the C calls
# ---------------------------------------------------------------------------

def fga_medium_grid_build(n, h, cp_nodes, cs_nodes, table):
    _check(lib().fga_medium_grid_build(n, h, _ptr(cp_nodes), _ptr(cs_nodes), _ptr(table), _stream()))


def make_mesh(eps, qmesh, pmesh, ymesh, branch_mask=7, one_way=True, cull_abs=0.0, merge_s=False) -> MeshC:
    m = MeshC()
    m.eps = eps
    m.nq[:], m.qlo[:], m.qh[:] = [int(v) for v in qmesh.n], list(qmesh.lo), list(qmesh.h)
    m.np[:], m.plo[:], m.ph[:] = [int(v) for v in pmesh.n], list(pmesh.lo), list(pmesh.h)
    m.ny[:], m.ylo[:], m.yh[:] = [int(v) for v in ymesh.n], list(ymesh.lo), list(ymesh.h)
    m.branch_mask, m.one_way, m.cull_abs = branch_mask, 1 if one_way else 0, cull_abs
    m.merge_s = 1 if merge_s else 0
    return m


def mesh_for(work, one_way=True, branch_mask=7, merge_s=False) -> MeshC:
    """merge_s: one S beam per (q, p, direction) carrying the SH and SV weights."""
    return make_mesh(work.eps, work.qmesh, work.pmesh, work.ymesh, branch_mask=branch_mask, one_way=one_way,
                     cull_abs=work.cull_abs, merge_s=merge_s)


def fga_decompose(medium: Medium, mesh: MeshC, f, g=None, beams: BeamSet = None, ws=None) -> BeamSet:
    """Step 1.  f (and g): complex [3][z][y][x] arrays on the mesh's y grid
    (numpy/torch complex, or device float64 already interleaved)."""
    L = lib()
    if beams is None:
        nq = mesh.nq[0] * mesh.nq[1] * mesh.nq[2]
        npm = mesh.np[0] * mesh.np[1] * mesh.np[2]
        nbranch = bin(mesh.branch_mask & 7).count("1")
        beams = BeamSet(nq * npm * nbranch * (1 if mesh.one_way else 2))
    fd = _complex_dev(f)
    gd = _complex_dev(g) if g is not None else None
    ws = _workspace(L.fga_decompose_workspace_bytes(C.byref(mesh), 1 if g is not None else 0), ws)
    _check(L.fga_decompose(C.byref(medium.c), C.byref(mesh), _ptr(fd), _ptr(gd), C.byref(beams.c),
                           _ptr(ws), ws.numel(), _stream()))
    return beams


def point_source(eps, x0, M, nq, qhalf=None, ndir=64, nshell=4, shell_lo=0.2, shell_hi=2.5, ricker=True,
                 rho0=0.0, branch_mask=7, cull_abs=0.0, merge_s=False) -> PointSourceC:
    """Point moment-tensor source parameters (M = xx, yy, zz, xy, xz, yz)."""
    s = PointSourceC()
    s.eps = eps
    s.x0[:] = [float(v) for v in x0]
    s.M[:] = [float(v) for v in M]
    s.rho0 = rho0
    s.nq = nq
    s.qhalf = 4.0 * eps ** 0.5 if qhalf is None else qhalf
    s.ndir, s.nshell = ndir, nshell
    s.shell_lo, s.shell_hi = shell_lo, shell_hi
    s.ricker = 1 if ricker else 0
    s.branch_mask = branch_mask
    s.cull_abs = cull_abs
    s.merge_s = 1 if merge_s else 0
    return s


def fga_decompose_point_source(medium: Medium, src: PointSourceC, beams: BeamSet = None, ws=None) -> BeamSet:
    """Step 1 for a point moment-tensor source (closed-form weights)."""
    L = lib()
    if beams is None:
        beams = BeamSet(int(L.fga_point_source_candidates(C.byref(src))))
    ws = _workspace(L.fga_decompose_point_source_workspace_bytes(C.byref(src)), ws)
    _check(L.fga_decompose_point_source(C.byref(medium.c), C.byref(src), C.byref(beams.c), _ptr(ws), ws.numel(),
                                        _stream()))
    return beams


def point_force(eps, x0, d, nq, qhalf, ndir, nshell, omega, t0, width, t_ref, shell_lo=0.2, shell_hi=2.5,
                rho0=0.0, branch_mask=7, cull_abs=0.0, merge_s=False) -> PointForceC:
    """Point force d F(t), F(t) = cos(omega (t + t0)) exp(-(t + t0)^2/width^2); beams launched at t_ref."""
    s = PointForceC()
    s.eps = eps
    s.x0[:] = [float(v) for v in x0]
    s.d[:] = [float(v) for v in d]
    s.rho0 = rho0
    s.nq, s.qhalf, s.ndir, s.nshell = nq, qhalf, ndir, nshell
    s.shell_lo, s.shell_hi = shell_lo, shell_hi
    s.omega, s.t0, s.width, s.t_ref = omega, t0, width, t_ref
    s.branch_mask = branch_mask
    s.cull_abs = cull_abs
    s.merge_s = 1 if merge_s else 0
    return s


def fga_decompose_point_force(medium: Medium, src: PointForceC, beams: BeamSet = None, ws=None) -> BeamSet:
    """Step 1 for a point force with its time function (closed-form weights)."""
    L = lib()
    if beams is None:
        beams = BeamSet(int(L.fga_point_force_candidates(C.byref(src))))
    ws = _workspace(L.fga_decompose_point_force_workspace_bytes(C.byref(src)), ws)
    _check(L.fga_decompose_point_force(C.byref(medium.c), C.byref(src), C.byref(beams.c), _ptr(ws), ws.numel(),
                                       _stream()))
    return beams


def fga_evolve(medium: Medium, beams: BeamSet, dt: float, nsteps: int, receivers=None, eps: float = None,
               tau: float = 25.0, stride: int = 1, chunk: int = 0, cutoff_abs: float = 0.0, compact: bool = False,
               batch: int = 0, precision: int = FGA_FP64, seis=None, ws=None, resort: int = 0, gen_max: int = 0,
               child_cut: float = 0.0, coords: int = FGA_COORDS_CARTESIAN, s_vector: bool = False):
    """Step 2.  Returns (seis or None, stats dict).  receivers: (n,3) array;
    seis is complex [n][nsteps/stride][3] as a float64 tensor [n, ns, 3, 2].
    resort: steps between spatial reorderings (0 default, < 0 never).
    gen_max, child_cut: interface generation cap and child amplitude cut of
    layered media (0: library defaults 3 and 1e-3; child_cut < 0 keeps all).
    s_vector: frame-free S amplitudes (homogeneous and grid media)."""
    torch = _torch()
    L = lib()
    opts = EvolveOptsC(chunk, cutoff_abs, 1 if compact else 0, batch, resort, gen_max, child_cut,
                       1 if s_vector else 0)
    rec = None
    xyz = None
    if receivers is not None:
        xyz = _dev(receivers, torch.float64)
        rec = ReceiversC(xyz.shape[0], xyz.data_ptr(), stride, eps, tau, precision, coords)
        ns = nsteps // stride
        if seis is None:
            seis = torch.empty((xyz.shape[0], ns, 3, 2), dtype=torch.float64, device="cuda")
    ws = _workspace(L.fga_evolve_workspace_bytes(C.byref(beams.c), nsteps, C.byref(opts),
                                                 C.byref(rec) if rec is not None else None), ws)
    stats = EvolveStatsC()
    _check(L.fga_evolve(C.byref(medium.c), C.byref(beams.c), dt, nsteps, C.byref(opts),
                        C.byref(rec) if rec is not None else None, _ptr(seis), _ptr(ws), ws.numel(), _stream(),
                        C.byref(stats)))
    return seis, {"beam_steps": stats.beam_steps, "evals": stats.evals, "culled": stats.culled,
                  "quarantined": stats.quarantined, "crossings": stats.crossings, "spawned": stats.spawned,
                  "capped": stats.capped}


def fga_reconstruct_points(beams: BeamSet, eps: float, tau: float, xyz, precision: int = FGA_FP64, out=None,
                           ws=None):
    """Step 3 at points.  Returns (float64 tensor [n,3,2], evals)."""
    torch = _torch()
    L = lib()
    x = _dev(xyz, torch.float64)
    n = x.shape[0]
    if out is None:
        out = torch.empty((n, 3, 2), dtype=torch.float64, device="cuda")
    ws = _workspace(L.fga_reconstruct_points_workspace_bytes(C.byref(beams.c), n), ws)
    ev = C.c_int64(0)
    _check(L.fga_reconstruct_points(C.byref(beams.c), eps, tau, n, _ptr(x), precision, _ptr(out), _ptr(ws),
                                    ws.numel(), _stream(), C.byref(ev)))
    return out, ev.value


def fga_reconstruct_points_noalloc(beams: BeamSet, eps: float, tau: float, xyz, out,
                                   precision: int = FGA_FP64, want_evals: bool = True):
    """Step 3 at points without any allocation in the call: xyz (device
    float64 [n,3]) and out (device float64 [n,3,2]) are caller tensors; the
    library's fixed per-device scratch holds everything else.  Returns
    (out, evals or None)."""
    L = lib()
    n = int(xyz.shape[0])
    ev = C.c_int64(0)
    _check(L.fga_reconstruct_points_noalloc(C.byref(beams.c), eps, tau, n, _ptr(xyz), precision, _ptr(out),
                                            _stream(), C.byref(ev) if want_evals else None))
    return out, (ev.value if want_evals else None)


def fga_reconstruct_grid(beams: BeamSet, eps: float, tau: float, mesh, precision: int = FGA_FP64, out=None,
                         ws=None, add: bool = False):
    """Step 3 on the grid mesh.lo + i*mesh.h.  Returns (float64 tensor
    [3, nz, ny, nx, 2], evals).  add: sum into `out` (fga_reconstruct_grid_add)."""
    torch = _torch()
    L = lib()
    n = (C.c_int * 3)(*[int(v) for v in mesh.n])
    lo = (C.c_double * 3)(*[float(v) for v in mesh.lo])
    h = (C.c_double * 3)(*[float(v) for v in mesh.h])
    if out is None:
        out = torch.empty((3, n[2], n[1], n[0], 2), dtype=torch.float64, device="cuda")
    ws = _workspace(L.fga_reconstruct_grid_workspace_bytes(C.byref(beams.c), n, eps, tau, h), ws)
    ev = C.c_int64(0)
    if add and out is None:
        raise ValueError("add=True needs the partial sum in out")
    fn = L.fga_reconstruct_grid_add if add else L.fga_reconstruct_grid
    _check(fn(C.byref(beams.c), eps, tau, n, lo, h, precision, _ptr(out), _ptr(ws), ws.numel(), _stream(),
              C.byref(ev)))
    return out, ev.value


def workspace_bytes(kind: str, **kw) -> int:
    """Workspace size of one call, for callers that preallocate."""
    L = lib()
    if kind == "decompose":
        return L.fga_decompose_workspace_bytes(C.byref(kw["mesh"]), 1 if kw.get("with_g") else 0)
    if kind == "evolve":
        opts = EvolveOptsC(kw.get("chunk", 0), kw.get("cutoff_abs", 0.0), 1 if kw.get("compact") else 0,
                           kw.get("batch", 0), kw.get("resort", 0), kw.get("gen_max", 0), kw.get("child_cut", 0.0))
        rec = None
        if kw.get("n_receivers"):
            rec = ReceiversC(kw["n_receivers"], 0, kw.get("stride", 1), kw["eps"], kw.get("tau", 25.0),
                             kw.get("precision", FGA_FP64), kw.get("coords", FGA_COORDS_CARTESIAN))
        return L.fga_evolve_workspace_bytes(C.byref(kw["beams"].c), kw["nsteps"], C.byref(opts),
                                            C.byref(rec) if rec is not None else None)
    if kind == "grid":
        mesh = kw["mesh"]
        n = (C.c_int * 3)(*[int(v) for v in mesh.n])
        h = (C.c_double * 3)(*[float(v) for v in mesh.h])
        return L.fga_reconstruct_grid_workspace_bytes(C.byref(kw["beams"].c), n, kw["eps"], kw["tau"], h)
    raise ValueError(kind)


def fga_profile_enable(on: bool = True) -> None:
    _check(lib().fga_profile_enable(1 if on else 0))


def fga_profile_read(kernel: int, reset: bool = False):
    """(launches, total milliseconds) of one kernel since profiling was enabled."""
    n = C.c_int64(0)
    ms = C.c_double(0.0)
    _check(lib().fga_profile_read(kernel, C.byref(n), C.byref(ms), 1 if reset else 0))
    return n.value, ms.value


def to_complex(t) -> np.ndarray:
    """float64 tensor with a trailing (re, im) axis -> complex numpy array."""
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

def make_request(medium: Medium, mesh, f, receivers, tau: float, dt: float, nsteps: int, stride: int = 1,
                 precision: int = FGA_FP64, source: "PointSourceC" = None, coords: int = FGA_COORDS_CARTESIAN):
    """A forward-solve request: host initial data f (complex [3, nz, ny, nx])
    and receivers (n, 3).  Returns (RequestC, seismogram array it fills:
    complex [n, nsteps // stride, 3]); both must stay alive until completion."""
    f = np.ascontiguousarray(np.asarray(f if f is not None else np.zeros(1), dtype=np.complex128))
    x = np.ascontiguousarray(np.asarray(receivers, dtype=np.float64).reshape(-1, 3))
    seis = np.zeros((x.shape[0], nsteps // stride, 3), dtype=np.complex128)
    r = RequestC()
    r.medium = medium.c
    if mesh is not None:
        r.mesh = mesh
    r.f = f.ctypes.data
    r.n_receivers = x.shape[0]
    r.receivers = x.ctypes.data
    r.tau, r.dt, r.nsteps, r.stride = tau, dt, nsteps, stride
    r.seis_out = seis.ctypes.data
    r.precision = precision
    r.receiver_coords = coords
    if source is not None:
        r.point_source = 1
        r.source = source
    return r, seis, (f, x, medium)


class Server:
    """fga_server: admits queued forward solves by device footprint into at
    most max_active concurrent slots, each on its own stream."""

    def __init__(self, hbm_budget: int, max_active: int):
        _torch()
        self._s = C.c_void_p()
        _check(lib().fga_server_create(int(hbm_budget), int(max_active), C.byref(self._s)))
        self._keep = {}

    @staticmethod
    def footprint(req: RequestC) -> int:
        return int(lib().fga_server_footprint(C.byref(req)))

    def submit(self, req: RequestC, keep=()) -> int:
        i = C.c_uint64(0)
        _check(lib().fga_server_submit(self._s, C.byref(req), C.byref(i)))
        self._keep[i.value] = (req, keep)
        return i.value

    def poll(self, max_n: int = 64, wait_ms: int = 0):
        out = (CompletionC * max_n)()
        n = C.c_int(0)
        _check(lib().fga_server_poll(self._s, out, max_n, C.byref(n), int(wait_ms)))
        res = []
        for k in range(n.value):
            c = out[k]
            self._keep.pop(c.id, None)
            res.append({"id": c.id, "status": c.status, "t_submit": c.t_submit, "t_start": c.t_start,
                        "t_done": c.t_done, "footprint": c.footprint, "beams": c.beams,
                        "beam_steps": c.beam_steps, "evals": c.evals})
        return res

    def status(self):
        q, r, pk = C.c_int(0), C.c_int(0), C.c_int(0)
        h = C.c_size_t(0)
        _check(lib().fga_server_status(self._s, C.byref(q), C.byref(r), C.byref(h), C.byref(pk)))
        return {"queued": q.value, "running": r.value, "held": h.value, "peak_running": pk.value}

    def close(self):
        if self._s:
            _check(lib().fga_server_destroy(self._s))
            self._s = C.c_void_p()
