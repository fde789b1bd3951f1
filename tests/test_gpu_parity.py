"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Bar (FP64 path): relative L2 <= 1e-10 for every floating-point output, exact
equality for integer outputs (beam lineage sets, in-window term counts).
"""
import math
import sys

import numpy as np
import pytest

import fga_inputs as fi
import oracle as om

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fga():
    import paper_1810_06760_amd as m
    m.lib()
    return m


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def oracle_to_dict(ob):
    return {"Q": ob["Q"], "P": ob["P"], "ZQ": ob["ZQ"], "ZP": ob["ZP"], "a": ob["a"], "S": ob["S"], "w": ob["w"],
            "e": ob["e"], "branch": ob["branch"], "sigma": ob["sigma"], "layer": ob["layer"], "gen": ob["gen"],
            "flags": ob["alive"], "lineage": ob["lineage"]}


def phys_amp_gpu(d):
    """physical amplitude vectors of exported GPU beams"""
    n = len(d["Q"])
    A = np.zeros((n, 3), dtype=np.complex128)
    for i in range(n):
        P = d["P"][i]
        if d["branch"][i] == 0:
            A[i] = d["a"][i, 0] * P / np.linalg.norm(P)
        else:
            e = d["e"][i]
            nsh = np.cross(e, P); nsh /= np.linalg.norm(nsh)
            nsv = np.cross(P / np.linalg.norm(P), nsh)
            A[i] = d["a"][i, 0] * nsv + d["a"][i, 1] * nsh
    return A


def by_lineage(d):
    """GPU export reordered by lineage (evolve keeps beams in spatial order)."""
    o = np.argsort(d["lineage"], kind="stable")
    return {k: v[o] for k, v in d.items()}


def compare_states(g, ob, tol=RTOL):
    g = by_lineage(g)
    assert np.array_equal(g["lineage"], ob["lineage"])
    for k in ("Q", "P", "ZQ", "ZP", "S"):
        err = rel_l2(g[k], ob[k]) if k != "S" else np.max(np.abs(g[k] - ob[k]))
        assert err <= (tol if k != "S" else 1e-12), (k, err)
    err = rel_l2(phys_amp_gpu(g), om.amplitude_vectors(ob))
    assert err <= tol, ("A", err)


def small_c1(nq=4, np_=2, ny=16):
    return fi.homogeneous_packet(nq=nq, np_=np_, ny=ny, nout=0)


def small_c2(nq=4, np_=2, ny=16, nmed=32):
    return fi.smooth_medium_packet(nq=nq, np_=np_, ny=ny, nmed=nmed, nout=0, nrec=8)


@pytest.mark.parametrize("case", ["homogeneous", "grid"])
def test_evolve_parity(case):
    m = fga()
    w = small_c1() if case == "homogeneous" else small_c2()
    say("evolve parity", case)
    ob = om.decompose(w)
    med_o = om.medium_for(w)
    med_g = m.medium_for(w)
    bs = m.BeamSet(len(ob) + 5)
    bs.load(oracle_to_dict(ob))
    nsteps, dt = (100, 0.005) if case == "homogeneous" else (150, 2e-3)
    m.fga_evolve(med_g, bs, dt, nsteps, chunk=37)
    om.evolve(med_o, ob, dt, nsteps)
    compare_states(bs.export(), ob)


def test_s_frame_switch_parity():
    """S beams whose momentum swings through the frame axis switch frames
    identically on both sides (bump-free check with a steep grid medium)."""
    m = fga()
    say("s frame switch")
    n = 16
    mesh = fi.node_grid(n)
    ax = mesh.axis(0)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    cp = 1.7 * (1.0 + 0.25 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z))
    med_o = om.grid(cp, mesh, cs_ratio=0.6)
    med_g = m.Medium.grid(cp, mesh, cs_ratio=0.6)
    g = np.random.default_rng(11)
    nb = 64
    ob = np.zeros(nb, dtype=om.BEAM_DTYPE)
    ob["Q"] = g.random((nb, 3))
    d = g.standard_normal((nb, 3))
    d[:, 2] += 3.0
    ob["P"] = d / np.linalg.norm(d, axis=1)[:, None] * 1.3
    for i in range(3):
        ob["ZQ"][:, i, i] = 1.0
        ob["ZP"][:, i, i] = -1j
    ob["a"][:, 0] = 2 ** 1.5
    ob["a"][:, 1] = 0.3j
    ob["w"] = 1.0
    ob["e"][:, 0] = 1.0    # x axis, far from P (mostly along z)
    ob["branch"] = 2
    ob["sigma"] = np.where(np.arange(nb) % 2 == 0, 1, -1)
    ob["alive"] = 1
    ob["lineage"] = np.arange(nb)
    om.reframe(ob)
    bs = m.BeamSet(nb)
    bs.load(oracle_to_dict(ob))
    m.fga_evolve(med_g, bs, 4e-3, 200)
    om.evolve(med_o, ob, 4e-3, 200)
    gexp = by_lineage(bs.export())
    assert np.array_equal(gexp["e"], ob["e"])
    compare_states(gexp, ob)


def test_decompose_parity():
    """Step 1 on the full homogeneous packet mesh (8^3 q x 4^3 p x 3 branches)."""
    m = fga()
    say("decompose parity")
    w = fi.homogeneous_packet(ny=32, nout=0)
    ob = om.decompose(w)
    bs = m.fga_decompose(m.medium_for(w), m.mesh_for(w), w.f)
    g = bs.export()
    assert bs.count == len(ob) == 3 * 8 ** 3 * 4 ** 3
    assert np.array_equal(g["lineage"], ob["lineage"])
    assert np.array_equal(g["branch"], ob["branch"])
    assert rel_l2(g["w"], ob["w"]) <= RTOL
    assert np.array_equal(g["Q"], ob["Q"]) and np.array_equal(g["P"], ob["P"])
    assert np.array_equal(g["e"], ob["e"])
    compare_states(g, ob)


def test_decompose_cull_parity():
    """Culling by |psi| makes the same beam set on both sides (beams within
    1e-9 relative of the threshold are not counted either way)."""
    m = fga()
    say("decompose cull parity")
    w = fi.homogeneous_packet(ny=32, nout=0)
    ob_all = om.decompose(w)
    psi_abs = np.abs(ob_all["w"])
    thr = np.quantile(psi_abs, 0.6)
    norm = w.qmesh.cell_volume * w.pmesh.cell_volume * (2 * math.pi * w.eps) ** -4.5
    w.cull_abs = thr / norm
    bs = m.fga_decompose(m.medium_for(w), m.mesh_for(w), w.f)
    g = bs.export()
    keep_o = set(ob_all["lineage"][psi_abs >= thr].tolist())
    amb = set(ob_all["lineage"][np.abs(psi_abs - thr) <= 1e-9 * thr].tolist())
    keep_g = set(g["lineage"].tolist())
    assert keep_o - amb <= keep_g and keep_g - amb <= keep_o
    assert np.all(np.diff(g["lineage"]) > 0)


def two_way_velocity(w):
    """A seeded initial velocity on the work's quadrature mesh: a second
    Gaussian packet (own polarisation, amplitude 2, wave vector (1, 0.5, 0))."""
    d = fi.unit_vector(fi.rng(2, 77))
    return 2.0 * fi.gaussian_plane_wave(w.ymesh, w.eps, (0.45, 0.5, 0.55), 0.12, (1.0, 0.5, 0.0), d)


@pytest.mark.parametrize("case,cull", [("homogeneous", False), ("grid", False), ("grid", True)])
def test_decompose_two_way_parity(case, cull):
    """Step 1 with both directions and u_t(0) = g != 0 (eq:psi, eq:alpha^k):
    psi_{b,+-} = 1/2 FBI[f].n_b +- (i eps/(2|p|)) FBI[g/c_b].n_b, with c_b
    taken from the medium at the quadrature points; with a cull at the median
    |psi| the kept sets agree outside a 1e-9 band around the threshold."""
    m = fga()
    say("decompose two-way parity", case, cull)
    w = small_c1(nq=4, np_=3, ny=16) if case == "homogeneous" else small_c2(nq=4, np_=3, ny=16, nmed=16)
    w.cull_abs = 0.0
    g = two_way_velocity(w)
    ob_all = om.decompose_two_way(w, g)
    n_all, n_cand = len(ob_all), 6 * w.qmesh.count * w.pmesh.count
    assert n_all == n_cand, (n_all, n_cand)
    norm = w.qmesh.cell_volume * w.pmesh.cell_volume * (2 * math.pi * w.eps) ** -4.5
    if cull:
        psi_abs = np.abs(ob_all["w"])
        thr = np.quantile(psi_abs, 0.5)
        w.cull_abs = thr / norm
    bs = m.fga_decompose(m.medium_for(w), m.mesh_for(w, one_way=False), w.f, g=g)
    gexp = bs.export()
    assert np.all(np.diff(gexp["lineage"]) > 0)
    if not cull:
        assert bs.count == len(ob_all)
        assert np.array_equal(gexp["lineage"], ob_all["lineage"])
        assert np.array_equal(gexp["sigma"], ob_all["sigma"])
        assert rel_l2(gexp["w"], ob_all["w"]) <= RTOL
        compare_states(gexp, ob_all)
        return
    keep_o = set(ob_all["lineage"][psi_abs >= thr].tolist())
    amb = set(ob_all["lineage"][np.abs(psi_abs - thr) <= 1e-9 * thr].tolist())
    keep_g = set(gexp["lineage"].tolist())
    assert keep_o - amb <= keep_g and keep_g - amb <= keep_o
    both = np.isin(ob_all["lineage"], gexp["lineage"])
    sel = np.isin(gexp["lineage"], ob_all["lineage"][both])
    assert rel_l2(gexp["w"][sel], ob_all["w"][both]) <= RTOL


def evolved_beams(w, nsteps, dt):
    ob = om.decompose(w)
    om.evolve(om.medium_for(w), ob, dt, nsteps)
    return ob


def test_points_parity():
    m = fga()
    say("points parity")
    w = small_c1(nq=5, np_=3, ny=16)
    ob = evolved_beams(w, 40, 0.005)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    x = fi.uniform_points(300, np.random.default_rng(2), -0.2, 1.2)
    for tau in (25.0, 4.0):
        uo, co = om.sum_points(ob, x, w.eps, tau)
        ug, cg = m.fga_reconstruct_points(bs, w.eps, tau, x)
        assert cg == co
        assert rel_l2(m.to_complex(ug), uo) <= RTOL


@pytest.mark.parametrize("prec", ["FGA_FP32", "FGA_FP32_ACC32"])
def test_points_mixed_precision(prec):
    """Receiver sums in the mixed modes (FP64 arguments, FP32 exp/sin/cos;
    FP64 products and sums, or FP32 products and per-lane sums) against the
    oracle: relative L2 <= 1e-3, exact in-window count."""
    m = fga()
    say("points mixed", prec)
    w = small_c1(nq=5, np_=3, ny=16)
    ob = evolved_beams(w, 40, 0.005)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    x = fi.uniform_points(300, np.random.default_rng(2), -0.2, 1.2)
    uo, co = om.sum_points(ob, x, w.eps, 16.0)
    ug, cg = m.fga_reconstruct_points(bs, w.eps, 16.0, x, precision=getattr(m, prec))
    assert cg == co
    err = rel_l2(m.to_complex(ug), uo)
    say("  rel L2", err)
    assert err <= 1e-3


def test_points_tile_skip():
    """Points spread far beyond the beams with a narrow window: most beam
    tiles lie outside every point group's reach and are skipped whole; the
    sums and in-window counts still match the direct sum exactly."""
    m = fga()
    say("points tile skip")
    w = small_c1(nq=6, np_=3, ny=16)
    ob = evolved_beams(w, 20, 0.005)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    x = fi.uniform_points(500, np.random.default_rng(5), -1.5, 2.5)
    for tau in (1.0, 3.0):
        uo, co = om.sum_points(ob, x, w.eps, tau)
        ug, cg = m.fga_reconstruct_points(bs, w.eps, tau, x)
        assert cg == co and co > 0
        assert rel_l2(m.to_complex(ug), uo) <= RTOL


@pytest.mark.parametrize("npts", [1, 17, 65])
def test_points_ragged_and_dead(npts):
    """Ragged point groups, a ragged last beam tile and dead beams: the
    in-window count is exact and idle lanes never add a term."""
    m = fga()
    say("points ragged", npts)
    w = small_c1(nq=5, np_=3, ny=16)
    ob = evolved_beams(w, 10, 0.005)
    ob = ob[:4096 + 64 * 3 + 7].copy()
    ob["alive"][::7] = 0
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    x = fi.uniform_points(npts, np.random.default_rng(npts), 0.0, 1.0)
    uo, co = om.sum_points(ob, x, w.eps, 25.0)
    ug, cg = m.fga_reconstruct_points(bs, w.eps, 25.0, x)
    assert cg == co
    assert rel_l2(m.to_complex(ug), uo) <= RTOL


@pytest.mark.parametrize("n,tau", [(20, 25.0), (37, 6.0)])
def test_grid_parity(n, tau):
    """Step 3 on a grid with ragged tiles: the tile GEMMs on the matrix cores
    against the oracle's direct windowed sum at every grid point."""
    m = fga()
    say("grid parity", n, tau)
    w = small_c1(nq=5, np_=3, ny=16)
    ob = evolved_beams(w, 30, 0.005)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    grid = fi.cell_centred(n, -0.1, 1.1)
    ug, cg = m.fga_reconstruct_grid(bs, w.eps, tau, grid)
    uo, co = om.sum_points(ob, grid.points(), w.eps, tau)
    assert cg == co
    ug = m.to_complex(ug).reshape(3, -1).T
    assert rel_l2(ug, uo) <= RTOL


@pytest.mark.parametrize("prec", ["FGA_FP32", "FGA_BF16X3", "FGA_FP16X3", "FGA_FP16X2"])
def test_grid_mixed_precision(prec):
    """Mixed-precision tile GEMMs (FP32 factors from FP64-reduced arguments,
    FP32 accumulation; hi+lo split operands for BF16/FP16) against the
    oracle's FP64 direct sum: relative L2 <= 1e-3, exact in-window count."""
    m = fga()
    say("grid mixed", prec)
    w = small_c1(nq=5, np_=3, ny=16)
    ob = evolved_beams(w, 30, 0.005)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    grid = fi.cell_centred(37, -0.1, 1.1)
    tau = 16.0
    ug, cg = m.fga_reconstruct_grid(bs, w.eps, tau, grid, precision=getattr(m, prec))
    uo, co = om.sum_points(ob, grid.points(), w.eps, tau)
    assert cg == co
    err = rel_l2(m.to_complex(ug).reshape(3, -1).T, uo)
    say("  rel L2", err)
    assert err <= 1e-3
    if prec in ("FGA_FP32", "FGA_BF16X3"):
        assert err <= 1e-4   # FP32 factors and 16-bit hi+lo splits carry ~1e-5


@pytest.mark.parametrize("prec", ["FGA_FP64", "FGA_BF16X3", "FGA_FP16X2"])
def test_grid_add_in_waves(prec):
    """A beam set summed in three waves (fga_reconstruct_grid then
    fga_reconstruct_grid_add twice) against the oracle's direct sum over all
    beams; the in-window counts of the waves add up to the oracle's."""
    m = fga()
    say("grid in waves", prec)
    w = small_c1(nq=5, np_=3, ny=16)
    ob = evolved_beams(w, 30, 0.005)
    grid = fi.cell_centred(37, -0.1, 1.1)
    tau = 16.0
    cuts = [0, len(ob) // 3, 2 * len(ob) // 3 + 5, len(ob)]
    ug, ctot = None, 0
    for k in range(3):
        part = ob[cuts[k]:cuts[k + 1]]
        bs = m.BeamSet(len(part))
        bs.load(oracle_to_dict(part))
        ug, c = m.fga_reconstruct_grid(bs, w.eps, tau, grid, precision=getattr(m, prec), out=ug, add=k > 0)
        ctot += c
    uo, co = om.sum_points(ob, grid.points(), w.eps, tau)
    assert ctot == co
    err = rel_l2(m.to_complex(ug).reshape(3, -1).T, uo)
    say("  rel L2", err)
    assert err <= {"FGA_FP64": RTOL, "FGA_BF16X3": 1e-4}.get(prec, 1e-3)


def test_seismogram_parity():
    """Receivers sampled after every step during the evolution."""
    m = fga()
    say("seismogram parity")
    w = small_c2(nq=4, np_=2, ny=16)
    ob = om.decompose(w)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    rec = w.receivers
    nsteps, dt, tau = 24, 2e-3, 25.0
    seis, st = m.fga_evolve(m.medium_for(w), bs, dt, nsteps, receivers=rec, eps=w.eps, tau=tau, stride=2, chunk=5,
                            batch=97)
    med_o = om.medium_for(w)
    ref = np.zeros((len(rec), nsteps // 2, 3), dtype=np.complex128)
    cnt = 0
    for s in range(nsteps // 2):
        om.evolve(med_o, ob, dt, 2)
        u, c = om.sum_points(ob, rec, w.eps, tau)
        ref[:, s, :] = u
        cnt += c
    assert st["evals"] == cnt
    assert st["beam_steps"] == nsteps * len(ob)
    assert rel_l2(m.to_complex(seis), ref) <= RTOL


def amp_measure(ob):
    """|w| max(|a0|, |a1|) of oracle beams (the cutoff's measure)."""
    return np.abs(ob["w"]) * np.max(np.abs(ob["a"]), axis=1)


@pytest.mark.parametrize("compact", [False, True])
def test_evolve_cutoff_parity(compact):
    """Culling after every step (the benchmark spec: beams whose amplitude falls below
    the cutoff are dropped): the oracle steps all beams one step at a time,
    drops those with |w| max|a| < cutoff after each step and sums the rest at
    the receivers; the GPU (chunks of 7 steps, receivers every step) must
    drop the same lineages (no decision within 1e-9 of the threshold), count
    them, keep the survivors' states and give the same seismograms."""
    m = fga()
    say("evolve cutoff parity, compact", compact)
    w = small_c2(nq=4, np_=3, ny=16)
    ob = om.decompose(w)
    n0 = len(ob)
    cut = float(np.quantile(amp_measure(ob), 0.35))
    bs = m.BeamSet(n0)
    bs.load(oracle_to_dict(ob))
    rec = w.receivers
    nsteps, dt = 60, 2e-3
    seis, st = m.fga_evolve(m.medium_for(w), bs, dt, nsteps, receivers=rec, eps=w.eps, tau=w.tau, chunk=7,
                            cutoff_abs=cut, compact=compact, resort=-1)
    med_o = om.medium_for(w)
    ref = np.zeros((len(rec), nsteps, 3), dtype=np.complex128)
    closest = np.inf
    steps = 0
    for s in range(nsteps):
        live = ob["alive"] == 1
        steps += int(live.sum())
        om.evolve(med_o, ob, dt, 1)
        meas = amp_measure(ob)
        closest = min(closest, float(np.min(np.abs(meas[live] / cut - 1.0))))
        ob["alive"][live & (meas < cut)] = 0
        ref[:, s, :], _ = om.sum_points(ob, rec, w.eps, w.tau)
    assert closest > 1e-9, closest                       # no decision at the threshold
    kept = ob["alive"] == 1
    say("  %d beams, %d culled by the oracle, %d by the GPU" % (n0, n0 - kept.sum(), st["culled"]))
    assert 0 < st["culled"] == n0 - int(kept.sum())
    assert st["beam_steps"] == steps
    g = bs.export()
    if compact:
        assert bs.count == int(kept.sum())
        assert np.all(g["flags"] == m.FGA_FLAG_ALIVE)
    else:
        assert bs.count == n0
        assert np.array_equal(g["flags"] == m.FGA_FLAG_ALIVE, kept)
        g = {k: v[g["flags"] == m.FGA_FLAG_ALIVE] for k, v in g.items()}
    compare_states(g, om.take_beams(ob, np.nonzero(kept)[0]))
    assert rel_l2(m.to_complex(seis), ref) <= RTOL


@pytest.mark.parametrize("case", ["homogeneous", "grid"])
def test_quarantine_non_finite_beam(case):
    """A beam loaded with a NaN in dzQ (its amplitude turns non-finite in the
    first step) is quarantined and counted, takes no further step, and no
    seismogram sample takes a NaN from it; every other beam and the
    seismograms equal the oracle's without that beam."""
    m = fga()
    say("quarantine", case)
    w = small_c1(nq=4, np_=2) if case == "homogeneous" else small_c2(nq=4, np_=2, ny=16)
    ob = om.decompose(w)
    bad = len(ob) // 3
    d = oracle_to_dict(ob)
    d["ZQ"] = d["ZQ"].copy()
    d["ZQ"][bad, 1, 1] = np.nan
    bs = m.BeamSet(len(ob))
    bs.load(d)
    rec = fi.uniform_points(12, fi.rng(1, 55)) if w.receivers is None else w.receivers
    nsteps, dt = 20, 2e-3
    seis, st = m.fga_evolve(m.medium_for(w), bs, dt, nsteps, receivers=rec, eps=w.eps, tau=w.tau, chunk=6,
                            resort=-1)
    assert st["quarantined"] == 1 and st["culled"] == 0
    g = bs.export()
    assert g["flags"][bad] == m.FGA_FLAG_QUARANTINED
    others = np.arange(len(ob)) != bad
    assert np.all(g["flags"][others] == m.FGA_FLAG_ALIVE)
    assert st["beam_steps"] == nsteps * (len(ob) - 1) + 1
    ob["alive"][bad] = 0
    med_o = om.medium_for(w)
    ref = np.zeros((len(rec), nsteps, 3), dtype=np.complex128)
    for s in range(nsteps):
        om.evolve(med_o, ob, dt, 1)
        ref[:, s, :], _ = om.sum_points(ob, rec, w.eps, w.tau)
    out = m.to_complex(seis)
    assert np.all(np.isfinite(out))
    assert rel_l2(out, ref) <= RTOL
    compare_states({k: v[others] for k, v in g.items()}, om.take_beams(ob, np.nonzero(others)[0]))


@pytest.mark.parametrize("prec", ["FGA_FP32", "FGA_FP32_ACC32"])
def test_seismogram_mixed_precision(prec):
    m = fga()
    say("seismogram mixed", prec)
    w = small_c2(nq=4, np_=2, ny=16)
    ob = om.decompose(w)
    bs = m.BeamSet(len(ob))
    bs.load(oracle_to_dict(ob))
    rec = w.receivers
    nsteps, dt, tau = 24, 2e-3, 16.0
    seis, st = m.fga_evolve(m.medium_for(w), bs, dt, nsteps, receivers=rec, eps=w.eps, tau=tau, stride=3,
                            precision=getattr(m, prec))
    med_o = om.medium_for(w)
    ref = np.zeros((len(rec), nsteps // 3, 3), dtype=np.complex128)
    for s in range(nsteps // 3):
        om.evolve(med_o, ob, dt, 3)
        ref[:, s, :] = om.sum_points(ob, rec, w.eps, tau)[0]
    assert rel_l2(m.to_complex(seis), ref) <= 1e-3


def test_empty_beam_set():
    m = fga()
    say("empty beams")
    bs = m.BeamSet(4)
    x = np.array([[0.5, 0.5, 0.5]])
    u, c = m.fga_reconstruct_points(bs, 1 / 32, 25.0, x)
    assert c == 0 and np.all(m.to_complex(u) == 0)
    g, c = m.fga_reconstruct_grid(bs, 1 / 32, 25.0, fi.cell_centred(5, 0, 1))
    assert c == 0 and np.all(m.to_complex(g) == 0)
    seis, st = m.fga_evolve(m.Medium.homogeneous(1.7, 1.0), bs, 0.01, 3, receivers=x, eps=1 / 32)
    assert np.all(m.to_complex(seis) == 0) and st["beam_steps"] == 0


# ---------------------------------------------------------------------------
# layered media: interface splitting (Sec. 3.1)
# ---------------------------------------------------------------------------

LAYERED = {
    "flat": (0, [0.42, 0.58], [1.7, 2.2, 1.9], [1.0, 1.3, 1.1], [1.0, 1.35, 1.2], None),
    "sphere": (1, [0.95, 0.8], [1.7, 2.1, 2.4], [1.0, 1.2, 1.4], [1.0, 1.25, 1.5], None),
    # linear speeds per layer (c = c_l (1 + g_l v), v = z or |x|): curved rays
    "flat_grad": (0, [0.42, 0.58], [1.7, 2.2, 1.9], [1.0, 1.3, 1.1], [1.0, 1.35, 1.2], [0.5, -0.4, 0.3]),
    "sphere_grad": (1, [0.95, 0.8], [1.7, 2.1, 2.4], [1.0, 1.2, 1.4], [1.0, 1.25, 1.5], [-0.3, 0.35, 0.0]),
    # a traction-free surface closing the outermost region
    "flat_free": (0, [0.42, 0.58], [1.7, 2.2, 1.9], [1.0, 1.3, 1.1], [1.0, 1.35, 1.2], None),
    "sphere_free": (1, [0.95, 0.8], [1.7, 2.1, 2.4], [1.0, 1.2, 1.4], [1.0, 1.25, 1.5], [-0.3, 0.35, 0.0]),
    # a Gaussian low-velocity region in the middle layer (the crosswell model's form, eq:true_c)
    "flat_anom": (0, [0.42, 0.58], [1.7, 2.2, 1.9], [1.0, 1.3, 1.1], [1.0, 1.35, 1.2], None),
    "sphere_anom": (1, [0.95, 0.8], [1.7, 2.1, 2.4], [1.0, 1.2, 1.4], [1.0, 1.25, 1.5], None),
}
SURFACE = {"flat_free": 0.72, "sphere_free": 1.12}
ANOMALY = {"flat_anom": {1: (0.2, 40.0, (0.5, 0.0, 0.5), (1.0, 0.0, 1.0))},
           "sphere_anom": {0: (0.15, 30.0, (0.5, 0.5, 0.7), (1.0, 1.0, 1.0))}}


def initial_layers(ob, geometry, bounds):
    """Layer index of each beam centre (interfaces: flat z = b_i, layer i
    below; spheres |x| = b_i, layer i outside)."""
    if geometry == 0:
        v = ob["Q"][:, 2]
        return np.array([sum(1 for b in bounds if z > b) for z in v], dtype=np.int32)
    r = np.linalg.norm(ob["Q"], axis=1)
    return np.array([sum(1 for b in bounds if x < b) for x in r], dtype=np.int32)


def layered_case(name, nq=4, np_=2):
    geo, bounds, cp, cs, rho, grad = LAYERED[name]
    w = small_c1(nq=nq, np_=np_, ny=16)
    ob = om.decompose(w)
    ob["layer"] = initial_layers(ob, geo, bounds)
    sf = SURFACE.get(name, 0.0)
    if sf > 0.0:
        # the beams start inside the free surface (the medium ends there)
        lev = ob["Q"][:, 2] if geo == 0 else np.linalg.norm(ob["Q"], axis=1)
        ob = om.take_beams(ob, np.nonzero(lev < sf)[0])
    an = ANOMALY.get(name)
    return (w, ob, om.layered(geo, bounds, cp, cs, rho, grad=grad, surface=sf, anomaly=an),
            fga().Medium.layered(geo, bounds, cp, cs, rho, grad=grad, surface=sf, anomaly=an))


def alive_by_lineage(d):
    keep = (d["flags"] & 1) == 1 if "flags" in d else d["alive"] == 1
    return {k: v[keep] for k, v in d.items()}


@pytest.mark.parametrize("name", ["flat", "sphere", "flat_grad", "sphere_grad", "flat_free", "sphere_free",
                                  "flat_anom", "sphere_anom"])
def test_interface_parity(name):
    """Beams crossing flat or spherical interfaces, between constant or
    linear-gradient layers, or reflected at a traction-free surface, split
    into the same children (lineage, generation, layer, branch) with the
    same states."""
    m = fga()
    say("interface parity", name)
    w, ob, med_o, med_g = layered_case(name)
    nsteps, dt = 60, 0.005
    out, ncap = om.evolve_layered(med_o, ob, dt, nsteps, gmax=3, child_cut=1e-3)
    ref = alive_by_lineage(oracle_to_dict(out))
    ref = {k: v[np.argsort(ref["lineage"], kind="stable")] for k, v in ref.items()}
    assert (ref["gen"] > 0).sum() > 50, "test geometry should produce children"
    bs = m.BeamSet(len(out) + 256)
    bs.load(oracle_to_dict(ob))
    _, st = m.fga_evolve(med_g, bs, dt, nsteps)
    g = alive_by_lineage(bs.export())
    g = by_lineage(g)
    assert np.array_equal(g["lineage"], ref["lineage"])
    for k in ("gen", "layer", "branch", "sigma"):
        assert np.array_equal(g[k], ref[k]), k
    assert st["capped"] == ncap
    assert st["spawned"] == int((out["gen"] > 0).sum())
    for k in ("Q", "P", "ZQ", "ZP"):
        assert rel_l2(g[k], ref[k]) <= RTOL, k
    keep = out["alive"] == 1
    A_ref = om.amplitude_vectors(out[keep][np.argsort(out["lineage"][keep], kind="stable")])
    assert rel_l2(phys_amp_gpu(g), A_ref) <= RTOL


@pytest.mark.parametrize("name,batch", [("flat", 0), ("flat", 100), ("sphere_grad", 0), ("sphere_free", 0),
                                        ("flat_anom", 0)])
def test_interface_seismogram_parity(name, batch):
    """Receiver sums during a layered run, children included; batch 100 splits
    each step's sum over several ragged beam batches (a layered run sums
    (chunk + stride - 1) / stride + 1 = 7 times the batch at once here)."""
    m = fga()
    say("interface seismograms, %s, batch %d" % (name, batch))
    w, ob, med_o, med_g = layered_case(name)
    rec = fi.uniform_points(9, np.random.default_rng(9), 0.2, 0.8)
    nsteps, dt, tau, stride = 30, 0.005, 25.0, 3
    bs = m.BeamSet(8 * len(ob))
    bs.load(oracle_to_dict(ob))
    seis, st = m.fga_evolve(med_g, bs, dt, nsteps, receivers=rec, eps=w.eps, tau=tau, stride=stride, batch=batch)
    say("beams %d -> %d" % (len(ob), bs.count))
    ref = np.zeros((len(rec), nsteps // stride, 3), dtype=np.complex128)
    cnt = 0
    cur = ob.copy()
    for s in range(nsteps // stride):
        cur, _ = om.evolve_layered(med_o, cur, dt, stride, gmax=3, child_cut=1e-3)
        cur = cur[cur["alive"] == 1].copy()
        u, c = om.sum_points(cur, rec, w.eps, tau)
        ref[:, s, :] = u
        cnt += c
    assert st["spawned"] > 0
    assert st["evals"] == cnt
    assert rel_l2(m.to_complex(seis), ref) <= RTOL


def test_spherical_receivers_parity():
    """Stations given as (r, longitude, latitude) (opening of Sec. 3) are
    mapped by the library; a layered run in the spherical-shell model samples
    them as the oracle does at its own mapping of the same coordinates."""
    m = fga()
    say("spherical receivers")
    w, ob, med_o, med_g = layered_case("sphere")
    g = np.random.default_rng(19)
    rtp = np.stack([g.uniform(0.75, 0.95, 11), g.uniform(0.6, 1.0, 11), g.uniform(0.45, 0.8, 11)], axis=1)
    nsteps, dt, tau, stride = 24, 0.005, 25.0, 2
    bs = m.BeamSet(4 * len(ob))
    bs.load(oracle_to_dict(ob))
    seis, st = m.fga_evolve(med_g, bs, dt, nsteps, receivers=rtp, eps=w.eps, tau=tau, stride=stride,
                            coords=m.FGA_COORDS_SPHERICAL)
    x = om.spherical_to_cartesian(rtp)
    ref = np.zeros((len(rtp), nsteps // stride, 3), dtype=np.complex128)
    cnt = 0
    cur = ob.copy()
    for s in range(nsteps // stride):
        cur, _ = om.evolve_layered(med_o, cur, dt, stride, gmax=3, child_cut=1e-3)
        cur = cur[cur["alive"] == 1].copy()
        ref[:, s, :], c = om.sum_points(cur, x, w.eps, tau)
        cnt += c
    assert st["evals"] == cnt > 0
    assert rel_l2(m.to_complex(seis), ref) <= RTOL


def test_interface_capacity_error():
    """Children that do not fit the beam capacity stop the call with
    FGA_ECAPACITY instead of being dropped."""
    m = fga()
    say("interface capacity")
    w, ob, med_o, med_g = layered_case("flat")
    bs = m.BeamSet(len(ob) + 3)
    bs.load(oracle_to_dict(ob))
    with pytest.raises(RuntimeError, match="capacity"):
        m.fga_evolve(med_g, bs, 0.005, 60)


# ---------------------------------------------------------------------------
# point moment-tensor source
# ---------------------------------------------------------------------------

SRC_M = [1.0, 0.5, -0.3, 0.2, 0.1, -0.4]


@pytest.mark.parametrize("medium", ["homogeneous", "grid", "layered"])
def test_point_source_parity(medium):
    """Closed-form point-source beams: same lineage set after the cull, same
    states and weights (Ricker-weighted, both directions, 3 branches)."""
    m = fga()
    say("point source", medium)
    eps = 1.0 / 32
    if medium == "homogeneous":
        mo, mg = om.homogeneous(math.sqrt(3), 1.0, 1.2), m.Medium.homogeneous(math.sqrt(3), 1.0)
        x0, rho0 = [0.5, 0.45, 0.55], 1.2
    elif medium == "grid":
        w = small_c2(nmed=16)
        mo, mg = om.medium_for(w), m.medium_for(w)
        x0, rho0 = [0.43, 0.52, 0.61], 1.0
    else:
        geo, bounds, cp, cs, rho, grad = LAYERED["sphere"]
        mo, mg = om.layered(geo, bounds, cp, cs, rho), m.Medium.layered(geo, bounds, cp, cs, rho)
        x0, rho0 = [0.3, 0.4, 0.75], 0.0
    kw = dict(nq=5, ndir=40, nshell=3, ricker=True, rho0=rho0)
    ob = om.point_source_beams(mo, om.point_source(eps, x0, SRC_M, **kw))
    bs = m.fga_decompose_point_source(mg, m.point_source(eps, x0, SRC_M, **kw))
    g = bs.export()
    assert np.array_equal(g["lineage"], ob["lineage"])
    for k in ("branch", "sigma", "layer"):
        assert np.array_equal(g[k], ob[k]), k
    assert rel_l2(g["Q"], ob["Q"]) <= 1e-14
    assert rel_l2(g["P"], ob["P"]) <= 1e-14
    assert rel_l2(g["w"], ob["w"]) <= RTOL
    assert np.array_equal(g["e"], ob["e"])


@pytest.mark.parametrize("medium", ["homogeneous", "grid"])
def test_point_force_parity(medium):
    """Point force with its time function (Sec. 2.3 eq:ex_homo, Duhamel
    weights in closed form): the same lineage set, states and weights as the
    oracle; evolved with receivers, the same seismograms."""
    m = fga()
    say("point force", medium)
    eps = 1.0 / 64
    if medium == "homogeneous":
        mo, mg = om.homogeneous(math.sqrt(3), 1.0, 1.0), m.Medium.homogeneous(math.sqrt(3), 1.0)
        x0 = [0.5, 0.5, 0.5]
    else:
        w = small_c2(nmed=16)
        mo, mg = om.medium_for(w), m.medium_for(w)
        x0 = [0.43, 0.52, 0.61]
    kw = dict(nq=5, qhalf=0.3, ndir=24, nshell=3, omega=64.0, t0=0.01, width=0.05, t_ref=-0.01, shell_lo=0.3,
              shell_hi=1.7)
    d = [1.0, 1.0, 1.0]
    ob = om.point_force_beams(mo, om.point_force(eps, x0, d, **kw))
    bs = m.fga_decompose_point_force(mg, m.point_force(eps, x0, d, **kw))
    g = bs.export()
    assert np.array_equal(g["lineage"], ob["lineage"])
    for k in ("branch", "sigma", "layer"):
        assert np.array_equal(g[k], ob[k]), k
    assert rel_l2(g["Q"], ob["Q"]) <= 1e-14
    assert rel_l2(g["w"], ob["w"]) <= RTOL
    rec = fi.uniform_points(7, fi.rng(1, 66), 0.3, 0.7)
    nsteps, dt, stride = 24, 2e-3, 4
    seis, _ = m.fga_evolve(mg, bs, dt, nsteps, receivers=rec, eps=eps, tau=25.0, stride=stride)
    ref = np.zeros((len(rec), nsteps // stride, 3), dtype=np.complex128)
    for k in range(nsteps // stride):
        om.evolve(mo, ob, dt, stride)
        ref[:, k, :], _ = om.sum_points(ob, rec, eps, 25.0)
    assert rel_l2(m.to_complex(seis), ref) <= RTOL


def source_psi_abs(b, eps, nq, qhalf, ndir, nshell, cP, cS, lo=0.2, hi=2.5):
    """|psi| of point-source beams in a homogeneous medium: |w| / (dq dp (2 pi eps)^{-9/2})."""
    dq = (2 * qhalf / nq) ** 3
    Nq, Np = nq ** 3, ndir * nshell
    out = np.empty(len(b))
    for k, (lin, br) in enumerate(zip(b["lineage"], b["branch"])):
        cb = cP if br == 0 else cS
        xs, ws = om.gauss_legendre(nshell, lo * cP / cb, hi * cP / cb)
        sh = ((lin // Nq) % Np) // ndir
        dp = xs[sh] ** 2 * ws[sh] * 4 * math.pi / ndir
        out[k] = abs(b["w"][k]) / (dq * dp * (2 * math.pi * eps) ** -4.5)
    return out


def test_point_source_cull_and_evolve():
    """With a cull threshold on |psi| the kept sets agree (outside a 1e-9
    band), and the source's beams evolve and sum at receivers like the
    oracle's."""
    m = fga()
    say("point source cull + seismograms")
    eps = 1.0 / 32
    mo, mg = om.homogeneous(math.sqrt(3), 1.0, 1.0), m.Medium.homogeneous(math.sqrt(3), 1.0)
    x0 = [0.5, 0.5, 0.5]
    kw = dict(nq=4, ndir=24, nshell=3, qhalf=4 * eps ** 0.5)
    full = om.point_source_beams(mo, om.point_source(eps, x0, SRC_M, **kw))
    psi = source_psi_abs(full, eps, 4, kw["qhalf"], 24, 3, math.sqrt(3), 1.0)
    thr = float(np.quantile(psi, 0.5))
    ob = om.point_source_beams(mo, om.point_source(eps, x0, SRC_M, cull_abs=thr, **kw))
    bs = m.fga_decompose_point_source(mg, m.point_source(eps, x0, SRC_M, cull_abs=thr, **kw))
    g = bs.export()
    amb = set(full["lineage"][np.abs(psi - thr) <= 1e-9 * thr].tolist())
    so, sg = set(ob["lineage"].tolist()), set(g["lineage"].tolist())
    assert so - amb <= sg and sg - amb <= so
    assert 0.3 * len(full) < len(so) < 0.7 * len(full)
    ob = ob[np.isin(ob["lineage"], g["lineage"])]
    rec = fi.uniform_points(6, np.random.default_rng(3), 0.3, 0.7)
    nsteps, dt, tau = 20, 0.005, 25.0
    seis, st = m.fga_evolve(mg, bs, dt, nsteps, receivers=rec, eps=eps, tau=tau, stride=5)
    ref = np.zeros((len(rec), nsteps // 5, 3), dtype=np.complex128)
    cur = ob.copy()
    for s in range(nsteps // 5):
        om.evolve(mo, cur, dt, 5)
        ref[:, s, :] = om.sum_points(cur, rec, eps, tau)[0]
    assert rel_l2(m.to_complex(seis), ref) <= RTOL
