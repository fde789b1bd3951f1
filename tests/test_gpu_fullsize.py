"""Parity at the workloads' full sizes.  Smooth random medium (the benchmark), eps = 1/128,
q 32^3 x p 8^3 x 3 branches (49 M beams after the cull), 1000 FP64 RK4
steps with 256 receivers sampled after every step, 128^3 grid at T = 1, run
in the launch configuration the benchmark times (the evolution as 4 calls of
250 steps sharing one workspace).

Outputs the oracle can compute one by one are compared with it: every beam
of 200 seeded (q, p) pairs, decomposed and evolved 1000 steps by the oracle,
against the GPU beam of the same lineage (the GPU set is re-sorted in space
during the run).  Sums over all 49 M beams are beyond the oracle; for them
the test checks properties that hold at any size: the MFMA grid tiles and
the ALU point sums (independent kernels) agree at 512 seeded grid points,
and the last seismogram sample, summed from the records the integrator
emits, equals a point sum at the receivers over the final beams.  The
homogeneous packet, the mixed-precision 256^3 grid and the layered Earth
have tests of their own below."""
import sys

import numpy as np
import pytest

import fga_inputs as fi
import oracle as om
from test_gpu_parity import alive_by_lineage, by_lineage, compare_states, oracle_to_dict, phys_amp_gpu, rel_l2

pytestmark = pytest.mark.gpu

RTOL = 1e-10
SEGMENTS = 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("merge", [False, True])
def test_smooth_medium_full_size(merge):
    """merge: SH and SV as one S beam per (q, p), as the benchmark runs them;
    the sampled oracle beams are then merged by the oracle's own merge."""
    import torch
    import paper_1810_06760_amd as m
    m.lib()
    say("full size: smooth medium, 32^3 x 8^3 x 3, 1000 steps, 256 receivers, 128^3 grid, merged", merge)
    w = fi.smooth_medium_packet()
    med = m.medium_for(w)
    mesh = m.mesh_for(w, merge_s=merge)
    beams = m.BeamSet(w.qmesh.count * w.pmesh.count * 3)
    m.fga_decompose(med, mesh, m._complex_dev(w.f), beams=beams)
    n0 = beams.count
    say("  decomposed", n0)
    assert n0 > (3.0e7 if merge else 4.5e7)
    seg = w.nsteps // SEGMENTS
    nrec = len(w.receivers)
    ws = m._workspace(m.workspace_bytes("evolve", beams=beams, nsteps=seg, n_receivers=nrec, eps=w.eps, tau=w.tau))
    seis = torch.empty((nrec, w.nsteps, 3, 2), dtype=torch.float64, device="cuda")
    steps = 0
    for s0 in range(0, w.nsteps, seg):
        part, st = m.fga_evolve(med, beams, w.dt, seg, receivers=w.receivers, eps=w.eps, tau=w.tau, ws=ws)
        seis[:, s0:s0 + seg].copy_(part)
        steps += st["beam_steps"]
        say("  steps", s0 + seg)
    assert beams.count == n0 and steps == n0 * w.nsteps
    grid, evg = m.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid)
    torch.cuda.synchronize()
    say("  grid done, evals", evg)

    # sampled beams: oracle decompose + 1000 steps
    g = np.random.default_rng(4243)
    pick = g.choice(w.qmesh.count * w.pmesh.count, size=200, replace=False)
    iq, ip = pick % w.qmesh.count, pick // w.qmesh.count
    ob = om.decompose(w, iq=iq, ip=ip)
    if merge:
        ob = om.merge_s_beams(ob, w.qmesh.count * w.pmesh.count)
    om.evolve(om.medium_for(w), ob, w.dt, w.nsteps)
    say("  oracle beams", len(ob))
    lin = torch.from_numpy(ob["lineage"].astype(np.int64)).cuda()
    idx = torch.isin(beams.lineage[:beams.count], lin).nonzero().squeeze(1)
    assert idx.numel() == len(ob)
    compare_states(beams.export(idx), ob)

    # MFMA grid tiles against ALU point sums at sampled grid points
    n = w.out_grid.n[0]
    sel = g.choice(w.out_grid.count, size=512, replace=False)
    pts = w.out_grid.points()[sel]
    up, _ = m.fga_reconstruct_points(beams, w.eps, w.tau, pts)
    G = m.to_complex(grid)                      # [3][z][y][x]
    zi, yi, xi = sel // (n * n), (sel // n) % n, sel % n
    ug = G[:, zi, yi, xi].T
    err = rel_l2(ug, m.to_complex(up))
    say("  grid vs points", err)
    assert err <= RTOL

    # last seismogram sample against a point sum at the receivers
    ur, _ = m.fga_reconstruct_points(beams, w.eps, w.tau, w.receivers)
    err = rel_l2(m.to_complex(seis[:, -1]), m.to_complex(ur))
    say("  seismogram vs points", err)
    assert err <= RTOL


@pytest.mark.timeout(600)
def test_homogeneous_full_size():
    """The homogeneous packet at its full size (eps = 1/32, q 8^3 x p 4^3 x 3
    branches = 98,304 beams, 100 steps to T = 0.5, 32^3 grid), evolved in 4
    calls of 25 steps: every beam against the oracle, and the grid at 2048
    seeded points against the oracle's direct sum over all beams."""
    import torch
    import paper_1810_06760_amd as m
    m.lib()
    say("full size: homogeneous packet, 8^3 x 4^3 x 3, 100 steps, 32^3 grid")
    w = fi.homogeneous_packet()
    med = m.medium_for(w)
    beams = m.fga_decompose(med, m.mesh_for(w), m._complex_dev(w.f))
    seg = w.nsteps // SEGMENTS
    ws = m._workspace(m.workspace_bytes("evolve", beams=beams, nsteps=seg))
    for s0 in range(0, w.nsteps, seg):
        m.fga_evolve(med, beams, w.dt, seg, ws=ws)
    grid, _ = m.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid)
    torch.cuda.synchronize()
    ob = om.decompose(w)
    om.evolve(om.medium_for(w), ob, w.dt, w.nsteps)
    say("  beams", beams.count, len(ob))
    compare_states(beams.export(), ob)
    n = w.out_grid.n[0]
    sel = np.random.default_rng(4244).choice(w.out_grid.count, size=2048, replace=False)
    uo, _ = om.sum_points(ob, w.out_grid.points()[sel], w.eps, w.tau)
    G = m.to_complex(grid)
    ug = G[:, sel // (n * n), (sel // n) % n, sel % n].T
    err = rel_l2(ug, uo)
    say("  grid vs oracle", err)
    assert err <= RTOL


@pytest.mark.timeout(600)
def test_mixed_grid_256():
    """The mixed-precision workload's 256^3 grid (eps = 1/512, tau = 16) over
    one wave of its packet (q 16^3 x p 8^3 x 3 branches, 250 FP64 steps in the
    smooth random medium), so that every tile's candidate list is thousands of
    beams long and its work is split into several items.  The FP64 tiles
    agree with point sums at 512 seeded grid points to 1e-10; every mixed
    variant is within 1e-3 of the FP64 tiles over the whole grid (relative
    L2), and all report the same in-window count."""
    import torch
    import paper_1810_06760_amd as m
    m.lib()
    say("mixed grid: eps 1/512, q 16^3 x p 8^3 x 3, 250 steps, 256^3 grid")
    w, slabs = fi.mixed_waves(nq=16, waves=1)
    med = m.medium_for(w)
    mesh = m.make_mesh(w.eps, slabs[0], w.pmesh, w.ymesh, cull_abs=w.cull_abs)
    beams = m.fga_decompose(med, mesh, m._complex_dev(w.f))
    m.fga_evolve(med, beams, w.dt, w.nsteps)
    say("  beams", beams.count)
    ref, ev = m.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid)
    torch.cuda.synchronize()
    say("  fp64 tiles, evals", ev)
    n = w.out_grid.n[0]
    sel = np.random.default_rng(4245).choice(w.out_grid.count, size=512, replace=False)
    up, _ = m.fga_reconstruct_points(beams, w.eps, w.tau, w.out_grid.points()[sel])
    zi, yi, xi = sel // (n * n), (sel // n) % n, sel % n
    err = rel_l2(m.to_complex(ref)[:, zi, yi, xi].T, m.to_complex(up))
    say("  fp64 tiles vs points", err)
    assert err <= RTOL
    nref = float(torch.linalg.vector_norm(ref))
    for prec in ("FGA_FP32", "FGA_BF16X3", "FGA_FP16X3", "FGA_FP16X2"):
        u, evm = m.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid, precision=getattr(m, prec))
        e = float(torch.linalg.vector_norm(u - ref)) / nref
        say("  %s vs fp64 tiles: %.3g" % (prec, e))
        assert evm == ev
        assert e <= 1e-3
        del u


@pytest.mark.timeout(900)
def test_mixed_grid_256_against_oracle():
    """The mixed-precision workload at its own sizes (eps = 1/512, q 50^3 x
    p 8^3 x 3 branches, second of its four z-slab waves, 250 FP64 RK4 steps
    in the smooth random medium, 256^3 grid with tau = 16) on a seeded subset
    the oracle can decompose and evolve: 2,000 (q, p) pairs of the wave,
    decomposed by the oracle's own quadrature on the 256^3 y mesh.  The GPU
    takes the beams of the same lineages from its decomposition of the whole
    wave, evolves them and sums them on the full 256^3 grid with every
    variant; at 2,000 seeded grid points the FP64 tiles equal the oracle's
    direct sum to 1e-10 and every mixed variant is within 1e-3 of it."""
    import torch
    import paper_1810_06760_amd as m
    m.lib()
    say("mixed grid vs oracle: eps 1/512, q 50^3 x p 8^3 x 3, wave 2 of 4, 2000-pair subset")
    w, slabs = fi.mixed_waves(nq=50, waves=4)
    qm = slabs[1]
    med = m.medium_for(w)
    mesh = m.make_mesh(w.eps, qm, w.pmesh, w.ymesh, cull_abs=w.cull_abs)
    full = m.fga_decompose(med, mesh, m._complex_dev(w.f))
    say("  wave beams", full.count)
    g = np.random.default_rng(4401)
    pick = g.choice(qm.count * w.pmesh.count, size=2000, replace=False)
    iq, ip = pick % qm.count, pick // qm.count
    Ft = om.fbi(w.f, w.ymesh, qm.points()[iq], w.pmesh.points()[ip], w.eps)
    ob = om.make_beams(qm, w.pmesh, Ft, w.eps, iq, ip, one_way=True, cull_abs=w.cull_abs)
    # the GPU beams of the subset's lineages (kept by the GPU's own cull)
    lin_gpu = full.lineage[:full.count].cpu().numpy()
    base = (ip * qm.count + iq).astype(np.int64)
    want = np.sort(np.concatenate([base + b * 2 * w.pmesh.count * qm.count for b in range(3)]))
    slots = np.searchsorted(lin_gpu, want)
    slots = slots[(slots < len(lin_gpu)) & (lin_gpu[np.minimum(slots, len(lin_gpu) - 1)] == want)]
    sub = full.export(torch.from_numpy(slots).to("cuda"))
    del full
    torch.cuda.empty_cache()
    assert np.array_equal(sub["lineage"], ob["lineage"]), (len(sub["lineage"]), len(ob))
    beams = m.BeamSet(len(ob))
    beams.load(sub)
    m.fga_evolve(med, beams, w.dt, w.nsteps, resort=-1)
    om.evolve(om.medium_for(w), ob, w.dt, w.nsteps)
    say("  subset beams", len(ob))
    n = w.out_grid.n[0]
    sel = np.random.default_rng(4402).choice(w.out_grid.count, size=2000, replace=False)
    ref, _ = om.sum_points(ob, w.out_grid.points()[sel], w.eps, w.tau)
    zi, yi, xi = (torch.from_numpy(v).to("cuda") for v in (sel // (n * n), (sel // n) % n, sel % n))
    for prec, tol in (("FGA_FP64", RTOL), ("FGA_FP32", 1e-3), ("FGA_BF16X3", 1e-3), ("FGA_FP16X3", 1e-3),
                      ("FGA_FP16X2", 1e-3)):
        u, _ = m.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid, precision=getattr(m, prec))
        got = m.to_complex(u[:, zi, yi, xi])
        e = rel_l2(got.T, ref)
        say("  %s vs oracle at 2000 grid points: %.3g" % (prec, e))
        assert e <= tol
        del u


@pytest.mark.timeout(900)
def test_layered_earth_full_size():
    """The layered Earth workload at its full size: a point moment-tensor
    source at eps = 1/256 (q 8^3 x 1600 directions x 4 shells x 3 branches x
    2 directions = 19,660,800 beams) in the 4-shell model with interface
    splitting (generation cap 3) and 512 surface receivers sampled after
    every step, for 400 of its 2000 steps in calls of 100 steps as the
    benchmark runs them (the set grows past 10^8 beams).  The oracle
    decomposes the full source and evolves the beams of 48 seeded initial
    lineages with all their descendants; the GPU beams of the same lineages
    match them (lineage, generation, layer, branch and sigma exactly; states
    and amplitudes to 1e-10).  The last seismogram sample equals a point sum
    at the receivers over the final beams; the stations are given to the
    library in spherical coordinates and to the point sum as the oracle maps
    them."""
    import torch
    import paper_1810_06760_amd as m
    m.lib()
    e = fi.layered_earth()
    nsteps, seg = 400, 100
    say("full size: layered Earth, %d of %d steps" % (nsteps, e["nsteps"]))
    med_g = m.Medium.layered(1, e["bounds"], e["cp"], e["cs"], e["rho"])
    kw = dict(nq=e["nq"], ndir=e["ndir"], nshell=e["nshell"])
    src = m.point_source(e["eps"], e["x0"], e["M"], **kw)
    ncand = int(m.lib().fga_point_source_candidates(m.C.byref(src)))
    beams = m.BeamSet(12 * ncand)
    m.fga_decompose_point_source(med_g, src, beams=beams)
    n0 = beams.count
    say("  decomposed", n0)
    rec = m._dev(e["receivers_rtp"], torch.float64)        # stations as (r, longitude, latitude)
    nrec = rec.shape[0]
    ws = m._workspace(m.workspace_bytes("evolve", beams=beams, nsteps=seg, n_receivers=nrec, eps=e["eps"],
                                        tau=e["tau"], coords=m.FGA_COORDS_SPHERICAL))
    seis = torch.empty((nrec, nsteps, 3, 2), dtype=torch.float64, device="cuda")
    for s0 in range(0, nsteps, seg):
        part, _ = m.fga_evolve(med_g, beams, e["dt"], seg, receivers=rec, eps=e["eps"], tau=e["tau"], ws=ws,
                               coords=m.FGA_COORDS_SPHERICAL)
        seis[:, s0:s0 + seg].copy_(part)
        say("  steps", s0 + seg, "beams", beams.count)
    torch.cuda.synchronize()

    med_o = om.layered(1, e["bounds"], e["cp"], e["cs"], e["rho"])
    ob_all = om.point_source_beams(med_o, om.point_source(e["eps"], e["x0"], e["M"], **kw))
    assert len(ob_all) == n0
    pick = np.sort(np.random.default_rng(4246).choice(len(ob_all), size=48, replace=False))
    ob = ob_all[pick].copy()
    del ob_all
    out, _ = om.evolve_layered(med_o, ob, e["dt"], nsteps, gmax=3, child_cut=1e-3)
    ref = alive_by_lineage(oracle_to_dict(out))
    ref = {k: v[np.argsort(ref["lineage"], kind="stable")] for k, v in ref.items()}
    say("  oracle beams", len(out), "alive", len(ref["lineage"]), "max generation", int(out["gen"].max()))
    assert int(out["gen"].max()) >= 2, "the sample should include interface children"
    lin = torch.from_numpy(ref["lineage"].astype(np.int64)).cuda()
    idx = torch.isin(beams.lineage[:beams.count], lin).nonzero().squeeze(1)
    g = by_lineage(alive_by_lineage(beams.export(idx)))
    assert np.array_equal(g["lineage"], ref["lineage"])
    for k in ("gen", "layer", "branch", "sigma"):
        assert np.array_equal(g[k], ref[k]), k
    for k in ("Q", "P", "ZQ", "ZP"):
        assert rel_l2(g[k], ref[k]) <= RTOL, k
    keep = out["alive"] == 1
    A_ref = om.amplitude_vectors(out[keep][np.argsort(out["lineage"][keep], kind="stable")])
    assert rel_l2(phys_amp_gpu(g), A_ref) <= RTOL

    ur, _ = m.fga_reconstruct_points(beams, e["eps"], e["tau"], om.spherical_to_cartesian(e["receivers_rtp"]))
    err = rel_l2(m.to_complex(seis[:, -1]), m.to_complex(ur))
    say("  seismogram vs points", err)
    assert err <= RTOL
