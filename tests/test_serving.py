"""The request server: continuous admission by device footprint, overlap of
admitted solves, and results that do not depend on what runs beside them."""
import sys

import numpy as np
import pytest

import fga_inputs as fi


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fga():
    import paper_1810_06760_amd as m
    m.lib()
    return m


def build_requests(m):
    """Six requests over two resident models (homogeneous, smooth grid),
    with different meshes, receiver counts, step counts and strides."""
    reqs = []
    rng = np.random.default_rng(77)
    grid_w = fi.smooth_medium_packet(nq=4, np_=2, ny=16, nmed=16, nout=0, nrec=4)
    grid_med = m.medium_for(grid_w)
    homog_w = fi.homogeneous_packet(nq=4, np_=2, ny=16, nout=0)
    homog_med = m.medium_for(homog_w)
    specs = [("h", 4, 2, 5, 24, 2), ("g", 4, 2, 7, 30, 3), ("h", 5, 2, 9, 20, 1),
             ("g", 3, 2, 3, 40, 4), ("h", 4, 3, 6, 16, 2), ("g", 5, 2, 8, 24, 2)]
    for kind, nq, np_, nrec, nsteps, stride in specs:
        if kind == "h":
            w = fi.homogeneous_packet(nq=nq, np_=np_, ny=16, nout=0)
            med = homog_med
        else:
            w = fi.smooth_medium_packet(nq=nq, np_=np_, ny=16, nmed=16, nout=0, nrec=4)
            med = grid_med
        x = fi.uniform_points(nrec, rng, 0.2, 0.8)
        dt = 0.005 if kind == "h" else 2e-3
        reqs.append((med, m.mesh_for(w), w.f, x, 25.0, dt, nsteps, stride))
    return reqs, (grid_med, homog_med)


def point_source_requests(m, meds):
    """Two point-source requests (sweep generator, shrunk meshes)."""
    out = []
    for i in range(2):
        rq = fi.sweep_request(i, nsteps=20)
        src = m.point_source(1.0 / 32, rq["x0"], rq["M"], nq=4, ndir=24, nshell=2)
        out.append(dict(medium=meds[i], receivers=rq["receivers"][:9], tau=25.0, dt=2e-3, nsteps=20, stride=2,
                        source=src))
    return out


def run_server(m, reqs, budget, slots):
    srv = m.Server(budget, slots)
    seis = {}
    try:
        for i, (med, mesh, f, x, tau, dt, nsteps, stride) in enumerate(reqs):
            r, s, keep = m.make_request(med, mesh, f, x, tau, dt, nsteps, stride)
            rid = srv.submit(r, keep=(keep, s))
            seis[rid] = (i, s)
        done = []
        while len(done) < len(reqs):
            got = srv.poll(16, wait_ms=20000)
            assert got, "server made no progress"
            done += got
        st = srv.status()
    finally:
        srv.close()
    out = [None] * len(reqs)
    for c in done:
        assert c["status"] == 0, c
        i, s = seis[c["id"]]
        out[i] = s
    return out, done, st


@pytest.mark.gpu
def test_results_alone_equal_results_in_mix():
    m = fga()
    say("serving alone vs mix")
    reqs, keep = build_requests(m)
    fps = [m.Server.footprint(m.make_request(*r)[0]) for r in reqs]
    alone = []
    for r in reqs:
        out, _, _ = run_server(m, [r], max(fps), 1)
        alone.append(out[0])
    budget = sum(sorted(fps)[-3:])
    mix, done, st = run_server(m, reqs, budget, 3)
    assert st["peak_running"] >= 2
    assert st["held"] == 0 and st["queued"] == 0
    for a, b in zip(alone, mix):
        assert np.array_equal(a, b)
    # solves started while others were still running (continuous admission)
    done.sort(key=lambda c: c["t_start"])
    overlap = sum(1 for k in range(1, len(done)) if done[k]["t_start"] < max(c["t_done"] for c in done[:k]))
    assert overlap >= 1


@pytest.mark.gpu
def test_server_matches_direct_calls():
    """A served solve equals decompose + evolve called directly."""
    m = fga()
    say("serving vs direct")
    reqs, keep = build_requests(m)
    med, mesh, f, x, tau, dt, nsteps, stride = reqs[1]
    out, _, _ = run_server(m, [reqs[1]], 1 << 34, 1)
    bs = m.fga_decompose(med, mesh, f)
    seis, _ = m.fga_evolve(med, bs, dt, nsteps, receivers=x, eps=mesh.eps, tau=tau, stride=stride)
    direct = m.to_complex(seis)
    assert np.array_equal(out[0], direct)


@pytest.mark.gpu
def test_mixed_precision_requests():
    """Served solves in mixed mode stay within 1e-3 of the FP64 ones."""
    m = fga()
    say("serving mixed")
    reqs, keep = build_requests(m)
    srv = m.Server(1 << 34, 2)
    outs = {}
    try:
        for i, r in enumerate(reqs[:3]):
            for prec in (m.FGA_FP64, m.FGA_FP32):
                rq, s, k = m.make_request(*r, precision=prec)
                outs[srv.submit(rq, keep=(k, s))] = (i, prec, s)
        got = []
        while len(got) < 6:
            got += srv.poll(8, wait_ms=20000)
    finally:
        srv.close()
    assert all(c["status"] == 0 for c in got)
    res = {(i, p): s for i, p, s in outs.values()}
    for i in range(3):
        a, b = res[(i, m.FGA_FP32)], res[(i, m.FGA_FP64)]
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b)


@pytest.mark.gpu
def test_point_source_requests_match_direct_calls():
    m = fga()
    say("serving point sources")
    reqs, meds = build_requests(m)
    srv = m.Server(1 << 34, 2)
    outs = {}
    try:
        for k, r in enumerate(point_source_requests(m, meds)):
            rq, s, keep = m.make_request(r["medium"], None, None, r["receivers"], r["tau"], r["dt"], r["nsteps"],
                                         r["stride"], source=r["source"])
            outs[srv.submit(rq, keep=(keep, s, r))] = (k, s, r)
        got = []
        while len(got) < 2:
            got += srv.poll(4, wait_ms=20000)
    finally:
        srv.close()
    assert all(c["status"] == 0 for c in got)
    for k, s, r in outs.values():
        bs = m.fga_decompose_point_source(r["medium"], r["source"])
        seis, _ = m.fga_evolve(r["medium"], bs, r["dt"], r["nsteps"], receivers=r["receivers"], eps=1.0 / 32,
                               tau=r["tau"], stride=r["stride"])
        assert np.array_equal(s, m.to_complex(seis))


@pytest.mark.gpu
def test_budget_limits_concurrency():
    """With a budget that fits one request at a time, solves run one by one
    even with several free slots; a request above the budget is refused."""
    m = fga()
    say("serving budget")
    reqs, keep = build_requests(m)
    trio = [reqs[0], reqs[1], reqs[0]]     # footprints of similar size
    fps = sorted(m.Server.footprint(m.make_request(*r)[0]) for r in trio)
    budget = fps[0] + fps[1] - 1           # no two of them fit together
    assert fps[2] <= budget
    out, done, st = run_server(m, trio, budget, 3)
    assert st["peak_running"] == 1
    srv = m.Server(min(fps) - 1, 2)
    try:
        r, s, k = m.make_request(*reqs[0])
        with pytest.raises(RuntimeError, match="budget"):
            srv.submit(r, keep=(k, s))
    finally:
        srv.close()


def test_footprint_is_a_host_query():
    """fga_server_footprint needs no GPU and grows with the request."""
    m = fga()
    reqs = []
    w = fi.homogeneous_packet(nq=4, np_=2, ny=16, nout=0)
    small = m.make_request(m.medium_for(w), m.mesh_for(w), w.f, np.zeros((4, 3)), 25.0, 0.005, 20, 1)[0]
    more_rec = m.make_request(m.medium_for(w), m.mesh_for(w), w.f, np.zeros((400, 3)), 25.0, 0.005, 20, 1)[0]
    w2 = fi.homogeneous_packet(nq=6, np_=2, ny=16, nout=0)
    more_beams = m.make_request(m.medium_for(w2), m.mesh_for(w2), w2.f, np.zeros((4, 3)), 25.0, 0.005, 20, 1)[0]
    f0, f1, f2 = (m.Server.footprint(r) for r in (small, more_rec, more_beams))
    assert 0 < f0 < f1 and f0 < f2


@pytest.mark.gpu
@pytest.mark.parametrize("precision,merge", [("fp64", False), ("mixed", False), ("mixed32", False), ("fp64", True),
                                             ("mixed32", True)])
def test_served_solve_matches_oracle(precision, merge):
    """A served point-source solve in a smooth grid medium (the sweep's model
    recipe) against the oracle's decompose -> evolve -> sum at the receivers
    (Steps 1-3): relative L2 <= 1e-10 in FP64, <= 1e-3 with the mixed
    receiver sums; a second, larger request served beside it changes nothing.
    merge: the served source makes one S beam per (q, p, direction) (as the
    serving benchmark does); the oracle's separate SH and SV beams give the
    same field."""
    import oracle as om
    m = fga()
    say("served solve vs oracle", precision, "merged" if merge else "")
    nodes = fi.sweep_model(1, nmed=32)
    mesh = fi.node_grid(32)
    med = m.Medium.grid(nodes, mesh, cs_ratio=1.0 / np.sqrt(3.0))
    rq = fi.sweep_request(3, nsteps=30)
    eps, nsteps, dt, stride = 1.0 / 32, 30, 2e-3, 3
    src = m.point_source(eps, rq["x0"], rq["M"], nq=3, ndir=16, nshell=2, merge_s=merge)
    x = rq["receivers"][:10]
    prec = {"fp64": m.FGA_FP64, "mixed": m.FGA_FP32, "mixed32": m.FGA_FP32_ACC32}[precision]
    other = m.point_source(eps, rq["x0"] + 0.05, rq["M"], nq=4, ndir=24, nshell=2, merge_s=merge)
    srv = m.Server(1 << 32, 2)
    try:
        r, seis, keep = m.make_request(med, None, None, x, 25.0, dt, nsteps, stride, precision=prec, source=src)
        r2, seis2, keep2 = m.make_request(med, None, None, rq["receivers"][:40], 25.0, dt, nsteps, 1,
                                          precision=prec, source=other)
        srv.submit(r2, keep=(keep2, seis2))
        srv.submit(r, keep=(keep, seis))
        got = []
        while len(got) < 2:
            got += srv.poll(4, wait_ms=20000)
    finally:
        srv.close()
    assert all(c["status"] == 0 for c in got)
    med_o = om.grid(nodes, mesh, cs_ratio=1.0 / np.sqrt(3.0))
    src_o = om.point_source(eps, rq["x0"], rq["M"], nq=3, ndir=16, nshell=2)
    ob = om.point_source_beams(med_o, src_o)
    ref = np.zeros((len(x), nsteps // stride, 3), dtype=np.complex128)
    for s in range(nsteps // stride):
        om.evolve(med_o, ob, dt, stride)
        ref[:, s, :], _ = om.sum_points(ob, x, eps, 25.0)
    err = np.linalg.norm(seis - ref) / np.linalg.norm(ref)
    say("  rel-L2 vs oracle %.2e (%d beams)" % (err, len(ob)))
    assert err <= (1e-10 if precision == "fp64" else 1e-3)
