#!/usr/bin/env python
"""Benchmark of the FGA hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input:
  decompose (FBI weights of the initial packet on the 32^3 q x 8^3 p mesh,
  3 branches) -> evolve (1,000 FP64 RK4 steps of every beam in the smooth
  random medium, with 3-component seismograms at 256 receivers after every
  step) -> reconstruct (wavefield at T = 1 on the 128^3 grid, FP64 tile GEMMs
  on the matrix cores).
Inputs (medium table, initial data, receivers) are resident in HBM before the
timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload smooth|homogeneous] [--scale S]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 operations per unit of algorithmic work, counted in the gfx950 code (FMA = 2):
#   one RK4 beam-step (4 right-hand sides + the update), per medium kind,
#   one receiver/point term (window test excluded), one grid term.
FLOP_BEAM_STEP = {"homogeneous": 1647, "grid": 4186, "layered": 1647}  # grad c = 0: the step of rk4_step_pc
FLOP_POINT_EVAL = 79      # FP64 flops per in-window receiver term (window test, exponent, phase, table
                          # exp and sincos, 12 accumulating FMAs), FMA = 2, counted in the gfx950 code
FLOP_GRID_EVAL = 24       # 3 complex multiply-adds
PEAK_FP64 = 78.6e12       # FP64 vector and FP64 matrix peak, MI355X
# grid summation variants: (library code, dense MFMA peak of the operand type)
GRID_PREC = {"fp64": (0, 78.6e12), "fp32": (1, 157.3e12), "bf16x3": (2, 2.5e15), "fp16x3": (3, 2.5e15),
             "fp16x2": (4, 2.5e15)}
HBM_PEAK = 8.0e12
# HBM bytes per launch of a kernel on the default workload (smooth, scale 1), from rocprofv3
# FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB copy calibration; valid only while the kernel's
# source is unchanged (sha256 prefix), else reported as null
TRAFFIC = {"sum_points": {"source": "paper_1810_06760_amd/csrc/k_points.hip", "sha256": "59bdb0187dd2497e",
                          "bytes_per_launch": 2.0397e+10}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="smooth", choices=["smooth", "homogeneous", "layered", "mixed"])
    ap.add_argument("--waves", type=int, default=4, help="beam waves of the mixed-precision workload")
    ap.add_argument("--batch", type=int, default=0, help="beams per receiver-sum batch in the evolution (0: library default)")
    ap.add_argument("--chunk", type=int, default=0, help="RK4 steps per integrator launch (0: library default)")
    ap.add_argument("--resort", type=int, default=0,
                    help="steps between spatial re-sorts of the beams in the evolution (0: library default, <0 never)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="fraction of the q mesh per axis and of the time steps (quick runs only)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--segments", type=int, default=4, help="evolution calls per step (progress between them)")
    ap.add_argument("--cpu-beams", type=int, default=48, help="(q,p) pairs in the oracle sample")
    ap.add_argument("--serve", action="store_true",
                    help="serving run instead: a seeded sweep of forward-solve requests over 4 resident models, "
                         "saturated and at Poisson arrivals; prints solves/s with p50/p99 latency")
    ap.add_argument("--requests", type=int, default=48, help="requests per serving phase")
    ap.add_argument("--slots", type=int, default=4, help="concurrent request slots of the server")
    ap.add_argument("--hbm-budget-gb", type=float, default=240.0, help="server device-memory budget")
    ap.add_argument("--load", type=float, default=0.8, help="Poisson arrival rate as a fraction of saturated")
    ap.add_argument("--serve-precision", default="fp64", choices=["fp64", "mixed"],
                    help="receiver sums of the served solves (mixed: FP32 exp/sin/cos of FP64-reduced arguments; "
                         "the run then also reports its error against FP64 solves of the first 8 requests)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (the known-size kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--grid-precision", default="fp64", choices=list(GRID_PREC),
                    help="grid summation variant (mixed variants also report their error against FP64)")
    return ap.parse_args()


def make_workload(name: str, scale: float):
    import fga_inputs as fi
    if name == "smooth":
        nq = max(2, int(round(32 * scale)))
        nsteps = max(4, int(round(1000 * scale)))
        w = fi.smooth_medium_packet(nq=nq, nsteps=nsteps, dt=1.0 / nsteps)
        label = "smooth random medium cp=sqrt3(1+0.2g), eps=1/128, q %d^3 x p 8^3 x 3 branches, " \
                "%d RK4 steps to T=1, 256 receivers x %d samples, 128^3 grid at T=1, FP64" % (nq, nsteps, nsteps)
    else:
        w = fi.homogeneous_packet()
        label = "homogeneous cp=sqrt3 cs=1, eps=1/32, q 8^3 x p 4^3 x 3 branches, 100 RK4 steps to T=0.5, " \
                "32^3 grid, FP64"
    return w, label


def gpu_run(w, args):
    import torch
    import paper_1810_06760_amd as fga

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    med = fga.medium_for(w)
    mesh = fga.mesh_for(w)
    f = fga._complex_dev(w.f)
    rec = fga._dev(w.receivers, torch.float64) if w.receivers is not None else None
    nq = w.qmesh.count * w.pmesh.count * 3
    beams = fga.BeamSet(nq)
    ws_dec = fga._workspace(fga.workspace_bytes("decompose", mesh=mesh))
    state = {"ws_ev": None, "ws_grid": None, "seis": None, "grid": None}

    nseg = max(1, min(args.segments, w.nsteps))
    seg = -(-w.nsteps // nseg)

    def step():
        fga.fga_decompose(med, mesh, f, beams=beams, ws=ws_dec)
        if state["ws_ev"] is None:
            state["ws_ev"] = fga._workspace(fga.workspace_bytes(
                "evolve", beams=beams, nsteps=seg, n_receivers=0 if rec is None else rec.shape[0],
                eps=w.eps, tau=w.tau, batch=args.batch, chunk=args.chunk))
            if rec is not None:
                state["seis"] = torch.empty((rec.shape[0], w.nsteps, 3, 2), dtype=torch.float64, device=dev)
        # the evolution in a few calls of `seg` steps (progress lines between)
        st = {"beam_steps": 0, "evals": 0}
        for s0 in range(0, w.nsteps, seg):
            n = min(seg, w.nsteps - s0)
            part, st_k = fga.fga_evolve(med, beams, w.dt, n, receivers=rec, eps=w.eps, tau=w.tau,
                                        ws=state["ws_ev"], batch=args.batch, resort=args.resort, chunk=args.chunk)
            if rec is not None:
                state["seis"][:, s0:s0 + n].copy_(part)
            st["beam_steps"] += st_k["beam_steps"]
            st["evals"] += st_k["evals"]
            print("bench: steps %d..%d done" % (s0, s0 + n), file=sys.stderr, flush=True)
        ev_grid = 0
        if w.out_grid is not None:
            if state["ws_grid"] is None:
                state["ws_grid"] = fga._workspace(fga.workspace_bytes("grid", beams=beams, mesh=w.out_grid,
                                                                      eps=w.eps, tau=w.tau))
            state["grid"], ev_grid = fga.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid,
                                                              precision=GRID_PREC[args.grid_precision][0],
                                                              out=state["grid"], ws=state["ws_grid"])
        return beams.count, st, ev_grid

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        print("bench: warmup step %d done in %.1f s" % (i + 1, time.perf_counter() - t), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    fga.fga_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = {"beams": 0, "beam_steps": 0, "ev_rec": 0, "ev_grid": 0}
    for _ in range(args.steps):
        nb, st, evg = step()
        tot["beams"] += nb
        tot["beam_steps"] += st["beam_steps"]
        tot["ev_rec"] += st["evals"]
        tot["ev_grid"] += evg
        print("bench: timed step done, %d beams" % nb, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {fga.KERNEL_NAMES[k]: fga.fga_profile_read(k) for k in fga.KERNEL_NAMES}
    fga.fga_profile_enable(False)
    if args.grid_precision != "fp64" and w.out_grid is not None:
        # error of the mixed variant against the FP64 path (itself at oracle parity), same final beams
        ref, _ = fga.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid, precision=0, ws=state["ws_grid"])
        tot["grid_rel_l2_vs_fp64"] = float(torch.linalg.vector_norm(state["grid"] - ref) /
                                           torch.linalg.vector_norm(ref))
    return t1 - t0, tot, prof


def traffic_for(name, default_workload):
    """Measured HBM bytes per launch, if taken on this workload and this kernel source."""
    import hashlib
    t = TRAFFIC.get(name)
    if t is None or not default_workload:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest()[:16] != t["sha256"]:
            return None
    return t["bytes_per_launch"]


def roofline(tot, prof, medium_kind, grid_peak=PEAK_FP64, default_workload=False):
    """Dominant kernel: algorithmic FLOPs per launch / mean launch time."""
    work = {
        "integrate": tot["beam_steps"] * FLOP_BEAM_STEP[medium_kind],
        "sum_points": tot["ev_rec"] * FLOP_POINT_EVAL,
        "grid_tile": tot["ev_grid"] * FLOP_GRID_EVAL,
    }
    name = max(work, key=lambda k: prof.get(k, (0, 0.0))[1])
    launches, ms = prof[name]
    if launches == 0 or ms <= 0:
        return None, name
    achieved = work[name] / launches / (ms / launches * 1e-3)
    bound = "mfma" if name == "grid_tile" else "alu"
    peak = grid_peak if name == "grid_tile" else PEAK_FP64
    return {"bound": bound, "kernel": name, "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic_for(name, default_workload),
            "launches": launches, "avg_launch_ms": ms / launches}, name


def cpu_baseline(w, tot_per_step, npairs, args):
    """The oracle on a bounded sample of the same workload, scaled to the
    whole step by the per-unit rates of its stages."""
    import oracle as om
    g = np.random.default_rng(4242)
    nqp = w.qmesh.count * w.pmesh.count
    pick = g.choice(nqp, size=min(args.cpu_beams, nqp), replace=False)
    iq, ip = pick % w.qmesh.count, pick // w.qmesh.count
    med = om.medium_for(w)
    t = time.perf_counter()
    F = om.fbi(w.f, w.ymesh, w.qmesh.points()[iq], w.pmesh.points()[ip], w.eps)
    t_fbi = (time.perf_counter() - t) / len(pick)
    beams = om.make_beams(w.qmesh, w.pmesh, F, w.eps, iq, ip, cull_abs=0.0)
    nsteps = min(w.nsteps, 200)
    t_ev = t_rec = 0.0
    n_rec = 0
    for s in range(nsteps):
        t = time.perf_counter()
        om.evolve(med, beams, w.dt, 1)
        t_ev += time.perf_counter() - t
        if w.receivers is not None:
            t = time.perf_counter()
            _, c = om.sum_points(beams, w.receivers, w.eps, w.tau)
            t_rec += time.perf_counter() - t
            n_rec += len(beams) * len(w.receivers)
    rate_step = t_ev / (nsteps * len(beams))
    rate_rec = t_rec / n_rec if n_rec else 0.0
    t_grid = 0.0
    if w.out_grid is not None:
        pts = w.out_grid.points()
        sel = g.choice(len(pts), size=min(4096, len(pts)), replace=False)
        t = time.perf_counter()
        om.sum_points(beams, pts[sel], w.eps, w.tau)
        t_grid = (time.perf_counter() - t) / (len(sel) * len(beams))
    # whole-step CPU time: FBI per (q,p) pair, per beam-step, per (beam, receiver, sample)
    # pair tested, per (beam, grid point) pair tested
    full = (t_fbi * npairs + rate_step * tot_per_step["beam_steps"]
            + rate_rec * tot_per_step["beams"] * (len(w.receivers) if w.receivers is not None else 0) * w.nsteps
            + t_grid * tot_per_step["beams"] * (w.out_grid.count if w.out_grid is not None else 0))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": tot_per_step["beam_steps"] / full, "unit": "beam-steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d random (q,p) pairs (%d beams): FBI, %d RK4 steps with 256-receiver sums per step, "
                      "4096 random grid points; stage rates scaled to the full step (FBI per pair, per "
                      "beam-step, per beam-receiver pair, per beam-grid point pair)"
                      % (len(pick), len(beams), nsteps),
            "seconds_per_step_extrapolated": full}


def layered(args):
    """Layered spherical Earth-like model (4 shells) with a point moment-tensor
    source (Ricker, eps = 1/256): decompose, then 2000 RK4 steps with
    interface splitting (generation cap 3) and 512 surface receivers sampled
    every step.  --scale shrinks the direction count and the step count."""
    import torch
    import fga_inputs as fi
    import paper_1810_06760_amd as fga
    torch.cuda.set_device(0)
    sc = args.scale
    e = fi.layered_earth(ndir=max(16, int(round(1600 * sc))), nsteps=max(8, int(round(2000 * sc))))
    med = fga.Medium.layered(1, e["bounds"], e["cp"], e["cs"], e["rho"])
    src = fga.point_source(e["eps"], e["x0"], e["M"], nq=e["nq"], ndir=e["ndir"], nshell=e["nshell"])
    ncand = int(fga.lib().fga_point_source_candidates(fga.C.byref(src)))
    beams = fga.BeamSet(12 * ncand)   # room for interface children (generation cap 3)
    rec = fga._dev(e["receivers"], torch.float64)
    nseg = max(1, min(args.segments, e["nsteps"]))
    seg = -(-e["nsteps"] // nseg)
    state = {"ws": None, "seis": torch.empty((rec.shape[0], e["nsteps"], 3, 2), dtype=torch.float64, device="cuda")}

    def step():
        fga.fga_decompose_point_source(med, src, beams=beams)
        n0 = beams.count
        if state["ws"] is None:
            state["ws"] = fga._workspace(fga.workspace_bytes("evolve", beams=beams, nsteps=seg,
                                                             n_receivers=rec.shape[0], eps=e["eps"], tau=e["tau"],
                                                             batch=args.batch))
        tot = {"beam_steps": 0, "evals": 0, "crossings": 0, "spawned": 0, "capped": 0}
        for s0 in range(0, e["nsteps"], seg):
            n = min(seg, e["nsteps"] - s0)
            part, st = fga.fga_evolve(med, beams, e["dt"], n, receivers=rec, eps=e["eps"], tau=e["tau"],
                                      ws=state["ws"], batch=args.batch, resort=args.resort)
            state["seis"][:, s0:s0 + n].copy_(part)
            for k in tot:
                tot[k] += st[k]
            print("bench: steps %d..%d done, %d beams" % (s0, s0 + n, beams.count), file=sys.stderr, flush=True)
        return n0, tot

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fga.fga_profile_enable(True)
    t0 = time.perf_counter()
    acc = {"beam_steps": 0, "evals": 0, "crossings": 0, "spawned": 0, "capped": 0, "beams": 0}
    for _ in range(args.steps):
        n0, tot = step()
        acc["beams"] += n0
        for k in tot:
            acc[k] += tot[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {fga.KERNEL_NAMES[k]: fga.fga_profile_read(k) for k in fga.KERNEL_NAMES}
    fga.fga_profile_enable(False)
    K = args.steps
    roof, _ = roofline({"beam_steps": acc["beam_steps"], "ev_rec": acc["evals"], "ev_grid": 0}, prof, "layered")
    line = {
        "metric": "beam-steps/s + beam-point evals/s; served solves/s, p50/p99 at rel-L2<=1e-3",
        "value": acc["beam_steps"] / elapsed, "unit": "beam-steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "layered spherical Earth-like model, 4 shells (radii %s), point moment-tensor "
                               "source with Ricker wavelet at r = %.3f, eps = 1/256, q %d^3 x %d directions x %d "
                               "shells x 3 branches x 2 directions, %d RK4 steps to T = 1.5 with interface "
                               "splitting (generation cap 3), %d surface receivers x %d samples, FP64"
                               % (", ".join("%.3f" % r for r in e["bounds"]), float(np.linalg.norm(e["x0"])),
                                  e["nq"], e["ndir"], e["nshell"], e["nsteps"], rec.shape[0], e["nsteps"]),
                   "beams": int(acc["beams"] / K), "parallelism": "single GPU"},
        "beam_point_evals_per_s": acc["evals"] / elapsed,
        "interface_hits_per_step": acc["crossings"] // K, "children_per_step": acc["spawned"] // K,
        "capped_per_step": acc["capped"] // K, "beams_at_end": int(beams.count),
        "kernel_ms_per_step": {k: v[1] / K for k, v in prof.items()},
        "roofline": roof,
    }
    print(json.dumps(line), flush=True)


def serve(args):
    """Serving sweep: 4 resident smooth models (128^3), requests from the
    seeded sweep generator; phase 1 submits all requests at once (saturated
    throughput), phase 2 submits them at Poisson arrivals with rate
    load x saturated throughput and reports latency percentiles."""
    import torch
    import fga_inputs as fi
    import paper_1810_06760_amd as fga
    torch.cuda.set_device(0)
    models = [fga.Medium.grid(fi.sweep_model(j), fi.node_grid(128), cs_ratio=1.0 / math.sqrt(3.0)) for j in range(4)]
    reqs = [fi.sweep_request(i) for i in range(args.requests)]

    prec = fga.FGA_FP32 if args.serve_precision == "mixed" else fga.FGA_FP64

    def request(rq, precision=None):
        src = fga.point_source(rq["eps"], rq["x0"], rq["M"], nq=rq["nq"], ndir=rq["ndir"], nshell=rq["nshell"])
        return fga.make_request(models[rq["model"]], None, None, rq["receivers"], rq["tau"], rq["dt"],
                                rq["nsteps"], 1, precision=prec if precision is None else precision, source=src)

    budget = int(args.hbm_budget_gb * 2 ** 30)
    # warm-up: one solve (module load, first allocations)
    srv = fga.Server(budget, 1)
    r, sz, keep = request(reqs[0])
    srv.submit(r, keep=(keep, sz))
    assert srv.poll(1, wait_ms=600000)[0]["status"] == 0
    srv.close()

    def phase(arrivals):
        srv = fga.Server(budget, args.slots)
        held = []
        done = []
        t0 = time.perf_counter()
        try:
            for k, rq in enumerate(reqs):
                wait = arrivals[k] - (time.perf_counter() - t0)
                if wait > 0:
                    done += srv.poll(64, wait_ms=int(wait * 1000))
                    rest = arrivals[k] - (time.perf_counter() - t0)
                    if rest > 0:
                        time.sleep(rest)
                r, sz, keep = request(rq)
                srv.submit(r, keep=(keep, sz))
                held.append((r, sz, keep))
            while len(done) < len(reqs):
                got = srv.poll(64, wait_ms=600000)
                if not got:
                    raise RuntimeError("serving made no progress")
                done += got
                print("bench: %d of %d solves done" % (len(done), len(reqs)), file=sys.stderr, flush=True)
            st = srv.status()
        finally:
            srv.close()
        bad = [c for c in done if c["status"] != 0]
        if bad:
            raise RuntimeError("failed solves: %s" % bad[:3])
        seis_by_req = {}
        for k, (r, sz, keep) in enumerate(held):
            seis_by_req[k] = sz
        lat = np.array([c["t_done"] - c["t_submit"] for c in done])
        span = max(c["t_done"] for c in done) - min(c["t_submit"] for c in done)
        return {"seis": seis_by_req, "solves_per_s": len(done) / span, "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "makespan_s": span, "peak_running": st["peak_running"],
                "beam_steps": int(sum(c["beam_steps"] for c in done)), "evals": int(sum(c["evals"] for c in done)),
                "beams": [int(c["beams"]) for c in done]}

    sat = phase([0.0] * len(reqs))
    print("bench: saturated phase %.1f s, %.3f solves/s" % (sat["makespan_s"], sat["solves_per_s"]),
          file=sys.stderr, flush=True)
    rate = args.load * sat["solves_per_s"]
    gen = np.random.default_rng(5999)
    arrivals = np.cumsum(gen.exponential(1.0 / rate, len(reqs)))
    arrivals -= arrivals[0]
    poi = phase(list(arrivals))
    beams = np.array(sat["beams"])
    err = None
    if prec != fga.FGA_FP64:
        # the same first 8 requests in FP64, one slot
        srv = fga.Server(budget, args.slots)
        ref = {}
        try:
            for k in range(min(8, len(reqs))):
                r, sz, keep = request(reqs[k], fga.FGA_FP64)
                ref[srv.submit(r, keep=(keep, sz))] = (k, sz)
            got = []
            while len(got) < len(ref):
                got += srv.poll(16, wait_ms=600000)
        finally:
            srv.close()
        err = max(float(np.linalg.norm(sat["seis"][k] - sz) / np.linalg.norm(sz)) for k, sz in ref.values())
    line = {
        "metric": "served solves/s, p50/p99 latency",
        "value": poi["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 1,
        "ms_per_step": 1e3 / poi["solves_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fga.FGA_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "tomography sweep: %d requests over 4 resident 128^3 smooth random models, point "
                               "moment-tensor sources (Ricker) at random positions, eps in {1/32, 1/64, 1/128}, "
                               "128..1024 receivers x 250 samples, 250 FP64 RK4 steps, %s receiver sums; "
                               "Poisson arrivals at %.2f x saturated rate"
                               % (len(reqs), "FP64" if prec == fga.FGA_FP64 else "mixed (FP32 exp/sin/cos)",
                                  args.load),
                   "slots": args.slots, "hbm_budget_gb": args.hbm_budget_gb, "parallelism": "single GPU"},
        "p50_s": poi["p50_s"], "p99_s": poi["p99_s"], "arrival_rate": rate,
        "saturated": {k: sat[k] for k in ("solves_per_s", "p50_s", "p99_s", "makespan_s", "peak_running")},
        "poisson_peak_running": poi["peak_running"],
        "beams_per_request": {"min": int(beams.min()), "median": int(np.median(beams)), "max": int(beams.max())},
        "beam_steps_per_s_saturated": sat["beam_steps"] / sat["makespan_s"],
        "evals_per_s_saturated": sat["evals"] / sat["makespan_s"],
    }
    if err is not None:
        line["max_rel_l2_vs_fp64_first8"] = err
    print(json.dumps(line), flush=True)


def mixed(args):
    """Mixed-precision grid summation at eps = 1/512: the smooth random
    medium (128^3 table) and packet form of the default workload, q 50^3 x p 8^3 x 3 branches in waves (q slabs along z);
    each wave is decomposed, evolved 250 FP64 RK4 steps to T = 0.25 and summed
    onto the 256^3 grid (tau = 16) by every variant (FP64, FP32, BF16 hi+lo,
    FP16 hi+lo, FP16 rows x hi+lo factors), each added into its own output.  Reports per variant the
    tile-kernel time, algorithmic evals/s and its fraction of the operand
    type's dense MFMA peak, and the relative L2 error against the FP64 sum
    (itself at oracle parity).  --scale shrinks the q mesh per axis."""
    import torch
    import fga_inputs as fi
    import paper_1810_06760_amd as fga

    nq = max(4, int(round(50 * args.scale)))
    w, slabs = fi.mixed_waves(nq=nq, waves=args.waves)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    med = fga.medium_for(w)
    f = fga._complex_dev(w.f)
    cap = max(q.count for q in slabs) * w.pmesh.count * 3
    beams = fga.BeamSet(cap)
    n = w.out_grid.n
    variants = ["fp64", "fp32", "bf16x3", "fp16x3", "fp16x2"]
    outs = {v: torch.zeros((3, n[2], n[1], n[0], 2), dtype=torch.float64, device=dev) for v in variants}
    stats = {v: {"tile_ms": 0.0, "call_s": 0.0, "evals": 0} for v in variants}
    ws = {}
    tot = {"beams": 0, "beam_steps": 0, "decompose_s": 0.0, "evolve_s": 0.0}
    torch.cuda.synchronize()
    fga.fga_profile_enable(True)
    t0 = time.perf_counter()
    for k, qm in enumerate(slabs):
        mesh = fga.make_mesh(w.eps, qm, w.pmesh, w.ymesh, cull_abs=w.cull_abs)
        t = time.perf_counter()
        if "dec" not in ws:
            ws["dec"] = fga._workspace(fga.workspace_bytes("decompose", mesh=mesh))
        fga.fga_decompose(med, mesh, f, beams=beams, ws=ws["dec"])
        tot["decompose_s"] += time.perf_counter() - t
        t = time.perf_counter()
        if "ev" not in ws:
            ws["ev"] = fga._workspace(fga.workspace_bytes("evolve", beams=beams, nsteps=w.nsteps))
        _, st = fga.fga_evolve(med, beams, w.dt, w.nsteps, ws=ws["ev"])
        torch.cuda.synchronize()
        tot["evolve_s"] += time.perf_counter() - t
        tot["beams"] += beams.count
        tot["beam_steps"] += st["beam_steps"]
        print("bench: wave %d/%d: %d beams decomposed and evolved" % (k + 1, len(slabs), beams.count),
              file=sys.stderr, flush=True)
        for v in variants:
            gw = fga._workspace(fga.workspace_bytes("grid", beams=beams, mesh=w.out_grid, eps=w.eps, tau=w.tau),
                                ws.get("grid"))
            ws["grid"] = gw
            fga.fga_profile_read(fga.FGA_K_GRID_TILE, reset=True)
            t = time.perf_counter()
            _, ev = fga.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid, precision=GRID_PREC[v][0],
                                             out=outs[v], ws=gw, add=k > 0)
            torch.cuda.synchronize()
            stats[v]["call_s"] += time.perf_counter() - t
            stats[v]["tile_ms"] += fga.fga_profile_read(fga.FGA_K_GRID_TILE, reset=True)[1]
            stats[v]["evals"] += ev
            print("bench: wave %d/%d: grid %s done" % (k + 1, len(slabs), v), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fga.fga_profile_enable(False)
    ref = outs["fp64"]
    nref = float(torch.linalg.vector_norm(ref))
    var = {}
    for v in variants:
        s_ = stats[v]
        ach = FLOP_GRID_EVAL * s_["evals"] / (s_["tile_ms"] * 1e-3)
        var[v] = {"tile_kernel_s": s_["tile_ms"] * 1e-3, "call_s": s_["call_s"], "evals": s_["evals"],
                  "evals_per_s": s_["evals"] / (s_["tile_ms"] * 1e-3),
                  "achieved_tflops_algorithmic": ach / 1e12, "peak_tflops": GRID_PREC[v][1] / 1e12,
                  "frac_algorithmic": ach / GRID_PREC[v][1],
                  "mfma_flops_per_term": {"x3": 72, "x2": 48}.get(v[-2:], 24),
                  "rel_l2_vs_fp64": float(torch.linalg.vector_norm(outs[v] - ref)) / nref}
    dom = max(variants, key=lambda v: stats[v]["tile_ms"])
    line = {
        "metric": "beam-steps/s + beam-point evals/s; served solves/s, p50/p99 at rel-L2<=1e-3",
        "value": tot["beam_steps"] / elapsed,
        "unit": "beam-steps/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * elapsed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32/bf16/f16", "data": "synthetic",
        "config": {"workload": "mixed-precision grid: smooth random medium and packet at eps=1/512, q %d^3 x p 8^3 x 3 "
                               "branches in %d waves, 250 FP64 RK4 steps to T=0.25, 256^3 grid (tau=16) summed by "
                               "FP64, FP32, BF16 hi+lo, FP16 hi+lo and FP16 x (hi+lo) tile GEMMs" % (nq, len(slabs)),
                   "beams": tot["beams"], "waves": len(slabs), "parallelism": "single GPU"},
        "beam_point_evals_per_s": sum(stats[v]["evals"] for v in variants) / elapsed,
        "decompose_s": tot["decompose_s"], "evolve_s": tot["evolve_s"],
        "variants": var,
        "roofline": {"bound": "mfma", "kernel": "grid_tile/" + dom,
                     "achieved": var[dom]["achieved_tflops_algorithmic"], "peak": var[dom]["peak_tflops"],
                     "unit": "TFLOP/s", "frac": var[dom]["frac_algorithmic"], "traffic": None},
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d (WORLD_SIZE %d) is not supported"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve(args)
        return
    if args.workload == "layered":
        layered(args)
        return
    if args.workload == "mixed":
        mixed(args)
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8}), flush=True)
        return
    w, label = make_workload(args.workload, args.scale)
    elapsed, tot, prof = gpu_run(w, args)
    K = args.steps
    per = {k: v / K for k, v in tot.items() if k != "grid_rel_l2_vs_fp64"}
    value = tot["beam_steps"] / elapsed
    kind = "grid" if w.medium_nodes is not None else "homogeneous"
    roof, dom = roofline(tot, prof, kind, GRID_PREC[args.grid_precision][1],
                         default_workload=(args.workload == "smooth" and args.scale == 1.0))
    line = {
        "metric": "beam-steps/s + beam-point evals/s; served solves/s, p50/p99 at rel-L2<=1e-3",
        "value": value,
        "unit": "beam-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": label, "beams": int(per["beams"]), "global_batch": int(per["beams"]),
                   "parallelism": "single GPU"},
        "beam_point_evals_per_s": (tot["ev_rec"] + tot["ev_grid"]) / elapsed,
        "receiver_evals_per_step": int(per["ev_rec"]),
        "grid_evals_per_step": int(per["ev_grid"]),
        "kernel_ms_per_step": {k: v[1] / K for k, v in prof.items()},
        "roofline": roof,
    }
    if args.grid_precision != "fp64":
        line["grid_precision"] = args.grid_precision
        line["grid_rel_l2_vs_fp64"] = tot.get("grid_rel_l2_vs_fp64")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, per, w.qmesh.count * w.pmesh.count, args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
