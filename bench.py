#!/usr/bin/env python
"""Benchmark of the FGA hot path on one MI355X.

Default workload: the smooth random medium (cp = sqrt3 (1 + 0.2 g) on a 128^3
node grid), eps = 1/128, the Gaussian packet decomposed on the 32^3 q x 8^3 p
mesh with 3 branches (49,095,784 beams after the cull), RK4 with dt = 1e-3 to
T = 1 and 3-component seismograms at 256 receivers after every step, the
wavefield on the 128^3 grid.

One bench step = one FP64 RK4 time step of the whole beam set together with
its seismogram sample at the 256 receivers (integrator + receiver sums, the
library's chunked launches).  The beams are decomposed and advanced untimed to
the window (t = 0.5 by default: --window is the fraction of the horizon), W
warm-up steps follow, then K steps are timed with inputs resident in HBM.
Decompose and the 128^3 grid sum (at the window's end) are one-time per
solve and are timed on their own (decompose_s, grid_s).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload smooth|homogeneous|layered|mixed]
                  [--scale S] [--serve ...]
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

# Algorithmic FP64 work per unit (FMA = 2), the method's hand counts:
#   one RK4 beam-step (4 right-hand sides of the ray, variational and amplitude
#   equations + the RK4 combination): 3.2 kflop in a homogeneous medium,
#   4.0 kflop in a grid medium (trilinear medium terms);
#   one in-window receiver/point term: ~60 flop (exponent, phase, complex
#   exponential, 3 complex multiply-adds);
#   one in-window grid term: 3 complex multiply-adds = 24 flop.
FLOP_BEAM_STEP = {"homogeneous": 3200, "grid": 4000, "layered": 3200}
FLOP_POINT_EVAL = 60
FLOP_GRID_EVAL = 24
PEAK_FP64 = 78.6e12       # FP64 vector and FP64 matrix peak, MI355X
# grid summation variants: (library code, dense MFMA peak of the operand type)
GRID_PREC = {"fp64": (0, 78.6e12), "fp32": (1, 157.3e12), "bf16x3": (2, 2.5e15), "fp16x3": (3, 2.5e15),
             "fp16x2": (4, 2.5e15)}
HBM_PEAK = 8.0e12
# HBM bytes per launch of the dominant kernel in the default bench window (smooth
# workload, scale 1, K = 20 after W = 5), from rocprofv3 FETCH_SIZE / WRITE_SIZE
# scaled by a 1 GiB copy calibration; valid only while the kernel's source is
# unchanged (sha256 prefix) and the beam set is the one profiled, else null
TRAFFIC = {
    "sum_points": {"source": "paper_1810_06760_amd/csrc/k_points.hip", "sha256": "262f9ec0539f99f6",
                   "beams": 33044152, "bytes_per_launch": 2.3741e10},
    "integrate": {"source": "paper_1810_06760_amd/csrc/k_integrate.hip", "sha256": "b905efd85e76b798",
                  "beams": 33044152, "bytes_per_launch": 9.9295e9},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed RK4 steps (each with its receiver sample)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed RK4 steps right before the timed ones")
    ap.add_argument("--window", type=float, default=0.5,
                    help="the timed steps start at this fraction of the horizon T (untimed advance before)")
    ap.add_argument("--segment", type=int, default=250, help="RK4 steps per evolution call (progress between)")
    ap.add_argument("--workload", default="smooth",
                    choices=["smooth", "homogeneous", "layered", "crosswell", "mixed", "pointforce"])
    ap.add_argument("--waves", type=int, default=4, help="beam waves of the mixed-precision workload")
    ap.add_argument("--batch", type=int, default=0, help="beams per receiver-sum batch in the evolution (0: library default)")
    ap.add_argument("--chunk", type=int, default=0, help="RK4 steps per integrator launch (0: library default)")
    ap.add_argument("--resort", type=int, default=0,
                    help="steps between spatial re-sorts of the beams in the evolution (0: library default, <0 never)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="fraction of the q mesh per axis and of the time steps (quick runs only)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--segments", type=int, default=4, help="evolution calls per step (progress between them)")
    ap.add_argument("--cpu-beams", type=int, default=12288, help="(q,p) pairs in the oracle sample")
    ap.add_argument("--cpu-steps", type=int, default=1000, help="RK4 steps of the oracle sample")
    ap.add_argument("--serve", action="store_true",
                    help="serving run instead: a seeded sweep of forward-solve requests over 4 resident models, "
                         "saturated and at Poisson arrivals; prints solves/s with p50/p99 latency")
    ap.add_argument("--requests", type=int, default=48, help="requests per serving phase")
    ap.add_argument("--sweep", default="small", choices=["small", "stated"],
                    help="serving requests: 'stated' = eps 1/64..1/512, 1e5..5e7 beams, 2000 samples (the "
                         "tomography sweep's own sizes); 'small' = eps 1/32..1/128, 250 samples")
    ap.add_argument("--slots", type=int, default=4, help="concurrent request slots of the server")
    ap.add_argument("--hbm-budget-gb", type=float, default=240.0, help="server device-memory budget")
    ap.add_argument("--load", type=float, default=0.8, help="Poisson arrival rate as a fraction of saturated")
    ap.add_argument("--serve-precision", default="fp64", choices=["fp64", "mixed", "mixed32"],
                    help="receiver sums of the served solves (mixed: FP32 exp/sin/cos of FP64-reduced arguments, "
                         "FP64 products and sums; mixed32: FP32 products and per-lane sums as well; the mixed runs "
                         "also report their error against FP64 solves of the 8 smallest requests)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (the known-size kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--unmerged", action="store_true",
                    help="SH and SV as two beams per (q, p, direction) (default: one S beam carrying both)")
    ap.add_argument("--medium-interp", default="trilinear", choices=["trilinear", "cubic"],
                    help="smooth workload: trilinear node fields (default) or the C2 cubic B-spline medium")
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
    """Decompose, advance untimed to the window, then time K RK4 steps of the
    whole beam set (each with its receiver sample); decompose and the grid sum
    are timed on their own, once per solve."""
    import torch
    import paper_1810_06760_amd as fga

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    med = fga.medium_for(w)
    mesh = fga.mesh_for(w, merge_s=not args.unmerged)
    f = fga._complex_dev(w.f)
    rec = fga._dev(w.receivers, torch.float64) if w.receivers is not None else None
    nq = w.qmesh.count * w.pmesh.count * 3
    beams = fga.BeamSet(nq)
    ws_dec = fga._workspace(fga.workspace_bytes("decompose", mesh=mesh))
    seg = max(1, args.segment)
    ws_ev = None
    seis = {}

    def decompose():
        torch.cuda.synchronize()
        t = time.perf_counter()
        fga.fga_decompose(med, mesh, f, beams=beams, ws=ws_dec)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def evolve(nsteps, what):
        """nsteps RK4 steps in calls of at most `seg` steps; returns summed stats."""
        nonlocal ws_ev
        if ws_ev is None:
            ws_ev = fga._workspace(fga.workspace_bytes(
                "evolve", beams=beams, nsteps=seg, n_receivers=0 if rec is None else rec.shape[0],
                eps=w.eps, tau=w.tau, batch=args.batch, chunk=args.chunk))
        tot = {"beam_steps": 0, "evals": 0}
        done = 0
        while done < nsteps:
            n = min(seg, nsteps - done)
            out = None
            if rec is not None:
                if n not in seis:
                    seis[n] = torch.empty((rec.shape[0], n, 3, 2), dtype=torch.float64, device=dev)
                out = seis[n]
            _, st = fga.fga_evolve(med, beams, w.dt, n, receivers=rec, eps=w.eps, tau=w.tau, seis=out,
                                   ws=ws_ev, batch=args.batch, resort=args.resort, chunk=args.chunk)
            tot["beam_steps"] += st["beam_steps"]
            tot["evals"] += st["evals"]
            done += n
            print("bench: %s: %d of %d steps done" % (what, done, nsteps), file=sys.stderr, flush=True)
        return tot

    W, K = args.warmup, args.steps
    advance = int(round(args.window * w.nsteps))
    advance = max(0, min(advance, w.nsteps - W - K))
    decompose()                      # first call: module load, allocations
    t_dec = decompose()
    n0 = beams.count
    print("bench: decomposed %d beams in %.3f s" % (n0, t_dec), file=sys.stderr, flush=True)
    if advance:
        evolve(advance, "untimed advance to the window")
    if W:
        evolve(W, "warmup")
    torch.cuda.synchronize()
    fga.fga_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = evolve(K, "timed window")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {fga.KERNEL_NAMES[k]: fga.fga_profile_read(k) for k in fga.KERNEL_NAMES}
    fga.fga_profile_enable(False)
    tot = {"beams": beams.count, "beams_decomposed": n0, "beam_steps": st["beam_steps"], "ev_rec": st["evals"],
           "decompose_s": t_dec, "advance_steps": advance, "t_window": ((advance + W) * w.dt, (advance + W + K) * w.dt)}
    if w.out_grid is not None:
        ws_grid = fga._workspace(fga.workspace_bytes("grid", beams=beams, mesh=w.out_grid, eps=w.eps, tau=w.tau))
        out, _ = fga.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid,
                                          precision=GRID_PREC[args.grid_precision][0], ws=ws_grid)
        fga.fga_profile_enable(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out, ev_grid = fga.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid,
                                                precision=GRID_PREC[args.grid_precision][0], out=out, ws=ws_grid)
        torch.cuda.synchronize()
        tot["grid_s"] = time.perf_counter() - t
        tot["grid_tile"] = fga.fga_profile_read(fga.FGA_K_GRID_TILE)
        fga.fga_profile_enable(False)
        tot["ev_grid"] = ev_grid
        if args.grid_precision != "fp64":
            # error of the mixed variant against the FP64 path (itself at oracle parity), same beams
            ref, _ = fga.fga_reconstruct_grid(beams, w.eps, w.tau, w.out_grid, precision=0, ws=ws_grid)
            tot["grid_rel_l2_vs_fp64"] = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
        print("bench: %s grid sum at t = %.3f in %.3f s" % (w.out_grid.n, tot["t_window"][1], tot["grid_s"]),
              file=sys.stderr, flush=True)
    return t1 - t0, tot, prof


def traffic_for(name, default_workload, beams):
    """Measured HBM bytes per launch, if taken on this workload, beam set and kernel source."""
    import hashlib
    t = TRAFFIC.get(name)
    if t is None or not default_workload or t["beams"] != beams:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest()[:16] != t["sha256"]:
            return None
    return t["bytes_per_launch"]


def roofline(tot, prof, medium_kind, default_workload=False):
    """Dominant kernel of the timed window (integrator or receiver sums):
    algorithmic flops per launch / mean launch duration (hipEvents recorded on
    the launch's own stream by the library)."""
    work = {
        "integrate": tot["beam_steps"] * FLOP_BEAM_STEP[medium_kind],
        "sum_points": tot["ev_rec"] * FLOP_POINT_EVAL,
    }
    name = max(work, key=lambda k: prof.get(k, (0, 0.0))[1])
    launches, ms = prof[name]
    if launches == 0 or ms <= 0:
        return None, name
    achieved = work[name] / (ms * 1e-3)
    return {"bound": "alu", "kernel": name, "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
            "traffic": traffic_for(name, default_workload, tot.get("beams")),
            "launches": launches, "avg_launch_ms": ms / launches,
            "flop_per_unit": FLOP_BEAM_STEP[medium_kind] if name == "integrate" else FLOP_POINT_EVAL,
            "units_per_launch": (tot["beam_steps"] if name == "integrate" else tot["ev_rec"]) / launches}, name


def cpu_baseline(w, args):
    """The oracle on a bounded sample of the same workload (about 10-20 s of
    host work): 12288 random (q, p) pairs decomposed by FBI quadrature (SH and SV
    merged unless --unmerged), then RK4 steps
    in the same medium, each followed by the sum at the 256 receivers.  The
    per-beam-step time (integrator + one receiver sample) gives beam-steps/s
    at the threads the oracle uses."""
    import oracle as om
    g = np.random.default_rng(4242)
    nqp = w.qmesh.count * w.pmesh.count
    pick = g.choice(nqp, size=min(args.cpu_beams, nqp), replace=False)
    iq, ip = pick % w.qmesh.count, pick // w.qmesh.count
    med = om.medium_for(w)
    F = om.fbi(w.f, w.ymesh, w.qmesh.points()[iq], w.pmesh.points()[ip], w.eps)
    beams = om.make_beams(w.qmesh, w.pmesh, F, w.eps, iq, ip, cull_abs=0.0)
    if not args.unmerged:
        beams = om.merge_s_beams(beams, nqp)
    nsteps = min(w.nsteps, args.cpu_steps)
    t_ev = t_rec = 0.0
    for s in range(nsteps):
        t = time.perf_counter()
        om.evolve(med, beams, w.dt, 1)
        t_ev += time.perf_counter() - t
        if w.receivers is not None:
            t = time.perf_counter()
            om.sum_points(beams, w.receivers, w.eps, w.tau)
            t_rec += time.perf_counter() - t
    per_beam_step = (t_ev + t_rec) / (nsteps * len(beams))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / per_beam_step, "unit": "beam-steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d random (q,p) pairs x 3 branches (%d beams%s) of the same workload, %d RK4 steps from "
                      "t = 0 each followed by the %d-receiver sum; %.1f s integrate + %.1f s receiver sums"
                      % (len(pick), len(beams), "" if args.unmerged else ", SH and SV merged", nsteps,
                         0 if w.receivers is None else len(w.receivers), t_ev, t_rec),
            "seconds": t_ev + t_rec}


def layered(args):
    """Layered spherical Earth-like model (4 shells) with a point moment-tensor
    source (Ricker, eps = 1/256): decompose, then 2000 RK4 steps with
    interface splitting (generation cap 3) and 512 surface receivers sampled
    every step.  --scale shrinks the direction count and the step count.
    --workload crosswell runs the crosswell model of Sec. 4 the same way
    (fga_inputs.crosswell: the ninth source, 32 receivers in the other well)."""
    import torch
    import fga_inputs as fi
    import paper_1810_06760_amd as fga
    torch.cuda.set_device(0)
    sc = args.scale
    cross = args.workload == "crosswell"
    if cross:
        # the crosswell model (Sec. 4): flat layers under a free surface, the low-velocity region
        e = fi.crosswell(ndir=max(16, int(round(1600 * sc))), nsteps=max(8, int(round(2000 * sc))))
        med = fga.Medium.layered(0, e["bounds"], e["cp"], e["cs"], e["rho"], surface=e["surface"],
                                 anomaly=e["anomaly"])
    else:
        e = fi.layered_earth(ndir=max(16, int(round(1600 * sc))), nsteps=max(8, int(round(2000 * sc))))
        med = fga.Medium.layered(1, e["bounds"], e["cp"], e["cs"], e["rho"])
    src = fga.point_source(e["eps"], e["x0"], e["M"], nq=e["nq"], ndir=e["ndir"], nshell=e["nshell"],
                           merge_s=not args.unmerged)
    ncand = int(fga.lib().fga_point_source_candidates(fga.C.byref(src)))
    beams = fga.BeamSet(12 * ncand)   # room for interface children (generation cap 3)
    if cross:
        rec, coords = fga._dev(e["receivers"], torch.float64), fga.FGA_COORDS_CARTESIAN
    else:   # stations as (r, longitude, latitude)
        rec, coords = fga._dev(e["receivers_rtp"], torch.float64), fga.FGA_COORDS_SPHERICAL
    nseg = max(1, min(args.segments, e["nsteps"]))
    seg = -(-e["nsteps"] // nseg)
    state = {"ws": None, "seis": torch.empty((rec.shape[0], e["nsteps"], 3, 2), dtype=torch.float64, device="cuda")}

    def step():
        fga.fga_decompose_point_source(med, src, beams=beams)
        n0 = beams.count
        if state["ws"] is None:
            state["ws"] = fga._workspace(fga.workspace_bytes("evolve", beams=beams, nsteps=seg,
                                                             n_receivers=rec.shape[0], eps=e["eps"], tau=e["tau"],
                                                             batch=args.batch, coords=coords))
        tot = {"beam_steps": 0, "evals": 0, "crossings": 0, "spawned": 0, "capped": 0}
        for s0 in range(0, e["nsteps"], seg):
            n = min(seg, e["nsteps"] - s0)
            part, st = fga.fga_evolve(med, beams, e["dt"], n, receivers=rec, eps=e["eps"], tau=e["tau"],
                                      ws=state["ws"], batch=args.batch, resort=args.resort, coords=coords)
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
        "config": {"s_beams": "separate SH and SV" if args.unmerged else "SH and SV merged per (q, p, direction)",
                   "workload": ("crosswell model (Sec. 4 eq:true_c, 100 m / 1000 m/s units): 3 flat layers "
                                "under a free surface, Gaussian low-velocity region, explosion with Ricker "
                                "wavelet at depth %.0f m, eps = 1/128, q %d^3 x %d directions x %d shells x "
                                "3 branches x 2 directions, %d RK4 steps to T = 2 (0.2 s) with interface and "
                                "surface splitting (generation cap 3), %d well receivers x %d samples, FP64"
                                % (100 * (3.0 - e["x0"][2]), e["nq"], e["ndir"], e["nshell"], e["nsteps"],
                                   rec.shape[0], e["nsteps"])) if cross else
                               ("layered spherical Earth-like model, 4 shells (radii %s), point moment-tensor "
                                "source with Ricker wavelet at r = %.3f, eps = 1/256, q %d^3 x %d directions x %d "
                                "shells x 3 branches x 2 directions, %d RK4 steps to T = 1.5 with interface "
                                "splitting (generation cap 3), %d surface receivers x %d samples, FP64"
                                % (", ".join("%.3f" % r for r in e["bounds"]), float(np.linalg.norm(e["x0"])),
                                   e["nq"], e["ndir"], e["nshell"], e["nsteps"], rec.shape[0], e["nsteps"])),
                   "beams": int(acc["beams"] / K), "parallelism": "single GPU"},
        "beam_point_evals_per_s": acc["evals"] / elapsed,
        "interface_hits_per_step": acc["crossings"] // K, "children_per_step": acc["spawned"] // K,
        "capped_per_step": acc["capped"] // K, "beams_at_end": int(beams.count),
        "kernel_ms_per_step": {k: v[1] / K for k, v in prof.items()},
        "roofline": roof,
    }
    print(json.dumps(line), flush=True)


def pointforce(args):
    """The accuracy experiment of Sec. 2.3 in box units (c_S = 1): a point
    force d F(t), d = (1, 1, 1), F(t) = cos(256 (t + T0)) exp(-(t + T0)^2 / (1/32)^2)
    (1.4702 Hz, eps_S = 1/256), homogeneous c_P = sqrt(3), c_S = 1, rho = 1;
    two-way point-force beams launched at t = -T0 (q 14^3 x 2000 directions x
    40 shells x 3 branches x 2 directions, cull 1e-4), RK4 to t = 0.25 (6.93 s)
    and the field on the 128^2 grid of the plane y = 1/2.  One step = one
    whole solve; reports its parts and the relative L2 error against the
    closed-form solution (eq:ex_anal; evaluated by tests/point_force_exact.py)."""
    import torch
    import paper_1810_06760_amd as fga
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import point_force_exact as pfe
    torch.cuda.set_device(0)
    eps, cp, cs = 1.0 / 256, math.sqrt(3.0), 1.0
    omega, t0, sig, T = 256.0, 0.1768 / (128.0 / 4.619), 1.0 / 32, 0.25
    x0, d = (0.5, 0.5, 0.5), (1.0, 1.0, 1.0)
    qhalf = 4 * math.sqrt(eps) + 3 * cp * sig
    nq = int(math.ceil(2 * qhalf / math.sqrt(eps)))
    pc = omega * eps / cp
    A = 1.0 / sig ** 2 + cp * cp / (2 * eps)
    psi_scale = eps / (2 * pc) * math.sqrt(3.0) / cp * math.sqrt(math.pi / A)
    src = fga.point_force(eps, x0, d, nq=nq, qhalf=qhalf, ndir=2000, nshell=40, omega=omega, t0=t0, width=sig,
                          t_ref=-t0, shell_lo=0.3 * pc, shell_hi=1.7 * pc, cull_abs=1e-4 * psi_scale,
                          merge_s=not args.unmerged)
    med = fga.Medium.homogeneous(cp, cs, 1.0)
    ncand = int(fga.lib().fga_point_force_candidates(fga.C.byref(src)))
    beams = fga.BeamSet(ncand // 12)
    n = 128
    ax = (np.arange(n) + 0.5) / n
    X, Z = np.meshgrid(ax, ax, indexing="xy")
    pts = np.stack([X.ravel(), np.full(n * n, 0.5), Z.ravel()], axis=1)
    xyz = fga._dev(pts, torch.float64)
    nsteps = 64
    ws_ev = fga._workspace(fga.workspace_bytes("evolve", beams=beams, nsteps=nsteps))

    def solve():
        t = {}
        torch.cuda.synchronize()
        a = time.perf_counter()
        fga.fga_decompose_point_force(med, src, beams=beams)
        torch.cuda.synchronize()
        b = time.perf_counter()
        _, st = fga.fga_evolve(med, beams, (T + t0) / nsteps, nsteps, ws=ws_ev)
        torch.cuda.synchronize()
        c = time.perf_counter()
        u, ev = fga.fga_reconstruct_points(beams, eps, 25.0, xyz)
        torch.cuda.synchronize()
        e = time.perf_counter()
        t.update(decompose_s=b - a, evolve_s=c - b, reconstruct_s=e - c, beam_steps=st["beam_steps"], evals=ev)
        return u, t

    for i in range(args.warmup):
        solve()
        print("bench: warm-up solve %d done" % (i + 1), file=sys.stderr, flush=True)
    fga.fga_profile_enable(True)
    t0w = time.perf_counter()
    parts = []
    for i in range(args.steps):
        u, t = solve()
        parts.append(t)
        print("bench: solve %d done" % (i + 1), file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0w
    prof = {fga.KERNEL_NAMES[k]: fga.fga_profile_read(k) for k in fga.KERNEL_NAMES}
    fga.fga_profile_enable(False)
    got = fga.to_complex(u)
    ref = pfe.displacement(pts, T, x0, d, cp, cs, 1.0, omega, t0, sig)
    err = float(np.linalg.norm(got.real - ref) / np.linalg.norm(ref))
    K = args.steps
    roof, _ = roofline({"beam_steps": sum(p["beam_steps"] for p in parts), "ev_rec": sum(p["evals"] for p in parts)},
                       prof, "homogeneous")
    line = {
        "metric": "beam-steps/s + beam-point evals/s; served solves/s, p50/p99 at rel-L2<=1e-3",
        "value": sum(p["beam_steps"] for p in parts) / elapsed, "unit": "beam-steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"s_beams": "separate SH and SV" if args.unmerged else "SH and SV merged per (q, p, direction)",
                   "workload": "point force with its time function in a homogeneous medium (the accuracy "
                               "experiment of Sec. 2.3 in box units, eps_S = 1/256): %d beams of %d candidates "
                               "(q %d^3 x 2000 directions x 40 shells x 3 branches x 2 directions), %d RK4 steps "
                               "to t = 0.25, field on a 128^2 plane; one step = one whole solve"
                               % (beams.count, ncand, nq, nsteps),
                   "beams": beams.count, "parallelism": "single GPU"},
        "rel_l2_vs_exact": err,
        "paper_rel_l2_vs_exact": 0.0384,
        "solve_parts_s": {k: float(np.mean([p[k] for p in parts])) for k in ("decompose_s", "evolve_s",
                                                                             "reconstruct_s")},
        "beam_point_evals_per_s": sum(p["evals"] for p in parts) / elapsed,
        "kernel_ms_per_step": {k: v[1] / K for k, v in prof.items() if v[0]},
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
    stated = args.sweep == "stated"
    if stated:
        # each eps of the stated sweep equally often (i mod 4), in a seeded random order
        order = np.random.default_rng(5998).permutation(args.requests)
        reqs = [fi.sweep5_request(int(i), eps_index=int(i) % 4) for i in order]
    else:
        reqs = [fi.sweep_request(i) for i in range(args.requests)]

    prec = {"fp64": fga.FGA_FP64, "mixed": fga.FGA_FP32, "mixed32": fga.FGA_FP32_ACC32}[args.serve_precision]

    def request(rq, precision=None):
        src = fga.point_source(rq["eps"], rq["x0"], rq["M"], nq=rq["nq"], ndir=rq["ndir"], nshell=rq["nshell"],
                               merge_s=not args.unmerged)
        return fga.make_request(models[rq["model"]], None, None, rq["receivers"], rq["tau"], rq["dt"],
                                rq["nsteps"], 1, precision=prec if precision is None else precision, source=src)

    budget = int(args.hbm_budget_gb * 2 ** 30)
    # warm-up: one solve of the smallest request (module load, first allocations)
    srv = fga.Server(budget, 1)
    r, sz, keep = request(min(reqs, key=lambda q: q["ndir"] * q["nshell"] / q["eps"]))
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
                # until request k arrives, collect completions (a line at least every 30 s)
                while True:
                    wait = arrivals[k] - (time.perf_counter() - t0)
                    if wait <= 0:
                        break
                    got = srv.poll(64, wait_ms=max(1, int(min(wait, 30.0) * 1000)))
                    done += got
                    print("bench: %.1f s, %d of %d solves done, next arrival in %.1f s"
                          % (time.perf_counter() - t0, len(done), len(reqs),
                             max(0.0, arrivals[k] - (time.perf_counter() - t0))), file=sys.stderr, flush=True)
                r, sz, keep = request(rq)
                srv.submit(r, keep=(keep, sz))
                held.append((r, sz, keep))
                print("bench: request %d of %d submitted at %.1f s, %d done" % (k + 1, len(reqs),
                      time.perf_counter() - t0, len(done)), file=sys.stderr, flush=True)
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
        # the same requests in FP64 (the 8 smallest), one slot
        srv = fga.Server(budget, args.slots)
        ref = {}
        small = sorted(range(len(reqs)), key=lambda k: reqs[k]["ndir"] * reqs[k]["nshell"] / reqs[k]["eps"])[:8]
        try:
            for k in small:
                r, sz, keep = request(reqs[k], fga.FGA_FP64)
                ref[srv.submit(r, keep=(keep, sz))] = (k, sz)
            got = []
            while len(got) < len(ref):
                got += srv.poll(16, wait_ms=600000)
                print("bench: FP64 reference %d of %d solves done" % (len(got), len(ref)), file=sys.stderr, flush=True)
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
        "config": {"s_beams": "separate SH and SV" if args.unmerged else "SH and SV merged per (q, p, direction)",
                   "workload": "tomography sweep: %d requests over 4 resident 128^3 smooth random models, point "
                               "moment-tensor sources (Ricker) at random positions, %s, "
                               "128..1024 receivers, %s receiver sums; Poisson arrivals at %.2f x saturated rate"
                               % (len(reqs),
                                  "eps in {1/64, 1/128, 1/256, 1/512} (each 1/4 of the requests; 9.8e4, 8.0e5, "
                                  "6.4e6, 5.1e7 candidate beams), 2000 FP64 RK4 steps to T = 1 with a sample after "
                                  "every step" if stated else
                                  "eps in {1/32, 1/64, 1/128}, 250 FP64 RK4 steps with a sample after every step",
                                  {fga.FGA_FP64: "FP64", fga.FGA_FP32: "mixed (FP32 exp/sin/cos, FP64 sums)",
                                   fga.FGA_FP32_ACC32: "mixed (FP32 exp/sin/cos, FP32 products and per-lane "
                                   "sums)"}[prec], args.load),
                   "slots": args.slots, "hbm_budget_gb": args.hbm_budget_gb, "parallelism": "single GPU"},
        "p50_s": poi["p50_s"], "p99_s": poi["p99_s"], "arrival_rate": rate,
        "saturated": {k: sat[k] for k in ("solves_per_s", "p50_s", "p99_s", "makespan_s", "peak_running")},
        "poisson_peak_running": poi["peak_running"],
        "beams_per_request": {"min": int(beams.min()), "median": int(np.median(beams)), "max": int(beams.max())},
        "beam_steps_per_s_saturated": sat["beam_steps"] / sat["makespan_s"],
        "evals_per_s_saturated": sat["evals"] / sat["makespan_s"],
    }
    if err is not None:
        line["max_rel_l2_vs_fp64_smallest8"] = err
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
        mesh = fga.make_mesh(w.eps, qm, w.pmesh, w.ymesh, cull_abs=w.cull_abs, merge_s=not args.unmerged)
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
        "config": {"s_beams": "separate SH and SV" if args.unmerged else "SH and SV merged per (q, p, direction)",
                   "workload": "mixed-precision grid: smooth random medium and packet at eps=1/512, q %d^3 x p 8^3 x 3 "
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
    if args.workload in ("layered", "crosswell"):
        layered(args)
        return
    if args.workload == "mixed":
        mixed(args)
        return
    if args.workload == "pointforce":
        pointforce(args)
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
    if args.medium_interp == "cubic" and w.medium_nodes is not None:
        w.medium_smooth = True
        label = label.replace("eps=1/128", "C2 cubic B-spline medium, eps=1/128")
    elapsed, tot, prof = gpu_run(w, args)
    K = args.steps
    value = tot["beam_steps"] / elapsed
    kind = "grid" if w.medium_nodes is not None else "homogeneous"
    roof, dom = roofline(tot, prof, kind, default_workload=(args.workload == "smooth" and args.scale == 1.0
                                                             and K == 20 and args.warmup == 5
                                                             and args.medium_interp == "trilinear"))
    t_a, t_b = tot["t_window"]
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
        "config": {"s_beams": "separate SH and SV" if args.unmerged else "SH and SV merged per (q, p, direction)",
                   "workload": label + "; one step = one RK4 step of all beams with its receiver sample, "
                               "timed over t = %.3f..%.3f after an untimed advance; decompose and the grid "
                               "sum timed separately per solve" % (t_a, t_b),
                   "beams": int(tot["beams"]), "parallelism": "single GPU"},
        "beam_point_evals_per_s": tot["ev_rec"] / elapsed,
        "receiver_evals_per_step": int(tot["ev_rec"] / K),
        "kernel_ms_per_step": {k: v[1] / K for k, v in prof.items() if v[0]},
        "kernel_launches": {k: v[0] for k, v in prof.items() if v[0]},
        "decompose_s": tot["decompose_s"],
        "beams_decomposed": tot["beams_decomposed"],
        "roofline": roof,
    }
    if "grid_s" in tot:
        gl, gms = tot["grid_tile"]
        gpeak = GRID_PREC[args.grid_precision][1]
        line["grid"] = {"n": list(w.out_grid.n), "t": t_b, "precision": args.grid_precision, "s": tot["grid_s"],
                        "tile_kernel_s": gms * 1e-3, "evals": tot["ev_grid"],
                        "evals_per_s": tot["ev_grid"] / (gms * 1e-3) if gms > 0 else None,
                        "frac_of_peak": FLOP_GRID_EVAL * tot["ev_grid"] / (gms * 1e-3) / gpeak if gms > 0 else None}
        if "grid_rel_l2_vs_fp64" in tot:
            line["grid"]["rel_l2_vs_fp64"] = tot["grid_rel_l2_vs_fp64"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args)
        print("bench: cpu baseline done (%.1f s)" % line["cpu_baseline"]["seconds"], file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
