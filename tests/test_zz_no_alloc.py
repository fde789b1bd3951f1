"""The allocation-free point sum (fga_reconstruct_points_noalloc, for callers
that cannot allocate device memory) against the workspace entry point
fga_reconstruct_points on the same beams and points (Step 3, eq:FGA): two
calls in a row, the second with fewer beams and fewer points, FP64 to
relative L2 <= 1e-10 with equal in-window term counts, the mixed path to
1e-10 of the mixed workspace path; sizes beyond the fixed scratch are
rejected before any device work.
"""
import numpy as np
import pytest

import fga_inputs as fi

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_noalloc_matches_workspace_entry_point():
    import torch
    import paper_1810_06760_amd as fga
    fga.lib()
    say("noalloc: two calls against fga_reconstruct_points")
    w = fi.smooth_medium_packet(nq=6, np_=3, ny=16, nmed=16, nout=0, nrec=0)
    med = fga.medium_for(w)
    beams = fga.fga_decompose(med, fga.mesh_for(w), w.f)
    fga.fga_evolve(med, beams, 2e-3, 60, resort=-1)
    n_all = beams.count
    assert n_all > 1000
    g = np.random.default_rng(31)
    cases = [(n_all, 300), (n_all // 3 + 17, 37)]      # second call: fewer beams, fewer points
    for k, (nb, npts) in enumerate(cases):
        beams.c.count = nb
        xyz = torch.from_numpy(g.random((npts, 3))).to("cuda")
        for prec in (fga.FGA_FP64, fga.FGA_FP32):
            ref, ev_ref = fga.fga_reconstruct_points(beams, w.eps, w.tau, xyz, precision=prec)
            out = torch.full((npts, 3, 2), float("nan"), dtype=torch.float64, device="cuda")
            got, ev = fga.fga_reconstruct_points_noalloc(beams, w.eps, w.tau, xyz, out, precision=prec)
            torch.cuda.synchronize()
            a, b = fga.to_complex(got), fga.to_complex(ref)
            say("  call %d: %d beams, %d points, precision %d: rel-L2 %.2e, evals %d / %d"
                % (k, nb, npts, prec, rel_l2(a, b), ev, ev_ref))
            assert np.all(np.isfinite(a))
            assert rel_l2(a, b) <= 1e-10
            assert ev == ev_ref and ev > 0
    beams.c.count = n_all


def test_noalloc_rejects_sizes_beyond_scratch():
    import torch
    import paper_1810_06760_amd as fga
    L = fga.lib()
    cap = int(L.fga_reconstruct_points_noalloc_max_bytes())
    assert cap == 64 << 20
    beams = fga.BeamSet(64)
    xyz = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    out = torch.zeros((1, 3, 2), dtype=torch.float64, device="cuda")
    n_big = cap // 48 + 1            # more points than the partial sums of one tile can hold
    st = L.fga_reconstruct_points_noalloc(fga.C.byref(beams.c), 1.0 / 64, 25.0, n_big, fga._ptr(xyz),
                                          fga.FGA_FP64, fga._ptr(out), fga._stream(), None)
    assert st == 2, st              # FGA_ENOMEM, nothing launched
    assert b"scratch" in L.fga_last_error()
