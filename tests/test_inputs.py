"""Host-side input generators (no method arithmetic): the wave split of the
mixed-precision workload covers the q mesh exactly once."""
import numpy as np

import fga_inputs as fi


def test_mixed_waves_partition_the_q_mesh():
    w, slabs = fi.mixed_waves(nq=10, ny=16, nout=16, waves=4)
    full = w.qmesh.points()
    parts = np.concatenate([s.points() for s in slabs])
    assert len(parts) == len(full) == w.qmesh.count
    key = lambda a: np.lexsort((a[:, 0], a[:, 1], a[:, 2]))
    # same points (a slab's origin is formed as lo + k h, so equal up to rounding)
    assert np.abs(parts[key(parts)] - full[key(full)]).max() <= 1e-14
    assert sum(s.n[2] for s in slabs) == 10
    assert max(s.n[2] for s in slabs) - min(s.n[2] for s in slabs) <= 1
    # the medium and packet are the smooth-medium workload's, at the requested eps
    w2 = fi.smooth_medium_packet(nq=10, ny=16, nout=16, nrec=0, eps=1.0 / 512)
    assert np.array_equal(w.medium_nodes, w2.medium_nodes) and np.array_equal(w.f, w2.f)


def test_crosswell_model_recipe():
    """The crosswell model's nondimensional recipe (Sec. 4, eq:true_c): depth
    d maps to z = 3 - d/100, the layer speeds and interfaces, the anomaly in
    the middle layer, the wells and their spacings."""
    import math
    import fga_inputs as fi
    c = fi.crosswell()
    assert c["bounds"] == [1.0, 2.0] and c["surface"] == 3.0
    assert c["cp"] == [2.2, 2.0, 1.8]                       # deepest layer first
    assert all(abs(s - p / math.sqrt(3.0)) < 1e-15 for s, p in zip(c["cs"], c["cp"]))
    amp, beta, x0, wts = c["anomaly"][1]
    assert amp == 0.1 and abs(beta - 1e4 / 450.0) < 1e-12   # 1/450 m^-2 in (100 m)^-2
    assert tuple(x0) == (0.75, 0.0, 1.5) and tuple(wts) == (1.0, 0.0, 1.0)   # 75 m, 150 m depth, y-invariant
    src, rec = c["sources"], c["receivers"]
    assert src.shape == (16, 3) and rec.shape == (32, 3)
    assert np.all(src[:, 0] == 0.0) and np.all(rec[:, 0] == 1.5)
    assert np.allclose(-np.diff(src[:, 2]) * 100, 16.0) and np.allclose(-np.diff(rec[:, 2]) * 100, 8.0)
    assert np.all(src[:, 2] < 3.0) and np.all(rec[:, 2] < 3.0)     # below the surface
    assert np.allclose(c["x0"], src[8])
    assert fi.crosswell(true_model=False)["anomaly"] is None  # the initial model eq:ini_c
