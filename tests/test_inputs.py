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
