"""The beam-set entry points of the C ABI: fga_beams_export and
fga_beams_import copy the planes [0, count) exactly (to host arrays and
back), and fga_beams_info counts alive, quarantined, per-branch and child
beams as the exported planes do."""
import numpy as np
import pytest

import fga_inputs as fi
import oracle as om
from test_gpu_parity import fga, layered_case, oracle_to_dict, say

pytestmark = pytest.mark.gpu


def test_export_import_round_trip():
    m = fga()
    say("beams export/import")
    torch = pytest.importorskip("torch")
    w = fi.smooth_medium_packet(nq=4, np_=2, ny=16, nmed=16, nout=0, nrec=0)
    bs = m.fga_decompose(m.medium_for(w), m.mesh_for(w), w.f)
    m.fga_evolve(m.medium_for(w), bs, 2e-3, 10)
    n = bs.count
    d = bs.export()
    # the C export against the planes read directly
    F = bs.f64[:, :n].cpu().numpy()
    assert np.array_equal(d["Q"], F[m.FGA_Q:m.FGA_Q + 3].T)
    assert np.array_equal(d["S"], F[m.FGA_S])
    assert np.array_equal(d["lineage"], bs.lineage[:n].cpu().numpy())
    assert np.array_equal(d["flags"], bs.i32[m.FGA_FLAGS, :n].cpu().numpy())
    # import into a larger set, then the planes [0, n) are the same bits
    b2 = m.BeamSet(n + 100)
    b2.load(d)
    assert b2.count == n
    assert torch.equal(b2.f64[:, :n], bs.f64[:, :n])
    assert torch.equal(b2.i32[:, :n], bs.i32[:, :n])
    assert torch.equal(b2.lineage[:n], bs.lineage[:n])
    # too many beams for the capacity: FGA_ECAPACITY from the library
    small = m.BeamSet(3)
    with pytest.raises(ValueError, match="capacity"):
        small.load(d)
    F = np.zeros((m.FGA_NF64, 4))
    I = np.zeros((m.FGA_NI32, 4), dtype=np.int32)
    L = np.zeros(4, dtype=np.int64)
    with pytest.raises(Exception, match="capacity"):
        m._check(m.lib().fga_beams_import(m.C.byref(small.c), 4, F.ctypes.data, I.ctypes.data, L.ctypes.data,
                                          m._stream()))
    assert small.count == 0


def test_info_counts():
    m = fga()
    say("beams info")
    w, ob, med_o, med_g = layered_case("flat")
    bs = m.BeamSet(8 * len(ob))
    bs.load(oracle_to_dict(ob))
    m.fga_evolve(med_g, bs, 0.005, 40)
    d = bs.export()
    info = bs.info()
    alive = (d["flags"] & m.FGA_FLAG_ALIVE) != 0
    assert info["count"] == bs.count
    assert info["alive"] == int(alive.sum())
    assert info["quarantined"] == int(((d["flags"] & m.FGA_FLAG_QUARANTINED) != 0).sum())
    assert info["by_branch"] == [int((alive & (d["branch"] == b)).sum()) for b in range(3)]
    assert info["children"] == int((alive & (d["gen"] > 0)).sum()) > 0
