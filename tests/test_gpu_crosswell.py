"""The crosswell model of the tomography example (Sec. 4, eq:true_c and the
initial model eq:ini_c; fga_inputs.crosswell): three flat layers under a
traction-free surface, the middle one with the Gaussian low-velocity region,
a point explosion (Ricker) in one well and 32 receivers in the other.  The
GPU's point-source beams, their evolution with interface and surface
splitting, and the seismograms at the receivers against the oracle's, at a
reduced beam count and duration.

Bar: relative L2 <= 1e-10, integers exact.
"""
import numpy as np
import pytest

import fga_inputs as fi
import oracle as om
from test_gpu_parity import RTOL, fga, oracle_to_dict, rel_l2, say

pytestmark = pytest.mark.gpu


def media(c):
    m = fga()
    args = (0, c["bounds"], c["cp"], c["cs"], c["rho"])
    kw = dict(surface=c["surface"], anomaly=c["anomaly"])
    return om.layered(*args, **kw), m.Medium.layered(*args, **kw)


@pytest.mark.parametrize("true_model", [True, False])
def test_crosswell_seismogram_parity(true_model):
    m = fga()
    say("crosswell", true_model)
    c = fi.crosswell(eps=1.0 / 64, true_model=true_model)
    mo, mg = media(c)
    kw = dict(nq=4, ndir=48, nshell=3, ricker=True, cull_abs=1e-6)
    ob = om.point_source_beams(mo, om.point_source(c["eps"], c["x0"], c["M"], **kw))
    bs = m.fga_decompose_point_source(mg, m.point_source(c["eps"], c["x0"], c["M"], **kw))
    g = bs.export()
    assert np.array_equal(g["lineage"], ob["lineage"]) and np.array_equal(g["layer"], ob["layer"])
    assert rel_l2(g["w"], ob["w"]) <= RTOL
    rec = c["receivers"]
    nsteps, dt, stride = 80, 0.01, 4
    big = m.BeamSet(12 * bs.count)
    big.load(g)
    seis, st = m.fga_evolve(mg, big, dt, nsteps, receivers=rec, eps=c["eps"], tau=c["tau"], stride=stride)
    ref = np.zeros((len(rec), nsteps // stride, 3), dtype=np.complex128)
    cur = ob.copy()
    cnt = 0
    for s in range(nsteps // stride):
        cur, _ = om.evolve_layered(mo, cur, dt, stride, gmax=3, child_cut=1e-3)
        cur = cur[cur["alive"] == 1].copy()
        u, k = om.sum_points(cur, rec, c["eps"], c["tau"])
        ref[:, s, :] = u
        cnt += k
    say("beams %d -> %d, children %d" % (len(ob), big.count, st["spawned"]))
    assert st["spawned"] > 0 and st["evals"] == cnt > 0
    assert np.abs(ref[:, -4:]).max() > 0          # the waves reach the receiver well
    assert rel_l2(m.to_complex(seis), ref) <= RTOL
