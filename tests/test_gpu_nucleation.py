"""Nucleation from a probability field (Sec. 3.4) end to end on the GPU: sites from the
library's Poisson-disk sampler, nucleated in the library and in the FP64 oracle, stepped and
compared (cell types and labels bit-exact, populations within 1e-12, bubbles within 1e-12)."""
import sys

import numpy as np
import pytest

from oracle import Oracle
from synth.workloads import _mk
from tests.parity_util import compare_bubbles, compare_states

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dim", [2, 3])
def test_field_nucleation_fp64_parity(dim):
    from paper_1908_04262_amd import Sim, poisson_nuclei
    if dim == 2:
        wl = _mk(name="fieldnuc", dim=2, nx=96, ny=72, nz=1, precision="fp64", tau=0.8, sigma=1e-3, S0=2.0,
                 nuclei=None)
        shape = (1, 72, 96)
    else:
        wl = _mk(name="fieldnuc", dim=3, nx=56, ny=40, nz=44, precision="fp64", tau=0.7, sigma=5e-4, S0=1.5,
                 nuclei=None)
        shape = (44, 40, 56)
    # a nucleation field rising along x
    P = np.broadcast_to(np.linspace(0.1, 1.0, shape[2], dtype=np.float32), shape).copy()
    c, r = poisson_nuclei(wl, P, 40, 2.0, 4.0, 1.0, 30, 17)
    assert len(r) > 3
    p0 = wl["p_atm"] + (2.0 if dim == 3 else 1.0) * wl["sigma"] / r
    _say(f"field nucleation {dim}D: {len(r)} nuclei")
    orc = Oracle(wl)
    gpu = Sim(wl)
    orc.nucleate(c, r, p0)
    gpu.nucleate(c, r, p0)
    compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-12, tol_geom=1e-10)
    compare_bubbles(gpu, orc, 1e-12)
    for k in range(2):
        orc.step(10)
        gpu.step(10)
        out = compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-10)
        compare_bubbles(gpu, orc, 1e-12)
    _say(f"field nucleation {dim}D: {out}")
