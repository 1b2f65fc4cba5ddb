"""GPU parity of the body-force term (Eq. collision, external force; Guo-Zheng-Shi form)
against the FP64 oracle on the same seeded inputs.

Binary64: foams under gravity (2D, 3D Newtonian, 3D power law) with cell types and labels
bit-exact and populations within 1e-12 of max|f|, bubbles and ledgers within 1e-12; a
periodic box under uniform acceleration bit-identical to the oracle. Binary32 and 16-bit
storage: random closed-box power-law flow under a body force (bulk and near-wall
kernels) within n times the storage form's rounding bound of the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from synth import place_nuclei, small_case
from synth.workloads import _mk
from tests.parity_util import compare_bubbles, compare_states

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(wl):
    from paper_1908_04262_amd import Sim
    return Sim(wl)


@pytest.mark.parametrize("case,accel,steps,chunk", [
    ("foam2d", (0.0, -2e-5, 0.0), 120, 40),
    ("c2_small", (1e-5, 0.0, -3e-5), 30, 10),
    ("c3_small", (0.0, 1e-5, -2e-5), 30, 10),
])
def test_force_fp64_parity(case, accel, steps, chunk):
    wl = small_case(case, precision="fp64", accel=accel)
    _say(f"fp64 force parity {case} a={accel}: nucleate")
    orc = Oracle(wl)
    gpu = _sim(wl)
    c, r, p0 = place_nuclei(wl)
    orc.nucleate(c, r, p0)
    gpu.nucleate(c, r, p0)
    done = 0
    out = None
    while done < steps:
        _say(f"fp64 force parity {case}: steps {done}..{done + chunk}")
        gpu.step(chunk)
        orc.step(chunk)
        done += chunk
        out = compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-10)
        compare_bubbles(gpu, orc, 1e-12)
    _say(f"fp64 force parity {case}: {out}")


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_acceleration_box_fp64_identical(dim):
    a = (2e-5, -1e-5, 3e-5 if dim == 3 else 0.0)
    wl = _mk(name="accel", dim=dim, nx=10, ny=7, nz=6 if dim == 3 else 1, gas_from=-1, nuclei=None,
             tau=0.8, periodic=[1, 1, 1], S0=0.5, accel=a)
    orc = Oracle(wl)
    gpu = _sim(wl)
    _say(f"uniform acceleration box {dim}D fp64")
    orc.step(60)
    gpu.step(60)
    compare_states(gpu, orc, tol_pop=0.0, tol_cell=0.0)
    f = gpu.read("f")
    e = np.array(orc.lattice()[0], float)
    j = np.tensordot(e.T, f, axes=(1, 0))
    for k in range(3):
        assert abs(j[k].mean() - 60 * a[k]) <= 1e-12 + 1e-10 * abs(60 * a[k])


_STORE_EPS = {"fp32": 2.0 ** -17, "f16s": 2.0 ** -11, "bf16s": 2.0 ** -8, "f16s_g16": 2.0 ** -11}


@pytest.mark.parametrize("prec", ["fp32", "f16s", "bf16s", "f16s_g16"])
def test_force_closed_box_flow_matches_oracle(prec):
    """Random populations in a closed box with power-law relaxation and a body force;
    rows of 72 cells put every cell through the bulk kernel or the near-wall kernel."""
    nsteps = 5
    a = (3e-4, -2e-4, 1e-4)
    wl = _mk(name="box", dim=3, nx=72, ny=20, nz=18, gas_from=-1, nuclei=None, S0=1.3,
             rheology="power_law", pl_n=0.6, tau=0.8, precision=prec, accel=a)
    orc = Oracle(dict(wl, precision="fp64"))
    gpu = _sim(wl)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    wg = np.array([0.25] + [0.125] * 6)
    c0 = 1.3 * 5e-3 / 3.0
    rng = np.random.default_rng(13)
    shape = orc.shape
    f = w[:, None, None, None] * (1.0 + 3e-3 * rng.uniform(-1, 1, (19,) + shape))
    g = (wg * c0)[:, None, None, None] * (1.0 + 1e-2 * rng.uniform(-1, 1, (7,) + shape))
    for o in (orc, gpu):
        o.write("f", f)
        o.write("g", g)
    m = orc.read("type") == 2
    f0 = orc.read("f")
    orc.step(nsteps)
    gpu.step(nsteps)
    fo, fg = orc.read("f"), gpu.read("f")
    # scale: the change the steps made (perturbation and force together)
    sf = np.abs(fo[:, m] - f0[:, m]).max()
    ef = np.abs(fg[:, m] - fo[:, m]).max() / sf
    tol = nsteps * _STORE_EPS[prec]
    _say(f"closed box with force {prec}: deviation / change {ef:.2e} (bound {tol:.2e})")
    assert ef < tol, (ef, tol)
