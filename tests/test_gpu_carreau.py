"""GPU parity of the Carreau-Yasuda relaxation (Eq. carreauTau in full) against the FP64
oracle on the same seeded inputs.

Binary64: foams with Carreau-Yasuda liquid (2D, 3D, 3D under gravity) with cell types and
labels bit-exact, populations within 1e-12 of max|f|, bubbles and ledgers within 1e-12.
Binary32 and 16-bit storage: random closed-box Carreau-Yasuda flow within n times the
storage form's rounding bound of the oracle after n steps (bulk and near-wall kernels).
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from synth import place_nuclei, small_case
from synth.workloads import _mk
from tests.parity_util import compare_bubbles, compare_states

pytestmark = pytest.mark.gpu

CY = dict(rheology="carreau_yasuda", cy_tau0=1.2, cy_tau_inf=0.6, cy_lambda=1000.0, cy_a=2.0, cy_n=0.4)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(wl):
    from paper_1908_04262_amd import Sim
    return Sim(wl)


@pytest.mark.parametrize("case,extra,steps,chunk", [
    ("foam2d", {}, 120, 40),
    ("c3_small", {}, 30, 10),
    ("c3_small", {"accel": (0.0, 0.0, -3e-5)}, 30, 10),
])
def test_carreau_fp64_parity(case, extra, steps, chunk):
    wl = small_case(case, precision="fp64", **CY, **extra)
    _say(f"fp64 Carreau-Yasuda parity {case} {extra}: nucleate")
    orc = Oracle(wl)
    gpu = _sim(wl)
    c, r, p0 = place_nuclei(wl)
    orc.nucleate(c, r, p0)
    gpu.nucleate(c, r, p0)
    done = 0
    out = None
    while done < steps:
        _say(f"fp64 Carreau-Yasuda parity {case}: steps {done}..{done + chunk}")
        gpu.step(chunk)
        orc.step(chunk)
        done += chunk
        out = compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-10)
        compare_bubbles(gpu, orc, 1e-12)
    _say(f"fp64 Carreau-Yasuda parity {case}: {out}")


_STORE_EPS = {"fp32": 2.0 ** -17, "f16s": 2.0 ** -11, "bf16s": 2.0 ** -8, "f16s_g16": 2.0 ** -11}


@pytest.mark.parametrize("prec", ["fp32", "f16s", "bf16s", "f16s_g16"])
def test_carreau_closed_box_flow_matches_oracle(prec):
    """Random populations in a closed box (rows of 72 cells: bulk and near-wall kernels)
    with Carreau-Yasuda relaxation; shear rates of the perturbation put lambda gdot near 1,
    where the relaxation time moves most."""
    nsteps = 5
    wl = _mk(name="box", dim=3, nx=72, ny=20, nz=18, gas_from=-1, nuclei=None, S0=1.3,
             precision=prec, **CY)
    orc = Oracle(dict(wl, precision="fp64"))
    gpu = _sim(wl)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    wg = np.array([0.25] + [0.125] * 6)
    c0 = 1.3 * 5e-3 / 3.0
    rng = np.random.default_rng(14)
    shape = orc.shape
    f = w[:, None, None, None] * (1.0 + 3e-3 * rng.uniform(-1, 1, (19,) + shape))
    g = (wg * c0)[:, None, None, None] * (1.0 + 1e-2 * rng.uniform(-1, 1, (7,) + shape))
    for o in (orc, gpu):
        o.write("f", f)
        o.write("g", g)
    m = orc.read("type") == 2
    sf = np.abs(f[:, m] - w[:, None]).max()
    orc.step(nsteps)
    gpu.step(nsteps)
    ef = np.abs(gpu.read("f")[:, m] - orc.read("f")[:, m]).max() / sf
    tol = nsteps * _STORE_EPS[prec]
    _say(f"closed box Carreau-Yasuda {prec}: deviation / initial perturbation {ef:.2e} (bound {tol:.2e})")
    assert ef < tol, (ef, tol)
