"""Workloads at their full sizes, checked through properties that hold at any size:

* the benchmark workload (384^3 power-law foam, 2000 nuclei, seed 3) in the launch
  configuration bench.py times (binary16 f and g with the learned curvature; binary32 with
  the plain fit), 40 steps;
* the 128^3 binary32 foam with 32 nuclei and disjoining pressure, its full 5000 steps;
* the 256^3 foam with 500 nuclei and the learned curvature (binary32), 1000 steps.

The properties:

* liquid mass (populations of liquid cells plus M of interface cells, plus the lost-liquid
  ledger) conserved to 1e-6 relative (1e-5 over the runs of 1000 steps and more);
* the ideal-gas law p = m RT / max(V, 1/2) on every bubble (binary64 table, 1e-12);
* every bubble's volume equal to the sum over its cells of 1 - alpha (gas cells 1), summed
  on the host from the label and fill-fraction fields read back (1e-6 relative);
* the connected components of the gas and interface cells (lattice neighbourhood, from
  scipy.ndimage) carry one bubble id each, and distinct components distinct ids (the
  atmosphere aside).
"""
import sys

import numpy as np
import pytest
from scipy import ndimage

from synth import place_nuclei, workload

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _liquid(sim):
    T = sim.read("type")
    f = sim.read("f")
    rho_l = f.sum(axis=0)[T == 2].sum()
    del f
    M = sim.read("mass")
    return rho_l + M[T == 1].sum() + sim.ledgers()["lost_liquid"]


@pytest.mark.parametrize("name,prec,curv,steps,min_bubbles", [
    ("c3_foam_384", "f16s_g16", "mlp", 40, 1500),
    ("c3_foam_384", "fp32", "plain", 40, 1500),
    ("c2_3d_128", "fp32", "plain", 5000, 1),
    ("c4_foam_256", "fp32", "mlp", 1000, 100),
])
def test_full_size_foam_properties(name, prec, curv, steps, min_bubbles):
    from paper_1908_04262_amd import CurvatureNet, Sim
    wl = workload(name, precision=prec, curvature=curv)
    _say(f"full size {name} {prec}/{curv}: create and nucleate")
    sim = Sim(wl)
    if curv == "mlp":
        net = CurvatureNet(5)
        net.train(n_train=65536, n_val=4096, epochs=1, batch=2048, lr=2e-3, data_seed=6)
        sim.attach_mlp(net)
    sim.nucleate(*place_nuclei(wl))
    m0 = _liquid(sim)
    _say(f"full size {name} {prec}/{curv}: {steps} steps")
    sim.step(steps)
    sim.sync()
    m1 = _liquid(sim)
    assert abs(m1 - m0) / m0 < (1e-6 if steps < 1000 else 1e-5), (m0, m1)

    b = sim.bubbles()
    ids, V, m, p = b["id"], b["V"], b["m"], b["p"]
    live = ids > 0
    assert live.sum() >= min_bubbles
    RT = wl["RT"]
    want_p = m[live] * RT / np.maximum(V[live], 0.5)
    assert np.allclose(p[live], want_p, rtol=1e-12, atol=0)

    _say(f"full size {name} {prec}/{curv}: volumes and components from the fields")
    T = sim.read("type")
    lab = sim.read("label")
    al = sim.read("alpha")
    bub = (T == 0) | (T == 1)
    share = np.where(T == 0, 1.0, 1.0 - al)
    sel = bub & (lab > 0)
    vsum = np.bincount(lab[sel].ravel(), weights=share[sel].ravel(), minlength=int(ids.max()) + 1)
    got = vsum[ids[live]]
    assert np.allclose(got, V[live], rtol=1e-6, atol=1e-9), np.abs(got / V[live] - 1).max()

    comp, nc = ndimage.label(bub, structure=ndimage.generate_binary_structure(3, 2))
    idx = np.arange(1, nc + 1)
    lo = np.asarray(ndimage.minimum(lab, labels=comp, index=idx))
    hi = np.asarray(ndimage.maximum(lab, labels=comp, index=idx))
    assert np.array_equal(lo, hi), "a component carries more than one bubble id"
    ids_of = lo.astype(np.int64)
    bubbles_only = ids_of[ids_of > 0]
    assert len(np.unique(bubbles_only)) == len(bubbles_only), "two components share a bubble id"
    assert set(bubbles_only.tolist()) == set(ids[live].tolist())
    npi = int(np.count_nonzero(sim.read("pi"))) if wl.get("k_pi", 0.0) > 0.0 else 0
    _say(f"full size {name} {prec}/{curv}: {nc} components, {live.sum()} bubbles, "
         f"mass drift {abs(m1 - m0) / m0:.2e}, {npi} cells with disjoining pressure")
    sim.close()
