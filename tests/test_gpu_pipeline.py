"""The overlapped step pipeline (labelling, normals and curvature of a step on two more
streams beside the next step's bulk sweep) gives the same state, bit for bit, however the
steps are issued: in one mf_step call, one step per call (every call joins the streams), and
with the profiling events on. Binary16 storage with the learned curvature (the stencil words
come from the excess pass then) and binary64 with the plain fit; both with topology changes
(foam with coalescence)."""
import sys

import numpy as np
import pytest

from synth import place_nuclei, small_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def net():
    from paper_1908_04262_amd import CurvatureNet
    n = CurvatureNet(5)
    n.train(n_train=16384, n_val=2048, epochs=1, batch=2048, lr=2e-3, data_seed=6)
    return n


def _state(sim):
    return {k: sim.read(k) for k in ("type", "label", "f", "g", "mass", "alpha", "kappa")}, sim.bubbles()


@pytest.mark.parametrize("prec,curv", [("f16s_g16", "mlp"), ("fp64", "plain")])
def test_issue_pattern_does_not_change_results(net, prec, curv):
    from paper_1908_04262_amd import Sim
    wl = small_case("c3_small", precision=prec, curvature=curv, S0=3.0)
    runs = []
    for mode in ("one_call", "per_step", "profiled"):
        _say(f"pipeline {prec}/{curv}: {mode}")
        sim = Sim(wl)
        if curv == "mlp":
            sim.attach_mlp(net)
        sim.nucleate(*place_nuclei(wl))
        if mode == "one_call":
            sim.step(24)
        elif mode == "per_step":
            for _ in range(24):
                sim.step(1)
        else:
            sim.profile(True)
            sim.step(24)
            ms, n = sim.profile_get(1)
            assert n == 24 and ms > 0
            sim.profile(False)
        sim.sync()
        runs.append(_state(sim))
        sim.close()
    (a, ba), rest = runs[0], runs[1:]
    for b, bb in rest:
        for k in a:
            assert np.array_equal(a[k], b[k]), k
        for k in ba:
            assert np.array_equal(ba[k], bb[k]), k
