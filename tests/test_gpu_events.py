"""GPU parity on the paths that only some states reach: disjoining pressure on thin
lamellae (Sec. 3.3, Eq. rhobplusdisjoining, Appendix A Algorithm 1), bubble merge,
split, burst into the headspace and collapse (Sec. 3.5), a 1000-step 3D run, and the
partial relabelling of a time step against a full relabelling of the same state.

Binary64 throughout, through the C ABI, against the FP64 oracle on the same nuclei:
cell types and bubble labels bit-exact and the bubble table and ledgers within 1e-12
after every step of the topology cases; populations within 1e-12 of max|f|, cell fields
within 1e-10 (curvature and disjoining pressure included) at every full comparison.
Each case also asserts that the oracle run really contains the events it is there for,
so that a change of the recipe cannot silently turn it into a run without them.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from synth import place_nuclei, small_case
from tests.parity_util import compare_bubbles, compare_states

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(wl):
    from paper_1908_04262_amd import Sim
    orc = Oracle(wl)
    gpu = Sim(wl)
    c, r, p0 = place_nuclei(wl)
    orc.nucleate(c, r, p0)
    gpu.nucleate(c, r, p0)
    return gpu, orc


def _cheap_compare(gpu, orc, tol):
    """types and labels bit-exact, bubble table and ledgers within tol"""
    Tg, To = gpu.read("type"), orc.read("type")
    nt = int((Tg != To).sum())
    assert nt == 0, f"{nt} cell types differ"
    nl = int((gpu.read("label") != orc.read("label")).sum())
    assert nl == 0, f"{nl} bubble labels differ"
    compare_bubbles(gpu, orc, tol)


@pytest.mark.parametrize("d_max,min_cells", [(2.0, 20), (3.0, 120)])
def test_disjoining_pressure_on_lamellae(d_max, min_cells):
    """Nine bubbles two cells apart: the films between them carry a disjoining pressure.
    The set of interface cells with Pi != 0 must be the oracle's exactly, and Pi itself
    within 1e-10 of max|Pi|, every 10 steps for 100 steps."""
    wl = small_case("lamella3d", d_max=d_max)
    _say(f"lamellae d_max={d_max}: nucleate")
    gpu, orc = _pair(wl)
    total = 0
    for k in range(11):
        if k:
            gpu.step(10)
            orc.step(10)
        _say(f"lamellae d_max={d_max}: step {10 * k}")
        out = compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-10)
        compare_bubbles(gpu, orc, 1e-12)
        T = orc.read("type")
        pg, po = gpu.read("pi"), orc.read("pi")
        on_o = (T == 1) & (po != 0.0)
        on_g = (T == 1) & (pg != 0.0)
        assert np.array_equal(on_o, on_g), int((on_o != on_g).sum())
        n = int(on_o.sum())
        assert n >= min_cells, f"only {n} interface cells carry a disjoining pressure"
        assert (po[on_o] > 0.0).all() and po.max() <= 5e-3 * d_max
        total += n
        _say(f"  {n} cells with Pi != 0, max {po.max():.3e}, diff {out['pi']:.2e}")
    _say(f"lamellae d_max={d_max}: {total} cell-snapshots with Pi != 0")


def _events(orc, prev):
    b = orc.bubbles()
    led = orc.ledgers()
    ids = tuple(int(i) for i in b["id"])
    ev = []
    if prev is not None:
        pids, pnext, patm, pcoll = prev
        if led["next_id"] > pnext:
            ev.append("split")
        gone = set(pids) - set(ids)
        if gone and led["collapsed_gas"] > pcoll:
            ev.append("collapse")
        elif gone and len(ids) < len(pids) and led["next_id"] == pnext:
            ev.append("merge_or_burst")
    return ev, (ids, led["next_id"], led["atm_gas"], led["collapsed_gas"])


@pytest.mark.parametrize("case,full_every,expect", [
    ("neck3d", 5, {"merge_or_burst": 2, "split": 1}),
    ("burst3d", 10, {"merge_or_burst": 2}),
    ("dissolve3d", 20, {"collapse": 3}),
])
def test_topology_events_3d(case, full_every, expect):
    """Merge, split, burst and collapse in 3D. After every step: types and labels
    bit-exact, bubbles and ledgers within 1e-12; every full_every steps: populations
    and cell fields too."""
    wl = small_case(case)
    steps = wl["steps"]
    _say(f"{case}: nucleate, {steps} steps")
    gpu, orc = _pair(wl)
    _, prev = _events(orc, None)
    seen = {}
    atm_jump = 0.0
    for k in range(1, steps + 1):
        gpu.step(1)
        orc.step(1)
        ev, cur = _events(orc, prev)
        for e in ev:
            seen[e] = seen.get(e, 0) + 1
            _say(f"{case}: step {k}: {e}, ids {cur[0]}")
        if "merge_or_burst" in ev:
            atm_jump = max(atm_jump, cur[2] - prev[2])
        prev = cur
        _cheap_compare(gpu, orc, 1e-12)
        if k % full_every == 0 or ev:
            compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-10)
    for e, n in expect.items():
        assert seen.get(e, 0) >= n, (case, seen)
    if case == "burst3d":
        # the bubble that reaches the headspace hands its gas to the atmosphere
        assert atm_jump > 1.0, atm_jump
    if case == "dissolve3d":
        assert orc.bubbles()["id"].size == 0
    _say(f"{case}: events {seen}")


@pytest.mark.timeout(900)
def test_fp64_parity_3d_1000_steps():
    """Config-2 physics (disjoining pressure on) on the 70x40x36 grid for 1000 steps; the
    run contains a burst into the headspace near step 580."""
    wl = small_case("c2_small", precision="fp64")
    _say("c2_small fp64, 1000 steps")
    gpu, orc = _pair(wl)
    n0 = len(orc.bubbles()["id"])
    for k in range(10):
        gpu.step(100)
        orc.step(100)
        out = compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-10)
        compare_bubbles(gpu, orc, 1e-12)
        _say(f"  step {100 * (k + 1)}: f {out['f']:.2e} kappa {out['kappa']:.2e} pi {out['pi']:.2e}")
    assert len(orc.bubbles()["id"]) < n0


@pytest.mark.parametrize("case,prec,steps,every", [
    ("neck3d", "fp64", 30, 3),
    ("burst3d", "fp64", 90, 15),
    ("dissolve3d", "fp64", 150, 25),
    ("neck3d", "f16s_g16", 30, 3),
    ("burst3d", "f16s_g16", 90, 15),
])
def test_partial_relabelling_equals_full(case, prec, steps, every):
    """A time step relabels only the components its conversions may have changed (the ids
    the topology test marks) and updates every other bubble on the fast path. The state it
    leaves must be the one a full relabelling of the same cells gives: at every checkpoint
    the run is relabelled from scratch (mf_refresh with relabel, which lists every gas and
    interface cell and applies no flux), and the bubble ids of every cell and the bubble
    table (volume, gas, pressure, alive flags) must come out unchanged, bit for bit."""
    from paper_1908_04262_amd import Sim
    wl = small_case(case, precision=prec)
    sim = Sim(wl)
    sim.nucleate(*place_nuclei(wl))
    done, events = 0, 0
    ids_before = None
    while done < steps:
        sim.step(every)
        done += every
        lab = sim.read("label")
        b = sim.bubbles()
        led = sim.ledgers()
        ids = set(b["id"].tolist())
        if ids_before is not None and ids != ids_before:
            events += 1
        ids_before = ids
        sim.refresh(relabel=True)
        assert np.array_equal(sim.read("label"), lab), f"{case} step {done}: ids differ"
        b2 = sim.bubbles()
        for k in ("id", "V", "m", "p"):
            assert np.array_equal(b[k], b2[k]), (case, done, k)
        led2 = sim.ledgers()
        for k in ("n_bubbles", "next_id", "atm_gas", "collapsed_gas", "lost_liquid"):
            assert led2[k] == led[k], (case, done, k, led[k], led2[k])
        assert led2["status"] == 0
    _say(f"partial relabelling {case} {prec}: {steps} steps, bubble set changed between "
         f"{events} of {steps // every - 1} checkpoints")
    assert events >= 1, "the run has no topology event"
    sim.close()
