"""GPU tests of the boundary calls beyond the time step itself: checkpoints, the totals
and bubble statistics computed on the device, fault injection and the device status
word, the paper-literal gas flux (Sec. 3.2, Eq. gascurrent) against the oracle, and
network files.
"""
import math
import os
import sys
import tempfile

import numpy as np
import pytest

from oracle import Oracle
from synth import place_nuclei, small_case
from tests.parity_util import compare_bubbles, compare_states

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(wl):
    from paper_1908_04262_amd import Sim
    return Sim(wl)


_FIELDS = ("type", "label", "f", "g", "mass", "alpha", "rho", "kappa", "pi", "ux", "uy", "uz")


def _same_state(a, b):
    for name in _FIELDS:
        x, y = a.read(name), b.read(name)
        assert np.array_equal(x, y), (name, np.abs(x.astype(float) - y.astype(float)).max())
    ba, bb = a.bubbles(), b.bubbles()
    for k in ba:
        assert np.array_equal(ba[k], bb[k]), k
    la, lb = a.ledgers(), b.ledgers()
    for k in la:
        assert la[k] == lb[k], (k, la[k], lb[k])


@pytest.mark.parametrize("case,prec,first,second", [
    ("c2_small", "fp64", 500, 500),
    ("c3_small", "f16s_g16", 150, 150),
])
def test_checkpoint_continues_bit_for_bit(case, prec, first, second):
    """first steps + save + load into a fresh context + second steps equals first + second
    steps in one context, bit for bit in every field, the bubble table and the ledgers
    (binary64 on config-2 physics, and binary16 storage with the learned curvature, whose
    network weights travel in the checkpoint)."""
    from paper_1908_04262_amd import CurvatureNet
    mlp = prec == "f16s_g16"
    wl = small_case(case, precision=prec, curvature="mlp" if mlp else "plain")
    net = CurvatureNet(9) if mlp else None
    ref = _sim(wl)
    run = _sim(wl)
    for s in (ref, run):
        if mlp:
            s.attach_mlp(net)
        s.nucleate(*place_nuclei(wl))
    _say(f"checkpoint {case} {prec}: {first} + save/load + {second}")
    ref.step(first + second)
    run.step(first)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "state.ckpt")
        run.save(path)
        run.close()
        fresh = _sim(wl)
        fresh.load(path)
    fresh.step(second)
    assert fresh.ledgers()["step"] == first + second
    _same_state(ref, fresh)


def test_checkpoint_rejects_other_parameters():
    from paper_1908_04262_amd import MifoamError
    wl = small_case("c2_small")
    a = _sim(wl)
    a.nucleate(*place_nuclei(wl))
    b = _sim(dict(wl, tau=0.75))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "state.ckpt")
        a.save(path)
        with pytest.raises(MifoamError, match="MF_EINVAL.*other parameters"):
            b.load(path)
        with open(os.path.join(d, "junk"), "wb") as fp:
            fp.write(b"not a checkpoint")
        with pytest.raises(MifoamError, match="MF_EINVAL"):
            a.load(os.path.join(d, "junk"))


@pytest.mark.parametrize("case,prec,tol", [("c2_small", "fp64", 1e-12), ("c3_small", "fp32", 1e-5)])
def test_device_totals_and_bubble_statistics(case, prec, tol):
    """The liquid mass, dissolved gas and bubble gas summed by the library equal the FP64
    oracle's (binary64: 1e-12; binary32 after 30 steps: 1e-5), and the cell count
    and gas-volume centroid of every bubble equal what the GPU's own fields give."""
    wl = small_case(case, precision=prec)
    gpu = _sim(wl)
    orc = Oracle(small_case(case, precision="fp64"))
    c, r, p0 = place_nuclei(wl)
    gpu.nucleate(c, r, p0)
    orc.nucleate(c, r, p0)
    for k in range(3):
        gpu.step(10)
        orc.step(10)
        tg, to = gpu.totals(), orc.totals()
        for key in ("liquid", "dissolved", "bubble_gas"):
            assert abs(tg[key] - to[key]) <= tol * abs(to[key]), (key, tg[key], to[key])
        T, lab, al = gpu.read("type"), gpu.read("label"), gpu.read("alpha")
        b = gpu.bubbles()
        zz, yy, xx = np.mgrid[0:T.shape[0], 0:T.shape[1], 0:T.shape[2]]
        for i, bid in enumerate(b["id"]):
            on = ((T == 0) | (T == 1)) & (lab == bid)
            assert b["n_cells"][i] == int(on.sum())
            w = np.where(T == 0, 1.0, 1.0 - al)[on]
            want = np.array([(w * xx[on]).sum(), (w * yy[on]).sum(), (w * zz[on]).sum()]) / w.sum()
            assert np.abs(b["centroid"][i] - want).max() < 1e-9, (bid, b["centroid"][i], want)
            assert abs(w.sum() - b["V"][i]) <= 1e-9 * b["V"][i] + (1e-5 if prec != "fp64" else 0.0)
    _say(f"totals {case} {prec}: {tg['liquid']:.6f} {tg['dissolved']:.6f} {tg['bubble_gas']:.6f}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "f16s_g16"])
def test_non_finite_population_is_reported(prec):
    """Fault injection from the host: a NaN written into one population of a liquid cell
    deep in the liquid (far from every interface, so nothing but that cell's neighbour
    reads it within one step) makes the next collision raise the non-finite-density bit
    of the status word; mf_sync reports MF_ENUMERIC and leaves the state readable."""
    from paper_1908_04262_amd import MifoamError
    wl = small_case("c2_small", precision=prec)
    gpu = _sim(wl)
    gpu.nucleate(*place_nuclei(wl))
    gpu.step(3)
    gpu.sync()
    T = gpu.read("type")
    nz, ny, nx = T.shape
    # a liquid cell whose 7^3 neighbourhood is all liquid
    from scipy.ndimage import minimum_filter
    deep = minimum_filter((T == 2).astype(np.uint8), size=7, mode="constant", cval=0) == 1
    z, y, x = np.argwhere(deep)[0]
    cell = int(x + nx * (y + ny * z))
    _say(f"poke NaN {prec} at cell {(x, y, z)}")
    gpu.poke("f", cell, 1, float("nan"))
    gpu.step(1)
    with pytest.raises(MifoamError, match="MF_ENUMERIC.*non-finite"):
        gpu.sync()
    assert gpu.ledgers()["status"] != 0
    with pytest.raises(MifoamError, match="MF_EINVAL"):
        gpu.poke("f", gpu.N, 0, 1.0)
    with pytest.raises(MifoamError, match="MF_EINVAL"):
        gpu.poke("f", cell, 19, 1.0)
    with pytest.raises(MifoamError, match="MF_EINVAL"):
        gpu.poke("label", cell, 0, 1.0)
    gpu.close()


@pytest.mark.parametrize("case,steps,chunk", [("c2_small", 60, 20), ("foam2d", 120, 40), ("neck3d", 30, 5)])
def test_paper_flux_mode_matches_oracle(case, steps, chunk):
    """The gas flux of Eq. gascurrent as printed, in binary64 against the oracle in the same
    mode: types and labels bit-exact, populations 1e-12, bubbles and ledgers 1e-12. The
    difference from the ledger mode is reported."""
    wl = small_case(case, precision="fp64", flux_mode="paper")
    gpu = _sim(wl)
    orc = Oracle(wl)
    led = _sim(dict(wl, flux_mode="ledger"))
    c, r, p0 = place_nuclei(wl)
    for s in (gpu, orc, led):
        s.nucleate(c, r, p0)
    done = 0
    while done < steps:
        gpu.step(chunk)
        orc.step(chunk)
        led.step(chunk)
        done += chunk
        compare_states(gpu, orc, tol_pop=1e-12, tol_cell=1e-10)
        compare_bubbles(gpu, orc, 1e-12)
    tp, tl = gpu.totals(), led.totals()
    gp = tp["dissolved"] + tp["bubble_gas"] + tp["atm_gas"] + tp["collapsed_gas"]
    gl = tl["dissolved"] + tl["bubble_gas"] + tl["atm_gas"] + tl["collapsed_gas"]
    _say(f"paper flux {case}: bubble gas {tp['bubble_gas']:.6e} (ledger {tl['bubble_gas']:.6e}), "
         f"total gas {gp:.6e} (ledger {gl:.6e}, relative drift of the printed form {(gp - gl) / gl:+.2e})")


def test_network_file_round_trip():
    from paper_1908_04262_amd import CurvatureNet, generate_stencils
    net = CurvatureNet(13)
    rng = np.random.default_rng(2)
    net.set_params(net.params() + rng.normal(size=net.nparam).astype(np.float32) * 0.01)
    X, _ = generate_stencils(3, 0, 256)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        net.save(path)
        back = CurvatureNet.load(path)
    assert np.array_equal(back.params()[:125 * 64], net.params()[:125 * 64])
    assert np.array_equal(back.params()[128 * 64:], net.params()[128 * 64:])
    assert np.array_equal(back.eval(X), net.eval(X))
