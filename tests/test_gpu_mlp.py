"""GPU tests of the learned curvature closure against the FP64 reference (oracle/mlp.py).

* the GPU stencil generator reproduces the reference generator (same counter-based
  stream): fill fractions within one sub-sample (1e-3 plus noise rounding), labels 1e-9;
* the MFMA forward pass matches the reference forward (same bfloat16 roundings) to 1e-3;
* the GPU gradient matches the reference backward: relative L2 <= 2e-2, cosine >= 0.999;
* a short training run lowers the validation error, and the trained network has a
  smaller curvature error than the plain paraboloid fit on held-out stencils (seed 44);
* inside the time step, the network curvature of each interface cell matches the
  reference forward on the stencil read back from the GPU state.
"""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from oracle import mlp as M
from synth import place_nuclei, small_case
from synth.workloads import _mk

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_generator_matches_reference():
    from paper_1908_04262_amd import generate_stencils
    _say("generator")
    Xg, Kg = generate_stencils(44, 10, 48)
    Xo, Ko = M.generate(44, 10, 48)
    assert np.abs(Kg - Ko).max() <= 1e-6 * np.abs(Ko).max() + 1e-9
    assert np.abs(Xg - Xo).max() <= 2e-3


def test_forward_matches_reference():
    from paper_1908_04262_amd import CurvatureNet, generate_stencils
    _say("forward")
    net = CurvatureNet(3)
    rng = np.random.default_rng(1)
    theta = M.init_params(5) * 3.0 + rng.normal(size=M.NPARAM) * 0.05
    theta[M.NFEAT * M.H:M.NPAD * M.H] = 0.0
    net.set_params(theta.astype(np.float32))
    th32 = net.params().astype(np.float64)
    X, _ = generate_stencils(7, 0, 200)
    kg = net.eval(X)
    out, _ = M.forward(th32, M.canonicalise(X.astype(np.float64)))
    ko = out / 8
    assert np.abs(kg - ko).max() <= 1e-3 * np.abs(ko).max() + 1e-4


def test_gradient_matches_reference():
    from paper_1908_04262_amd import CurvatureNet, generate_stencils
    _say("gradient")
    net = CurvatureNet(3)
    th32 = net.params().astype(np.float64)
    X, K = generate_stencils(9, 0, 256)
    loss_g, gg = net.grad(X, 8 * K)
    loss_o, go = M.loss_and_grad(th32, M.canonicalise(X.astype(np.float64)), 8 * K.astype(np.float64))
    assert abs(loss_g / loss_o - 1) < 1e-3
    sl = [(0, M.NPAD * M.H), (M.NPAD * M.H, M.NPAD * M.H + M.H),
          (M.NPAD * M.H + M.H, M.NPAD * M.H + M.H + M.H * M.H)]
    for a, b in sl + [(b0, M.NPARAM) for b0 in [M.NPARAM - M.H - 1]]:
        x, y = gg[a:b].astype(np.float64), go[a:b]
        rel = np.linalg.norm(x - y) / np.linalg.norm(y)
        cos = x @ y / (np.linalg.norm(x) * np.linalg.norm(y))
        assert rel <= 2e-2 and cos >= 0.999, (a, b, rel, cos)


def _plain_kappa(stencils):
    """the plain paraboloid fit of the oracle on 5x5x5 stencils (periodic 9^3 box)"""
    wl = _mk(name="st", dim=3, nx=9, ny=9, nz=9, gas_from=-1, periodic=[1, 1, 1], nuclei=None)
    o = Oracle(wl)
    out = []
    for s in stencils:
        a = np.ones((9, 9, 9))
        a[2:7, 2:7, 2:7] = np.asarray(s, dtype=np.float64).reshape(5, 5, 5)
        T = np.where(a <= 0.0, 0, np.where(a >= 1.0, 2, 1)).astype(np.uint8)
        o.write("type", T)
        o.write("alpha", a)
        out.append(o.curvature(o.cell(4, 4, 4)))
    return np.array(out)


def test_training_gain_over_plain_fit():
    from paper_1908_04262_amd import CurvatureNet, generate_stencils
    _say("training")
    net = CurvatureNet(7)
    rmse = net.train(n_train=131072, n_val=8192, epochs=4, batch=2048, lr=2e-3, data_seed=4)
    _say("val rmse", rmse)
    assert rmse < 0.03
    X, K = generate_stencils(44, 0, 400)
    km = net.eval(X)
    kp = _plain_kappa(X)
    e_mlp = math.sqrt(((km - K) ** 2).mean())
    e_plain = math.sqrt(((kp - K) ** 2).mean())
    _say("test rms: mlp", e_mlp, "plain", e_plain)
    assert e_mlp < e_plain


def _stencil_from_state(T, alpha, lab, x, y, z):
    """5x5x5 stencil of cell (x,y,z) with the rules of the step: walls and off-domain
    cells read the centre value, another bubble's gas/interface cell invalidates it"""
    nz, ny, nx = T.shape
    ac = min(1.0, max(0.0, alpha[z, y, x]))
    own = lab[z, y, x]
    out = np.empty(125)
    ok = True
    for j in range(125):
        dx, dy, dz = j % 5 - 2, (j // 5) % 5 - 2, j // 25 - 2
        X, Y, Z = x + dx, y + dy, z + dz
        if not (0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz) or T[Z, Y, X] == 3:
            out[j] = ac
            ok = False
            continue
        t = T[Z, Y, X]
        if t == 2:
            out[j] = 1.0
        else:
            if lab[Z, Y, X] != own:
                ok = False
            out[j] = 0.0 if t == 0 else min(1.0, max(0.0, alpha[Z, Y, X]))
    return out, ok


@pytest.fixture(scope="module")
def trained_net():
    from paper_1908_04262_amd import CurvatureNet
    _say("training a network for the in-step tests")
    net = CurvatureNet(7)
    net.train(n_train=65536, n_val=4096, epochs=2, batch=2048, lr=2e-3, data_seed=4)
    return net


def test_in_step_inference_matches_reference(trained_net):
    from paper_1908_04262_amd import Sim
    _say("in-step inference")
    net = trained_net
    th = net.params().astype(np.float64)
    wl = small_case("c2_small", precision="fp32", curvature="mlp", nx=64)
    sim = Sim(wl)
    sim.attach_mlp(net)
    sim.nucleate(*place_nuclei(wl))
    sim.step(5)
    T, al, lab, kap = sim.read("type"), sim.read("alpha"), sim.read("label"), sim.read("kappa")
    cells = np.argwhere(T == 1)
    St, idx = [], []
    for (z, y, x) in cells:
        s, ok = _stencil_from_state(T, al, lab, x, y, z)
        if ok:
            St.append(s)
            idx.append((z, y, x))
    assert len(St) > 100
    out, _ = M.forward(th, M.canonicalise(np.array(St)))
    ko = out / 8
    kg = np.array([kap[c] for c in idx])
    use = np.abs(ko) <= 0.49
    assert use.sum() > 100
    bad = np.flatnonzero(use & (np.abs(kg - ko) > 2e-3))
    for b in bad[:8]:
        z, y, x = idx[b]
        _say("mismatch", (x, y, z), "gpu", kg[b], "ref", ko[b], "label", lab[z, y, x],
             "alpha", al[z, y, x], "n", len(bad), "of", use.sum())
    assert np.abs(kg[use] - ko[use]).max() <= 2e-3


def _liquid(s):
    t = s.totals()
    return t["liquid"] + t["lost_liquid"]


@pytest.mark.parametrize("prec", ["f16s", "bf16s"])
def test_16bit_storage_with_learned_curvature(trained_net, prec):
    """16-bit offsets + learned curvature against the FP64 oracle with plain curvature:
    liquid mass within 1e-6 relative, bubble volumes within 1% while no topology change
    has happened (after one, trajectories may legitimately part)."""
    from paper_1908_04262_amd import Sim
    wl = small_case("c2_small", precision=prec, curvature="mlp")
    wl64 = small_case("c2_small", precision="fp64")
    _say(f"{prec} + mlp c2_small vs fp64 oracle")
    gpu = Sim(wl)
    gpu.attach_mlp(trained_net)
    orc = Oracle(wl64)
    c, r, p0 = place_nuclei(wl)
    gpu.nucleate(c, r, p0)
    orc.nucleate(c, r, p0)
    m0 = _liquid(gpu)
    compared = 0
    for k in range(4):
        gpu.step(10)
        orc.step(10)
        bg, bo = gpu.bubbles(), orc.bubbles()
        if list(bg["id"]) == list(bo["id"]) and orc.ledgers()["next_id"] == len(r) + 1:
            dv = np.abs(bg["V"] - bo["V"]) / bo["V"]
            _say(f"  step {10 * (k + 1)}: max volume deviation {dv.max():.2e}")
            assert dv.max() < 0.01, dv.max()
            compared += 1
        dm = abs(_liquid(gpu) - m0) / m0
        assert dm < 1e-6, dm
    assert compared >= 1


@pytest.mark.timeout(900)
def test_headline_form_against_fp64_oracle(trained_net):
    """The benchmark's production form, binary16 f and g (precision 4) with the learned
    curvature, against the FP64 oracle with the plain fit on config-2 physics: liquid mass
    within 1e-6 relative and every bubble volume within 1% for 500 steps (the oracle's
    first topology change comes later, near step 580)."""
    from paper_1908_04262_amd import Sim
    wl = small_case("c2_small", precision="f16s_g16", curvature="mlp")
    wl64 = small_case("c2_small", precision="fp64")
    _say("f16s_g16 + mlp c2_small vs fp64 oracle, 500 steps")
    gpu = Sim(wl)
    gpu.attach_mlp(trained_net)
    orc = Oracle(wl64)
    c, r, p0 = place_nuclei(wl)
    gpu.nucleate(c, r, p0)
    orc.nucleate(c, r, p0)
    m0 = _liquid(gpu)
    worst = 0.0
    for k in range(10):
        gpu.step(50)
        orc.step(50)
        bg, bo = gpu.bubbles(), orc.bubbles()
        assert orc.ledgers()["next_id"] == len(r) + 1 and len(bo["id"]) == len(r)
        assert list(bg["id"]) == list(bo["id"]), (bg["id"], bo["id"])
        dv = np.abs(bg["V"] - bo["V"]) / bo["V"]
        dm = abs(_liquid(gpu) - m0) / m0
        worst = max(worst, dv.max())
        _say(f"  step {50 * (k + 1)}: max volume deviation {dv.max():.2e}, mass drift {dm:.2e}")
        assert dv.max() < 0.01, dv.max()
        assert dm < 1e-6, dm
    _say(f"worst volume deviation over 500 steps {worst:.2e}")


@pytest.mark.timeout(900)
def test_config4_crop_fp32_learned_curvature(trained_net):
    """Config 4's foam (config-2 physics: tau 0.7, sigma 5e-4, supersaturation 1.5,
    disjoining pressure; radii U[3,5], separation 12) with binary32 storage and the learned
    curvature, on a 64^3 crop with the bubble density of the 256^3 run (8 bubbles), against
    the FP64 oracle with the plain fit: liquid mass within 1e-6 relative and every bubble
    volume within 0.5% for 300 steps while the oracle's bubble ids are unchanged."""
    from paper_1908_04262_amd import Sim
    from synth import workload
    n = 64
    wl64 = workload("c4_foam_256", nx=n, ny=n, nz=n, precision="fp64", curvature="plain", max_ids=1024)
    wl64["gas_from"] = int(0.75 * n)
    wl64["nuclei"] = dict(wl64["nuclei"], n=8)
    wl = dict(wl64, precision="fp32", curvature="mlp")
    _say("config-4 crop 64^3, fp32 + mlp vs fp64 oracle, 300 steps")
    gpu = Sim(wl)
    gpu.attach_mlp(trained_net)
    orc = Oracle(wl64)
    c, r, p0 = place_nuclei(wl64)
    gpu.nucleate(c, r, p0)
    orc.nucleate(c, r, p0)
    m0 = _liquid(gpu)
    compared, worst = 0, 0.0
    for k in range(6):
        gpu.step(50)
        orc.step(50)
        bg, bo = gpu.bubbles(), orc.bubbles()
        dm = abs(_liquid(gpu) - m0) / m0
        assert dm < 1e-6, dm
        if list(bg["id"]) == list(bo["id"]) and orc.ledgers()["next_id"] == len(r) + 1:
            dv = np.abs(bg["V"] - bo["V"]) / bo["V"]
            worst = max(worst, dv.max())
            assert dv.max() < 0.005, dv.max()
            compared += 1
        _say(f"  step {50 * (k + 1)}: mass drift {dm:.2e}, compared {compared}, worst volume {worst:.2e}")
    assert compared >= 2
