"""Pins of the oracle's lattice Boltzmann core against closed forms.

P1 lattice isotropy and equilibrium moments (Sec. 2, Eq. equilibrium; Sec. 3.1 ADE
equilibrium), P2 rest state, P3 shear-wave decay at nu = c_s^2 (tau - 1/2) (Eq. tau),
P4 Gaussian-pulse spreading at D = c_s^2 (tau_g - 1/2) (Eq. diffusionconst), P18 the
implicit power-law relaxation time (Eq. carreauTau, power-law limit).
"""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import Oracle
from oracle.oracle import powerlaw_tau
from synth.workloads import _mk


def _box(dim, n, **kw):
    base = dict(name="t", dim=dim, nx=n[0], ny=n[1], nz=n[2] if dim == 3 else 1,
                gas_from=-1, nuclei=None)
    base.update(kw)
    return _mk(**base)


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_isotropy(dim):
    o = Oracle(_box(dim, (6, 6, 6)))
    e, w, wg, opp = o.lattice()
    Q = len(w)
    assert Q == (9 if dim == 2 else 19)
    # the velocity set: every vector with components in {-1,0,1} and |e|^2 <= 2 in 3D,
    # all nine in 2D (Sec. 2 lists the D3Q19 groups)
    want = {v for v in itertools.product((-1, 0, 1), repeat=dim)
            if dim == 2 or sum(c * c for c in v) <= 2}
    got = {tuple(int(c) for c in row[:dim]) for row in e}
    assert got == want and len(got) == Q
    assert tuple(e[0]) == (0, 0, 0)
    for i in range(Q):
        assert np.array_equal(e[opp[i]], -e[i])
    # weights printed in Fig. latticesfluid
    if dim == 2:
        assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=0)
    else:
        assert np.allclose(w, [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, rtol=0, atol=0)
    # isotropy up to fourth order with c_s^2 = 1/3
    ef = e[:, :dim].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ ef).max() < 1e-16
    M2 = np.einsum("i,ia,ib->ab", w, ef, ef)
    assert np.allclose(M2, np.eye(dim) / 3, atol=1e-16)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, ef, ef, ef, ef)
    d = np.eye(dim)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(M4, iso, atol=1e-16)
    # ADE lattice: rest + axis directions, c_s^2 = 1/3 (D2Q5) or 1/4 (D3Q7), Sec. 3.1
    cs2 = 1 / 3 if dim == 2 else 1 / 4
    eg = ef[: len(wg)]
    assert abs(wg.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia,ib->ab", wg, eg, eg), np.eye(dim) * cs2, atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments(dim):
    o = Oracle(_box(dim, (6, 6, 6)))
    e, w, wg, opp = o.lattice()
    ef = e.astype(float)
    rng = np.random.default_rng(5)
    for _ in range(50):
        rho = rng.uniform(0.8, 1.2)
        u = np.zeros(3)
        u[:dim] = rng.uniform(-0.1, 0.1, dim)
        f = np.array([o.feq(i, rho, u) for i in range(len(w))])
        assert abs(f.sum() - rho) < 2e-15
        assert np.abs(f @ ef - rho * u).max() < 2e-15
        P = np.einsum("i,ia,ib->ab", f, ef, ef)[:dim, :dim]
        want = rho / 3 * np.eye(dim) + rho * np.outer(u[:dim], u[:dim])
        assert np.abs(P - want).max() < 2e-15
        c = rng.uniform(0, 0.02)
        g = np.array([o.geq(i, c, u) for i in range(len(wg))])
        assert abs(g.sum() - c) < 1e-17
        assert np.abs(g @ ef[: len(wg)] - c * u).max() < 1e-17


@pytest.mark.parametrize("rheology", ["newtonian", "power_law"])
def test_rest_state(rheology):
    """A closed liquid box at rest stays at rest: u stays exactly zero and the
    populations stay at w_i up to rounding (sum w_i is 1 + 2^-52 in binary64)."""
    wl = _box(3, (10, 9, 8), rheology=rheology, pl_n=0.6, S0=1.3)
    o = Oracle(wl)
    _, w, wg, _ = o.lattice()
    o.step(300)
    f = o.read("f")
    T = o.read("type")
    fl = T == 2
    dev = np.abs(f[:, fl] - w[:, None]).max()
    assert dev < 1e-13
    fl_f = f[:, fl]
    e, *_ = o.lattice()
    j = np.einsum("ia,in->an", e.astype(float), fl_f)
    assert np.all(j == 0.0)
    c = o.read("conc")[fl]
    c0 = wl["S0"] * wl["kH"] * wl["p_atm"]
    assert np.abs(c - c0).max() < 1e-16


@pytest.mark.parametrize("dim,tau", [(2, 0.6), (2, 0.8), (2, 1.0), (3, 0.8)])
def test_shear_wave_viscosity(dim, tau):
    """u_x = U sin(k y) decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3 (Eq. tau)."""
    L = 64
    n = (4, L, 4)
    wl = _box(dim, n, tau=tau, periodic=[1, 1, 1], S0=0.0)
    o = Oracle(wl)
    e, w, wg, opp = o.lattice()
    Q = len(w)
    U = 1e-3
    k = 2 * math.pi / L
    f = np.zeros((Q,) + o.shape)
    for y in range(L):
        u = (U * math.sin(k * y), 0.0, 0.0)
        for i in range(Q):
            f[i, :, y, :] = o.feq(i, 1.0, u)
    o.write("f", f)
    ys = np.arange(L)
    amps, ts = [], []
    for t in range(0, 401, 50):
        if t:
            o.step(50)
        f = o.read("f")
        rho = f.sum(0)
        ux = np.einsum("i,i...->...", e[:, 0].astype(float), f) / rho
        prof = ux.mean(axis=(0, 2))
        amps.append(2 / L * (prof * np.sin(k * ys)).sum())
        ts.append(t)
    slope = np.polyfit(ts, np.log(amps), 1)[0]
    nu_fit = -slope / k ** 2
    nu = (tau - 0.5) / 3
    assert abs(nu_fit / nu - 1) < 0.01


@pytest.mark.parametrize("dim", [2, 3])
def test_ade_gaussian_variance(dim):
    """A Gaussian concentration pulse at rest spreads its variance by 2 D t per axis,
    with D = c_s^2 (tau_g - 1/2) (Eq. diffusionconst)."""
    n = (48, 48, 48) if dim == 2 else (32, 32, 32)
    D = 0.05
    wl = _box(dim, n, periodic=[1, 1, 1], D=D, S0=0.0)
    o = Oracle(wl)
    e, w, wg, opp = o.lattice()
    s0 = 3.0
    zz, yy, xx = np.meshgrid(*(np.arange(s) for s in o.shape), indexing="ij")
    cx = [(s - 1) / 2 for s in (n[0], n[1], n[2] if dim == 3 else 1)]
    r2 = (xx - cx[0]) ** 2 + (yy - cx[1]) ** 2
    if dim == 3:
        r2 = r2 + (zz - cx[2]) ** 2
    c = 1e-3 * np.exp(-r2 / (2 * s0 * s0))
    g = np.stack([wg[i] * c for i in range(len(wg))])
    o.write("g", g)

    def var_x():
        cc = o.read("conc")
        m = cc.sum()
        return ((xx - cx[0]) ** 2 * cc).sum() / m

    # the first steps carry the initial layer of an equilibrium start; measure after it
    o.step(25)
    v0 = var_x()
    t = 75 if dim == 2 else 50
    o.step(t)
    v1 = var_x()
    assert abs((v1 - v0) / (2 * D * t) - 1) < 0.005


def test_powerlaw_tau_implicit_root():
    """tau solves tau - 1/2 = 3 nu_ref (gdot(tau)/gdot_ref)^(n-1) with
    gdot = 3 |Pi_neq| / (sqrt(2) rho tau), clamped to [tau_min, tau_max]; checked against
    a bracketing root solve of that equation over nine decades of |Pi_neq|."""
    wl = _mk(name="pl", dim=3, nx=4, ny=4, nz=4, gas_from=-1, rheology="power_law",
             pl_n=0.6, pl_nu_ref=0.1, pl_gdot_ref=1e-3, tau_min=0.51, tau_max=2.0)
    rng = np.random.default_rng(9)
    for _ in range(300):
        rho = rng.uniform(0.9, 1.1)
        pn = 10 ** rng.uniform(-9, 0)

        def h(tau):
            gdot = 3 * pn / (math.sqrt(2) * rho * tau)
            return tau - 0.5 - 3 * wl["pl_nu_ref"] * (gdot / wl["pl_gdot_ref"]) ** (wl["pl_n"] - 1)

        lo, hi = wl["tau_min"], wl["tau_max"]
        if h(lo) >= 0:
            want = lo
        elif h(hi) <= 0:
            want = hi
        else:
            want = brentq(h, lo, hi, xtol=1e-15, rtol=1e-15)
        assert abs(powerlaw_tau(wl, rho, pn) - want) < 1e-12
    # fluid at rest: zero shear rate gives the upper clamp for shear thinning
    assert powerlaw_tau(wl, 1.0, 0.0) == 2.0
    # n = 1 is Newtonian: tau = 1/2 + 3 nu_ref whatever the shear
    wl1 = dict(wl, pl_n=1.0)
    assert abs(powerlaw_tau(wl1, 1.0, 1e-4) - 0.8) < 1e-15
