"""Pins of the oracle's Carreau-Yasuda relaxation (Eq. carreauTau in full; the power-law
limit is pinned in test_oracle_lattice.py and test_oracle_force.py).

C1 the implicit relaxation time against an independent bracketing root solve of
   (tau - tau_inf)/(tau0 - tau_inf) = (1 + (lambda gdot)^a)^((n-1)/a), gdot = (3/sqrt 2)|Pi|/(rho tau);
C2 the limits: zero shear, lambda = 0, n = 1 and tau0 = tau_inf give tau0; high shear tends to
   tau_inf;
C3 with lambda = 0 a foam runs exactly as the Newtonian one at tau0;
C4 a channel driven by a body force reaches the steady profile obtained by integrating the
   model's own stress-shear relation rho nu(gdot) gdot = rho a |y - y_c| across the channel.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

from oracle import Oracle
from oracle.oracle import cy_tau
from synth import place_nuclei, small_case
from synth.workloads import _mk

K = 3.0 / math.sqrt(2.0)


def _wl(**kw):
    base = dict(name="cy", dim=2, nx=8, ny=8, nz=1, gas_from=-1, nuclei=None, rheology="carreau_yasuda",
                cy_tau0=1.2, cy_tau_inf=0.6, cy_lambda=1000.0, cy_a=2.0, cy_n=0.4)
    base.update(kw)
    return _mk(**base)


def _ref_tau(wl, rho, pn):
    t0, ti, lam, a, n = (wl[k] for k in ("cy_tau0", "cy_tau_inf", "cy_lambda", "cy_a", "cy_n"))
    if pn == 0:
        return t0

    def G(t):
        gd = K * pn / (rho * t)
        return t - (ti + (t0 - ti) * (1 + (lam * gd) ** a) ** ((n - 1) / a))
    return brentq(G, ti, t0, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)


@pytest.mark.parametrize("params", [
    dict(),
    dict(cy_n=0.2, cy_a=1.0, cy_lambda=50.0, cy_tau0=1.0, cy_tau_inf=0.7),
    dict(cy_n=0.7, cy_a=3.5, cy_lambda=5000.0, cy_tau0=2.0, cy_tau_inf=1.2),
])
def test_cy_tau_root(params):
    wl = _wl(**params)
    for rho in (0.97, 1.0, 1.04):
        for pn in np.geomspace(1e-9, 1e-1, 25):
            got = cy_tau(wl, rho, pn)
            want = _ref_tau(wl, rho, pn)
            assert abs(got - want) <= 1e-13 * want, (rho, pn, got, want)
            lo, hi = wl["cy_tau_inf"], wl["cy_tau0"]
            assert lo <= got <= hi


def test_cy_tau_limits():
    wl = _wl()
    assert cy_tau(wl, 1.0, 0.0) == wl["cy_tau0"]
    for pn in (1e-6, 1e-3):
        assert cy_tau(_wl(cy_lambda=0.0), 1.0, pn) == 1.2
        assert abs(cy_tau(_wl(cy_n=1.0), 1.0, pn) - 1.2) <= 4e-16
        assert cy_tau(_wl(cy_tau_inf=1.2), 1.0, pn) == 1.2
    # strong shear: the relaxation time approaches tau_inf, with the model's algebraic tail
    t = cy_tau(wl, 1.0, 10.0)
    assert 0.6 < t < 0.6 + 0.6 * (1000.0 * K * 10.0 / 0.6) ** (0.4 - 1) * 1.01


def test_cy_lambda_zero_is_newtonian():
    base = small_case("foam2d", precision="fp64")
    runs = []
    for rh in ({"rheology": "newtonian", "tau": 0.9},
               {"rheology": "carreau_yasuda", "tau": 0.5001, "cy_tau0": 0.9, "cy_tau_inf": 0.6,
                "cy_lambda": 0.0}):
        wl = dict(base, **rh)
        o = Oracle(wl)
        c, r, p0 = place_nuclei(wl)
        o.nucleate(c, r, p0)
        o.step(30)
        runs.append((o.read("f"), o.read("type"), o.read("label")))
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    assert np.array_equal(runs[0][0], runs[1][0])


def _cy_channel_profile(wl, a, H):
    """u(y) of steady channel flow between walls at y = 1/2 and y = H + 1/2 from the stress
    balance rho nu(gdot) gdot = rho a |y - y_c| with nu = (tau(gdot) - 1/2)/3 and the explicit
    Carreau-Yasuda tau(gdot) (Eq. carreauTau as a function of the shear rate)."""
    t0, ti, lam, al, n = (wl[k] for k in ("cy_tau0", "cy_tau_inf", "cy_lambda", "cy_a", "cy_n"))

    def nu(g):
        return ((ti + (t0 - ti) * (1 + (lam * g) ** al) ** ((n - 1) / al)) - 0.5) / 3.0

    def gdot(s):
        if s == 0:
            return 0.0
        return brentq(lambda g: nu(g) * g - s, 0.0, 10.0, xtol=1e-18, rtol=1e-14)

    yc = (H + 1) / 2.0
    y = np.arange(H + 2, dtype=float)
    u = np.zeros_like(y)
    for k in range(1, H + 1):
        d0, d1 = abs(0.5 - yc), abs(y[k] - yc)
        # u(y) = integral from the wall of gdot, symmetric about y_c
        u[k] = quad(lambda dd: gdot(a * dd), d1, d0, limit=200)[0]
    return u


def test_cy_channel_profile():
    H = 16
    a = 5e-5
    wl = _mk(name="cyc", dim=2, nx=3, ny=H + 2, nz=1, gas_from=-1, nuclei=None, periodic=[1, 0, 1],
             precision="fp64", rheology="carreau_yasuda", cy_tau0=1.2, cy_tau_inf=0.6, cy_lambda=1000.0,
             cy_a=2.0, cy_n=0.4, accel=(a, 0.0, 0.0))
    o = Oracle(wl)
    o.step(8000)
    f = o.read("f")
    e = np.array(o.lattice()[0], float)
    T = o.read("type")
    rho = f.sum(axis=0)
    jx = np.tensordot(e[:, 0], f, axes=(0, 0))
    fluid = T == 2
    ux = np.where(fluid, jx / np.where(fluid, rho, 1.0) - 0.5 * a, 0.0)
    u = ux.sum(axis=(0, 2)) / np.maximum(fluid.sum(axis=(0, 2)), 1)
    ref = _cy_channel_profile(wl, a, H)
    fl = slice(1, H + 1)
    err = np.abs(u[fl] - ref[fl]).max() / ref[fl].max()
    # the viscosity varies by a factor of two across the channel (tau from 0.9 at the walls to
    # 1.2 at the centre), so a wrong exponent or shear-rate factor moves the profile by far more
    assert err < 1e-2, err
