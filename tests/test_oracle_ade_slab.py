"""Pin of the oracle's dissolved-gas transport against the paper's advection-diffusion
validation (Sec. 4.1, Table validatonParameters, Eq. diffusionanalytical; values in
tests/golden/ade_slab_sec41.txt): a liquid slab with a uniform gas source between two gas
regions at the Henry value reaches the parabola 8 D (c - k_H p_g) / (q L^2) = 1 - x'^2.

It ties together the source term (w_i q in the ADE update), the diffusivity of the D2Q5
lattice (D = c_s^2 (tau_g - 1/2), Eq. diffusionconst) and the Henry rebuild at the
interface (Eqs. henryslaw, reconstructdiffusion): a wrong source weight or sign moves the
curvature, a wrong tau_g the curvature as well, and a wrong Henry value the end values.
The slab is at rest here; the paper moves it at v_x, which leaves the steady profile in
the slab's own frame unchanged.
"""
import pathlib

import numpy as np

from oracle import Oracle
from synth.workloads import _mk

G, I, L, W = 0, 1, 2, 3
GOLDEN = pathlib.Path(__file__).parent / "golden" / "ade_slab_sec41.txt"


def _fixture():
    vals = {}
    for line in GOLDEN.read_text().splitlines():
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_ade_slab_steady_state():
    fx = _fixture()
    D, q, kH, pg, nu = fx["D"], fx["q"], fx["k_H"], fx["p_g"], fx["nu"]
    Ls = int(fx["L"])  # interface cell to interface cell, both included
    ng, ny = 6, 4
    nx = Ls + 2 * ng
    # periodic box: the two gas regions join through the boundary into the atmosphere (id 0)
    wl = _mk(name="slab", dim=2, nx=nx, ny=ny, nz=1, periodic=[1, 1, 1], gas_from=-1, nuclei=None,
             tau=3 * nu + 0.5, D=D, q=q, kH=kH, p_atm=pg, sigma=0.0, S0=1.0)
    o = Oracle(wl)
    _, _, wg, _ = o.lattice()
    T = np.full((1, ny, nx), L, np.uint8)
    T[0, :, :ng] = G
    T[0, :, ng + Ls:] = G
    T[0, :, ng] = I
    T[0, :, ng + Ls - 1] = I
    lab = np.where(T == L, -1, 0).astype(np.int32)
    M = np.where(T == L, 1.0, np.where(T == I, 0.5, 0.0))
    # start near the answer (any start reaches the same steady state; this one in fewer steps)
    x = np.arange(nx)
    xc = ng + (Ls - 1) / 2
    c0 = kH * pg + q * (Ls - 1) ** 2 / (8 * D) * (1 - (2 * (x - xc) / (Ls - 1)) ** 2)
    c0 = np.where((x >= ng) & (x < ng + Ls), c0, kH * pg)
    cc = np.broadcast_to(c0, (1, ny, nx))
    o.write("type", T)
    o.write("label", lab)
    o.write("mass", M)
    o.write("alpha", M)
    o.write("rho", np.ones((1, ny, nx)))
    o.write("g", np.stack([wg[i] * cc for i in range(len(wg))]))
    o.set_bubble(0, 0.0, 0.0, pg)
    o.geometry()
    o.step(12000)

    assert np.array_equal(o.read("type"), T)  # the interfaces stay where they are
    assert np.abs(o.read("ux")).max() < 1e-12  # and the liquid at rest
    cv = o.read("conc")[0]
    assert np.abs(cv - cv[0]).max() < 1e-15 * cv.max()  # uniform along y
    c = cv[0]
    liq = np.arange(ng + 1, ng + Ls - 1)
    assert np.abs(c[liq] - c[liq[::-1]]).max() < 1e-12  # symmetric about the centre
    # the fitted parabola: curvature -q / (2D), zeros of c - k_H p_g a distance L apart
    A = np.vstack([np.ones(len(liq)), liq, liq ** 2]).T
    c_0, c_1, c_2 = np.linalg.lstsq(A, c[liq], rcond=None)[0]
    assert abs(c_2 / (-q / (2 * D)) - 1) < 5e-3
    cmax = c_0 - c_1 ** 2 / (4 * c_2)
    half = np.sqrt((cmax - kH * pg) / (-c_2))
    assert abs(2 * half - Ls) < 0.5
    # Eq. diffusionanalytical at the centre (x' = 0) with the printed L
    assert abs(8 * D * (cmax - kH * pg) / (q * Ls ** 2) - 1) < 1e-2
    # and across the slab
    xp = 2 * (liq - xc) / Ls
    lhs = 8 * D * (c[liq] - kH * pg) / (q * Ls ** 2)
    assert np.abs(lhs - (1 - xp ** 2)).max() < 1e-2
