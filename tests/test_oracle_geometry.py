"""Pins of the oracle's interface geometry.

P16 PLIC plane offset (analytic Scardovelli-Zaleski inverse, Sec. 3.3) against the
inclusion-exclusion volume of a cut unit cube in exact rational arithmetic;
P15 the ray traversal of Appendix A (Algorithm 1, generalised to 3D) against exact
rational ray/grid crossing parameters, and the disjoining pressure of two flat films of
known gap (Sec. 3.3, Eq. for Pi); P9 curvature of voxelised circles and spheres;
nucleation volume (Sec. 3.4).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import Oracle
from oracle.oracle import plic_offset, traverse
from synth.workloads import _mk


def exact_liquid_fraction(dim, m, s):
    """vol{p in [-1/2,1/2]^dim : m.p >= s} exactly, by inclusion-exclusion over the
    cube vertices: vol{x in [0,1]^d : n.x <= a} = sum_v (-1)^|v| max(a - n.v, 0)^d
    / (d! prod n_i) for n_i > 0; zero components drop out of the constraint."""
    mf = [Fraction(abs(c)) for c in m[:dim]]
    sf = Fraction(s)
    a = sf + sum(mf) / 2
    nz = [c for c in mf if c != 0]
    d = len(nz)
    if d == 0:
        return Fraction(1) if sf <= 0 else Fraction(0)
    tot = Fraction(0)
    for v in itertools.product((0, 1), repeat=d):
        t = a - sum(ni * vi for ni, vi in zip(nz, v))
        if t > 0:
            tot += (-1) ** sum(v) * t ** d
    den = math.factorial(d)
    for ni in nz:
        den *= ni
    gas = tot / den
    gas = min(max(gas, Fraction(0)), Fraction(1))
    return 1 - gas


def _random_normals(rng, dim, k):
    out = []
    for _ in range(k):
        v = rng.normal(size=dim)
        out.append(v / np.linalg.norm(v))
    # special directions: axis-aligned, two equal components, one zero component
    if dim == 2:
        out += [np.array([1.0, 0.0]), np.array([0.0, -1.0]),
                np.array([1, 1]) / math.sqrt(2), np.array([-0.6, 0.8])]
    else:
        out += [np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]),
                np.array([0.6, 0.0, -0.8]), np.array([1, 1, 1]) / math.sqrt(3),
                np.array([1, -1, 0]) / math.sqrt(2), np.array([0.2, 0.2, 0.96]) /
                np.linalg.norm([0.2, 0.2, 0.96])]
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_plic_offset_exact_volume(dim):
    rng = np.random.default_rng(31 + dim)
    normals = _random_normals(rng, dim, 60)
    alphas = list(rng.uniform(0, 1, 40)) + [0.0, 1.0, 0.5, 1e-9, 1 - 1e-9, 0.02, 0.97]
    worst = 0.0
    for m in normals:
        m3 = list(m) + [0.0] * (3 - dim)
        for a in alphas:
            s = plic_offset(dim, a, m3)
            got = exact_liquid_fraction(dim, m3, s)
            worst = max(worst, abs(float(got) - a))
            # sign convention: the plane sits on the liquid side when alpha < 1/2
            if a < 0.5 - 1e-12:
                assert s >= 0.0
            if a > 0.5 + 1e-12:
                assert s <= 0.0
    assert worst < 1e-12


def exact_traversal(dim, m, dmax):
    """cells entered by the ray beta*m from the centre of cell 0 (exact crossing
    parameters (k - 1/2)/|m_a|); returns the cells and the smallest relative gap between
    two distinct crossing parameters among the events used"""
    events = []
    for a in range(dim):
        ma = Fraction(m[a])
        if ma == 0:
            continue
        for k in range(1, dmax + 2):
            events.append(((Fraction(2 * k - 1, 2)) / abs(ma), a, 1 if ma > 0 else -1))
    events.sort()
    pos = [0, 0, 0]
    cells, gaps = [], []
    i = 0
    while len(cells) < dmax:
        b = events[i][0]
        j = i
        while j < len(events) and events[j][0] == b:
            pos[events[j][1]] += events[j][2]
            j += 1
        if j < len(events):
            gaps.append(float((events[j][0] - b) / b))
        cells.append(tuple(pos))
        i = j
    return cells, min(gaps) if gaps else 1.0


@pytest.mark.parametrize("dim", [2, 3])
def test_traversal_exact(dim):
    rng = np.random.default_rng(77 + dim)
    dmax = 6
    compared = 0
    normals = _random_normals(rng, dim, 400)
    for m in normals:
        cells, gap = exact_traversal(dim, m, dmax)
        if gap < 1e-9:  # a near-tie that rounding may resolve either way
            continue
        got = traverse(dim, list(m), dmax)
        assert [tuple(int(c) for c in r) for r in got] == cells, (m, got, cells)
        compared += 1
    assert compared > 380


def _film_state(gap_rows, aa, ab, dmax=4.0, kpi=0.005):
    """Two flat films in 2D: bubble 1 below, a liquid layer, bubble 2 above."""
    nx, ny = 8, 24
    wl = _mk(name="film", dim=2, nx=nx, ny=ny, nz=1, gas_from=-1, periodic=[1, 0, 0],
             k_pi=kpi, d_max=dmax, nuclei=None)
    o = Oracle(wl)
    T = np.full((1, ny, nx), 2, np.uint8)
    lab = np.full((1, ny, nx), -1, np.int32)
    al = np.ones((1, ny, nx))
    T[0, 0, :] = 3
    T[0, ny - 1, :] = 3
    ya = 6
    yb = ya + gap_rows + 1
    T[0, 1:ya, :] = 0
    lab[0, 1:ya, :] = 1
    al[0, 1:ya, :] = 0.0
    T[0, ya, :] = 1
    lab[0, ya, :] = 1
    al[0, ya, :] = aa
    T[0, yb, :] = 1
    lab[0, yb, :] = 2
    al[0, yb, :] = ab
    T[0, yb + 1:ny - 1, :] = 0
    lab[0, yb + 1:ny - 1, :] = 2
    al[0, yb + 1:ny - 1, :] = 0.0
    o.write("type", T)
    o.write("label", lab)
    o.write("alpha", al)
    o.write("mass", al)
    o.set_bubble(1, 1.0, 10.0, 1 / 3)
    o.set_bubble(2, 1.0, 10.0, 1 / 3)
    o.geometry()
    return o, ya, yb


@pytest.mark.parametrize("gap_rows,aa,ab", [(0, 0.3, 0.6), (1, 0.5, 0.5), (1, 0.2, 0.9),
                                             (2, 0.4, 0.1), (3, 0.5, 0.5)])
def test_flat_film_disjoining(gap_rows, aa, ab):
    """Liquid film between two flat interfaces: the gap is (rows between the interface
    cells) + alpha_a + alpha_b and Pi = k_Pi (d_max - gap) when gap < d_max."""
    dmax, kpi = 4.0, 0.005
    o, ya, yb = _film_state(gap_rows, aa, ab, dmax, kpi)
    Pi = o.read("pi")[0]
    gap = (yb - ya - 1) + aa + ab
    want = kpi * (dmax - gap) if gap < dmax else 0.0
    assert np.allclose(Pi[ya, :], want, rtol=0, atol=1e-15)
    assert np.allclose(Pi[yb, :], want, rtol=0, atol=1e-15)
    # without the disjoining constant there is no pressure
    o2, _, _ = _film_state(gap_rows, aa, ab, dmax, 0.0)
    assert np.all(o2.read("pi") == 0.0)


def _voxel_case(dim, R, offset):
    n = int(2 * R + 10)
    wl = _mk(name="vox", dim=dim, nx=n, ny=n, nz=n if dim == 3 else 1, gas_from=-1,
             nuclei=None)
    o = Oracle(wl)
    c = np.array([[n / 2 + offset[0], n / 2 + offset[1], (n / 2 + offset[2]) if dim == 3 else 0.0]])
    o.nucleate(c, np.array([R]), np.array([1 / 3]))
    return o


@pytest.mark.parametrize("dim,R", [(2, 5.0), (2, 8.0), (2, 12.0), (3, 4.0), (3, 6.0), (3, 9.0)])
def test_nucleation_volume(dim, R):
    o = _voxel_case(dim, R, (0.31, -0.17, 0.23))
    V = o.bubbles()["V"][0]
    want = math.pi * R * R if dim == 2 else 4 / 3 * math.pi * R ** 3
    assert abs(V / want - 1) < (0.01 if dim == 2 else 0.005)


@pytest.mark.parametrize("dim,R,tol", [(2, 6.0, 0.07), (2, 10.0, 0.04), (2, 16.0, 0.03),
                                       (3, 5.0, 0.07), (3, 8.0, 0.05), (3, 12.0, 0.05)])
def test_curvature_voxelised(dim, R, tol):
    """Mean curvature on the interface of a voxelised circle / sphere: 1/(2R) in 2D
    (half the circle curvature, so that 2 sigma kappa = sigma/R) and 1/R in 3D, positive
    for a gas bubble."""
    o = _voxel_case(dim, R, (0.27, 0.41, -0.12))
    T = o.read("type")
    kap = o.read("kappa")
    al = o.read("alpha")
    sel = (T == 1) & (al > 0.02) & (al < 0.98)
    want = 1 / (2 * R) if dim == 2 else 1 / R
    mean = kap[sel].mean()
    assert abs(mean / want - 1) < tol
    # per-cell scatter stays a fraction of the curvature itself
    assert kap[sel].std() / want < 0.2
    assert np.all(kap[sel] > 0)
