"""Pins of the learned-curvature reference (oracle/mlp.py) against mathematics outside it.

* ellipsoid mean curvature (closed form) against the divergence of the unit normal of the
  implicit function computed by finite differences, and 1/R on spheres;
* closest-point solve: the point lies on the surface and o - q is parallel to the normal;
* canonical orientation: invariant under all 48 cube symmetries, and orders the gradient;
* backward pass against central finite differences of the loss;
* generated stencils: labels within the trained range, centre cell cut, spheres give
  |kappa| = 1/R consistent with the stencil's own paraboloid (checked loosely).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import mlp as M


def _implicit_H(q, a, h=1e-4):
    """mean curvature from H = -div(grad F / |grad F|) / 2 by central differences"""
    def n(p):
        g = 2 * p / (a * a)
        return g / np.linalg.norm(g)

    div = 0.0
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        div += (n(q + e)[i] - n(q - e)[i]) / (2 * h)
    return abs(div) / 2


def test_ellipsoid_curvature_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(40):
        a = np.exp(rng.uniform(math.log(2), math.log(40), 3))
        d = rng.normal(size=3)
        q = d / math.sqrt(((d / a) ** 2).sum())
        assert abs(M.ellipsoid_mean_curvature(q, a) / _implicit_H(q, a) - 1) < 1e-6
    for R in (2.0, 7.5, 39.0):
        q = np.array([R, 0, 0]) @ np.eye(3)
        assert abs(M.ellipsoid_mean_curvature(q, np.array([R, R, R])) * R - 1) < 1e-14


def test_closest_point_geometry():
    rng = np.random.default_rng(4)
    for _ in range(40):
        a = np.exp(rng.uniform(math.log(2), math.log(40), 3))
        d = rng.normal(size=3)
        on = d / math.sqrt(((d / a) ** 2).sum())
        o = on + rng.normal(size=3) * 0.6
        q = M.closest_point(o, a)
        assert abs(((q / a) ** 2).sum() - 1) < 1e-12
        nrm = q / (a * a)
        r = o - q
        cross = np.cross(r, nrm)
        assert np.linalg.norm(cross) <= 1e-9 * max(1.0, np.linalg.norm(r) * np.linalg.norm(nrm))


def _apply_symmetry(s, perm, flips):
    """apply a cube symmetry to a [z][y][x] stencil: flip lattice axes, then permute"""
    t = s
    for ax in range(3):
        if flips[ax]:
            t = np.flip(t, axis=2 - ax)
    return np.transpose(t, axes=[2 - perm[2], 2 - perm[1], 2 - perm[0]])


def test_canonical_form_invariant():
    rng = np.random.default_rng(5)
    for _ in range(10):
        s = rng.uniform(0, 1, (5, 5, 5))
        base = M.canonicalise(s.reshape(1, -1))[0]
        c = base.reshape(5, 5, 5)
        g = [0.5 * (c[2, 2, 3] - c[2, 2, 1]), 0.5 * (c[2, 3, 2] - c[2, 1, 2]),
             0.5 * (c[3, 2, 2] - c[1, 2, 2])]
        assert g[0] >= g[1] >= g[2] >= 0
        for perm in itertools.permutations(range(3)):
            for flips in itertools.product((0, 1), repeat=3):
                t = _apply_symmetry(s, perm, flips)
                assert np.array_equal(M.canonicalise(t.reshape(1, -1))[0], base)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(6)
    theta = M.init_params(11) + rng.normal(size=M.NPARAM) * 0.01
    theta[M.NFEAT * M.H:M.NPAD * M.H] = 0.0
    X = rng.uniform(0, 1, (16, M.NFEAT))
    t = rng.normal(size=16)
    loss, g = M.loss_and_grad(theta, X, t, rounding=False)
    idx = rng.choice(M.NPARAM, 60, replace=False)
    idx = [i for i in idx if not (M.NFEAT * M.H <= i < M.NPAD * M.H)] + [M.NPARAM - 1]
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (M.loss_and_grad(tp, X, t, False)[0] - M.loss_and_grad(tm, X, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i]))


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 1e-3, 0.0])
    r = M.bf16(vals)
    for v, b in zip(vals, r):
        # bfloat16 keeps 8 significant bits: the rounded value is the nearest such number
        if v == 0:
            assert b == 0
            continue
        e = math.floor(math.log2(abs(v)))
        ulp = 2.0 ** (e - 7)
        assert abs(b - v) <= ulp / 2 + 1e-12
        assert (abs(b) / ulp) == int(abs(b) / ulp)


def test_generated_stencils():
    X, K = M.generate(44, 0, 24)
    assert np.all(np.abs(K) <= 0.5)
    assert np.all((X[:, 62] > 0) & (X[:, 62] < 1))
    assert np.all((X >= 0) & (X <= 1))
    # both phases appear and the sign of kappa follows the side the gas is on: the
    # centre cell of a bubble-like (gas inside) surface has liquid on the outside
    assert (K > 0).any() and (K < 0).any()


# ------------------------------------------------------------ generator geometry pins
def _body_rotation(q):
    """rotation of the body frame from its quaternion (w, x, y, z), through scipy"""
    from scipy.spatial.transform import Rotation
    w, x, y, z = q
    return Rotation.from_quat([x, y, z, w]).as_matrix()


def _cell_fraction(centre, c, Rm, a, n=24):
    """fraction of the unit cell around `centre` inside the body, by n^3 midpoints"""
    s = (np.arange(n) + 0.5) / n - 0.5
    g = np.stack(np.meshgrid(s, s, s, indexing="ij"), -1).reshape(-1, 3) + centre
    yb = (g - c) @ Rm
    return float(((yb / a) ** 2).sum(-1).__lt__(1.0).mean())


def _closest_surface_point(o, a):
    """point of the ellipsoid surface nearest to o (body frame): coarse search over the
    spherical parametrisation, then Nelder-Mead"""
    from scipy.optimize import minimize

    def pt(v):
        th, ph = v
        return a * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])

    th = np.linspace(0.01, math.pi - 0.01, 60)
    ph = np.linspace(-math.pi, math.pi, 120)
    best = min(((float(((pt((t, p)) - o) ** 2).sum()), (t, p)) for t in th for p in ph))[1]
    r = minimize(lambda v: ((pt(v) - o) ** 2).sum(), best, method="Nelder-Mead",
                 options=dict(xatol=1e-12, fatol=1e-16, maxiter=20000))
    return pt(r.x)


def _generated(n, seed=44):
    geo = []
    X, K = M.generate(seed, 0, n, noise=0.0, geometry=geo)
    return X, K, geo


def test_generator_stencil_is_the_voxelised_body():
    """Every fill fraction of a noiseless stencil equals the fraction of that cell inside
    the body (or outside, for liquid inside the body), computed here from the body alone
    with its own rotation (scipy), cell order (dz outer, dx inner) and 24^3 sampling.
    The generator samples cut cells 10^3 times, so cells agree to the sampling error, and
    the sums over the stencil (its volume) agree more closely."""
    X, K, geo = _generated(24)
    worst, mean_err = 0.0, []
    for k in range(len(X)):
        g = geo[k]
        Rm = _body_rotation(g["q"])
        al = np.empty(125)
        for j in range(125):
            cell = np.array([j % 5 - 2, (j // 5) % 5 - 2, j // 25 - 2], float)
            f = _cell_fraction(cell, g["c"], Rm, g["a"])
            al[j] = 1.0 - f if g["gas_inside"] else f
        d = np.abs(X[k] - al)
        worst = max(worst, d.max())
        mean_err.append(d.mean())
        assert abs(X[k].sum() - al.sum()) < 0.25, (k, X[k].sum(), al.sum())
    assert worst < 0.08, worst
    assert np.mean(mean_err) < 4e-3, np.mean(mean_err)


def test_generator_label_is_the_curvature_nearest_the_centre():
    """The label is the mean curvature (Eq. rhob convention: positive with gas inside) at
    the body's surface point nearest the centre-cell centre: found here by a direct
    search over the surface and evaluated by finite differences of the implicit normal."""
    X, K, geo = _generated(24)
    for k in range(len(X)):
        g = geo[k]
        Rm = _body_rotation(g["q"])
        o = Rm.T @ (-g["c"])
        q = _closest_surface_point(o, g["a"])
        H = _implicit_H(q, g["a"], h=1e-5)
        want = H if g["gas_inside"] else -H
        assert abs(K[k] - want) <= 1e-5 * abs(want) + 1e-9, (k, K[k], want)
        # the centre cell is cut by the surface, so the nearest point lies within it
        assert np.abs(Rm @ q + g["c"]).max() <= 0.5 + 1e-9


def _plain_fit_kappa(stencil):
    """the oracle's plain paraboloid fit at the centre of a 5x5x5 stencil (placed in a
    periodic 9^3 box; the fit reads at most two cells from the centre)"""
    from oracle import Oracle
    from synth.workloads import _mk
    wl = _mk(name="st", dim=3, nx=9, ny=9, nz=9, gas_from=-1, periodic=[1, 1, 1], nuclei=None)
    o = Oracle(wl)
    a = np.ones((9, 9, 9))
    a[2:7, 2:7, 2:7] = np.asarray(stencil, dtype=np.float64).reshape(5, 5, 5)
    T = np.where(a <= 0.0, 0, np.where(a >= 1.0, 2, 1)).astype(np.uint8)
    o.write("type", T)
    o.write("alpha", a)
    return o.curvature(o.cell(4, 4, 4))


def test_generator_spheres_agree_with_the_plain_fit():
    """On noiseless sphere stencils the oracle's own plain fit, which knows nothing of the
    generator, recovers the label 1/R with its sign (gas side) to the accuracy the plain
    fit has on voxelised spheres."""
    X, K, geo = _generated(160, seed=45)
    rel = []
    for k in range(len(X)):
        a = geo[k]["a"]
        if not (a[0] == a[1] == a[2]) or a[0] > 12.0:
            continue
        kp = _plain_fit_kappa(X[k])
        assert abs(abs(K[k]) * a[0] - 1.0) < 1e-6
        rel.append((kp - K[k]) / abs(K[k]))
    rel = np.array(rel)
    assert rel.size >= 15, rel.size
    assert np.median(np.abs(rel)) < 0.12, np.median(np.abs(rel))
    assert (np.abs(rel) < 0.5).mean() >= 0.9
