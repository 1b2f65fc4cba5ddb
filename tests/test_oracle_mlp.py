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
