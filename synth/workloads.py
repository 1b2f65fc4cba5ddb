"""Seeded workload definitions and nucleus placement (input data only).

Every run in this repository starts from a parameter dictionary returned by
``workload(name)`` or ``small_case(name)`` and from the nucleus list returned by
``place_nuclei``.  The physical constants that the benchmark configurations leave
open are filled from the parameter sets printed in the paper's figure captions
(Sec. 4.3-4.5: k_H = 5e-3, RT = 50, k_Pi = 5e-3); the remaining gaps (liquid level,
diffusivity, supersaturation, power-law reference viscosity) are fixed below.  Randomness: SplitMix64 (Steele, Lea and Flood, 2014) as the integer
stream and U(0,1) = (u >> 11) * 2**-53.

Nucleus placement is a fixed list (``fixed``: (x, y, z, r) per nucleus), one nucleus at the
grid centre with a seeded sub-cell offset (``center="jitter"``), or dart throwing: per attempt draw r ~ U[r_min, r_max], then the
centre coordinates in axis order, each uniform over the liquid box that keeps the
sphere ``r + 2`` cells away from walls and from the headspace; accept if the centre
distance to every accepted nucleus is at least ``min_sep`` (or r_i + r_j + 4 when
``min_sep`` is None).
"""
from __future__ import annotations

import copy
import math

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (2.0 ** -53)

    def uniform_range(self, lo: float, hi: float) -> float:
        return lo + (hi - lo) * self.uniform()


_COMMON = dict(
    periodic=[0, 0, 0],
    precision="fp64",
    rheology="newtonian",
    tau=0.8,
    pl_n=1.0,
    pl_nu_ref=0.1,
    pl_gdot_ref=1e-3,
    tau_min=0.51,
    tau_max=2.0,
    sigma=0.0,
    D=0.05,
    q=0.0,
    kH=5e-3,
    RT=50.0,
    k_pi=0.0,
    d_max=4.0,
    S0=1.0,
    p_atm=1.0 / 3.0,
    eps=1e-3,
    cleanup=1,
    max_ids=4096,
    curvature="plain",
    steps=100,
    seed=0,
    nuclei=None,
)


def _mk(**kw):
    d = copy.deepcopy(_COMMON)
    d.update(kw)
    if d.get("gas_from") is None:
        last = d["ny"] if d["dim"] == 2 else d["nz"]
        d["gas_from"] = int(math.floor(0.75 * last))
    return d


# The five benchmark configurations (lattice units; grids include the wall layer).
WORKLOADS = {
    # 2D D2Q9 + D2Q5, one bubble of radius 8 at the centre with a seeded sub-cell offset.
    "c1_2d_128": _mk(
        name="c1_2d_128", dim=2, nx=128, ny=128, nz=1, precision="fp64", tau=0.8,
        sigma=1e-3, D=0.05, S0=1.2, steps=1000, seed=1,
        nuclei=dict(n=1, r_min=8.0, r_max=8.0, center="jitter", p0=1.05 / 3.0),
    ),
    # 3D D3Q19 + D3Q7, 32 bubbles, disjoining pressure on lamellae thinner than 2 cells.
    "c2_3d_128": _mk(
        name="c2_3d_128", dim=3, nx=128, ny=128, nz=128, precision="fp32", tau=0.7,
        sigma=5e-4, S0=1.5, k_pi=5e-3, d_max=2.0, steps=5000, seed=2,
        nuclei=dict(n=32, r_min=3.0, r_max=5.0, min_sep=12.0),
    ),
    # 3D 384^3 power-law foam with 2000 bubbles and coalescence.
    "c3_foam_384": _mk(
        name="c3_foam_384", dim=3, nx=384, ny=384, nz=384, precision="fp32",
        rheology="power_law", pl_n=0.6, pl_nu_ref=0.1, pl_gdot_ref=1e-3,
        tau_min=0.51, tau_max=2.0, tau=0.8, sigma=5e-4, S0=1.5, k_pi=0.0,
        steps=10000, seed=3, max_ids=16384,
        nuclei=dict(n=2000, r_min=2.0, r_max=4.0, min_sep=None),
    ),
    # 256^3 foam run of the learned-curvature configuration (config-2 style).
    "c4_foam_256": _mk(
        name="c4_foam_256", dim=3, nx=256, ny=256, nz=256, precision="fp32", tau=0.7,
        sigma=5e-4, S0=1.5, k_pi=5e-3, d_max=2.0, steps=5000, seed=41,
        curvature="mlp", max_ids=8192,
        nuclei=dict(n=500, r_min=3.0, r_max=5.0, min_sep=12.0),
    ),
}


def workload(name: str, **overrides) -> dict:
    d = copy.deepcopy(WORKLOADS[name])
    d.update(overrides)
    return d


def small_case(name: str, **overrides) -> dict:
    """Small seeded cases that the oracle finishes in seconds (parity tests)."""
    cases = {
        # config-1 physics on a 48x48 grid (several 64-wide tiles are not needed in 2D;
        # the ragged tail is the 48-wide row).
        "c1_small": _mk(
            name="c1_small", dim=2, nx=48, ny=48, nz=1, tau=0.8, sigma=1e-3, S0=1.2,
            steps=200, seed=1,
            nuclei=dict(n=1, r_min=6.0, r_max=6.0, center="jitter", p0=1.05 / 3.0),
        ),
        "c1_full": copy.deepcopy(WORKLOADS["c1_2d_128"]),
        # 2D foam with several bubbles that grow and coalesce.
        "foam2d": _mk(
            name="foam2d", dim=2, nx=96, ny=80, nz=1, tau=0.8, sigma=1e-3, S0=3.0,
            kH=5e-3, RT=50.0, steps=300, seed=11,
            nuclei=dict(n=8, r_min=2.5, r_max=4.0, min_sep=None),
        ),
        # 3D config-2 physics on a small ragged grid.
        "c2_small": _mk(
            name="c2_small", dim=3, nx=70, ny=40, nz=36, precision="fp64", tau=0.7,
            sigma=5e-4, S0=1.5, k_pi=5e-3, d_max=2.0, steps=60, seed=2,
            nuclei=dict(n=6, r_min=3.0, r_max=5.0, min_sep=10.0),
        ),
        # 3D power-law foam (config-3 physics) on a small grid.
        "c3_small": _mk(
            name="c3_small", dim=3, nx=72, ny=40, nz=40, precision="fp64",
            rheology="power_law", pl_n=0.6, pl_nu_ref=0.1, pl_gdot_ref=1e-3,
            tau_min=0.51, tau_max=2.0, tau=0.8, sigma=5e-4, S0=1.5,
            steps=60, seed=3,
            nuclei=dict(n=12, r_min=2.0, r_max=4.0, min_sep=None),
        ),
        # Topology and lamella cases (3D, binary64): nuclei at given places. Bubbles a
        # lamella of two cells apart in a 3 x 3 layer (disjoining pressure acts on the
        # films between them; saturated liquid, so they neither grow nor shrink much).
        "lamella3d": _mk(
            name="lamella3d", dim=3, nx=53, ny=50, nz=31, precision="fp64", tau=0.7,
            sigma=5e-4, S0=1.0, k_pi=5e-3, d_max=2.0, steps=100, seed=0,
            nuclei=dict(n=9, fixed=_grid_layer(53, 50, 11.3, 3, 4.0, 2.0)),
        ),
        # two growing bubbles two cells apart: the film between them breaks (merge), the
        # disjoining pressure opens the neck again (split into a new id), and they join
        # once more
        "neck3d": _mk(
            name="neck3d", dim=3, nx=46, ny=34, nz=34, precision="fp64", tau=0.7,
            sigma=5e-4, S0=1.5, k_pi=5e-3, d_max=2.0, steps=30, seed=0,
            nuclei=dict(n=2, fixed=[(17.5, 16.3, 14.2, 4.0), (27.5, 16.6, 14.0, 4.0)]),
        ),
        # growth at supersaturation 2: two bubbles merge, a third one under the liquid
        # surface grows into the headspace and bursts
        "burst3d": _mk(
            name="burst3d", dim=3, nx=46, ny=34, nz=34, precision="fp64", tau=0.7,
            sigma=5e-4, S0=2.0, steps=100, seed=0,
            nuclei=dict(n=3, fixed=[(12.3, 12.2, 10.4, 4.0), (22.1, 12.5, 10.2, 4.0),
                                    (30.4, 23.6, 25 - 5.6, 3.0)]),
        ),
        # dissolution in undersaturated liquid: three small bubbles shrink and vanish
        "dissolve3d": _mk(
            name="dissolve3d", dim=3, nx=38, ny=30, nz=29, precision="fp64", tau=0.7,
            sigma=2e-3, D=0.1, S0=0.2, steps=340, seed=0,
            nuclei=dict(n=3, fixed=[(10.3, 10.2, 9.4, 2.0), (24.1, 17.5, 10.2, 2.6),
                                    (14.4, 21.6, 12.1, 3.2)]),
        ),
    }
    d = cases[name]
    d.update(overrides)
    return d


def _grid_layer(nx, ny, z, n, r, gap):
    """n x n nuclei of radius r in the plane at height z, centre spacing 2r + gap, with
    small fixed sub-cell offsets so that no two spheres voxelise alike."""
    sp = 2.0 * r + gap
    out = []
    for j in range(n):
        for i in range(n):
            out.append((nx / 2 + (i - (n - 1) / 2) * sp + 0.13 * j,
                        ny / 2 + (j - (n - 1) / 2) * sp - 0.07 * i, z + 0.1 * i, r))
    return out


def _liquid_box(wl: dict, r: float):
    """Bounds of admissible centre coordinates for a nucleus of radius r."""
    dims = [wl["nx"], wl["ny"], wl["nz"]][: wl["dim"]]
    lo, hi = [], []
    for a, n in enumerate(dims):
        wall = 0 if wl["periodic"][a] else 1
        lo.append(wall + r + 2.0 - 0.5)
        top = n - 1 - wall
        if a == wl["dim"] - 1 and wl["gas_from"] >= 0:
            top = min(top, wl["gas_from"] - 1)
        hi.append(top - r - 2.0 + 0.5)
    return lo, hi


def place_nuclei(wl: dict):
    """Return (centers[n,3], radii[n], p0[n]) for the workload's nucleus recipe."""
    spec = wl["nuclei"]
    dim = wl["dim"]
    if not spec:
        return np.zeros((0, 3)), np.zeros(0), np.zeros(0)
    rng = SplitMix64(wl["seed"])
    n = spec["n"]
    centers, radii = [], []
    if spec.get("fixed") is not None:
        for (x, y, z, r) in spec["fixed"]:
            centers.append([x, y, z if dim == 3 else 0.0])
            radii.append(r)
    elif spec.get("center") == "jitter":
        # one nucleus at the grid centre plus a seeded sub-cell offset in [-1/2, 1/2)
        r = spec["r_min"]
        c = [0.5 * (wl["nx"] - 1) + 0.5, 0.5 * (wl["ny"] - 1) + 0.5, 0.0]
        c = [math.floor(c[0]), math.floor(c[1]), 0.0]
        for a in range(dim):
            c[a] += rng.uniform() - 0.5
        if dim == 3:
            c[2] = math.floor(0.5 * wl["nz"]) + rng.uniform() - 0.5
        centers.append(c)
        radii.append(r)
    else:
        acc = np.zeros((0, 3))
        accr = np.zeros(0)
        attempts = 0
        while len(radii) < n:
            attempts += 1
            if attempts > 1_000_000:
                raise ValueError(f"could not place {n} nuclei (placed {len(radii)})")
            r = rng.uniform_range(spec["r_min"], spec["r_max"])
            lo, hi = _liquid_box(wl, r)
            c = [0.0, 0.0, 0.0]
            for a in range(dim):
                c[a] = rng.uniform_range(lo[a], hi[a])
            if len(radii):
                d2 = ((acc[:, :dim] - np.array(c[:dim])) ** 2).sum(axis=1)
                if spec.get("min_sep") is None:
                    need = accr + r + 4.0
                else:
                    need = np.full(len(accr), float(spec["min_sep"]))
                if np.any(d2 < need * need):
                    continue
            centers.append(c)
            radii.append(r)
            acc = np.vstack([acc, np.array(c)[None, :]])
            accr = np.append(accr, r)
    centers = np.array(centers, dtype=np.float64).reshape(-1, 3)
    radii = np.array(radii, dtype=np.float64)
    if spec.get("p0") is not None:
        p0 = np.full(len(radii), float(spec["p0"]))
    else:
        # Initial nucleus pressure: ambient plus the Laplace jump of a sphere (3D)
        # or a circle (2D) of the nucleus radius.
        jump = (2.0 if dim == 3 else 1.0) * wl["sigma"] / radii
        p0 = wl["p_atm"] + jump
    return centers, radii, p0


def batch_workloads(seed: int = 5, n: int = 48, sizes=(64, 96, 128, 160), precision: str = "f16s_g16",
                    curvature: str = "mlp"):
    """The batched ensemble: n independent 3D foaming domains with edge lengths drawn
    uniformly from `sizes`, Poisson(0.02 per 1000 cells) nuclei of radius U[2,4],
    supersaturation U[1.2, 2.0] and relaxation time U[0.6, 1.0]; binary16 storage and
    the learned curvature by default. Domain k places its nuclei with seed
    SplitMix64(seed) -> k-th draw."""
    rng = SplitMix64(seed)
    out = []
    for k in range(n):
        edge = sizes[min(len(sizes) - 1, int(rng.uniform() * len(sizes)))]
        mean = 0.02 * edge ** 3 / 1000.0
        # Poisson by inversion of the cumulative distribution
        u, kk, pk = rng.uniform(), 0, math.exp(-mean)
        cdf = pk
        while u > cdf and kk < 100000:
            kk += 1
            pk *= mean / kk
            cdf += pk
        S0 = rng.uniform_range(1.2, 2.0)
        tau = rng.uniform_range(0.6, 1.0)
        dseed = rng.next_u64() & 0x7FFFFFFF
        out.append(_mk(
            name=f"batch{k:02d}_{edge}", dim=3, nx=edge, ny=edge, nz=edge, precision=precision,
            tau=tau, sigma=5e-4, S0=S0, k_pi=0.0, steps=3000, seed=dseed, curvature=curvature,
            max_ids=4096, nuclei=dict(n=max(1, kk), r_min=2.0, r_max=4.0, min_sep=None),
        ))
    return out
