"""Pins of the oracle's nucleation-site sampler (Sec. 3.4: nucleation probability field and
Poisson-disk sampling).

N1 every pair of sites keeps |x_i - x_j| >= r_i + r_j + gap (brute force over all pairs, with
   the minimum image on periodic axes) and every sphere lies inside the liquid region;
N2 regions where the field is zero receive no site;
N3 with equal radii and the field at one, the packing fraction of the centre-distance disks
   lies between 0.40 (the active-list method fills to about 0.49 in 2D; a sampler that
   misplaced its shells would leave wide gaps) and the hexagonal bound 0.9069;
N4 a field of 0.2 over half the box keeps about a fifth of the sites the other half keeps
   (binomial thinning of the filled set);
N5 the radii lie in [r_min, r_max] and max_n caps the count.
"""
import itertools
import math

import numpy as np
import pytest

from oracle.nucleation import poisson_nuclei


def _check(dim, n, periodic, gas_from, cen, rad, gap):
    ext = [n[0], n[1], n[2]][:dim]
    for i, j in itertools.combinations(range(len(rad)), 2):
        d2 = 0.0
        for a in range(dim):
            d = cen[i][a] - cen[j][a]
            if periodic[a]:
                d -= ext[a] * round(d / ext[a])
            d2 += d * d
        assert math.sqrt(d2) >= rad[i] + rad[j] + gap - 1e-12, (i, j)
    for c, r in zip(cen, rad):
        for a in range(dim):
            if periodic[a]:
                assert 0.0 <= c[a] < ext[a]
                continue
            top = ext[a] - 3
            if a == dim - 1 and gas_from >= 0:
                top = min(top, gas_from - 2)
            assert c[a] - r >= 2.0 - 1e-12 and c[a] + r <= top + 1e-12


@pytest.mark.parametrize("dim,n,periodic,gas_from,seed", [
    (2, (120, 90, 1), (0, 0, 0), 70, 1),
    (2, (100, 100, 1), (1, 0, 0), -1, 2),
    (3, (40, 36, 44), (0, 0, 0), 33, 3),
    (3, (32, 32, 32), (1, 1, 0), -1, 4),
])
def test_sites_keep_distance_and_containment(dim, n, periodic, gas_from, seed):
    cen, rad = poisson_nuclei(dim, n, periodic, gas_from, None, 100000, 2.0, 4.0, 1.0, 30, seed)
    assert len(rad) > 10
    _check(dim, n, periodic, gas_from, cen, rad, 1.0)
    assert all(2.0 <= r <= 4.0 for r in rad)
    cap, _ = poisson_nuclei(dim, n, periodic, gas_from, None, 7, 2.0, 4.0, 1.0, 30, seed)
    assert len(cap) == 7 and cap == cen[:7]


def test_zero_probability_regions_stay_empty():
    nx, ny = 160, 120
    P = np.zeros((ny, nx), np.float32)
    P[:, : nx // 2] = 1.0
    P[40:60, 100:120] = 0.7
    cen, rad = poisson_nuclei(2, (nx, ny, 1), (0, 0, 0), -1, P.ravel(), 100000, 1.5, 3.0, 1.0, 30, 9)
    for c in cen:
        cx, cy = int(math.floor(c[0] + 0.5)), int(math.floor(c[1] + 0.5))
        assert P[cy, cx] > 0.0
    assert any(c[0] >= 100 for c in cen)  # the island keeps some of its sites


def test_packing_fraction_equal_radii():
    L, r, gap = 200, 3.0, 1.0
    cen, rad = poisson_nuclei(2, (L, L, 1), (1, 1, 0), -1, None, 100000, r, r, gap, 30, 5)
    d = 2 * r + gap
    phi = len(rad) * math.pi * (d / 2) ** 2 / (L * L)
    assert 0.40 < phi < 0.9069, phi


def test_thinned_half_holds_fewer_sites():
    nx, ny = 240, 120
    P = np.ones((ny, nx), np.float32)
    P[:, nx // 2:] = 0.2
    counts = []
    for seed in (11, 12, 13):
        cen, rad = poisson_nuclei(2, (nx, ny, 1), (1, 1, 0), -1, P.ravel(), 100000, 2.0, 2.0, 1.0, 30, seed)
        left = sum(1 for c in cen if c[0] < nx / 2)
        counts.append((left, len(cen) - left))
    # each site of the thinned half survives with probability 0.2: about 0.2 of the other half
    for lf, rt in counts:
        assert 0.1 * lf < rt < 0.32 * lf, counts
