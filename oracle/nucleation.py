"""Nucleation sites from a nucleation probability field by Poisson-disk sampling (Sec. 3.4):
plain Python reference.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU-baseline leg
use this module; it shares no code with the library.

Reading of Sec. 3.4 (the paper names the field, Poisson-disk sampling after the cited
active-list method and a minimum distance of "the radius plus one cell"):
  * sites are sphere (disk) centres with radii drawn uniformly in [r_min, r_max]; two sites
    keep |x_i - x_j| >= r_i + r_j + gap (gap = one cell by default), so that the spheres do
    not overlap and a liquid film of at least one cell separates them, which is the purpose
    the paper gives;
  * a sphere lies inside the liquid region: at least one cell from every wall layer of a
    closed axis and from the headspace (cells whose last coordinate is >= gas_from);
    distances wrap on periodic axes (minimum image);
  * the active-list scheme first fills the liquid region: the first site is the first of up to
    10000 uniform candidates that fits; then, while sites are active, an active site i is drawn
    uniformly and up to `attempts` candidates are tried in the shell [d, 2d],
    d = r_i + r_new + gap, around it (uniform direction, uniform distance); the first candidate
    that fits is placed and becomes active, and a site whose attempts all fail is retired;
  * the field P (one value per cell, in [0, 1]) then thins the filled set: in placement order,
    a site whose nearest cell has probability P is kept with probability P, until max_n are
    kept. Thinning keeps the minimum distance and makes the expected number of sites in a
    region P times what the filled set holds there (filtering candidates instead would hardly
    thin, since the attempts retry until something fits).
Random numbers: one SplitMix64 stream (Steele, Lea and Flood 2014) from the seed, u = (z >> 11)
2^-53 in [0, 1), drawn in a fixed order (below); directions by rejection from the cube
[-1, 1]^d (accept 1e-4 < |v|^2 <= 1), so no trigonometric function enters.
Pinned by the distance and containment properties on every pair and site, by P = 0 regions
staying empty, by the packing fraction of the filled set and by the density of thinned
regions.
"""
import math

MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed):
        self.s = seed & MASK

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    def u(self):
        return (self.next() >> 11) * 2.0 ** -53


def poisson_nuclei(dim, n, periodic, gas_from, prob, max_n, r_min, r_max, gap, attempts, seed):
    """n = (nx, ny, nz); prob: sequence of N floats in cell order (x fastest) or None.
    Returns (centres [k][3], radii [k]) in placement order."""
    nx, ny, nz = n[0], n[1], (n[2] if dim == 3 else 1)
    ext = [nx, ny, nz][:dim]
    per = [bool(periodic[a]) for a in range(dim)]
    last = dim - 1
    rng = SplitMix64(seed)

    def inside(x, r):
        for a in range(dim):
            if per[a]:
                continue
            lo = 1.0 + r + 1.0
            hi = (ext[a] - 2) - r - 1.0
            if a == last and gas_from >= 0:
                hi = min(hi, (gas_from - 1) - r - 1.0)
            if x[a] < lo or x[a] > hi:
                return False
        return True

    def dist2(x, y):
        s = 0.0
        for a in range(dim):
            d = x[a] - y[a]
            if per[a]:
                L = float(ext[a])
                d = d - L * math.floor(d / L + 0.5)
            s = s + d * d
        return s

    def far(x, r, sites, radii):
        for y, ry in zip(sites, radii):
            m = r + ry + gap
            if dist2(x, y) < m * m:
                return False
        return True

    def pval(x):
        if prob is None:
            return 1.0
        c = [int(math.floor(x[a] + 0.5)) for a in range(dim)]
        for a in range(dim):
            c[a] = c[a] % ext[a] if per[a] else min(max(c[a], 0), ext[a] - 1)
        idx = c[0] + nx * (c[1] + (ny * c[2] if dim == 3 else 0))
        return float(prob[idx])

    def wrap(x):
        return [x[a] - ext[a] * math.floor(x[a] / ext[a]) if per[a] else x[a] for a in range(dim)]

    sites, radii, active = [], [], []
    if max_n <= 0:
        return [], []
    # first site: uniform candidates over the box
    for _ in range(10000):
        x = [rng.u() * ext[a] for a in range(dim)]
        r = r_min + rng.u() * (r_max - r_min)
        if inside(x, r):
            sites.append(x)
            radii.append(r)
            active.append(0)
            break
    while active:
        k = int(rng.u() * len(active))
        i = active[k]
        placed = False
        for _ in range(attempts):
            r = r_min + rng.u() * (r_max - r_min)
            while True:
                v = [2.0 * rng.u() - 1.0 for _ in range(dim)]
                q = 0.0
                for a in range(dim):
                    q = q + v[a] * v[a]
                if 1e-4 < q <= 1.0:
                    break
            nv = math.sqrt(q)
            d = radii[i] + r + gap
            rho = d * (1.0 + rng.u())
            x = wrap([sites[i][a] + (rho / nv) * v[a] for a in range(dim)])
            if inside(x, r) and far(x, r, sites, radii):
                sites.append(x)
                radii.append(r)
                active.append(len(sites) - 1)
                placed = True
                break
        if not placed:
            active[k] = active[-1]
            active.pop()
    # thinning by the probability field, in placement order
    kept_c, kept_r = [], []
    for x, r in zip(sites, radii):
        if len(kept_r) >= max_n:
            break
        pu = rng.u()
        if pu < pval(x):
            kept_c.append(x + [0.0] * (3 - dim))
            kept_r.append(r)
    return kept_c, kept_r
