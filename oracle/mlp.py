"""Learned curvature closure: FP64 reference (test infrastructure only).

What is computed (the closure the library trains and runs on the GPU):
  * training stencils: 5x5x5 fill fractions around a cell cut by the surface of a
    voxelised sphere or ellipsoid (semi-axes log-uniform in [2, 40] cells, random
    rotation, random sub-cell position of the surface point, fill noise N(0, 0.01) on cut
    cells), labelled with the exact mean curvature of the surface point closest to the
    centre cell's centre (positive when the gas is inside, as for a bubble);
  * canonicalisation: the cube symmetry (axis flips, then axis permutation) that maps the
    central-difference gradient of the stencil to m_x >= m_y >= m_z >= 0;
  * network 125-64-64-1 with GELU, inputs and hidden activations rounded to bfloat16
    before each product (as the GPU does), accumulation in FP64 here; kappa = out / 8.
Random numbers: SplitMix64 (Steele, Lea & Flood 2014) as a counter-based stream per
sample and attempt; U(0,1) = (u >> 11) 2^-53; normals by the cosine branch of Box-Muller.
"""
from __future__ import annotations

import math

import numpy as np

MASK = (1 << 64) - 1
GOLD = 0x9E3779B97F4A7C15
NFEAT = 125
NPAD = 128
H = 64
LOG2, LOG40 = math.log(2.0), math.log(40.0)


# ---------------------------------------------------------------- random numbers
class Stream:
    """SplitMix64 stream of one sample attempt: state = seed + (counter + 1) * C."""

    def __init__(self, seed, sample, attempt):
        ctr = (sample * 16 + attempt + 1) & MASK
        self.s = (seed + ctr * 0xD1B54A32D192ED03) & MASK

    def u64(self):
        self.s = (self.s + GOLD) & MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    def uniform(self):
        return (self.u64() >> 11) * (2.0 ** -53)

    def normal(self):
        u1 = self.uniform()
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


def _rotation(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_mean_curvature(q, a):
    """|H| at a point q of x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 (textbook closed form)."""
    a2 = a * a
    num = abs(q @ q - a2.sum())
    s = (q * q / (a2 * a2)).sum()
    return num / (2.0 * a2.prod() * s ** 1.5)


def closest_point(o, a, iters=200):
    """point of the ellipsoid closest to o: q_i = o_i a_i^2 / (a_i^2 + t) with
    sum (q_i / a_i)^2 = 1, a decreasing function of t on (-min a_i^2, inf); bisection"""
    a2 = a * a

    def g(t):
        return (((o * a) / (a2 + t)) ** 2).sum() - 1.0

    lo = -a2.min() * (1 - 1e-15)
    hi = max(1.0, float(np.abs(o).max() * a.max()))
    while g(hi) > 0:
        hi *= 2
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    t = 0.5 * (lo + hi)
    return o * a2 / (a2 + t)


def _inside_frac(cell, c, Rm, a):
    """liquid-independent: fraction of the cell inside the body (27-point test, then
    10^3 midpoint sub-samples for cut cells)"""
    def F(pts):
        yb = (pts - c) @ Rm  # body frame: R^T (x - c)
        return ((yb / a) ** 2).sum(axis=-1) - 1.0

    o = np.array([-0.5, 0.0, 0.5])
    g = np.stack(np.meshgrid(o, o, o, indexing="ij"), -1).reshape(-1, 3) + cell
    f = F(g)
    if np.all(f < 0):
        return 1.0
    if np.all(f > 0):
        return 0.0
    s = (np.arange(10) + 0.5) / 10 - 0.5
    sub = np.stack(np.meshgrid(s, s, s, indexing="ij"), -1).reshape(-1, 3) + cell
    return float((F(sub) < 0).sum()) / 1000.0


def generate(seed, first, n, noise=0.01, geometry=None):
    """stencils [n, 125] (dz outer, dx inner, offsets -2..2) and exact curvature [n];
    with a list as geometry, each sample's body is appended to it as a dict (centre c
    relative to the centre cell's centre, unit quaternion q = (w, x, y, z) of the body
    frame, semi-axes a, gas_inside) so that tests can rebuild the stencil and its label
    independently"""
    X = np.zeros((n, NFEAT))
    K = np.zeros(n)
    offs = np.arange(-2, 3)
    cells = np.stack(np.meshgrid(offs, offs, offs, indexing="ij"), -1).reshape(-1, 3)[:, ::-1]
    for k in range(n):
        sample = first + k
        for attempt in range(16):
            st = Stream(seed, sample, attempt)
            sphere = st.uniform() < 0.5
            if sphere:
                r = math.exp(LOG2 + st.uniform() * (LOG40 - LOG2))
                a = np.array([r, r, r])
            else:
                a = np.array([math.exp(LOG2 + st.uniform() * (LOG40 - LOG2)) for _ in range(3)])
            qv = np.array([st.normal() for _ in range(4)])
            qv /= np.linalg.norm(qv)
            Rm = _rotation(qv)
            d = np.array([st.normal() for _ in range(3)])
            pb = d / math.sqrt(((d / a) ** 2).sum())
            u = np.array([st.uniform() - 0.5 for _ in range(3)])
            gas_inside = st.uniform() < 0.5
            c = u - Rm @ pb
            frac = np.array([_inside_frac(cl.astype(float), c, Rm, a) for cl in cells])
            alpha = 1.0 - frac if gas_inside else frac
            if not (0.0 < alpha[62] < 1.0):
                continue
            ob = Rm.T @ (-c)
            qc = closest_point(ob, a)
            kap = ellipsoid_mean_curvature(qc, a)
            if not gas_inside:
                kap = -kap
            if abs(kap) > 0.5:
                continue
            for j in range(NFEAT):
                if 0.0 < alpha[j] < 1.0:
                    alpha[j] = min(1.0, max(0.0, alpha[j] + noise * st.normal()))
            X[k] = alpha
            K[k] = kap
            if geometry is not None:
                geometry.append(dict(c=c.copy(), q=qv.copy(), a=a.copy(), gas_inside=bool(gas_inside)))
            break
        else:
            raise RuntimeError(f"sample {sample}: no valid attempt")
    return X, K


# ---------------------------------------------------------------- canonical form
def canonicalise(X):
    """apply to each stencil the symmetry mapping its central gradient to
    m_x >= m_y >= m_z >= 0 (flip negative axes, then sort axes by |m| descending,
    lower axis first on ties)"""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 5, 5, 5)  # [z][y][x]
    out = np.empty_like(X)
    for b in range(X.shape[0]):
        s = X[b]
        g = np.array([0.5 * (s[2, 2, 3] - s[2, 2, 1]),
                      0.5 * (s[2, 3, 2] - s[2, 1, 2]),
                      0.5 * (s[3, 2, 2] - s[1, 2, 2])])
        t = s
        for ax, arr_axis in ((0, 2), (1, 1), (2, 0)):
            if g[ax] < 0:
                t = np.flip(t, axis=arr_axis)
        ag = np.abs(g)
        order = sorted(range(3), key=lambda i: (-ag[i], i))  # new axis a <- old axis order[a]
        # array axes are (z, y, x) = (2, 1, 0); new array axis for new lattice axis a is 2 - a
        t = np.transpose(t, axes=[2 - order[2], 2 - order[1], 2 - order[0]])
        out[b] = t
    return out.reshape(-1, NFEAT)


# ---------------------------------------------------------------- network
def bf16(x):
    """round to bfloat16 (nearest even) through binary32, as the GPU does"""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def unpack(theta):
    """flat parameter vector (binary32 master layout of the library) -> tensors"""
    t = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = t[o:o + NPAD * H].reshape(NPAD, H); o += NPAD * H
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + H * H].reshape(H, H); o += H * H
    b2 = t[o:o + H]; o += H
    W3 = t[o:o + H]; o += H
    b3 = t[o]; o += 1
    return W1, b1, W2, b2, W3, b3


NPARAM = NPAD * H + H + H * H + H + H + 1


def forward(theta, Xc, rounding=True):
    """Xc: canonical stencils [B,125]; returns (out, cache); kappa = out / 8"""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    rd = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    A = np.zeros((Xc.shape[0], NPAD))
    A[:, :NFEAT] = np.clip(Xc, 0.0, 1.0)
    Ab = rd(A)
    W1b, W2b, W3b = rd(W1), rd(W2), rd(W3)
    z1 = Ab @ W1b + b1
    h1 = rd(gelu(z1))
    z2 = h1 @ W2b + b2
    h2 = rd(gelu(z2))
    out = h2 @ W3b + b3
    return out, (Ab, W1b, W2b, W3b, z1, h1, z2, h2)


def loss_and_grad(theta, Xc, target, rounding=True):
    """mean squared error of out against target (= 8 kappa) and its gradient; the
    bfloat16 roundings pass gradients straight through"""
    out, (Ab, W1b, W2b, W3b, z1, h1, z2, h2) = forward(theta, Xc, rounding)
    B = Xc.shape[0]
    r = out - target
    loss = float((r * r).mean())
    dout = 2.0 * r / B
    dW3 = h2.T @ dout
    db3 = dout.sum()
    dz2 = np.outer(dout, W3b) * gelu_grad(z2)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2b.T) * gelu_grad(z1)
    dW1 = Ab.T @ dz1
    db1 = dz1.sum(0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3]])
    return loss, g


def init_params(seed):
    """uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases; padded inputs
    carry zero weights"""
    st = Stream(seed, 0, 0)
    th = np.zeros(NPARAM)
    W1, b1, W2, b2, W3, b3 = unpack(th)
    vals = []
    for fan, shape in ((NFEAT, (NPAD, H)), (H, (H, H)), (H, (H,))):
        lim = 1.0 / math.sqrt(fan)
        n = int(np.prod(shape))
        vals.append(np.array([(2.0 * st.uniform() - 1.0) * lim for _ in range(n)]).reshape(shape))
    vals[0][NFEAT:, :] = 0.0
    return np.concatenate([vals[0].ravel(), np.zeros(H), vals[1].ravel(), np.zeros(H),
                           vals[2].ravel(), [0.0]])
