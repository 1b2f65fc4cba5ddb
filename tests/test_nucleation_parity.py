"""The library's nucleation-site sampler (mf_poisson_nuclei, host code behind the C ABI)
against the oracle's (Sec. 3.4): identical sites bit for bit on the same seeds, grids and
probability fields; argument checks. No GPU is involved."""
import os

import numpy as np
import pytest

from oracle.nucleation import poisson_nuclei as oracle_nuclei
from synth.workloads import _mk


def _lib_ready():
    from paper_1908_04262_amd.mifoam import LIBPATH
    return os.path.exists(LIBPATH)


def _field(kind, n):
    nx, ny, nz = n
    if kind is None:
        return None
    rng = np.random.default_rng(3)
    if kind == "random":
        return rng.uniform(0, 1, (nz, ny, nx)).astype(np.float32)
    P = np.ones((nz, ny, nx), np.float32)
    P[:, :, nx // 2:] = 0.25
    P[:, : ny // 3, :] = 0.0
    return P


@pytest.mark.parametrize("dim,n,periodic,gas_from,kind,radii,seed", [
    (2, (90, 70, 1), (0, 0, 0), 55, None, (2.0, 4.0), 1),
    (2, (96, 64, 1), (1, 0, 0), -1, "random", (1.5, 3.5), 2),
    (3, (36, 30, 40), (0, 0, 0), 30, "halves", (2.0, 4.0), 3),
    (3, (28, 28, 28), (1, 1, 1), -1, "random", (2.0, 3.0), 4),
    (3, (40, 24, 24), (0, 1, 0), 20, None, (3.0, 3.0), 5),
])
def test_sites_match_oracle(dim, n, periodic, gas_from, kind, radii, seed):
    if not _lib_ready():
        pytest.skip("libmifoam.so not built")
    from paper_1908_04262_amd import poisson_nuclei
    wl = _mk(name="nuc", dim=dim, nx=n[0], ny=n[1], nz=n[2], periodic=list(periodic), gas_from=gas_from,
             nuclei=None)
    P = _field(kind, (n[0], n[1], n[2] if dim == 3 else 1))
    for max_n in (100000, 9):
        c_lib, r_lib = poisson_nuclei(wl, P, max_n, radii[0], radii[1], 1.0, 30, seed)
        c_or, r_or = oracle_nuclei(dim, n, periodic, gas_from, None if P is None else P.ravel(), max_n,
                                   radii[0], radii[1], 1.0, 30, seed)
        assert len(r_lib) == len(r_or) > 0
        assert np.array_equal(np.asarray(r_or), r_lib)
        assert np.array_equal(np.asarray(c_or), c_lib)


def test_argument_checks():
    if not _lib_ready():
        pytest.skip("libmifoam.so not built")
    from paper_1908_04262_amd import MifoamError, poisson_nuclei
    wl = _mk(name="nuc", dim=2, nx=40, ny=40, nz=1, gas_from=-1, nuclei=None)
    for kw in (dict(r_min=0.0), dict(r_min=3.0, r_max=2.0), dict(gap=-1.0), dict(attempts=0)):
        with pytest.raises(MifoamError):
            poisson_nuclei(wl, **kw)
    bad = np.ones((40, 40), np.float32)
    bad[3, 3] = 1.5
    with pytest.raises(MifoamError):
        poisson_nuclei(wl, bad)
    c, r = poisson_nuclei(wl, max_n=0)
    assert len(r) == 0
