"""Helpers that run the oracle and the GPU library on the same seeded input and compare."""
import numpy as np

G, I, L, W = 0, 1, 2, 3


def fluid_mask(T):
    return (T == L) | (T == I)


def rel_maxdiff(a, b, mask):
    """max |a - b| over masked cells divided by max |b| (populations: leading axis Q)."""
    if a.ndim == mask.ndim + 1:
        a = a[:, mask]
        b = b[:, mask]
    else:
        a = a[mask]
        b = b[mask]
    if a.size == 0:
        return 0.0
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


def compare_states(gpu, orc, tol_pop, tol_cell, exact_types=True, tol_geom=None):
    """Compare a GPU Sim and an Oracle; returns a dict of the measured differences.

    tol_geom bounds the curvature and the disjoining pressure of the interface cells
    (default: tol_cell). In 3D binary64 they carry 1e-10: the least-squares fit amplifies
    the last-bit differences of cbrt / acos in the PLIC inverse (libm on the host, the
    device library on the GPU)."""
    if tol_geom is None:
        tol_geom = tol_cell
    Tg, To = gpu.read("type"), orc.read("type")
    out = {}
    out["type_mismatch"] = int((Tg != To).sum())
    Lg, Lo = gpu.read("label"), orc.read("label")
    out["label_mismatch"] = int((Lg != Lo).sum())
    if exact_types:
        assert out["type_mismatch"] == 0, f"{out['type_mismatch']} cell types differ"
        assert out["label_mismatch"] == 0, f"{out['label_mismatch']} bubble labels differ"
    m = fluid_mask(To) & fluid_mask(Tg)
    mi = (To == I) & (Tg == I)
    out["f"] = rel_maxdiff(gpu.read("f"), orc.read("f"), m)
    out["g"] = rel_maxdiff(gpu.read("g"), orc.read("g"), m)
    for name in ("mass", "alpha", "rho", "kappa", "pi"):
        out[name] = rel_maxdiff(gpu.read(name), orc.read(name), mi)
    assert out["f"] <= tol_pop, out
    assert out["g"] <= tol_pop, out
    for name in ("mass", "alpha", "rho"):
        assert out[name] <= tol_cell, (name, out)
    for name in ("kappa", "pi"):
        assert out[name] <= tol_geom, (name, out)
    return out


def compare_bubbles(gpu, orc, tol):
    bg, bo = gpu.bubbles(), orc.bubbles()
    assert list(bg["id"]) == list(bo["id"]), (bg["id"], bo["id"])
    for k in ("V", "m", "p"):
        if bo[k].size:
            d = np.abs(bg[k] - bo[k]) / np.maximum(np.abs(bo[k]), 1e-300)
            assert d.max() <= tol, (k, d.max())
    lg, lo = gpu.ledgers(), orc.ledgers()
    assert lg["next_id"] == lo["next_id"]
    for k in ("lost_liquid", "atm_gas", "collapsed_gas"):
        assert abs(lg[k] - lo[k]) <= tol * max(abs(lo[k]), 1e-12), (k, lg[k], lo[k])
