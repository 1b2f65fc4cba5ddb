"""ctypes wrapper around the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FIELDS = dict(type=0, label=1, rho=2, ux=3, uy=4, uz=5, alpha=6, mass=7, conc=8,
              kappa=9, pi=10, f=11, g=12)

TYPE_G, TYPE_I, TYPE_L, TYPE_W = 0, 1, 2, 3


class OrParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("periodic", C.c_int32 * 3), ("gas_from", C.c_int32), ("rheology", C.c_int32),
        ("cleanup", C.c_int32), ("max_ids", C.c_int32),
        ("tau", C.c_double), ("D", C.c_double), ("sigma", C.c_double), ("kH", C.c_double),
        ("RT", C.c_double), ("k_pi", C.c_double), ("d_max", C.c_double),
        ("p_atm", C.c_double), ("q", C.c_double), ("eps", C.c_double), ("S0", C.c_double),
        ("pl_n", C.c_double), ("pl_nu_ref", C.c_double), ("pl_gdot_ref", C.c_double),
        ("tau_min", C.c_double), ("tau_max", C.c_double), ("accel", C.c_double * 3),
        ("cy_tau0", C.c_double), ("cy_tau_inf", C.c_double), ("cy_lambda", C.c_double),
        ("cy_a", C.c_double), ("cy_n", C.c_double), ("flux_mode", C.c_int32),
    ]


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(HERE, "liboracle.so")
    src = os.path.join(HERE, "fslbm_oracle.c")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        from .build import build
        build()
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.or_create.restype = vp
    lib.or_create.argtypes = [C.POINTER(OrParams)]
    lib.or_destroy.argtypes = [vp]
    lib.or_error.restype = C.c_char_p
    lib.or_error.argtypes = [vp]
    lib.or_nucleate.argtypes = [vp, C.c_int, vp, vp, vp]
    lib.or_step.argtypes = [vp, C.c_int]
    lib.or_ncells.restype = C.c_int64
    lib.or_ncells.argtypes = [vp]
    lib.or_read.argtypes = [vp, C.c_int, vp]
    lib.or_write.argtypes = [vp, C.c_int, vp]
    lib.or_set_bubble.argtypes = [vp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int]
    lib.or_geometry.argtypes = [vp]
    lib.or_bubbles.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    lib.or_ledgers.argtypes = [vp, vp]
    for fn in ("or_feq", "or_geq"):
        getattr(lib, fn).restype = C.c_double
        getattr(lib, fn).argtypes = [vp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.or_curvature.restype = C.c_double
    lib.or_curvature.argtypes = [vp, C.c_int64]
    lib.or_disjoining.restype = C.c_double
    lib.or_disjoining.argtypes = [vp, C.c_int64]
    lib.or_plic_offset.restype = C.c_double
    lib.or_plic_offset.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.or_powerlaw_tau.restype = C.c_double
    lib.or_powerlaw_tau.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double]
    lib.or_lattice.argtypes = [vp, vp, vp, vp, vp]
    lib.or_cy_tau.restype = C.c_double
    lib.or_cy_tau.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double]
    lib.or_powerlaw_tau_iter.restype = C.c_double
    lib.or_powerlaw_tau_iter.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double, C.c_int]
    lib.or_relabel.argtypes = [vp]
    lib.or_traverse.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, vp]
    _LIB = lib
    return lib


def make_params(wl: dict) -> OrParams:
    p = OrParams()
    p.dim = wl["dim"]
    p.nx, p.ny = wl["nx"], wl["ny"]
    p.nz = wl["nz"] if wl["dim"] == 3 else 1
    for a in range(3):
        p.periodic[a] = int(wl["periodic"][a])
    p.gas_from = int(wl["gas_from"])
    p.rheology = {"newtonian": 0, "power_law": 1, "carreau_yasuda": 2}[wl["rheology"]]
    p.cleanup = int(wl["cleanup"])
    p.max_ids = int(wl["max_ids"])
    for k in ("tau", "D", "sigma", "kH", "RT", "k_pi", "d_max", "p_atm", "q", "eps", "S0",
              "pl_n", "pl_nu_ref", "pl_gdot_ref", "tau_min", "tau_max"):
        setattr(p, k, float(wl[k]))
    for a, v in enumerate(wl.get("accel", (0.0, 0.0, 0.0))):
        p.accel[a] = float(v)
    for k, d in (("cy_tau0", 0.8), ("cy_tau_inf", 0.8), ("cy_lambda", 0.0), ("cy_a", 2.0), ("cy_n", 1.0)):
        setattr(p, k, float(wl.get(k, d)))
    p.flux_mode = {"ledger": 0, "paper": 1}[wl.get("flux_mode", "ledger")]
    return p


class Oracle:
    """One simulation state held by the C oracle."""

    def __init__(self, wl: dict):
        self.lib = load_library()
        self.wl = dict(wl)
        self.params = make_params(wl)
        self.h = self.lib.or_create(C.byref(self.params))
        self.N = int(self.lib.or_ncells(self.h))
        self.dim = wl["dim"]
        self.Q = 9 if self.dim == 2 else 19
        self.Qg = 5 if self.dim == 2 else 7
        self.shape = (self.params.nz, self.params.ny, self.params.nx)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.or_destroy(h)
            self.h = None

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError("oracle: " + self.lib.or_error(self.h).decode())

    def nucleate(self, centers, radii, p0):
        centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        radii = np.ascontiguousarray(radii, dtype=np.float64)
        p0 = np.ascontiguousarray(p0, dtype=np.float64)
        self._check(self.lib.or_nucleate(self.h, len(radii), centers.ctypes.data,
                                         radii.ctypes.data, p0.ctypes.data))

    def step(self, n=1):
        self._check(self.lib.or_step(self.h, int(n)))

    def read(self, name):
        fid = FIELDS[name]
        if name == "type":
            out = np.empty(self.N, np.uint8)
        elif name == "label":
            out = np.empty(self.N, np.int32)
        elif name == "f":
            out = np.empty(self.Q * self.N, np.float64)
        elif name == "g":
            out = np.empty(self.Qg * self.N, np.float64)
        else:
            out = np.empty(self.N, np.float64)
        self._check(self.lib.or_read(self.h, fid, out.ctypes.data))
        if name == "f":
            return out.reshape((self.Q,) + self.shape)
        if name == "g":
            return out.reshape((self.Qg,) + self.shape)
        return out.reshape(self.shape)

    def write(self, name, arr):
        fid = FIELDS[name]
        dt = {"type": np.uint8, "label": np.int32}.get(name, np.float64)
        a = np.ascontiguousarray(arr, dtype=dt).ravel()
        self._check(self.lib.or_write(self.h, fid, a.ctypes.data))

    def set_bubble(self, bid, m, V, p, alive=True):
        self._check(self.lib.or_set_bubble(self.h, bid, m, V, p, int(alive)))

    def geometry(self):
        self.lib.or_geometry(self.h)

    def bubbles(self):
        cap = self.params.max_ids
        ids = np.empty(cap, np.int32)
        m = np.empty(cap)
        V = np.empty(cap)
        p = np.empty(cap)
        k = self.lib.or_bubbles(self.h, cap, ids.ctypes.data, m.ctypes.data, V.ctypes.data,
                                p.ctypes.data)
        return dict(id=ids[:k].copy(), m=m[:k].copy(), V=V[:k].copy(), p=p[:k].copy())

    def ledgers(self):
        out = np.empty(5)
        self.lib.or_ledgers(self.h, out.ctypes.data)
        return dict(lost_liquid=out[0], atm_gas=out[1], collapsed_gas=out[2],
                    next_id=int(out[3]), step=int(out[4]))

    def feq(self, i, rho, u):
        u = list(u) + [0.0] * (3 - len(u))
        return self.lib.or_feq(self.h, i, rho, *u)

    def geq(self, i, c, u):
        u = list(u) + [0.0] * (3 - len(u))
        return self.lib.or_geq(self.h, i, c, *u)

    def lattice(self):
        e = np.zeros((19, 3), np.int32)
        w = np.zeros(19)
        wg = np.zeros(7)
        opp = np.zeros(19, np.int32)
        Q = self.lib.or_lattice(self.h, e.ctypes.data, w.ctypes.data, wg.ctypes.data,
                                opp.ctypes.data)
        return e[:Q], w[:Q], wg[: self.Qg], opp[:Q]

    def relabel(self):
        self._check(self.lib.or_relabel(self.h))

    def curvature(self, cell):
        return self.lib.or_curvature(self.h, int(cell))

    def disjoining(self, cell):
        return self.lib.or_disjoining(self.h, int(cell))

    def cell(self, x, y, z=0):
        return x + self.params.nx * (y + self.params.ny * z)

    def totals(self):
        """Liquid mass (sum of rho over L plus M over I), dissolved and bubble gas."""
        T = self.read("type")
        f = self.read("f")
        rho_all = f.sum(axis=0)
        M = self.read("mass")
        liquid = rho_all[T == TYPE_L].sum() + M[T == TYPE_I].sum()
        conc = self.read("conc")
        dissolved = conc[(T == TYPE_L) | (T == TYPE_I)].sum()
        b = self.bubbles()
        led = self.ledgers()
        return dict(liquid=liquid, dissolved=dissolved, bubble_gas=b["m"].sum(), **led)


def plic_offset(dim, alpha, m):
    lib = load_library()
    m = list(m) + [0.0] * (3 - len(m))
    return lib.or_plic_offset(dim, alpha, m[0], m[1], m[2])


def powerlaw_tau(wl, rho, pn, iters=None):
    lib = load_library()
    p = make_params(wl)
    if iters is None:
        return lib.or_powerlaw_tau(C.byref(p), rho, pn)
    return lib.or_powerlaw_tau_iter(C.byref(p), rho, pn, int(iters))


def cy_tau(wl, rho, pn):
    """Carreau-Yasuda relaxation time of the oracle (Eq. carreauTau)."""
    lib = load_library()
    return lib.or_cy_tau(C.byref(make_params(wl)), rho, pn)


def traverse(dim, m, dmax):
    lib = load_library()
    m = list(m) + [0.0] * (3 - len(m))
    out = np.zeros(3 * dmax, np.int32)
    lib.or_traverse(dim, m[0], m[1], m[2], dmax, out.ctypes.data)
    return out.reshape(dmax, 3)
