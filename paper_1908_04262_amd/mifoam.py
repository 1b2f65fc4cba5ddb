"""Python binding of libmifoam (argument marshalling only).

Every step of the method runs in the HIP kernels of libmifoam.so; this module only
converts parameter dictionaries to ``mf_params``, hands the library a device
workspace allocated by PyTorch and the current PyTorch stream, and copies fields back.
Importing fails loudly when the built library is absent.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmifoam.so")

PRECISIONS = {"fp64": 0, "fp32": 1, "f16s": 2, "bf16s": 3, "f16s_g16": 4}
FLUX_MODES = {"ledger": 0, "paper": 1}
FIELDS = dict(type=0, label=1, rho=2, ux=3, uy=4, uz=5, alpha=6, mass=7, conc=8,
              kappa=9, pi=10, f=11, g=12)
STATUS = {0: "MF_OK", -1: "MF_EINVAL", -2: "MF_ENOMEM", -3: "MF_EHIP", -4: "MF_ECAPACITY",
          -5: "MF_ENUMERIC", -6: "MF_ESTATE", -7: "MF_EUNSUPPORTED", -8: "MF_EINTERNAL"}


class MfParams(C.Structure):
    _fields_ = [
        ("struct_size", C.c_size_t),
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("periodic", C.c_int32 * 3), ("gas_from", C.c_int32), ("precision", C.c_int32),
        ("rheology", C.c_int32), ("curvature", C.c_int32), ("cleanup", C.c_int32),
        ("max_ids", C.c_int32),
        ("tau", C.c_double), ("D", C.c_double), ("sigma", C.c_double), ("kH", C.c_double),
        ("RT", C.c_double), ("k_pi", C.c_double), ("d_max", C.c_double),
        ("p_atm", C.c_double), ("q", C.c_double), ("eps", C.c_double), ("S0", C.c_double),
        ("pl_n", C.c_double), ("pl_nu_ref", C.c_double), ("pl_gdot_ref", C.c_double),
        ("tau_min", C.c_double), ("tau_max", C.c_double), ("accel", C.c_double * 3),
        ("cy_tau0", C.c_double), ("cy_tau_inf", C.c_double), ("cy_lambda", C.c_double),
        ("cy_a", C.c_double), ("cy_n", C.c_double), ("flux_mode", C.c_int32),
    ]


class MfBubble(C.Structure):
    _fields_ = [("id", C.c_int32), ("alive", C.c_int32), ("volume", C.c_double),
                ("gas_mass", C.c_double), ("pressure", C.c_double), ("n_cells", C.c_int32),
                ("reserved", C.c_int32), ("centroid", C.c_double * 3)]


class MfTotals(C.Structure):
    _fields_ = [("step", C.c_int64), ("lost_liquid", C.c_double), ("atm_gas", C.c_double),
                ("collapsed_gas", C.c_double), ("next_id", C.c_int32),
                ("n_bubbles", C.c_int32), ("n_interface", C.c_int32), ("status", C.c_int32),
                ("liquid_mass", C.c_double), ("dissolved_gas", C.c_double), ("bubble_gas", C.c_double)]


class MfMlpTrainSpec(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("n_train", C.c_int64), ("n_val", C.c_int64),
                ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("noise", C.c_double), ("data_seed", C.c_uint64)]


# every symbol include/mifoam.h declares
EXPORTS = ["mf_abi_version", "mf_last_error", "mf_workspace_bytes", "mf_create", "mf_destroy",
           "mf_nucleate", "mf_step", "mf_sync", "mf_read_field", "mf_write_field",
           "mf_set_bubble", "mf_refresh", "mf_read_bubbles", "mf_totals_get",
           "mf_profile_enable", "mf_profile_get", "mf_mlp_param_count", "mf_mlp_create",
           "mf_mlp_destroy", "mf_mlp_train", "mf_mlp_get_params", "mf_mlp_set_params",
           "mf_mlp_generate", "mf_mlp_eval", "mf_mlp_eval_noalloc", "mf_mlp_grad", "mf_attach_mlp", "mf_tune",
           "mf_set_sweep_variant", "mf_batch_create", "mf_batch_tune", "mf_batch_step",
           "mf_batch_destroy", "mf_poisson_nuclei", "mf_save", "mf_load", "mf_debug_poke",
           "mf_mlp_save", "mf_mlp_load"]
SWEEP_VARIANTS = 8

_LIB = None


def load_library():
    """Load libmifoam.so from the package directory (built by build.py)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIBPATH):
        raise ImportError(f"libmifoam.so is not built ({LIBPATH}); run __graft_entry__.build()")
    # PyTorch ships its own HIP runtime under the same soname; load it first so that the
    # library and PyTorch (which supplies device memory and streams) share one runtime
    import torch  # noqa: F401
    lib = C.CDLL(LIBPATH)
    vp = C.c_void_p
    lib.mf_abi_version.restype = C.c_int
    lib.mf_last_error.restype = C.c_char_p
    lib.mf_last_error.argtypes = [vp]
    lib.mf_workspace_bytes.argtypes = [C.POINTER(MfParams), C.POINTER(C.c_size_t)]
    lib.mf_create.argtypes = [C.POINTER(MfParams), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.mf_destroy.argtypes = [vp]
    lib.mf_nucleate.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.mf_step.argtypes = [vp, C.c_int32]
    lib.mf_sync.argtypes = [vp]
    lib.mf_read_field.argtypes = [vp, C.c_int32, vp, C.c_size_t, C.c_int32]
    lib.mf_write_field.argtypes = [vp, C.c_int32, vp, C.c_size_t]
    lib.mf_set_bubble.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32]
    lib.mf_refresh.argtypes = [vp, C.c_int32]
    lib.mf_read_bubbles.argtypes = [vp, C.POINTER(MfBubble), C.c_int32, C.POINTER(C.c_int32)]
    lib.mf_totals_get.argtypes = [vp, C.POINTER(MfTotals)]
    lib.mf_profile_enable.argtypes = [vp, C.c_int32]
    lib.mf_profile_get.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.mf_mlp_param_count.restype = C.c_int
    lib.mf_mlp_create.argtypes = [C.c_uint64, C.POINTER(vp)]
    lib.mf_mlp_destroy.argtypes = [vp]
    lib.mf_mlp_train.argtypes = [vp, C.POINTER(MfMlpTrainSpec), vp, C.POINTER(C.c_double)]
    lib.mf_mlp_get_params.argtypes = [vp, vp]
    lib.mf_mlp_set_params.argtypes = [vp, vp]
    lib.mf_mlp_generate.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_double, vp, vp, vp]
    lib.mf_mlp_eval.argtypes = [vp, vp, C.c_int64, vp, vp]
    lib.mf_mlp_eval_noalloc.argtypes = [vp, vp, C.c_int64, vp, vp]
    lib.mf_mlp_grad.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_double), vp]
    lib.mf_attach_mlp.argtypes = [vp, vp]
    lib.mf_tune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), vp]
    lib.mf_poisson_nuclei.argtypes = [C.POINTER(MfParams), vp, C.c_int32, C.c_double, C.c_double, C.c_double,
                                      C.c_int32, C.c_uint64, vp, vp, C.POINTER(C.c_int32)]
    lib.mf_set_sweep_variant.argtypes = [vp, C.c_int32]
    lib.mf_batch_create.argtypes = [C.c_int32, vp, C.POINTER(vp)]
    lib.mf_batch_tune.argtypes = [vp, C.c_int32, vp]
    lib.mf_batch_step.argtypes = [vp, C.c_int32]
    lib.mf_batch_destroy.argtypes = [vp]
    lib.mf_save.argtypes = [vp, C.c_char_p]
    lib.mf_load.argtypes = [vp, C.c_char_p]
    lib.mf_debug_poke.argtypes = [vp, C.c_int32, C.c_int64, C.c_int32, C.c_double]
    lib.mf_mlp_save.argtypes = [vp, C.c_char_p]
    lib.mf_mlp_load.argtypes = [C.POINTER(vp), C.c_char_p]
    _LIB = lib
    return lib


def make_params(wl: dict) -> MfParams:
    p = MfParams()
    p.struct_size = C.sizeof(MfParams)
    p.dim = wl["dim"]
    p.nx, p.ny = wl["nx"], wl["ny"]
    p.nz = wl["nz"] if wl["dim"] == 3 else 1
    for a in range(3):
        p.periodic[a] = int(wl["periodic"][a])
    p.gas_from = int(wl["gas_from"])
    p.precision = PRECISIONS[wl["precision"]]
    p.rheology = {"newtonian": 0, "power_law": 1, "carreau_yasuda": 2}[wl["rheology"]]
    p.curvature = 1 if wl.get("curvature") == "mlp" else 0
    p.cleanup = int(wl["cleanup"])
    p.max_ids = int(wl["max_ids"])
    for k in ("tau", "D", "sigma", "kH", "RT", "k_pi", "d_max", "p_atm", "q", "eps", "S0",
              "pl_n", "pl_nu_ref", "pl_gdot_ref", "tau_min", "tau_max"):
        setattr(p, k, float(wl[k]))
    for a, v in enumerate(wl.get("accel", (0.0, 0.0, 0.0))):
        p.accel[a] = float(v)
    for k, d in (("cy_tau0", 0.8), ("cy_tau_inf", 0.8), ("cy_lambda", 0.0), ("cy_a", 2.0), ("cy_n", 1.0)):
        setattr(p, k, float(wl.get(k, d)))
    p.flux_mode = FLUX_MODES[wl.get("flux_mode", "ledger")]
    return p


class MifoamError(RuntimeError):
    pass


def poisson_nuclei(wl: dict, prob=None, max_n=1 << 20, r_min=2.0, r_max=4.0, gap=1.0, attempts=30, seed=0):
    """Nucleation sites of the grid wl describes, by Poisson-disk sampling of the
    probability field prob (host array of one value per cell, x fastest; None: all ones).
    Returns (centres [n, 3], radii [n]) as float64 arrays; host code only."""
    import numpy as np

    lib = load_library()
    p = make_params(wl)
    pr = None
    if prob is not None:
        pr = np.ascontiguousarray(prob, dtype=np.float32).ravel()
        ncell = int(p.nx) * int(p.ny) * (int(p.nz) if int(p.dim) == 3 else 1)
        if pr.size != ncell:
            raise ValueError(f"prob holds {pr.size} values, the grid {ncell} cells")
    cap = int(max_n)
    cen = np.zeros((max(cap, 1), 3), np.float64)
    rad = np.zeros(max(cap, 1), np.float64)
    n = C.c_int32()
    rc = lib.mf_poisson_nuclei(C.byref(p), None if pr is None else pr.ctypes.data, cap, float(r_min), float(r_max),
                               float(gap), int(attempts), int(seed) & ((1 << 64) - 1), cen.ctypes.data,
                               rad.ctypes.data, C.byref(n))
    if rc != 0:
        raise MifoamError(f"mf_poisson_nuclei failed with status {rc}")
    return cen[: n.value].copy(), rad[: n.value].copy()


class Sim:
    """One foaming domain on one GPU (a libmifoam context)."""

    def __init__(self, wl: dict, device: int = 0):
        import torch

        self.lib = load_library()
        self.wl = dict(wl)
        self.params = make_params(wl)
        self.dim = wl["dim"]
        self.Q = 9 if self.dim == 2 else 19
        self.Qg = 5 if self.dim == 2 else 7
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = int(np.prod(self.shape))
        self.device = torch.device("cuda", device)
        nbytes = C.c_size_t()
        self._check(self.lib.mf_workspace_bytes(C.byref(self.params), C.byref(nbytes)), None)
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._check(self.lib.mf_create(C.byref(self.params), C.c_void_p(self.workspace.data_ptr()),
                                       nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)), None)
        self.h = h

    def _check(self, rc, h="self"):
        if rc != 0:
            handle = None if h is None else self.h
            msg = self.lib.mf_last_error(handle)
            raise MifoamError(f"{STATUS.get(rc, rc)}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            self.lib.mf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nucleate(self, centers, radii, p0):
        c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        r = np.ascontiguousarray(radii, dtype=np.float64)
        p = np.ascontiguousarray(p0, dtype=np.float64)
        self._check(self.lib.mf_nucleate(self.h, len(r), c.ctypes.data, r.ctypes.data, p.ctypes.data))

    def step(self, n: int = 1):
        self._check(self.lib.mf_step(self.h, int(n)))

    def sync(self):
        self._check(self.lib.mf_sync(self.h))

    def read(self, name):
        fid = FIELDS[name]
        if name == "type":
            out = np.empty(self.N, np.uint8)
        elif name == "label":
            out = np.empty(self.N, np.int32)
        elif name == "f":
            out = np.empty(self.Q * self.N)
        elif name == "g":
            out = np.empty(self.Qg * self.N)
        else:
            out = np.empty(self.N)
        self._check(self.lib.mf_read_field(self.h, fid, out.ctypes.data, out.nbytes, 0))
        if name == "f":
            return out.reshape((self.Q,) + self.shape)
        if name == "g":
            return out.reshape((self.Qg,) + self.shape)
        return out.reshape(self.shape)

    def write(self, name, arr):
        dt = {"type": np.uint8, "label": np.int32}.get(name, np.float64)
        a = np.ascontiguousarray(arr, dtype=dt).ravel()
        self._check(self.lib.mf_write_field(self.h, FIELDS[name], a.ctypes.data, a.nbytes))

    def set_bubble(self, bid, m, V, p, alive=True):
        self._check(self.lib.mf_set_bubble(self.h, bid, m, V, p, int(alive)))

    def refresh(self, relabel=False):
        self._check(self.lib.mf_refresh(self.h, int(relabel)))

    def bubbles(self):
        cap = self.params.max_ids
        arr = (MfBubble * cap)()
        n = C.c_int32()
        self._check(self.lib.mf_read_bubbles(self.h, arr, cap, C.byref(n)))
        k = min(n.value, cap)
        return dict(id=np.array([arr[i].id for i in range(k)], np.int32),
                    m=np.array([arr[i].gas_mass for i in range(k)]),
                    V=np.array([arr[i].volume for i in range(k)]),
                    p=np.array([arr[i].pressure for i in range(k)]),
                    n_cells=np.array([arr[i].n_cells for i in range(k)], np.int32),
                    centroid=np.array([list(arr[i].centroid) for i in range(k)]).reshape(k, 3))

    def ledgers(self):
        t = MfTotals()
        self._check(self.lib.mf_totals_get(self.h, C.byref(t)))
        return dict(lost_liquid=t.lost_liquid, atm_gas=t.atm_gas, collapsed_gas=t.collapsed_gas,
                    next_id=t.next_id, step=t.step, n_bubbles=t.n_bubbles,
                    n_interface=t.n_interface, status=t.status, liquid=t.liquid_mass,
                    dissolved=t.dissolved_gas, bubble_gas=t.bubble_gas)

    def save(self, path):
        self._check(self.lib.mf_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._check(self.lib.mf_load(self.h, os.fsencode(path)))

    def poke(self, name, cell, comp, value):
        """overwrite one element of a field in its storage form (fault-injection tests)"""
        self._check(self.lib.mf_debug_poke(self.h, FIELDS[name], int(cell), int(comp), float(value)))

    def attach_mlp(self, net):
        self._check(self.lib.mf_attach_mlp(self.h, net.h))

    def profile(self, on=True):
        self._check(self.lib.mf_profile_enable(self.h, int(on)))

    def profile_get(self, group):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.mf_profile_get(self.h, int(group), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def tune(self, reps=5):
        """Time the bulk-sweep launch variants on the current state and keep the fastest;
        returns (variant, ms per launch of each variant, -1 where not applicable)."""
        best = C.c_int32()
        ms = np.zeros(SWEEP_VARIANTS, np.float32)
        self._check(self.lib.mf_tune(self.h, int(reps), C.byref(best), ms.ctypes.data))
        return best.value, ms

    def set_sweep_variant(self, v):
        self._check(self.lib.mf_set_sweep_variant(self.h, int(v)))

    def totals(self):
        """Liquid mass (rho over liquid cells plus M over interface cells), dissolved and
        bubble gas (summed by the library on the device), and the ledgers."""
        return self.ledgers()


class Batch:
    """Several domains (Sim objects) advanced together, one launch per kernel for all
    domains of a group."""

    def __init__(self, sims):
        self.lib = load_library()
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s.h.value for s in self.sims])
        h = C.c_void_p()
        _check_plain(self.lib, self.lib.mf_batch_create(len(self.sims), arr, C.byref(h)))
        self.h = h

    def tune(self, reps=5):
        v = np.zeros(len(self.sims), np.int32)
        _check_plain(self.lib, self.lib.mf_batch_tune(self.h, int(reps), v.ctypes.data))
        return v

    def step(self, n=1):
        _check_plain(self.lib, self.lib.mf_batch_step(self.h, int(n)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.mf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_plain(lib, rc):
    if rc != 0:
        msg = lib.mf_last_error(None)
        raise MifoamError(f"{STATUS.get(rc, rc)}: {msg.decode() if msg else ''}")


class CurvatureNet:
    """The learned curvature closure (a libmifoam network object)."""

    def __init__(self, init_seed: int = 7):
        self.lib = load_library()
        self.nparam = self.lib.mf_mlp_param_count()
        h = C.c_void_p()
        _check_plain(self.lib, self.lib.mf_mlp_create(C.c_uint64(init_seed), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.mf_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = np.empty(self.nparam, np.float32)
        _check_plain(self.lib, self.lib.mf_mlp_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        assert t.size == self.nparam
        _check_plain(self.lib, self.lib.mf_mlp_set_params(self.h, t.ctypes.data))

    def train(self, n_train, n_val, epochs=8, batch=4096, lr=1e-3, noise=0.01, data_seed=4):
        spec = MfMlpTrainSpec()
        spec.struct_size = C.sizeof(MfMlpTrainSpec)
        spec.n_train, spec.n_val, spec.epochs, spec.batch = n_train, n_val, epochs, batch
        spec.lr, spec.noise, spec.data_seed = lr, noise, data_seed
        rmse = C.c_double()
        _check_plain(self.lib, self.lib.mf_mlp_train(self.h, C.byref(spec), _stream_ptr(), C.byref(rmse)))
        return rmse.value

    def save(self, path):
        _check_plain(self.lib, self.lib.mf_mlp_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        """a network read from a file written by save()"""
        net = cls.__new__(cls)
        net.lib = load_library()
        net.nparam = net.lib.mf_mlp_param_count()
        h = C.c_void_p()
        _check_plain(net.lib, net.lib.mf_mlp_load(C.byref(h), os.fsencode(path)))
        net.h = h
        return net

    def eval(self, stencils):
        X = np.ascontiguousarray(stencils, dtype=np.float32).reshape(-1, 125)
        out = np.empty(X.shape[0], np.float32)
        _check_plain(self.lib, self.lib.mf_mlp_eval(self.h, X.ctypes.data, X.shape[0], out.ctypes.data,
                                                    _stream_ptr()))
        return out

    def eval_noalloc(self, stencils_dev, kappa_dev, n=None):
        """curvature of device stencils (torch float32 [n, 125] on the GPU) into a device
        tensor kappa_dev (float32 [n]) through the allocation-free entry point; enqueued
        on the current stream"""
        n = stencils_dev.shape[0] if n is None else int(n)
        _check_plain(self.lib, self.lib.mf_mlp_eval_noalloc(self.h, C.c_void_p(stencils_dev.data_ptr()), n,
                                                            C.c_void_p(kappa_dev.data_ptr()), _stream_ptr()))

    def grad(self, stencils, target8):
        X = np.ascontiguousarray(stencils, dtype=np.float32).reshape(-1, 125)
        t = np.ascontiguousarray(target8, dtype=np.float32)
        g = np.empty(self.nparam, np.float32)
        loss = C.c_double()
        _check_plain(self.lib, self.lib.mf_mlp_grad(self.h, X.ctypes.data, t.ctypes.data, X.shape[0],
                                                    g.ctypes.data, C.byref(loss), _stream_ptr()))
        return loss.value, g


def generate_stencils(seed, first, n, noise=0.01):
    """stencils [n,125] and exact curvature [n] from the library's GPU generator"""
    lib = load_library()
    X = np.empty((n, 125), np.float32)
    k = np.empty(n, np.float32)
    _check_plain(lib, lib.mf_mlp_generate(C.c_uint64(seed), first, n, noise, X.ctypes.data, k.ctypes.data,
                                          _stream_ptr()))
    return X, k
