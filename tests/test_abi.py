"""The C-ABI library loads and exports every symbol include/mifoam.h declares (no GPU
compute calls here); parameter validation runs on the host."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mifoam.h")).read()
    return sorted(set(re.findall(r"\b(mf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_exports():
    from paper_1908_04262_amd.mifoam import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_library_exports_every_symbol():
    from paper_1908_04262_amd.mifoam import LIBPATH, load_library
    if not os.path.exists(LIBPATH):
        pytest.skip("libmifoam.so not built (run __graft_entry__.build())")
    lib = load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    want = int(re.search(r"#define MF_ABI_VERSION (\d+)", open(os.path.join(ROOT, "include", "mifoam.h")).read()).group(1))
    assert lib.mf_abi_version() == want


def test_workspace_and_validation_on_host():
    from paper_1908_04262_amd.mifoam import LIBPATH, load_library, make_params
    from synth import workload
    if not os.path.exists(LIBPATH):
        pytest.skip("libmifoam.so not built")
    lib = load_library()
    p = make_params(workload("c3_foam_384"))
    n = C.c_size_t()
    assert lib.mf_workspace_bytes(C.byref(p), C.byref(n)) == 0
    # two FP32 population buffers of 19 + 7 planes dominate: ~11.8 GB at 384^3
    assert 11.5e9 < n.value < 20e9
    bad = make_params(workload("c3_foam_384"))
    bad.tau = 0.4
    bad.rheology = 0
    assert lib.mf_workspace_bytes(C.byref(bad), C.byref(n)) == -1
    assert b"tau" in lib.mf_last_error(None)
    bad2 = make_params(workload("c3_foam_384"))
    bad2.struct_size = 8
    assert lib.mf_workspace_bytes(C.byref(bad2), C.byref(n)) == -1
    # body force: bounded components, none out of the plane of a 2D domain
    ok = make_params(workload("c3_foam_384", accel=(0.0, 0.0, -3e-5)))
    assert lib.mf_workspace_bytes(C.byref(ok), C.byref(n)) == 0
    big = make_params(workload("c3_foam_384", accel=(0.0, 0.02, 0.0)))
    assert lib.mf_workspace_bytes(C.byref(big), C.byref(n)) == -1
    assert b"acceleration" in lib.mf_last_error(None)
    nan = make_params(workload("c3_foam_384", accel=(float("nan"), 0.0, 0.0)))
    assert lib.mf_workspace_bytes(C.byref(nan), C.byref(n)) == -1
    # Carreau-Yasuda: shear thinning with a unique relaxation time
    cy = dict(rheology="carreau_yasuda", cy_tau0=1.2, cy_tau_inf=0.6, cy_lambda=1000.0, cy_a=2.0, cy_n=0.4)
    good = make_params(workload("c3_foam_384", **cy))
    assert lib.mf_workspace_bytes(C.byref(good), C.byref(n)) == 0
    for badkw in (dict(cy_tau_inf=0.5), dict(cy_tau0=0.55), dict(cy_n=1.5), dict(cy_a=0.0),
                  dict(cy_lambda=-1.0), dict(cy_tau0=3.0, cy_n=0.1)):
        b = make_params(workload("c3_foam_384", **dict(cy, **badkw)))
        assert lib.mf_workspace_bytes(C.byref(b), C.byref(n)) == -1, badkw
        assert b"Carreau" in lib.mf_last_error(None)
    plane = make_params(workload("c1_2d_128", accel=(0.0, -1e-5, 1e-5)))
    assert lib.mf_workspace_bytes(C.byref(plane), C.byref(n)) == -1
    assert b"2D" in lib.mf_last_error(None)
