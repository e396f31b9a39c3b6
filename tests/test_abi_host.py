"""CPU-side checks of the boundary: the library is built for gfx950, loads,
and exports every function declared in include/ga.h (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2102_11536_amd", "libga.so")


def declared():
    src = open(os.path.join(ROOT, "include", "ga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ga_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("ga_setup_patch", "ga_apply_MK", "ga_apply_Pinv", "ga_mass_solve", "ga_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2102_11536_amd.build import build_library
        build_library()
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in declared():
        assert re.search(rf"\bT {n}\b", out), n


def test_binding_names_match_header():
    from paper_2102_11536_amd import ga
    assert sorted(ga.EXPORTS) == declared()


def test_stability_limit_host_function():
    # a host-only entry point: pinned against the lambda = -1 root of the
    # printed type-k characteristic polynomial, (4 alpha - 2)/(2 beta - gamma)
    from paper_2102_11536_amd import ga
    lib = ga.load_library()
    for rho in (0.0, 0.5, 0.8):
        a = (2 - rho) / (1 + rho)
        b = (5 - 3 * rho) / ((1 + rho) ** 2 * (2 - rho))
        g = a + 0.5
        assert abs(lib.ga_stability_limit(rho) - (4 * a - 2) / (2 * b - g)) < 1e-13
    assert abs(lib.ga_stability_limit(0.5) - 108 / 31) < 1e-13


def test_code_object_targets_gfx950():
    # the fat binary of the library (built here from source) names its target
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_profile_mask_host_checks():
    # host-only: the kinds mask is range-checked before any event is touched
    from paper_2102_11536_amd import ga
    lib = ga.load_library()
    assert lib.ga_profile(16) == -1
    assert lib.ga_profile(-1) == -1
    assert lib.ga_profile(0) == 0


def _declarations():
    src = open(os.path.join(ROOT, "include", "ga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(?:int|double|const char\*)\s+(ga_[A-Za-z0-9_]+)\s*\(([^)]*)\)\s*;", src):
        params = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        out[m.group(1)] = params
    return out


def test_binding_argument_counts_match_header():
    # every ctypes prototype has as many arguments as the header declares
    from paper_2102_11536_amd import ga
    lib = ga.load_library()
    decl = _declarations()
    assert sorted(decl) == declared()
    for name, params in decl.items():
        assert len(getattr(lib, name).argtypes) == len(params), (name, params)


def test_apply_signatures_take_a_precision():
    # the operator and preconditioner applies take the arithmetic (GA_FP64 / GA_FP32 /
    # GA_BF16) right after nrhs, as the boundary specifies
    decl = _declarations()
    mk = decl["ga_apply_MK"]
    assert mk[2].endswith("nrhs") and mk[3] == "int prec", mk
    pv = decl["ga_apply_Pinv"]
    assert pv[1].endswith("nrhs") and pv[2] == "int prec", pv
    src = open(os.path.join(ROOT, "include", "ga.h")).read()
    assert re.search(r"GA_FP64 = 0, GA_FP32 = 1, GA_BF16 = 2", src)
    assert re.search(r"GA_PINV_MFMA = 2", src)


def test_argument_checks_before_device_work():
    # host-side validation: null handles and bad precisions are refused with
    # GA_EINVAL before any device call
    from paper_2102_11536_amd import ga
    lib = ga.load_library()
    null = ctypes.c_void_p()
    assert lib.ga_apply_MK(null, b"M", 1, 0, 1.0, null, null, null) == ga.GA_EINVAL
    assert lib.ga_apply_Pinv(null, 1, 2, null, null, null) == ga.GA_EINVAL
    assert lib.ga_patch_set_layers(null, 0, 0) == ga.GA_EINVAL
    assert lib.ga_patch_set_pinv(null, ga.GA_PINV_MFMA) == ga.GA_EINVAL
