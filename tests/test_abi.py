"""The C-ABI library loads on a machine without a GPU and exports every entry point
that include/bemc.h declares; host-side argument checks return errors without touching
the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bemc.h")
LIB = os.path.join(ROOT, "paper_1606_03743_amd", "libbemc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bemc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1606_03743_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("bemc_create", "bemc_upload_geometry", "bemc_upload_densities", "bemc_eval",
              "bemc_collocation_matvec", "bemc_server_start", "bemc_server_submit"):
        assert f in fns


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (bemc_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        getattr(lib, f)


def test_binding_lists_every_symbol():
    from paper_1606_03743_amd import bemc

    assert sorted(bemc.EXPORTED) == declared_functions()


def test_null_argument_errors(lib):
    lib.bemc_last_error.restype = ctypes.c_char_p
    assert lib.bemc_create(0, None) == -1
    assert b"NULL" in lib.bemc_last_error()
    assert lib.bemc_eval(None, None, 0, 0, 0, None, None, None) == -1
    assert lib.bemc_destroy(None) == -1
    lib.bemc_coulomb_constant.restype = ctypes.c_double
    import scipy.constants as sc
    import math

    assert abs(lib.bemc_coulomb_constant() * 4 * math.pi * sc.epsilon_0 - 1) < 1e-15
    assert lib.bemc_rule_size(33) == 33 and lib.bemc_rule_size(7) == 7 and lib.bemc_rule_size(5) == -1


def test_missing_library_fails_loudly(monkeypatch):
    """No silent fallback: without the built library the binding raises."""
    from paper_1606_03743_amd import bemc

    monkeypatch.setattr(bemc, "_lib", None)
    monkeypatch.setattr(bemc, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libbemc.so"))
    with pytest.raises(RuntimeError, match="missing"):
        bemc.load_library()


def test_null_argument_errors_of_newer_entry_points(lib):
    assert lib.bemc_eval_gradient(None, None, 0, 0, 0, None, None) == -1
    assert lib.bemc_set_dr_rules(None, 1, None, None) == -1
    assert lib.bemc_solve_densities(None, None, None, ctypes.c_double(1e-10), 10, 10, 0, None, None) == -1


@pytest.mark.parametrize("lang,std", [("c", "c99"), ("c++", "c++17")])
def test_header_is_plain_c_and_cxx(lang, std):
    """The boundary header needs no HIP or torch include and compiles as C99 and C++."""
    compiler = "gcc" if lang == "c" else "g++"
    r = subprocess.run([compiler, f"-std={std}", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-x", lang, HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_c_program_links_against_the_library(tmp_path, lib):
    """A plain C caller: declares nothing itself, links libbemc.so, and gets errors (not
    crashes) for invalid calls on a machine without a GPU."""
    src = tmp_path / "caller.c"
    src.write_text(
        '#include "bemc.h"\n#include <stdio.h>\n'
        "int main(void) {\n"
        "    bemc_handle h = 0;\n"
        "    int rc = bemc_create(0, 0);\n"
        '    printf("%d %d %s\\n", rc, bemc_rule_size(12), bemc_last_error());\n'
        "    (void)h;\n"
        "    return rc == BEMC_E_INVALID_ARG && bemc_rule_size(12) == 12 ? 0 : 1;\n"
        "}\n")
    exe = tmp_path / "caller"
    libdir = os.path.dirname(LIB)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                        "-L", libdir, "-lbemc", f"-Wl,-rpath,{libdir}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr


def test_issue_probe_library():
    """The benchmark's issue-rate probe is a library of its own (not part of the boundary):
    it loads without a GPU, exports its one entry point, rejects a null output, and libbemc.so
    does not carry it."""
    probe = os.path.join(ROOT, "paper_1606_03743_amd", "libissue_probe.so")
    if not os.path.exists(probe):
        from paper_1606_03743_amd import build

        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", probe], capture_output=True, text=True, check=True).stdout
    assert re.search(r" T issue_probe_rates$", out, re.M)
    lib = ctypes.CDLL(probe)
    lib.issue_probe_rates.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert lib.issue_probe_rates(0, None) == -1
    main = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    assert "issue_probe_rates" not in main


@pytest.mark.gpu
def test_issue_probe_rates_on_device():
    """The probe measures positive rates; the FP64 reciprocal square root issues slower than
    the FP64 FMA, and the one-in-nine stream lies between the two."""
    import torch

    assert torch.cuda.is_available()
    probe = os.path.join(ROOT, "paper_1606_03743_amd", "libissue_probe.so")
    lib = ctypes.CDLL(probe)
    lib.issue_probe_rates.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    r = (ctypes.c_double * 6)()
    assert lib.issue_probe_rates(0, r) == 0
    fma64, rsq64, mix64, fma32, rsq32, mix32 = list(r)
    print(f"issue rates: fma64 {fma64:.3e} rsq64 {rsq64:.3e} mix64 {mix64:.3e} "
          f"fma32 {fma32:.3e} rsq32 {rsq32:.3e} mix32 {mix32:.3e}")
    assert all(v > 1e9 for v in r)
    assert rsq64 < fma64 and rsq64 < mix64 <= 1.05 * fma64
    assert rsq32 < fma32
