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
