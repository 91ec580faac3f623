"""The C-ABI library loads without a GPU and exports every function the header declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hinv.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hinv_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_paper_operations():
    names = declared_functions()
    for op in ("hinv_forward", "hinv_gradient", "hinv_inc_forward", "hinv_inc_adjoint",
               "hinv_hessian_apply", "hinv_prior_apply", "hinv_prior_solve", "hinv_prior_sample",
               "hinv_map_newton", "hinv_lowrank_eig", "hinv_posterior_sample"):
        assert op in names


def test_library_exports_every_declared_symbol():
    from paper_1909_03948_amd import hinv
    lib = hinv.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(hinv.EXPORTS) == set(declared_functions())


def test_status_strings_without_gpu():
    from paper_1909_03948_amd import hinv
    lib = hinv.load()
    assert lib.hinv_status_string(hinv.HINV_ENOCONV).decode().startswith("iterative")
    assert lib.hinv_status_string(12345).decode() == "unknown status"
