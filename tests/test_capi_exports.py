"""The C-ABI library loads on any host and exports every symbol include/simm.h declares
(no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simm.h")
LIB = os.path.join(ROOT, "paper_2006_16117_amd", "libsimm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(simm_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("simm_pencil_create_banded", "simm_shift_build", "simm_indicators", "simm_project", "simm_run",
                 "simm_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_the_header():
    import paper_2006_16117_amd.simm as S
    assert set(declared_functions()) <= set(S.EXPORTS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_params_default_without_gpu():
    import paper_2006_16117_amd.simm as S
    p = S.params_default()
    assert p.eps0 == 1e-8 and p.delta0 == 0.05 and p.tau == 1e-8 and p.gauss_per_edge == 8
