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
                 "simm_multiplicities", "simm_gradient", "simm_last_error"):
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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_band_sum_of_the_gradient_wrapper():
    """The autograd wrapper forms A0 + p A1 + diag(d) as a band: check it against dense
    matrices (host logic only)."""
    import numpy as np
    import oracle.simm as O
    import paper_2006_16117_amd.simm as S
    from workloads import random_band_matrix, random_band_pencil
    n = 37
    pen, _ = random_band_pencil(n, 3, 11)
    a1 = random_band_matrix(n, 5, 12, 0.1)
    d = np.arange(n) * (0.5 - 0.25j)
    kl, ku, band = S._band_sum(n, [(3, 3, pen.a_band), (5, 5, 0.3 * a1), (0, 0, d.reshape(1, -1))])
    assert (kl, ku) == (5, 5)
    dense = O.band_to_dense(n, 3, 3, pen.a_band) + 0.3 * O.band_to_dense(n, 5, 5, a1) + np.diag(d)
    assert np.array_equal(O.band_to_dense(n, kl, ku, band), dense)
    # A1's entries are real and confined to its band
    A1 = O.band_to_dense(n, 5, 5, a1)
    assert np.all(A1.imag == 0)
    i, j = np.nonzero(A1)
    assert np.all(np.abs(i - j) <= 5) and len(i) == sum(n - abs(k) for k in range(-5, 6))
