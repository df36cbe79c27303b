"""simm_project_noalloc (projection with the library's static scratch, no device
allocation) against simm_project, through the C ABI (needs an MI355X).  Collected last
(file name), so that a failure here hides no other test."""
import sys

import numpy as np
import pytest

from workloads.gen import random_band_pencil

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2006_16117_amd.simm as S
    return S


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_project_noalloc_matches_project(S, prec):
    import torch
    n, m = 3001, 37
    pen, f = random_band_pencil(n, 3, 901, b_kind="tridiag", b_offdiag=0.3)
    say("project_noalloc", f"n={n} m={m} prec={prec}: shift build")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.1 + 0.05j, f, m)
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(11)
    for c in (301, 77):      # two calls in a row, the second smaller
        Y = torch.randn((c, m), dtype=torch.complex128, generator=g).to(dev)     # column-major m x c: Y.T
        X_ref = torch.empty((c, n), dtype=torch.complex128, device=dev)
        X_new = torch.full((c, n), complex(7.0, 7.0), dtype=torch.complex128, device=dev)
        nr_ref = torch.empty(c, dtype=torch.float64, device=dev)
        nr_new = torch.full((c,), -1.0, dtype=torch.float64, device=dev)
        nr_only = torch.full((c,), -1.0, dtype=torch.float64, device=dev)
        say(f"  c={c}: simm_project, then simm_project_noalloc (X and norms), then norms only")
        S.simm_project(sh, Y.T, X_ref.T, nr_ref, precision=prec)
        S.simm_project_noalloc(sh, Y.T, X_new.T, nr_new, precision=prec)
        S.simm_project_noalloc(sh, Y.T, None, nr_only, precision=prec)
        torch.cuda.synchronize()
        # the same kernels with the same launch shapes: bit for bit the same values
        assert torch.equal(X_new, X_ref)
        assert torch.equal(nr_new, nr_ref)
        assert torch.equal(nr_only, nr_ref)
        # and the reference itself against the basis (numpy, FP64)
        V = sh.basis()[:, :m]
        Xn = V @ Y.T.cpu().numpy()
        tol = 1e-13 if prec == 0 else 1e-5
        assert np.linalg.norm(X_ref.T.cpu().numpy() - Xn) <= tol * np.linalg.norm(Xn)


def test_project_noalloc_rejects_too_large(S):
    import torch
    n, m = 300000, 2
    pen, f = random_band_pencil(n, 1, 902, b_kind="identity")
    say("project_noalloc", f"size limit: n={n} m={m}")
    P = S.Pencil.from_workload(pen)
    sh = S.simm_shift_build(P, 0.1 + 0.05j, f, m)
    dev = torch.device("cuda:0")
    c = 500        # (2 ceil(n/128) + 32) c doubles > 2^21
    Y = torch.zeros((c, m), dtype=torch.complex128, device=dev)
    nr = torch.empty(c, dtype=torch.float64, device=dev)
    with pytest.raises(S.SimmError) as e:
        S.simm_project_noalloc(sh, Y.T, None, nr)
    assert e.value.status == -8 and "scratch" in str(e.value)
    # X alone needs no scratch
    X = torch.empty((c, n), dtype=torch.complex128, device=dev)
    S.simm_project_noalloc(sh, Y.T, X.T, None)
    torch.cuda.synchronize()
    assert float(X.abs().max()) == 0.0
