"""The multi-cycle driver (abi_chebfi_solve) against the dense spectrum.

On the small workload (1503 plane waves, 32 bands, 2 atoms) the lowest 20
eigenvalues of the dense operator (the oracle's explicit H, diagonalised by
LAPACK) are the exact answer the cycles converge to:

* FP64 cycles to residuals <= 1e-8: Ritz values <= 1e-9 Ha from the dense ones;
* mixed cycles handing over to the FP64 refinement: the same bound, with at
  least one refinement cycle (the mixed form alone stalls near 1e-5);
* mixed cycles without refinement within the 12-cycle budget: <= 1e-6 Ha
  (the mixed budget);
* argument errors.
"""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import to_dev

pytestmark = pytest.mark.gpu

NCONV = 20


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


@functools.lru_cache(maxsize=None)
def _case():
    s = W.make_system(1)
    H = O.Hamiltonian.from_system(s)
    lam = np.linalg.eigvalsh(H.dense())
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    return s, lam, X, v0


def test_solve_fp64():
    s, lam, X, v0 = _case()
    with B.System(s) as g:
        Xd = to_dev(X)
        ev, res, info = g.solve(Xd, to_dev(v0), 8, 60, NCONV, 1e-8)
    assert info["converged"] and info["refine_cycles"] == 0
    assert res[:NCONV].max() <= 1e-8
    assert np.abs(ev[:NCONV] - lam[:NCONV]).max() <= 1e-9


def test_solve_mixed_with_refinement():
    import torch
    s, lam, X, v0 = _case()
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Xd = to_dev(X).to(torch.complex64)
        ev, res, info = g.solve(Xd, to_dev(v0), 8, 60, NCONV, 1e-8, refine_degree=4)
    assert info["converged"] and info["refine_cycles"] >= 1
    assert np.abs(ev[:NCONV] - lam[:NCONV]).max() <= 1e-9


def test_solve_mixed_budget():
    import torch
    s, lam, X, v0 = _case()
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Xd = to_dev(X).to(torch.complex64)
        ev, res, info = g.solve(Xd, to_dev(v0), 8, 12, NCONV, 1e-8)
    assert info["cycles"] <= 12 and info["refine_cycles"] == 0
    assert np.abs(ev[:NCONV] - lam[:NCONV]).max() <= 1e-6


def test_solve_argument_errors():
    import torch
    s, lam, X, v0 = _case()
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Xd = to_dev(X)
        for kw in (dict(refine_degree=4), dict(nconv=s.nband + 1), dict(tol=0.0)):
            args = dict(degree=8, max_cycles=4, nconv=NCONV, tol=1e-8)
            args.update(kw)
            with pytest.raises(B.ChebfiError) as ei:
                g.solve(Xd, to_dev(v0), **args)
            assert ei.value.code == B.ABI_ERR_ARG
        with pytest.raises(TypeError):
            g.solve(Xd, to_dev(v0).to(torch.complex64), 8, 4, NCONV, 1e-8)
