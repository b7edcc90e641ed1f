"""Block LOBPCG on the GPU against the oracle's (the paper's comparison solver).

* one pass (every block runs all its line minimisations, tol = 0) from the
  same seeded start block, S = I and the PAW-like S: Ritz values <= 1e-9 Ha,
  residual norms <= 1e-8 absolute (a pass chains up to 1 + 2 nline
  Rayleigh-Ritz steps per block; Ritz values are second order in the vectors'
  rounding, residuals first order), Psi S-orthonormal to 1e-10;
* passes to convergence reach the lowest pairs of the dense pencil (1e-8 Ha);
* argument errors: complex64 blocks, a block count that does not divide nband.
"""
import functools

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import SMALL, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [  # name, nband, nblocks, nline
    ("tiny_k", 8, 2, 3),
    ("odd15", 18, 3, 4),
    ("n25", 70, 2, 3),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


@functools.lru_cache(maxsize=None)
def case(name, paw):
    kw = dict(SMALL[name])
    tag = kw.pop("tag")
    s = W.make_system(tag, q_scale=W.PAW_Q_SCALE if paw else 0.0, **kw)
    H = O.Hamiltonian.from_system(s)
    return s, H, O.Overlap.from_system(H, s)


@pytest.mark.parametrize("paw", [False, True])
@pytest.mark.parametrize("name,nband,nblocks,nline", CASES)
def test_one_pass(name, nband, nblocks, nline, paw):
    s, H, S = case(name, paw)
    X = W.random_block(H.npw, nband, s.tag + 50)
    ref = O.lobpcg_pass(H.apply, S.apply, H.sphere.kinetic, X, nblocks, nline, 0.0)
    with B.System(s) as g:
        Xd = to_dev(X)
        ev, res, info = g.lobpcg(Xd, nblocks, nline, max_passes=1, tol=0.0)
        Psi = to_host(Xd)
        SPsi = to_host(g.apply_S(Xd))
    assert info["passes"] == 1 and info["line_steps"] == nblocks * nline
    assert np.abs(ev - ref["eval"]).max() <= 1e-9
    assert np.abs(res - ref["res"]).max() <= 1e-8
    assert np.abs(Psi.conj().T @ SPsi - np.eye(nband)).max() <= 1e-10


@pytest.mark.parametrize("paw", [False, True])
def test_converges_to_dense_pencil(paw):
    s, H, S = case("tiny_k", paw)
    lam = scipy.linalg.eigh(H.dense(), S.dense(), eigvals_only=True)
    X = W.random_block(H.npw, 8, 91)
    with B.System(s) as g:
        ev, res, info = g.lobpcg(to_dev(X), 2, 4, max_passes=20, nconv=6, tol=1e-9)
    assert info["converged"]
    assert np.abs(ev[:6] - lam[:6]).max() <= 1e-8
    assert res[:6].max() <= 1e-9


def test_argument_errors():
    import torch
    s, H, S = case("tiny_k", False)
    X = to_dev(W.random_block(H.npw, 8, 92))
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        with pytest.raises(B.ChebfiError) as e:
            g.lobpcg(X.to(torch.complex64), 2, 2)
        assert e.value.code == B.ABI_ERR_ARG
        with pytest.raises(B.ChebfiError) as e:
            g.lobpcg(X, 3, 2)
        assert e.value.code == B.ABI_ERR_ARG
