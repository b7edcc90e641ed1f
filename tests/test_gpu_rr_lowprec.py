"""The split-BF16 Rayleigh-Ritz of the mixed form (needs an MI355X).

Columns scaled to unit norm, G and H_s as split-BF16 products accumulated in
FP32, Cholesky / reduction / eigensolve in FP64, split-BF16 rotations; a block
whose equilibrated Gram matrix has a squared Cholesky pivot below 0.5 is first
orthonormalised with that factor and its Gram matrix taken again (two passes).
A split-BF16 product carries a relative error of about 2^-17 (two 8-bit
significands per operand, the lo x lo term dropped), so against the FP64
oracle's Rayleigh-Ritz of the same complex64 block the Ritz values are within
2^-17 ||H_s|| times a small factor after two passes, and within that times the
Gram matrix's condition number after one.  Bars: Ritz values within
2e-5 max|lambda| (two passes; the emulated error on these blocks is at most
3.4e-6 max|lambda|) or 1e-4 max|lambda| (one pass, condition number below 20:
emulated 1.2e-5); Ritz vectors orthonormal to 1e-4; residual norms within
1e-4 max|lambda| of || H psi - lambda psi || recomputed by the oracle.  The
smallest squared pivots of the three blocks (0.023, 0.25 and 0.60 in FP64)
put the first two on the two-pass branch and the third on the one-pass one.
A block with two nearly parallel columns (equilibrated Gram matrix
conditioned beyond what the split products resolve, condition ~3e6) makes the call fall back
to the FP64 form and say so in flags; its Ritz values then meet the FP64 bar
(1e-8 Ha) against the oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import hamiltonian, system, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


def _filtered(name, nb, seed):
    """A filtered complex64 block (rounded to complex128 for the oracle)."""
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, nb, seed)
    a, b, a0 = O.filter_bounds(H, X, W.random_vector(H.npw, s.tag))
    Y = O.cheb_filter(H, X, 6, a, b, a0)
    Y = Y / np.linalg.norm(Y, axis=0)[None, :]
    return H, s, Y.astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("name,nb,two_pass", [("n27", 37, True), ("c1", 32, False),
                                              ("n25", 70, True)])
def test_lowprec_rr_against_oracle(name, nb, two_pass):
    import torch
    H, s, Y = _filtered(name, nb, 71)
    ref = O.rayleigh_ritz(H, Y)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Yd = to_dev(Y).to(torch.complex64)
        hp = torch.empty_like(Yd)
        ev, res, flags, C = g.rayleigh_ritz(Yd, hp, want_coef=True, lowprec=True)
        Psi = to_host(Yd).astype(np.complex128)
        C = C.cpu().numpy()
    assert flags == (B.RR_LOWPREC | B.RR_TWO_PASS if two_pass else B.RR_LOWPREC)
    scale = np.abs(ref["eval"]).max()
    assert np.all(np.diff(ev) >= -1e-4 * scale)
    assert np.abs(ev - ref["eval"]).max() <= (2e-5 if two_pass else 1e-4) * scale
    assert np.abs(Psi.conj().T @ Psi - np.eye(nb)).max() <= 1e-4
    r = np.linalg.norm(H(Psi) - Psi * ev[None, :], axis=0)
    assert np.abs(r - res).max() <= 1e-4 * scale
    # the coefficients reproduce the Ritz vectors from the input block
    assert np.abs(Y @ C - Psi).max() <= 1e-4 * np.abs(Psi).max()


def test_lowprec_rr_falls_back_on_near_dependent_columns():
    import torch
    H, s, Y = _filtered("n27", 37, 72)
    rng = np.random.default_rng([2604, 11139, 73])
    # column 5 = column 3 + 3e-3 noise: the equilibrated Gram matrix has an
    # eigenvalue near 1e-5 (a squared Cholesky pivot near 9e-6, below the
    # split form's 1e-4), which FP64 still resolves (condition ~3e6)
    noise = rng.standard_normal(H.npw) + 1j * rng.standard_normal(H.npw)
    Y[:, 5] = Y[:, 3] + 3e-3 * noise / np.linalg.norm(noise)
    Y = Y.astype(np.complex64).astype(np.complex128)
    ref = O.rayleigh_ritz(H, Y)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Yd = to_dev(Y).to(torch.complex64)
        ev, res, flags = g.rayleigh_ritz(Yd, lowprec=True)
    assert flags == B.RR_FELL_BACK
    assert np.abs(ev - ref["eval"]).max() <= 1e-8
