"""Pins for the oracle's filter adjoint (CPU only).

* central finite differences (h = 1e-5) of L = Re<W, p(H) X> along random
  directions in V(r), in the real and imaginary parts of D and in X;
* dX = p(H) W exactly (p has real coefficients and H is Hermitian);
* sum_r dV(r) = Re<W, p'(H) X>: a uniform shift of V shifts H by the identity,
  with p'(H) evaluated from a dense eigendecomposition and NumPy's Chebyshev
  series derivative.
"""
import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest

import oracle as O
import workloads as W


def tiny(tag=131, **kw):
    base = dict(a=6.0, ecut=4.0, n=12, natom=2, nband=5, kpt_red=(0.1, 0.2, 0.3), d_scale=20.0)
    base.update(kw)
    return W.make_system(tag, **base)


def _setup(degree=5):
    s = tiny()
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 5, 131)
    Wt = W.random_block(H.npw, 5, 131, stream=3)
    v0 = W.random_vector(H.npw, 131)
    a, b, a0 = O.filter_bounds(H, X, v0)
    return s, H, X, Wt, (a, b, a0), degree


def _loss(s, X, Wt, bounds, degree, vloc=None, dij=None):
    s2 = tiny()
    if vloc is not None:
        s2.vloc = vloc
    if dij is not None:
        s2.dij = dij
    H = O.Hamiltonian.from_system(s2)
    return O.filter_loss(H, X, Wt, degree, *bounds)


def test_fd_potential():
    s, H, X, Wt, bounds, m = _setup()
    dV, _, _ = O.filter_backward(H, X, Wt, m, *bounds)
    rng = np.random.default_rng(1)
    h = 1e-5
    for _ in range(3):
        d = rng.standard_normal(s.vloc.shape)
        fd = (_loss(s, X, Wt, bounds, m, vloc=s.vloc + h * d)
              - _loss(s, X, Wt, bounds, m, vloc=s.vloc - h * d)) / (2 * h)
        an = float(dV @ d)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)


@pytest.mark.parametrize("part", ["re", "im"])
def test_fd_nonlocal(part):
    s, H, X, Wt, bounds, m = _setup()
    _, dD, _ = O.filter_backward(H, X, Wt, m, *bounds)
    rng = np.random.default_rng(2)
    h = 1e-5
    for _ in range(3):
        d = rng.standard_normal(s.dij.shape) * (1.0 if part == "re" else 1j)
        fd = (_loss(s, X, Wt, bounds, m, dij=s.dij + h * d)
              - _loss(s, X, Wt, bounds, m, dij=s.dij - h * d)) / (2 * h)
        # grad convention dRe + i dIm: directional derivative = Re(conj(grad) . d)
        an = float(np.real(np.vdot(dD, d)))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)


def test_fd_block():
    s, H, X, Wt, bounds, m = _setup()
    _, _, dX = O.filter_backward(H, X, Wt, m, *bounds)
    rng = np.random.default_rng(3)
    h = 1e-5
    for _ in range(2):
        d = rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)
        fd = (O.filter_loss(H, X + h * d, Wt, m, *bounds)
              - O.filter_loss(H, X - h * d, Wt, m, *bounds)) / (2 * h)
        an = float(np.real(np.vdot(dX, d)))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)


def test_dx_is_filter_of_w():
    s, H, X, Wt, bounds, m = _setup(degree=7)
    _, _, dX = O.filter_backward(H, X, Wt, m, *bounds)
    ref = O.cheb_filter(H, Wt, m, *bounds)
    assert np.abs(dX - ref).max() <= 1e-11 * np.abs(ref).max()


def test_uniform_potential_shift_closed_form():
    s, H, X, Wt, bounds, m = _setup(degree=6)
    dV, _, _ = O.filter_backward(H, X, Wt, m, *bounds)
    a, b, a0 = bounds
    e, c = (b - a) / 2, (b + a) / 2
    coef = np.zeros(m + 1)
    coef[-1] = 1.0
    dcoef = npcheb.chebder(coef)
    lam, V = np.linalg.eigh(H.dense())
    tm = npcheb.chebval((a0 - c) / e, coef)
    dp = npcheb.chebval((lam - c) / e, dcoef) / e / tm  # p'(lambda)
    ref = float(np.real(np.vdot(Wt, V @ (dp[:, None] * (V.conj().T @ X)))))
    assert abs(dV.sum() - ref) <= 1e-10 * abs(ref)
