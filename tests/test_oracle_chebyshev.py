"""Pins for the oracle's filter and bounds (CPU only).

* sigma_k = T_{k-1}(tau)/T_k(tau) with T_k(tau) = (-1)^k cosh(k arccosh(-tau));
* the filter on an exact eigenvector scales it by T_m((lam-c)/e)/T_m(tau),
  with T_m evaluated by NumPy's Chebyshev series (independent of the recurrence);
* on a tiny basis the filter equals V p(Lambda) V^H X from a dense eigensolve;
* degree 1 is the affine (sigma_1/e)(H - c) X;
* free electron: elementwise p(kin);
* Lanczos satisfies H V_k = V_k T_k + beta_k v_{k+1} e_k^T, its Ritz values
  interlace the dense spectrum, and b bounds lambda_max on the test systems;
* Rayleigh-quotient bounds lie inside the spectrum.
"""
import math

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest

import oracle as O
import workloads as W


def tiny(tag=111, **kw):
    base = dict(a=6.0, ecut=4.0, n=12, natom=2, nband=8, kpt_red=(0.1, 0.2, 0.3), d_scale=20.0)
    base.update(kw)
    return W.make_system(tag, **base)


def p_of(lam, degree, a, b, a0):
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    coef = np.zeros(degree + 1)
    coef[-1] = 1.0
    return npcheb.chebval((lam - c) / e, coef) / npcheb.chebval((a0 - c) / e, coef)


def test_sigmas_closed_form():
    a, b, a0 = 1.0, 9.0, -2.0
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    tau = (a0 - c) / e
    sig = O.cheb_sigmas(12, a, b, a0)
    T = [(-1) ** k * math.cosh(k * math.acosh(-tau)) for k in range(13)]
    for k in range(1, 13):
        assert abs(sig[k - 1] - T[k - 1] / T[k]) < 1e-14 * abs(T[k - 1] / T[k])


@pytest.mark.parametrize("degree", [1, 2, 5, 12])
def test_filter_dense_and_eigenvector(degree):
    s = tiny()
    H = O.Hamiltonian.from_system(s)
    lam, V = np.linalg.eigh(H.dense())
    a, b, a0 = float(lam[20]), float(lam[-1]) + 0.3, float(lam[0]) - 0.1
    X = W.random_block(H.npw, 5, 111)
    Y = O.cheb_filter(H, X, degree, a, b, a0)
    ref = V @ (p_of(lam, degree, a, b, a0)[:, None] * (V.conj().T @ X))
    assert np.abs(Y - ref).max() <= 1e-11 * np.abs(ref).max()
    v = V[:, 3]
    yv = O.cheb_filter(H, v, degree, a, b, a0)
    assert np.abs(yv - p_of(lam[3], degree, a, b, a0) * v).max() < 1e-11 * abs(p_of(lam[3], degree, a, b, a0))


def test_degree_one_affine():
    s = tiny()
    H = O.Hamiltonian.from_system(s)
    a, b, a0 = 1.0, 6.0, -1.0
    X = W.random_block(H.npw, 3, 112)
    e, c = (b - a) / 2, (b + a) / 2
    s1 = e / (a0 - c)
    ref = (s1 / e) * (H(X) - c * X)
    assert np.abs(O.cheb_filter(H, X, 1, a, b, a0) - ref).max() < 1e-14 * np.abs(ref).max()


def test_free_electron_elementwise():
    s = W.make_system(1, vloc_scale=0.0, d_scale=0.0)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 2, 1)
    a, b, a0 = 5.0, 20.0, 0.0
    Y = O.cheb_filter(H, X, 8, a, b, a0)
    ref = p_of(H.sphere.kinetic, 8, a, b, a0)[:, None] * X
    assert np.abs(Y - ref).max() < 1e-12 * np.abs(ref).max()


def test_lanczos_relation_and_bounds():
    s = tiny(tag=113)
    H = O.Hamiltonian.from_system(s)
    lam = np.linalg.eigvalsh(H.dense())
    v0 = W.random_vector(H.npw, 113)
    al, be, V, stopped = O.lanczos(H, v0, 10)
    assert not stopped and len(al) == 10 and len(be) == 10 and V.shape[1] == 11
    assert np.abs(V.conj().T @ V - np.eye(11)).max() < 1e-13
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    HV = H(V[:, :10])
    resid = HV - V[:, :10] @ T
    resid[:, -1] -= be[-1] * V[:, 10]
    assert np.abs(resid).max() < 1e-12 * np.abs(HV).max()
    theta = np.linalg.eigvalsh(T)
    assert theta[-1] <= lam[-1] + 1e-12 and theta[0] >= lam[0] - 1e-12
    b, _, _ = O.lanczos_upper_bound(H, v0, 10)
    assert b >= lam[-1]
    X = W.random_block(H.npw, 8, 113)
    a_, b_, a0_ = O.filter_bounds(H, X, v0)
    assert lam[0] <= a0_ <= a_ <= lam[-1] and b_ == b


def test_lanczos_stops_on_invariant_start():
    s = W.make_system(1, vloc_scale=0.0, d_scale=0.0)
    H = O.Hamiltonian.from_system(s)
    v0 = np.zeros(H.npw, dtype=np.complex128)
    v0[7] = 1.0
    b, al, be = O.lanczos_upper_bound(H, v0, 10)
    assert len(al) == 1 and b == H.sphere.kinetic[7]
