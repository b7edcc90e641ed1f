"""Pins for the oracle Hamiltonian (CPU only).

* dense explicit matrix (definition of V_L from the Fourier coefficients of V)
  against the matrix-free FFT apply, with a shifted k-point;
* Hermiticity;
* free electron: V = 0 and D = 0 gives H X = kin * X exactly;
* constant potential: V = c adds exactly c;
* projector normalisation and phase against closed forms from the Poisson sum
  of a Gaussian (a dropped 1/2, 1/sqrt(Omega) or a flipped phase sign fails);
* translating atoms and V by a grid vector conjugates H by a diagonal phase.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def tiny(tag=101, **kw):
    base = dict(a=6.0, ecut=4.0, n=12, natom=2, nband=8, kpt_red=(0.1, 0.2, 0.3))
    base.update(kw)
    return W.make_system(tag, **base)


@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.1, 0.2, 0.3)])
def test_dense_equals_matrix_free(kpt):
    s = tiny(kpt_red=kpt, d_scale=30.0)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 6, 101)
    ref = H.dense() @ X
    got = H(X)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # each part separately
    Hd = H.dense_local() @ X
    assert np.abs(H.local_apply(X) - Hd).max() <= 1e-13 * np.abs(Hd).max()


def test_hermitian():
    s = tiny(d_scale=10.0)
    H = O.Hamiltonian.from_system(s)
    Hd = H.dense()
    assert np.abs(Hd - Hd.conj().T).max() < 1e-14 * np.abs(Hd).max()
    x = W.random_block(H.npw, 1, 102)[:, 0]
    y = W.random_block(H.npw, 1, 103)[:, 0]
    lhs = np.vdot(x, H(y))
    rhs = np.vdot(H(x), y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_free_electron_exact():
    s = W.make_system(1, vloc_scale=0.0, d_scale=0.0)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 4, 1)
    assert np.array_equal(H(X), H.sphere.kinetic[:, None] * X)


def test_constant_potential_shift():
    s = tiny(d_scale=0.0)
    s.vloc = np.full_like(s.vloc, -1.75)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 3, 104)
    assert np.abs(H.local_apply(X) + 1.75 * X).max() < 1e-14 * 1.75 * np.abs(X).max() * 10


def _image_sum(d, a, fn):
    tot = 0.0
    for l1 in range(-3, 4):
        for l2 in range(-3, 4):
            for l3 in range(-3, 4):
                x = d + a * np.array([l1, l2, l3])
                tot = tot + fn(x)
    return tot


def test_projector_closed_forms():
    """sum_G conj(p(R1)) p(R2) from Poisson summation of Gaussians (rc = 1).

    (1/Omega) sum_G exp(-G^2 rc^2) e^{iG.x} = (8 pi^1.5 rc^3)^-1 sum_L exp(-|x+L|^2/(4 rc^2))
    and the q_c moment gives the factor i (x+L)_c / (2 rc).  The sphere cut at
    |q|^2 < 20 leaves a tail of relative size ~1e-8.
    """
    s = W.make_system(1)
    H = O.Hamiltonian.from_system(s)
    P = H.P
    rc = s.rc
    pref = 1.0 / (8.0 * math.pi ** 1.5 * rc ** 3)
    # self overlaps
    assert abs(np.vdot(P[:, 0], P[:, 0]).real - pref) < 1e-7 * pref
    assert abs(np.vdot(P[:, 1], P[:, 1]).real - pref / 2.0) < 1e-7 * pref
    # cross-atom, s-s and s-p: sum conj(p(R1)) p(R2) with d = R1 - R2
    d = s.tau[0] - s.tau[1]
    ss = _image_sum(d, s.a, lambda x: pref * math.exp(-np.dot(x, x) / (4 * rc * rc)))
    got_ss = np.vdot(P[:, 0], P[:, 4])
    assert abs(got_ss - ss) < 1e-7 * pref
    for c in range(3):
        sp = _image_sum(d, s.a, lambda x: pref * 1j * x[c] / (2 * rc)
                        * math.exp(-np.dot(x, x) / (4 * rc * rc)))
        got_sp = np.vdot(P[:, 0], P[:, 4 + 1 + c])
        assert abs(got_sp - sp) < 1e-7 * pref, c


def test_translation_covariance():
    s = tiny(tag=105, kpt_red=(0.0, 0.0, 0.0), d_scale=20.0)
    H = O.Hamiltonian.from_system(s)
    shift = np.array([3, 5, 7])  # grid steps
    t = shift * (s.a / s.ngrid[0])
    s2 = tiny(tag=105, kpt_red=(0.0, 0.0, 0.0), d_scale=20.0)
    s2.tau = s.tau + t
    n = s.ngrid[0]
    v = s.vloc.reshape(n, n, n)  # (i3, i2, i1)
    s2.vloc = np.roll(v, shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2)).reshape(-1)
    H2 = O.Hamiltonian.from_system(s2)
    phi = np.exp(-1j * (H.sphere.gcart @ t))
    A = H.dense()
    B = H2.dense()
    ref = (phi[:, None] * A) * phi.conj()[None, :]
    assert np.abs(B - ref).max() < 1e-12 * np.abs(A).max()
    assert np.allclose(np.linalg.eigvalsh(A), np.linalg.eigvalsh(B), atol=1e-11)
