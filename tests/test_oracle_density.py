"""Pins for the oracle density (CPU only).

* Parseval: sum_r rho(r) = sum_n w_n ||psi_n||^2;
* a single plane wave gives the uniform density 1/n^3 per grid point;
* Hellmann-Feynman: for an exact eigenvector psi (unit norm) of the dense H,
  d lambda / d V(r) = rho_psi(r), checked by central differences of the dense
  eigenvalue along random directions of V.
"""
import numpy as np

import oracle as O
import workloads as W


def tiny(tag=141, **kw):
    base = dict(a=6.0, ecut=4.0, n=12, natom=2, nband=5, kpt_red=(0.1, 0.2, 0.3), d_scale=10.0)
    base.update(kw)
    return W.make_system(tag, **base)


def test_parseval_and_plane_wave():
    s = tiny()
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 4, 141)
    w = np.array([1.0, 0.5, 2.0, 0.0])
    rho = O.density(H, X, w)
    assert abs(rho.sum() - (np.linalg.norm(X, axis=0) ** 2 * w).sum()) <= 1e-12 * rho.sum()
    e = np.zeros((H.npw, 1), dtype=np.complex128)
    e[17, 0] = 1.0
    rho1 = O.density(H, e)
    assert np.abs(rho1 - 1.0 / rho1.size).max() <= 1e-15


def test_hellmann_feynman():
    s = tiny()
    H = O.Hamiltonian.from_system(s)
    lam, V = np.linalg.eigh(H.dense())
    n = 2
    rho = O.density(H, V[:, n:n + 1])
    rng = np.random.default_rng(4)
    h = 1e-5
    for _ in range(3):
        d = rng.standard_normal(s.vloc.shape)
        lp = np.linalg.eigvalsh(O.Hamiltonian(s.lattice, s.kpt_red, s.ecut, s.ngrid,
                                              s.vloc + h * d, s.tau, s.dij, s.rc).dense())[n]
        lm = np.linalg.eigvalsh(O.Hamiltonian(s.lattice, s.kpt_red, s.ecut, s.ngrid,
                                              s.vloc - h * d, s.tau, s.dij, s.rc).dense())[n]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - rho @ d) <= 1e-7 * abs(rho @ d)
