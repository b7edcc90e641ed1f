"""Pins for the oracle's orthonormalisation and Rayleigh-Ritz (CPU only).

* with M = N the Ritz values are the dense eigenvalues;
* Q = Y U^-1 is orthonormal and Y = Q U;
* Ritz values depend only on span(Y) (Y -> Y A);
* Cauchy interlacing: eps_n >= lambda_n;
* free electron with X = the lowest plane waves gives the sorted kinetic
  energies with the r3 multiplicities;
* residual norms vanish on an exact invariant subspace;
* filtering then Rayleigh-Ritz: a higher degree gives smaller residuals (the
  trend of the paper's degree/residual table).
"""
import numpy as np

import oracle as O
import workloads as W


def tiny(tag=121, **kw):
    base = dict(a=6.0, ecut=4.0, n=12, natom=2, nband=8, kpt_red=(0.1, 0.2, 0.3), d_scale=20.0)
    base.update(kw)
    return W.make_system(tag, **base)


def test_full_basis_gives_dense_spectrum():
    s = tiny()
    H = O.Hamiltonian.from_system(s)
    lam = np.linalg.eigvalsh(H.dense())
    Y = W.random_block(H.npw, H.npw, 121)
    rr = O.rayleigh_ritz(H, Y)
    assert np.abs(rr["eval"] - lam).max() < 1e-10
    res = O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"])
    assert res.max() < 1e-9


def test_orthonormalisation_and_invariance():
    s = tiny()
    H = O.Hamiltonian.from_system(s)
    lam = np.linalg.eigvalsh(H.dense())
    Y = W.random_block(H.npw, 10, 122)
    G = O.gram(Y)
    U = O.cholesky_upper(G)
    assert np.allclose(np.tril(U, -1), 0) and np.all(np.diag(U).real > 0)
    assert np.abs(U.conj().T @ U - G).max() < 1e-12 * np.abs(G).max()
    rr = O.rayleigh_ritz(H, Y)
    Psi = rr["Psi"]
    assert np.abs(Psi.conj().T @ Psi - np.eye(10)).max() < 1e-12
    rng = np.random.default_rng(5)
    A = rng.standard_normal((10, 10)) + 1j * rng.standard_normal((10, 10))
    rr2 = O.rayleigh_ritz(H, Y @ A)
    assert np.abs(rr2["eval"] - rr["eval"]).max() < 1e-10
    assert np.all(rr["eval"] >= lam[:10] - 1e-12)


def test_free_electron_lowest_plane_waves():
    s = W.make_system(1, vloc_scale=0.0, d_scale=0.0)
    H = O.Hamiltonian.from_system(s)
    order = np.argsort(H.sphere.kinetic, kind="stable")[:27]  # shells 0..3: 1+6+12+8
    Y = np.zeros((H.npw, 27), dtype=np.complex128)
    Y[order, np.arange(27)] = 1.0
    rr = O.rayleigh_ritz(H, Y)
    unit = 0.5 * (2 * np.pi / s.a) ** 2
    want = np.array([0] * 1 + [1] * 6 + [2] * 12 + [3] * 8) * unit
    assert np.abs(rr["eval"] - want).max() < 1e-14 * 10
    assert O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"]).max() < 1e-13


def test_higher_degree_smaller_residual():
    s = tiny(tag=123)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 8, 123)
    v0 = W.random_vector(H.npw, 123)
    a, b, a0 = O.filter_bounds(H, X, v0)
    worst = []
    for deg in (4, 14):
        Y = O.cheb_filter(H, X, deg, a, b, a0)
        rr = O.rayleigh_ritz(H, Y)
        worst.append(O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"])[:4].max())
    assert worst[1] < worst[0]


def test_repeated_cycles_converge_to_dense_spectrum():
    """Subspace iteration (bounds from the current block, filter, Rayleigh-Ritz,
    repeated) converges to the lowest eigenpairs of the dense operator."""
    s = tiny(tag=124, nband=10)
    H = O.Hamiltonian.from_system(s)
    lam = np.linalg.eigvalsh(H.dense())
    X = W.random_block(H.npw, 10, 124)
    v0 = W.random_vector(H.npw, 124)
    for _ in range(30):
        a, b, a0 = O.filter_bounds(H, X, v0)
        rr = O.rayleigh_ritz(H, O.cheb_filter(H, X, 8, a, b, a0))
        X = rr["Psi"]
        res = O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"])
        if res[:6].max() < 1e-10:
            break
    assert res[:6].max() < 1e-10
    assert np.abs(rr["eval"][:6] - lam[:6]).max() < 1e-12
