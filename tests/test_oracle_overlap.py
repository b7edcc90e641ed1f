"""Pins for the oracle's generalised problem H psi = lambda S psi (CPU only).

* Q = 0 gives S = S^-1 = I exactly and the S = I routines' results;
* one atom with only the s channel: S^-1 is the Sherman-Morrison closed form
  I - q p p^H / (1 + q |p|^2);
* the Woodbury S^-1 inverts the explicit matrix I + P Q P^H, which is
  Hermitian and positive definite for the indefinite Q of the recipe;
* Rayleigh-Ritz over the whole basis gives the generalised eigenvalues of the
  dense pencil (scipy.linalg.eigh(H, S), a different algorithm);
* the filter of an exact generalised eigenvector scales it by
  T_m((lam - c)/e) / T_m((a0 - c)/e) (NumPy's Chebyshev series);
* the S-Lanczos run over the whole Krylov space returns lambda_max(H, S),
  and its basis is S-orthonormal;
* the generalised Rayleigh quotient of an eigenvector is its eigenvalue;
* filter + Rayleigh-Ritz cycles converge to the lowest generalised pairs.
"""
import numpy as np
import numpy.polynomial.chebyshev as npcheb
import scipy.linalg

import oracle as O
import workloads as W
from oracle.overlap import (
    Overlap,
    filter_bounds_gen,
    lanczos_gen,
    lanczos_upper_bound_gen,
    rayleigh_quotients_gen,
    rayleigh_ritz_gen,
    residual_norms_gen,
    sinv_h,
)


def tiny(tag=131, **kw):
    base = dict(a=6.0, ecut=4.0, n=12, natom=2, nband=8, kpt_red=(0.1, 0.2, 0.3), d_scale=20.0,
                q_scale=W.PAW_Q_SCALE)
    base.update(kw)
    return W.make_system(tag, **base)


def dense_pencil(s):
    H = O.Hamiltonian.from_system(s)
    S = Overlap.from_system(H, s)
    return H, S, H.dense(), S.dense()


def test_zero_q_is_identity():
    s = tiny(q_scale=0.0)
    assert s.qij is None
    H = O.Hamiltonian.from_system(s)
    S = Overlap.from_system(H, s)
    X = W.random_block(H.npw, 5, 131)
    assert np.array_equal(S.apply(X), X)
    assert np.array_equal(S.inv_apply(X), X)
    v0 = W.random_vector(H.npw, 131)
    al, be, _, _ = O.lanczos(H, v0, 10)
    ag, bg, _, _ = lanczos_gen(H.apply, S.apply, S.inv_apply, v0, 10)
    assert np.abs(al - ag).max() < 1e-12 and np.abs(be - bg).max() < 1e-12
    r1 = O.rayleigh_ritz(H, X)
    r2 = rayleigh_ritz_gen(H.apply, S.apply, X)
    assert np.abs(r1["eval"] - r2["eval"]).max() < 1e-12
    assert np.abs(r1["Psi"] - r2["Psi"]).max() < 1e-12


def test_sherman_morrison_single_channel():
    s = tiny(natom=1)
    H = O.Hamiltonian.from_system(s)
    q = 7.5
    Q = np.zeros((1, 4, 4), dtype=np.complex128)
    Q[0, 0, 0] = q
    S = Overlap(H, Q)
    p = H.P[:, 0]
    X = W.random_block(H.npw, 3, 132)
    closed = X - np.outer(p, p.conj() @ X) * (q / (1.0 + q * np.vdot(p, p).real))
    assert np.abs(S.inv_apply(X) - closed).max() < 1e-13 * np.abs(X).max()
    assert np.abs(S.apply(X) - (X + q * np.outer(p, p.conj() @ X))).max() < 1e-13 * np.abs(X).max()


def test_woodbury_inverts_dense_overlap():
    s = tiny()
    H, S, Hd, Sd = dense_pencil(s)
    assert np.linalg.eigvalsh(S.Q).min() < 0  # the recipe's Q is indefinite
    assert np.abs(Sd - Sd.conj().T).max() < 1e-15
    ev = np.linalg.eigvalsh(Sd)
    assert ev.min() > 0.5 and ev.max() > 1.05
    X = W.random_block(H.npw, 6, 133)
    assert np.abs(S.apply(X) - Sd @ X).max() < 1e-12 * np.abs(X).max()
    assert np.abs(Sd @ S.inv_apply(X) - X).max() < 1e-12 * np.abs(X).max()
    assert np.abs(S.inv_apply(X) - np.linalg.solve(Sd, X)).max() < 1e-12 * np.abs(X).max()


def test_full_basis_gives_generalised_spectrum():
    s = tiny()
    H, S, Hd, Sd = dense_pencil(s)
    lam = scipy.linalg.eigh(Hd, Sd, eigvals_only=True)
    assert np.abs(lam - np.linalg.eigvalsh(Hd)).max() > 1e-3  # S really changes the spectrum
    Y = W.random_block(H.npw, H.npw, 134)
    rr = rayleigh_ritz_gen(H.apply, S.apply, Y)
    assert np.abs(rr["eval"] - lam).max() < 1e-10
    Psi = rr["Psi"]
    assert np.abs(Psi.conj().T @ (Sd @ Psi) - np.eye(H.npw)).max() < 1e-10
    assert residual_norms_gen(rr["HPsi"], rr["SPsi"], rr["eval"]).max() < 1e-9


def test_filter_scales_generalised_eigenvectors():
    s = tiny()
    H, S, Hd, Sd = dense_pencil(s)
    lam, V = scipy.linalg.eigh(Hd, Sd)
    a, b, a0 = lam[6], lam[-1] + 0.5, lam[0]
    degree = 7
    e, c = (b - a) / 2.0, (b + a) / 2.0
    coef = np.zeros(degree + 1)
    coef[-1] = 1.0
    for i in (0, 3, 10, len(lam) - 1):
        y = O.cheb_filter(sinv_h(H, S), V[:, i:i + 1], degree, a, b, a0)
        ratio = npcheb.chebval((lam[i] - c) / e, coef) / npcheb.chebval((a0 - c) / e, coef)
        assert np.abs(y[:, 0] - ratio * V[:, i]).max() < 1e-10 * max(1.0, abs(ratio))
        rq = rayleigh_quotients_gen(V[:, i:i + 1], Hd @ V[:, i:i + 1], Sd @ V[:, i:i + 1])
        assert abs(rq[0] - lam[i]) < 1e-10


def test_lanczos_full_krylov_space():
    s = tiny(ecut=2.0)
    H, S, Hd, Sd = dense_pencil(s)
    N = H.npw
    lam = scipy.linalg.eigh(Hd, Sd, eigvals_only=True)
    v0 = W.random_vector(N, 135)
    alphas, betas, V, stopped = lanczos_gen(H.apply, S.apply, S.inv_apply, v0, N)
    k = len(alphas)
    G = V[:, :k].conj().T @ Sd @ V[:, :k]
    assert np.abs(G - np.eye(k)).max() < 1e-10
    T = np.diag(alphas) + np.diag(betas[:k - 1], 1) + np.diag(betas[:k - 1], -1)
    theta = np.linalg.eigvalsh(T)
    assert abs(theta[-1] - lam[-1]) < 1e-8 and abs(theta[0] - lam[0]) < 1e-8
    b10, _, _ = lanczos_upper_bound_gen(H.apply, S.apply, S.inv_apply, v0, 10)
    assert b10 >= lam[-1] - 1e-9


def test_cycles_converge_to_lowest_generalised_pairs():
    s = tiny(ecut=5.0)
    H, S, Hd, Sd = dense_pencil(s)
    lam = scipy.linalg.eigh(Hd, Sd, eigvals_only=True)
    M, nconv = 12, 6
    X = W.random_block(H.npw, M, 136)
    v0 = W.random_vector(H.npw, 136)
    res_first = None
    for cycle in range(12):
        a, b, a0 = filter_bounds_gen(H, S, X, v0)
        Y = O.cheb_filter(sinv_h(H, S), X, 8, a, b, a0)
        rr = rayleigh_ritz_gen(H.apply, S.apply, Y)
        res = residual_norms_gen(rr["HPsi"], rr["SPsi"], rr["eval"])
        res_first = res[:nconv].max() if res_first is None else res_first
        X = rr["Psi"]
    assert np.abs(rr["eval"][:nconv] - lam[:nconv]).max() < 1e-9
    assert res[:nconv].max() < 1e-6 < res_first
