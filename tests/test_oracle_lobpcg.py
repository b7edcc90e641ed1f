"""Pins for the oracle's block LOBPCG (CPU only).

* the Teter-Payne-Allan diagonal: K = 65/81 at x = 1, K = 1 at x = 0, and
  K -> 1/(2x) for large x, on a band made of one plane wave;
* one block, one line minimisation: the Ritz values are the lowest m Ritz
  values of the plain generalised Rayleigh-Ritz on [Psi_RR, K W] (the
  2m-sized step written with the textbook routine);
* Ritz values never increase from pass to pass and stay above the exact
  generalised eigenvalues (each Rayleigh-Ritz basis contains the current Psi;
  Cauchy interlacing);
* passes converge to the lowest pairs of the dense pencil (H, S) with one and
  with three blocks; the result is S-orthonormal.
"""
import numpy as np
import scipy.linalg

import oracle as O
import workloads as W


def tiny(tag=141, **kw):
    base = dict(a=6.0, ecut=5.0, n=12, natom=2, nband=12, kpt_red=(0.1, 0.2, 0.3), d_scale=20.0,
                q_scale=W.PAW_Q_SCALE)
    base.update(kw)
    return W.make_system(tag, **base)


def pencil(s):
    H = O.Hamiltonian.from_system(s)
    S = O.Overlap.from_system(H, s)
    return H, S, scipy.linalg.eigh(H.dense(), S.dense(), eigvals_only=True)


def test_tpa_closed_form():
    kin = np.array([0.0, 0.5, 2.0, 1e3])
    Psi = np.zeros((4, 1), dtype=np.complex128)
    Psi[1, 0] = 3.0  # E_kin(psi) = 0.5
    Wv = np.ones((4, 1), dtype=np.complex128)
    K = O.tpa_precondition(kin, Psi, Wv)[:, 0].real
    assert K[0] == 1.0
    assert abs(K[1] - 65.0 / 81.0) < 1e-15
    x = 4.0
    p = 27 + 18 * x + 12 * x ** 2 + 8 * x ** 3
    assert abs(K[2] - p / (p + 16 * x ** 4)) < 1e-15
    assert abs(K[3] * 2 * 2000.0 - 1.0) < 2e-3


def test_single_step_is_rayleigh_ritz_on_psi_and_kw():
    s = tiny()
    H, S, lam = pencil(s)
    m = 6
    X = W.random_block(H.npw, m, 142)
    r = O.lobpcg_pass(H.apply, S.apply, H.sphere.kinetic, X, 1, 1, 0.0)
    rr0 = O.rayleigh_ritz_gen(H.apply, S.apply, X)
    Xr = rr0["Psi"]
    Wr = rr0["HPsi"] - rr0["SPsi"] * rr0["eval"][None, :]
    KW = O.tpa_precondition(H.sphere.kinetic, Xr, Wr)
    rr = O.rayleigh_ritz_gen(H.apply, S.apply, np.hstack([Xr, KW]))
    assert np.abs(r["eval"] - rr["eval"][:m]).max() < 1e-10
    assert r["steps"] == [1]


def test_monotone_and_above_exact():
    s = tiny()
    H, S, lam = pencil(s)
    M = 8
    X = W.random_block(H.npw, M, 143)
    prev = None
    for _ in range(4):
        r = O.lobpcg_pass(H.apply, S.apply, H.sphere.kinetic, X, 1, 2, 0.0)
        assert np.all(r["eval"] >= lam[:M] - 1e-10)
        if prev is not None:
            assert np.all(r["eval"] <= prev + 1e-10)
        prev = r["eval"]
        X = r["Psi"]


def test_converges_to_dense_pencil():
    s = tiny()
    H, S, lam = pencil(s)
    Sd = S.dense()
    for nblocks in (1, 3):
        X = W.random_block(H.npw, 12, 144)
        for _ in range(12):
            r = O.lobpcg_pass(H.apply, S.apply, H.sphere.kinetic, X, nblocks, 4, 1e-11)
            X = r["Psi"]
            if r["res"][:8].max() < 1e-9:
                break
        assert np.abs(r["eval"][:8] - lam[:8]).max() < 1e-10
        assert r["res"][:8].max() < 1e-9
        assert np.abs(X.conj().T @ Sd @ X - np.eye(12)).max() < 1e-10
