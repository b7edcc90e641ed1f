"""Cholesky orthonormalisation, Rayleigh-Ritz and residuals (oracle, S = I).

Paper: S-orthogonalisation computes S_Psi = Psi^H (S Psi), its Cholesky factor
S_Psi = U^H U and Psi <- Psi U^-1 (Algorithm "S-ortho"); the Rayleigh-Ritz
procedure projects H on the trial block, solves the small generalised
Hermitian problem H_Psi X = Lambda S_Psi X and rotates Psi, H Psi by X
(Algorithms "Rayleigh-Ritz procedure", "Matrix-free Rayleigh-Ritz procedure",
"RR"); the cycle ends with W = (H - Lambda S) Psi and its column norms
(Algorithm "Parallel Chebyshev filtering of degree k").

Readings: the transposes printed in those algorithms are conjugate transposes
(the matrices are Hermitian and the solver is a Hermitian one); the small
matrices are symmetrised (A + A^H)/2 before factorisation; U is the upper
factor with a real positive diagonal; Ritz values are returned ascending.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def gram(Y) -> np.ndarray:
    G = Y.conj().T @ Y
    return 0.5 * (G + G.conj().T)


def cholesky_upper(G) -> np.ndarray:
    """U upper triangular with real positive diagonal, G = U^H U."""
    return scipy.linalg.cholesky(G, lower=False)


def rayleigh_ritz(apply_H, Y):
    """Returns dict(eval, Psi, HPsi, U, Z) for the block Y (N x M).

    Q = Y U^-1 (Cholesky of the Gram), H_s = Q^H (H Q), H_s = Z Lambda Z^H,
    Psi = Q Z, H Psi = (H Q) Z.
    """
    Y = np.asarray(Y, dtype=np.complex128)
    U = cholesky_upper(gram(Y))
    Q = scipy.linalg.solve_triangular(U.T, Y.T, lower=True).T  # Q U = Y
    HQ = apply_H(Q)
    Hs = Q.conj().T @ HQ
    Hs = 0.5 * (Hs + Hs.conj().T)
    lam, Z = scipy.linalg.eigh(Hs)
    return dict(eval=lam, Psi=Q @ Z, HPsi=HQ @ Z, U=U, Z=Z, Hs=Hs)


def residual_norms(Psi, HPsi, lam) -> np.ndarray:
    """||H psi_n - lambda_n psi_n||_2 per column."""
    R = HPsi - Psi * lam[None, :]
    return np.linalg.norm(R, axis=0)
