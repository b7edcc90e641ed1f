"""Generalised problem H psi = lambda S psi with a projector overlap S (oracle).

Paper: with PAW or ultrasoft pseudopotentials the pseudo wave functions are
not orthonormal and the Kohn-Sham problem carries an overlap operator S != I
(sections "Introduction" and "Problem setup"); S is applied beside H
(the HX_SX kernel), its inverse by a Woodbury formula (the Sinv kernel,
section "Main computational kernels", cost O(N_projs^2) + O(N_projs N) per
band, section "Floating-point operation count").  The filter applies a
polynomial of S^-1 H (Algorithm "Parallel Chebyshev filtering of degree k":
Rayleigh quotients from H Psi and S Psi, then per step S^-1 H Psi, the
recurrence, H Psi and S Psi again), and the Rayleigh-Ritz step uses the
S-Gram S_Psi = Psi^H (S Psi) (Algorithms "S-ortho" and "RR"), the residual
being W = (H - Lambda S) Psi.

Readings where the paper is silent (the PAW datasets are not part of it):

* S = I + sum_R P_R Q_R P_R^H with the projectors of H and one Hermitian 4x4
  Q_R per atom (the same block structure as D); S must be positive definite;
* S^-1 = I - P K P^H with K = Q (I + B Q)^-1 = (I + Q B)^-1 Q, B = P^H P (the
  Woodbury identity in the form that also holds for a singular Q);
* Rayleigh quotients RQ_i = Re(x_i^H H x_i) / Re(x_i^H S x_i);
* the Lanczos run for the upper bound works on S^-1 H in the S inner product
  <u, v>_S = u^H S v (in which S^-1 H is self-adjoint), with full
  S-reorthogonalisation; otherwise as for S = I (b = theta_max + beta_last,
  early stop at beta_j <= 1e-12 max(1, |alpha_j|));
* residual norms are Euclidean: ||H psi_n - lambda_n S psi_n||_2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import Hamiltonian
from .chebyshev import _tridiag_max


class Overlap:
    """S = I + P Q P^H for the projectors P of a Hamiltonian."""

    def __init__(self, H: Hamiltonian, qij):
        self.P = H.P
        self.qij = np.asarray(qij, dtype=np.complex128).reshape(-1, 4, 4)
        if self.qij.shape[0] != H.tau.shape[0]:
            raise ValueError("one 4x4 Q per atom")
        n = H.nproj
        Q = np.zeros((n, n), dtype=np.complex128)
        for r in range(self.qij.shape[0]):
            Q[4 * r:4 * r + 4, 4 * r:4 * r + 4] = self.qij[r]
        self.Q = Q
        self.B = self.P.conj().T @ self.P
        # Woodbury: S^-1 = I - P K P^H, K = (I + Q B)^-1 Q
        self.K = np.linalg.solve(np.eye(n) + Q @ self.B, Q) if n else Q

    @classmethod
    def from_system(cls, H: Hamiltonian, sys) -> "Overlap":
        q = sys.qij if sys.qij is not None else np.zeros((sys.natom, 4, 4))
        return cls(H, q)

    def apply(self, X):
        """S X = X + P (Q (P^H X))."""
        X = np.asarray(X, dtype=np.complex128)
        X2 = X.reshape(self.P.shape[0], -1)
        return (X2 + self.P @ (self.Q @ (self.P.conj().T @ X2))).reshape(X.shape)

    __call__ = apply

    def inv_apply(self, X):
        """S^-1 X = X - P (K (P^H X))."""
        X = np.asarray(X, dtype=np.complex128)
        X2 = X.reshape(self.P.shape[0], -1)
        return (X2 - self.P @ (self.K @ (self.P.conj().T @ X2))).reshape(X.shape)

    def dense(self) -> np.ndarray:
        return np.eye(self.P.shape[0]) + self.P @ self.Q @ self.P.conj().T


def sinv_h(H: Hamiltonian, S: Overlap):
    """The operator the filter is a polynomial of: X -> S^-1 (H X)."""
    return lambda X: S.inv_apply(H.apply(X))


def rayleigh_quotients_gen(X, HX, SX) -> np.ndarray:
    X = np.asarray(X).reshape(X.shape[0], -1)
    num = np.real(np.einsum("ij,ij->j", X.conj(), np.asarray(HX).reshape(X.shape)))
    den = np.real(np.einsum("ij,ij->j", X.conj(), np.asarray(SX).reshape(X.shape)))
    return num / den


def lanczos_gen(apply_H, apply_S, apply_Sinv, v0, nsteps: int = 10):
    """Lanczos on A = S^-1 H in the S inner product, full S-reorthogonalisation.

    Returns (alphas, betas, V, stopped) as the S = I routine does; the columns of
    V are S-orthonormal and alphas[j] = Re(v_j^H H v_j).
    """
    v = np.asarray(v0, dtype=np.complex128)
    v = v / np.sqrt(np.real(np.vdot(v, apply_S(v))))
    V, SV = [v], [apply_S(v)]
    alphas, betas = [], []
    beta_prev = 0.0
    v_prev = np.zeros_like(v)
    for j in range(nsteps):
        w = apply_Sinv(apply_H(V[j])) - beta_prev * v_prev
        alpha = float(np.real(np.vdot(SV[j], w)))
        w = w - alpha * V[j]
        Vm, SVm = np.stack(V, axis=1), np.stack(SV, axis=1)
        w = w - Vm @ (SVm.conj().T @ w)
        Sw = apply_S(w)
        beta = float(np.sqrt(max(np.real(np.vdot(w, Sw)), 0.0)))
        alphas.append(alpha)
        if beta <= 1e-12 * max(1.0, abs(alpha)):
            return np.array(alphas), np.array(betas), Vm, True
        betas.append(beta)
        v_prev = V[j]
        beta_prev = beta
        V.append(w / beta)
        SV.append(Sw / beta)
    return np.array(alphas), np.array(betas), np.stack(V, axis=1), False


def lanczos_upper_bound_gen(apply_H, apply_S, apply_Sinv, v0, nsteps: int = 10):
    alphas, betas, _, stopped = lanczos_gen(apply_H, apply_S, apply_Sinv, v0, nsteps)
    if stopped:
        return _tridiag_max(alphas, betas), alphas, betas
    return _tridiag_max(alphas, betas[:-1]) + betas[-1], alphas, betas


def filter_bounds_gen(H: Hamiltonian, S: Overlap, X, v0, nlanczos: int = 10):
    """(a, b, a0): generalised Rayleigh quotients of X and the S-Lanczos bound."""
    rq = rayleigh_quotients_gen(X, H.apply(X), S.apply(X))
    b, _, _ = lanczos_upper_bound_gen(H.apply, S.apply, S.inv_apply, v0, nlanczos)
    return float(rq.max()), float(b), float(rq.min())


def rayleigh_ritz_gen(apply_H, apply_S, Y):
    """Returns dict(eval, Psi, HPsi, SPsi, U, Z): S_Psi = Y^H S Y = U^H U,
    Q = Y U^-1, H_s = Q^H (H Q) = Z Lambda Z^H, Psi = Q Z (S-orthonormal)."""
    Y = np.asarray(Y, dtype=np.complex128)
    G = Y.conj().T @ apply_S(Y)
    G = 0.5 * (G + G.conj().T)
    U = scipy.linalg.cholesky(G, lower=False)
    Q = scipy.linalg.solve_triangular(U.T, Y.T, lower=True).T  # Q U = Y
    HQ = apply_H(Q)
    SQ = apply_S(Q)
    Hs = Q.conj().T @ HQ
    Hs = 0.5 * (Hs + Hs.conj().T)
    lam, Z = scipy.linalg.eigh(Hs)
    return dict(eval=lam, Psi=Q @ Z, HPsi=HQ @ Z, SPsi=SQ @ Z, U=U, Z=Z, Hs=Hs)


def residual_norms_gen(HPsi, SPsi, lam) -> np.ndarray:
    """||H psi_n - lambda_n S psi_n||_2 per column."""
    return np.linalg.norm(HPsi - SPsi * lam[None, :], axis=0)
