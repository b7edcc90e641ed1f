"""Adjoint of the Chebyshev filter (oracle).

The paper does not differentiate the solver; this follows the reverse mode of
the filter recurrence it describes (the "axpy" recurrence of section "Parallel
implementation design") for the loss L = sum_n Re<W_n, Y_{m,n}>, <u,v> = u^H v.

Forward, with gamma_0 = sigma_1/e, gamma_k = 2 sigma_{k+1}/e, delta_k =
sigma_k sigma_{k+1} (k >= 1):
    Y_1 = gamma_0 (H - c) Y_0,   Y_{k+1} = gamma_k (H - c) Y_k - delta_k Y_{k-1}.
Reverse (A_k = dL/dY_k with the gradient convention dRe + i dIm):
    A_m = W;  for k = m-1 .. 0:  A_k += gamma_k (H - c) A_{k+1},
                                 A_{k-1} -= delta_k A_{k+1} (k >= 1);
    dX = A_0.
Each forward term gamma_k (H - c) Y_k contributes gamma_k Re<A_{k+1}, dH Y_k>:
    dV(r)  += gamma_k sum_n Re[conj(A~_{k+1,n}(r)) Y~_{k,n}(r)] / n^3,
    dD_R   += gamma_k (P_R^H A_{k+1}) (P_R^H Y_k)^H,
where ~ is the unnormalised inverse FFT of the scattered sphere vector and D
entries are treated as independent complex numbers (no Hermitian projection).
The bounds (a, b, a0) are held fixed.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .chebyshev import cheb_sigmas
from .hamiltonian import _WORKERS


def filter_coefficients(degree: int, a: float, b: float, a0: float):
    """(gamma[0..m-1], delta[0..m-1], c) of the scaled recurrence (delta[0] unused)."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sig = cheb_sigmas(degree, a, b, a0)
    gamma = np.empty(degree)
    delta = np.zeros(degree)
    gamma[0] = sig[0] / e
    for k in range(1, degree):
        gamma[k] = 2.0 * sig[k] / e
        delta[k] = sig[k - 1] * sig[k]
    return gamma, delta, c


def filter_iterates(H, X, degree, a, b, a0):
    """[Y_0, ..., Y_m] of the forward recurrence."""
    gamma, delta, c = filter_coefficients(degree, a, b, a0)
    Y = [np.asarray(X, dtype=np.complex128)]
    Y.append(gamma[0] * (H(Y[0]) - c * Y[0]))
    for k in range(1, degree):
        Y.append(gamma[k] * (H(Y[k]) - c * Y[k]) - delta[k] * Y[k - 1])
    return Y


def _real_space(H, Z):
    """Unnormalised inverse FFT of the scattered sphere columns, (n3, n2, n1, nb)."""
    box = H.to_box(Z)
    return scipy.fft.ifftn(box, axes=(0, 1, 2), norm="forward", workers=_WORKERS)


def filter_backward(H, X, W, degree, a, b, a0):
    """Returns (dV (n1*n2*n3,), dD (natom, 4, 4), dX (npw, nb)) of L = Re<W, Y_m>."""
    gamma, delta, c = filter_coefficients(degree, a, b, a0)
    X = np.asarray(X, dtype=np.complex128).reshape(H.npw, -1)
    W = np.asarray(W, dtype=np.complex128).reshape(H.npw, -1)
    Y = filter_iterates(H, X, degree, a, b, a0)
    n1, n2, n3 = H.ngrid
    ntot = n1 * n2 * n3
    natom = H.tau.shape[0]
    dV = np.zeros(ntot)
    dD = np.zeros((natom, 4, 4), dtype=np.complex128)
    A = [None] * (degree + 1)
    A[degree] = W.copy()
    for k in range(degree - 1, -1, -1):
        Ak1 = A[k + 1]
        # parameter gradients of the term gamma_k (H - c) Y_k
        ra = _real_space(H, Ak1)
        ry = _real_space(H, Y[k])
        dV += gamma[k] * np.real(np.conj(ra) * ry).sum(axis=3).reshape(-1) / ntot
        ca = (H.P.conj().T @ Ak1).reshape(natom, 4, -1)
        cy = (H.P.conj().T @ Y[k]).reshape(natom, 4, -1)
        dD += gamma[k] * np.einsum("rib,rjb->rij", ca, cy.conj())
        # reverse recurrence
        contrib = gamma[k] * (H(Ak1) - c * Ak1)
        A[k] = contrib if A[k] is None else A[k] + contrib
        if k >= 1:
            A[k - 1] = -delta[k] * Ak1
    return dV, dD, A[0]


def filter_loss(H, X, W, degree, a, b, a0) -> float:
    Y = filter_iterates(H, X, degree, a, b, a0)[-1]
    return float(np.real(np.vdot(W, Y)))
