"""Chebyshev spectral filter and its bounds (oracle).

Paper: the filtering solver starts from Rayleigh quotients (one H application),
takes their minimum and maximum, then applies k filter steps, each one H
application combined through a recurrence of the form X <- aX + Y
(Algorithm "Spectral polynomial filtering of degree k", Algorithm "Parallel
Chebyshev filtering of degree k", section "Parallel implementation design").
The Rayleigh quotient of band i is (H psi_i)^H psi_i / (S psi_i)^H psi_i, S = I.

Readings (the cited filter papers are not part of the text):

* bounds: lower edge of the damped interval a = max_i RQ_i, scaling point
  a0 = min_i RQ_i, upper edge b from a 10-step Lanczos run started from a given
  vector v0 with full reorthogonalisation: b = theta_max(T) + beta_last; the run
  stops early (b = theta_max) when beta_j <= 1e-12 * max(1, |alpha_j|);
* filter: the scaled three-term Chebyshev recurrence
  e = (b - a)/2, c = (b + a)/2, sigma_1 = e/(a0 - c),
  sigma_{k+1} = 1/(2/sigma_1 - sigma_k),
  Y_1 = (sigma_1/e)(H - c)Y_0,
  Y_{k+1} = (2 sigma_{k+1}/e)(H - c)Y_k - sigma_k sigma_{k+1} Y_{k-1},
  whose output is T_m((H - c)/e) X / T_m((a0 - c)/e); "degree m" counts the m
  H applications inside the filter.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def rayleigh_quotients(X, HX) -> np.ndarray:
    X = np.asarray(X).reshape(X.shape[0], -1)
    HX = np.asarray(HX).reshape(X.shape)
    num = np.real(np.einsum("ij,ij->j", X.conj(), HX))
    den = np.real(np.einsum("ij,ij->j", X.conj(), X))
    return num / den


def lanczos(apply_H, v0, nsteps: int = 10):
    """Lanczos with full reorthogonalisation.

    Returns (alphas, betas, V, stopped): alphas[j] = Re(v_j^H H v_j); betas[j]
    is the norm of the j-th residual (one entry per completed step, so the
    last one is beta_last unless the run stopped early); V holds the
    orthonormal basis as columns (one more column than alphas unless stopped).
    """
    v = np.asarray(v0, dtype=np.complex128) / np.linalg.norm(v0)
    V = [v]
    alphas, betas = [], []
    beta_prev = 0.0
    v_prev = np.zeros_like(v)
    for j in range(nsteps):
        w = apply_H(V[j]) - beta_prev * v_prev
        alpha = float(np.real(np.vdot(V[j], w)))
        w = w - alpha * V[j]
        Vm = np.stack(V, axis=1)
        w = w - Vm @ (Vm.conj().T @ w)
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        if beta <= 1e-12 * max(1.0, abs(alpha)):
            return np.array(alphas), np.array(betas), np.stack(V, axis=1), True
        betas.append(beta)
        v_prev = V[j]
        beta_prev = beta
        V.append(w / beta)
    return np.array(alphas), np.array(betas), np.stack(V, axis=1), False


def lanczos_upper_bound(apply_H, v0, nsteps: int = 10):
    """Returns (b, alphas, betas) with b = theta_max(T) + beta_last."""
    alphas, betas, _, stopped = lanczos(apply_H, v0, nsteps)
    if stopped:
        return _tridiag_max(alphas, betas), alphas, betas
    return _tridiag_max(alphas, betas[:-1]) + betas[-1], alphas, betas


def _tridiag_max(alphas, offdiag) -> float:
    d = np.asarray(alphas, dtype=np.float64)
    e = np.asarray(offdiag, dtype=np.float64)
    if d.size == 1:
        return float(d[0])
    return float(scipy.linalg.eigvalsh_tridiagonal(d, e)[-1])


def filter_bounds(apply_H, X, v0, nlanczos: int = 10):
    """(a, b, a0) from the Rayleigh quotients of X and a Lanczos run from v0."""
    rq = rayleigh_quotients(X, apply_H(X))
    b, _, _ = lanczos_upper_bound(apply_H, v0, nlanczos)
    return float(rq.max()), float(b), float(rq.min())


def cheb_sigmas(degree: int, a: float, b: float, a0: float) -> np.ndarray:
    """sigma_1 .. sigma_degree (index 0 holds sigma_1)."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    s1 = e / (a0 - c)
    s = [s1]
    for _ in range(1, degree):
        s.append(1.0 / (2.0 / s1 - s[-1]))
    return np.array(s)


def cheb_filter(apply_H, X, degree: int, a: float, b: float, a0: float):
    """Y_m = T_m((H - c)/e) X / T_m((a0 - c)/e) by the scaled recurrence."""
    if degree < 1 or not b > a or a0 > a:
        raise ValueError("need degree >= 1, b > a, a0 <= a")
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sig = cheb_sigmas(degree, a, b, a0)
    X = np.asarray(X, dtype=np.complex128)
    y_prev = X
    y = (sig[0] / e) * (apply_H(X) - c * X)
    for k in range(1, degree):
        s_k, s_k1 = sig[k - 1], sig[k]
        y_next = (2.0 * s_k1 / e) * (apply_H(y) - c * y) - (s_k * s_k1) * y_prev
        y_prev, y = y, y_next
    return y
