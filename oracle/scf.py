"""Outer self-consistent-field step (oracle).

Paper: each SCF iteration solves H Psi = Lambda S Psi per k-point, computes the
occupations f from the eigenvalues on the host, accumulates the electronic
density from f and Psi with FFTs on the GPU, and stops once converged
(Algorithm "Self-consistent field in DFT" and the paragraph after it).  The
new Hamiltonian that the next iteration solves is not described there (it is
the host code's part); the readings below define a minimal one.

Readings where the paper is silent:

* occupations: Fermi-Dirac, f_n = occ_max / (1 + exp((eps_n - mu)/kT)), mu by
  bisection so that sum_n f_n = N_el (occ_max = 2: spin-degenerate bands);
* density per volume n(r) = rho(r) n1 n2 n3 / Omega, rho the grid density of
  the FFT step (sum_r rho(r) = sum_n f_n);
* potential of the next iteration: V(r) = V_ion(r) + V_H(r) + v_x(r) with the
  Hartree potential V_H(G) = 4 pi n(G) / |G|^2 (G != 0, V_H(0) = 0),
  n(G) = n^-3 sum_r n(r) e^{-i G.r}, G = sum_d m_d b_d with the box window of
  the sphere (m_d in [-n_d/2, n_d/2 - 1] for even n_d), and the LDA
  (Slater) exchange v_x = -(3 n / pi)^(1/3) (n <= 0 gives 0);
* mixing V_in <- V_in + K (V_out - V_in): K = alpha (linear mixing) or, with a
  screening wave number q0 > 0, Kerker's preconditioner (Kerker, 1981)
  K(G) = alpha |G|^2 / (|G|^2 + q0^2) for G != 0 and K(0) = alpha, applied on the
  FFT box; converged when max_r |V_out - V_in| <= tol.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .hamiltonian import Hamiltonian, density
from .sphere import reciprocal_vectors


def occupations(eval, nelec: float, kT: float, occ_max: float = 2.0):
    """(f, mu) with sum f = nelec (bisection on mu, to machine precision)."""
    e = np.asarray(eval, dtype=np.float64)
    if not 0.0 <= nelec <= occ_max * e.size:
        raise ValueError("nelec out of range")

    def total(mu):
        return float((occ_max / (1.0 + np.exp(np.clip((e - mu) / kT, -700, 700)))).sum())

    lo, hi = e.min() - 50.0 * kT - 1.0, e.max() + 50.0 * kT + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if total(mid) < nelec:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    f = occ_max / (1.0 + np.exp(np.clip((e - mu) / kT, -700, 700)))
    return f, mu


def g_squared(lattice, ngrid) -> np.ndarray:
    """|G|^2 on the FFT box, shape (n3, n2, n1)."""
    B = reciprocal_vectors(np.asarray(lattice, dtype=np.float64))
    n1, n2, n3 = ngrid
    m = [np.where(np.arange(n) < (n + 1) // 2, np.arange(n), np.arange(n) - n) for n in ngrid]
    m3, m2, m1 = np.meshgrid(m[2], m[1], m[0], indexing="ij")
    G = m1[..., None] * B[0] + m2[..., None] * B[1] + m3[..., None] * B[2]
    return np.einsum("...i,...i->...", G, G)


def hartree(n_r, lattice, ngrid) -> np.ndarray:
    """V_H on the grid (i1 fastest) from the density per volume n(r)."""
    n1, n2, n3 = ngrid
    nG = scipy.fft.fftn(np.asarray(n_r, dtype=np.float64).reshape(n3, n2, n1)) / (n1 * n2 * n3)
    g2 = g_squared(lattice, ngrid)
    vG = np.zeros_like(nG)
    nz = g2 > 0
    vG[nz] = 4.0 * np.pi * nG[nz] / g2[nz]
    return np.real(scipy.fft.ifftn(vG, norm="forward")).reshape(-1)


def lda_exchange(n_r) -> np.ndarray:
    n = np.maximum(np.asarray(n_r, dtype=np.float64), 0.0)
    return -np.cbrt(3.0 * n / np.pi)


def scf_potential(rho, vion, lattice, ngrid) -> np.ndarray:
    """V_out = V_ion + V_H[n] + v_x[n] with n = rho n^3 / Omega."""
    omega = abs(np.linalg.det(np.asarray(lattice, dtype=np.float64)))
    n_r = np.asarray(rho) * (np.prod(ngrid) / omega)
    return np.asarray(vion) + hartree(n_r, lattice, ngrid) + lda_exchange(n_r)


def mix(vin, vout, alpha, q0, lattice, ngrid) -> np.ndarray:
    """V_in + K (V_out - V_in) with the linear (q0 = 0) or Kerker factor K(G)."""
    d = np.asarray(vout, dtype=np.float64) - np.asarray(vin, dtype=np.float64)
    if q0 <= 0.0:
        return np.asarray(vin) + alpha * d
    n1, n2, n3 = ngrid
    dG = scipy.fft.fftn(d.reshape(n3, n2, n1))
    g2 = g_squared(lattice, ngrid)
    k = np.where(g2 > 0, alpha * g2 / (g2 + q0 * q0), alpha)
    return np.asarray(vin) + np.real(scipy.fft.ifftn(k * dG)).reshape(-1)


def scf_iteration(H: Hamiltonian, Psi, vion, nelec, kT, alpha, solve, q0=0.0):
    """One SCF iteration at the potential H.vloc: (Psi, eval, rho, V_out, V_next, dv).

    `solve(H, Psi) -> (eval, Psi)` runs the eigensolver at fixed potential."""
    ev, Psi = solve(H, Psi)
    f, _ = occupations(ev, nelec, kT)
    rho = density(H, Psi, f)
    vout = scf_potential(rho, vion, H.lattice, H.ngrid)
    dv = float(np.abs(vout - H.vloc).max())
    vnext = mix(H.vloc, vout, alpha, q0, H.lattice, H.ngrid)
    return Psi, ev, rho, vout, vnext, dv
