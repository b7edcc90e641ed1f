"""Plane-wave Hamiltonian H = K + V_loc + V_nl (oracle, S = I).

Paper: H and S are N x N Hermitian in the plane-wave basis (section "Problem
setup"); H is applied matrix-free, the local potential through batched FFTs
(section "Batch processing", Algorithm "Batched bands kernel execution") and
the nonlocal part V_nl = sum_{R,i,j} |p_i^R> D_ij^R <p_j^R| through products
with the projector matrix P = <g|p_i^R> (section "Low-level operations").
The kinetic part is the diagonal 0.5 |k+G|^2 (section "Single-step benchmarks:
GPU kernel rooflines" names its multiply-add as the memory-bound piece).

Readings where the paper is silent:

* FFT convention: psi(r_i) = sum_G c_G exp(+2 pi i m.i/n) unnormalised,
  c'_G = n^-3 sum_r exp(-2 pi i m.i/n) (V psi)(r); only the composite operator
  matters.  The grid defines the operator: index differences wrap modulo n
  (aliasing is part of H on grids smaller than twice the sphere).
* Projectors, four per atom (s, px, py, pz), q = k + G, g = exp(-|q|^2 rc^2/2):
  p_s = g e^{-i G.R} / sqrt(Omega), p_c = rc q_c g e^{-i G.R} / sqrt(Omega);
  column index 4 R + i.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from .sphere import GSphere, gsphere

_WORKERS = max(1, len(os.sched_getaffinity(0)))
_CHUNK = 32  # bands per FFT batch (bounds the box memory)


class Hamiltonian:
    """Dense-definition and matrix-free forms of the same operator."""

    def __init__(self, lattice, kpt_red, ecut, ngrid, vloc, tau, dij, rc=1.0):
        self.lattice = np.asarray(lattice, dtype=np.float64)
        self.sphere: GSphere = gsphere(self.lattice, kpt_red, ecut, ngrid)
        self.ngrid = tuple(int(x) for x in ngrid)
        self.vloc = np.asarray(vloc, dtype=np.float64).reshape(-1)
        self.tau = np.asarray(tau, dtype=np.float64).reshape(-1, 3)
        self.dij = np.asarray(dij, dtype=np.complex128).reshape(-1, 4, 4)
        self.rc = float(rc)
        self.omega = abs(np.linalg.det(self.lattice))
        self.P = self._projectors()

    @classmethod
    def from_system(cls, sys) -> "Hamiltonian":
        return cls(sys.lattice, sys.kpt_red, sys.ecut, sys.ngrid, sys.vloc, sys.tau,
                   sys.dij, sys.rc)

    @property
    def npw(self) -> int:
        return self.sphere.npw

    @property
    def nproj(self) -> int:
        return 4 * self.tau.shape[0]

    # -- tables -----------------------------------------------------------
    def _projectors(self) -> np.ndarray:
        q = self.sphere.qcart
        G = self.sphere.gcart
        g = np.exp(-0.5 * (self.rc ** 2) * np.einsum("ij,ij->i", q, q))
        P = np.zeros((self.npw, self.nproj), dtype=np.complex128)
        for r, R in enumerate(self.tau):
            phase = np.exp(-1j * (G @ R)) / np.sqrt(self.omega)
            P[:, 4 * r + 0] = g * phase
            for c in range(3):
                P[:, 4 * r + 1 + c] = self.rc * q[:, c] * g * phase
        return P

    def d_blockdiag(self) -> np.ndarray:
        n = self.nproj
        D = np.zeros((n, n), dtype=np.complex128)
        for r in range(self.tau.shape[0]):
            D[4 * r:4 * r + 4, 4 * r:4 * r + 4] = self.dij[r]
        return D

    # -- matrix-free parts -----------------------------------------------
    def kinetic_apply(self, X):
        X = np.asarray(X)
        return self.sphere.kinetic.reshape(-1, *([1] * (X.ndim - 1))) * X

    def to_box(self, X):
        """Scatter sphere coefficients into zeroed boxes, shape (n3, n2, n1, nb)."""
        X2 = np.asarray(X).reshape(self.npw, -1)
        n1, n2, n3 = self.ngrid
        box = np.zeros((n1 * n2 * n3, X2.shape[1]), dtype=np.complex128)
        box[self.sphere.box_index] = X2
        return box.reshape(n3, n2, n1, X2.shape[1])

    def local_apply(self, X):
        """V_loc X = gather(FFT_fwd(V * FFT_inv(scatter X))) / n^3."""
        X = np.asarray(X)
        X2 = X.reshape(self.npw, -1)
        n1, n2, n3 = self.ngrid
        ntot = n1 * n2 * n3
        out = np.empty(X2.shape, dtype=np.complex128)
        v = self.vloc.reshape(n3, n2, n1, 1)
        for c0 in range(0, X2.shape[1], _CHUNK):
            c1 = min(X2.shape[1], c0 + _CHUNK)
            box = self.to_box(X2[:, c0:c1])
            # unnormalised inverse transform (exponent +), then forward / n^3
            real = scipy.fft.ifftn(box, axes=(0, 1, 2), norm="forward", workers=_WORKERS)
            real *= v
            back = scipy.fft.fftn(real, axes=(0, 1, 2), norm="forward", workers=_WORKERS)
            out[:, c0:c1] = back.reshape(ntot, c1 - c0)[self.sphere.box_index]
        return out.reshape(X.shape)

    def nonlocal_apply(self, X):
        """P (D (P^H X)) with D block-diagonal per atom."""
        X = np.asarray(X)
        X2 = X.reshape(self.npw, -1)
        C = self.P.conj().T @ X2
        C2 = np.einsum("rij,rjb->rib", self.dij, C.reshape(-1, 4, X2.shape[1]))
        return (self.P @ C2.reshape(self.nproj, -1)).reshape(X.shape)

    def apply(self, X):
        return self.kinetic_apply(X) + self.local_apply(X) + self.nonlocal_apply(X)

    __call__ = apply

    # -- dense definition --------------------------------------------------
    def vhat(self) -> np.ndarray:
        """Fourier coefficients V^[g] = n^-3 sum_r V(r) e^{-2 pi i g.i/n}, (n3,n2,n1)."""
        n1, n2, n3 = self.ngrid
        return np.fft.fftn(self.vloc.reshape(n3, n2, n1)) / (n1 * n2 * n3)

    def dense_local(self) -> np.ndarray:
        n1, n2, n3 = self.ngrid
        m = self.sphere.miller.astype(np.int64)
        d1 = np.mod(m[:, None, 0] - m[None, :, 0], n1)
        d2 = np.mod(m[:, None, 1] - m[None, :, 1], n2)
        d3 = np.mod(m[:, None, 2] - m[None, :, 2], n3)
        return self.vhat()[d3, d2, d1]

    def dense(self) -> np.ndarray:
        """Explicit N x N matrix: diag(kinetic) + V_L + P D P^H."""
        H = self.dense_local().astype(np.complex128)
        H[np.diag_indices(self.npw)] += self.sphere.kinetic
        H += self.P @ self.d_blockdiag() @ self.P.conj().T
        return H


def density(H: Hamiltonian, Psi, weights=None) -> np.ndarray:
    """rho(r) = sum_n w_n |psi~_n(r)|^2 / n^3 on the grid (i1 fastest).

    psi~ is the unnormalised inverse FFT of the scattered sphere vector, so a
    unit-norm band contributes sum_r |psi~(r)|^2 / n^3 = 1 (Parseval).  This is
    the density the SCF loop builds from the wave functions through FFTs
    (paper: Algorithm "SCF", density step); with w_n = 1 for the lowest p
    bands it is the Hellmann-Feynman derivative of their eigenvalue sum with
    respect to V_loc(r).
    """
    Psi = np.asarray(Psi, dtype=np.complex128).reshape(H.npw, -1)
    w = np.ones(Psi.shape[1]) if weights is None else np.asarray(weights, dtype=np.float64)
    n1, n2, n3 = H.ngrid
    ntot = n1 * n2 * n3
    rho = np.zeros(ntot)
    for c0 in range(0, Psi.shape[1], _CHUNK):
        c1 = min(Psi.shape[1], c0 + _CHUNK)
        box = H.to_box(Psi[:, c0:c1])
        real = scipy.fft.ifftn(box, axes=(0, 1, 2), norm="forward", workers=_WORKERS)
        rho += (np.abs(real) ** 2 * w[c0:c1]).sum(axis=3).reshape(-1) / ntot
    return rho
