"""Block LOBPCG (oracle) — the paper's comparison solver.

Paper: LOBPCG splits the M bands into b blocks; each block is S-deflated against
the blocks before it, orthonormalised and rotated by Rayleigh-Ritz, then k line
minimisations follow, each forming the residual W = (H - Lambda S) Psi
(stopping when the block has converged), preconditioning it with a diagonal K,
deflating it, applying H and S to it, and running an S-orthonormalisation and
Rayleigh-Ritz on [Psi, W] (first step, 2m-sized) or [Psi, W, P] (3m-sized),
P being the conjugate directions; after the last block a global S-ortho and
Rayleigh-Ritz of all M bands (Algorithms "LOBPCG with b blocks and k line
minimizations" and "Parallel LOBPCG with b blocks and k line minimizations",
section "Main computational kernels").

Readings where the paper is silent:

* preconditioner: the Teter-Payne-Allan polynomial per band,
  K_G = p(x) / (p(x) + 16 x^4), p(x) = 27 + 18 x + 12 x^2 + 8 x^3,
  x = 0.5|k+G|^2 / E_kin(psi_n), E_kin(psi) = sum_G 0.5|k+G|^2 |c_G|^2 / sum_G |c_G|^2
  (published by Teter, Payne and Allan, 1989);
* S-deflation of a block X against the S-orthonormal earlier bands Q:
  X <- X - Q (Q^H S X);
* before the small Gram is formed each column of W and P is scaled to unit
  S-norm (the basis spans the same space; the Gram stays well conditioned);
* S-ortho + Rayleigh-Ritz of a basis Z: Z^H S Z = U^H U (Cholesky),
  U^-H (Z^H H Z) U^-1 = Y Lambda Y^H, coefficients C = U^-1 Y[:, :m] of the
  lowest m pairs (the same Ritz pairs as the generalised pencil); if the
  Cholesky factorisation fails on [Psi, W, P] the step drops P;
* conjugate directions P_new = W C_W + P C_P (the rows of C that multiply W
  and P), and Psi_new = Psi C_Psi + P_new;
* a block counts as converged when all its residual norms
  ||H psi - lambda S psi||_2 are <= tol;
* the block size is M/b (b divides M).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def tpa_precondition(kin, Psi, W):
    """K W with the Teter-Payne-Allan diagonal of each band (column)."""
    num = (kin[:, None] * np.abs(Psi) ** 2).sum(axis=0)
    den = (np.abs(Psi) ** 2).sum(axis=0)
    ek = num / den
    x = kin[:, None] / ek[None, :]
    p = 27.0 + 18.0 * x + 12.0 * x ** 2 + 8.0 * x ** 3
    return W * (p / (p + 16.0 * x ** 4))


def _ortho_rr(Z, HZ, SZ, m):
    """(lam[:m], C) from the S-ortho + Rayleigh-Ritz of the basis Z, or None if the
    Gram is not positive definite."""
    G = Z.conj().T @ SZ
    G = 0.5 * (G + G.conj().T)
    try:
        U = scipy.linalg.cholesky(G, lower=False)
    except np.linalg.LinAlgError:
        return None
    Hs = Z.conj().T @ HZ
    Hs = 0.5 * (Hs + Hs.conj().T)
    Ui = scipy.linalg.solve_triangular(U, np.eye(U.shape[0]), lower=False)
    R = Ui.conj().T @ Hs @ Ui
    lam, Y = scipy.linalg.eigh(0.5 * (R + R.conj().T))
    return lam[:m], Ui @ Y[:, :m]


def _snormalise(X, HX, SX):
    d = np.sqrt(np.real(np.einsum("ij,ij->j", X.conj(), SX)))
    return X / d, HX / d, SX / d


def lobpcg_pass(apply_H, apply_S, kin, Psi, nblocks: int, nline: int, tol: float):
    """One pass of the algorithm over all blocks; returns dict(eval, Psi, res, steps).

    steps[i] = line minimisations block i ran (it stops early once converged).
    """
    Psi = np.array(Psi, dtype=np.complex128)
    N, M = Psi.shape
    if M % nblocks:
        raise ValueError("nblocks must divide the number of bands")
    m = M // nblocks
    HPsi = np.zeros_like(Psi)
    SPsi = np.zeros_like(Psi)
    steps = []
    for i in range(nblocks):
        sl = slice(i * m, (i + 1) * m)
        X = Psi[:, sl]
        Q = Psi[:, : i * m]
        if i > 0:
            X = X - Q @ (Q.conj().T @ apply_S(X))
        HX, SX = apply_H(X), apply_S(X)
        lam, C = _ortho_rr(X, HX, SX, m)
        X, HX, SX = X @ C, HX @ C, SX @ C
        P = HP = SP = None
        done = 0
        for _ in range(nline):
            Wr = HX - SX * lam[None, :]
            if np.linalg.norm(Wr, axis=0).max() <= tol:
                break
            W = tpa_precondition(kin, X, Wr)
            if i > 0:
                W = W - Q @ (Q.conj().T @ apply_S(W))
            HW, SW = apply_H(W), apply_S(W)
            W, HW, SW = _snormalise(W, HW, SW)
            out = None
            if P is not None:
                Pn, HPn, SPn = _snormalise(P, HP, SP)
                out = _ortho_rr(np.hstack([X, W, Pn]), np.hstack([HX, HW, HPn]),
                                np.hstack([SX, SW, SPn]), m)
                if out is not None:
                    lam, C = out
                    Cw, Cp = C[m:2 * m], C[2 * m:]
                    P, HP, SP = W @ Cw + Pn @ Cp, HW @ Cw + HPn @ Cp, SW @ Cw + SPn @ Cp
            if out is None:
                out = _ortho_rr(np.hstack([X, W]), np.hstack([HX, HW]), np.hstack([SX, SW]), m)
                if out is None:
                    raise np.linalg.LinAlgError("S-Gram of [Psi, W] is not positive definite")
                lam, C = out
                Cw = C[m:]
                P, HP, SP = W @ Cw, HW @ Cw, SW @ Cw
            Cx = C[:m]
            X, HX, SX = X @ Cx + P, HX @ Cx + HP, SX @ Cx + SP
            done += 1
        Psi[:, sl], HPsi[:, sl], SPsi[:, sl] = X, HX, SX
        steps.append(done)
    if nblocks > 1:
        # global S-ortho + Rayleigh-Ritz of all M bands (H Psi, S Psi carried along)
        lam, C = _ortho_rr(Psi, HPsi, SPsi, M)
        Psi, HPsi, SPsi = Psi @ C, HPsi @ C, SPsi @ C
    res = np.linalg.norm(HPsi - SPsi * lam[None, :], axis=0)
    return dict(eval=lam, Psi=Psi, res=res, steps=steps)
