"""Pins for the oracle's SCF step (CPU only).

* occupations: they sum to N_el; two levels symmetric about mu with one
  level's worth of electrons put mu at the midpoint; a small kT gives the
  step function (whole bands below the gap, empty above);
* Hartree: a density A cos(G0.r) gives 4 pi A / |G0|^2 cos(G0.r) (closed form,
  on a sheared cell so that G0 mixes reciprocal vectors), a constant density
  gives zero;
* LDA exchange: v_x(pi/3) = -1, v_x(8 pi/3) = -2, zero for n <= 0;
* normalisation: a grid density with sum_r rho = N is N / Omega per volume, and
  the potential of a modulated density is V_ion + the closed-form V_H + v_x;
* Kerker mixing: q0 = 0 is linear mixing; a plane-wave potential residual is
  scaled by alpha G0^2/(G0^2 + q0^2), a constant one by alpha;
* the loop's fixed point: iterated on a tiny cell until max |V_out - V_in| is
  below 1e-7, the eigenvalues equal those of the dense H at that potential and
  the potential reproduces itself.
"""
import numpy as np

import oracle as O
import workloads as W
from oracle.scf import (g_squared, hartree, lda_exchange, mix, occupations, scf_iteration,
                        scf_potential)


def test_occupations():
    e = np.array([-1.0, -0.5, 0.2, 0.3, 1.0])
    f, mu = occupations(e, 4.0, 0.05)
    assert abs(f.sum() - 4.0) < 1e-12 and np.all(np.diff(f) <= 0)
    f, mu = occupations(np.array([-0.3, 0.5]), 2.0, 0.1)
    assert abs(mu - 0.1) < 1e-12 and abs(f[0] + f[1] - 2.0) < 1e-12
    f, mu = occupations(e, 4.0, 1e-4)
    assert np.allclose(f, [2, 2, 0, 0, 0], atol=1e-12) and -0.5 < mu < 0.2


def test_hartree_closed_form():
    lat = np.array([[7.0, 0.0, 0.0], [1.5, 8.0, 0.0], [0.5, -1.0, 9.0]])
    ngrid = (12, 15, 16)
    B = O.reciprocal_vectors(lat)
    n1, n2, n3 = ngrid
    i3, i2, i1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    frac = np.stack([i1 / n1, i2 / n2, i3 / n3], axis=-1)
    r = frac @ lat
    m = np.array([1, -2, 1])
    G0 = m @ B
    A = 0.37
    n_r = A * np.cos(r @ G0)
    vh = hartree(n_r.reshape(-1), lat, ngrid)
    ref = 4.0 * np.pi * A / (G0 @ G0) * np.cos(r @ G0)
    assert np.abs(vh - ref.reshape(-1)).max() < 1e-13
    assert np.abs(hartree(np.full(n1 * n2 * n3, 0.2), lat, ngrid)).max() < 1e-14
    g2 = g_squared(lat, ngrid)
    assert g2[0, 0, 0] == 0.0 and abs(g2[0, 0, 1] - B[0] @ B[0]) < 1e-14


def test_lda_exchange():
    v = lda_exchange(np.array([np.pi / 3, 8 * np.pi / 3, 0.0, -1e-3]))
    assert np.allclose(v, [-1.0, -2.0, 0.0, 0.0], atol=1e-15, rtol=1e-15)


def test_potential_normalisation():
    lat = np.eye(3) * 6.0
    ngrid = (8, 8, 8)
    N = 5.0
    rho = np.full(512, N / 512)
    v = scf_potential(rho, np.zeros(512), lat, ngrid)
    n = N / 216.0
    assert np.allclose(v, -np.cbrt(3 * n / np.pi), atol=1e-14)
    # a modulated density: V_ion + 4 pi A/|G0|^2 cos + v_x of the total, term by term
    x = (np.arange(8) / 8.0 * 6.0)[None, None, :] * np.ones((8, 8, 1))
    G0 = 2 * np.pi / 6.0
    A = 0.2 * n
    dens = (n + A * np.cos(G0 * x)).reshape(-1)
    vion = np.linspace(-1.0, 0.5, 512)
    v = scf_potential(dens * 216.0 / 512, vion, lat, ngrid)
    ref = vion + 4 * np.pi * A / G0 ** 2 * np.cos(G0 * x).reshape(-1) - np.cbrt(3 * dens / np.pi)
    assert np.abs(v - ref).max() < 1e-13


def test_fixed_point_of_the_loop():
    s = W.make_system(151, a=6.0, ecut=4.0, n=12, natom=2, nband=8, kpt_red=(0.0, 0.0, 0.0))
    H = O.Hamiltonian.from_system(s)
    vion = H.vloc.copy()
    X = W.random_block(H.npw, 8, 151)

    def solve(Hm, Psi):
        lam, V = np.linalg.eigh(Hm.dense())
        return lam[:8], V[:, :8]

    for _ in range(200):
        X, ev, rho, vout, vnext, dv = scf_iteration(H, X, vion, 6.0, 0.02, 0.4, solve)
        if dv < 1e-7:
            break
        H.vloc = vnext
    assert dv < 1e-7
    assert np.abs(ev - np.linalg.eigvalsh(H.dense())[:8]).max() < 1e-12
    assert np.abs(scf_potential(rho, vion, H.lattice, H.ngrid) - H.vloc).max() < 1e-7


def test_kerker_mixing():
    lat = np.array([[6.0, 0.0, 0.0], [1.0, 7.0, 0.0], [0.0, 0.5, 8.0]])
    ngrid = (10, 12, 15)
    n1, n2, n3 = ngrid
    i3, i2, i1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    r = np.stack([i1 / n1, i2 / n2, i3 / n3], axis=-1) @ lat
    G0 = np.array([2, 1, -1]) @ O.reciprocal_vectors(lat)
    vin = np.linspace(-1, 1, n1 * n2 * n3)
    d = (0.3 + 0.7 * np.cos(r @ G0)).reshape(-1)
    alpha, q0 = 0.4, 1.3
    got = mix(vin, vin + d, alpha, q0, lat, ngrid)
    g2 = G0 @ G0
    ref = vin + alpha * 0.3 + alpha * g2 / (g2 + q0 ** 2) * 0.7 * np.cos(r @ G0).reshape(-1)
    assert np.abs(got - ref).max() < 1e-13
    assert np.abs(mix(vin, vin + d, alpha, 0.0, lat, ngrid) - (vin + alpha * d)).max() < 1e-15
