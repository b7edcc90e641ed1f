"""G-sphere of plane waves and its FFT-box index map (oracle).

Paper: the cut-off energy fixes the FFT grid, and plane-wave data are moved
into the FFT box layout before the batched transforms (section "Low-level
operations"); the basis is the set of plane waves of a k-point (section
"Problem setup").  The paper does not spell the maps out; the reading here:

* G_m = m1 b1 + m2 b2 + m3 b3 with b = 2 pi (A^-1)^T, A the lattice rows;
* plane wave m belongs to the basis iff 0.5 |k + G_m|^2 < E_cut (strict), the
  cartesian components of q = k + G evaluated as
  ``(m1+k1)*b1c + (m2+k2)*b2c + (m3+k3)*b3c`` and the energy as
  ``0.5*(qx*qx + qy*qy + qz*qz)`` in float64;
* box coordinate i_d = m_d mod n_d, box index i1 + n1*(i2 + n2*i3);
* the basis is ordered by ascending box index;
* every m_d must lie in the window [-n/2, n/2-1] (even n) or
  [-(n-1)/2, (n-1)/2] (odd n), otherwise the grid is rejected.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def reciprocal_vectors(lattice: np.ndarray) -> np.ndarray:
    """Rows b_j with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def box_window(n: int):
    if n % 2 == 0:
        return -(n // 2), n // 2 - 1
    return -((n - 1) // 2), (n - 1) // 2


@dataclasses.dataclass
class GSphere:
    miller: np.ndarray  # (npw, 3) int32
    box_index: np.ndarray  # (npw,) int64
    kinetic: np.ndarray  # (npw,) 0.5 |k+G|^2
    qcart: np.ndarray  # (npw, 3) k+G, cartesian
    gcart: np.ndarray  # (npw, 3) G, cartesian
    ngrid: tuple

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])


def gsphere(lattice, kpt_red, ecut: float, ngrid) -> GSphere:
    B = reciprocal_vectors(lattice)
    k = np.asarray(kpt_red, dtype=np.float64)
    # A generous search range: |m_d| <= |a_d| * qmax / (2 pi) + |k_d| + 2.
    qmax = np.sqrt(2.0 * ecut)
    alen = np.linalg.norm(np.asarray(lattice, dtype=np.float64), axis=1)
    reach = [int(np.ceil(alen[d] * qmax / (2.0 * np.pi) + abs(k[d]))) + 2 for d in range(3)]
    r1 = np.arange(-reach[0], reach[0] + 1)
    r2 = np.arange(-reach[1], reach[1] + 1)
    r3 = np.arange(-reach[2], reach[2] + 1)
    m3, m2, m1 = np.meshgrid(r3, r2, r1, indexing="ij")
    m1 = m1.ravel(); m2 = m2.ravel(); m3 = m3.ravel()
    f1 = m1 + k[0]; f2 = m2 + k[1]; f3 = m3 + k[2]
    qx = f1 * B[0, 0] + f2 * B[1, 0] + f3 * B[2, 0]
    qy = f1 * B[0, 1] + f2 * B[1, 1] + f3 * B[2, 1]
    qz = f1 * B[0, 2] + f2 * B[1, 2] + f3 * B[2, 2]
    e = 0.5 * (qx * qx + qy * qy + qz * qz)
    inside = e < ecut
    m = np.stack([m1[inside], m2[inside], m3[inside]], axis=1)
    n1, n2, n3 = (int(x) for x in ngrid)
    for d, n in enumerate((n1, n2, n3)):
        lo, hi = box_window(n)
        if m.shape[0] and (m[:, d].min() < lo or m[:, d].max() > hi):
            raise ValueError("G-sphere does not fit the FFT box")
    i1 = np.mod(m[:, 0], n1); i2 = np.mod(m[:, 1], n2); i3 = np.mod(m[:, 2], n3)
    box = i1.astype(np.int64) + n1 * (i2.astype(np.int64) + n2 * i3.astype(np.int64))
    order = np.argsort(box, kind="stable")
    m = m[order]
    q = np.stack([qx[inside][order], qy[inside][order], qz[inside][order]], axis=1)
    g = m.astype(np.float64) @ B
    return GSphere(
        miller=m.astype(np.int32),
        box_index=box[order],
        kinetic=e[inside][order],
        qcart=q,
        gcart=g,
        ngrid=(n1, n2, n3),
    )
