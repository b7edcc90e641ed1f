"""Synthetic plane-wave systems shaped like the paper's workloads.

The paper benchmarks ABINIT on a Ti solid-liquid interface and on a Ga2O3
crystal with PAW datasets (section "Benchmark test cases"); neither structure,
dataset nor code is available, so these seeded systems stand in for them.  A
system is a cubic cell with Gaussian-well local potentials and four Gaussian
s+p projectors per atom:

* atoms: uniform in [0, a)^3, sequential rejection with minimum-image distance
  >= 3 bohr;
* V_loc(r) = sum_R sum_{L in a{-2..2}^3} -4 exp(-|r - R - L|^2 / (2 * 0.8^2)),
  sampled at r = (i/n) a on the FFT grid, flat with i1 fastest;
* D per atom: 4x4 Hermitian, real diagonal U[-1,1], upper entries with real and
  imaginary parts U[-1,1];
* blocks: complex128 with independent N(0,1) real and imaginary parts, stored
  column-major (plane waves fastest).

Every random draw comes from ``numpy.random.SeedSequence([2604, 11139, tag])``
split into independent child streams, so both sides of a parity test read the
very same arrays.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional, Sequence

import numpy as np

# Stream indices of SeedSequence(...).spawn(N_STREAMS).
ATOMS, DMAT, XBLOCK, WBLOCK, V0, FD, EXTRA, QMAT = range(8)
N_STREAMS = 8

WELL_DEPTH = -4.0
WELL_SIGMA = 0.8
MIN_SEPARATION = 3.0
PROJ_RC = 1.0
Q_SHIFT = 1.5
PAW_Q_SCALE = 10.0  # q_scale of the PAW-like variants: S spectrum about [0.8, 1.8]

# The workloads: sizes follow the paper's regime of a few percent of bands per
# plane wave; ids 1-3 are single systems of growing size.
CONFIGS: Dict[int, dict] = {
    1: dict(a=10.0, ecut=10.0, n=32, natom=2, nband=32, degree=8, cycles=1),
    2: dict(a=20.0, ecut=15.0, n=36, natom=64, nband=512, degree=10, cycles=4),
    3: dict(a=30.0, ecut=20.0, n=64, natom=216, nband=2048, degree=12, cycles=4),
}


@dataclasses.dataclass
class System:
    """Inputs that define one Hamiltonian (cubic cell)."""

    a: float
    ecut: float
    ngrid: tuple
    kpt_red: np.ndarray  # (3,) reduced coordinates
    tau: np.ndarray  # (natom, 3) cartesian bohr
    rc: float
    vloc: np.ndarray  # (n1*n2*n3,) float64, i1 fastest
    dij: np.ndarray  # (natom, 4, 4) complex128, Hermitian
    nband: int
    degree: int
    cycles: int
    tag: int
    qij: Optional[np.ndarray] = None  # (natom, 4, 4) complex128, Hermitian; None: S = I

    @property
    def lattice(self) -> np.ndarray:
        """Rows are the lattice vectors a1, a2, a3 (bohr)."""
        return np.eye(3) * self.a

    @property
    def natom(self) -> int:
        return int(self.tau.shape[0])

    @property
    def nproj(self) -> int:
        return 4 * self.natom


def streams(tag: int) -> Sequence[np.random.Generator]:
    """Independent generators for one workload tag."""
    ss = np.random.SeedSequence([2604, 11139, int(tag)])
    return [np.random.default_rng(s) for s in ss.spawn(N_STREAMS)]


def _place_atoms(rng: np.random.Generator, natom: int, a: float) -> np.ndarray:
    pos = np.zeros((natom, 3))
    count = 0
    tries = 0
    while count < natom:
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("atom placement did not converge")
        cand = rng.uniform(0.0, a, size=3)
        if count:
            d = pos[:count] - cand
            d -= a * np.round(d / a)
            if np.min(np.einsum("ij,ij->i", d, d)) < MIN_SEPARATION ** 2:
                continue
        pos[count] = cand
        count += 1
    return pos


def _gaussian_wells(tau: np.ndarray, a: float, ngrid) -> np.ndarray:
    """Periodic Gaussian wells on the grid (separable per axis for a cubic cell)."""
    n1, n2, n3 = ngrid
    v = np.zeros((n3, n2, n1))
    images = np.arange(-2, 3) * a
    s2 = 2.0 * WELL_SIGMA ** 2
    axes = [np.arange(n) * (a / n) for n in (n1, n2, n3)]
    for R in tau:
        g = []
        for d in range(3):
            diff = axes[d][:, None] - R[d] - images[None, :]
            g.append(np.exp(-(diff ** 2) / s2).sum(axis=1))
        v += WELL_DEPTH * (g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :])
    return v.reshape(-1)


def _hermitian_d(rng: np.random.Generator, natom: int) -> np.ndarray:
    d = np.zeros((natom, 4, 4), dtype=np.complex128)
    for r in range(natom):
        diag = rng.uniform(-1.0, 1.0, size=4)
        up_re = rng.uniform(-1.0, 1.0, size=6)
        up_im = rng.uniform(-1.0, 1.0, size=6)
        k = 0
        for i in range(4):
            d[r, i, i] = diag[i]
            for j in range(i + 1, 4):
                d[r, i, j] = up_re[k] + 1j * up_im[k]
                d[r, j, i] = np.conj(d[r, i, j])
                k += 1
    return d


def make_system(
    tag: int = 1,
    *,
    a: Optional[float] = None,
    ecut: Optional[float] = None,
    n: Optional[int] = None,
    natom: Optional[int] = None,
    nband: Optional[int] = None,
    degree: Optional[int] = None,
    cycles: Optional[int] = None,
    kpt_red=(0.0, 0.0, 0.0),
    vloc_scale: float = 1.0,
    d_scale: float = 1.0,
    q_scale: float = 0.0,
) -> System:
    """Build a seeded system.  ``tag`` selects the workload and the seed.

    Keyword overrides make small variants (test systems) from the same recipe;
    ``vloc_scale`` / ``d_scale`` scale the potential and D (0 gives the free
    electron, 100 makes the weak nonlocal term visible); ``q_scale`` > 0 adds
    the overlap matrices Q_R = q_scale (H_R + Q_SHIFT I) of a PAW-like system
    (H_R drawn like D), otherwise S = I.
    """
    base = dict(CONFIGS.get(tag, CONFIGS[1]))
    for k, v in dict(a=a, ecut=ecut, n=n, natom=natom, nband=nband, degree=degree,
                     cycles=cycles).items():
        if v is not None:
            base[k] = v
    rngs = streams(tag)
    A = float(base["a"])
    ngrid = (int(base["n"]),) * 3
    tau = _place_atoms(rngs[ATOMS], int(base["natom"]), A)
    vloc = _gaussian_wells(tau, A, ngrid) * vloc_scale
    dij = _hermitian_d(rngs[DMAT], int(base["natom"])) * d_scale
    return System(
        a=A,
        ecut=float(base["ecut"]),
        ngrid=ngrid,
        kpt_red=np.asarray(kpt_red, dtype=np.float64),
        tau=tau,
        rc=PROJ_RC,
        vloc=vloc,
        dij=dij,
        nband=int(base["nband"]),
        degree=int(base["degree"]),
        cycles=int(base["cycles"]),
        tag=int(tag),
        qij=(_hermitian_d(rngs[QMAT], int(base["natom"])) + Q_SHIFT * np.eye(4)) * q_scale
        if q_scale > 0 else None,
    )


# The batched workload: independent small cells with k-point offsets (uneven
# plane-wave counts), as many k-points and cells handled in one launch.
BATCH = dict(tag=4, nsys=16, a=(8, 16), ecut=12.0, natom=(1, 8), nband=(32, 64, 128, 256),
             degree=8)
BATCH_TAG0 = 4000  # system i of the batch draws from tag BATCH_TAG0 + i


def smooth_235(m: int) -> int:
    """Smallest integer >= m whose only prime factors are 2, 3 and 5."""
    n = max(int(m), 1)
    while True:
        r = n
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return n
        n += 1


def make_batch(nsys: Optional[int] = None) -> list:
    """The batched workload: `nsys` (16) cubic cells, a ~ U{8..16} bohr,
    E_cut 12 Ha, k ~ U[0, 0.5)^3 (reduced), grid n = smallest {2,3,5}-smooth
    >= 3a, 1-8 atoms, nband in {32, 64, 128, 256}, degree 8."""
    nsys = BATCH["nsys"] if nsys is None else int(nsys)
    rng = streams(BATCH["tag"])[EXTRA]
    out = []
    for i in range(nsys):
        a = int(rng.integers(BATCH["a"][0], BATCH["a"][1] + 1))
        k = rng.uniform(0.0, 0.5, size=3)
        natom = int(rng.integers(BATCH["natom"][0], BATCH["natom"][1] + 1))
        nband = int(rng.choice(BATCH["nband"]))
        out.append(make_system(BATCH_TAG0 + i, a=float(a), ecut=BATCH["ecut"],
                               n=smooth_235(3 * a), natom=natom, nband=nband,
                               degree=BATCH["degree"], cycles=1, kpt_red=tuple(k)))
    return out


def random_block(npw: int, nband: int, tag: int, stream: int = XBLOCK) -> np.ndarray:
    """complex128 (npw, nband), column-major, N(0,1) real and imaginary parts."""
    rng = streams(tag)[stream]
    re = rng.standard_normal((nband, npw))
    im = rng.standard_normal((nband, npw))
    return np.asfortranarray((re + 1j * im).T)


def random_vector(npw: int, tag: int, stream: int = V0) -> np.ndarray:
    """complex128 (npw,) start vector with N(0,1) parts."""
    rng = streams(tag)[stream]
    return rng.standard_normal(npw) + 1j * rng.standard_normal(npw)
