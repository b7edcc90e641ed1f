"""Pins for the oracle's G-sphere and index maps (CPU only).

The sphere is pinned by an integer formulation at Gamma (sum m^2 < 2 E_cut a^2 /
(2 pi)^2), by the free-electron shell multiplicities r3(n) (golden fixture),
by the inversion symmetry at Gamma, by a brute-force loop on a tiny shifted
k-point, and by the continuum plane-wave count.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _r3_table():
    rows = []
    with open(os.path.join(GOLDEN, "r3_sums_of_three_squares.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, r = line.split()
            rows.append((int(n), int(r)))
    return dict(rows)


@pytest.mark.parametrize("tag,expect", [(1, 1503), (2, 22119), (3, 115313)])
def test_gamma_sphere_matches_integer_count(tag, expect):
    s = W.make_system(tag)
    sp = O.gsphere(s.lattice, s.kpt_red, s.ecut, s.ngrid)
    assert sp.npw == expect
    # integer formulation: sum m^2 < 2 Ecut a^2 / (2 pi)^2 ; no lattice point
    # lies within 1e-9 of the boundary, so float rounding cannot flip membership
    bound = 2.0 * s.ecut * s.a ** 2 / (2.0 * math.pi) ** 2
    r = int(math.ceil(math.sqrt(bound))) + 1
    ax = np.arange(-r, r + 1)
    m3, m2, m1 = np.meshgrid(ax, ax, ax, indexing="ij")
    n2 = (m1 ** 2 + m2 ** 2 + m3 ** 2).ravel()
    assert np.count_nonzero(n2 < bound) == expect
    assert np.min(np.abs(n2 - bound)) > 1e-9 * bound
    got = set(map(tuple, sp.miller.tolist()))
    want = set(zip(m1.ravel()[n2 < bound], m2.ravel()[n2 < bound], m3.ravel()[n2 < bound]))
    assert got == want


def test_free_electron_shells_follow_r3():
    r3 = _r3_table()
    s = W.make_system(1)
    sp = O.gsphere(s.lattice, s.kpt_red, s.ecut, s.ngrid)
    unit = 0.5 * (2.0 * math.pi / s.a) ** 2
    shell = np.rint(sp.kinetic / unit).astype(int)
    assert np.allclose(sp.kinetic, shell * unit, rtol=1e-13, atol=0)
    for n, count in r3.items():
        assert np.count_nonzero(shell == n) == count, n


def test_gamma_inversion_symmetry_and_maps():
    s = W.make_system(2)
    sp = O.gsphere(s.lattice, s.kpt_red, s.ecut, s.ngrid)
    got = set(map(tuple, sp.miller.tolist()))
    assert all((-a, -b, -c) in got for a, b, c in got)
    # box index: ascending, unique, recomputed from miller with wrap
    n1, n2, n3 = s.ngrid
    m = sp.miller.astype(np.int64)
    box = (m[:, 0] % n1) + n1 * ((m[:, 1] % n2) + n2 * (m[:, 2] % n3))
    assert np.array_equal(box, sp.box_index)
    assert np.all(np.diff(sp.box_index) > 0)


def test_shifted_kpoint_brute_force():
    """Pure-Python triple loop over the box window on a tiny cell."""
    a, ecut, n = 5.0, 3.0, 10
    k = (0.25, -0.1, 0.45)
    sp = O.gsphere(np.eye(3) * a, k, ecut, (n, n, n))
    lo, hi = -(n // 2), n // 2 - 1
    want = []
    for m3 in range(lo, hi + 1):
        for m2 in range(lo, hi + 1):
            for m1 in range(lo, hi + 1):
                q = [(m1 + k[0]) * 2 * math.pi / a, (m2 + k[1]) * 2 * math.pi / a,
                     (m3 + k[2]) * 2 * math.pi / a]
                if 0.5 * sum(x * x for x in q) < ecut:
                    want.append(((m1 % n) + n * ((m2 % n) + n * (m3 % n)), (m1, m2, m3)))
    want.sort()
    assert [w[1] for w in want] == list(map(tuple, sp.miller.tolist()))
    for kin, mm in zip(sp.kinetic, sp.miller):
        q = (mm + np.array(k)) * 2 * math.pi / a
        assert abs(kin - 0.5 * np.dot(q, q)) < 1e-13


def test_count_close_to_continuum():
    s = W.make_system(3)
    sp = O.gsphere(s.lattice, s.kpt_red, s.ecut, s.ngrid)
    vol = s.a ** 3 * (2.0 * s.ecut) ** 1.5 / (6.0 * math.pi ** 2)
    assert abs(sp.npw - vol) / vol < 0.01


def test_grid_too_small_rejected():
    with pytest.raises(ValueError):
        O.gsphere(np.eye(3) * 10.0, (0, 0, 0), 10.0, (12, 12, 12))
