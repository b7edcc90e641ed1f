"""Host-side checks of the C ABI (no GPU): symbol exports and the basis maps.

The library's basis maps must equal the oracle's bit for bit (integers), and its
kinetic table must agree to rounding.
"""
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:abi_status|const char \*)\s*(abi_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = declared_symbols()
    assert "abi_cheb_filter" in names and "abi_rayleigh_ritz" in names
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(B.EXPORTS) == names
    # every entry point has its argument types declared to ctypes (a missing
    # declaration passes Python floats as ints or fails at the call)
    for n in sorted(names):
        assert getattr(L, n).argtypes is not None, n


@pytest.mark.parametrize("tag,kw", [
    (1, {}), (2, {}), (3, {}),
    (201, dict(a=9.0, ecut=12.0, n=30, natom=1, kpt_red=(0.31, 0.05, 0.44))),
    (202, dict(a=11.0, ecut=12.0, n=27, natom=1, kpt_red=(0.12, 0.49, 0.2))),
    (203, dict(a=8.0, ecut=12.0, n=25, natom=1, kpt_red=(0.0, 0.25, 0.0))),
])
def test_gsphere_bit_exact(tag, kw):
    s = W.make_system(tag, **kw)
    sp = O.gsphere(s.lattice, s.kpt_red, s.ecut, s.ngrid)
    miller, box, kin = B.gsphere_host(s)
    assert np.array_equal(miller, sp.miller)
    assert np.array_equal(box.astype(np.int64), sp.box_index)
    assert np.abs(kin - sp.kinetic).max() <= 1e-14 * max(1.0, sp.kinetic.max())


def test_grid_errors():
    s = W.make_system(1)
    s.ngrid = (12, 12, 12)  # sphere reaches |m| = 7 > 5
    with pytest.raises(B.ChebfiError) as e:
        B.gsphere_host(s)
    assert e.value.code == B.ABI_ERR_GRID
    s.ngrid = (32, 32, 28 + 3)  # 31 is prime
    with pytest.raises(B.ChebfiError) as e:
        B.gsphere_host(s)
    assert e.value.code == B.ABI_ERR_GRID
    s.ngrid = (32, 32, 100)  # larger than the LDS passes take (edges up to 96)
    with pytest.raises(B.ChebfiError) as e:
        B.gsphere_host(s)
    assert e.value.code == B.ABI_ERR_GRID


def test_occupations_host_call():
    """Fermi-Dirac occupations are a host computation: library vs oracle."""
    import oracle as O
    from paper_2604_11139_amd import binding as B
    rng = np.random.default_rng(8)
    e = np.sort(rng.uniform(-1.0, 1.0, 37))
    for nelec, kT in ((10.0, 0.01), (7.3, 0.2), (0.0, 0.05), (74.0, 0.05)):
        f, mu = B.occupations(e, nelec, kT)
        fo, muo = O.occupations(e, nelec, kT)
        assert abs(f.sum() - nelec) <= 1e-10
        assert np.abs(f - fo).max() <= 1e-10
    with pytest.raises(B.ChebfiError):
        B.occupations(e, 75.0, 0.01)
