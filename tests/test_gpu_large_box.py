"""FFT boxes above 64 points per edge (up to 96, needs an MI355X).

Boxes above 64 take the runtime-size FFT passes with up to 24 values per
thread per Stockham stage and planes of up to 152 KB of LDS (FP64 96 x 97).
Against the FP64 oracle: H X to 1e-10 (FP64) / 2e-6 (mixed) per column, a
degree-3 filter to 1e-9 (FP64); a cubic 96^3 box and a non-cubic 72 x 80 x 90
one (all three plans, radix 2/3/4/5).
"""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import col_rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


@functools.lru_cache(maxsize=None)
def _system(name):
    if name == "cubic96":
        return W.make_system(301, a=12.0, ecut=6.0, n=96, natom=2, nband=9,
                             kpt_red=(0.1, 0.2, 0.3))
    s = W.make_system(302, a=12.0, ecut=6.0, n=72, natom=3, nband=7, kpt_red=(0.3, 0.0, 0.15))
    s.ngrid = (72, 80, 90)
    s.vloc = W.systems._gaussian_wells(s.tau, s.a, s.ngrid)
    return s


@functools.lru_cache(maxsize=None)
def _ham(name):
    return O.Hamiltonian.from_system(_system(name))


@pytest.mark.parametrize("name", ["cubic96", "noncubic72"])
def test_large_box_apply_H_and_filter(name):
    import torch
    s = _system(name)
    H = _ham(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    ref = H(X)
    with B.System(s) as g:
        got = to_host(g.apply_H(to_dev(X)))
        assert col_rel_err(got, ref) <= 1e-10
        v0 = W.random_vector(H.npw, s.tag)
        a, b, a0 = O.filter_bounds(H, X, v0)
        Y = to_host(g.cheb_filter(to_dev(X), 3, a, b, a0))
    assert col_rel_err(Y, O.cheb_filter(H, X, 3, a, b, a0)) <= 1e-9
    Xm = X.astype(np.complex64).astype(np.complex128)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        got = to_host(g.apply_H(to_dev(Xm).to(torch.complex64))).astype(np.complex128)
    assert col_rel_err(got, H(Xm)) <= 2e-6
