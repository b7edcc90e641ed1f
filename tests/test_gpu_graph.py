"""The captured filter (ABI_TUNE_FILTER_GRAPH = 1, needs an MI355X).

abi_cheb_filter records its launches into a HIP graph on the first call with
given blocks and replays it afterwards, with each step's coefficients read
from a device table uploaded before the replay.  Every replay must equal the
eager filter bit for bit: replays with new bounds, with the program's own
eager work and synchronisations between them, alternating block pairs, the
H X form, and replays after a work buffer was reallocated by another call.
"""
import numpy as np
import pytest

import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import hamiltonian, system, to_dev

pytestmark = pytest.mark.gpu

BOUNDS = [(0.5, 9.0, -1.5), (0.8, 11.0, -1.2), (0.3, 7.5, -2.0)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


def _block(name, precision, seed):
    import torch
    s = system(name)
    H = hamiltonian(name)
    X = to_dev(W.random_block(H.npw, s.nband, seed))
    if precision == "mixed":
        X = X.to(torch.complex64)
    return s, X


def _eager(s, prec, X, degree, bounds, hx=None):
    with B.System(s, precision=prec) as g:
        g.set_tuning(B.TUNE_FILTER_GRAPH, 0)
        return g.cheb_filter(X, degree, *bounds, hx=hx).clone()


@pytest.mark.parametrize("name,precision,degree", [("n27", "fp64", 5), ("n27", "mixed", 6),
                                                   ("c1", "mixed", 8), ("odd15", "fp64", 3)])
def test_graph_replays_equal_eager(name, precision, degree):
    import torch
    prec = B.ABI_PREC_MIXED if precision == "mixed" else B.ABI_PREC_FP64
    s, X = _block(name, precision, 61)
    ref = [_eager(s, prec, X, degree, bd) for bd in BOUNDS]
    with B.System(s, precision=prec) as g:
        assert g.get_tuning(B.TUNE_FILTER_GRAPH) == 0
        g.set_tuning(B.TUNE_FILTER_GRAPH, 1)
        Y = torch.empty_like(X)
        other = torch.empty_like(X)
        for rep in range(3):
            for k, bd in enumerate(BOUNDS):
                g.cheb_filter(X, degree, *bd, out=Y)
                torch.cuda.synchronize()
                assert torch.equal(Y, ref[k]), (rep, k)
                # the program's own eager work between replays
                g.apply_H(X, out=other)
                other.mul_(0.5)
                torch.cuda.synchronize()


def test_graph_alternating_blocks_and_hx():
    """X -> Y, Y -> X as a loop does (two graphs), and the H X form."""
    import torch
    s, X0 = _block("n27", "mixed", 62)
    prec = B.ABI_PREC_MIXED
    bd = BOUNDS[0]
    # eager references of the alternating chain
    with B.System(s, precision=prec) as g:
        g.set_tuning(B.TUNE_FILTER_GRAPH, 0)
        a = X0.clone()
        chain = []
        for _ in range(4):
            b = g.cheb_filter(a, 4, *bd)
            b = b / b.abs().amax()
            chain.append(b.clone())
            a = b
        HX = g.apply_H(X0)
        ref_hx = g.cheb_filter(X0, 4, *bd, hx=HX).clone()
    with B.System(s, precision=prec) as g:
        g.set_tuning(B.TUNE_FILTER_GRAPH, 1)
        A = X0.clone()
        Bb = torch.empty_like(A)
        for i in range(4):
            src, dst = (A, Bb) if i % 2 == 0 else (Bb, A)
            g.cheb_filter(src, 4, *bd, out=dst)
            dst.div_(dst.abs().amax())
            torch.cuda.synchronize()
            assert torch.equal(dst, chain[i]), i
        HXd = g.apply_H(X0)
        Y = torch.empty_like(X0)
        for _ in range(3):
            g.cheb_filter(X0, 4, *bd, out=Y, hx=HXd)
            torch.cuda.synchronize()
            assert torch.equal(Y, ref_hx)


def test_graph_after_buffer_reallocation():
    """A larger call on the same handle reallocates work buffers: the next
    filter must not replay the stale graph (it runs eagerly and records anew)."""
    import torch
    s, X = _block("n27", "fp64", 63)
    prec = B.ABI_PREC_FP64
    bd = BOUNDS[1]
    ref = _eager(s, prec, X, 5, bd)
    H = hamiltonian("n27")
    big = to_dev(W.random_block(H.npw, 4 * s.nband, 64))
    with B.System(s, precision=prec) as g:
        g.set_tuning(B.TUNE_FILTER_GRAPH, 1)
        Y = torch.empty_like(X)
        g.cheb_filter(X, 5, *bd, out=Y)
        g.cheb_filter(X, 5, *bd, out=Y)   # replay
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
        g.cheb_filter(big, 5, *bd)        # grows the iterate and FFT buffers
        torch.cuda.synchronize()
        for _ in range(2):
            g.cheb_filter(X, 5, *bd, out=Y)
            torch.cuda.synchronize()
            assert torch.equal(Y, ref)
