"""FP32-mixed form against the FP64 oracle (needs an MI355X).

The mixed form runs the FFT passes, the recurrence and the projector products in
single precision on complex64 blocks and keeps the bounds' Lanczos run, the
Cholesky factorisation, the eigensolver and the Rayleigh-Ritz step in FP64.
There is no closed form for its rounding error, so it is compared with the FP64
oracle within error budgets derived from FP32 rounding (unit roundoff 6e-8):

* one H application: per column ||diff||/||ref|| <= 2e-6 (FFT of 3 passes of
  log2 n radix stages plus FP32-accumulated projector sums);
* degree-m filter: <= 5e-6 * m per column;
* Rayleigh-Ritz of a complex64 block: the FP64 pencil of that block, so FP64
  tolerance (1e-8 Ha) against the oracle run on the same rounded block;
* a full cycle (bounds, filter, Rayleigh-Ritz): Ritz values within 1e-6 Ha of
  the FP64 oracle's cycle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import col_rel_err, hamiltonian, system, to_dev, to_host

pytestmark = pytest.mark.gpu

NAMES = ["odd15", "n27", "c1"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


def _mixed(name):
    return B.System(system(name), precision=B.ABI_PREC_MIXED)


def _c64(X):
    return to_dev(X).to(dtype=__import__("torch").complex64)


@pytest.mark.parametrize("name", NAMES)
def test_mixed_apply_H(name):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag).astype(np.complex64).astype(np.complex128)
    with _mixed(name) as g:
        got = to_host(g.apply_H(_c64(X)))
    assert got.dtype == np.complex64
    assert col_rel_err(got.astype(np.complex128), H(X)) <= 2e-6


@pytest.mark.parametrize("name,generic", [("noncubic", False), ("n27", True), ("c1", True)])
def test_mixed_apply_H_generic_fft(name, generic):
    """Runtime-size FFT passes in the mixed form (the last pass adds the projector
    part computed before it): a non-cubic box, and cubic boxes forced onto them."""
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, 12).astype(np.complex64).astype(np.complex128)
    with _mixed(name) as g:
        g.set_tuning(B.TUNE_GENERIC_FFT, int(generic))
        got = to_host(g.apply_H(_c64(X)))
    assert col_rel_err(got.astype(np.complex128), H(X)) <= 2e-6


@pytest.mark.parametrize("nb", [1, 2, 65])
def test_mixed_apply_H_band_counts(nb):
    """One, two and 65 bands: expansion tiles with one, two and one-past-a-tile
    columns, FFT batches of one band."""
    name = "n27"
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, nb, 13).astype(np.complex64).astype(np.complex128)
    with _mixed(name) as g:
        got = to_host(g.apply_H(_c64(X)))
    assert got.shape == X.shape
    assert col_rel_err(got.astype(np.complex128), H(X)) <= 2e-6


def test_mixed_apply_H_config2_ragged():
    """77 bands of the medium workload: one full 64-band FFT batch and a ragged
    one, a full and a ragged expansion tile (128 x 64)."""
    s = W.make_system(2)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 77, 2).astype(np.complex64).astype(np.complex128)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        got = to_host(g.apply_H(_c64(X)))
    assert col_rel_err(got.astype(np.complex128), H(X)) <= 2e-6


def test_mixed_apply_H_every_gemm_variant():
    """Every projection (0..16) and expansion (0..15) tile variant the tuning
    parameters select, on 300 bands of the medium workload (256 projectors: two
    row tiles; ragged column tiles; split-K over 22119 plane waves), against the
    oracle's H X.  The autotuner may pick any of them."""
    s = W.make_system(2)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 300, 5).astype(np.complex64).astype(np.complex128)
    ref = H(X)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Xd = _c64(X)
        p0, e0 = g.get_tuning(B.TUNE_PROJ), g.get_tuning(B.TUNE_EXPAND)
        for param, variants, keep in ((B.TUNE_PROJ, range(17), (B.TUNE_EXPAND, e0)),
                                      (B.TUNE_EXPAND, range(16), (B.TUNE_PROJ, p0))):
            g.set_tuning(*keep)
            for v in variants:
                g.set_tuning(param, v)
                err = col_rel_err(to_host(g.apply_H(Xd)).astype(np.complex128), ref)
                print(f"tuning {param} = {v}: {err:.3e}", flush=True)
                assert err <= 2e-6, (param, v, err)


@pytest.mark.parametrize("name,degree", [("odd15", 3), ("n27", 6), ("c1", 8)])
def test_mixed_filter(name, degree):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag).astype(np.complex64).astype(np.complex128)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds(H, X, v0)
    ref = O.cheb_filter(H, X, degree, a, b, a0)
    with _mixed(name) as g:
        got = to_host(g.cheb_filter(_c64(X), degree, a, b, a0)).astype(np.complex128)
    assert col_rel_err(got, ref) <= 5e-6 * degree


@pytest.mark.parametrize("name", ["n27", "noncubic"])
def test_mixed_filter_chained_planes(name):
    """Projection variants 15 and 16 read the bf16 planes of each step's input,
    which the previous step's last FFT pass writes (specialised passes on the
    27^3 box, runtime-size ones on the non-cubic box); the split they write is
    the one the block-reading variant 14 forms while staging, so the three
    filters agree to the products' rounding."""
    import torch
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, 40, 17)
    a, b, a0 = O.filter_bounds(H, X, W.random_vector(H.npw, s.tag))
    outs = {}
    with _mixed(name) as g:
        for v in (14, 15, 16):
            g.set_tuning(B.TUNE_PROJ, v)
            outs[v] = to_host(g.cheb_filter(_c64(X), 6, a, b, a0)).astype(np.complex128)
            torch.cuda.synchronize()
    for v in (15, 16):
        assert np.isfinite(outs[v]).all()
        err = col_rel_err(outs[v], outs[14])
        print(f"variant {v} vs 14: {err:.3e}", flush=True)
        assert err <= 1e-6, (v, err)


@pytest.mark.parametrize("name", NAMES)
def test_mixed_bounds(name):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag).astype(np.complex64).astype(np.complex128)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds(H, X, v0)
    with _mixed(name) as g:
        ga, gb, ga0 = g.spectral_bounds(_c64(X), to_dev(v0))
    assert abs(ga - a) <= 2e-6 * max(1.0, abs(a))
    assert abs(ga0 - a0) <= 2e-6 * max(1.0, abs(a0))
    assert abs(gb - b) <= 1e-10 * abs(b)


@pytest.mark.parametrize("name", NAMES)
def test_mixed_rayleigh_ritz_is_fp64(name):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds(H, X, v0)
    Y = O.cheb_filter(H, X, 6, a, b, a0).astype(np.complex64).astype(np.complex128)
    rr = O.rayleigh_ritz(H, Y)
    with _mixed(name) as g:
        Yd = _c64(Y)
        ev, res, flags = g.rayleigh_ritz(Yd)
    assert np.abs(ev - rr["eval"]).max() <= 1e-8


@pytest.mark.parametrize("name", NAMES)
def test_mixed_cycle_eigenvalues(name):
    """Two cycles: Ritz values within 1e-6 Ha of the FP64 oracle's cycles."""
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    Xr = X.copy()
    for _ in range(2):
        a, b, a0 = O.filter_bounds(H, Xr, v0)
        rr = O.rayleigh_ritz(H, O.cheb_filter(H, Xr, s.degree, a, b, a0))
        Xr = rr["Psi"]
    with _mixed(name) as g:
        Xd = _c64(X)
        v0d = to_dev(v0)
        for _ in range(2):
            ga, gb, ga0 = g.spectral_bounds(Xd, v0d)
            Yd = g.cheb_filter(Xd, s.degree, ga, gb, ga0)
            ev, res, _ = g.rayleigh_ritz(Yd)
            Xd = Yd
    assert np.abs(ev - rr["eval"]).max() <= 1e-6


def test_c64_needs_mixed_handle():
    import torch
    s = system("tiny_k")
    with B.System(s) as g:
        X = torch.zeros((2, g.npw), dtype=torch.complex64, device="cuda")
        with pytest.raises(B.ChebfiError) as e:
            g.apply_H(X)
        assert e.value.code == B.ABI_ERR_STATE
