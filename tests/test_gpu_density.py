"""Density and the full-chain gradient of a Ritz-value sum (needs an MI355X).

* density of a block vs the oracle (FP64 <= 1e-12 relative, complex64 <= 1e-6);
* the Hellmann-Feynman density of the lowest p Ritz vectors vs the oracle's
  (same filter and Rayleigh-Ritz in FP64; p at a spectral gap);
* the gradient of L(V) = sum_{n<=p} eps_n through filter and Rayleigh-Ritz:
  rho_p (the derivative with the filtered block held fixed) plus the filter
  adjoint with W = 2 R_p C_p^H (R_p residuals, C_p Ritz coefficients, from
  d eps_n = 2 Re<dY c_n, r_n>), checked by central differences of the GPU
  pipeline (relative error <= 1e-6).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import hamiltonian, system, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["c1", "n27", "noncubic"])
def test_density_vs_oracle(name):
    import torch
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, 21)
    w = np.linspace(0.0, 2.0, s.nband)
    ref = O.density(H, X, w)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        rho = g.density(to_dev(X), w).cpu().numpy()
        rho32 = g.density(to_dev(X).to(torch.complex64), w).cpu().numpy()
    assert np.abs(rho - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(rho32 - ref).max() <= 1e-6 * np.abs(ref).max()


def _pipeline(g, Xd, degree, bounds, p):
    """sum of the lowest p Ritz values after filter + Rayleigh-Ritz (FP64)."""
    Y = g.cheb_filter(Xd, degree, *bounds)
    ev, _, _ = g.rayleigh_ritz(Y)
    return float(ev[:p].sum())


def _gap_index(ev, lo, hi):
    gaps = np.diff(ev[lo:hi])
    return lo + int(np.argmax(gaps)) + 1


def test_hf_density_vs_oracle():
    H = hamiltonian("c1")
    s = system("c1")
    X = W.random_block(H.npw, s.nband, 22)
    v0 = W.random_vector(H.npw, 22)
    a, b, a0 = O.filter_bounds(H, X, v0)
    Y = O.cheb_filter(H, X, s.degree, a, b, a0)
    rr = O.rayleigh_ritz(H, Y)
    p = _gap_index(rr["eval"], 4, s.nband // 2)
    ref = O.density(H, rr["Psi"][:, :p])
    with B.System(s) as g:
        Yd = to_dev(Y)
        ev, _, _ = g.rayleigh_ritz(Yd)
        rho = g.density(Yd[:p]).cpu().numpy()
    assert np.abs(ev - rr["eval"]).max() <= 1e-8
    assert np.abs(rho - ref).max() <= 1e-8 * np.abs(ref).max()
    assert abs(rho.sum() - p) <= 1e-10 * p


def test_ritz_sum_gradient_chain():
    import torch
    s = system("n27")
    H = hamiltonian("n27")
    degree = 6
    X = W.random_block(H.npw, s.nband, 23)
    v0 = W.random_vector(H.npw, 23)
    with B.System(s) as g:
        Xd = to_dev(X)
        bounds = g.spectral_bounds(Xd, to_dev(v0))
        Yd = g.cheb_filter(Xd, degree, *bounds)
        hp = torch.empty_like(Yd)
        ev, res, _, C = g.rayleigh_ritz(Yd, hp, want_coef=True)
        p = _gap_index(ev, 3, s.nband // 2)
        Psi, HPsi = to_host(Yd), to_host(hp)
        R = HPsi[:, :p] - Psi[:, :p] * ev[:p][None, :]
        Cp = C.cpu().numpy()[:, :p]
        Wm = 2.0 * R @ Cp.conj().T
        dV_chain, _, _ = g.filter_backward(Xd, to_dev(Wm), degree, *bounds, ckpt_every=0,
                                           want_dx=False)
        rho = g.density(Yd[:p])
        grad = (rho + dV_chain).cpu().numpy()
        V0 = torch.from_numpy(s.vloc).cuda()
        rng = np.random.default_rng(27)
        h = 1e-5
        worst = 0.0
        for _ in range(6):
            d = rng.standard_normal(s.vloc.shape)
            dd = torch.from_numpy(d).cuda()
            g.update_potential(V0 + h * dd, None)
            lp = _pipeline(g, Xd, degree, bounds, p)
            g.update_potential(V0 - h * dd, None)
            lm = _pipeline(g, Xd, degree, bounds, p)
            fd = (lp - lm) / (2 * h)
            an = float(grad @ d)
            worst = max(worst, abs(fd - an) / abs(an))
        g.update_potential(V0, None)
    assert worst <= 1e-6, worst
