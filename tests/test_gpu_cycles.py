"""Four filter / Rayleigh-Ritz cycles on the large workload against the FP64
oracle's run of the same cycles (tests/golden/config3_cycles.json, written by
tests/golden/make_config3_reference.py from the oracle alone).

Workload: cubic a = 30 bohr, E_cut = 20 Ha, 115313 plane waves, 64^3 grid,
216 atoms, 2048 bands, degree 12, from the seeded start block; each cycle
takes its bounds from the current block (Rayleigh quotients, 10-step Lanczos
from the seeded v0), filters and applies Rayleigh-Ritz, whose Ritz vectors
start the next cycle.

* FP64: bounds of every cycle <= 1e-9 relative; Ritz values of every cycle
  <= 1e-8 Ha; residual norms of the last cycle <= 1e-8; the Hellmann-Feynman
  density rho_p of the lowest p Ritz vectors (p at the largest gap between
  bands 1000 and 1048) at the stored points <= 1e-8 of max rho.
* FP32-mixed (complex64 blocks and filter, FP64 bounds and Rayleigh-Ritz):
  Ritz values of the last cycle within 1e-6 Ha of the oracle's, for all bands
  and for the lowest half.
* Gradient of sum_{n<=p} eps_n with respect to V_loc through the last mixed
  filter and Rayleigh-Ritz, with checkpoints every 4th step: rho_p plus the
  filter adjoint with W = 2 R_p C_p^H.  Against the oracle's rho_p it may
  differ by the filter term, which is bounded by the residuals of the lowest
  p Ritz pairs: |grad - rho_p| <= 4 max_{n<=p} ||r_n|| max rho at every stored
  point, and the gradient sums to p within the same bound.
* The filter term itself, at full size: (1) the GPU adjoint with the GPU's own
  W on three of its columns (the filter acts on each column alone) against the
  oracle's adjoint of the same columns, <= 1e-5 m relative (the mixed adjoint
  bar); (2) central differences (h = 1e-3 Ha) of sum_{n<=p} eps_n through the
  mixed filter and the FP64 Rayleigh-Ritz from the same block and bounds, along
  three seeded directions dV: <grad, dV> within 1e-6 relative, and, along the
  direction where the filter term is largest, within 5% of that term, which
  rho_p alone misses by more than half of it.
"""
import functools
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import to_dev

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config3_cycles.json")


@functools.lru_cache(maxsize=None)
def _ref():
    return json.load(open(GOLD))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


def _cycles(g, X, v0, s, ncyc, want_last=False, lowprec_cycles=0, flags=None):
    """Runs ncyc cycles in place on X; returns per-cycle (bounds, eval, res)
    and, with want_last, the last cycle's input block and its outputs.  The
    first lowprec_cycles cycles ask for the split-BF16 Rayleigh-Ritz; their
    flags are appended to the list flags."""
    import torch
    out = []
    last = None
    hp = torch.empty_like(X)
    for c in range(ncyc):
        bounds = g.spectral_bounds(X, v0)
        Xin = X.clone() if (want_last and c == ncyc - 1) else None
        Y = g.cheb_filter(X, s.degree, *bounds)
        if want_last and c == ncyc - 1:
            ev, res, _, C = g.rayleigh_ritz(Y, hp, want_coef=True)
            last = (Xin, Y, hp, C, bounds)
        else:
            ev, res, fl = g.rayleigh_ritz(Y, lowprec=c < lowprec_cycles)
            if flags is not None and c < lowprec_cycles:
                flags.append(fl)
        X.copy_(Y)
        del Y
        out.append((bounds, np.asarray(ev), np.asarray(res)))
    return out, last


def test_fp64_cycles_match_oracle():
    ref = _ref()
    s = W.make_system(3)
    with B.System(s) as g:
        X = to_dev(W.random_block(g.npw, s.nband, s.tag))
        v0 = to_dev(W.random_vector(g.npw, s.tag))[0]
        runs, _ = _cycles(g, X, v0, s, len(ref["cycles"]))
        p = ref["p"]
        rho = g.density(X[:p]).cpu().numpy()
    for (bounds, ev, res), rc in zip(runs, ref["cycles"]):
        rb = np.array(rc["bounds"])
        assert np.all(np.abs(np.array(bounds) - rb) <= 1e-9 * np.abs(rb).max())
        assert np.abs(ev - np.array(rc["eval"])).max() <= 1e-8
    assert np.abs(runs[-1][2] - np.array(ref["last_residuals"])).max() <= 1e-8
    pts = np.array(ref["rho_points"])
    assert np.abs(rho[pts] - np.array(ref["rho_values"])).max() <= 1e-8 * ref["rho_max"]
    assert abs(rho.sum() - p) <= 1e-9 * p


def test_mixed_cycles_and_gradient_vs_oracle():
    import torch
    ref = _ref()
    s = W.make_system(3)
    p = ref["p"]
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        X = to_dev(W.random_block(g.npw, s.nband, s.tag)).to(torch.complex64)
        v0 = to_dev(W.random_vector(g.npw, s.tag))[0]
        runs, (Xin, Y, HY, C, bounds) = _cycles(g, X, v0, s, len(ref["cycles"]), want_last=True)
        ev, res = runs[-1][1], runs[-1][2]
        d = np.abs(ev - np.array(ref["cycles"][-1]["eval"]))
        assert d.max() <= 1e-6, d.max()
        assert d[: s.nband // 2].max() <= 1e-6
        # gradient of the sum of the lowest p Ritz values through filter + RR
        lam = torch.as_tensor(ev[:p], dtype=torch.float32, device="cuda")
        R = HY[:p] - Y[:p] * lam[:, None]          # rows = bands (p, npw)
        Cp = C[:, :p].to(torch.complex64)           # (M, p): Psi_p = Y_in C_p
        Wm = 2.0 * (Cp.conj() @ R)                  # rows: W = 2 R_p C_p^H, (M, npw)
        dV, _, _ = g.filter_backward(Xin, Wm.contiguous(), s.degree, *bounds, ckpt_every=4,
                                     want_dx=False)
        rho = g.density(Y[:p])
        grad = (rho + dV).cpu().numpy()
        rmax = float(res[:p].max())
        dV = dV.cpu().numpy()
        rho = rho.cpu().numpy()
        # (1) three columns of the GPU's W alone
        cols = [0, p // 2, p - 1]
        Wc = torch.zeros_like(Wm)
        Wc[cols] = Wm[cols]
        dVc, _, _ = g.filter_backward(Xin, Wc.contiguous(), s.degree, *bounds, ckpt_every=4,
                                      want_dx=False)
        dVc = dVc.cpu().numpy()
        Xc = Xin[cols].cpu().numpy().T.astype(np.complex128)
        Wcc = Wm[cols].cpu().numpy().T.astype(np.complex128)
        # (2) central differences of sum_{n<=p} eps_n along seeded directions
        V0 = torch.from_numpy(np.ascontiguousarray(s.vloc.reshape(-1))).to("cuda")
        rng = np.random.default_rng([2604, 11139, 55])
        dirs = [rng.standard_normal(V0.numel()) for _ in range(3)]
        h = 1e-3
        fd = []
        for dv in dirs:
            vals = []
            for t in (h, -h):
                g.update_potential(vloc=V0 + t * torch.from_numpy(dv).to("cuda"))
                Yt = g.cheb_filter(Xin, s.degree, *bounds)
                evt, _, _ = g.rayleigh_ritz(Yt)
                vals.append(float(np.sum(np.asarray(evt)[:p], dtype=np.float64)))
                del Yt
            fd.append((vals[0] - vals[1]) / (2 * h))
        g.update_potential(vloc=V0)
    pts = np.array(ref["rho_points"])
    tol = 4.0 * rmax * ref["rho_max"]
    assert np.abs(grad[pts] - np.array(ref["rho_values"])).max() <= tol
    assert abs(grad.sum() - p) <= 4.0 * rmax * p
    H = O.Hamiltonian.from_system(s)
    dV_ref, _, _ = O.filter_backward(H, Xc, Wcc, s.degree, *bounds)
    dV_ref = np.asarray(dV_ref).reshape(dVc.shape)
    assert np.abs(dVc - dV_ref).max() <= 1e-5 * s.degree * np.abs(dV_ref).max()
    chain = [float(np.dot(dV, dv)) for dv in dirs]
    for f, dv in zip(fd, dirs):
        assert abs(f - float(np.dot(grad, dv))) <= 1e-6 * abs(f)
    k = int(np.argmax(np.abs(chain)))
    assert abs(fd[k] - float(np.dot(grad, dirs[k]))) <= 0.05 * abs(chain[k])
    assert abs(fd[k] - float(np.dot(rho, dirs[k]))) >= 0.5 * abs(chain[k])


def test_mixed_lowprec_rr_cycles_vs_oracle():
    """The mixed form as the solver runs it before an FP64 refinement: all but
    the last cycle with the split-BF16 Rayleigh-Ritz, the last with the FP64
    one.  Ritz values within the mixed form's 1e-6 Ha of the oracle's cycles."""
    import torch
    ref = _ref()
    s = W.make_system(3)
    ncyc = len(ref["cycles"])
    flags = []
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        X = to_dev(W.random_block(g.npw, s.nband, s.tag)).to(torch.complex64)
        v0 = to_dev(W.random_vector(g.npw, s.tag))[0]
        runs, _ = _cycles(g, X, v0, s, ncyc, lowprec_cycles=ncyc - 1, flags=flags)
    assert all(f & B.RR_LOWPREC for f in flags) and len(flags) == ncyc - 1
    for (bounds, ev, res), rc in zip(runs[:-1], ref["cycles"][:-1]):
        # intermediate cycles: split-BF16 rounding of the Rayleigh-Ritz products
        rv = np.array(rc["eval"])
        assert np.abs(ev - rv).max() <= 1e-4 * np.abs(rv).max()
    d = np.abs(runs[-1][1] - np.array(ref["cycles"][-1]["eval"]))
    assert d.max() <= 1e-6, d.max()
