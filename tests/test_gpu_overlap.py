"""Parity of the generalised problem H psi = lambda S psi (S = I + P Q P^H).

Against the FP64 oracle (which inverts S by the Woodbury identity
K = (I + Q B)^-1 Q, a different route from the library's eigen-decomposition
of R Q R^H), on the PAW-like variants of the small systems:

* smallest eigenvalue of S: dense eigvalsh of the oracle's S, <= 1e-10;
* S X and S^-1 X per column: FP64 <= 1e-12; complex64 blocks <= 1e-6
  (split-BF16 projection, FP32 storage);
* bounds (generalised Rayleigh quotients, S-Lanczos): <= 1e-10 relative;
* filter on S^-1 H: FP64 <= 1e-9 per column, mixed <= 5e-6 x degree (the
  S = I budgets: the carried projections add products of the same size);
* Rayleigh-Ritz with the S-Gram: Ritz values <= 1e-8 Ha, residual norms
  ||H psi - lambda S psi|| <= 1e-8 absolute, Psi S-orthonormal to 1e-10;
* Q = 0 through the generalised path equals the S = I path to rounding;
* the solver loop converges to the lowest pairs of the dense pencil (H, S);
* full size (115313 plane waves, 2048 bands, degree 12, 864 projectors):
  sampled filter columns against the oracle (column-independent filter), and
  the FP64 S-Lanczos bound and sampled Ritz pairs' properties;
* errors: an S that is not positive definite, the adjoint and the batched
  filter with S != I are refused;
* one band (matrix-vector products) and a ragged band count; the band halves
  pipelined on two streams give the one-stream result bit for bit.
"""
import functools

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import SMALL, col_rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

NAMES = ["tiny_k", "odd15", "n27", "n25", "c1"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


@functools.lru_cache(maxsize=None)
def paw(name, q_scale=W.PAW_Q_SCALE):
    kw = dict(SMALL[name])
    tag = kw.pop("tag")
    return W.make_system(tag, q_scale=q_scale, **kw)


@functools.lru_cache(maxsize=None)
def oracle_pair(name):
    s = paw(name)
    H = O.Hamiltonian.from_system(s)
    return H, O.Overlap.from_system(H, s)


def _c64(X):
    import torch
    return to_dev(X).to(torch.complex64)


def _r64(X):
    return np.asarray(X).astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("name", NAMES)
def test_overlap_spectrum(name):
    H, S = oracle_pair(name)
    ref = np.linalg.eigvalsh(S.dense()).min()
    with B.System(paw(name)) as g:
        has, smin = g.overlap_info()
    assert has and abs(smin - ref) <= 1e-10


@pytest.mark.parametrize("name", NAMES)
def test_apply_S_and_Sinv(name):
    H, S = oracle_pair(name)
    s = paw(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    with B.System(s) as g:
        Xd = to_dev(X)
        got_s = to_host(g.apply_S(Xd))
        got_i = to_host(g.apply_Sinv(Xd))
        back = to_host(g.apply_S(g.apply_Sinv(Xd)))
    assert col_rel_err(got_s, S.apply(X)) <= 1e-12
    assert col_rel_err(got_i, S.inv_apply(X)) <= 1e-12
    assert col_rel_err(back, X) <= 1e-12


@pytest.mark.parametrize("name", ["odd15", "c1"])
def test_apply_S_and_Sinv_mixed(name):
    H, S = oracle_pair(name)
    s = paw(name)
    X = _r64(W.random_block(H.npw, s.nband, s.tag))
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        got_s = to_host(g.apply_S(_c64(X))).astype(np.complex128)
        got_i = to_host(g.apply_Sinv(_c64(X))).astype(np.complex128)
    assert col_rel_err(got_s, S.apply(X)) <= 1e-6
    assert col_rel_err(got_i, S.inv_apply(X)) <= 1e-6


@pytest.mark.parametrize("name", NAMES)
def test_bounds(name):
    H, S = oracle_pair(name)
    s = paw(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    ref = O.filter_bounds_gen(H, S, X, v0)
    with B.System(s) as g:
        got = g.spectral_bounds(to_dev(X), to_dev(v0))
    for x, r in zip(got, ref):
        assert abs(x - r) <= 1e-10 * max(1.0, abs(r))


@pytest.mark.parametrize("name,degree", [("tiny_k", 1), ("tiny_k", 2), ("odd15", 5),
                                         ("n27", 8), ("n25", 3), ("c1", 8)])
def test_filter(name, degree):
    H, S = oracle_pair(name)
    s = paw(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds_gen(H, S, X, v0)
    ref = O.cheb_filter(O.sinv_h(H, S), X, degree, a, b, a0)
    with B.System(s) as g:
        got = to_host(g.cheb_filter(to_dev(X), degree, a, b, a0))
    assert col_rel_err(got, ref) <= 1e-9


@pytest.mark.parametrize("name,degree", [("odd15", 3), ("n27", 6), ("c1", 8)])
def test_filter_mixed(name, degree):
    H, S = oracle_pair(name)
    s = paw(name)
    X = _r64(W.random_block(H.npw, s.nband, s.tag))
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds_gen(H, S, X, v0)
    ref = O.cheb_filter(O.sinv_h(H, S), X, degree, a, b, a0)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        got = to_host(g.cheb_filter(_c64(X), degree, a, b, a0)).astype(np.complex128)
    assert col_rel_err(got, ref) <= 5e-6 * degree


@pytest.mark.parametrize("name", ["tiny_k", "n27", "c1"])
def test_rayleigh_ritz(name):
    H, S = oracle_pair(name)
    s = paw(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds_gen(H, S, X, v0)
    Y = O.cheb_filter(O.sinv_h(H, S), X, 6, a, b, a0)
    rr = O.rayleigh_ritz_gen(H.apply, S.apply, Y)
    res = O.residual_norms_gen(rr["HPsi"], rr["SPsi"], rr["eval"])
    with B.System(s) as g:
        Yd = to_dev(Y)
        ev, rn, _ = g.rayleigh_ritz(Yd)
        Psi = to_host(Yd)
        SPsi = to_host(g.apply_S(Yd))
    assert np.abs(ev - rr["eval"]).max() <= 1e-8
    assert np.abs(rn - res).max() <= 1e-8
    assert np.abs(Psi.conj().T @ SPsi - np.eye(s.nband)).max() <= 1e-10


def test_zero_q_matches_plain_path():
    s0 = W.make_system(103, **{k: v for k, v in SMALL["n27"].items() if k != "tag"})
    sq = W.make_system(103, q_scale=1.0, **{k: v for k, v in SMALL["n27"].items() if k != "tag"})
    sq.qij = np.zeros_like(sq.qij)
    H = O.Hamiltonian.from_system(s0)
    X = W.random_block(H.npw, s0.nband, 5)
    v0 = W.random_vector(H.npw, 5)
    with B.System(s0) as g0, B.System(sq) as gq:
        assert gq.overlap_info() == (True, 1.0)
        bd0 = g0.spectral_bounds(to_dev(X), to_dev(v0))
        bdq = gq.spectral_bounds(to_dev(X), to_dev(v0))
        y0 = to_host(g0.cheb_filter(to_dev(X), 7, *bd0))
        yq = to_host(gq.cheb_filter(to_dev(X), 7, *bd0))
    assert np.allclose(bd0, bdq, rtol=1e-12, atol=0)
    assert col_rel_err(yq, y0) <= 1e-12


def test_solver_converges_to_dense_pencil():
    s = paw("tiny_k")
    H, S = oracle_pair("tiny_k")
    lam = scipy.linalg.eigh(H.dense(), S.dense(), eigvals_only=True)
    nconv = 5
    X = W.random_block(H.npw, s.nband, 77)
    v0 = W.random_vector(H.npw, 77)
    with B.System(s) as g:
        Xd = to_dev(X)
        ev, res, info = g.solve(Xd, to_dev(v0), degree=8, max_cycles=30, nconv=nconv, tol=1e-9)
    assert info["converged"]
    assert np.abs(ev[:nconv] - lam[:nconv]).max() <= 1e-8
    assert res[:nconv].max() <= 1e-9


def test_indefinite_overlap_is_refused():
    s = paw("odd15")
    bad = W.make_system(102, q_scale=1.0, **{k: v for k, v in SMALL["odd15"].items()
                                             if k != "tag"})
    bad.qij = -1e4 * np.repeat(np.eye(4)[None], bad.natom, axis=0).astype(np.complex128)
    with pytest.raises(B.ChebfiError) as e:
        B.System(bad)
    assert e.value.code == B.ABI_ERR_NOT_HPD
    with B.System(s) as g:
        X = to_dev(W.random_block(g.npw, 3, 9))
        with pytest.raises(B.ChebfiError) as e:
            g.filter_backward(X, X.clone(), 3, 1.0, 5.0, 0.0)
        assert e.value.code == B.ABI_ERR_STATE
    with pytest.raises(B.ChebfiError) as e:
        B.Batch([s])
    assert e.value.code == B.ABI_ERR_ARG


COLS = [0, 1023, 2047]


def test_fullsize_filter_sampled_columns():
    """The large workload with the overlap, mixed form (the timed configuration)."""
    import torch
    s = W.make_system(3, q_scale=W.PAW_Q_SCALE)
    H = O.Hamiltonian.from_system(s)
    S = O.Overlap.from_system(H, s)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Xd = to_dev(X)
        bounds = g.spectral_bounds(Xd, to_dev(v0))
        Xd = Xd.to(torch.complex64)
        Yd = g.cheb_filter(Xd, s.degree, *bounds)
        got = Yd[COLS].cpu().numpy().T.astype(np.complex128)
        del Yd, Xd
    Xs = _r64(X[:, COLS])
    ref = O.cheb_filter(O.sinv_h(H, S), Xs, s.degree, *bounds)
    assert col_rel_err(got, ref) <= 5e-6 * s.degree


@pytest.mark.parametrize("nband", [1, 37])
def test_filter_single_and_ragged(nband):
    """One band (the matrix-vector products) and a ragged band count."""
    H, S = oracle_pair("n27")
    s = paw("n27")
    X = W.random_block(H.npw, nband, 61)
    v0 = W.random_vector(H.npw, 61)
    a, b, a0 = O.filter_bounds_gen(H, S, X, v0)
    ref = O.cheb_filter(O.sinv_h(H, S), X, 5, a, b, a0)
    with B.System(s) as g:
        got = to_host(g.cheb_filter(to_dev(X), 5, a, b, a0))
        gs = to_host(g.apply_Sinv(to_dev(X)))
    assert col_rel_err(got, ref) <= 1e-9
    assert col_rel_err(gs, S.inv_apply(X)) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_stream_halves_match_one_stream(precision):
    """The pipelined band halves on two streams (130 bands: halves of 96 and 34) give the
    one-stream result bit for bit."""
    import torch
    H, S = oracle_pair("n27")
    s = paw("n27")
    X = W.random_block(H.npw, 130, 62)
    if precision == "mixed":
        X = _r64(X)
    prec = B.ABI_PREC_MIXED if precision == "mixed" else B.ABI_PREC_FP64
    outs = []
    for ov in (0, 1):
        with B.System(s, precision=prec) as g:
            g.set_tuning(B.TUNE_OVERLAP, ov)
            Xd = to_dev(X)
            if precision == "mixed":
                Xd = Xd.to(torch.complex64)
            outs.append(to_host(g.cheb_filter(Xd, 4, 1.0, 9.0, -0.5)))
    assert np.array_equal(outs[0], outs[1])


def test_fullsize_bounds_and_rayleigh_ritz_properties():
    """The large workload with the overlap, FP64: the S-Lanczos bound depends on v0 only
    (oracle 1e-10); after a filter and the S-Gram Rayleigh-Ritz, sampled Ritz vectors
    have generalised Rayleigh quotients equal to their Ritz values (1e-8 Ha), the
    library's residual norms ||H psi - lambda S psi|| (1e-8) and S-orthonormality
    (1e-10)."""
    s = W.make_system(3, q_scale=W.PAW_Q_SCALE)
    H = O.Hamiltonian.from_system(s)
    S = O.Overlap.from_system(H, s)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    cols = [0, 1, 2, 1024, 2046, 2047]
    with B.System(s) as g:
        Xd = to_dev(X)
        a, b, a0 = g.spectral_bounds(Xd, to_dev(v0))
        Yd = g.cheb_filter(Xd, s.degree, a, b, a0)
        del Xd
        ev, res, flags = g.rayleigh_ritz(Yd)
        Psi = Yd[cols].cpu().numpy().T
        del Yd
    ref_b, _, _ = O.lanczos_upper_bound_gen(H.apply, S.apply, S.inv_apply, v0, 10)
    assert abs(b - ref_b) <= 1e-10 * abs(ref_b)
    assert flags == 0 and np.all(np.diff(ev) >= 0)
    HPsi, SPsi = H(Psi), S.apply(Psi)
    rq = O.rayleigh_quotients_gen(Psi, HPsi, SPsi)
    assert np.abs(rq - ev[cols]).max() <= 1e-8
    r = np.linalg.norm(HPsi - SPsi * ev[cols][None, :], axis=0)
    assert np.abs(r - res[cols]).max() <= 1e-8
    assert np.abs(Psi.conj().T @ SPsi - np.eye(len(cols))).max() <= 1e-10
