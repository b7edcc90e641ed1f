"""Parity of the HIP path against the FP64 oracle (needs an MI355X).

Tolerances (FP64 path): H X per column ||diff|| / ||ref|| <= 1e-10; filter
output per column <= 1e-9 (relative, a degree-m polynomial compounds
rounding); bounds <= 1e-10 relative; Ritz values <= 1e-8 Ha absolute.
Basis maps are compared bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import SMALL, col_rel_err, hamiltonian, system, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


def _sys(name, **kw):
    return B.System(system(name, **kw))


@pytest.mark.parametrize("name", list(SMALL))
def test_tables(name):
    H = hamiltonian(name)
    with _sys(name) as g:
        miller, box = g.gsphere()
        assert np.array_equal(miller, H.sphere.miller)
        assert np.array_equal(box.astype(np.int64), H.sphere.box_index)
        P = to_host(g.projectors())
        assert P.shape == H.P.shape
        assert np.abs(P - H.P).max() <= 1e-14 * np.abs(H.P).max()


@pytest.mark.parametrize("name", list(SMALL))
def test_apply_H(name):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    with _sys(name) as g:
        got = to_host(g.apply_H(to_dev(X)))
    assert col_rel_err(got, H(X)) <= 1e-10


@pytest.mark.parametrize("parts", ["local", "nonlocal", "free"])
def test_apply_H_parts(parts):
    scales = {"local": (1.0, 0.0), "nonlocal": (0.0, 100.0), "free": (0.0, 0.0)}[parts]
    H = hamiltonian("n27", *scales)
    s = system("n27", *scales)
    X = W.random_block(H.npw, s.nband, 7)
    with B.System(s) as g:
        got = to_host(g.apply_H(to_dev(X)))
    if parts == "free":
        assert np.array_equal(got, H.sphere.kinetic[:, None] * X)
    else:
        ref = H(X)
        part = H.local_apply(X) if parts == "local" else H.nonlocal_apply(X)
        assert col_rel_err(got, ref) <= 1e-10
        # the isolated part itself is resolved well above rounding
        assert np.linalg.norm(got - H.kinetic_apply(X) - part) <= 1e-10 * np.linalg.norm(part)


@pytest.mark.parametrize("name,generic", [("noncubic", False), ("n27", True), ("c1", True)])
def test_apply_H_generic_fft(name, generic):
    """Runtime-size FFT passes: a non-cubic box, and cubic boxes forced onto them."""
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, 11)
    with B.System(s) as g:
        g.set_tuning(B.TUNE_GENERIC_FFT, int(generic))
        assert g.get_tuning(B.TUNE_GENERIC_FFT) == int(generic)
        got = to_host(g.apply_H(to_dev(X)))
    assert col_rel_err(got, H(X)) <= 1e-10


def test_apply_H_config2_ragged():
    s = W.make_system(2)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, 77, 2)  # 77 bands: one full 64-column tile and a ragged tail
    with B.System(s) as g:
        got = to_host(g.apply_H(to_dev(X)))
    assert col_rel_err(got, H(X)) <= 1e-10


@pytest.mark.parametrize("name,degree", [("tiny_k", 1), ("tiny_k", 2), ("odd15", 3), ("n27", 4),
                                         ("c1", 8)])
def test_cheb_filter(name, degree):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds(H, X, v0)
    ref = O.cheb_filter(H, X, degree, a, b, a0)
    with _sys(name) as g:
        got = to_host(g.cheb_filter(to_dev(X), degree, a, b, a0))
    assert col_rel_err(got, ref) <= 1e-9


@pytest.mark.parametrize("name,degree,precision", [("tiny_k", 1, "fp64"), ("n27", 4, "fp64"),
                                                   ("c1", 8, "fp64"), ("n27", 6, "mixed"),
                                                   ("c1", 8, "mixed")])
def test_cheb_filter_from_given_hx(name, degree, precision):
    """The filter started from a given H X (the oracle's, so independent of the
    library's H application): the oracle's filter to 1e-9 (FP64) / the mixed
    filter budget 5e-6 m."""
    import torch
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    if precision == "mixed":
        X = X.astype(np.complex64).astype(np.complex128)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds(H, X, v0)
    ref = O.cheb_filter(H, X, degree, a, b, a0)
    HX = H(X)
    prec = B.ABI_PREC_MIXED if precision == "mixed" else B.ABI_PREC_FP64
    with B.System(s, precision=prec) as g:
        Xd, HXd = to_dev(X), to_dev(HX)
        if precision == "mixed":
            Xd, HXd = Xd.to(torch.complex64), HXd.to(torch.complex64)
        got = to_host(g.cheb_filter(Xd, degree, a, b, a0, hx=HXd)).astype(np.complex128)
        with pytest.raises(B.ChebfiError) as e:
            g.cheb_filter(Xd, degree, a, b, a0, out=HXd, hx=HXd)  # HX aliasing Y
        assert e.value.code == B.ABI_ERR_ARG
    tol = 5e-6 * degree if precision == "mixed" else 1e-9
    assert col_rel_err(got, ref) <= tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_filter_overlap_is_bitwise_neutral(precision):
    """The FFT passes on a second stream beside the projection give the same bits."""
    import torch
    s = system("n25")
    H = hamiltonian("n25")
    X = W.random_block(H.npw, s.nband, 31)
    prec = B.ABI_PREC_MIXED if precision == "mixed" else B.ABI_PREC_FP64
    outs = []
    for ov in (0, 1):
        with B.System(s, precision=prec) as g:
            g.set_tuning(B.TUNE_OVERLAP, ov)
            Xd = to_dev(X)
            if precision == "mixed":
                Xd = Xd.to(torch.complex64)
            outs.append(g.cheb_filter(Xd, 7, 0.5, 9.0, -1.5).cpu())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("name", ["tiny_k", "n25", "c1"])
def test_spectral_bounds(name):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    ref = O.filter_bounds(H, X, v0)
    with _sys(name) as g:
        got = g.spectral_bounds(to_dev(X), to_dev(v0))
    for x, y in zip(got, ref):
        assert abs(x - y) <= 1e-10 * max(1.0, abs(y))


def test_spectral_bounds_invariant_start():
    """Lanczos from an eigenvector stops after one step: b = its eigenvalue."""
    s = system("c1", 0.0, 0.0)
    H = hamiltonian("c1", 0.0, 0.0)
    X = W.random_block(H.npw, 4, 1)
    v0 = np.zeros(H.npw, dtype=np.complex128)
    v0[11] = 2.0
    ref = O.filter_bounds(H, X, v0)
    with B.System(s) as g:
        got = g.spectral_bounds(to_dev(X), to_dev(v0))
    assert abs(got[1] - H.sphere.kinetic[11]) <= 1e-12 and abs(ref[1] - got[1]) <= 1e-12


def _principal_sines(A, B_):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B_)
    s = np.linalg.svd(qa.conj().T @ qb, compute_uv=False)
    return np.sqrt(np.maximum(0.0, 1.0 - np.min(s) ** 2))


@pytest.mark.parametrize("name", ["odd15", "n27", "c1"])
def test_rayleigh_ritz(name):
    H = hamiltonian(name)
    s = system(name)
    X = W.random_block(H.npw, s.nband, s.tag)
    v0 = W.random_vector(H.npw, s.tag)
    a, b, a0 = O.filter_bounds(H, X, v0)
    Y = O.cheb_filter(H, X, 6, a, b, a0)
    rr = O.rayleigh_ritz(H, Y)
    res_ref = O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"])
    import torch
    with _sys(name) as g:
        Yd = to_dev(Y)
        hp = torch.empty_like(Yd)
        ev, res, flags = g.rayleigh_ritz(Yd, hp)
        Psi = to_host(Yd)
        HPsi = to_host(hp)
    assert flags == 0
    assert np.abs(ev - rr["eval"]).max() <= 1e-8
    assert np.abs(Psi.conj().T @ Psi - np.eye(s.nband)).max() <= 1e-9
    assert np.abs(res - res_ref).max() <= 1e-8
    assert col_rel_err(HPsi, H(Psi)) <= 1e-9
    # same lowest invariant subspace where the spectrum has a gap
    lam = rr["eval"]
    gaps = np.diff(lam[: s.nband // 2 + 1])
    p = int(np.argmax(gaps)) + 1
    assert _principal_sines(Psi[:, :p], rr["Psi"][:, :p]) <= 1e-7


@pytest.mark.parametrize("nb", [1, 2])
def test_rayleigh_ritz_one_and_two_bands(nb):
    """The smallest blocks: 1 x 1 and 2 x 2 Hermitian Grams (one partial tile),
    Cholesky and eigensolver of size 1 and 2."""
    s = system("n27")
    H = hamiltonian("n27")
    X = W.random_block(H.npw, nb, 7)
    rr = O.rayleigh_ritz(H, X)
    res_ref = O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"])
    import torch
    with B.System(s) as g:
        Yd = to_dev(X)
        ev, res, flags = g.rayleigh_ritz(Yd)
        Psi = to_host(Yd)
    assert flags == 0
    assert np.abs(ev - rr["eval"]).max() <= 1e-10 * max(1.0, np.abs(rr["eval"]).max())
    assert np.abs(Psi.conj().T @ Psi - np.eye(nb)).max() <= 1e-12
    assert np.abs(res - res_ref).max() <= 1e-9 * max(1.0, np.abs(res_ref).max())


@pytest.mark.parametrize("nb", [77, 130])
def test_rayleigh_ritz_ragged_tiles(nb):
    """Rayleigh-Ritz of 77 and 130 bands of the medium workload: the Hermitian
    Gram products span two and three 64-wide tiles with ragged last ones (only
    the upper tiles are formed, the rest is mirrored)."""
    s = W.make_system(2)
    H = O.Hamiltonian.from_system(s)
    X = W.random_block(H.npw, nb, 5)
    rr = O.rayleigh_ritz(H, X)
    res_ref = O.residual_norms(rr["Psi"], rr["HPsi"], rr["eval"])
    import torch
    with B.System(s) as g:
        Yd = to_dev(X)
        hp = torch.empty_like(Yd)
        ev, res, flags = g.rayleigh_ritz(Yd, hp)
        Psi = to_host(Yd)
    assert flags == 0
    assert np.abs(ev - rr["eval"]).max() <= 1e-8 * max(1.0, np.abs(rr["eval"]).max())
    assert np.abs(Psi.conj().T @ Psi - np.eye(nb)).max() <= 1e-9
    assert np.abs(res - res_ref).max() <= 1e-8 * max(1.0, np.abs(res_ref).max())


def test_rayleigh_ritz_rank_deficient():
    s = system("tiny_k")
    H = hamiltonian("tiny_k")
    X = W.random_block(H.npw, 6, 3)
    X[:, 5] = X[:, 1]  # duplicate column: Gram matrix singular
    with B.System(s) as g:
        with pytest.raises(B.ChebfiError) as e:
            g.rayleigh_ritz(to_dev(X))
    assert e.value.code == B.ABI_ERR_NOT_HPD


@pytest.mark.parametrize("m", [1, 2, 7, 33, 64, 65, 95, 96, 130, 300, 1000])
def test_zheev(m):
    import torch
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    A = A + A.conj().T
    w, Z = B.zheev(torch.from_numpy(A).cuda())
    w = w.cpu().numpy()
    Z = Z.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    scale = np.abs(ref).max()
    assert np.abs(w - ref).max() <= 1e-12 * scale * max(1, np.sqrt(m))
    assert np.abs(A @ Z - Z * w[None, :]).max() <= 1e-11 * scale
    assert np.abs(Z.conj().T @ Z - np.eye(m)).max() <= 1e-11


def test_zheev_degenerate():
    import torch
    rng = np.random.default_rng(9)
    m = 40
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    lam = np.repeat(np.arange(8, dtype=np.float64), 5)  # 8 five-fold clusters
    A = (Q * lam[None, :]) @ Q.conj().T
    w, Z = B.zheev(torch.from_numpy(A).cuda())
    w = w.cpu().numpy()
    Z = Z.cpu().numpy()
    assert np.abs(w - lam).max() <= 1e-12 * 8
    assert np.abs(A @ Z - Z * w[None, :]).max() <= 1e-11 * 8
    assert np.abs(Z.conj().T @ Z - np.eye(m)).max() <= 1e-11


@pytest.mark.parametrize("m", [2048, 2560, 3000])
def test_zheev_large(m):
    """The Rayleigh-Ritz size of the large workload, the largest size whose
    clusters' inverse iteration runs in LDS, and one above it (global-memory
    arrays); one past the eigensolver's limit (8192) is an argument error."""
    import torch
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    A = A + A.conj().T
    w, Z = B.zheev(torch.from_numpy(A).cuda())
    w = w.cpu().numpy()
    Z = Z.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    scale = np.abs(ref).max()
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 1e-12 * scale * np.sqrt(m)
    assert np.abs(A @ Z - Z * w[None, :]).max() <= 1e-11 * scale
    assert np.abs(Z.conj().T @ Z - np.eye(m)).max() <= 1e-11
    if m == 3000:
        with pytest.raises(B.ChebfiError) as e:
            B.zheev(torch.zeros((8193, 8193), dtype=torch.complex128, device="cuda"))
        assert e.value.code == B.ABI_ERR_ARG


@pytest.mark.parametrize("kind,m", [("repeated", 600), ("near", 600), ("repeated", 2700)])
def test_zheev_clusters_large(kind, m):
    """Wide clusters: 12 eigenvalues of multiplicity 50 (exactly repeated), or
    spread by 1e-10 inside each cluster (closer than the inverse iteration's
    cluster gap, distinct to the multisection); at m = 2700 with 2100 more
    distinct eigenvalues, so that the clusters' inverse iteration keeps its
    arrays in global memory (above the LDS size)."""
    import torch
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    lam = np.repeat(np.arange(12, dtype=np.float64) - 5.5, 50)
    if kind == "near":
        lam = lam + 1e-10 * np.tile(np.arange(50), 12)
    if m > 600:
        # distinct values between the clusters (gaps well above the cluster gap)
        lam = np.concatenate([lam, np.linspace(-6.0, 6.0, m - 600) + 0.0123])
    A = (Q * lam[None, :]) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    w, Z = B.zheev(torch.from_numpy(A).cuda())
    w = w.cpu().numpy()
    Z = Z.cpu().numpy()
    assert np.abs(w - np.sort(lam)).max() <= 1e-12 * 6 * np.sqrt(m)
    assert np.abs(A @ Z - Z * w[None, :]).max() <= 1e-11 * 6
    assert np.abs(Z.conj().T @ Z - np.eye(m)).max() <= 1e-11


def test_zheev_max_size():
    """M = 8192 (the paper's largest band count, the eigensolver's limit): A =
    Q diag(lam) Q^H with Q = I - 2 u u^H (|u| = 1) a Householder reflection, so
    the eigenvalues are lam exactly; lam holds 8 clusters of 16 equal values
    among distinct ones.  Residual and orthogonality formed on the GPU (FP64
    complex products)."""
    import torch
    m = 8192
    rng = np.random.default_rng(8192)
    lam = np.sort(np.concatenate([np.repeat(np.linspace(-3.0, 3.0, 8), 16),
                                  rng.uniform(-4.0, 4.0, m - 128)]))
    u = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    u /= np.linalg.norm(u)
    dev = "cuda"
    ut = torch.from_numpy(u).to(dev)
    lt = torch.from_numpy(lam).to(dev).to(torch.complex128)
    # A = (I - 2 u u^H) D (I - 2 u u^H) = D - 2 u (D u)^H - 2 (D u) u^H + 4 (u^H D u) u u^H
    Du = lt * ut
    A = torch.diag(lt) - 2.0 * torch.outer(ut, Du.conj()) - 2.0 * torch.outer(Du, ut.conj())
    A = A + 4.0 * (ut.conj() @ Du) * torch.outer(ut, ut.conj())
    A = 0.5 * (A + A.conj().T)
    w, Z = B.zheev(A.clone())
    Z = Z.contiguous()
    w = w.cpu().numpy()
    scale = np.abs(lam).max()
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - lam).max() <= 1e-12 * scale * np.sqrt(m)
    wt = torch.from_numpy(w).to(dev).to(torch.complex128)
    R = A @ Z - Z * wt[None, :]
    assert R.abs().max().item() <= 1e-11 * scale
    O = Z.conj().T @ Z
    O.diagonal().sub_(1.0)
    assert O.abs().max().item() <= 1e-10
    del A, Z, R, O


@pytest.mark.parametrize("m", [1, 31, 33, 100, 257])
def test_zpotrf(m):
    import scipy.linalg
    import torch
    rng = np.random.default_rng(100 + m)
    X = rng.standard_normal((m + 5, m)) + 1j * rng.standard_normal((m + 5, m))
    G = X.conj().T @ X
    U = B.zpotrf_upper(torch.from_numpy(G).cuda()).cpu().numpy()
    ref = scipy.linalg.cholesky(G, lower=False)
    assert np.abs(U - ref).max() <= 1e-12 * np.abs(ref).max() * max(1.0, np.sqrt(m))


def test_zpotrf_not_hpd():
    import torch
    G = np.eye(40, dtype=np.complex128)
    G[17, 17] = -1.0
    with pytest.raises(B.ChebfiError) as e:
        B.zpotrf_upper(torch.from_numpy(G).cuda())
    assert e.value.code == B.ABI_ERR_NOT_HPD
    assert "18" in str(e.value)


def test_argument_errors():
    import torch
    s = system("tiny_k")
    with B.System(s) as g:
        X = torch.zeros((4, g.npw), dtype=torch.complex128, device="cuda")
        with pytest.raises(B.ChebfiError) as e:
            g.cheb_filter(X, 0, 1.0, 2.0, 0.0)
        assert e.value.code == B.ABI_ERR_ARG
        with pytest.raises(B.ChebfiError) as e:
            g.cheb_filter(X, 3, 2.0, 1.0, 0.0)
        assert e.value.code == B.ABI_ERR_ARG
        with pytest.raises(B.ChebfiError) as e:
            g.cheb_filter(X, 3, 1.0, 2.0, 1.5)
        assert e.value.code == B.ABI_ERR_ARG
