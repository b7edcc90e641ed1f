"""The autotuner (needs an MI355X): it keeps a launch choice, persists it in its
JSON cache under the problem's key, and a second handle of the same problem
takes the cached choice without timing; the tuned H application and filter
stay within the mixed form's parity bars against the FP64 oracle (H X: per
column 2e-6; degree-m filter: 5e-6 m)."""
import json

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import col_rel_err, hamiltonian, system, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


def test_autotune_persists_and_reloads(tmp_path):
    import torch
    name = "n25"
    s = system(name)
    H = hamiltonian(name)
    X = W.random_block(H.npw, s.nband, 51).astype(np.complex64).astype(np.complex128)
    cache = tmp_path / "tune.json"
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        Xd = to_dev(X).to(torch.complex64)
        choice, cached = g.autotune(Xd, cache)
        assert not cached
        got = to_host(g.apply_H(Xd))
        a, b, a0 = O.filter_bounds(H, X, W.random_vector(H.npw, s.tag))
        Yf = to_host(g.cheb_filter(Xd, 6, a, b, a0))
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert "npw=%d" % H.npw in key and "nband=%d" % s.nband in key and key.endswith("c64")
    assert {k: val[k] for k in choice} == choice
    assert col_rel_err(got.astype(np.complex128), H(X)) <= 2e-6
    assert col_rel_err(Yf.astype(np.complex128), O.cheb_filter(H, X, 6, a, b, a0)) <= 5e-6 * 6
    with B.System(s, precision=B.ABI_PREC_MIXED) as g2:
        choice2, cached2 = g2.autotune(to_dev(X).to(torch.complex64), cache)
        assert cached2 and choice2 == choice
    # another band count is another entry
    with B.System(s, precision=B.ABI_PREC_MIXED) as g3:
        _, cached3 = g3.autotune(to_dev(X[:, :9]).to(torch.complex64), cache)
        assert not cached3
    assert len(json.load(open(cache))) == 2


def test_autotune_fp64_block():
    s = system("c1")
    H = hamiltonian("c1")
    X = W.random_block(H.npw, s.nband, 52)
    with B.System(s) as g:
        choice, cached = g.autotune(to_dev(X))
        assert not cached and choice["fft_batch"] >= 1
        got = to_host(g.apply_H(to_dev(X)))
    assert col_rel_err(got, H(X)) <= 1e-10
