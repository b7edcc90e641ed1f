"""The no-allocation H application against abi_apply_H (needs an MI355X).

abi_apply_H_noalloc carves every work buffer out of the library's static
per-device scratch array instead of allocating.  Its output must meet the
parity bar of abi_apply_H's own tests against it (FP64: per column
||diff|| / ||ref|| <= 1e-10; mixed: <= 2e-6) on two calls in a row, the
second with fewer bands, including cases where the scratch array limits the
FFT box batch; a call whose buffers exceed the array fails with
ABI_ERR_NOMEM.
"""
import numpy as np
import pytest

import workloads as W
from paper_2604_11139_amd import binding as B

from gpu_util import col_rel_err, system, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    yield
    torch.cuda.synchronize()


def _system(name):
    return W.make_system(2) if name == "c2" else system(name)


# (system, precision, bands of the first call, bands of the second call)
CASES = [
    ("c1", B.ABI_PREC_FP64, 32, 7),
    ("c1", B.ABI_PREC_MIXED, 32, 5),
    ("odd15", B.ABI_PREC_FP64, 19, 1),
    ("n27", B.ABI_PREC_MIXED, 37, 2),
    ("c2", B.ABI_PREC_FP64, 256, 100),   # box batch limited by the scratch array
    ("c2", B.ABI_PREC_MIXED, 128, 65),
]


@pytest.mark.parametrize("name,prec,nb1,nb2", CASES)
def test_noalloc_apply_H_matches_apply_H(name, prec, nb1, nb2):
    import torch
    s = _system(name)
    dt = torch.complex128 if prec == B.ABI_PREC_FP64 else torch.complex64
    tol = 1e-10 if prec == B.ABI_PREC_FP64 else 2e-6
    print(f"no-alloc apply_H: {name} precision {prec} bands {nb1} then {nb2}", flush=True)
    with B.System(s, precision=prec) as g:
        X = torch.from_numpy(W.random_block(g.npw, nb1, 41).T.copy()).to("cuda").to(dt)
        for nb in (nb1, nb2):
            Xn = X[:nb].contiguous()
            ref = g.apply_H(Xn)
            out = torch.full_like(Xn, float("nan"))
            g.apply_H_noalloc(Xn, out)
            torch.cuda.synchronize()
            got, want = to_host(out), to_host(ref)
            assert np.isfinite(got).all()
            err = col_rel_err(got.astype(np.complex128), want.astype(np.complex128))
            assert err <= tol, (name, nb, err)


def test_noalloc_rejects_work_beyond_scratch():
    import torch
    s = _system("c2")
    with B.System(s, precision=B.ABI_PREC_MIXED) as g:
        # the projector part alone is 22119 x 512 complex64 = 90 MB > 64 MiB
        X = torch.zeros((512, g.npw), dtype=torch.complex64, device="cuda")
        out = torch.empty_like(X)
        with pytest.raises(B.ChebfiError) as e:
            g.apply_H_noalloc(X, out)
        assert e.value.code == B.ABI_ERR_NOMEM
        assert "scratch" in str(e.value)
        # the handle still works for a size that fits
        g.apply_H_noalloc(X[:8].contiguous(), out[:8])
        torch.cuda.synchronize()
        assert np.isfinite(to_host(out[:8])).all()
