"""Helpers shared by the GPU tests (layout conversion, cached oracle objects)."""
import functools

import numpy as np

import oracle as O
import workloads as W


def to_dev(X):
    """numpy (npw, nband) -> torch (nband, npw) complex128 on cuda:0."""
    import torch
    X = np.asarray(X, dtype=np.complex128)
    if X.ndim == 1:
        X = X[:, None]
    return torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda:0")


def to_host(t):
    """torch (nband, npw) -> numpy (npw, nband)."""
    return np.ascontiguousarray(t.detach().cpu().numpy().T)


def col_rel_err(got, ref):
    """max over columns of ||got - ref|| / ||ref||."""
    num = np.linalg.norm(got - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return float(np.max(num / np.maximum(den, 1e-300)))


SMALL = {
    "tiny_k": dict(tag=101, a=6.0, ecut=4.0, n=12, natom=2, nband=8, kpt_red=(0.1, 0.2, 0.3)),
    "odd15": dict(tag=102, a=7.0, ecut=5.0, n=15, natom=3, nband=19, kpt_red=(0.25, 0.0, 0.4)),
    "n27": dict(tag=103, a=10.0, ecut=6.0, n=27, natom=2, nband=37, kpt_red=(0.0, 0.33, 0.1)),
    "n25": dict(tag=104, a=9.0, ecut=6.0, n=25, natom=4, nband=70, kpt_red=(0.45, 0.45, 0.0)),
    "c1": dict(tag=1),
}


@functools.lru_cache(maxsize=None)
def system(name, vloc_scale=1.0, d_scale=1.0):
    if name == "noncubic":
        # 12 x 15 x 16 box: exercises the runtime-size FFT passes
        s = W.make_system(105, a=7.0, ecut=4.0, n=16, natom=2, nband=11,
                          kpt_red=(0.2, 0.1, 0.3), vloc_scale=vloc_scale, d_scale=d_scale)
        s.ngrid = (12, 15, 16)
        s.vloc = W.systems._gaussian_wells(s.tau, s.a, s.ngrid) * vloc_scale
        return s
    kw = dict(SMALL[name])
    tag = kw.pop("tag")
    return W.make_system(tag, vloc_scale=vloc_scale, d_scale=d_scale, **kw)


@functools.lru_cache(maxsize=None)
def hamiltonian(name, vloc_scale=1.0, d_scale=1.0):
    return O.Hamiltonian.from_system(system(name, vloc_scale, d_scale))
