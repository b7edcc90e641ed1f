"""ctypes binding of ``libchebfi.so`` (argument marshalling only).

Every computation runs in the HIP library; this module only converts Python
and torch objects to the pointers and sizes of the C ABI (include/chebfi.h).
PyTorch provides device memory and the current HIP stream.

Blocks of wave functions are torch complex128 tensors of shape (nband, npw)
with unit stride along the plane waves: row b is band b, which is exactly the
column-major npw x nband layout of the ABI with ld = tensor.stride(0).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchebfi.so")

ABI_OK = 0
ABI_ERR_ARG = -1
ABI_ERR_GRID = -2
ABI_ERR_NOT_HPD = -3
ABI_ERR_DEVICE = -4
ABI_ERR_NOMEM = -5
ABI_ERR_STATE = -6
ABI_C128 = 0
ABI_C64 = 1
ABI_PREC_FP64 = 0
ABI_PREC_MIXED = 1

EXPORTS = [
    "abi_gsphere_count", "abi_gsphere_build", "abi_set_system", "abi_system_info",
    "abi_get_gsphere", "abi_get_projectors", "abi_destroy", "abi_apply_H",
    "abi_spectral_bounds", "abi_cheb_filter", "abi_cheb_filter_hx", "abi_rayleigh_ritz",
    "abi_zpotrf_upper",
    "abi_zheev", "abi_profile_enable", "abi_profile_read", "abi_update_potential",
    "abi_filter_backward", "abi_density", "abi_last_error", "abi_set_system_batch",
    "abi_batch_system", "abi_cheb_filter_batch", "abi_batch_autotune", "abi_batch_use_graph",
    "abi_batch_use_overlap",
    "abi_destroy_batch", "abi_chebfi_solve", "abi_apply_S", "abi_apply_Sinv", "abi_overlap_info",
    "abi_lobpcg_solve", "abi_density_add", "abi_occupations", "abi_scf_potential", "abi_scf_solve",
    "abi_get_potential", "abi_set_tuning", "abi_get_tuning", "abi_apply_H_noalloc",
    "abi_autotune",
]

PROFILE_CLASSES = ["proj_gemm", "expand_gemm", "fft_a", "fft_b", "fft_c", "dapply", "gram",
                   "chol", "eig", "rot", "split"]


class ChebfiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chebfi error {code}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("abi_version", c_int32),
        ("lattice", c_double * 9),
        ("kpt_red", c_double * 3),
        ("ecut", c_double),
        ("ngrid", c_int32 * 3),
        ("vloc", POINTER(c_double)),
        ("natom", c_int32),
        ("tau_cart", POINTER(c_double)),
        ("rc", c_double),
        ("dij", POINTER(c_double)),
        ("precision", c_int32),
        ("qij", POINTER(c_double)),
    ]


(TUNE_PROJ, TUNE_EXPAND, TUNE_FFT_BATCH, TUNE_OVERLAP, TUNE_GENERIC_FFT, TUNE_MIXED_GEMM,
 TUNE_FILTER_GRAPH) = range(7)
RR_FELL_BACK, RR_LOWPREC, RR_TWO_PASS = 1, 2, 4

_lib = None


def lib():
    """Loads the library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2604_11139_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    sig = {
        "abi_gsphere_count": [POINTER(Desc), POINTER(c_int64)],
        "abi_gsphere_build": [POINTER(Desc), c_int64, vp, vp, vp],
        "abi_set_system": [POINTER(Desc), vp, POINTER(vp)],
        "abi_system_info": [vp, POINTER(c_int64), POINTER(c_int32), POINTER(c_int32)],
        "abi_get_gsphere": [vp, vp, vp],
        "abi_get_projectors": [vp, vp, vp],
        "abi_destroy": [vp],
        "abi_apply_H": [vp, vp, vp, c_int64, c_int64, c_int32, vp],
        "abi_spectral_bounds": [vp, vp, c_int64, c_int64, c_int32, vp, c_int32, vp, vp],
        "abi_cheb_filter": [vp, vp, vp, c_int64, c_int64, c_int32, c_int32, c_double, c_double,
                            c_double, vp],
        "abi_cheb_filter_hx": [vp, vp, vp, vp, c_int64, c_int64, c_int32, c_int32, c_double,
                               c_double, c_double, vp],
        "abi_rayleigh_ritz": [vp, vp, vp, c_int64, c_int64, c_int32, vp, vp, vp, vp, vp],
        "abi_zpotrf_upper": [c_int64, vp, c_int64, vp],
        "abi_zheev": [c_int64, vp, c_int64, vp, vp, c_int64, vp],
        "abi_profile_enable": [vp, c_int32],
        "abi_update_potential": [vp, vp, vp, vp],
        "abi_density": [vp, vp, c_int64, c_int64, c_int32, vp, vp, vp],
        "abi_filter_backward": [vp, vp, vp, c_int64, c_int64, c_int32, c_int32, c_double,
                                c_double, c_double, c_int32, vp, vp, vp, vp],
        "abi_profile_read": [vp, c_int32, vp, vp, vp],
        "abi_set_tuning": [vp, c_int32, c_int32],
        "abi_apply_H_noalloc": [vp, vp, vp, c_int64, c_int64, c_int32, vp],
        "abi_autotune": [vp, vp, c_int64, c_int64, c_int32, c_char_p, POINTER(c_int32), vp],
        "abi_get_tuning": [vp, c_int32, POINTER(c_int32)],
        "abi_set_system_batch": [vp, c_int32, vp, POINTER(vp)],
        "abi_batch_system": [vp, c_int32, POINTER(vp)],
        "abi_cheb_filter_batch": [vp, vp, vp, vp, vp, c_int32, c_int32, vp, vp, vp, vp],
        "abi_batch_autotune": [vp, vp, vp, vp, vp, c_int32, c_int32, vp, vp, vp, vp, vp],
        "abi_batch_use_graph": [vp, c_int32],
        "abi_batch_use_overlap": [vp, c_int32],
        "abi_destroy_batch": [vp],
        "abi_chebfi_solve": [vp, vp, c_int64, c_int64, c_int32, vp, c_int32, c_int32, c_int32,
                             c_double, c_int32, vp, vp, vp, vp],
        "abi_apply_S": [vp, vp, vp, c_int64, c_int64, c_int32, vp],
        "abi_apply_Sinv": [vp, vp, vp, c_int64, c_int64, c_int32, vp],
        "abi_overlap_info": [vp, POINTER(c_int32), POINTER(c_double)],
        "abi_lobpcg_solve": [vp, vp, c_int64, c_int64, c_int32, c_int32, c_int32, c_int32,
                             c_int32, c_double, vp, vp, vp, vp],
        "abi_density_add": [vp, vp, c_int64, c_int64, c_int32, vp, vp, vp],
        "abi_occupations": [c_int64, vp, c_double, c_double, c_double, vp, vp],
        "abi_scf_potential": [vp, vp, vp, vp, vp],
        "abi_get_potential": [vp, vp, vp],
        "abi_scf_solve": [vp, vp, c_int64, c_int64, c_int32, vp, vp, c_double, c_double, c_double,
                          c_double, c_int32, c_int32, c_int32, c_double, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = c_int32
    L.abi_last_error.argtypes = []
    L.abi_last_error.restype = c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc != ABI_OK:
        raise ChebfiError(rc, lib().abi_last_error().decode(errors="replace"))


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _block(t, npw: int):
    """(pointer, nband, ld, dtype code) of a (nband, npw) complex CUDA tensor."""
    import torch
    if t.dtype == torch.complex128:
        code = ABI_C128
    elif t.dtype == torch.complex64:
        code = ABI_C64
    else:
        raise TypeError("blocks must be complex128 or complex64 tensors")
    if not t.is_cuda:
        raise TypeError("blocks must live on the GPU")
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.shape[1] != npw or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError("block must be (nband, npw) with unit stride along plane waves")
    ld = int(t.stride(0)) if t.shape[0] > 1 else npw  # a one-row stride is arbitrary
    if ld < npw:
        raise ValueError("block rows overlap (stride(0) < npw)")
    return c_void_p(t.data_ptr()), int(t.shape[0]), ld, code


class _DescHolder:
    """Keeps the numpy arrays referenced by a Desc alive."""

    def __init__(self, lattice, kpt_red, ecut, ngrid, vloc, tau, dij, rc, precision, qij=None):
        self.vloc = np.ascontiguousarray(np.asarray(vloc, dtype=np.float64).reshape(-1))
        self.tau = np.ascontiguousarray(np.asarray(tau, dtype=np.float64).reshape(-1, 3))
        d = np.ascontiguousarray(np.asarray(dij, dtype=np.complex128).reshape(-1, 4, 4))
        self.dij = np.ascontiguousarray(d.view(np.float64).reshape(-1))
        self.desc = Desc()
        self.desc.abi_version = 1
        lat = np.asarray(lattice, dtype=np.float64).reshape(-1)
        for i in range(9):
            self.desc.lattice[i] = float(lat[i])
        for i in range(3):
            self.desc.kpt_red[i] = float(kpt_red[i])
            self.desc.ngrid[i] = int(ngrid[i])
        self.desc.ecut = float(ecut)
        self.desc.vloc = self.vloc.ctypes.data_as(POINTER(c_double))
        self.desc.natom = int(self.tau.shape[0])
        self.desc.tau_cart = self.tau.ctypes.data_as(POINTER(c_double))
        self.desc.rc = float(rc)
        self.desc.dij = self.dij.ctypes.data_as(POINTER(c_double))
        self.desc.precision = int(precision)
        self.qij = None
        if qij is not None:
            q = np.ascontiguousarray(np.asarray(qij, dtype=np.complex128).reshape(-1, 4, 4))
            if q.shape[0] != self.desc.natom:
                raise ValueError("qij needs one 4x4 matrix per atom")
            self.qij = np.ascontiguousarray(q.view(np.float64).reshape(-1))
            self.desc.abi_version = 2
            self.desc.qij = self.qij.ctypes.data_as(POINTER(c_double))

    @classmethod
    def from_system(cls, s, precision=ABI_PREC_FP64):
        return cls(s.lattice, s.kpt_red, s.ecut, s.ngrid, s.vloc, s.tau, s.dij, s.rc, precision,
                   getattr(s, "qij", None))


def gsphere_host(s):
    """Host-only basis build: (miller (npw,3) int32, box_index (npw,) int32, kinetic)."""
    h = _DescHolder.from_system(s)
    n = c_int64(0)
    _check(lib().abi_gsphere_count(ctypes.byref(h.desc), ctypes.byref(n)))
    npw = n.value
    miller = np.zeros((npw, 3), dtype=np.int32)
    box = np.zeros(npw, dtype=np.int32)
    kin = np.zeros(npw, dtype=np.float64)
    _check(lib().abi_gsphere_build(ctypes.byref(h.desc), npw, miller.ctypes.data_as(c_void_p),
                                   box.ctypes.data_as(c_void_p), kin.ctypes.data_as(c_void_p)))
    return miller, box, kin


class System:
    """One Hamiltonian resident on the current GPU."""

    def __init__(self, s, precision=ABI_PREC_FP64):
        h = _DescHolder.from_system(s, precision)
        handle = c_void_p()
        _check(lib().abi_set_system(ctypes.byref(h.desc), _stream(), ctypes.byref(handle)))
        self._h = handle
        self._own = True
        self._info()

    @classmethod
    def _borrow(cls, handle, owner):
        """A view of a handle owned by `owner` (a Batch): never destroyed here."""
        obj = cls.__new__(cls)
        obj._h = handle
        obj._own = False
        obj._owner = owner
        obj._info()
        return obj

    def _info(self):
        npw = c_int64(0)
        nproj = c_int32(0)
        grid = (c_int32 * 3)()
        _check(lib().abi_system_info(self._h, ctypes.byref(npw), ctypes.byref(nproj), grid))
        self.npw = npw.value
        self.nproj = nproj.value
        self.ngrid = tuple(grid)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and self._own:
            _check(lib().abi_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- tables ------------------------------------------------------------
    def gsphere(self):
        miller = np.zeros((self.npw, 3), dtype=np.int32)
        box = np.zeros(self.npw, dtype=np.int32)
        _check(lib().abi_get_gsphere(self._h, miller.ctypes.data_as(c_void_p),
                                     box.ctypes.data_as(c_void_p)))
        return miller, box

    def projectors(self):
        import torch
        P = torch.empty((self.nproj, self.npw), dtype=torch.complex128, device="cuda")
        _check(lib().abi_get_projectors(self._h, c_void_p(P.data_ptr()), _stream()))
        return P  # row j = projector column j

    # -- hot path ------------------------------------------------------------
    def _out_like(self, X, out):
        import torch
        if out is None:
            out = torch.empty_strided(X.shape, X.stride(), dtype=X.dtype, device=X.device)
        if out.dtype != X.dtype or out.shape != X.shape or (X.dim() == 2 and X.shape[0] > 1
                                                             and out.stride() != X.stride()):
            raise ValueError("out must match X's dtype, shape and stride")
        return out

    def apply_H(self, X, out=None):
        px, nb, ld, code = _block(X, self.npw)
        out = self._out_like(X, out)
        po, _, _, _ = _block(out, self.npw)
        _check(lib().abi_apply_H(self._h, px, po, nb, ld, code, _stream()))
        return out

    def apply_H_noalloc(self, X, out):
        """H X into the preallocated `out` through the entry point that allocates
        nothing (work buffers in the library's per-device scratch array)."""
        px, nb, ld, code = _block(X, self.npw)
        po, nbo, ldo, codeo = _block(out, self.npw)
        if (nbo, ldo, codeo) != (nb, ld, code):
            raise ValueError("out must match X in bands, stride and dtype")
        _check(lib().abi_apply_H_noalloc(self._h, px, po, nb, ld, code, _stream()))
        return out

    def apply_S(self, X, out=None):
        px, nb, ld, code = _block(X, self.npw)
        out = self._out_like(X, out)
        po, _, _, _ = _block(out, self.npw)
        _check(lib().abi_apply_S(self._h, px, po, nb, ld, code, _stream()))
        return out

    def apply_Sinv(self, X, out=None):
        px, nb, ld, code = _block(X, self.npw)
        out = self._out_like(X, out)
        po, _, _, _ = _block(out, self.npw)
        _check(lib().abi_apply_Sinv(self._h, px, po, nb, ld, code, _stream()))
        return out

    def overlap_info(self):
        """(has_overlap, smallest eigenvalue of S)."""
        h = c_int32(0)
        m = c_double(0.0)
        _check(lib().abi_overlap_info(self._h, ctypes.byref(h), ctypes.byref(m)))
        return bool(h.value), float(m.value)

    def cheb_filter(self, X, degree, a, b, a0, out=None, hx=None):
        """Degree-m filter of X; hx: H X of the same shape and dtype (its first
        step then reuses it instead of applying H)."""
        px, nb, ld, code = _block(X, self.npw)
        out = self._out_like(X, out)
        po, _, _, _ = _block(out, self.npw)
        if hx is None:
            _check(lib().abi_cheb_filter(self._h, px, po, nb, ld, code, int(degree), float(a),
                                         float(b), float(a0), _stream()))
        else:
            self._out_like(X, hx)  # same shape, dtype and layout as X
            ph, _, _, _ = _block(hx, self.npw)
            _check(lib().abi_cheb_filter_hx(self._h, px, ph, po, nb, ld, code, int(degree),
                                            float(a), float(b), float(a0), _stream()))
        return out

    def spectral_bounds(self, X, v0, nlanczos=10):
        """(a, b, a0); v0 must be complex128 (the Lanczos run is FP64)."""
        px, nb, ld, code = _block(X, self.npw)
        pv, _, _, vcode = _block(v0, self.npw)
        if vcode != ABI_C128:
            raise TypeError("v0 must be complex128")
        out = (c_double * 3)()
        _check(lib().abi_spectral_bounds(self._h, px, nb, ld, code, pv, int(nlanczos), out,
                                         _stream()))
        return float(out[0]), float(out[1]), float(out[2])

    def update_potential(self, vloc=None, dij=None):
        """Replace V_loc (float64, n1*n2*n3, i1 fastest) and/or D (complex128 (natom,4,4))."""
        import torch
        pv = c_void_p(0)
        pd = c_void_p(0)
        keep = []
        if vloc is not None:
            v = vloc.detach().to(device="cuda", dtype=torch.float64).contiguous().reshape(-1)
            if v.numel() != self.ngrid[0] * self.ngrid[1] * self.ngrid[2]:
                raise ValueError("vloc has the wrong size")
            keep.append(v)
            pv = c_void_p(v.data_ptr())
        if dij is not None:
            d = dij.detach().to(device="cuda", dtype=torch.complex128).contiguous()
            if d.numel() != 4 * self.nproj:
                raise ValueError("dij has the wrong size")
            keep.append(d)
            pd = c_void_p(d.data_ptr())
        _check(lib().abi_update_potential(self._h, pv, pd, _stream()))
        torch.cuda.current_stream().synchronize()

    def filter_backward(self, X, W, degree, a, b, a0, ckpt_every=4, want_dx=True):
        """(dV, dD, dX) of L = sum_n Re<W_n, filter(X)_n> (dX None unless want_dx)."""
        import torch
        px, nb, ld, code = _block(X, self.npw)
        self._out_like(X, W)
        pw, _, _, _ = _block(W, self.npw)
        n3 = self.ngrid[0] * self.ngrid[1] * self.ngrid[2]
        dV = torch.empty(n3, dtype=torch.float64, device=X.device)
        dD = torch.empty((max(self.nproj // 4, 1), 4, 4), dtype=torch.complex128, device=X.device)
        dX = None
        pdx = c_void_p(0)
        if want_dx:
            dX = self._out_like(X, None)
            pdx = c_void_p(dX.data_ptr())
        _check(lib().abi_filter_backward(self._h, px, pw, nb, ld, code, int(degree), float(a),
                                         float(b), float(a0), int(ckpt_every),
                                         c_void_p(dV.data_ptr()), c_void_p(dD.data_ptr()), pdx,
                                         _stream()))
        return dV, dD[: self.nproj // 4], dX

    def density(self, Psi, weights=None):
        """rho(r) = sum_n w_n |psi~_n(r)|^2 / n^3 (float64, n1*n2*n3, i1 fastest)."""
        import torch
        pp, nb, ld, code = _block(Psi, self.npw)
        rho = torch.empty(self.ngrid[0] * self.ngrid[1] * self.ngrid[2], dtype=torch.float64,
                          device=Psi.device)
        pw = c_void_p(0)
        w = None
        if weights is not None:
            w = torch.as_tensor(weights, dtype=torch.float64, device=Psi.device).contiguous()
            if w.numel() != nb:
                raise ValueError("weights must have nband entries")
            pw = c_void_p(w.data_ptr())
        _check(lib().abi_density(self._h, pp, nb, ld, code, pw, c_void_p(rho.data_ptr()),
                                 _stream()))
        return rho

    def density_add(self, Psi, rho, weights=None):
        """rho += sum_n w_n |psi~_n(r)|^2 / n^3 (rho: float64 CUDA tensor of n1*n2*n3)."""
        import torch
        pp, nb, ld, code = _block(Psi, self.npw)
        pw = c_void_p(0)
        w = None
        if weights is not None:
            w = torch.as_tensor(weights, dtype=torch.float64, device=Psi.device).contiguous()
            pw = c_void_p(w.data_ptr())
        _check(lib().abi_density_add(self._h, pp, nb, ld, code, pw, c_void_p(rho.data_ptr()),
                                     _stream()))
        return rho

    def potential(self):
        """The handle's V_loc (float64 CUDA tensor, n1*n2*n3, i1 fastest)."""
        import torch
        v = torch.empty(self.ngrid[0] * self.ngrid[1] * self.ngrid[2], dtype=torch.float64,
                        device="cuda")
        _check(lib().abi_get_potential(self._h, c_void_p(v.data_ptr()), _stream()))
        return v

    def scf_potential(self, rho, vion):
        """V_ion + V_H[rho] + v_x[rho] on the grid (float64 CUDA tensors)."""
        import torch
        rho = rho.contiguous()
        vion = vion.contiguous()
        vout = torch.empty_like(rho)
        _check(lib().abi_scf_potential(self._h, c_void_p(rho.data_ptr()),
                                       c_void_p(vion.data_ptr()), c_void_p(vout.data_ptr()),
                                       _stream()))
        return vout

    def scf(self, X, v0, vion, nelec, kT, alpha, degree, cycles_per_iter, max_iter, tol, q0=0.0):
        """SCF iterations in place on X and on the handle's V_loc.  Returns
        (eval, rho, dv, info dict)."""
        import torch
        px, nb, ld, code = _block(X, self.npw)
        pv, _, _, _ = _block(v0.reshape(1, -1) if v0.dim() == 1 else v0, self.npw)
        vion = vion.contiguous()
        rho = torch.empty(self.ngrid[0] * self.ngrid[1] * self.ngrid[2], dtype=torch.float64,
                          device=X.device)
        ev = np.zeros(nb)
        dv = c_double(0.0)
        info = np.zeros(4, dtype=np.int32)
        _check(lib().abi_scf_solve(self._h, px, nb, ld, code, pv, c_void_p(vion.data_ptr()),
                                   float(nelec), float(kT), float(alpha), float(q0), int(degree),
                                   int(cycles_per_iter), int(max_iter), float(tol),
                                   ev.ctypes.data_as(c_void_p), c_void_p(rho.data_ptr()),
                                   ctypes.byref(dv), info.ctypes.data_as(c_void_p), _stream()))
        return ev, rho, float(dv.value), {"iterations": int(info[0]),
                                          "converged": bool(info[1])}

    def solve(self, X, v0, degree, max_cycles, nconv, tol, refine_degree=0):
        """In place: X <- Ritz vectors after cycles of bounds, filter and
        Rayleigh-Ritz until the lowest nconv residuals are <= tol.  Returns
        (eval, resnorm, info dict)."""
        px, nb, ld, code = _block(X, self.npw)
        pv, _, _, vcode = _block(v0.reshape(1, -1) if v0.dim() == 1 else v0, self.npw)
        if vcode != ABI_C128:
            raise TypeError("v0 must be complex128")
        ev = np.zeros(nb)
        res = np.zeros(nb)
        info = np.zeros(4, dtype=np.int32)
        _check(lib().abi_chebfi_solve(self._h, px, nb, ld, code, pv, int(degree), int(max_cycles),
                                      int(nconv), float(tol), int(refine_degree),
                                      ev.ctypes.data_as(c_void_p), res.ctypes.data_as(c_void_p),
                                      info.ctypes.data_as(c_void_p), _stream()))
        return ev, res, {"cycles": int(info[0]), "refine_cycles": int(info[1]),
                         "converged": bool(info[2])}

    def lobpcg(self, X, nblocks, nline, max_passes=1, nconv=None, tol=0.0):
        """In place: X <- Ritz vectors after passes of block LOBPCG (complex128).
        Returns (eval, resnorm, info dict)."""
        px, nb, ld, code = _block(X, self.npw)
        nconv = nb if nconv is None else int(nconv)
        ev = np.zeros(nb)
        res = np.zeros(nb)
        info = np.zeros(4, dtype=np.int32)
        _check(lib().abi_lobpcg_solve(self._h, px, nb, ld, code, int(nblocks), int(nline),
                                      int(max_passes), nconv, float(tol),
                                      ev.ctypes.data_as(c_void_p), res.ctypes.data_as(c_void_p),
                                      info.ctypes.data_as(c_void_p), _stream()))
        return ev, res, {"passes": int(info[0]), "line_steps": int(info[1]),
                         "converged": bool(info[2])}

    def profile(self, on=True):
        _check(lib().abi_profile_enable(self._h, 1 if on else 0))

    def set_tuning(self, param, value):
        """Sets one launch choice (TUNE_* parameter) of this handle."""
        _check(lib().abi_set_tuning(self._h, int(param), int(value)))

    def autotune(self, X, cache_path=None):
        """Times the launch choices on H applications of X and keeps the fastest
        (looked up in / stored to the cache file, if any).  Returns
        ({param: value}, from_cache)."""
        px, nb, ld, code = _block(X, self.npw)
        fc = c_int32(0)
        cp = None if cache_path is None else str(cache_path).encode()
        _check(lib().abi_autotune(self._h, px, nb, ld, code, cp, ctypes.byref(fc), _stream()))
        names = {"proj": TUNE_PROJ, "expand": TUNE_EXPAND, "fft_batch": TUNE_FFT_BATCH,
                 "overlap": TUNE_OVERLAP}
        return {k: self.get_tuning(v) for k, v in names.items()}, bool(fc.value)

    def get_tuning(self, param):
        v = c_int32(0)
        _check(lib().abi_get_tuning(self._h, int(param), ctypes.byref(v)))
        return v.value

    def profile_read(self):
        """{class: (total_ms, work, count)} for the launches timed so far."""
        n = len(PROFILE_CLASSES)
        ms = np.zeros(n)
        wk = np.zeros(n)
        ct = np.zeros(n, dtype=np.int64)
        _check(lib().abi_profile_read(self._h, n, ms.ctypes.data_as(c_void_p),
                                      wk.ctypes.data_as(c_void_p), ct.ctypes.data_as(c_void_p)))
        return {c: (float(ms[i]), float(wk[i]), int(ct[i])) for i, c in enumerate(PROFILE_CLASSES)}

    def rayleigh_ritz(self, Y, hpsi=None, want_coef=False, lowprec=False):
        """In place: Y <- Ritz vectors.  Returns (eval, resnorm, flags) and, with
        want_coef, the coefficient matrix C (torch (nband, nband), Psi = Y_in C).
        lowprec: the split-BF16 form for a complex64 block (RR_LOWPREC in flags
        when it ran, with RR_TWO_PASS when it orthonormalised first;
        RR_FELL_BACK when the FP64 form ran instead)."""
        import torch
        py, nb, ld, code = _block(Y, self.npw)
        ph = c_void_p(0)
        if hpsi is not None:
            self._out_like(Y, hpsi)
            ph, _, _, _ = _block(hpsi, self.npw)
        ev = np.zeros(nb, dtype=np.float64)
        rn = np.zeros(nb, dtype=np.float64)
        fl = c_int32(RR_LOWPREC if lowprec else 0)
        coef = None
        pc = c_void_p(0)
        if want_coef:
            coef = torch.empty((nb, nb), dtype=torch.complex128, device=Y.device)
            pc = c_void_p(coef.data_ptr())
        _check(lib().abi_rayleigh_ritz(self._h, py, ph, nb, ld, code, ev.ctypes.data_as(c_void_p),
                                       rn.ctypes.data_as(c_void_p), pc, ctypes.byref(fl),
                                       _stream()))
        if want_coef:
            return ev, rn, fl.value, coef.t()  # stored column-major
        return ev, rn, fl.value


def occupations(eval, nelec, kT, occ_max=2.0):
    """(f, mu): Fermi-Dirac occupations with sum f = nelec (host computation)."""
    e = np.ascontiguousarray(np.asarray(eval, dtype=np.float64))
    f = np.zeros_like(e)
    mu = c_double(0.0)
    _check(lib().abi_occupations(e.size, e.ctypes.data_as(c_void_p), float(nelec), float(kT),
                                 float(occ_max), f.ctypes.data_as(c_void_p), ctypes.byref(mu)))
    return f, float(mu.value)


# -- dense building blocks (matrices as torch (m, m) tensors, math layout) ------
def zpotrf_upper(A):
    """Upper Cholesky factor U (A = U^H U) of a Hermitian positive definite matrix."""
    m = A.shape[0]
    cm = A.t().contiguous()  # column-major storage
    _check(lib().abi_zpotrf_upper(m, c_void_p(cm.data_ptr()), m, _stream()))
    return cm.t()


def zheev(A):
    """(w ascending, Z) with A = Z diag(w) Z^H for a Hermitian matrix."""
    import torch
    m = A.shape[0]
    cm = A.t().contiguous()
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    Z = torch.empty((m, m), dtype=torch.complex128, device=A.device)
    _check(lib().abi_zheev(m, c_void_p(cm.data_ptr()), m, c_void_p(w.data_ptr()),
                           c_void_p(Z.data_ptr()), m, _stream()))
    return w, Z.t()


class Batch:
    """Many independent systems filtered together (abi_cheb_filter_batch)."""

    def __init__(self, systems, precision=ABI_PREC_MIXED):
        holders = [_DescHolder.from_system(s, precision) for s in systems]
        n = len(holders)
        arr = (Desc * n)(*[h.desc for h in holders])
        handle = c_void_p()
        _check(lib().abi_set_system_batch(ctypes.cast(arr, c_void_p), n, _stream(),
                                          ctypes.byref(handle)))
        self._h = handle
        self.systems = []
        for i in range(n):
            hi = c_void_p()
            _check(lib().abi_batch_system(self._h, i, ctypes.byref(hi)))
            self.systems.append(System._borrow(hi, self))

    def __len__(self):
        return len(self.systems)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            for s in self.systems:
                s._h = None
            _check(lib().abi_destroy_batch(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _args(self, Xs, out, bounds):
        n = len(self.systems)
        if len(Xs) != n or len(bounds) != n:
            raise ValueError("one block and one (a, b, a0) per system")
        if out is None:
            out = [self.systems[i]._out_like(Xs[i], None) for i in range(n)]
        xs, ys = (c_void_p * n)(), (c_void_p * n)()
        nb, ld = (c_int64 * n)(), (c_int64 * n)()
        a, b, a0 = (c_double * n)(), (c_double * n)(), (c_double * n)()
        code = None
        for i in range(n):
            px, nbi, ldi, ci = _block(Xs[i], self.systems[i].npw)
            self.systems[i]._out_like(Xs[i], out[i])
            py, _, _, _ = _block(out[i], self.systems[i].npw)
            if code is None:
                code = ci
            elif ci != code:
                raise TypeError("all blocks of a batch must share one dtype")
            xs[i], ys[i], nb[i], ld[i] = px, py, nbi, ldi
            a[i], b[i], a0[i] = (float(v) for v in bounds[i])
        return out, (xs, ys, nb, ld, code, a, b, a0)

    def cheb_filter(self, Xs, degree, bounds, out=None):
        """[Y_i] = degree-m filters of the blocks [X_i] with bounds [(a, b, a0)_i]."""
        out, (xs, ys, nb, ld, code, a, b, a0) = self._args(Xs, out, bounds)
        _check(lib().abi_cheb_filter_batch(self._h, ctypes.cast(xs, c_void_p),
                                           ctypes.cast(ys, c_void_p), ctypes.cast(nb, c_void_p),
                                           ctypes.cast(ld, c_void_p), code, int(degree),
                                           ctypes.cast(a, c_void_p), ctypes.cast(b, c_void_p),
                                           ctypes.cast(a0, c_void_p), _stream()))
        return out

    def autotune(self, Xs, degree, bounds, out=None):
        """Times the launch variants on these arguments and keeps the fastest."""
        out, (xs, ys, nb, ld, code, a, b, a0) = self._args(Xs, out, bounds)
        ch = (c_int32 * 4)()
        _check(lib().abi_batch_autotune(self._h, ctypes.cast(xs, c_void_p),
                                        ctypes.cast(ys, c_void_p), ctypes.cast(nb, c_void_p),
                                        ctypes.cast(ld, c_void_p), code, int(degree),
                                        ctypes.cast(a, c_void_p), ctypes.cast(b, c_void_p),
                                        ctypes.cast(a0, c_void_p), ctypes.cast(ch, c_void_p),
                                        _stream()))
        return {"fft_threads": ch[0], "proj_threads": ch[1], "radix_descending": bool(ch[2]),
                "variants_timed": ch[3]}

    def use_graph(self, on=True):
        _check(lib().abi_batch_use_graph(self._h, 1 if on else 0))

    def use_overlap(self, on=True):
        _check(lib().abi_batch_use_overlap(self._h, 1 if on else 0))


def _make_autograd():
    import torch

    class ChebFilterFunction(torch.autograd.Function):
        """Y = p(H[vloc, dij]) X with the library's adjoint as its backward.

        Inputs X (complex128 (nband, npw), or complex64 on a mixed-precision
        handle), vloc (float64, n1*n2*n3) and dij (complex128 (natom, 4, 4))
        are differentiable; the bounds are constants.
        """

        @staticmethod
        def forward(ctx, X, vloc, dij, system, degree, a, b, a0, ckpt_every):
            system.update_potential(vloc, dij)
            Y = system.cheb_filter(X.detach(), degree, a, b, a0)
            ctx.save_for_backward(X.detach(), vloc.detach(), dij.detach())
            ctx.system = system
            ctx.params = (degree, a, b, a0, ckpt_every)
            return Y

        @staticmethod
        def backward(ctx, gY):
            X, vloc, dij = ctx.saved_tensors
            degree, a, b, a0, ckpt = ctx.params
            ctx.system.update_potential(vloc, dij)
            dV, dD, dX = ctx.system.filter_backward(X, gY.contiguous(), degree, a, b, a0, ckpt,
                                                    want_dx=ctx.needs_input_grad[0])
            return (dX, dV.reshape(vloc.shape), dD.reshape(dij.shape), None, None, None, None,
                    None, None)

    return ChebFilterFunction


_autograd_fn = None


def cheb_filter_autograd(X, vloc, dij, system, degree, a, b, a0, ckpt_every=4):
    """Differentiable Chebyshev filter (torch.autograd.Function over the C ABI)."""
    global _autograd_fn
    if _autograd_fn is None:
        _autograd_fn = _make_autograd()
    return _autograd_fn.apply(X, vloc, dij, system, degree, a, b, a0, ckpt_every)
