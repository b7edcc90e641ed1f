// Block LOBPCG, the solver the paper compares the Chebyshev filter with
// (Algorithm "Parallel LOBPCG with b blocks and k line minimizations"), on the
// kernels of the hot path: H and S applications, FP64 Gram GEMMs, Cholesky,
// triangular inverse, the Hermitian eigensolver and FP64 rotations.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cplx.h"
#include "driver.h"
#include "kernels.h"

namespace chebfi {
namespace {

// S-ortho + Rayleigh-Ritz of a basis Z (npw x k, ld): Z^H S Z = U^H U,
// U^-H (Z^H H Z) U^-1 = Y diag(w) Y^H, C = U^-1 Y[:, :mout] (k x mout, ld k), w on the
// device (k values, ascending).  Returns false, with nothing else written, when the
// Gram is not positive definite.
bool ortho_rr_basis(abi_system_s *s, int64_t k, int64_t mout, const double2 *Z,
                    const double2 *HZ, const double2 *SZ, int64_t ld, double *w_dev, double2 *C,
                    hipStream_t st) {
  const int64_t npw = s->npw;
  const size_t kk = sizeof(double2) * (size_t)k * k;
  double2 *G = (double2 *)s->small1.get(kk);
  double2 *Hs = (double2 *)s->small2.get(kk);
  double2 *T = (double2 *)s->small3.get(kk);
  double2 *Y = (double2 *)s->small4.get(kk);
  int *info = (int *)s->lob_g.get(sizeof(double2) * 16);
  // Z^H S Z and Z^H H Z are Hermitian: only the upper tiles are formed
  const int splits = zgemm_herm_splits(k, npw);
  const double gflops = 8.0 * (double)k * k * npw;
  void *part = s->cpart.get(sizeof(double2) * (size_t)splits * k * k);
  int tok = s->prof.begin(PROF_GRAM, gflops, st);
  zgemm_herm(k, npw, Z, ld, SZ, ld, G, k, st, part, splits);
  s->prof.end(tok, st);
  launch_hermitize(k, G, k, st);
  tok = s->prof.begin(PROF_CHOL, 4.0 / 3.0 * (double)k * k * k, st);
  zpotrf_upper(k, G, k, info, nullptr, st);
  s->prof.end(tok, st);
  int h = 0;
  CHEBFI_HIP(hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, st));
  CHEBFI_HIP(hipStreamSynchronize(st));
  if (h != 0) return false;
  tok = s->prof.begin(PROF_GRAM, gflops, st);
  zgemm_herm(k, npw, Z, ld, HZ, ld, Hs, k, st, part, splits);
  s->prof.end(tok, st);
  launch_hermitize(k, Hs, k, st);
  tok = s->prof.begin(PROF_CHOL, 16.0 * (double)k * k * k, st);
  ztrtri_upper(k, G, k, s->eig2.get(ztrtri_work_bytes(k)), st);
  zgemm(OP_N, OP_N, k, k, k, Hs, k, G, k, T, k, double2{1, 0}, double2{0, 0}, st);
  zgemm(OP_C, OP_N, k, k, k, G, k, T, k, Hs, k, double2{1, 0}, double2{0, 0}, st);
  s->prof.end(tok, st);
  tok = s->prof.begin(PROF_EIG, 16.0 / 3.0 * (double)k * k * k, st);
  zheev(k, Hs, k, w_dev, Y, k, s->eig1.get(zheev_work_bytes(k)), st);
  s->prof.end(tok, st);
  zgemm(OP_N, OP_N, k, mout, k, G, k, Y, k, C, k, double2{1, 0}, double2{0, 0}, st);
  return true;
}

// X <- X - Q (Q^H S X) for the S-orthonormal bands Q (npw x nq) and a block X
// (npw x m); SX is work space that receives S X first (unused when S = I).
void s_deflate(abi_system_s *s, const double2 *Q, int64_t nq, double2 *X, double2 *SX, int64_t m,
               hipStream_t st) {
  const int64_t npw = s->npw;
  if (nq == 0) return;
  const double2 *sx = X;
  if (s->has_S) {
    apply_S(s, X, npw, SX, npw, m, st);
    sx = SX;
  }
  double2 *G = (double2 *)s->lob_g.get(sizeof(double2) * (size_t)nq * m);
  const int splits = zgemm_splits(nq, m, npw);
  void *part = s->cpart.get(sizeof(double2) * (size_t)splits * nq * m);
  zgemm(OP_C, OP_N, nq, m, npw, Q, npw, sx, npw, nullptr, 0, double2{1, 0}, double2{0, 0}, st,
        part, splits);
  zsum_parts(nq, m, part, splits, G, nq, double2{1, 0}, double2{0, 0}, st);
  zgemm(OP_N, OP_N, npw, m, nq, Q, npw, G, nq, X, npw, double2{-1, 0}, double2{1, 0}, st);
}

}  // namespace

// One pass of block LOBPCG (Algorithm "Parallel LOBPCG with b blocks and k line
// minimizations") on the block Psi (npw x M, ld), in place; returns the Ritz values and
// residual norms ||H psi - lambda S psi|| (host arrays of M) and the line minimisations
// each block ran.  FP64 throughout.
void lobpcg_pass_core(abi_system_s *s, double2 *Psi_io, int64_t ldio, int64_t M, int nblocks,
                      int nline, double tol, double *eval, double *res, int *steps,
                      hipStream_t st) {
  const int64_t npw = s->npw, m = M / nblocks;
  const bool gen = s->has_S;
  const size_t col = sizeof(double2) * (size_t)npw;
  double2 *Psi = (double2 *)s->lob_psi.get(col * M);
  double2 *HPsi = (double2 *)s->lob_hp.get(col * M);
  double2 *SPsi = gen ? (double2 *)s->lob_sp.get(col * M) : Psi;
  double2 *Z = (double2 *)s->lob_z.get(col * 3 * m);  // [X | W | P]
  double2 *HZ = (double2 *)s->lob_hz.get(col * 3 * m);
  double2 *SZ = gen ? (double2 *)s->lob_sz.get(col * 3 * m) : Z;
  double2 *T1 = (double2 *)s->lob_t1.get(col * m);
  double2 *T2 = (double2 *)s->lob_t2.get(col * m);
  double2 *C = (double2 *)s->lob_c.get(sizeof(double2) * (size_t)std::max(3 * m * m, M * M));
  // w: Ritz values of the last Rayleigh-Ritz (up to max(3m, M)), lam: current block's,
  // resd: residual norms
  double *w = (double *)s->lob_v.get(sizeof(double) * (size_t)(3 * M + 3 * m + 64));
  double *lam = w + std::max(3 * m, M);
  double *resd = lam + M;
  launch_copy_block(npw, M, Psi_io, ldio, Psi, npw, st);
  const size_t blk = (size_t)npw * m;
  std::vector<double> hres(M);
  auto rotate = [&](double2 *A, int64_t k) {
    // P <- A[:, m:k] C[m:k, :], X <- A[:, 0:k] C
    zgemm(OP_N, OP_N, npw, m, k - m, A + blk, npw, C + m, k, T1, npw, double2{1, 0},
          double2{0, 0}, st);
    zgemm(OP_N, OP_N, npw, m, k, A, npw, C, k, T2, npw, double2{1, 0}, double2{0, 0}, st);
    launch_copy_block(npw, m, T2, npw, A, npw, st);
    launch_copy_block(npw, m, T1, npw, A + 2 * blk, npw, st);
  };
  for (int i = 0; i < nblocks; ++i) {
    double2 *X = Z, *HX = HZ, *SX = SZ;
    double2 *W = Z + blk, *HW = HZ + blk, *SW = SZ + blk;
    double2 *P = Z + 2 * blk, *HP = HZ + 2 * blk, *SP = SZ + 2 * blk;
    launch_copy_block(npw, m, Psi + (size_t)i * blk, npw, X, npw, st);
    s_deflate(s, Psi, (int64_t)i * m, X, SX, m, st);
    apply_core(s, X, npw, nullptr, 0, HX, npw, m, 1.0, 0.0, 0.0, st);
    if (gen) apply_S(s, X, npw, SX, npw, m, st);
    if (!ortho_rr_basis(s, m, m, X, HX, SX, npw, w, C, st))
      throw Error{ABI_ERR_NOT_HPD, "LOBPCG: block Gram matrix not positive definite"};
    // X, HX (, SX) <- (.) C
    double2 *rot1[3] = {X, HX, SX};
    for (int r = 0; r < (gen ? 3 : 2); ++r) {
      zgemm(OP_N, OP_N, npw, m, m, rot1[r], npw, C, m, T2, npw, double2{1, 0}, double2{0, 0}, st);
      launch_copy_block(npw, m, T2, npw, rot1[r], npw, st);
    }
    CHEBFI_HIP(hipMemcpyAsync(lam, w, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    bool have_p = false;
    int done = 0;
    for (int n = 0; n < nline; ++n) {
      launch_resid_block(npw, m, HX, SX, npw, lam, W, npw, resd, st);
      CHEBFI_HIP(hipMemcpyAsync(hres.data(), resd, sizeof(double) * m, hipMemcpyDeviceToHost, st));
      CHEBFI_HIP(hipStreamSynchronize(st));
      double worst = 0.0;
      for (int64_t j = 0; j < m; ++j) worst = std::max(worst, hres[j]);
      if (worst <= tol) break;
      launch_tpa(npw, m, s->d_kin, X, npw, W, npw, st);
      s_deflate(s, Psi, (int64_t)i * m, W, SW, m, st);
      apply_core(s, W, npw, nullptr, 0, HW, npw, m, 1.0, 0.0, 0.0, st);
      if (gen) apply_S(s, W, npw, SW, npw, m, st);
      launch_snorm_scale(npw, m, W, HW, gen ? SW : nullptr, npw, st);
      int64_t k = 0;
      if (have_p) {
        launch_snorm_scale(npw, m, P, HP, gen ? SP : nullptr, npw, st);
        if (ortho_rr_basis(s, 3 * m, m, Z, HZ, SZ, npw, w, C, st)) k = 3 * m;
      }
      if (k == 0) {
        if (!ortho_rr_basis(s, 2 * m, m, Z, HZ, SZ, npw, w, C, st))
          throw Error{ABI_ERR_NOT_HPD, "LOBPCG: Gram matrix of [Psi, W] not positive definite"};
        k = 2 * m;
      }
      const int tok = s->prof.begin(PROF_ROT, 8.0 * (double)npw * m * (2 * k - m) * (gen ? 3 : 2),
                                    st);
      rotate(Z, k);
      rotate(HZ, k);
      if (gen) rotate(SZ, k);
      s->prof.end(tok, st);
      CHEBFI_HIP(hipMemcpyAsync(lam, w, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
      have_p = true;
      ++done;
    }
    launch_copy_block(npw, m, X, npw, Psi + (size_t)i * blk, npw, st);
    launch_copy_block(npw, m, HX, npw, HPsi + (size_t)i * blk, npw, st);
    if (gen) launch_copy_block(npw, m, SX, npw, SPsi + (size_t)i * blk, npw, st);
    if (steps) steps[i] = done;
  }
  double2 *Wres = (double2 *)s->lob_t3.get(col * M);
  if (nblocks > 1) {
    // global S-ortho + Rayleigh-Ritz of all M bands
    double2 *CM = (double2 *)s->lob_c.get(sizeof(double2) * (size_t)std::max(3 * m * m, M * M));
    if (!ortho_rr_basis(s, M, M, Psi, HPsi, SPsi, npw, w, CM, st))
      throw Error{ABI_ERR_NOT_HPD, "LOBPCG: global Gram matrix not positive definite"};
    double2 *rot2[3] = {Psi, HPsi, SPsi};
    for (int r = 0; r < (gen ? 3 : 2); ++r) {
      zgemm(OP_N, OP_N, npw, M, M, rot2[r], npw, CM, M, Wres, npw, double2{1, 0}, double2{0, 0},
            st);
      launch_copy_block(npw, M, Wres, npw, rot2[r], npw, st);
    }
    CHEBFI_HIP(hipMemcpyAsync(lam, w, sizeof(double) * M, hipMemcpyDeviceToDevice, st));
  }
  launch_resid_block(npw, M, HPsi, SPsi, npw, lam, Wres, npw, resd, st);
  launch_copy_block(npw, M, Psi, npw, Psi_io, ldio, st);
  CHEBFI_HIP(hipMemcpyAsync(eval, lam, sizeof(double) * M, hipMemcpyDeviceToHost, st));
  CHEBFI_HIP(hipMemcpyAsync(res, resd, sizeof(double) * M, hipMemcpyDeviceToHost, st));
  CHEBFI_HIP(hipStreamSynchronize(st));
}

}  // namespace chebfi
