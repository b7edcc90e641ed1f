// Host-side drivers shared by the entry points (driver.cpp, lobpcg.cpp).
#pragma once

#include <cstdint>

#include "internal.h"

namespace chebfi {

// Device copy of `count` host elements (allocation only when host is null);
// throws ABI_ERR_NOMEM on allocation failure.
template <typename T> inline T *upload(const T *host, size_t count) {
  T *dev = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&dev, sizeof(T) * count) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{ABI_ERR_NOMEM, "hipMalloc failed during set_system"};
  }
  if (host) CHEBFI_HIP(hipMemcpy(dev, host, sizeof(T) * count, hipMemcpyHostToDevice));
  return dev;
}

inline size_t elem_bytes(int32_t dtype) { return dtype == ABI_C64 ? sizeof(float2) : sizeof(double2); }

// Out = alpha (H - cshift) X - beta Xprev (Xprev may be null).  dtype ABI_C128: FP64;
// ABI_C64: complex64 blocks, FP32 FFT passes, split-BF16 MFMA projector products.
// Craw (optional) receives the raw projections P^H X (nproj x nband, contiguous, in
// the block's precision).
void apply_core(abi_system_s *s, const void *X, int64_t ldx, const void *Xprev, int64_t ldp,
                void *Out, int64_t ldo, int64_t nband, double alpha, double cshift, double beta,
                hipStream_t st, int32_t dtype = ABI_C128, void *Craw = nullptr);

// Out = S X and Out = S^-1 X (copies of X when S = I); Out must not overlap X.
void apply_S(abi_system_s *s, const void *X, int64_t ldx, void *Out, int64_t ldo, int64_t nband,
             hipStream_t st, int32_t dtype = ABI_C128);
void apply_Sinv(abi_system_s *s, const void *X, int64_t ldx, void *Out, int64_t ldo,
                int64_t nband, hipStream_t st, int32_t dtype = ABI_C128);

// One step of the filter on S^-1 H: Out = alpha (S^-1 H - cshift) X - beta Xprev and
// Cnext = P^H Out, given Ck = P^H X and Ckm1 = P^H Xprev (complex double, nproj x nband;
// Ckm1 null on the first step).
void gen_step(abi_system_s *s, const void *X, int64_t ldx, const void *Xprev, int64_t ldp,
              void *Out, int64_t ldo, int64_t nband, double alpha, double cshift, double beta,
              const double2 *Ck, const double2 *Ckm1, double2 *Cnext, hipStream_t st,
              int32_t dtype);

// Split-BF16 projector products of the mixed form with the handle's tile
// variants (s->pl_proj, s->pl_expand).  mixed_proj_splits: K-split count of the
// projection of nband bands; mixed_project: part[z] = P^H X over K chunk z
// (complex float, splits x nproj x nband); mixed_expand: Out = P C' (or Out +=
// P C' with accumulate) for complex float C' (nproj x nband, ld nproj).
// have_planes: X's bf16 planes are already in s->planes (no split pass).
// proj_chains_planes: the projection variant reads planes that the previous
// filter step's last FFT pass can write (15, 16).
int mixed_proj_splits(abi_system_s *s, int64_t nband);
bool proj_chains_planes(const abi_system_s *s);
void mixed_project(abi_system_s *s, const void *X, int64_t ldx, int64_t nband, void *part,
                   int splits, hipStream_t st, bool have_planes = false);
void mixed_expand(abi_system_s *s, const void *Cp, void *Out, int64_t ldo, int64_t nband,
                  hipStream_t st, bool accumulate);

// C = P^H X in complex double (nproj x nband, contiguous).
void project_c128(abi_system_s *s, const void *X, int64_t ldx, int64_t nband, double2 *C,
                  hipStream_t st, int32_t dtype);

// Overlap tables from Q (host, natom*16 complex): B = P^H P and the Woodbury kernel K.
void setup_overlap(abi_system_s *s, const double *qij, hipStream_t st);

// Split-BF16 Rayleigh-Ritz of a complex64 block (mixed handle, S = I): 0
// (nothing written) when the equilibrated Gram matrix is not safely positive
// definite at that precision, 1 after one Cholesky pass, 2 after two (the
// block orthonormalised first).
int rr_lowprec(abi_system_s *s, void *Y, int64_t ld, void *HPsi, int64_t ldh_in, int64_t M,
                double *eval, double *resnorm, void *coef, hipStream_t st);

// FP64 Rayleigh-Ritz on a complex128 block Y (in: filtered block, out: Psi).
void rr_core(abi_system_s *s, double2 *Y, int64_t ld, double2 *HPsi, int64_t ldh_in, int64_t M,
             double *eval, double *resnorm, void *coef, hipStream_t st);

// One pass of block LOBPCG on Psi (npw x M, ld) in place (FP64); host eval, res (M)
// and the line minimisations of each block (steps, nblocks entries, or null).
void lobpcg_pass_core(abi_system_s *s, double2 *Psi_io, int64_t ldio, int64_t M, int nblocks,
                      int nline, double tol, double *eval, double *res, int *steps,
                      hipStream_t st);

}  // namespace chebfi
