// Drivers of the hot-path operations on one handle: the H application (FFT
// passes + projector products), the overlap S and its Woodbury inverse, the
// step of the filter on S^-1 H, the overlap set-up and the FP64 Rayleigh-Ritz.
// Paper (arXiv 2604.11139): section "Main computational kernels" (HX, HX_SX,
// Sinv), Algorithm "Parallel Chebyshev filtering of degree k", Algorithms
// "S-ortho" and "RR".
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "cplx.h"
#include "driver.h"
#include "kernels.h"

namespace chebfi {
namespace {

// Projection variants 4 and 9..14 read the complex64 block itself (split into
// bf16 planes while staged); the others read planes made by a separate pass
// (15 and 16: the pipelined direct-to-LDS tiles of 2 x 4 and 4 x 2 waves).
static bool proj_reads_block(int variant) { return variant == 4 || (variant >= 9 && variant <= 14); }
static int proj_planes_variant(int variant) { return variant >= 15 ? variant - 2 : variant; }

}  // namespace

int mixed_proj_splits(abi_system_s *s, int64_t nband) {
  // 9..12 share the 128 x 128 tile of planes variant 7, 13 the 128 x 256 one of
  // 12, 14..16 the 128 x 128 one
  const int v = s->pl_proj == 13 ? 12 : s->pl_proj >= 9 ? 7 : s->pl_proj;
  return proj_planes_splits(v, s->nproj, nband, s->npw);
}

bool proj_chains_planes(const abi_system_s *s) {
  return s->pl_proj >= 15 && s->mixed_gemm == 0 && s->nproj > 0;
}

void mixed_project(abi_system_s *s, const void *X, int64_t ldx, int64_t nband, void *part,
                   int splits, hipStream_t st, bool have_planes) {
  const int64_t npw = s->npw;
  const int nproj = s->nproj;
  // a no-allocation call keeps to the block-reading tile (no planes buffer in
  // the scratch array); same tile and K split as 15
  const int v = (g_scratch_arena && s->pl_proj >= 15) ? 14 : s->pl_proj;
  const double flops = 8.0 * (double)nproj * (double)npw * (double)nband;
  if (proj_reads_block(v)) {
    const int tok = s->prof.begin(PROF_PROJ, flops, st);
    proj_gemm_f32_variant(v == 4 ? 0 : v - 8, nproj, nband, npw, s->d_PA, s->ldPA,
                          (int64_t)nproj * s->ldPA, X, ldx, part, splits, st);
    s->prof.end(tok, st);
    return;
  }
  void *xpl = s->planes.get(8 * (size_t)s->ldPA * nband);
  if (!have_planes) {
    const int tk = s->prof.begin(PROF_SPLIT, 16.0 * (double)npw * (double)nband, st);
    split_planes(npw, nband, X, ldx, xpl, s->ldPA, st);
    s->prof.end(tk, st);
  }
  const int tok = s->prof.begin(PROF_PROJ, flops, st);
  proj_gemm_planes(nproj, nband, npw, s->d_PA, s->ldPA, (int64_t)nproj * s->ldPA, xpl, s->ldPA,
                   s->ldPA * nband, part, splits, st, proj_planes_variant(v));
  s->prof.end(tok, st);
}

void mixed_expand(abi_system_s *s, const void *Cp, void *Out, int64_t ldo, int64_t nband,
                  hipStream_t st, bool accumulate) {
  const int nproj = s->nproj;
  split_planes(nproj, nband, Cp, nproj, s->cplanes.get(8 * (size_t)s->ldPB * nband), s->ldPB, st);
  expand_gemm_planes(s->npw, nband, nproj, s->d_PB, s->ldPB, s->npw * s->ldPB, s->cplanes.ptr,
                     s->ldPB, s->ldPB * nband, Out, ldo, st, s->pl_expand, accumulate);
}

namespace {

// Projector products of a block: part[z] = P^H X over plane-wave chunk z
// (returns the chunk count).  T = double: FP64 MFMA (a matrix-vector product
// for one band); T = float: complex64 block, split-BF16 MFMA (FP32 MFMA with
// mixed_gemm = 1), FP32 partials.
template <typename T>
int project_t(abi_system_s *s, const void *X, int64_t ldx, int64_t nband, hipStream_t st,
              C2<T> **part_out, bool have_planes = false) {
  typedef C2<T> V2;
  const bool fp32 = std::is_same<T, float>::value;
  const void *P = fp32 ? (const void *)s->d_Pf : (const void *)s->d_P;
  const int64_t npw = s->npw;
  const int nproj = s->nproj;
  const bool single = (nband == 1) && !fp32;
  const bool planes = fp32 && s->mixed_gemm == 0;
  const int splits = single ? 1
                     : planes ? mixed_proj_splits(s, nband)
                              : zgemm_splits(nproj, nband, npw);
  V2 *cpart = (V2 *)s->cpart.get(sizeof(V2) * (size_t)splits * nproj * nband);
  const double flops = 8.0 * (double)nproj * (double)npw * (double)nband;
  // the split-BF16 products time themselves (a planes variant's split pass apart)
  if (planes) {
    mixed_project(s, X, ldx, nband, cpart, splits, st, have_planes);
    *part_out = cpart;
    return splits;
  }
  const int tok = s->prof.begin(PROF_PROJ, flops, st);
  if (single)
    proj_gemv(npw, nproj, P, X, cpart, st);
  else if (fp32 && s->mixed_gemm == 2)
    proj_gemm_bf16x3(nproj, nband, npw, s->d_PA, s->ldPA, (int64_t)nproj * s->ldPA, X, ldx,
                     cpart, splits, st);
  else
    proj_gemm(nproj, nband, npw, P, X, ldx, cpart, splits, st, fp32);
  s->prof.end(tok, st);
  *part_out = cpart;
  return splits;
}

// Out += P C' for nproj x nband coefficients C' (ld nproj) of the block's type;
// store_only (split-BF16 products only): Out = P C'.
template <typename T>
void expand_t(abi_system_s *s, const C2<T> *cprime, void *Out, int64_t ldo, int64_t nband,
              hipStream_t st, bool store_only = false) {
  const bool fp32 = std::is_same<T, float>::value;
  const void *P = fp32 ? (const void *)s->d_Pf : (const void *)s->d_P;
  const int64_t npw = s->npw;
  const int nproj = s->nproj;
  const bool single = (nband == 1) && !fp32;
  const bool planes = fp32 && s->mixed_gemm == 0;
  CHEBFI_REQUIRE(!store_only || (planes && !single), ABI_ERR_STATE,
                 "store-only expansion needs the split-BF16 products");
  if (planes)
    split_planes(nproj, nband, cprime, nproj, s->cplanes.get(8 * (size_t)s->ldPB * nband),
                 s->ldPB, st);
  const double flops = 8.0 * (double)nproj * (double)npw * (double)nband;
  const int tok = s->prof.begin(PROF_EXPAND, flops, st);
  if (single)
    expand_gemv(npw, nproj, P, cprime, Out, st);
  else if (planes)
    expand_gemm_planes(npw, nband, nproj, s->d_PB, s->ldPB, npw * s->ldPB, s->cplanes.ptr,
                       s->ldPB, s->ldPB * nband, Out, ldo, st, s->pl_expand, !store_only);
  else if (fp32 && s->mixed_gemm == 2)
    expand_gemm_bf16x3(npw, nband, nproj, s->d_PB, s->ldPB, npw * s->ldPB, cprime, Out, ldo, st);
  else
    expand_gemm(npw, nband, nproj, P, cprime, Out, ldo, st, fp32);
  s->prof.end(tok, st);
}

// Local part, kinetic term and recurrence on the FFT grid:
// Out = alpha ((0.5|k+G|^2 + V_loc) X - cshift X) - beta Xprev   (Xprev may be null).
// E (optional, ld lde): the projector part P C', added to Out on the sphere.
template <typename T>
void local_t(abi_system_s *s, const void *X, int64_t ldx, const void *Xprev, int64_t ldp,
             void *Out, int64_t ldo, int64_t nband, double alpha, double cshift, double beta,
             hipStream_t st, const void *E = nullptr, int64_t lde = 0, void *ypl = nullptr) {
  typedef C2<T> V2;
  const bool fp32 = std::is_same<T, float>::value;
  const void *V = fp32 ? (const void *)s->d_Vf : (const void *)s->d_V;
  const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
  int fb = (int)std::min<int64_t>(s->fft_batch * (fp32 ? 2 : 1), nband);
  if (ScratchArena *a = g_scratch_arena) {
    // no-allocation call: as many boxes as the scratch array has room for
    const size_t room = a->remaining() > a->reserve + 256 ? a->remaining() - a->reserve - 256 : 0;
    fb = (int)std::max<int64_t>(1, std::min<int64_t>(fb, room / (sizeof(V2) * (size_t)nbox)));
  }
  void *box = s->box.get(sizeof(V2) * (size_t)nbox * fb);
  for (int64_t b0 = 0; b0 < nband; b0 += fb) {
    const int nb = (int)std::min<int64_t>(fb, nband - b0);
    launch_local_potential<T>(s, X, ldx, Xprev, ldp, Out, ldo, (int)b0, nb, box, V, alpha, cshift,
                              beta, st, s->prof.on ? &s->prof : nullptr, E, lde, ypl, s->ldPA,
                              s->ldPA * nband);
  }
}

// Out = alpha * (H - cshift) X - beta * Xprev   (Xprev may be null).
// T = double: FP64 tables, FP64 MFMA; T = float: complex64 blocks, FP32 FFT
// passes and FP32 MFMA projector products (mixed form).
// Craw (optional): receives the raw projections P^H X (nproj x nband, contiguous, in the
// block's precision), the sum of the same split-K partials the D application reads.
template <typename T>
void apply_core_t(abi_system_s *s, const void *X, int64_t ldx, const void *Xprev, int64_t ldp,
                  void *Out, int64_t ldo, int64_t nband, double alpha, double cshift, double beta,
                  hipStream_t st, void *Craw = nullptr) {
  typedef C2<T> V2;
  const bool fp32 = std::is_same<T, float>::value;
  const int nproj = s->nproj;
  const bool single = (nband == 1) && !fp32;
  // the FFT passes run on the second stream beside the projection when they can
  const bool side = s->overlap && nproj > 0 && !single && s->aux;
  // otherwise, with the split-BF16 products, the projector part goes first: the
  // expansion stores E = P C' (no read of the output block) and the last FFT
  // pass adds E while it writes Out
  const bool pre = !side && nproj > 0 && fp32 && s->mixed_gemm == 0;
  // chained planes: X's planes from the previous step's last pass (or assumed
  // present while the autotuner times a chained step); this step's last pass
  // writes Out's (after the projection has read X's from the same buffer)
  const bool chain = pre && s->pl_chain && proj_chains_planes(s);
  const bool have_planes = chain && (s->pl_assume || (s->pl_have == X && X != nullptr));
  s->pl_have = nullptr;
  if (side) {
    CHEBFI_HIP(hipEventRecord(s->ev_fork, st));
    CHEBFI_HIP(hipStreamWaitEvent(s->aux, s->ev_fork, 0));
  }
  if (!pre)
    local_t<T>(s, X, ldx, Xprev, ldp, Out, ldo, nband, alpha, cshift, beta, side ? s->aux : st);
  if (side) CHEBFI_HIP(hipEventRecord(s->ev_join, s->aux));
  V2 *cprime = nullptr;
  if (nproj > 0) {
    // C = P^H X, C' = alpha D C
    V2 *cpart = nullptr;
    const int splits = project_t<T>(s, X, ldx, nband, st, &cpart, have_planes);
    if (Craw) launch_sum_parts(nproj, nband, cpart, splits, Craw, st, fp32);
    cprime = (V2 *)s->cprime.get(sizeof(V2) * (size_t)nproj * nband);
    const int tok =
        s->prof.begin(PROF_DAPPLY, (double)sizeof(V2) * nproj * nband * (splits + 1), st);
    launch_dapply(s->natom, nband, cpart, splits, s->d_D, alpha, cprime, st, fp32, s->coef_dev);
    s->prof.end(tok, st);
  }
  if (side) CHEBFI_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
  if (pre) {
    void *E = s->expout.get(sizeof(V2) * (size_t)s->npw * nband);
    expand_t<T>(s, cprime, E, s->npw, nband, st, true);  // E = P C'
    void *ypl = chain ? s->planes.get(8 * (size_t)s->ldPA * nband) : nullptr;
    local_t<T>(s, X, ldx, Xprev, ldp, Out, ldo, nband, alpha, cshift, beta, st, E, s->npw, ypl);
    if (chain) s->pl_have = Out;
  } else if (nproj > 0) {
    expand_t<T>(s, cprime, Out, ldo, nband, st);  // Out += P C'
  }
}

// ---- overlap S = I + P Q P^H and its Woodbury inverse ----------------------------

// Out = S X = X + P (Q (P^H X))  (Out must not overlap X).
template <typename T>
void apply_S_t(abi_system_s *s, const void *X, int64_t ldx, void *Out, int64_t ldo,
               int64_t nband, hipStream_t st) {
  typedef C2<T> V2;
  const bool fp32 = std::is_same<T, float>::value;
  launch_copy_block(s->npw, nband, X, ldx, Out, ldo, st, fp32);
  if (!s->has_S) return;
  V2 *cpart = nullptr;
  const int splits = project_t<T>(s, X, ldx, nband, st, &cpart);
  V2 *cprime = (V2 *)s->cprime.get(sizeof(V2) * (size_t)s->nproj * nband);
  launch_dapply(s->natom, nband, cpart, splits, s->d_Q, 1.0, cprime, st, fp32);
  expand_t<T>(s, cprime, Out, ldo, nband, st);
}

// Out = S^-1 X = X - P (K (P^H X))  (the Sinv kernel; Out must not overlap X).
template <typename T>
void apply_Sinv_t(abi_system_s *s, const void *X, int64_t ldx, void *Out, int64_t ldo,
                  int64_t nband, hipStream_t st) {
  typedef C2<T> V2;
  const bool fp32 = std::is_same<T, float>::value;
  launch_copy_block(s->npw, nband, X, ldx, Out, ldo, st, fp32);
  if (!s->has_S) return;
  const int n = s->nproj;
  V2 *cpart = nullptr;
  const int splits = project_t<T>(s, X, ldx, nband, st, &cpart);
  double2 *C = (double2 *)s->gen_e.get(sizeof(double2) * (size_t)n * nband);
  double2 *F = (double2 *)s->gen_f.get(sizeof(double2) * (size_t)n * nband);
  const int tok = s->prof.begin(PROF_DAPPLY, 8.0 * (double)n * n * nband, st);
  launch_parts_to_c128(n, nband, cpart, splits, fp32, C, st);
  zgemm(OP_N, OP_N, n, nband, n, s->d_K, n, C, n, F, n, double2{-1, 0}, double2{0, 0}, st);
  const V2 *fp = (const V2 *)F;
  if (fp32) {
    float2 *Ff = (float2 *)s->gen_ff.get(sizeof(float2) * (size_t)n * nband);
    launch_d2f(2 * (int64_t)n * nband, (const double *)F, (float *)Ff, st);
    fp = (const V2 *)Ff;
  }
  s->prof.end(tok, st);
  expand_t<T>(s, fp, Out, ldo, nband, st);
}

// One step of the filter on S^-1 H:
//   Out = alpha (S^-1 H - cshift) X - beta Xprev,   Cnext = P^H Out,
// given Ck = P^H X and Ckm1 = P^H Xprev (complex double, nproj x nband; Ckm1 null
// on the first step).  With H X = T + P D Ck (T: kinetic and local part) and
// S^-1 = I - P K P^H:  S^-1 H X = T + P F,  F = D Ck - K (P^H T + B D Ck).
// The local passes write Out = alpha (T - c X) - beta Xprev; its projection G
// gives P^H T = G / alpha + c Ck + (beta / alpha) Ckm1 without projecting T
// itself; then Out += alpha P F and Cnext = G + alpha B F.  One projection and
// one expansion of the block per step, as for S = I, plus three nproj x nproj
// products by nband.
// The projection reads the local passes' output, so the two are pipelined over
// two halves of the bands: the passes of the second half (second stream) run
// beside the projection of the first, and D Ck, B D Ck beside the first half's
// passes.
template <typename T>
void gen_step_t(abi_system_s *s, const void *X, int64_t ldx, const void *Xprev, int64_t ldp,
                void *Out, int64_t ldo, int64_t nband, double alpha, double cshift, double beta,
                const double2 *Ck, const double2 *Ckm1, double2 *Cnext, hipStream_t st) {
  typedef C2<T> V2;
  const bool fp32 = std::is_same<T, float>::value;
  const int n = s->nproj;
  const size_t eb = sizeof(V2);
  const bool side = s->overlap && s->aux && nband >= 128;
  // band ranges [0, h) and [h, nband)
  const int64_t h = side ? (nband / 2 + 31) / 32 * 32 : nband;
  auto at = [&](const void *p, int64_t ld, int64_t b) -> const void * {
    return p ? (const void *)((const char *)p + eb * (size_t)(b * ld)) : nullptr;
  };
  auto local_range = [&](int64_t b0, int64_t nb, hipStream_t sst) {
    local_t<T>(s, at(X, ldx, b0), ldx, at(Xprev, ldp, b0), ldp,
               (void *)at(Out, ldo, b0), ldo, nb, alpha, cshift, beta, sst);
  };
  if (side) {
    CHEBFI_HIP(hipEventRecord(s->ev_fork, st));
    CHEBFI_HIP(hipStreamWaitEvent(s->aux, s->ev_fork, 0));
    local_range(0, h, s->aux);
    CHEBFI_HIP(hipEventRecord(s->ev_half, s->aux));
    local_range(h, nband - h, s->aux);
    CHEBFI_HIP(hipEventRecord(s->ev_join, s->aux));
  } else {
    local_range(0, nband, st);
  }
  double2 *E = (double2 *)s->gen_e.get(sizeof(double2) * (size_t)n * nband);
  double2 *F = (double2 *)s->gen_f.get(sizeof(double2) * (size_t)n * nband);
  int tok = s->prof.begin(PROF_DAPPLY, 8.0 * (double)n * n * nband, st);
  launch_dapply(s->natom, nband, Ck, 1, s->d_D, 1.0, F, st, false);  // F = D Ck
  zgemm(OP_N, OP_N, n, nband, n, s->d_B, n, F, n, E, n, double2{1, 0}, double2{0, 0},
        st);  // E = B D Ck
  s->prof.end(tok, st);
  // G = P^H Out per band range; E += G / alpha + c Ck + (beta / alpha) Ckm1, Cnext = G
  for (int part = 0; part < 2; ++part) {
    const int64_t b0 = part == 0 ? 0 : h, nb = part == 0 ? h : nband - h;
    if (nb <= 0) continue;
    if (side) CHEBFI_HIP(hipStreamWaitEvent(st, part == 0 ? s->ev_half : s->ev_join, 0));
    V2 *cpart = nullptr;
    const int splits = project_t<T>(s, at(Out, ldo, b0), ldo, nb, st, &cpart);
    const size_t off = (size_t)n * b0;
    launch_gen_combine(n, nb, cpart, splits, fp32, Ck + off, Ckm1 ? Ckm1 + off : nullptr, alpha,
                       cshift, beta, E + off, Cnext + off, st);
  }
  tok = s->prof.begin(PROF_DAPPLY, 16.0 * (double)n * n * nband, st);
  zgemm(OP_N, OP_N, n, nband, n, s->d_K, n, E, n, F, n, double2{-alpha, 0}, double2{alpha, 0},
        st);  // F = alpha (D Ck - K E)
  zgemm(OP_N, OP_N, n, nband, n, s->d_B, n, F, n, Cnext, n, double2{1, 0}, double2{1, 0}, st);
  const V2 *fp = (const V2 *)F;
  if (fp32) {
    float2 *Ff = (float2 *)s->gen_ff.get(sizeof(float2) * (size_t)n * nband);
    launch_d2f(2 * (int64_t)n * nband, (const double *)F, (float *)Ff, st);
    fp = (const V2 *)Ff;
  }
  s->prof.end(tok, st);
  expand_t<T>(s, fp, Out, ldo, nband, st);
}

// Ck = P^H X in complex double (the first coefficients of a generalised filter).
template <typename T>
void project_c128_t(abi_system_s *s, const void *X, int64_t ldx, int64_t nband, double2 *C,
                    hipStream_t st) {
  C2<T> *cpart = nullptr;
  const int splits = project_t<T>(s, X, ldx, nband, st, &cpart);
  launch_parts_to_c128(s->nproj, nband, cpart, splits, std::is_same<T, float>::value, C, st);
}

}  // namespace

void apply_core(abi_system_s *s, const void *X, int64_t ldx, const void *Xprev, int64_t ldp,
                void *Out, int64_t ldo, int64_t nband, double alpha, double cshift, double beta,
                hipStream_t st, int32_t dtype, void *Craw) {
  if (dtype == ABI_C64)
    apply_core_t<float>(s, X, ldx, Xprev, ldp, Out, ldo, nband, alpha, cshift, beta, st, Craw);
  else
    apply_core_t<double>(s, X, ldx, Xprev, ldp, Out, ldo, nband, alpha, cshift, beta, st, Craw);
}

void apply_S(abi_system_s *s, const void *X, int64_t ldx, void *Out, int64_t ldo, int64_t nband,
             hipStream_t st, int32_t dtype) {
  if (dtype == ABI_C64)
    apply_S_t<float>(s, X, ldx, Out, ldo, nband, st);
  else
    apply_S_t<double>(s, X, ldx, Out, ldo, nband, st);
}

void apply_Sinv(abi_system_s *s, const void *X, int64_t ldx, void *Out, int64_t ldo,
                int64_t nband, hipStream_t st, int32_t dtype) {
  if (dtype == ABI_C64)
    apply_Sinv_t<float>(s, X, ldx, Out, ldo, nband, st);
  else
    apply_Sinv_t<double>(s, X, ldx, Out, ldo, nband, st);
}

// Builds the overlap tables from Q (host, natom*16 complex): B = P^H P,
// B = R^H R (Cholesky), R Q R^H = Z diag(mu) Z^H, so that S has the eigenvalues
// 1 and 1 + mu_i and S^-1 = I - P K P^H with K = W diag(mu/(1+mu)) W^H, W = R^-1 Z
// (the Woodbury formula, written through the eigenvalues of the small pencil so
// that an indefinite Q is allowed as long as S stays positive definite).
void setup_overlap(abi_system_s *s, const double *qij, hipStream_t st) {
  const int n = s->nproj;
  if (n == 0 || qij == nullptr) return;
  s->d_Q = upload(qij, (size_t)s->natom * 32);
  std::vector<double> Qd((size_t)2 * n * n, 0.0);
  for (int R = 0; R < s->natom; ++R)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        // column-major dense Q, Q[4R+i, 4R+j] = Q_R[i][j]
        const size_t dst = 2 * ((size_t)(4 * R + i) + (size_t)(4 * R + j) * n);
        Qd[dst] = qij[32 * R + 2 * (4 * i + j)];
        Qd[dst + 1] = qij[32 * R + 2 * (4 * i + j) + 1];
      }
  const size_t mm = sizeof(double2) * (size_t)n * n;
  double2 *Q = upload((const double2 *)Qd.data(), (size_t)n * n);
  DevBuf w1, w2, w3, wz, ws;
  double2 *R = (double2 *)w1.get(mm), *T = (double2 *)w2.get(mm), *A = (double2 *)w3.get(mm);
  double2 *Z = (double2 *)wz.get(mm);
  double *mu = (double *)ws.get(sizeof(double) * (size_t)n + 64);
  int *info = (int *)(mu + n);
  s->d_B = (double *)upload<double2>(nullptr, (size_t)n * n);
  s->d_K = (double *)upload<double2>(nullptr, (size_t)n * n);
  try {
    {
      const int splits = zgemm_splits(n, n, s->npw);
      DevBuf part;
      void *pp = part.get(sizeof(double2) * (size_t)splits * n * n);
      zgemm(OP_C, OP_N, n, n, s->npw, s->d_P, s->npw, s->d_P, s->npw, nullptr, 0, double2{1, 0},
            double2{0, 0}, st, pp, splits);
      zsum_parts(n, n, pp, splits, s->d_B, n, double2{1, 0}, double2{0, 0}, st);
      CHEBFI_HIP(hipStreamSynchronize(st));
    }
    launch_hermitize(n, s->d_B, n, st);
    launch_copy_block(n, n, s->d_B, n, R, n, st);
    DevBuf pw;
    zpotrf_upper(n, R, n, info, pw.get(zpotrf_work_bytes(n)), st);
    int hinfo = 0;
    CHEBFI_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
    CHEBFI_HIP(hipStreamSynchronize(st));
    if (hinfo != 0)
      throw Error{ABI_ERR_NOT_HPD, "projector Gram matrix P^H P is singular (pivot " +
                                       std::to_string(hinfo) + ")"};
    // A = R Q R^H
    zgemm(OP_N, OP_C, n, n, n, Q, n, R, n, T, n, double2{1, 0}, double2{0, 0}, st);
    zgemm(OP_N, OP_N, n, n, n, R, n, T, n, A, n, double2{1, 0}, double2{0, 0}, st);
    DevBuf ew;
    zheev(n, A, n, mu, Z, n, ew.get(zheev_work_bytes(n)), st);
    std::vector<double> hmu(n);
    CHEBFI_HIP(hipMemcpyAsync(hmu.data(), mu, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    CHEBFI_HIP(hipStreamSynchronize(st));
    s->s_min = std::min(1.0, 1.0 + hmu[0]);
    if (!(1.0 + hmu[0] > 1e-10))
      throw Error{ABI_ERR_NOT_HPD, "overlap operator S = I + P Q P^H is not positive definite "
                                   "(smallest eigenvalue " + std::to_string(1.0 + hmu[0]) + ")"};
    // W = R^-1 Z, K = W diag(mu / (1 + mu)) W^H
    DevBuf tw;
    ztrtri_upper(n, R, n, tw.get(ztrtri_work_bytes(n)), st);
    zgemm(OP_N, OP_N, n, n, n, R, n, Z, n, T, n, double2{1, 0}, double2{0, 0}, st);
    launch_woodbury_scale(n, T, n, mu, A, n, st);
    zgemm(OP_N, OP_C, n, n, n, A, n, T, n, s->d_K, n, double2{1, 0}, double2{0, 0}, st);
    launch_hermitize(n, s->d_K, n, st);
    CHEBFI_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(Q);
    throw;
  }
  CHEBFI_HIP(hipFree(Q));
  s->has_S = true;
}

// FP64 Rayleigh-Ritz on a complex128 block Y (in: filtered block, out: Psi).
// Rayleigh-Ritz of a complex64 block with split-BF16 products (mixed form,
// S = I): the columns are scaled to unit norm (Y_e = Y E, E = diag(1/||y_j||)),
// G = Y_e^H Y_e and H_s = Y_e^H (H Y_e) are split-BF16 products accumulated in
// FP32 (summed in FP64), the Cholesky factorisation, the reduction and the
// eigensolve run in FP64, and the rotations Psi = Y_e T, H Psi = (H Y_e) T
// (T = U^-1 Z) are split-BF16 products again.  The equilibrated Gram matrix of
// a filtered block is well conditioned even when G is not; a pivot of its
// Cholesky factor below kLowPivot (a condition number the split products'
// ~1e-5 relative error cannot resolve) returns false and nothing is written.
int rr_lowprec(abi_system_s *s, void *Y, int64_t ld, void *HPsi, int64_t ldh_in, int64_t M,
               double *eval, double *resnorm, void *coef, hipStream_t st) {
  // pivots^2 of the equilibrated Gram matrix's Cholesky factor: below kLowPivot
  // the split products cannot resolve the block (FP64 form instead); below
  // kTwoPass a second pass orthonormalises first (CholeskyQR2)
  constexpr double kLowPivot = 1e-4, kTwoPass = 0.5;
  const int64_t npw = s->npw;
  const size_t mm = sizeof(double2) * (size_t)M * M;
  double2 *G = (double2 *)s->small1.get(mm);
  double2 *Hs = (double2 *)s->small2.get(mm);
  double2 *T = (double2 *)s->small3.get(mm);
  double2 *Z = (double2 *)s->small4.get(mm);
  double *scal = (double *)s->scal.get(sizeof(double) * (size_t)(160 + 5 * M + 64));
  double *w_dev = scal + 160;
  double *r_dev = w_dev + M;
  double *nrm = r_dev + M, *inv = nrm + M;
  double *pmin_dev = inv + M;
  int *info = (int *)(pmin_dev + 1);
  const size_t blk = sizeof(float2) * (size_t)npw * M;
  float2 *Ye = (float2 *)s->blk4.get(blk);
  float2 *spare = (float2 *)s->blk1.get(blk);
  const int64_t ldm = (M + 31) / 32 * 32;
  const int splits = proj_planes_splits(7, M, M, npw);
  const double gflops = 8.0 * (double)M * M * npw;
  // (own planes buffer: a planes variant of the H application reuses s->planes)
  void *ypl = s->rr_planes.get(8 * (size_t)s->ldPA * M);
  void *part = nullptr;
  // G = Ye^H Ye as split-BF16 products, its Cholesky factor in G; 0 if a pivot
  // is too small, else the smallest pivot^2
  auto gram_chol = [&](const float2 *B) -> double {
    ypl = s->rr_planes.get(8 * (size_t)s->ldPA * M);
    split_planes(npw, M, B, npw, ypl, s->ldPA, st);
    part = s->cpart.get(sizeof(float2) * (size_t)splits * M * M);
    int tok = s->prof.begin(PROF_GRAM, gflops, st);
    rr_gram_f32(M, npw, ypl, s->ldPA, B, npw, part, splits, st);
    launch_parts_to_c128(M, M, part, splits, true, G, st);
    s->prof.end(tok, st);
    launch_hermitize(M, G, M, st);
    tok = s->prof.begin(PROF_CHOL, 4.0 / 3.0 * (double)M * M * M, st);
    zpotrf_upper(M, G, M, info, nullptr, st);
    s->prof.end(tok, st);
    launch_diag_min_sq(M, G, M, pmin_dev, st);
    // (the stream drained first, then blocking copies into host variables)
    CHEBFI_HIP(hipStreamSynchronize(st));
    int hinfo = 0;
    double pmin = 0.0;
    CHEBFI_HIP(hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost));
    CHEBFI_HIP(hipMemcpy(&pmin, pmin_dev, sizeof(double), hipMemcpyDeviceToHost));
    if (hinfo != 0) return 0.0;
    return pmin >= kLowPivot ? pmin : 0.0;
  };
  // Out = A C for the npw x M complex64 block A and the FP64 M x M matrix C
  // (rounded to complex64), both split into BF16 planes
  void *tpl = nullptr, *ytpl = nullptr;
  auto split_coef = [&](const double2 *C) {
    float2 *C32 = (float2 *)Hs;  // free whenever a coefficient matrix is split
    launch_c128_to_c64(M, M, C, M, C32, M, st);
    tpl = s->cplanes.get(8 * (size_t)ldm * M);
    split_planes(M, M, C32, M, tpl, ldm, st);
    ytpl = s->rr_planes.get(8 * (size_t)npw * ldm);
  };
  auto rotate = [&](const float2 *A, void *Out, int64_t ldo) {
    split_planes_t(npw, M, A, npw, ytpl, ldm, st);
    rr_rotate_planes(npw, M, ytpl, ldm, tpl, ldm, Out, ldo, st);
  };
  // equilibrated block Ye = Y E (E = diag of inverse column norms)
  launch_col_norms(npw, M, Y, ld, nrm, inv, st, true);
  launch_scale_cols_f(npw, M, Y, ld, inv, Ye, npw, st);
  double pmin = gram_chol(Ye);
  if (pmin == 0.0) return 0;
  void *trw = s->eig2.get(ztrtri_work_bytes(M));
  double2 *U1i = nullptr;
  if (pmin < kTwoPass) {
    // Q1 = Ye U1^-1, then the Gram matrix of Q1 (close to I)
    U1i = (double2 *)s->small5.get(mm);
    int tok = s->prof.begin(PROF_ROT, 16.0 * (double)npw * M * M, st);
    ztrtri_upper(M, G, M, trw, st);
    launch_copy_block(M, M, G, M, U1i, M, st);
    split_coef(U1i);
    rotate(Ye, spare, npw);
    s->prof.end(tok, st);
    std::swap(Ye, spare);
    if (gram_chol(Ye) == 0.0) return 0;
  }
  // H Ye (mixed H application) and H_s = Ye^H (H Ye)
  float2 *HYe = spare;
  apply_core(s, Ye, npw, nullptr, 0, HYe, npw, M, 1.0, 0.0, 0.0, st, ABI_C64);
  // (ypl still holds the planes of Ye from its Gram matrix)
  part = s->cpart.get(sizeof(float2) * (size_t)splits * M * M);  // apply_core may regrow it
  int tok = s->prof.begin(PROF_GRAM, gflops, st);
  rr_gram_f32(M, npw, ypl, s->ldPA, HYe, npw, part, splits, st);
  launch_parts_to_c128(M, M, part, splits, true, Hs, st);
  s->prof.end(tok, st);
  launch_hermitize(M, Hs, M, st);
  tok = s->prof.begin(PROF_CHOL, 16.0 * (double)M * M * M, st);
  ztrtri_upper(M, G, M, trw, st);
  zgemm(OP_N, OP_N, M, M, M, Hs, M, G, M, T, M, double2{1, 0}, double2{0, 0}, st);
  zgemm(OP_C, OP_N, M, M, M, G, M, T, M, Hs, M, double2{1, 0}, double2{0, 0}, st);
  s->prof.end(tok, st);
  void *ew = s->eig1.get(zheev_work_bytes(M));
  tok = s->prof.begin(PROF_EIG, 16.0 / 3.0 * (double)M * M * M, st);
  zheev(M, Hs, M, w_dev, Z, M, ew, st);
  s->prof.end(tok, st);
  // T = U^-1 Z; Psi = Ye T and H Psi = (H Ye) T as split-BF16 products
  tok = s->prof.begin(PROF_ROT, 8.0 * (double)M * M * M + 16.0 * (double)npw * M * M, st);
  zgemm(OP_N, OP_N, M, M, M, G, M, Z, M, T, M, double2{1, 0}, double2{0, 0}, st);
  split_coef(T);
  rotate(Ye, Y, ld);
  void *HP;
  int64_t ldh;
  if (HPsi) {
    HP = HPsi;
    ldh = ldh_in;
  } else {
    HP = s->blk3.get(blk);
    ldh = npw;
  }
  rotate(HYe, HP, ldh);
  s->prof.end(tok, st);
  if (coef) {
    // Psi = Y_in E [U1^-1] T
    const double2 *C = T;
    if (U1i) {
      zgemm(OP_N, OP_N, M, M, M, U1i, M, T, M, Z, M, double2{1, 0}, double2{0, 0}, st);
      C = Z;
    }
    launch_copy_block(M, M, C, M, coef, M, st);
    launch_scale_rows(M, M, coef, M, inv, st);
  }
  launch_residual_norms_f(npw, M, Y, ld, HP, ldh, w_dev, r_dev, st);
  CHEBFI_HIP(hipMemcpyAsync(eval, w_dev, sizeof(double) * M, hipMemcpyDeviceToHost, st));
  if (resnorm)
    CHEBFI_HIP(hipMemcpyAsync(resnorm, r_dev, sizeof(double) * M, hipMemcpyDeviceToHost, st));
  CHEBFI_HIP(hipStreamSynchronize(st));
  return U1i ? 2 : 1;
}

void rr_core(abi_system_s *s, double2 *Y, int64_t ld, double2 *HPsi, int64_t ldh_in, int64_t M,
             double *eval, double *resnorm, void *coef, hipStream_t st) {
  const int64_t npw = s->npw;
  const size_t mm = sizeof(double2) * (size_t)M * M;
  double2 *G = (double2 *)s->small1.get(mm);
  double2 *Hs = (double2 *)s->small2.get(mm);
  double2 *T = (double2 *)s->small3.get(mm);
  double2 *Z = (double2 *)s->small4.get(mm);
  double *scal = (double *)s->scal.get(sizeof(double) * (size_t)(160 + 3 * M + 64));
  double *w_dev = scal + 160;
  double *r_dev = w_dev + M;
  int *info = (int *)(r_dev + M);
  // Gram G = Y^H (S Y) -> U (Cholesky, upper); with S != I, S Y = Y + P Q C_Y from
  // the projections C_Y = P^H Y, which also give S Psi after the rotation
  const bool gen = s->has_S;
  const int n = s->nproj;
  double2 *CY = nullptr, *SY = Y;
  int64_t lds = ld;
  if (gen) {
    CY = (double2 *)s->gen_c.get(sizeof(double2) * (size_t)n * M);
    double2 *QC = (double2 *)s->gen_f.get(sizeof(double2) * (size_t)n * M);
    SY = (double2 *)s->blk5.get(sizeof(double2) * (size_t)npw * M);
    lds = npw;
    project_c128_t<double>(s, Y, ld, M, CY, st);
    launch_dapply(s->natom, M, CY, 1, s->d_Q, 1.0, QC, st, false);
    launch_copy_block(npw, M, Y, ld, SY, lds, st);
    expand_t<double>(s, QC, SY, lds, M, st);
  }
  // both products are Hermitian: only the tiles on and above the diagonal are formed
  const int splits = zgemm_herm_splits(M, npw);
  void *part = s->cpart.get(sizeof(double2) * (size_t)splits * M * M);
  const double gflops = 8.0 * (double)M * M * npw;
  int tok = s->prof.begin(PROF_GRAM, gflops, st);
  zgemm_herm(M, npw, Y, ld, SY, lds, G, M, st, part, splits);
  s->prof.end(tok, st);
  launch_hermitize(M, G, M, st);
  tok = s->prof.begin(PROF_CHOL, 4.0 / 3.0 * (double)M * M * M, st);
  zpotrf_upper(M, G, M, info, nullptr, st);
  s->prof.end(tok, st);
  int hinfo = 0;
  CHEBFI_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
  CHEBFI_HIP(hipStreamSynchronize(st));
  if (hinfo != 0)
    throw Error{ABI_ERR_NOT_HPD,
                "Gram matrix not positive definite at pivot " + std::to_string(hinfo)};
  // H Y and H_s = Y^H (H Y)
  double2 *HY = (double2 *)s->blk1.get(sizeof(double2) * (size_t)npw * M);
  apply_core(s, Y, ld, nullptr, 0, HY, npw, M, 1.0, 0.0, 0.0, st);
  part = s->cpart.get(sizeof(double2) * (size_t)splits * M * M);  // apply_core may regrow it
  tok = s->prof.begin(PROF_GRAM, gflops, st);
  zgemm_herm(M, npw, Y, ld, HY, npw, Hs, M, st, part, splits);
  s->prof.end(tok, st);
  launch_hermitize(M, Hs, M, st);
  // U^-1 and the reduced matrix U^-H H_s U^-1
  tok = s->prof.begin(PROF_CHOL, 16.0 * (double)M * M * M, st);
  void *trw = s->eig2.get(ztrtri_work_bytes(M));
  ztrtri_upper(M, G, M, trw, st);
  zgemm(OP_N, OP_N, M, M, M, Hs, M, G, M, T, M, double2{1, 0}, double2{0, 0}, st);
  zgemm(OP_C, OP_N, M, M, M, G, M, T, M, Hs, M, double2{1, 0}, double2{0, 0}, st);
  s->prof.end(tok, st);
  // eigen-decomposition (Hs overwritten), W = U^-1 Z
  void *ew = s->eig1.get(zheev_work_bytes(M));
  tok = s->prof.begin(PROF_EIG, 16.0 / 3.0 * (double)M * M * M, st);
  zheev(M, Hs, M, w_dev, Z, M, ew, st);
  s->prof.end(tok, st);
  tok = s->prof.begin(PROF_ROT, 8.0 * (double)M * M * M + 16.0 * (double)npw * M * M, st);
  zgemm(OP_N, OP_N, M, M, M, G, M, Z, M, T, M, double2{1, 0}, double2{0, 0}, st);
  // Psi = Y W, H Psi = (H Y) W
  double2 *Psi = (double2 *)s->blk2.get(sizeof(double2) * (size_t)npw * M);
  zgemm(OP_N, OP_N, npw, M, M, Y, ld, T, M, Psi, npw, double2{1, 0}, double2{0, 0}, st);
  double2 *HP;
  int64_t ldh;
  if (HPsi) {
    HP = HPsi;
    ldh = ldh_in;
  } else {
    HP = (double2 *)s->blk3.get(sizeof(double2) * (size_t)npw * M);
    ldh = npw;
  }
  zgemm(OP_N, OP_N, npw, M, M, HY, npw, T, M, HP, ldh, double2{1, 0}, double2{0, 0}, st);
  s->prof.end(tok, st);
  if (coef) launch_copy_block(M, M, T, M, coef, M, st);
  launch_copy_block(npw, M, Psi, npw, Y, ld, st);
  if (gen) {
    // S Psi = Psi + P Q (C_Y W): residuals || H psi - lambda S psi ||
    double2 *CP = (double2 *)s->gen_e.get(sizeof(double2) * (size_t)n * M);
    double2 *QC = (double2 *)s->gen_f.get(sizeof(double2) * (size_t)n * M);
    zgemm(OP_N, OP_N, n, M, M, CY, n, T, M, CP, n, double2{1, 0}, double2{0, 0}, st);
    launch_dapply(s->natom, M, CP, 1, s->d_Q, 1.0, QC, st, false);
    launch_copy_block(npw, M, Psi, npw, SY, lds, st);
    expand_t<double>(s, QC, SY, lds, M, st);
    launch_residual_norms(npw, M, SY, lds, HP, ldh, w_dev, r_dev, st);
  } else {
    launch_residual_norms(npw, M, Y, ld, HP, ldh, w_dev, r_dev, st);
  }
  CHEBFI_HIP(hipMemcpyAsync(eval, w_dev, sizeof(double) * M, hipMemcpyDeviceToHost, st));
  if (resnorm)
    CHEBFI_HIP(hipMemcpyAsync(resnorm, r_dev, sizeof(double) * M, hipMemcpyDeviceToHost, st));
  CHEBFI_HIP(hipStreamSynchronize(st));
}

void gen_step(abi_system_s *s, const void *X, int64_t ldx, const void *Xprev, int64_t ldp,
              void *Out, int64_t ldo, int64_t nband, double alpha, double cshift, double beta,
              const double2 *Ck, const double2 *Ckm1, double2 *Cnext, hipStream_t st,
              int32_t dtype) {
  if (dtype == ABI_C64)
    gen_step_t<float>(s, X, ldx, Xprev, ldp, Out, ldo, nband, alpha, cshift, beta, Ck, Ckm1,
                      Cnext, st);
  else
    gen_step_t<double>(s, X, ldx, Xprev, ldp, Out, ldo, nband, alpha, cshift, beta, Ck, Ckm1,
                       Cnext, st);
}

void project_c128(abi_system_s *s, const void *X, int64_t ldx, int64_t nband, double2 *C,
                  hipStream_t st, int32_t dtype) {
  if (dtype == ABI_C64)
    project_c128_t<float>(s, X, ldx, nband, C, st);
  else
    project_c128_t<double>(s, X, ldx, nband, C, st);
}


}  // namespace chebfi
