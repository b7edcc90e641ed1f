// Complex FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// Serves the dense contractions of the path: the nonlocal projections P^H X and
// P (D C) (section "Low-level operations" of arXiv 2604.11139: level-3 BLAS for
// the nonlocal operator), the Gram and subspace matrices Y^H Y, Y^H (H Y) and
// the rotations Y Z (Algorithms "S-ortho" and "RR").  A complex product is four
// real MFMA chains on separate real/imaginary LDS planes:
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B.
// Workgroup tile 64 x 64 complex, four waves of 32 x 32, K step 16; operands are
// staged global -> registers -> LDS with the next K step's loads in flight
// while the current one is multiplied.  Tall-skinny products (K = npw) are
// split along K; each chunk writes its own partial product and a separate pass
// adds the chunks in a fixed order, so results do not depend on scheduling.
#include "cplx.h"
#include "kernels.h"

namespace chebfi {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;

// One 16x16x4 MFMA per element type and the row of accumulator element r of a
// lane (column is lane % 16 for both).
template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef v4d acc;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mma<float> {
  typedef v4f acc;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// TAG only separates instantiations (1 = projector products of the H
// application) so that kernel traces report them apart from the dense ones.
template <typename T, int OPA, int OPB, bool SPLIT, int TAG>
__global__ __launch_bounds__(256) void zgemm_kernel(int64_t m, int64_t n, int64_t k,
                                                    const C2<T> *__restrict__ A, int64_t lda,
                                                    const C2<T> *__restrict__ B, int64_t ldb,
                                                    C2<T> *__restrict__ C, int64_t ldc,
                                                    double2 alpha, double2 beta, int64_t kchunk,
                                                    C2<T> *__restrict__ part) {
  typedef C2<T> V2;
  typedef typename Mma<T>::acc Acc;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t row0 = (int64_t)blockIdx.x * BM, col0 = (int64_t)blockIdx.y * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (kbeg + kchunk < k) ? kbeg + kchunk : k;

  Acc acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = Acc{0, 0, 0, 0};
      acc_im[i][j] = Acc{0, 0, 0, 0};
    }

  V2 ra[4], rb[4];
  // Index maps: the thread-fastest index follows each operand's contiguous axis.
  auto a_idx = [&](int c, int *kk, int *i) {
    if (OPA == OP_N) {
      *kk = tid >> 4;
      *i = (tid & 15) + 16 * c;
    } else {
      *kk = tid & 15;
      *i = (tid >> 4) + 16 * c;
    }
  };
  auto b_idx = [&](int c, int *kk, int *j) {
    if (OPB == OP_N) {
      *kk = tid & 15;
      *j = (tid >> 4) + 16 * c;
    } else {
      *kk = tid >> 4;
      *j = (tid & 15) + 16 * c;
    }
  };
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int kk, i;
      a_idx(c, &kk, &i);
      const int64_t gr = row0 + i, gk = k0 + kk;
      ra[c] = V2{0, 0};
      if (gr < m && gk < kend) ra[c] = (OPA == OP_N) ? A[gr + gk * lda] : A[gk + gr * lda];
      int j;
      b_idx(c, &kk, &j);
      const int64_t gc = col0 + j, gk2 = k0 + kk;
      rb[c] = V2{0, 0};
      if (gc < n && gk2 < kend) rb[c] = (OPB == OP_N) ? B[gk2 + gc * ldb] : B[gc + gk2 * ldb];
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int kk, i;
      a_idx(c, &kk, &i);
      As[0][kk][i] = ra[c].x;
      As[1][kk][i] = (OPA == OP_C) ? -ra[c].y : ra[c].y;
      int j;
      b_idx(c, &kk, &j);
      Bs[0][kk][j] = rb[c].x;
      Bs[1][kk][j] = (OPB == OP_C) ? -rb[c].y : rb[c].y;
    }
  };

  if (kbeg < kend) load_tiles(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    store_tiles();
    __syncthreads();
    if (k0 + BK < kend) load_tiles(k0 + BK);
#pragma unroll
    for (int kq = 0; kq < BK / 4; ++kq) {
      const int kk = kq * 4 + (lane >> 4);
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int ii = wm * 32 + s * 16 + (lane & 15);
        ar[s] = As[0][kk][ii];
        ai[s] = As[1][kk][ii];
        const int jj = wn * 32 + s * 16 + (lane & 15);
        br[s] = Bs[0][kk][jj];
        bi[s] = Bs[1][kk][jj];
      }
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          acc_re[si][sj] = Mma<T>::run(ar[si], br[sj], acc_re[si][sj]);
          acc_im[si][sj] = Mma<T>::run(ar[si], bi[sj], acc_im[si][sj]);
        }
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          acc_re[si][sj] = Mma<T>::run(-ai[si], bi[sj], acc_re[si][sj]);
          acc_im[si][sj] = Mma<T>::run(ai[si], br[sj], acc_im[si][sj]);
        }
    }
    __syncthreads();
  }

  const bool use_beta = (beta.x != 0.0 || beta.y != 0.0);
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wm * 32 + si * 16 + Mma<T>::row(lane, r);
        const int64_t col = col0 + wn * 32 + sj * 16 + (lane & 15);
        if (row < m && col < n) {
          const V2 v{acc_re[si][sj][r], acc_im[si][sj][r]};
          if (SPLIT) {
            part[(int64_t)blockIdx.z * m * n + row + col * m] = v;
          } else {
            const V2 al{(T)alpha.x, (T)alpha.y};
            V2 o = cmul(al, v);
            if (use_beta) o = cadd(o, cmul(V2{(T)beta.x, (T)beta.y}, C[row + col * ldc]));
            C[row + col * ldc] = o;
          }
        }
      }
}

__global__ void zsum_parts_kernel(int64_t m, int64_t n, const double2 *__restrict__ part,
                                  int splits, double2 *__restrict__ C, int64_t ldc, double2 alpha,
                                  double2 beta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t row = idx % m, col = idx / m;
  double2 s{0, 0};
  for (int z = 0; z < splits; ++z) s = cadd(s, part[(int64_t)z * m * n + idx]);
  double2 o = cmul(alpha, s);
  if (beta.x != 0.0 || beta.y != 0.0) o = cadd(o, cmul(beta, C[row + col * ldc]));
  C[row + col * ldc] = o;
}

template <typename T, int OPA, int OPB, int TAG>
void launch_t(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
              int64_t ldb, void *C, int64_t ldc, double2 alpha, double2 beta, hipStream_t st,
              void *part, int splits) {
  typedef C2<T> V2;
  const int64_t chunk = part ? ((k + splits - 1) / splits + BK - 1) / BK * BK : k;
  // every chunk index gets launched; a chunk past the end of K writes zeros
  const int zs = part ? splits : 1;
  dim3 grid((unsigned)((m + BM - 1) / BM), (unsigned)((n + BN - 1) / BN), (unsigned)zs);
  if (part) {
    hipLaunchKernelGGL((zgemm_kernel<T, OPA, OPB, true, TAG>), grid, dim3(256), 0, st, m, n, k,
                       (const V2 *)A, lda, (const V2 *)B, ldb, (V2 *)C, ldc, alpha, beta, chunk,
                       (V2 *)part);
  } else {
    hipLaunchKernelGGL((zgemm_kernel<T, OPA, OPB, false, TAG>), grid, dim3(256), 0, st, m, n, k,
                       (const V2 *)A, lda, (const V2 *)B, ldb, (V2 *)C, ldc, alpha, beta, chunk,
                       (V2 *)nullptr);
  }
  CHEBFI_HIP(hipGetLastError());
}

}  // namespace

int zgemm_splits(int64_t m, int64_t n, int64_t k) {
  const int64_t tiles = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
  int64_t s = (1024 + tiles - 1) / tiles;
  const int64_t kmax = (k + 511) / 512;  // keep at least ~512 K per chunk
  if (s > kmax) s = kmax;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

void zgemm(Op opa, Op opb, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
           const void *B, int64_t ldb, void *C, int64_t ldc, double2 alpha, double2 beta,
           hipStream_t st, void *part, int splits) {
  if (m <= 0 || n <= 0) return;
  if (opa == OP_N && opb == OP_N)
    launch_t<double, OP_N, OP_N, 0>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, st, part, splits);
  else if (opa == OP_C && opb == OP_N)
    launch_t<double, OP_C, OP_N, 0>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, st, part, splits);
  else if (opa == OP_N && opb == OP_C)
    launch_t<double, OP_N, OP_C, 0>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, st, part, splits);
  else
    launch_t<double, OP_C, OP_C, 0>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, st, part, splits);
}

void proj_gemm(int64_t nproj, int64_t nband, int64_t npw, const void *P, const void *X,
               int64_t ldx, void *part, int splits, hipStream_t st, bool fp32) {
  if (fp32)
    launch_t<float, OP_C, OP_N, 1>(nproj, nband, npw, P, npw, X, ldx, nullptr, 0, double2{1, 0},
                                   double2{0, 0}, st, part, splits);
  else
    launch_t<double, OP_C, OP_N, 1>(nproj, nband, npw, P, npw, X, ldx, nullptr, 0, double2{1, 0},
                                    double2{0, 0}, st, part, splits);
}

void expand_gemm(int64_t npw, int64_t nband, int64_t nproj, const void *P, const void *Cp,
                 void *Out, int64_t ldo, hipStream_t st, bool fp32) {
  if (fp32)
    launch_t<float, OP_N, OP_N, 1>(npw, nband, nproj, P, npw, Cp, nproj, Out, ldo, double2{1, 0},
                                   double2{1, 0}, st, nullptr, 1);
  else
    launch_t<double, OP_N, OP_N, 1>(npw, nband, nproj, P, npw, Cp, nproj, Out, ldo, double2{1, 0},
                                    double2{1, 0}, st, nullptr, 1);
}

namespace {

// c[j] = sum_i conj(P[i, j]) x[i]: one workgroup per projector (single band).
__global__ __launch_bounds__(256) void proj_gemv_kernel(int64_t npw, const double2 *__restrict__ P,
                                                        const double2 *__restrict__ x,
                                                        double2 *__restrict__ c) {
  __shared__ double sr[4], si[4];
  const int64_t j = blockIdx.x;
  const double2 *p = P + j * npw;
  double re = 0, im = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 a = p[i], b = x[i];
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sr[threadIdx.x >> 6] = re;
    si[threadIdx.x >> 6] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) c[j] = double2{sr[0] + sr[1] + sr[2] + sr[3], si[0] + si[1] + si[2] + si[3]};
}

// out[i] += sum_j P[i, j] c[j]: one thread per plane wave (single band).
__global__ __launch_bounds__(256) void expand_gemv_kernel(int64_t npw, int nproj,
                                                          const double2 *__restrict__ P,
                                                          const double2 *__restrict__ c,
                                                          double2 *__restrict__ out) {
  extern __shared__ double2 cs[];
  for (int j = threadIdx.x; j < nproj; j += blockDim.x) cs[j] = c[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npw) return;
  double2 s = out[i];
  for (int j = 0; j < nproj; ++j) s = cadd(s, cmul(P[i + (int64_t)j * npw], cs[j]));
  out[i] = s;
}

}  // namespace

void proj_gemv(int64_t npw, int nproj, const void *P, const void *x, void *c, hipStream_t st) {
  hipLaunchKernelGGL(proj_gemv_kernel, dim3((unsigned)nproj), dim3(256), 0, st, npw,
                     (const double2 *)P, (const double2 *)x, (double2 *)c);
  CHEBFI_HIP(hipGetLastError());
}

void expand_gemv(int64_t npw, int nproj, const void *P, const void *c, void *out, hipStream_t st) {
  hipLaunchKernelGGL(expand_gemv_kernel, dim3((unsigned)((npw + 255) / 256)), dim3(256),
                     sizeof(double2) * (size_t)nproj, st, npw, nproj, (const double2 *)P,
                     (const double2 *)c, (double2 *)out);
  CHEBFI_HIP(hipGetLastError());
}

void zsum_parts(int64_t m, int64_t n, const void *part, int splits, void *C, int64_t ldc,
                double2 alpha, double2 beta, hipStream_t st) {
  const int64_t total = m * n;
  if (total <= 0) return;
  hipLaunchKernelGGL(zsum_parts_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     m, n, (const double2 *)part, splits, (double2 *)C, ldc, alpha, beta);
  CHEBFI_HIP(hipGetLastError());
}

}  // namespace chebfi
