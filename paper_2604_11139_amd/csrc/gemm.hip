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
#include <algorithm>
#include <type_traits>

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

// Tile (ti, tj), ti <= tj, of the t-th upper-triangle tile in column order
// (t = tj (tj + 1) / 2 + ti).
__device__ __forceinline__ void upper_tile(int64_t t, int64_t &ti, int64_t &tj) {
  int64_t j = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  while (j * (j + 1) / 2 > t) --j;
  tj = j;
  ti = t - j * (j + 1) / 2;
}

// TAG only separates instantiations (1 = projector products of the H
// application) so that kernel traces report them apart from the dense ones.
// TRI: square product known to be Hermitian; the 1-D grid enumerates only the
// tiles on and above the diagonal (the split-K sum mirrors the rest).
template <typename T, int OPA, int OPB, bool SPLIT, int TAG, bool TRI = false>
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
  int64_t row0 = (int64_t)blockIdx.x * BM, col0 = (int64_t)blockIdx.y * BN;
  if constexpr (TRI) {
    static_assert(BM == BN, "square tiles");
    int64_t ti, tj;
    upper_tile(blockIdx.x, ti, tj);
    row0 = ti * BM;
    col0 = tj * BN;
  }
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
          acc_re[si][sj] = Mma<T>::run(br[sj], ar[si], acc_re[si][sj]);
          acc_im[si][sj] = Mma<T>::run(bi[sj], ar[si], acc_im[si][sj]);
        }
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          acc_re[si][sj] = Mma<T>::run(bi[sj], -ai[si], acc_re[si][sj]);
          acc_im[si][sj] = Mma<T>::run(br[sj], ai[si], acc_im[si][sj]);
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
        // transposed tile (B operand first): 16 lanes hold 16 consecutive rows
        const int64_t row = row0 + wm * 32 + si * 16 + (lane & 15);
        const int64_t col = col0 + wn * 32 + sj * 16 + Mma<T>::row(lane, r);
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

// Hermitian split-K sum: 32 x 32 blocks (bi <= bj) of the m x m parts are
// summed and written, and their conjugate transposes written to (bj, bi)
// through LDS, so that C is exactly Hermitian and only parts of tiles on and
// above the diagonal are read.
__global__ __launch_bounds__(256) void zsum_herm_kernel(int64_t m, const double2 *__restrict__ part,
                                                        int splits, double2 *__restrict__ C,
                                                        int64_t ldc) {
  __shared__ double2 t[32][33];
  int64_t bi, bj;
  upper_tile(blockIdx.x, bi, bj);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int c = ty; c < 32; c += 8) {
    const int64_t row = bi * 32 + tx, col = bj * 32 + c;
    double2 v{0, 0};
    if (row < m && col < m) {
      for (int z = 0; z < splits; ++z) v = cadd(v, part[(int64_t)z * m * m + row + col * m]);
      if (bi < bj || tx <= c) C[row + col * ldc] = v;
    }
    t[c][tx] = v;  // element (bi*32 + tx, bj*32 + c)
  }
  __syncthreads();
  for (int c = ty; c < 32; c += 8) {
    const int64_t row = bj * 32 + tx, col = bi * 32 + c;  // mirror of (col, row)
    if (row < m && col < m && (bi < bj || tx > c)) {
      const double2 v = t[tx][c];
      C[row + col * ldc] = double2{v.x, -v.y};
    }
  }
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

// Compute units of the current device (cached per device).
static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v <= 0)
      v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

// Split-K count for `tiles` output tiles when `per_cu` workgroups fit on a CU:
// the launch runs in ceil(tiles * s / slots) rounds of slots = CUs x per_cu
// workgroups, each 1/s of the K range long, so s minimises ceil(tiles s / slots) / s
// (the tail round of a launch that does not fill the chip costs a whole round),
// with at least 4 workgroups per slot-round in total and at most kmax chunks.
static int best_splits(int64_t tiles, int64_t kmax, int per_cu) {
  const int64_t slots = (int64_t)device_cus() * per_cu;
  if (kmax < 1) kmax = 1;
  const int64_t smax = std::min<int64_t>(64, kmax);
  int64_t best = 1;
  double best_cost = 1e300;
  for (int64_t sp = 1; sp <= smax; ++sp) {
    const int64_t wgs = tiles * sp;
    const double cost = (double)((wgs + slots - 1) / slots) / (double)sp;
    // prefer fewer chunks unless a larger count is clearly better (fewer partials)
    if (cost < best_cost * (1.0 - 1e-9)) {
      best_cost = cost;
      best = sp;
    }
    if (wgs >= 8 * slots) break;
  }
  return (int)best;
}

int zgemm_herm_splits(int64_t m, int64_t k) {
  const int64_t nt = (m + BM - 1) / BM;
  return best_splits(nt * (nt + 1) / 2, (k + 511) / 512, 2);
}

void zgemm_herm(int64_t m, int64_t k, const void *A, int64_t lda, const void *B, int64_t ldb,
                void *C, int64_t ldc, hipStream_t st, void *part, int splits) {
  if (m <= 0) return;
  CHEBFI_REQUIRE(part != nullptr && splits >= 1, ABI_ERR_ARG, "Hermitian product needs parts");
  const int64_t nt = (m + BM - 1) / BM;
  const int64_t chunk = ((k + splits - 1) / splits + BK - 1) / BK * BK;
  hipLaunchKernelGGL((zgemm_kernel<double, OP_C, OP_N, true, 0, true>),
                     dim3((unsigned)(nt * (nt + 1) / 2), 1, (unsigned)splits), dim3(256), 0, st, m,
                     m, k, (const double2 *)A, lda, (const double2 *)B, ldb, (double2 *)nullptr,
                     (int64_t)0, double2{1, 0}, double2{0, 0}, chunk, (double2 *)part);
  CHEBFI_HIP(hipGetLastError());
  const int64_t nb = (m + 31) / 32;
  hipLaunchKernelGGL(zsum_herm_kernel, dim3((unsigned)(nb * (nb + 1) / 2)), dim3(256), 0, st, m,
                     (const double2 *)part, splits, (double2 *)C, ldc);
  CHEBFI_HIP(hipGetLastError());
}

int zgemm_splits(int64_t m, int64_t n, int64_t k) {
  const int64_t tiles = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
  // keep at least ~512 K per chunk; two 256-thread workgroups per CU (66 KB LDS each)
  return best_splits(tiles, (k + 511) / 512, 2);
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

namespace {

// ---- split-BF16 complex GEMM (mixed form) ------------------------------------
// Each real operand x is carried as hi = bf16(x), lo = bf16(x - hi) and every
// real product as hi*hi + hi*lo + lo*hi, accumulated in FP32 (the bf16x3
// method of Henry, Tang and Heinecke, ARITH 2019; relative error ~2^-16).
// A is given as four bf16 planes (Re hi, Im hi, Re lo, Im lo), row-major with
// the contraction index contiguous; B is complex float, column-major, split
// while it is staged into LDS.  CONJ selects op(A) = A^H (the projection
// P^H Y, with A holding the rows of P^T) instead of A.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

constexpr int XBM = 64, XBN = 64, XBK = 32, XPAD = 8;

__device__ __forceinline__ u16 bf16_rn(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf16_val(u16 h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ v4f mfma_bf16(const v8bf &a, const v8bf &b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <bool CONJ, bool SPLIT>
__global__ __launch_bounds__(256) void zgemm_bf16x3_kernel(
    int64_t m, int64_t n, int64_t k, const u16 *__restrict__ Apl, int64_t lda, int64_t pstride,
    const float2 *__restrict__ B, int64_t ldb, float2 *__restrict__ C, int64_t ldc,
    int64_t kchunk, float2 *__restrict__ part) {
  __shared__ __align__(16) u16 As[4][XBM][XBK + XPAD];
  __shared__ __align__(16) u16 Bs[4][XBN][XBK + XPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t row0 = (int64_t)blockIdx.x * XBM, col0 = (int64_t)blockIdx.y * XBN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (kbeg + kchunk < k) ? kbeg + kchunk : k;

  v4f acc[2][2][4];  // [si][sj][rr, ii, ri, ir]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[i][j][q] = v4f{0, 0, 0, 0};

  uint4 ra[4];
  float2 rb[8];
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int idx = tid + 256 * c;
      const int kc = idx & 3, i = (idx >> 2) & 63, p = idx >> 8;
      const int64_t gr = row0 + i, ks = k0 + 8 * kc;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gr < m && ks < kend) {
        const u16 *src = Apl + (int64_t)p * pstride + gr * lda + ks;
        if (ks + 8 <= kend) {
          v = *reinterpret_cast<const uint4 *>(src);
        } else {
          u16 t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          for (int e = 0; e < 8 && ks + e < kend; ++e) t[e] = src[e];
          v = make_uint4(t[0] | ((unsigned)t[1] << 16), t[2] | ((unsigned)t[3] << 16),
                         t[4] | ((unsigned)t[5] << 16), t[6] | ((unsigned)t[7] << 16));
        }
      }
      ra[c] = v;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int idx = tid + 256 * c;
      const int kk = idx & 31, j = idx >> 5;
      const int64_t gc = col0 + j, gk = k0 + kk;
      rb[c] = (gc < n && gk < kend) ? B[gk + gc * ldb] : float2{0.f, 0.f};
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int idx = tid + 256 * c;
      const int kc = idx & 3, i = (idx >> 2) & 63, p = idx >> 8;
      *reinterpret_cast<uint4 *>(&As[p][i][8 * kc]) = ra[c];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int idx = tid + 256 * c;
      const int kk = idx & 31, j = idx >> 5;
      const u16 hr = bf16_rn(rb[c].x), hi = bf16_rn(rb[c].y);
      Bs[0][j][kk] = hr;
      Bs[1][j][kk] = hi;
      Bs[2][j][kk] = bf16_rn(rb[c].x - bf16_val(hr));
      Bs[3][j][kk] = bf16_rn(rb[c].y - bf16_val(hi));
    }
  };

  if (kbeg < kend) load_tiles(kbeg);
  const int kb = 8 * (lane >> 4);
  for (int64_t k0 = kbeg; k0 < kend; k0 += XBK) {
    store_tiles();
    __syncthreads();
    if (k0 + XBK < kend) load_tiles(k0 + XBK);
    v8bf a[2][4], b[2][4];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int ii = wm * 32 + s2 * 16 + (lane & 15);
      const int jj = wn * 32 + s2 * 16 + (lane & 15);
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        a[s2][p] = *reinterpret_cast<const v8bf *>(&As[p][ii][kb]);
        b[s2][p] = *reinterpret_cast<const v8bf *>(&Bs[p][jj][kb]);
      }
    }
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) {
        // planes: 0 Re hi, 1 Im hi, 2 Re lo, 3 Im lo
        v4f *q = acc[si][sj];
        q[0] = mfma_bf16(a[si][0], b[sj][0], q[0]);
        q[1] = mfma_bf16(a[si][1], b[sj][1], q[1]);
        q[2] = mfma_bf16(a[si][0], b[sj][1], q[2]);
        q[3] = mfma_bf16(a[si][1], b[sj][0], q[3]);
        q[0] = mfma_bf16(a[si][0], b[sj][2], q[0]);
        q[1] = mfma_bf16(a[si][1], b[sj][3], q[1]);
        q[2] = mfma_bf16(a[si][0], b[sj][3], q[2]);
        q[3] = mfma_bf16(a[si][1], b[sj][2], q[3]);
        q[0] = mfma_bf16(a[si][2], b[sj][0], q[0]);
        q[1] = mfma_bf16(a[si][3], b[sj][1], q[1]);
        q[2] = mfma_bf16(a[si][2], b[sj][1], q[2]);
        q[3] = mfma_bf16(a[si][3], b[sj][0], q[3]);
      }
    __syncthreads();
  }

#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wm * 32 + si * 16 + 4 * (lane >> 4) + r;
        const int64_t col = col0 + wn * 32 + sj * 16 + (lane & 15);
        if (row < m && col < n) {
          const float rr = acc[si][sj][0][r], ii = acc[si][sj][1][r];
          const float ri = acc[si][sj][2][r], ir = acc[si][sj][3][r];
          const float2 v = CONJ ? float2{rr + ii, ri - ir} : float2{rr - ii, ri + ir};
          if (SPLIT) {
            part[(int64_t)blockIdx.z * m * n + row + col * m] = v;
          } else {
            float2 o = C[row + col * ldc];
            o.x += v.x;
            o.y += v.y;
            C[row + col * ldc] = o;
          }
        }
      }
}

// Planes x planes form: both operands arrive as four bf16 planes with the
// contraction index contiguous (A rows, B columns), so every global load is a
// 16-byte vector and staging into LDS is a plain copy.  Tile BM x BN complex,
// NWM x NWN waves, K step 32.  Two accumulators per 16x16 complex tile: the
// sign of an imaginary plane is flipped in registers (bf16 sign bits), so
//   op(A) = A^H: Re += Ar Br + Ai Bi,   Im += Ar Bi + (-Ai) Br
//   op(A) = A  : Re += Ar Br + Ai (-Bi), Im += Ar Bi + Ai Br
// each real product being hi*hi + hi*lo + lo*hi.  Workgroups are numbered so
// that the tiles sharing an A panel run on the same XCD (consecutive
// workgroup ids go to different XCDs).
__device__ __forceinline__ v8bf bf16_neg(v8bf x) {
  typedef unsigned v4u __attribute__((ext_vector_type(4)));
  v4u u = __builtin_bit_cast(v4u, x);
  u ^= v4u{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(v8bf, u);
}

template <int BM, int BN, int NWM, int NWN, bool CONJ, bool SPLIT>
__global__ __launch_bounds__(64 * NWM * NWN) void zgemm_pl_kernel(
    int64_t m, int64_t n, int64_t k, const u16 *__restrict__ Apl, int64_t lda, int64_t psa,
    const u16 *__restrict__ Bpl, int64_t ldb, int64_t psb, float2 *__restrict__ C, int64_t ldc,
    int64_t kchunk, float2 *__restrict__ part, int accum) {
  constexpr int NT = 64 * NWM * NWN;
  constexpr int SM = BM / NWM / 16, SN = BN / NWN / 16;
  constexpr int CA = 16 * BM / NT, CB = 16 * BN / NT;  // 16-byte chunks per thread
  __shared__ __align__(16) u16 As[4][BM][XBK + XPAD];
  __shared__ __align__(16) u16 Bs[4][BN][XBK + XPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % NWM, wn = wave / NWM;
  // XCD-aware order: within the leading groups of 8 row panels, the column
  // tiles of one row panel get ids congruent mod 8 (same XCD); the remaining
  // row panels (fewer than 8) are numbered plainly.  A bijection on the grid.
  const unsigned ntn = gridDim.y, ntm = gridDim.x;
  const unsigned wid = blockIdx.x + ntm * blockIdx.y;
  const unsigned full = ntm & ~7u;
  unsigned tm, tn;
  if (wid < full * ntn) {
    const unsigned xcd = wid & 7u, loc = wid >> 3;
    tm = (loc / ntn) * 8u + xcd;
    tn = loc % ntn;
  } else {
    const unsigned r = wid - full * ntn, rest = ntm - full;
    tm = full + r % rest;
    tn = r / rest;
  }
  const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (kbeg + kchunk < k) ? kbeg + kchunk : k;

  v4f acc[SM][SN][2];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      acc[i][j][0] = v4f{0, 0, 0, 0};
      acc[i][j][1] = v4f{0, 0, 0, 0};
    }

  uint4 ra[CA], rb[CB];
  auto load_chunk = [&](const u16 *base, int64_t ld, int64_t ps, int64_t lim, int idx,
                        int64_t r0, int64_t k0) -> uint4 {
    const int kc = idx & 3, rr = (idx >> 2), i = rr >> 2;
    const int64_t gr = r0 + i, ks = k0 + 8 * kc;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (gr < lim && ks < kend) {
      const u16 *src = base + (int64_t)(rr & 3) * ps + gr * ld + ks;
      if (ks + 8 <= kend) {
        v = *reinterpret_cast<const uint4 *>(src);
      } else {
        u16 t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int e = 0; e < 8 && ks + e < kend; ++e) t[e] = src[e];
        v = make_uint4(t[0] | ((unsigned)t[1] << 16), t[2] | ((unsigned)t[3] << 16),
                       t[4] | ((unsigned)t[5] << 16), t[6] | ((unsigned)t[7] << 16));
      }
    }
    return v;
  };
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int c = 0; c < CA; ++c) ra[c] = load_chunk(Apl, lda, psa, m, tid + NT * c, row0, k0);
#pragma unroll
    for (int c = 0; c < CB; ++c) rb[c] = load_chunk(Bpl, ldb, psb, n, tid + NT * c, col0, k0);
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int idx = tid + NT * c, kc = idx & 3, rr = idx >> 2;
      *reinterpret_cast<uint4 *>(&As[rr & 3][rr >> 2][8 * kc]) = ra[c];
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int idx = tid + NT * c, kc = idx & 3, rr = idx >> 2;
      *reinterpret_cast<uint4 *>(&Bs[rr & 3][rr >> 2][8 * kc]) = rb[c];
    }
  };

  if (kbeg < kend) load_tiles(kbeg);
  const int kb = 8 * (lane >> 4);
  for (int64_t k0 = kbeg; k0 < kend; k0 += XBK) {
    store_tiles();
    __syncthreads();
    if (k0 + XBK < kend) load_tiles(k0 + XBK);
    // planes: 0 Re hi, 1 Im hi, 2 Re lo, 3 Im lo; slot 4/5: negated Im hi/lo
    v8bf a[SM][6], b[SN][6];
#pragma unroll
    for (int i = 0; i < SM; ++i) {
      const int ii = wm * (BM / NWM) + i * 16 + (lane & 15);
#pragma unroll
      for (int p = 0; p < 4; ++p) a[i][p] = *reinterpret_cast<const v8bf *>(&As[p][ii][kb]);
      if (CONJ) {
        a[i][4] = bf16_neg(a[i][1]);
        a[i][5] = bf16_neg(a[i][3]);
      }
    }
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      const int jj = wn * (BN / NWN) + j * 16 + (lane & 15);
#pragma unroll
      for (int p = 0; p < 4; ++p) b[j][p] = *reinterpret_cast<const v8bf *>(&Bs[p][jj][kb]);
      if (!CONJ) {
        b[j][4] = bf16_neg(b[j][1]);
        b[j][5] = bf16_neg(b[j][3]);
      }
    }
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        v4f re = acc[i][j][0], im = acc[i][j][1];
        // real part
        re = mfma_bf16(b[j][0], a[i][0], re);
        re = mfma_bf16(b[j][2], a[i][0], re);
        re = mfma_bf16(b[j][0], a[i][2], re);
        if (CONJ) {
          re = mfma_bf16(b[j][1], a[i][1], re);
          re = mfma_bf16(b[j][3], a[i][1], re);
          re = mfma_bf16(b[j][1], a[i][3], re);
        } else {
          re = mfma_bf16(b[j][4], a[i][1], re);
          re = mfma_bf16(b[j][5], a[i][1], re);
          re = mfma_bf16(b[j][4], a[i][3], re);
        }
        // imaginary part
        im = mfma_bf16(b[j][1], a[i][0], im);
        im = mfma_bf16(b[j][3], a[i][0], im);
        im = mfma_bf16(b[j][1], a[i][2], im);
        if (CONJ) {
          im = mfma_bf16(b[j][0], a[i][4], im);
          im = mfma_bf16(b[j][2], a[i][4], im);
          im = mfma_bf16(b[j][0], a[i][5], im);
        } else {
          im = mfma_bf16(b[j][0], a[i][1], im);
          im = mfma_bf16(b[j][2], a[i][1], im);
          im = mfma_bf16(b[j][0], a[i][3], im);
        }
        acc[i][j][0] = re;
        acc[i][j][1] = im;
      }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // the MFMA computed the transposed tile (B operand first): lane & 15
        // indexes rows, so 16 lanes store 16 consecutive rows of a column
        const int64_t row = row0 + wm * (BM / NWM) + i * 16 + (lane & 15);
        const int64_t col = col0 + wn * (BN / NWN) + j * 16 + 4 * (lane >> 4) + r;
        if (row < m && col < n) {
          const float2 v{acc[i][j][0][r], acc[i][j][1][r]};
          if (SPLIT) {
            part[(int64_t)blockIdx.z * m * n + row + col * m] = v;
          } else {
            if (accum) {
              float2 o = C[row + col * ldc];
              o.x += v.x;
              o.y += v.y;
              C[row + col * ldc] = o;
            } else {
              C[row + col * ldc] = v;
            }
          }
        }
      }
}

// Tile of this workgroup in the grid (tiles along x = rows, y = columns,
// z = K chunks).  Workgroups are handed to the eight XCDs round robin by linear
// id, so the first 8*floor(T/8) ids are remapped to give each XCD one
// contiguous range of a linear tile order (the rest keep their id).  That order
// runs over K chunks slowest, then over groups of `gm` row panels; within a
// group the row panel varies fastest, then the column.  The workgroups an XCD
// runs together then share a few A and B panels in its L2.
__device__ __forceinline__ void grouped_tile(unsigned gm, unsigned &tm, unsigned &tn,
                                             unsigned &tz) {
  const unsigned ntm = gridDim.x, ntn = gridDim.y;
  const unsigned lid = blockIdx.x + ntm * (blockIdx.y + ntn * blockIdx.z);
  const unsigned q = (ntm * ntn * gridDim.z) >> 3;
  const unsigned L = lid < 8u * q ? (lid & 7u) * q + (lid >> 3) : lid;
  const unsigned per_z = ntm * ntn;
  tz = L / per_z;
  const unsigned r = L - tz * per_z;
  const unsigned g = r / (gm * ntn);
  const unsigned rows = min(gm, ntm - g * gm);
  const unsigned rr = r - g * gm * ntn;
  tm = g * gm + rr % rows;
  tn = rr / rows;
}

// Double-buffered form of the planes x planes kernel: two LDS stages of
// 32-element K slices without padding; the 16-byte chunk kc of row i is
// stored at chunk position kc ^ ((i >> 1) & 3).  With that swizzle the
// 128-bit fragment reads (16 rows x 4 chunks per wave) and the staging
// writes (four lanes per row, consecutive rows of one plane) are free of
// bank conflicts on gfx950 (measured with the LDS conflict counters).  One
// barrier per K step: the next slice is written into the other stage while
// this one is multiplied.
template <int BM, int BN, int NWM, int NWN, bool CONJ, bool SPLIT, int DEPTH, bool BF32 = false>
__global__ __launch_bounds__(64 * NWM * NWN, 2) void zgemm_pl2_kernel(
    int64_t m, int64_t n, int64_t k, const u16 *__restrict__ Apl, int64_t lda, int64_t psa,
    const u16 *__restrict__ Bpl, int64_t ldb, int64_t psb, float2 *__restrict__ C, int64_t ldc,
    int64_t kchunk, float2 *__restrict__ part, int accum) {
  constexpr int NT = 64 * NWM * NWN;
  constexpr int SM = BM / NWM / 16, SN = BN / NWN / 16;
  constexpr int CA = 16 * BM / NT, CB = 16 * BN / NT;
  constexpr int NST = DEPTH == 0 ? 1 : 2;  // LDS stages
  __shared__ __align__(16) u16 As[NST][4][BM][XBK];
  __shared__ __align__(16) u16 Bs[NST][4][BN][XBK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % NWM, wn = wave / NWM;
  unsigned tm, tn, tz;
  grouped_tile(SPLIT ? gridDim.x : 4u, tm, tn, tz);
  const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
  const int64_t kbeg = (int64_t)tz * kchunk;
  const int64_t kend = (kbeg + kchunk < k) ? kbeg + kchunk : k;

  v4f acc[SM][SN][2];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      acc[i][j][0] = v4f{0, 0, 0, 0};
      acc[i][j][1] = v4f{0, 0, 0, 0};
    }

  uint4 ra[DEPTH == 0 ? 1 : DEPTH][CA], rb[DEPTH == 0 ? 1 : DEPTH][CB];
  // chunk idx of a staged slice with R rows: K chunk idx & 3, row
  // (idx >> 2) % R, plane (idx >> 2) / R
  auto load_chunk = [&](const u16 *base, int64_t ld, int64_t ps, int64_t lim, int idx,
                        int64_t r0, int64_t k0, int R) -> uint4 {
    const int kc = idx & 3, i = (idx >> 2) % R, pl = (idx >> 2) / R;
    const int64_t gr = r0 + i, ks = k0 + 8 * kc;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (gr < lim && ks < kend) {
      const u16 *src = base + (int64_t)pl * ps + gr * ld + ks;
      if (ks + 8 <= kend) {
        v = *reinterpret_cast<const uint4 *>(src);
      } else {
        u16 t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int e = 0; e < 8 && ks + e < kend; ++e) t[e] = src[e];
        v = make_uint4(t[0] | ((unsigned)t[1] << 16), t[2] | ((unsigned)t[3] << 16),
                       t[4] | ((unsigned)t[5] << 16), t[6] | ((unsigned)t[7] << 16));
      }
    }
    return v;
  };
  // BF32: B is a complex float block (column j = band j, ld ldb in complex
  // elements) split into its bf16 planes while staged.  Super-chunk sidx covers
  // 8 consecutive K elements (kc = sidx & 3) of row sidx >> 2 and is held raw
  // in four uint4 of rb.
  constexpr int CBF = 4 * BN / NT;
  static_assert(!BF32 || 4 * CBF == CB, "raw super-chunks must fill the B registers");
  auto load_b32 = [&](int r, int c, int64_t k0) {
    const int sidx = tid + NT * c, kc = sidx & 3, i = sidx >> 2;
    const int64_t gr = col0 + i, ks = k0 + 8 * kc;
    uint2 t[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = make_uint2(0, 0);
    if (gr < n && ks < kend) {
      const uint2 *src = reinterpret_cast<const uint2 *>(Bpl) + gr * ldb + ks;
      if (ks + 8 <= kend) {
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = src[e];
      } else {
        for (int e = 0; e < 8 && ks + e < kend; ++e) t[e] = src[e];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      rb[r][4 * c + q] = make_uint4(t[2 * q].x, t[2 * q].y, t[2 * q + 1].x, t[2 * q + 1].y);
  };
  auto load_tiles = [&](int r, int64_t k0) {
#pragma unroll
    for (int c = 0; c < CA; ++c)
      ra[r][c] = load_chunk(Apl, lda, psa, m, tid + NT * c, row0, k0, BM);
    if constexpr (BF32) {
#pragma unroll
      for (int c = 0; c < CBF; ++c) load_b32(r, c, k0);
    } else {
#pragma unroll
      for (int c = 0; c < CB; ++c)
        rb[r][c] = load_chunk(Bpl, ldb, psb, n, tid + NT * c, col0, k0, BN);
    }
  };
  auto store_tiles = [&](int r, int st) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int idx = tid + NT * c, kc = idx & 3, i = (idx >> 2) % BM, pl = (idx >> 2) / BM;
      *reinterpret_cast<uint4 *>(&As[st][pl][i][8 * (kc ^ ((i >> 1) & 3))]) = ra[r][c];
    }
    if constexpr (BF32) {
#pragma unroll
      for (int c = 0; c < CBF; ++c) {
        const int sidx = tid + NT * c, kc = sidx & 3, i = sidx >> 2;
        unsigned w[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint4 u = rb[r][4 * c + q];
          const float re0 = __uint_as_float(u.x), im0 = __uint_as_float(u.y);
          const float re1 = __uint_as_float(u.z), im1 = __uint_as_float(u.w);
          const u16 hr0 = bf16_rn(re0), hi0 = bf16_rn(im0), hr1 = bf16_rn(re1),
                    hi1 = bf16_rn(im1);
          w[0][q] = hr0 | ((unsigned)hr1 << 16);
          w[1][q] = hi0 | ((unsigned)hi1 << 16);
          w[2][q] = bf16_rn(re0 - bf16_val(hr0)) | ((unsigned)bf16_rn(re1 - bf16_val(hr1)) << 16);
          w[3][q] = bf16_rn(im0 - bf16_val(hi0)) | ((unsigned)bf16_rn(im1 - bf16_val(hi1)) << 16);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
          *reinterpret_cast<uint4 *>(&Bs[st][p][i][8 * (kc ^ ((i >> 1) & 3))]) =
              make_uint4(w[p][0], w[p][1], w[p][2], w[p][3]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int idx = tid + NT * c, kc = idx & 3, i = (idx >> 2) % BN, pl = (idx >> 2) / BN;
        *reinterpret_cast<uint4 *>(&Bs[st][pl][i][8 * (kc ^ ((i >> 1) & 3))]) = rb[r][c];
      }
    }
  };

  const int kq = lane >> 4;
  // multiply-accumulate of the K slice held in LDS stage st
  auto mma = [&](int st) {
    // negated imaginary planes of A (a[4], a[5]) carry the minus signs of the
    // complex product in both forms, so B needs no negated copies
    v8bf b[SN][4];
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      const int jj = wn * (BN / NWN) + j * 16 + (lane & 15);
      const int kb = 8 * (kq ^ ((jj >> 1) & 3));
#pragma unroll
      for (int p = 0; p < 4; ++p) b[j][p] = *reinterpret_cast<const v8bf *>(&Bs[st][p][jj][kb]);
    }
#pragma unroll
    for (int i = 0; i < SM; ++i) {
      v8bf a[6];
      const int ii = wm * (BM / NWM) + i * 16 + (lane & 15);
      const int kb = 8 * (kq ^ ((ii >> 1) & 3));
#pragma unroll
      for (int p = 0; p < 4; ++p) a[p] = *reinterpret_cast<const v8bf *>(&As[st][p][ii][kb]);
      a[4] = bf16_neg(a[1]);
      a[5] = bf16_neg(a[3]);
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        v4f re = acc[i][j][0], im = acc[i][j][1];
        // Re: hi*hi + lo*hi + hi*lo of Re x Re, then -/+ Im x Im
        re = mfma_bf16(b[j][0], a[0], re);
        re = mfma_bf16(b[j][2], a[0], re);
        re = mfma_bf16(b[j][0], a[2], re);
        re = mfma_bf16(b[j][1], a[CONJ ? 1 : 4], re);
        re = mfma_bf16(b[j][3], a[CONJ ? 1 : 4], re);
        re = mfma_bf16(b[j][1], a[CONJ ? 3 : 5], re);
        // Im: Im(B) Re(A) then +/- Re(B) Im(A)
        im = mfma_bf16(b[j][1], a[0], im);
        im = mfma_bf16(b[j][3], a[0], im);
        im = mfma_bf16(b[j][1], a[2], im);
        im = mfma_bf16(b[j][0], a[CONJ ? 4 : 1], im);
        im = mfma_bf16(b[j][2], a[CONJ ? 4 : 1], im);
        im = mfma_bf16(b[j][0], a[CONJ ? 5 : 3], im);
        acc[i][j][0] = re;
        acc[i][j][1] = im;
      }
    }
  };

  if constexpr (DEPTH == 0) {
    // one LDS stage (so that two workgroups fit a CU): registers carry slice
    // k+1 while slice k is multiplied; two barriers per K step
    if (kbeg < kend) {
      load_tiles(0, kbeg);
      store_tiles(0, 0);
    }
    __syncthreads();
    for (int64_t k0 = kbeg; k0 < kend; k0 += XBK) {
      const bool more = k0 + XBK < kend;
      if (more) load_tiles(0, k0 + XBK);
      mma(0);
      __syncthreads();
      if (more) {
        store_tiles(0, 0);
        __syncthreads();
      }
    }
  } else if constexpr (DEPTH == 1) {
    // loads for slice k+1 are issued before slice k is multiplied
    int cur = 0;
    if (kbeg < kend) {
      load_tiles(0, kbeg);
      store_tiles(0, 0);
    }
    __syncthreads();
    for (int64_t k0 = kbeg; k0 < kend; k0 += XBK) {
      const bool more = k0 + XBK < kend;
      if (more) load_tiles(0, k0 + XBK);
      mma(cur);
      if (more) store_tiles(0, cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  } else {
    // two register sets: loads for slice k+2 are issued before slice k is
    // multiplied, and slice k+1 (loaded one step earlier) is staged after it
    if (kbeg < kend) {
      load_tiles(0, kbeg);
      store_tiles(0, 0);
    }
    if (kbeg + XBK < kend) load_tiles(1, kbeg + XBK);
    __syncthreads();
    for (int64_t k0 = kbeg; k0 < kend; k0 += 2 * XBK) {
      if (k0 + 2 * XBK < kend) load_tiles(0, k0 + 2 * XBK);
      mma(0);
      if (k0 + XBK < kend) store_tiles(1, 1);
      __syncthreads();
      if (k0 + XBK >= kend) break;
      if (k0 + 3 * XBK < kend) load_tiles(1, k0 + 3 * XBK);
      mma(1);
      if (k0 + 2 * XBK < kend) store_tiles(0, 0);
      __syncthreads();
    }
  }

#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wm * (BM / NWM) + i * 16 + (lane & 15);
        const int64_t col = col0 + wn * (BN / NWN) + j * 16 + 4 * (lane >> 4) + r;
        if (row < m && col < n) {
          const float2 v{acc[i][j][0][r], acc[i][j][1][r]};
          if (SPLIT) {
            part[(int64_t)tz * m * n + row + col * m] = v;
          } else {
            if (accum) {
              float2 o = C[row + col * ldc];
              o.x += v.x;
              o.y += v.y;
              C[row + col * ldc] = o;
            } else {
              C[row + col * ldc] = v;
            }
          }
        }
      }
}

// ---- split-BF16 products with direct global -> LDS staging -------------------
// gfx950's global_load_lds moves 4 or 16 bytes per lane from global memory
// straight into LDS (lane l's bytes land at the wave's LDS address + l * size).
// Staging a K slice then takes no VGPRs and no ds_write instructions: the waves
// issue the next slice's loads and go on multiplying the current one, and the
// only wait is one vmcnt before the barrier that ends the step.
//
// Operands.  A: four bf16 planes, rows = output rows, K contiguous (row stride
// lda, plane stride psa), zero beyond the true K up to kpad (a multiple of 32).
// B (PLANES): the same layout with rows = output columns.  B (BF32): a complex
// float block, column j = output column j, K contiguous (ld ldb); it is staged
// raw and split into its four bf16 planes when a wave reads its fragment
// (v_cvt_pk_bf16_f32: round to nearest even, the rounding of the planes of A).
// K indices at or beyond kdata are read at kdata - 1 (a finite value that
// meets a zero of A); rows and columns beyond m, n are read at m - 1, n - 1 and
// their results are not stored.  So no load leaves the operands' storage.
//
// LDS, one stage: A as [plane][row][32] bf16 with the 16-byte chunk kc of row i
// at position kc ^ ((i >> 1) & 3) (B planes alike); B32 as [column][32]
// complex float with the 16-byte chunk c (two complex) of column j at position
// c ^ b32_mask(j).  A column's 256 bytes span all 64 banks, so only the
// position separates the lanes of a fragment read; the LDS serves a 16-byte
// read for lanes 0-7 together with lanes 16-23 (and 8-15 with 24-31): eight
// columns at two adjacent K quarters, i.e. chunks differing in bit 2.  The
// mask leaves that bit alone and moves bit 2 of the column to bit 3, so those
// sixteen reads fill all sixteen positions.  Both layouts make the fragment
// reads free of bank conflicts.
__device__ __forceinline__ int b32_mask(int j) { return (j & 3) | ((j & 4) << 1); }
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
typedef float f2v_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void dma16(const void *g, unsigned char *lds) {
  __builtin_amdgcn_global_load_lds(g, (lds_void_t *)lds, 16, 0, 0);
}
__device__ __forceinline__ void dma4(const void *g, unsigned char *lds) {
  __builtin_amdgcn_global_load_lds(g, (lds_void_t *)lds, 4, 0, 0);
}
// s_waitcnt vmcnt(N) (gfx9 encoding: vmcnt[3:0] at bits 3:0, vmcnt[5:4] at
// bits 15:14; expcnt and lgkmcnt left at their maxima)
template <int N> __device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// x (two floats) -> hi = bf16(x), lo = bf16(x - hi), both round to nearest even
__device__ __forceinline__ void split2(f2v_t x, bf2_t &hi, bf2_t &lo) {
  hi = __builtin_convertvector(x, bf2_t);
  lo = __builtin_convertvector(x - __builtin_convertvector(hi, f2v_t), bf2_t);
}
__device__ __forceinline__ v8bf cat4(bf2_t a, bf2_t b, bf2_t c, bf2_t d) {
  typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
  const bf4_t ab = __builtin_shufflevector(a, b, 0, 1, 2, 3);
  const bf4_t cd = __builtin_shufflevector(c, d, 0, 1, 2, 3);
  return __builtin_shufflevector(ab, cd, 0, 1, 2, 3, 4, 5, 6, 7);
}

// ROLE only names the instantiation: 0 for the filter's projector products, 1
// for the Rayleigh-Ritz products (same code, told apart in kernel traces).
template <int BM, int BN, int NWM, int NWN, bool CONJ, bool SPLIT, bool BF32, bool PIPE = false,
          bool PERSIST = false, int ROLE = 0>
__global__ __launch_bounds__(64 * NWM * NWN) void zgemm_dl_kernel(
    int64_t m, int64_t n, int64_t kdata, const u16 *__restrict__ Apl, int64_t lda, int64_t psa,
    const void *__restrict__ Bsrc, int64_t ldb, int64_t psb, float2 *__restrict__ C,
    int64_t ldc, int64_t kchunk, int64_t kpad, float2 *__restrict__ part, int accum) {
  constexpr int NW = NWM * NWN;
  constexpr int SM = BM / NWM / 16, SN = BN / NWN / 16;
  constexpr int A_BYTES = 4 * BM * 64;                       // 4 planes x BM rows x 32 bf16
  constexpr int B_BYTES = BF32 ? BN * 256 : 4 * BN * 64;     // BN columns x 32 complex float
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int QA = BM / 4 / NW;                    // 1 KB loads (16 rows of a plane) per wave
  constexpr int QB = BF32 ? BN / NW : BN / 4 / NW;   // BF32: 256 B loads (one column) per wave
  static_assert(QA * 4 * NW == BM && (BF32 ? QB * NW == BN : QB * 4 * NW == BN), "tile / waves");
  static_assert(SM >= 1 && SN >= 1, "wave tile");
  // the two stages are separate LDS objects, so that the compiler can tell the
  // loads streaming into one stage from the fragment reads of the other (one
  // array indexed by the step parity would make it wait for the loads first)
  __shared__ __align__(16) unsigned char stage0[STAGE];
  __shared__ __align__(16) unsigned char stage1[STAGE];

  static_assert(!(PERSIST && SPLIT), "the persistent form writes whole products");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % NWM, wn = wave / NWM;
  // Tiles.  One tile per workgroup, or (PERSIST) a sequence of tiles per
  // workgroup: the grid holds 8 W workgroups (W per XCD, the hardware handing
  // workgroup ids to the XCDs round robin); round `it` gives XCD x the W
  // consecutive tiles starting at (8 it + x) W.  Tiles are numbered by blocks
  // of PR row panels, column panel major inside a block, so that W = 32
  // consecutive tiles cover 4 row x 8 column panels: the workgroups an XCD
  // runs together share 4 A and 8 B panels in its L2 (2 and 16 in row panel
  // major order).
  constexpr int PR = 4;
  const int ntm = (int)((m + BM - 1) / BM), ntn = (int)((n + BN - 1) / BN);
  const int ntiles = ntm * ntn;
  const int wpx = (int)(gridDim.x >> 3), xcd = (int)(blockIdx.x & 7), wj = (int)(blockIdx.x >> 3);
  auto tile_of = [&](int it) -> int { return (it * 8 + xcd) * wpx + wj; };
  // tile number -> (row panel, column panel)
  auto tile_rc = [&](int t, int &tm, int &tn) {
    const int b = t / (PR * ntn);
    const int h = ntm - b * PR < PR ? ntm - b * PR : PR;
    const int u = t - b * PR * ntn;
    tn = u / h;
    tm = b * PR + (u - tn * h);
  };
  int64_t row0, col0, kbeg = 0, kend, tzv = 0;
  if constexpr (PERSIST) {
    const int t = tile_of(0);
    if (t >= ntiles) return;
    int tm0, tn0;
    tile_rc(t, tm0, tn0);
    row0 = (int64_t)tm0 * BM;
    col0 = (int64_t)tn0 * BN;
    kend = kpad;
  } else {
    unsigned tm, tn, tz;
    grouped_tile(SPLIT ? gridDim.x : 4u, tm, tn, tz);
    row0 = (int64_t)tm * BM;
    col0 = (int64_t)tn * BN;
    tzv = tz;
    kbeg = (int64_t)tz * kchunk;
    kend = (kbeg + kchunk < kpad) ? kbeg + kchunk : kpad;
  }
  const int ns = kend > kbeg ? (int)((kend - kbeg) >> 5) : 0;

  // Load addresses: a wave-uniform base (scalar registers) plus a 32-bit lane
  // offset fixed for the tile.  Load q of A covers rows r0 .. r0 + 15 of plane
  // p; lane l its row r0 + (l >> 2) (clamped to m - 1) and 16-byte chunk
  // (l & 3) ^ ((row >> 1) & 3) (the same for every q, r0 being a multiple of
  // 16).  B planes alike.  B32: load q covers column c = wave QB + q (clamped
  // to n - 1; uniform), lane l the dword l & 3 of the 16-byte chunk at
  // position l >> 2, which holds chunk (l >> 2) ^ b32_mask(c) of the column.
  static_assert(!BF32 || QB % 8 == 0, "B32 lane patterns repeat every 8 columns");
  const int kcl = (lane & 3) ^ ((lane >> 3) & 3);
  // byte offsets of this lane's loads within the tile being loaded (rows and
  // columns past m, n read row m - 1 / column n - 1: their results are not
  // stored); set when the loads move to a new tile
  uint32_t aofs[QA];
  uint32_t bofs[BF32 ? 8 : QB];
  auto set_offsets = [&](int64_t r0t, int64_t c0t) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int64_t r = ((wave * QA + q) % (BM / 16)) * 16 + (lane >> 2);
      const int64_t rr = r0t + r < m ? r : m - 1 - r0t;
      aofs[q] = (uint32_t)(2 * (rr * lda + 8 * kcl));
    }
    if constexpr (BF32) {
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        const int ch = (lane >> 2) ^ b32_mask(c8), w = lane & 3;
        bofs[c8] = (uint32_t)(4 * (2 * (2 * ch + (w >> 1)) + (w & 1)));
      }
    } else {
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int64_t r = ((wave * QB + q) % (BN / 16)) * 16 + (lane >> 2);
        const int64_t rr = c0t + r < n ? r : n - 1 - c0t;
        bofs[q] = (uint32_t)(2 * (rr * ldb + 8 * kcl));
      }
    }
  };
  set_offsets(row0, col0);
  // (uniform base + zero-extended 32-bit byte offset: the scalar-base form of
  // the load instruction).  TAIL: a B32 slice reaching past the data reads the
  // last complex of the column for K indices past it (meeting zeros of A).
  auto issue_k = [&](int64_t r0t, int64_t c0t, int64_t k0, unsigned char *st, auto tail_c) {
    constexpr bool TAIL = decltype(tail_c)::value;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int qq = wave * QA + q, p = qq / (BM / 16), r0 = (qq % (BM / 16)) * 16;
      const char *base = (const char *)(Apl + (int64_t)p * psa + r0t * lda + k0);
      dma16(base + aofs[q], st + p * BM * 64 + r0 * 64);
    }
    if constexpr (BF32) {
      const char *base = (const char *)((const float *)Bsrc + 2 * (c0t * ldb + k0));
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int c = wave * QB + q;
        const uint32_t cofs = (uint32_t)(8 * (c0t + c < n ? c : n - 1 - c0t) * ldb);
        uint32_t off = bofs[q & 7];
        if constexpr (TAIL) {
          if (k0 + (off >> 3) >= kdata) off = (uint32_t)(8 * (kdata - 1 - k0)) + (off & 4);
        }
        dma4(base + (cofs + off), st + A_BYTES + c * 256);
      }
    } else {
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int qq = wave * QB + q, p = qq / (BN / 16), r0 = (qq % (BN / 16)) * 16;
        const char *base = (const char *)((const u16 *)Bsrc + (int64_t)p * psb + c0t * ldb + k0);
        dma16(base + bofs[q], st + A_BYTES + p * BN * 64 + r0 * 64);
      }
    }
  };
  auto issue_t = [&](int64_t r0t, int64_t c0t, int s, unsigned char *st) {
    const int64_t k0 = kbeg + 32 * (int64_t)s;
    if (BF32 && k0 + 32 > kdata)
      issue_k(r0t, c0t, k0, st, std::integral_constant<bool, true>{});
    else
      issue_k(r0t, c0t, k0, st, std::integral_constant<bool, false>{});
  };
  auto issue = [&](int s, unsigned char *st) { issue_t(row0, col0, s, st); };

  // PIPE: the product's minus sign rides on a third accumulator (subtracted in
  // the epilogue) instead of negated planes, the A fragments of row block i + 1
  // are read while row block i is multiplied, and the reads are spread over
  // the MFMAs with scheduling groups
  constexpr int NACC = PIPE ? 3 : 2;
  v4f acc[SM][SN][NACC];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int c = 0; c < NACC; ++c) acc[i][j][c] = v4f{0, 0, 0, 0};

  const int kq = lane >> 4;
  auto b_frag = [&](const unsigned char *st, int j, v8bf *b) {
    const int jj = wn * (BN / NWN) + j * 16 + (lane & 15);
    if constexpr (BF32) {
      // eight complex of column jj (K 8 kq .. 8 kq + 7) -> four bf16 planes
      float4 q4[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int off = A_BYTES + jj * 256 + 16 * ((4 * kq + t) ^ b32_mask(jj));
        q4[t] = *reinterpret_cast<const float4 *>(st + off);
      }
      bf2_t rh[4], rl[4], ih[4], il[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        split2(f2v_t{q4[t].x, q4[t].z}, rh[t], rl[t]);
        split2(f2v_t{q4[t].y, q4[t].w}, ih[t], il[t]);
      }
      b[0] = cat4(rh[0], rh[1], rh[2], rh[3]);
      b[1] = cat4(ih[0], ih[1], ih[2], ih[3]);
      b[2] = cat4(rl[0], rl[1], rl[2], rl[3]);
      b[3] = cat4(il[0], il[1], il[2], il[3]);
    } else {
      const int kb = 16 * (kq ^ ((jj >> 1) & 3));
#pragma unroll
      for (int p = 0; p < 4; ++p)
        b[p] = *reinterpret_cast<const v8bf *>(st + (A_BYTES + p * BN * 64 + jj * 64 + kb));
    }
  };
  auto a_frag = [&](const unsigned char *st, int i, v8bf *a) {
    const int ii = wm * (BM / NWM) + i * 16 + (lane & 15);
    const int kb = 16 * (kq ^ ((ii >> 1) & 3));
#pragma unroll
    for (int p = 0; p < 4; ++p)
      a[p] = *reinterpret_cast<const v8bf *>(st + (p * BM * 64 + ii * 64 + kb));
  };
  auto mma = [&](const unsigned char *st) {
    v8bf b[SN][4];
#pragma unroll
    for (int j = 0; j < SN; ++j) b_frag(st, j, b[j]);
    if constexpr (PIPE) {
      v8bf a[2][4];
      a_frag(st, 0, a[0]);
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        if (i + 1 < SM) a_frag(st, i + 1, a[(i + 1) & 1]);
        const v8bf *ai = a[i & 1];
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          // planes 0 Re hi, 1 Im hi, 2 Re lo, 3 Im lo; acc 0 / 1 Re / Im with
          // plus signs, acc 2 the minus-signed product (Im A Im B for op(A) = A,
          // Im A Re B for op(A) = A^H)
          v4f re = acc[i][j][0], im = acc[i][j][1], ng = acc[i][j][2];
          re = mfma_bf16(b[j][0], ai[0], re);
          re = mfma_bf16(b[j][2], ai[0], re);
          re = mfma_bf16(b[j][0], ai[2], re);
          im = mfma_bf16(b[j][1], ai[0], im);
          im = mfma_bf16(b[j][3], ai[0], im);
          im = mfma_bf16(b[j][1], ai[2], im);
          if (CONJ) {
            re = mfma_bf16(b[j][1], ai[1], re);
            re = mfma_bf16(b[j][3], ai[1], re);
            re = mfma_bf16(b[j][1], ai[3], re);
            ng = mfma_bf16(b[j][0], ai[1], ng);
            ng = mfma_bf16(b[j][2], ai[1], ng);
            ng = mfma_bf16(b[j][0], ai[3], ng);
          } else {
            ng = mfma_bf16(b[j][1], ai[1], ng);
            ng = mfma_bf16(b[j][3], ai[1], ng);
            ng = mfma_bf16(b[j][1], ai[3], ng);
            im = mfma_bf16(b[j][0], ai[1], im);
            im = mfma_bf16(b[j][2], ai[1], im);
            im = mfma_bf16(b[j][0], ai[3], im);
          }
          acc[i][j][0] = re;
          acc[i][j][1] = im;
          acc[i][j][2] = ng;
        }
      }
      // order: the step's first fragments, then per row block the next block's
      // four reads spread over the first MFMAs, the conversions of BF32 B
      // fragments with the MFMAs
      constexpr int MF = 12 * SN;  // MFMAs per row block
      __builtin_amdgcn_sched_group_barrier(0x100, 4 * SN + 4, 0);
      if constexpr (BF32) {
        // the conversions of column block j + 1 run under the MFMAs of block j
        // in the first row block (about four VALU instructions per MFMA)
        __builtin_amdgcn_sched_group_barrier(0x002, 48, 0);
#pragma unroll
        for (int j = 0; j + 1 < SN; ++j)
#pragma unroll
          for (int r = 0; r < 12; ++r) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
          }
      }
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        if (BF32 && i == 0 && SM > 1) {
          // last column block of the first row block, with the next A reads
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          }
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        } else if (i + 1 < SM) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          }
          __builtin_amdgcn_sched_group_barrier(0x008, MF - 8, 0);
        } else {
          __builtin_amdgcn_sched_group_barrier(0x008, MF, 0);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        v8bf a[6];
        a_frag(st, i, a);
        a[4] = bf16_neg(a[1]);
        a[5] = bf16_neg(a[3]);
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          v4f re = acc[i][j][0], im = acc[i][j][1];
          re = mfma_bf16(b[j][0], a[0], re);
          re = mfma_bf16(b[j][2], a[0], re);
          re = mfma_bf16(b[j][0], a[2], re);
          re = mfma_bf16(b[j][1], a[CONJ ? 1 : 4], re);
          re = mfma_bf16(b[j][3], a[CONJ ? 1 : 4], re);
          re = mfma_bf16(b[j][1], a[CONJ ? 3 : 5], re);
          im = mfma_bf16(b[j][1], a[0], im);
          im = mfma_bf16(b[j][3], a[0], im);
          im = mfma_bf16(b[j][1], a[2], im);
          im = mfma_bf16(b[j][0], a[CONJ ? 4 : 1], im);
          im = mfma_bf16(b[j][2], a[CONJ ? 4 : 1], im);
          im = mfma_bf16(b[j][0], a[CONJ ? 5 : 3], im);
          acc[i][j][0] = re;
          acc[i][j][1] = im;
        }
      }
    }
  };

  // two stages: slice s + 1 streams into the other stage while slice s is
  // multiplied; the barrier after the wait both publishes slice s + 1 and
  // frees the stage that slice s + 2 will overwrite
  auto epilogue = [&](int64_t row0, int64_t col0) {
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int j = 0; j < SN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + wm * (BM / NWM) + i * 16 + (lane & 15);
          const int64_t col = col0 + wn * (BN / NWN) + j * 16 + 4 * (lane >> 4) + r;
          if (row < m && col < n) {
            float2 v{acc[i][j][0][r], acc[i][j][1][r]};
            if constexpr (PIPE) {
              if (CONJ)
                v.y -= acc[i][j][NACC - 1][r];
              else
                v.x -= acc[i][j][NACC - 1][r];
            }
            if (SPLIT) {
              part[tzv * m * n + row + col * m] = v;
            } else if (accum) {
              float2 o = C[row + col * ldc];
              o.x += v.x;
              o.y += v.y;
              C[row + col * ldc] = o;
            } else {
              C[row + col * ldc] = v;
            }
          }
        }
  };
  if constexpr (PERSIST) {
    // the steps of all the workgroup's tiles in one sequence: the last step of
    // a tile streams in the first slice of the next one, whose multiplication
    // then follows the stores of the finished tile
    if (ns == 0) return;
    int it = 0, sidx = 0;
    int64_t nrow0 = row0, ncol0 = col0;
    auto advance = [&]() -> bool {  // (tile, step) after the current one
      if (sidx + 1 < ns) return true;
      const int t = tile_of(it + 1);
      if (t >= ntiles) return false;
      int tm1, tn1;
      tile_rc(t, tm1, tn1);
      nrow0 = (int64_t)tm1 * BM;
      ncol0 = (int64_t)tn1 * BN;
      set_offsets(nrow0, ncol0);  // the current tile issues no more loads
      return true;
    };
    auto step = [&](unsigned char *cur, unsigned char *nxt) -> bool {
      wait_vmcnt<0>();
      __syncthreads();
      const bool more = advance();
      if (more) issue_t(nrow0, ncol0, sidx + 1 < ns ? sidx + 1 : 0, nxt);
      mma(cur);
      if (sidx + 1 < ns) {
        ++sidx;
        return true;
      }
      epilogue(row0, col0);
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
#pragma unroll
          for (int c = 0; c < NACC; ++c) acc[i][j][c] = v4f{0, 0, 0, 0};
      if (!more) return false;
      ++it;
      sidx = 0;
      row0 = nrow0;
      col0 = ncol0;
      return true;
    };
    issue(0, stage0);
    while (step(stage0, stage1) && step(stage1, stage0)) {
    }
    wait_vmcnt<0>();
  } else {
    if (ns > 0) issue(0, stage0);
    for (int s = 0; s < ns; s += 2) {
      wait_vmcnt<0>();
      __syncthreads();
      if (s + 1 < ns) issue(s + 1, stage1);
      mma(stage0);
      if (s + 1 >= ns) break;
      wait_vmcnt<0>();
      __syncthreads();
      if (s + 2 < ns) issue(s + 2, stage0);
      mma(stage1);
    }
    epilogue(row0, col0);
  }
}

// ---- three-stage form with 32 x 32 x 16 fragments ------------------------------
// The same products as zgemm_dl_kernel with a larger workgroup tile: K slices
// of 16 (v_mfma_f32_32x32x16_bf16), three LDS stages of 48 KB, eight waves of
// 64 x 64 complex (two per SIMD).  Slice s + 2 streams in while slice s is
// multiplied, so a step waits only for loads issued two steps earlier; the
// barrier carries no memory fence (a release fence on LDS would wait for the
// loads still streaming into the third stage) and the waits it needs are
// explicit: vmcnt for this wave's loads of the slice about to be read, and
// the LDS reads of the stage about to be refilled are complete because the
// multiplications that consumed them precede the barrier.
//
// LDS, one stage: A as [plane][row][16] bf16 with the 16-byte half h of row r
// at position h ^ dl3_swz(r) (B planes alike); B32 as [column][16] complex
// float with the 16-byte chunk c (two complex) of column j at position
// c ^ dl3_b32_mask(j).  A 16-byte read is served for lanes 0-7 together with
// lanes 16-23 (and 8-15 with 24-31), rows r and r + 16 of a fragment; eight
// rows of 32 bytes (or four columns of 128) fill one bank width, so the bit
// r >> 4 flips the half (the chunk's bit 0) and the sixteen reads fill all
// sixteen 16-byte positions: free of bank conflicts.
typedef float v16f __attribute__((ext_vector_type(16)));
__device__ __forceinline__ int dl3_swz(int r) { return ((r >> 2) & 1) ^ ((r >> 4) & 1); }
__device__ __forceinline__ int dl3_b32_mask(int j) { return (j & 7) ^ ((j >> 4) & 1); }

__device__ __forceinline__ v16f mfma32_bf16(const v8bf &a, const v8bf &b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// workgroup barrier without a memory fence; the empty asm statements keep the
// compiler from moving memory accesses across it
__device__ __forceinline__ void bar_nofence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int BM, int BN, int NWM, int NWN, bool CONJ, bool SPLIT, bool BF32>
__global__ __launch_bounds__(64 * NWM * NWN) void zgemm_dl3_kernel(
    int64_t m, int64_t n, int64_t kdata, const u16 *__restrict__ Apl, int64_t lda, int64_t psa,
    const void *__restrict__ Bsrc, int64_t ldb, int64_t psb, float2 *__restrict__ C,
    int64_t ldc, int64_t kchunk, int64_t kpad, float2 *__restrict__ part, int accum) {
  constexpr int NW = NWM * NWN;
  constexpr int WM = BM / NWM, WN = BN / NWN;     // wave tile
  constexpr int SM = WM / 32, SN = WN / 32;       // 32 x 32 blocks per wave
  constexpr int A_BYTES = 4 * BM * 32;                    // 4 planes x BM rows x 16 bf16
  constexpr int B_BYTES = BF32 ? BN * 128 : 4 * BN * 32;  // BN columns x 16 complex float
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int QA = BM / 8 / NW;                    // 1 KB loads (32 rows of a plane) per wave
  constexpr int QB = BF32 ? BN / 2 / NW : BN / 8 / NW;  // BF32: 256 B loads (two columns)
  constexpr int LOADS = QA + QB;                      // loads per wave per slice
  static_assert(QA * 8 * NW == BM && (BF32 ? QB * 2 * NW == BN : QB * 8 * NW == BN),
                "tile / waves");
  static_assert(SM >= 1 && SN >= 1 && SM * 32 == WM && SN * 32 == WN, "wave tile");
  __shared__ __align__(16) unsigned char stage0[STAGE];
  __shared__ __align__(16) unsigned char stage1[STAGE];
  __shared__ __align__(16) unsigned char stage2[STAGE];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % NWM, wn = wave / NWM;
  unsigned tm, tn, tz;
  grouped_tile(SPLIT ? gridDim.x : 4u, tm, tn, tz);
  const int64_t row0 = (int64_t)tm * BM, col0 = (int64_t)tn * BN;
  const int64_t kbeg = (int64_t)tz * kchunk;
  const int64_t kend = (kbeg + kchunk < kpad) ? kbeg + kchunk : kpad;
  const int ns = kend > kbeg ? (int)((kend - kbeg) >> 4) : 0;

  const u16 *asrc[QA];
  int aoff[QA];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int qq = wave * QA + q, p = qq / (BM / 32), r0 = (qq % (BM / 32)) * 32;
    const int r = r0 + (lane >> 1), h = (lane & 1) ^ dl3_swz(r);
    const int64_t gr = row0 + r < m ? row0 + r : m - 1;
    asrc[q] = Apl + (int64_t)p * psa + gr * lda + 8 * h;
    aoff[q] = p * BM * 32 + r0 * 32;
  }
  // B planes: per-load sources as for A.  B32: the column and the float index
  // of a lane's dword are formed at issue time (they are cheap, and holding 16
  // 64-bit sources would cost 32 VGPRs); load q of a wave covers columns
  // 2 (wave QB + q) + {0, 1}, lane l column (l >> 5), 16-byte position
  // (l >> 2) & 7, dword l & 3.
  const u16 *bsrc[BF32 ? 1 : QB];
  int boff[BF32 ? 1 : QB];
  if constexpr (!BF32) {
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int qq = wave * QB + q, p = qq / (BN / 32), r0 = (qq % (BN / 32)) * 32;
      const int r = r0 + (lane >> 1), h = (lane & 1) ^ dl3_swz(r);
      const int64_t gr = col0 + r < n ? col0 + r : n - 1;
      bsrc[q] = (const u16 *)Bsrc + (int64_t)p * psb + gr * ldb + 8 * h;
      boff[q] = A_BYTES + p * BN * 32 + r0 * 32;
    }
  }
  auto issue = [&](int s, unsigned char *st) {
    const int64_t k0 = kbeg + 16 * (int64_t)s;
#pragma unroll
    for (int q = 0; q < QA; ++q) dma16(asrc[q] + k0, st + aoff[q]);
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      if constexpr (BF32) {
        const int c = (wave * QB + q) * 2 + (lane >> 5);
        const int64_t gc = col0 + c < n ? col0 + c : n - 1;
        const int ch = ((lane >> 2) & 7) ^ dl3_b32_mask(c), w = lane & 3;
        int64_t kk = k0 + 2 * ch + (w >> 1);
        if (kk >= kdata) kk = kdata - 1;
        dma4((const float *)Bsrc + 2 * (gc * ldb + kk) + (w & 1),
             st + A_BYTES + (wave * QB + q) * 256);
      } else {
        dma16(bsrc[q] + k0, st + boff[q]);
      }
    }
  };

  v16f acc[SM][SN][2];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][j][c][e] = 0.f;

  const int hh = lane >> 5;  // K half of this lane's fragments
  auto b_frag = [&](const unsigned char *st, int j, v8bf *b) {
    const int jj = wn * WN + j * 32 + (lane & 31);
    if constexpr (BF32) {
      float4 q4[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int off = A_BYTES + jj * 128 + 16 * ((4 * hh + t) ^ dl3_b32_mask(jj));
        q4[t] = *reinterpret_cast<const float4 *>(st + off);
      }
      bf2_t rh[4], rl[4], ih[4], il[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        split2(f2v_t{q4[t].x, q4[t].z}, rh[t], rl[t]);
        split2(f2v_t{q4[t].y, q4[t].w}, ih[t], il[t]);
      }
      b[0] = cat4(rh[0], rh[1], rh[2], rh[3]);
      b[1] = cat4(ih[0], ih[1], ih[2], ih[3]);
      b[2] = cat4(rl[0], rl[1], rl[2], rl[3]);
      b[3] = cat4(il[0], il[1], il[2], il[3]);
    } else {
      const int kb = 16 * (hh ^ dl3_swz(jj));
#pragma unroll
      for (int p = 0; p < 4; ++p)
        b[p] = *reinterpret_cast<const v8bf *>(st + (A_BYTES + p * BN * 32 + jj * 32 + kb));
    }
  };
  auto a_frag = [&](const unsigned char *st, int i, v8bf *a) {
    const int ii = wm * WM + i * 32 + (lane & 31);
    const int kb = 16 * (hh ^ dl3_swz(ii));
#pragma unroll
    for (int p = 0; p < 4; ++p)
      a[p] = *reinterpret_cast<const v8bf *>(st + (p * BM * 32 + ii * 32 + kb));
    a[4] = bf16_neg(a[1]);
    a[5] = bf16_neg(a[3]);
  };
  auto mac = [&](const v8bf *a, const v8bf *b, v16f *q) {
    v16f re = q[0], im = q[1];
    re = mfma32_bf16(b[0], a[0], re);
    re = mfma32_bf16(b[2], a[0], re);
    re = mfma32_bf16(b[0], a[2], re);
    re = mfma32_bf16(b[1], a[CONJ ? 1 : 4], re);
    re = mfma32_bf16(b[3], a[CONJ ? 1 : 4], re);
    re = mfma32_bf16(b[1], a[CONJ ? 3 : 5], re);
    im = mfma32_bf16(b[1], a[0], im);
    im = mfma32_bf16(b[3], a[0], im);
    im = mfma32_bf16(b[1], a[2], im);
    im = mfma32_bf16(b[0], a[CONJ ? 4 : 1], im);
    im = mfma32_bf16(b[2], a[CONJ ? 4 : 1], im);
    im = mfma32_bf16(b[0], a[CONJ ? 5 : 3], im);
    q[0] = re;
    q[1] = im;
  };
  auto mma = [&](const unsigned char *st) {
    if constexpr (BF32) {
      // A fragments of every row block, then one column block of B at a time
      // (its converted fragments live only while its MFMAs run)
      v8bf a[SM][6];
#pragma unroll
      for (int i = 0; i < SM; ++i) a_frag(st, i, a[i]);
#pragma unroll
      for (int j = 0; j < SN; ++j) {
        v8bf b[4];
        b_frag(st, j, b);
#pragma unroll
        for (int i = 0; i < SM; ++i) mac(a[i], b, acc[i][j]);
      }
    } else {
      v8bf b[SN][4];
#pragma unroll
      for (int j = 0; j < SN; ++j) b_frag(st, j, b[j]);
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        v8bf a[6];
        a_frag(st, i, a);
#pragma unroll
        for (int j = 0; j < SN; ++j) mac(a, b[j], acc[i][j]);
      }
    }
  };

  // step s: slice s (stage s % 3) is complete once at most the loads of
  // slice s + 1 are outstanding; after the barrier every wave's part of it is
  // in LDS and every wave has finished slice s - 1, whose stage slice s + 2
  // then refills
  // (the stage of each step is a compile-time choice, so that every LDS access
  // names its stage array and the compiler can tell them apart)
  // Every step issues one slice (past the end: the last slice again, into a
  // stage no later step reads), so that the same vmcnt wait holds for every
  // step and the waits need no branches.
  auto step = [&](int s, auto cur_idx) {
    constexpr int CI = decltype(cur_idx)::value;
    wait_vmcnt<LOADS>();
    bar_nofence();
    issue(s + 2 < ns ? s + 2 : ns - 1, CI == 0 ? stage2 : CI == 1 ? stage0 : stage1);
    // keep the loads at the head of the step (the longest lead on their data)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (CI == 0)
      mma(stage0);
    else if constexpr (CI == 1)
      mma(stage1);
    else
      mma(stage2);
  };
  if (ns > 0) {
    issue(0, stage0);
    issue(ns > 1 ? 1 : 0, stage1);
    // all counters drained here: then the steady state's waits are exactly the
    // explicit ones (with the prologue's loads in flight, or only vmcnt drained,
    // the compiler adds a full vmcnt wait to the first step of every round of
    // three)
    __builtin_amdgcn_s_waitcnt(0);
    for (int s = 0; s < ns; s += 3) {
      step(s, std::integral_constant<int, 0>{});
      if (s + 1 >= ns) break;
      step(s + 1, std::integral_constant<int, 1>{});
      if (s + 2 >= ns) break;
      step(s + 2, std::integral_constant<int, 2>{});
    }
    // the last loads must land before the workgroup's LDS is released
    wait_vmcnt<0>();
  }

#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        // B operand first: lane & 31 indexes output rows, the accumulator
        // element e the column 8 (e / 4) + 4 (lane / 32) + e % 4
        const int64_t row = row0 + wm * WM + i * 32 + (lane & 31);
        const int64_t col = col0 + wn * WN + j * 32 + 8 * (e >> 2) + 4 * hh + (e & 3);
        if (row < m && col < n) {
          const float2 v{acc[i][j][0][e], acc[i][j][1][e]};
          if (SPLIT) {
            part[(int64_t)tz * m * n + row + col * m] = v;
          } else if (accum) {
            float2 o = C[row + col * ldc];
            o.x += v.x;
            o.y += v.y;
            C[row + col * ldc] = o;
          } else {
            C[row + col * ldc] = v;
          }
        }
      }
}

// complex float block (ld) -> four bf16 planes (Re hi, Im hi, Re lo, Im lo),
// row-major per band with stride ldp; rows .. ldp - 1 of each band are zero
// (the K padding the split-BF16 products read).
__global__ __launch_bounds__(256) void split_planes_kernel(int64_t rows, int64_t cols,
                                                           const float2 *__restrict__ X, int64_t ld,
                                                           u16 *__restrict__ pl, int64_t ldp,
                                                           int64_t ps) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ldp * cols) return;
  const int64_t i = idx % ldp, j = idx / ldp;
  const float2 v = i < rows ? X[i + j * ld] : float2{0.f, 0.f};
  const u16 hr = bf16_rn(v.x), hi = bf16_rn(v.y);
  const int64_t o = j * ldp + i;
  pl[o] = hr;
  pl[ps + o] = hi;
  pl[2 * ps + o] = bf16_rn(v.x - bf16_val(hr));
  pl[3 * ps + o] = bf16_rn(v.y - bf16_val(hi));
}

}  // namespace

void proj_gemm_bf16x3(int64_t nproj, int64_t nband, int64_t npw, const void *Apl, int64_t lda,
                      int64_t pstride, const void *Y, int64_t ldy, void *part, int splits,
                      hipStream_t st) {
  const int64_t chunk = ((npw + splits - 1) / splits + XBK - 1) / XBK * XBK;
  dim3 grid((unsigned)((nproj + XBM - 1) / XBM), (unsigned)((nband + XBN - 1) / XBN),
            (unsigned)splits);
  hipLaunchKernelGGL((zgemm_bf16x3_kernel<true, true>), grid, dim3(256), 0, st, nproj, nband, npw,
                     (const u16 *)Apl, lda, pstride, (const float2 *)Y, ldy, (float2 *)nullptr,
                     (int64_t)0, chunk, (float2 *)part);
  CHEBFI_HIP(hipGetLastError());
}

// Transposed split: tiles of 64 rows x 64 columns of X pass through LDS so that
// both the reads (rows contiguous) and the plane writes (columns contiguous)
// are coalesced.
__global__ __launch_bounds__(256) void split_planes_t_kernel(int64_t rows, int64_t cols,
                                                             const float2 *__restrict__ X,
                                                             int64_t ld, u16 *__restrict__ pl,
                                                             int64_t ldp, int64_t ps) {
  __shared__ float2 t[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    const int64_t i = i0 + ii, j = j0 + jj;
    t[jj][ii] = (i < rows && j < cols) ? X[i + j * ld] : float2{0.f, 0.f};
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int jj = e & 63, ii = e >> 6;
    const int64_t i = i0 + ii, j = j0 + jj;
    if (i >= rows || j >= ldp) continue;
    const float2 v = t[jj][ii];  // zero past cols
    const u16 hr = bf16_rn(v.x), hi = bf16_rn(v.y);
    const int64_t o = i * ldp + j;
    pl[o] = hr;
    pl[ps + o] = hi;
    pl[2 * ps + o] = bf16_rn(v.x - bf16_val(hr));
    pl[3 * ps + o] = bf16_rn(v.y - bf16_val(hi));
  }
}

void split_planes_t(int64_t rows, int64_t cols, const void *X, int64_t ld, void *planes,
                    int64_t ldp, hipStream_t st) {
  if (rows <= 0 || ldp <= 0) return;
  dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((ldp + 63) / 64));
  hipLaunchKernelGGL(split_planes_t_kernel, grid, dim3(256), 0, st, rows, cols,
                     (const float2 *)X, ld, (u16 *)planes, ldp, ldp * rows);
  CHEBFI_HIP(hipGetLastError());
}

void split_planes(int64_t rows, int64_t cols, const void *X, int64_t ld, void *planes,
                  int64_t ldp, hipStream_t st) {
  const int64_t total = ldp * cols;
  if (total <= 0) return;
  hipLaunchKernelGGL(split_planes_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     rows, cols, (const float2 *)X, ld, (u16 *)planes, ldp, ldp * cols);
  CHEBFI_HIP(hipGetLastError());
}

// Tile variants of the planes x planes kernel: {BM, BN, NWM, NWN}.
//   0: 128 x 128, 2 x 4 waves (64 x 32 per wave)
//   1: 128 x 128, 2 x 2 waves (64 x 64 per wave)
//   2:  64 x  64, 2 x 2 waves (32 x 32 per wave)
//   3:  64 x 128, 1 x 4 waves (64 x 32 per wave)
//   4: 128 x 128, 2 x 4 waves, double-buffered LDS (default)
//   5: as 4 with the global loads issued two K slices ahead
//   6: 128 x  64, 2 x 2 waves, one LDS stage (two workgroups per CU)
// accum: C += A B (else C = A B) when not split
template <bool CONJ, bool SPLIT>
static void launch_pl(int variant, dim3 grid_mn_z, int64_t m, int64_t n, int64_t k,
                      const void *Apl, int64_t lda, int64_t psa, const void *Bpl, int64_t ldb,
                      int64_t psb, void *C, int64_t ldc, int64_t chunk, void *part,
                      hipStream_t st, bool accum = true) {
  auto go = [&](auto kern, int bm, int bn, int nt) {
    dim3 grid((unsigned)((m + bm - 1) / bm), (unsigned)((n + bn - 1) / bn), grid_mn_z.z);
    hipLaunchKernelGGL(kern, grid, dim3(nt), 0, st, m, n, k, (const u16 *)Apl, lda, psa,
                       (const u16 *)Bpl, ldb, psb, (float2 *)C, ldc, chunk, (float2 *)part,
                       (int)accum);
  };
  // direct-to-LDS kernels: K runs to the next multiple of 32 (zero planes), in
  // chunks of a multiple of 32
  auto go_dl = [&](auto kern, int bm, int bn, int nt) {
    dim3 grid((unsigned)((m + bm - 1) / bm), (unsigned)((n + bn - 1) / bn), grid_mn_z.z);
    const int64_t kpad = (k + 31) / 32 * 32;
    const int64_t kch = grid_mn_z.z == 1 ? kpad : (chunk + 31) / 32 * 32;
    CHEBFI_REQUIRE(kpad <= lda && kpad <= ldb, ABI_ERR_ARG,
                   "split-BF16 planes must be zero-padded to a multiple of 32");
    CHEBFI_REQUIRE((int64_t)bm * lda < (1ll << 31) && (int64_t)bn * ldb < (1ll << 31), ABI_ERR_ARG,
                   "split-BF16 tile spans more than 2^31 elements");
    hipLaunchKernelGGL(kern, grid, dim3(nt), 0, st, m, n, k, (const u16 *)Apl, lda, psa,
                       (const void *)Bpl, ldb, psb, (float2 *)C, ldc, kch, kpad, (float2 *)part,
                       (int)accum);
  };
  switch (variant) {
    case 1: go(zgemm_pl_kernel<128, 128, 2, 2, CONJ, SPLIT>, 128, 128, 256); break;
    case 2: go(zgemm_pl_kernel<64, 64, 2, 2, CONJ, SPLIT>, 64, 64, 256); break;
    case 3: go(zgemm_pl_kernel<64, 128, 1, 4, CONJ, SPLIT>, 64, 128, 256); break;
    case 4: go(zgemm_pl2_kernel<128, 128, 2, 4, CONJ, SPLIT, 1>, 128, 128, 512); break;
    case 5: go(zgemm_pl2_kernel<128, 128, 2, 4, CONJ, SPLIT, 2>, 128, 128, 512); break;
    case 6: go(zgemm_pl2_kernel<128, 64, 2, 2, CONJ, SPLIT, 0>, 128, 64, 256); break;
    case 7: go_dl(zgemm_dl_kernel<128, 128, 2, 2, CONJ, SPLIT, false>, 128, 128, 256); break;
    case 8: go_dl(zgemm_dl_kernel<128, 128, 1, 4, CONJ, SPLIT, false>, 128, 128, 256); break;
    case 9: go_dl(zgemm_dl_kernel<128, 128, 2, 4, CONJ, SPLIT, false>, 128, 128, 512); break;
    case 10: go_dl(zgemm_dl_kernel<128, 128, 4, 2, CONJ, SPLIT, false>, 128, 128, 512); break;
    case 11: go_dl(zgemm_dl3_kernel<256, 128, 4, 2, CONJ, SPLIT, false>, 256, 128, 512); break;
    case 12: go_dl(zgemm_dl3_kernel<128, 256, 2, 4, CONJ, SPLIT, false>, 128, 256, 512); break;
    case 13: go_dl(zgemm_dl_kernel<128, 128, 2, 4, CONJ, SPLIT, false, true>, 128, 128, 512); break;
    case 14: go_dl(zgemm_dl_kernel<128, 128, 4, 2, CONJ, SPLIT, false, true>, 128, 128, 512); break;
    case 15:
      if constexpr (!SPLIT) {
        // persistent: one workgroup per CU, a whole number per XCD
        const int64_t tiles = ((m + 127) / 128) * ((n + 127) / 128);
        const int64_t per_xcd = std::max<int64_t>(
            1, std::min<int64_t>(device_cus() / 8, (tiles + 7) / 8));
        const int64_t kpad = (k + 31) / 32 * 32;
        CHEBFI_REQUIRE(kpad <= lda && kpad <= ldb, ABI_ERR_ARG,
                       "split-BF16 planes must be zero-padded to a multiple of 32");
        CHEBFI_REQUIRE(128 * lda < (1ll << 31) && 128 * ldb < (1ll << 31), ABI_ERR_ARG,
                       "split-BF16 tile spans more than 2^31 elements");
        hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 2, 4, CONJ, false, false, true, true>),
                           dim3((unsigned)(8 * per_xcd)), dim3(512), 0, st, m, n, k,
                           (const u16 *)Apl, lda, psa, (const void *)Bpl, ldb, psb, (float2 *)C,
                           ldc, kpad, kpad, (float2 *)nullptr, (int)accum);
      } else {
        go_dl(zgemm_dl_kernel<128, 128, 2, 4, CONJ, SPLIT, false, true>, 128, 128, 512);
      }
      break;
    default: go(zgemm_pl_kernel<128, 128, 2, 4, CONJ, SPLIT>, 128, 128, 512); break;
  }
  CHEBFI_HIP(hipGetLastError());
}

static int pl_bm(int variant) { return (variant == 2 || variant == 3) ? 64 : variant == 11 ? 256 : 128; }
static int pl_bn(int variant) { return (variant == 2 || variant == 6) ? 64 : variant == 12 ? 256 : 128; }
static bool pl_one_per_cu(int variant) { return variant == 4 || variant == 5 || variant >= 7; }

int proj_planes_splits(int variant, int64_t nproj, int64_t nband, int64_t npw) {
  // at least 1024 plane waves per chunk; the double-buffered 128 x 128 tiles hold
  // 128 KB of LDS (one workgroup per CU), the single-stage ones two per CU
  const int64_t tiles = ((nproj + pl_bm(variant) - 1) / pl_bm(variant)) *
                        ((nband + pl_bn(variant) - 1) / pl_bn(variant));
  const int per_cu = pl_one_per_cu(variant) ? 1 : 2;
  return best_splits(tiles, (npw + 1023) / 1024, per_cu);
}

void proj_gemm_planes(int64_t nproj, int64_t nband, int64_t npw, const void *Apl, int64_t lda,
                      int64_t psa, const void *Ypl, int64_t ldy, int64_t psy, void *part,
                      int splits, hipStream_t st, int variant) {
  const int64_t chunk = ((npw + splits - 1) / splits + XBK - 1) / XBK * XBK;
  launch_pl<true, true>(variant, dim3(1, 1, (unsigned)splits), nproj, nband, npw, Apl, lda, psa,
                        Ypl, ldy, psy, nullptr, 0, chunk, part, st);
}

void proj_gemm_planes_f32(int64_t nproj, int64_t nband, int64_t npw, const void *Apl, int64_t lda,
                          int64_t psa, const void *Y, int64_t ldy, void *part, int splits,
                          hipStream_t st) {
  const int64_t chunk = ((npw + splits - 1) / splits + XBK - 1) / XBK * XBK;
  dim3 grid((unsigned)((nproj + 127) / 128), (unsigned)((nband + 127) / 128), (unsigned)splits);
  hipLaunchKernelGGL((zgemm_pl2_kernel<128, 128, 2, 4, true, true, 1, true>), grid, dim3(512), 0,
                     st, nproj, nband, npw, (const u16 *)Apl, lda, psa, (const u16 *)Y, ldy,
                     (int64_t)0, (float2 *)nullptr, (int64_t)0, chunk, (float2 *)part, 1);
  CHEBFI_HIP(hipGetLastError());
}

// BF32 projection variants: 0 = double-buffered register-staged 128 x 128
// (split while staged), 1 = direct-to-LDS 128 x 128 with 2 x 2 waves,
// 2 = direct-to-LDS 128 x 128 with 1 x 4 waves.
void proj_gemm_f32_variant(int variant, int64_t nproj, int64_t nband, int64_t npw,
                           const void *Apl, int64_t lda, int64_t psa, const void *Y, int64_t ldy,
                           void *part, int splits, hipStream_t st) {
  if (variant == 0) {
    proj_gemm_planes_f32(nproj, nband, npw, Apl, lda, psa, Y, ldy, part, splits, st);
    return;
  }
  const int64_t chunk = ((npw + splits - 1) / splits + XBK - 1) / XBK * XBK;
  const int64_t kpad = (npw + 31) / 32 * 32;
  CHEBFI_REQUIRE(kpad <= lda, ABI_ERR_ARG, "projector planes must be zero-padded to 32");
  CHEBFI_REQUIRE(128 * lda < (1ll << 31), ABI_ERR_ARG, "projector planes too long");
  dim3 grid((unsigned)((nproj + 127) / 128), (unsigned)((nband + 127) / 128), (unsigned)splits);
  if (variant == 2)
    hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 1, 4, true, true, true>), grid, dim3(256), 0,
                       st, nproj, nband, npw, (const u16 *)Apl, lda, psa, Y, ldy, (int64_t)0,
                       (float2 *)nullptr, (int64_t)0, chunk, kpad, (float2 *)part, 1);
  else if (variant == 3)
    hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 2, 4, true, true, true>), grid, dim3(512), 0,
                       st, nproj, nband, npw, (const u16 *)Apl, lda, psa, Y, ldy, (int64_t)0,
                       (float2 *)nullptr, (int64_t)0, chunk, kpad, (float2 *)part, 1);
  else if (variant == 4)
    hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 4, 2, true, true, true>), grid, dim3(512), 0,
                       st, nproj, nband, npw, (const u16 *)Apl, lda, psa, Y, ldy, (int64_t)0,
                       (float2 *)nullptr, (int64_t)0, chunk, kpad, (float2 *)part, 1);
  else if (variant == 6)
    hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 2, 4, true, true, true, true>), grid, dim3(512),
                       0, st, nproj, nband, npw, (const u16 *)Apl, lda, psa, Y, ldy, (int64_t)0,
                       (float2 *)nullptr, (int64_t)0, chunk, kpad, (float2 *)part, 1);
  else if (variant == 5)
    hipLaunchKernelGGL((zgemm_dl3_kernel<128, 256, 2, 4, true, true, true>),
                       dim3(grid.x, (unsigned)((nband + 255) / 256), grid.z), dim3(512), 0, st,
                       nproj, nband, npw, (const u16 *)Apl, lda, psa, Y, ldy, (int64_t)0,
                       (float2 *)nullptr, (int64_t)0, chunk, kpad, (float2 *)part, 1);
  else
    hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 2, 2, true, true, true>), grid, dim3(256), 0,
                       st, nproj, nband, npw, (const u16 *)Apl, lda, psa, Y, ldy, (int64_t)0,
                       (float2 *)nullptr, (int64_t)0, chunk, kpad, (float2 *)part, 1);
  CHEBFI_HIP(hipGetLastError());
}

void expand_gemm_planes(int64_t npw, int64_t nband, int64_t nproj, const void *Apl, int64_t lda,
                        int64_t psa, const void *Cpl, int64_t ldc_pl, int64_t psc, void *Out,
                        int64_t ldo, hipStream_t st, int variant, bool accumulate) {
  launch_pl<false, false>(variant, dim3(1, 1, 1), npw, nband, nproj, Apl, lda, psa, Cpl, ldc_pl,
                          psc, Out, ldo, nproj, nullptr, st, accumulate);
}

void rr_gram_f32(int64_t m, int64_t npw, const void *Apl, int64_t lda, const void *Y,
                 int64_t ldy, void *part, int splits, hipStream_t st) {
  const int64_t chunk = ((npw + splits - 1) / splits + XBK - 1) / XBK * XBK;
  const int64_t kpad = (npw + 31) / 32 * 32;
  CHEBFI_REQUIRE(kpad <= lda, ABI_ERR_ARG, "block planes must be zero-padded to 32");
  CHEBFI_REQUIRE(128 * lda < (1ll << 31), ABI_ERR_ARG, "block planes too long");
  dim3 grid((unsigned)((m + 127) / 128), (unsigned)((m + 127) / 128), (unsigned)splits);
  hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 2, 4, true, true, true, true, false, 1>), grid,
                     dim3(512), 0, st, m, m, npw, (const u16 *)Apl, lda, m * lda, Y, ldy,
                     (int64_t)0, (float2 *)nullptr, (int64_t)0, chunk, kpad, (float2 *)part, 1);
  CHEBFI_HIP(hipGetLastError());
}

void rr_rotate_planes(int64_t npw, int64_t m, const void *Apl, int64_t lda, const void *Tpl,
                      int64_t ldt, void *Out, int64_t ldo, hipStream_t st) {
  const int64_t tiles = ((npw + 127) / 128) * ((m + 127) / 128);
  const int64_t per_xcd =
      std::max<int64_t>(1, std::min<int64_t>(device_cus() / 8, (tiles + 7) / 8));
  const int64_t kpad = (m + 31) / 32 * 32;
  CHEBFI_REQUIRE(kpad <= lda && kpad <= ldt, ABI_ERR_ARG,
                 "split-BF16 planes must be zero-padded to a multiple of 32");
  CHEBFI_REQUIRE(128 * lda < (1ll << 31) && 128 * ldt < (1ll << 31), ABI_ERR_ARG,
                 "split-BF16 tile spans more than 2^31 elements");
  hipLaunchKernelGGL((zgemm_dl_kernel<128, 128, 2, 4, false, false, false, true, true, 1>),
                     dim3((unsigned)(8 * per_xcd)), dim3(512), 0, st, npw, m, m, (const u16 *)Apl,
                     lda, npw * lda, (const void *)Tpl, ldt, ldt * m, (float2 *)Out, ldo, kpad,
                     kpad, (float2 *)nullptr, 0);
  CHEBFI_HIP(hipGetLastError());
}

void expand_gemm_bf16x3(int64_t npw, int64_t nband, int64_t nproj, const void *Apl, int64_t lda,
                        int64_t pstride, const void *Cp, void *Out, int64_t ldo, hipStream_t st) {
  dim3 grid((unsigned)((npw + XBM - 1) / XBM), (unsigned)((nband + XBN - 1) / XBN), 1);
  hipLaunchKernelGGL((zgemm_bf16x3_kernel<false, false>), grid, dim3(256), 0, st, npw, nband,
                     nproj, (const u16 *)Apl, lda, pstride, (const float2 *)Cp, nproj,
                     (float2 *)Out, ldo, nproj, (float2 *)nullptr);
  CHEBFI_HIP(hipGetLastError());
}

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
