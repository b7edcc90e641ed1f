// Local-potential part of H on a batch of bands: scatter sphere -> box,
// inverse 3D FFT, multiply by V_loc(r), forward 3D FFT, gather sphere.
//
// The paper applies V_loc to all bands with one batched FFT call instead of a
// per-band loop (arXiv 2604.11139, section "Batch processing", Algorithms
// "Per-band kernel execution" / "Batched bands kernel execution").  Here the
// batched 3D transform is split in three HBM passes, each holding one 2D slab
// of one band in LDS:
//   pass A  (band, i3 plane): scatter the plane's sphere rows into a zeroed
//           n1 x n2 plane, inverse FFT along x then y, store the plane;
//   pass B  (band, i2 slab):  load n1 x n3, inverse FFT along z, multiply by
//           V(r), forward FFT along z, store;
//   pass C  (band, i3 plane): load, forward FFT along y then x, gather the
//           sphere rows, scale 1/(n1 n2 n3) and combine with the kinetic term
//           and the Chebyshev recurrence:
//           out = alpha (local + (kin - cshift) yk) - beta yprev.
// Each 1D transform is a Stockham autosort FFT with radix-2/3/4/5 stages
// executed in place in LDS (every thread holds its butterflies' outputs in
// registers across a barrier).  Twiddles are FP64 tables built on the host.
#include <cstdlib>

#include "cplx.h"
#include "internal.h"
#include "kernels.h"
#include "fft_dev.h"

namespace chebfi {

namespace {

// ---- pass A: sphere plane -> inverse xy FFT -> box plane -------------------
// bf16 planes of the complex64 values a pass writes (the operand layout of the
// split-BF16 projection: planes re_hi, im_hi, re_lo, im_lo of ps elements each,
// band b at b * ld): hi = bf16(v) and lo = bf16(v - hi), both rounded to
// nearest even, the same values as the planes made by a separate split pass.
struct PlanesOut {
  unsigned short *p;
  int64_t ld, ps;
};
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}
// Out[idx] = value(idx) over the sphere rows [s0, s1) with nt threads, and with
// po.p (T = float) the bf16 planes of each value.  (Pairing neighbouring
// lanes' planes into 32-bit stores by a shuffle measured slower: the pass is
// bound by its HBM bytes, which the planes raise by a fifth either way.)
template <typename T, class F>
__device__ __forceinline__ void sphere_store(int s0, int s1, int nt, const PlanesOut &po,
                                             int64_t b, C2<T> *out, F value) {
  if constexpr (std::is_same<T, float>::value) {
    if (po.p) {
      unsigned short *pb = po.p + b * po.ld;
      for (int idx = s0 + threadIdx.x; idx < s1; idx += nt) {
        const C2<T> o = value(idx);
        out[idx] = o;
        const unsigned short hr = bf16_bits(o.x), hi = bf16_bits(o.y);
        unsigned short *q = pb + idx;
        q[0] = hr;
        q[po.ps] = hi;
        q[2 * po.ps] = bf16_bits(o.x - bf16_float(hr));
        q[3 * po.ps] = bf16_bits(o.y - bf16_float(hi));
      }
      return;
    }
  }
  for (int idx = s0 + threadIdx.x; idx < s1; idx += nt) out[idx] = value(idx);
}

template <typename T>
__global__ __launch_bounds__(512) void pass_a_kernel(const C2<T> *__restrict__ X, int64_t ldx, int band0,
                              const int32_t *__restrict__ box_index,
                              const int32_t *__restrict__ plane, BoxPlan plan,
                              const double2 *__restrict__ twg, C2<T> *__restrict__ box) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const int nxy = n1 * n2, L1 = n1 + 1;  // LDS plane rows padded to n1 + 1
  C2<T> *tw1 = buf + n2 * L1;
  C2<T> *tw2 = tw1 + n1;
  const int i3 = blockIdx.x;
  const int bl = blockIdx.y;
  load_twiddles<T>(tw1, twg, n1);
  load_twiddles<T>(tw2, twg + kMaxN, n2);
  for (int i = threadIdx.x; i < n2 * L1; i += blockDim.x) buf[i] = C2<T>{0, 0};
  __syncthreads();
  const int s0 = plane[i3], s1 = plane[i3 + 1];
  const C2<T> *xb = X + (int64_t)(band0 + bl) * ldx;
  const int off = i3 * nxy;
  for (int idx = s0 + threadIdx.x; idx < s1; idx += blockDim.x) {
    const int e = box_index[idx] - off;
    buf[e + e / n1] = xb[idx];
  }
  __syncthreads();
  lds_fft<T>(buf, plan.d[0], 1, n2, L1, tw1, +1);
  lds_fft<T>(buf, plan.d[1], L1, n1, 1, tw2, +1);
  C2<T> *dst = box + (int64_t)bl * nxy * n3 + off;
  for (int i = threadIdx.x; i < nxy; i += blockDim.x) dst[i] = buf[i + i / n1];
}

// ---- pass B: z pencils of one i2 slab, inverse FFT, * V, forward FFT -------
template <typename T, typename VT>
__global__ __launch_bounds__(512) void pass_b_kernel(C2<T> *__restrict__ box, const VT *__restrict__ V, BoxPlan plan,
                              const double2 *__restrict__ twg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const int nxz = n1 * n3, L1 = n1 + 1;  // LDS slab rows padded to n1 + 1
  C2<T> *tw3 = buf + n3 * L1;
  const int i2 = blockIdx.x;
  const int bl = blockIdx.y;
  load_twiddles<T>(tw3, twg + 2 * kMaxN, n3);
  C2<T> *src = box + (int64_t)bl * n1 * n2 * n3;
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    buf[i3 * L1 + i1] = src[i1 + n1 * (i2 + n2 * i3)];
  }
  __syncthreads();
  lds_fft<T>(buf, plan.d[2], L1, n1, 1, tw3, +1);
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    buf[i3 * L1 + i1] = cscale(buf[i3 * L1 + i1], (T)V[i1 + n1 * (i2 + n2 * i3)]);
  }
  __syncthreads();
  lds_fft<T>(buf, plan.d[2], L1, n1, 1, tw3, -1);
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    src[i1 + n1 * (i2 + n2 * i3)] = buf[i3 * L1 + i1];
  }
}

// a + b rounded on its own (never fused with the multiply that produced a), so
// that adding a precomputed block E equals storing the value and adding E later
template <typename V2> __device__ __forceinline__ V2 add_rounded(V2 a, V2 b) {
#pragma clang fp contract(off)
  return V2{a.x + b.x, a.y + b.y};
}

// ---- pass C: box plane -> forward xy FFT -> gather + recurrence combine ----
template <typename T>
__global__ __launch_bounds__(512) void pass_c_kernel(const C2<T> *__restrict__ box, BoxPlan plan,
                              const double2 *__restrict__ twg,
                              const int32_t *__restrict__ box_index,
                              const int32_t *__restrict__ plane, const double *__restrict__ kin,
                              int band0, const C2<T> *__restrict__ Yk, int64_t ldk,
                              const C2<T> *__restrict__ Yprev, int64_t ldp,
                              C2<T> *__restrict__ Out, int64_t ldo, T alpha, T cshift, T beta,
                              T scale, const C2<T> *__restrict__ E, int64_t lde,
                              const double *__restrict__ coef, PlanesOut po) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  if (coef) {  // (alpha, cshift, beta) of this step from device memory (captured filters)
    alpha = (T)coef[0];
    cshift = (T)coef[1];
    beta = (T)coef[2];
  }
  const int n1 = plan.d[0].n, n2 = plan.d[1].n;
  const int nxy = n1 * n2, L1 = n1 + 1;  // LDS plane rows padded to n1 + 1
  C2<T> *tw1 = buf + n2 * L1;
  C2<T> *tw2 = tw1 + n1;
  const int i3 = blockIdx.x;
  const int bl = blockIdx.y;
  load_twiddles<T>(tw1, twg, n1);
  load_twiddles<T>(tw2, twg + kMaxN, n2);
  const int off = i3 * nxy;
  const C2<T> *src = box + (int64_t)bl * nxy * plan.d[2].n + off;
  for (int i = threadIdx.x; i < nxy; i += blockDim.x) buf[i + i / n1] = src[i];
  __syncthreads();
  lds_fft<T>(buf, plan.d[1], L1, n1, 1, tw2, -1);
  lds_fft<T>(buf, plan.d[0], 1, n2, L1, tw1, -1);
  const int s0 = plane[i3], s1 = plane[i3 + 1];
  const int64_t b = band0 + bl;
  const C2<T> *yk = Yk + b * ldk;
  C2<T> *out = Out + b * ldo;
  const C2<T> *ex = E ? E + b * lde : nullptr;
  if (Yprev != nullptr) {
    const C2<T> *yp = Yprev + b * ldp;
    sphere_store<T>(s0, s1, (int)blockDim.x, po, b, out, [&](int idx) {
      const int e = box_index[idx] - off;
      C2<T> loc = cscale(buf[e + e / n1], scale);
      C2<T> x = yk[idx];
      const T kd = (T)kin[idx] - cshift;
      C2<T> h = cadd(loc, cscale(x, kd));
      C2<T> p = yp[idx];
      C2<T> o{alpha * h.x - beta * p.x, alpha * h.y - beta * p.y};
      if (ex) o = add_rounded(o, ex[idx]);
      return o;
    });
  } else {
    sphere_store<T>(s0, s1, (int)blockDim.x, po, b, out, [&](int idx) {
      const int e = box_index[idx] - off;
      C2<T> loc = cscale(buf[e + e / n1], scale);
      C2<T> x = yk[idx];
      const T kd = (T)kin[idx] - cshift;
      C2<T> h = cadd(loc, cscale(x, kd));
      C2<T> o = cscale(h, alpha);
      if (ex) o = add_rounded(o, ex[idx]);
      return o;
    });
  }
}

// ---- adjoint passes (runtime sizes) -----------------------------------------
// z-inverse FFT only: the box then holds the band in real space.
template <typename T>
__global__ __launch_bounds__(512) void pass_b_inv_kernel(C2<T> *__restrict__ box, BoxPlan plan,
                                                         const double2 *__restrict__ twg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const int nxz = n1 * n3, L1 = n1 + 1;  // LDS slab rows padded to n1 + 1
  C2<T> *tw3 = buf + n3 * L1;
  const int i2 = blockIdx.x;
  const int bl = blockIdx.y;
  load_twiddles<T>(tw3, twg + 2 * kMaxN, n3);
  C2<T> *src = box + (int64_t)bl * n1 * n2 * n3;
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    buf[i3 * L1 + i1] = src[i1 + n1 * (i2 + n2 * i3)];
  }
  __syncthreads();
  lds_fft<T>(buf, plan.d[2], L1, n1, 1, tw3, +1);
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    src[i1 + n1 * (i2 + n2 * i3)] = buf[i3 * L1 + i1];
  }
}

// Pass B of the adjoint H application: z-inverse of the adjoint band (box),
// the pointwise product Re[conj(adjoint) * forward] written over the forward
// band's real-space box (`fwd`, real part), then * V and the z-forward FFT.
template <typename T>
__global__ __launch_bounds__(512) void pass_b_adj_kernel(C2<T> *__restrict__ box,
                                                         C2<T> *__restrict__ fwd,
                                                         const T *__restrict__ V, BoxPlan plan,
                                                         const double2 *__restrict__ twg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const int nxz = n1 * n3, L1 = n1 + 1;  // LDS slab rows padded to n1 + 1
  C2<T> *tw3 = buf + n3 * L1;
  const int i2 = blockIdx.x;
  const int bl = blockIdx.y;
  load_twiddles<T>(tw3, twg + 2 * kMaxN, n3);
  C2<T> *src = box + (int64_t)bl * n1 * n2 * n3;
  C2<T> *fw = fwd + (int64_t)bl * n1 * n2 * n3;
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    buf[i3 * L1 + i1] = src[i1 + n1 * (i2 + n2 * i3)];
  }
  __syncthreads();
  lds_fft<T>(buf, plan.d[2], L1, n1, 1, tw3, +1);
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    const int64_t r = i1 + n1 * (i2 + n2 * i3);
    const C2<T> a = buf[i3 * L1 + i1], y = fw[r];
    fw[r] = C2<T>{a.x * y.x + a.y * y.y, (T)0};
    buf[i3 * L1 + i1] = cscale(a, V[r]);
  }
  __syncthreads();
  lds_fft<T>(buf, plan.d[2], L1, n1, 1, tw3, -1);
  for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    src[i1 + n1 * (i2 + n2 * i3)] = buf[i3 * L1 + i1];
  }
}

// dV[r] += scale * sum_b prod[b][r].x, bands summed in order.
template <typename T>
__global__ __launch_bounds__(256) void dv_reduce_kernel(int64_t nbox, int nb,
                                                        const C2<T> *__restrict__ prod,
                                                        double scale, double *__restrict__ dV) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbox) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += (double)prod[(int64_t)b * nbox + r].x;
  dV[r] += scale * acc;
}

// rho[r] += sum_b w[band0 + b] |box_b(r)|^2 * scale, bands summed in order.
template <typename T>
__global__ __launch_bounds__(256) void rho_accum_kernel(int64_t nbox, int nb, int band0,
                                                        const C2<T> *__restrict__ box,
                                                        const double *__restrict__ w,
                                                        double scale, double *__restrict__ rho) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbox) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) {
    const C2<T> v = box[(int64_t)b * nbox + r];
    const double wb = w ? w[band0 + b] : 1.0;
    acc += wb * ((double)v.x * v.x + (double)v.y * v.y);
  }
  rho[r] += scale * acc;
}

// ---- compile-time specialised passes for cubic boxes (building blocks in fft_dev.h) ----

template <typename T, int N>
__global__ __launch_bounds__(kCT) void cpass_a_kernel(const C2<T> *__restrict__ X, int64_t ldx,
                                                      int band0, const int32_t *__restrict__ box_index,
                                                      const int32_t *__restrict__ plane,
                                                      const double2 *__restrict__ twg,
                                                      C2<T> *__restrict__ box) {
  constexpr int NXY = N * N, LD = cld<N>();
  __shared__ C2<T> buf[N * LD];
  __shared__ C2<T> tw[N];
  const int i3 = blockIdx.x;
  const int bl = blockIdx.y;
  // a plane with no sphere points is left unwritten: the middle passes read it as zero
  if (plane[i3] == plane[i3 + 1]) return;
  for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(twg[i]);
  for (int i = threadIdx.x; i < N * LD; i += kCT) buf[i] = C2<T>{0, 0};
  __syncthreads();
  const int s0 = plane[i3], s1 = plane[i3 + 1];
  const C2<T> *xb = X + (int64_t)(band0 + bl) * ldx;
  const int off = i3 * NXY;
  for (int idx = s0 + threadIdx.x; idx < s1; idx += kCT) {
    const int e = box_index[idx] - off;
    buf[(e / N) * LD + e % N] = xb[idx];
  }
  __syncthreads();
  cfft<T, N, 0, 1, N, 1, LD, +1>(buf, tw);  // x: N pencils of stride-1 elements
  // y: pencil i1, element i2; the last stage writes the box plane
  C2<T> *dst = box + (int64_t)bl * NXY * N + off;
  auto ldm = [&](int pa, int e) { return buf[pa + e * LD]; };
  auto stm = [&](int pa, int e, C2<T> v) { buf[pa + e * LD] = v; };
  auto stg = [&](int pa, int e, C2<T> v) { dst[pa + e * N] = v; };
  cfft_io<T, N, 0, 1, N, +1, true, false>(tw, ldm, stg, ldm, stm);
}

template <typename T, typename VT, int N>
__global__ __launch_bounds__(kCT) void cpass_b_kernel(C2<T> *__restrict__ box,
                                                      const VT *__restrict__ V,
                                                      const double2 *__restrict__ twg,
                                                      uint64_t zocc) {
  constexpr int LD = cld<N>();
  __shared__ C2<T> buf[N * LD];
  __shared__ C2<T> tw[N];
  const int i2 = blockIdx.x;
  const int bl = blockIdx.y;
  for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(twg[2 * kMaxN + i]);
  __syncthreads();
  // z transforms of the slab (pencil i1, element i3): the first stage reads the
  // box, the forward transform's last stage applies V, the inverse's last
  // stage writes the box
  C2<T> *src = box + (int64_t)bl * N * N * N + (int64_t)N * i2;
  const VT *v = V + (int64_t)N * i2;
  constexpr int64_t ZS = (int64_t)N * N;
  auto ldm = [&](int pa, int e) { return buf[pa + e * LD]; };
  auto stm = [&](int pa, int e, C2<T> x) { buf[pa + e * LD] = x; };
  // reciprocal planes g3 without sphere points: zero in (pass A leaves them
  // unwritten), not written out (pass C does not read them)
  auto occ = [&](int e) { return ((zocc >> e) & 1ull) != 0; };
  auto ldg = [&](int pa, int e) { return occ(e) ? src[pa + e * ZS] : C2<T>{0, 0}; };
  auto stg = [&](int pa, int e, C2<T> x) {
    if (occ(e)) src[pa + e * ZS] = x;
  };
  auto stv = [&](int pa, int e, C2<T> x) { buf[pa + e * LD] = cscale(x, (T)v[pa + e * ZS]); };
  cfft_io<T, N, 0, 1, N, +1, false, true>(tw, ldg, stv, ldm, stm);
  cfft_io<T, N, 0, 1, N, -1, true, false>(tw, ldm, stg, ldm, stm);
}

// z-inverse FFT only (the box then holds the bands in real space).
template <typename T, int N>
__global__ __launch_bounds__(kCT) void cpass_b_inv_kernel(C2<T> *__restrict__ box,
                                                          const double2 *__restrict__ twg,
                                                          uint64_t zocc) {
  constexpr int LD = cld<N>();
  __shared__ C2<T> buf[N * LD];
  __shared__ C2<T> tw[N];
  const int i2 = blockIdx.x;
  const int bl = blockIdx.y;
  for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(twg[2 * kMaxN + i]);
  __syncthreads();
  C2<T> *src = box + (int64_t)bl * N * N * N + (int64_t)N * i2;
  constexpr int64_t ZS = (int64_t)N * N;
  auto ldm = [&](int pa, int e) { return buf[pa + e * LD]; };
  auto stm = [&](int pa, int e, C2<T> x) { buf[pa + e * LD] = x; };
  // input planes g3 without sphere points are zero; the output is real space (all z)
  auto ldg = [&](int pa, int e) {
    return ((zocc >> e) & 1ull) ? src[pa + e * ZS] : C2<T>{0, 0};
  };
  auto stg = [&](int pa, int e, C2<T> x) { src[pa + e * ZS] = x; };
  cfft_io<T, N, 0, 1, N, +1, false, false>(tw, ldg, stg, ldm, stm);
}

// Adjoint pass B: z-inverse of the adjoint band, Re[conj(adjoint) * forward]
// written over the forward band's real-space box (real part), then * V and the
// z-forward FFT of the adjoint band.
template <typename T, typename VT, int N>
__global__ __launch_bounds__(kCT) void cpass_b_adj_kernel(C2<T> *__restrict__ box,
                                                          C2<T> *__restrict__ fwd,
                                                          const VT *__restrict__ V,
                                                          const double2 *__restrict__ twg,
                                                          uint64_t zocc) {
  constexpr int LD = cld<N>();
  __shared__ C2<T> buf[N * LD];
  __shared__ C2<T> tw[N];
  const int i2 = blockIdx.x;
  const int bl = blockIdx.y;
  for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(twg[2 * kMaxN + i]);
  __syncthreads();
  const int64_t o = (int64_t)bl * N * N * N + (int64_t)N * i2;
  C2<T> *src = box + o;
  C2<T> *fw = fwd + o;
  const VT *v = V + (int64_t)N * i2;
  constexpr int64_t ZS = (int64_t)N * N;
  auto ldm = [&](int pa, int e) { return buf[pa + e * LD]; };
  auto stm = [&](int pa, int e, C2<T> x) { buf[pa + e * LD] = x; };
  // the adjoint band's planes g3 without sphere points: zero in, not written
  // out; the forward band's box is real space (all z)
  auto occ = [&](int e) { return ((zocc >> e) & 1ull) != 0; };
  auto ldg = [&](int pa, int e) { return occ(e) ? src[pa + e * ZS] : C2<T>{0, 0}; };
  auto stg = [&](int pa, int e, C2<T> x) {
    if (occ(e)) src[pa + e * ZS] = x;
  };
  // the z-inverse's last stage: Re[conj(a) y] over the forward box, a V into LDS
  auto stv = [&](int pa, int e, C2<T> a) {
    const int64_t r = pa + e * ZS;
    const C2<T> y = fw[r];
    fw[r] = C2<T>{a.x * y.x + a.y * y.y, (T)0};
    buf[pa + e * LD] = cscale(a, (T)v[r]);
  };
  cfft_io<T, N, 0, 1, N, +1, false, true>(tw, ldg, stv, ldm, stm);
  cfft_io<T, N, 0, 1, N, -1, true, false>(tw, ldm, stg, ldm, stm);
}

template <typename T, int N>
__global__ __launch_bounds__(kCT) void cpass_c_kernel(
    const C2<T> *__restrict__ box, const double2 *__restrict__ twg,
    const int32_t *__restrict__ box_index, const int32_t *__restrict__ plane,
    const double *__restrict__ kin, int band0, const C2<T> *__restrict__ Yk, int64_t ldk,
    const C2<T> *__restrict__ Yprev, int64_t ldp, C2<T> *__restrict__ Out, int64_t ldo, T alpha,
    T cshift, T beta, T scale, const C2<T> *__restrict__ E, int64_t lde,
    const double *__restrict__ coef, PlanesOut po) {
  constexpr int NXY = N * N, LD = cld<N>();
  __shared__ C2<T> buf[N * LD];
  __shared__ C2<T> tw[N];
  if (coef) {  // (alpha, cshift, beta) of this step from device memory (captured filters)
    alpha = (T)coef[0];
    cshift = (T)coef[1];
    beta = (T)coef[2];
  }
  const int i3 = blockIdx.x;
  const int bl = blockIdx.y;
  if (plane[i3] == plane[i3 + 1]) return;  // no sphere points to gather in this plane
  for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(twg[i]);
  __syncthreads();
  const int off = i3 * NXY;
  const C2<T> *src = box + (int64_t)bl * NXY * N + off;
  {  // y: pencil i1, element i2; the first stage reads the box plane
    auto ldm = [&](int pa, int e) { return buf[pa + e * LD]; };
    auto stm = [&](int pa, int e, C2<T> v) { buf[pa + e * LD] = v; };
    auto ldg = [&](int pa, int e) { return src[pa + e * N]; };
    cfft_io<T, N, 0, 1, N, -1, false, true>(tw, ldg, stm, ldm, stm);
  }
  cfft<T, N, 0, 1, N, 1, LD, -1>(buf, tw);
  const int s0 = plane[i3], s1 = plane[i3 + 1];
  const int64_t b = band0 + bl;
  const C2<T> *yk = Yk + b * ldk;
  C2<T> *out = Out + b * ldo;
  const C2<T> *ex = E ? E + b * lde : nullptr;
  if (Yprev != nullptr) {
    const C2<T> *yp = Yprev + b * ldp;
    sphere_store<T>(s0, s1, kCT, po, b, out, [&](int idx) {
      const int e = box_index[idx] - off;
      const C2<T> loc = cscale(buf[(e / N) * LD + e % N], scale);
      const C2<T> x = yk[idx];
      const T kd = (T)kin[idx] - cshift;
      const C2<T> h = cadd(loc, cscale(x, kd));
      const C2<T> p = yp[idx];
      C2<T> o{alpha * h.x - beta * p.x, alpha * h.y - beta * p.y};
      if (ex) o = add_rounded(o, ex[idx]);
      return o;
    });
  } else {
    sphere_store<T>(s0, s1, kCT, po, b, out, [&](int idx) {
      const int e = box_index[idx] - off;
      const C2<T> loc = cscale(buf[(e / N) * LD + e % N], scale);
      const C2<T> x = yk[idx];
      const T kd = (T)kin[idx] - cshift;
      C2<T> o = cscale(cadd(loc, cscale(x, kd)), alpha);
      if (ex) o = add_rounded(o, ex[idx]);
      return o;
    });
  }
}

template <typename T, int N>
void launch_cubic(const abi_system_s *s, const void *Yk, int64_t ldk, const void *Yprev,
                  int64_t ldp, void *Out, int64_t ldo, int band0, int nb, void *box, const void *V,
                  double alpha, double cshift, double beta, hipStream_t st, Profiler *prof,
                  double bytesA, double bytesB, double bytesC, const void *E, int64_t lde,
                  PlanesOut po) {
  typedef C2<T> V2;
  typedef typename std::conditional<std::is_same<T, double>::value, double, float>::type VT;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  V2 *bx = reinterpret_cast<V2 *>(box);
  int tok = prof ? prof->begin(PROF_FFT_A, bytesA, st) : -1;
  hipLaunchKernelGGL((cpass_a_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st,
                     reinterpret_cast<const V2 *>(Yk), ldk, band0, s->d_box, s->d_plane, tw, bx);
  CHEBFI_HIP(hipGetLastError());
  if (prof) prof->end(tok, st);
  tok = prof ? prof->begin(PROF_FFT_B, bytesB, st) : -1;
  hipLaunchKernelGGL((cpass_b_kernel<T, VT, N>), dim3(N, nb), dim3(kCT), 0, st, bx,
                     reinterpret_cast<const VT *>(V), tw, s->zocc);
  CHEBFI_HIP(hipGetLastError());
  if (prof) prof->end(tok, st);
  tok = prof ? prof->begin(PROF_FFT_C, bytesC, st) : -1;
  const T scale = (T)(1.0 / ((double)N * N * N));
  hipLaunchKernelGGL((cpass_c_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st, bx, tw, s->d_box,
                     s->d_plane, s->d_kin, band0, reinterpret_cast<const V2 *>(Yk), ldk,
                     reinterpret_cast<const V2 *>(Yprev), ldp, reinterpret_cast<V2 *>(Out), ldo,
                     (T)alpha, (T)cshift, (T)beta, scale, reinterpret_cast<const V2 *>(E), lde,
                     s->coef_dev, po);
  CHEBFI_HIP(hipGetLastError());
  if (prof) prof->end(tok, st);
}

template <typename T, int N>
void adjoint_cubic(const abi_system_s *s, const void *Ak1, int64_t lda1, const void *Yk,
                   int64_t ldy, void *Ak, int64_t ldak, bool accumulate, int band0, int nb,
                   void *box1, void *box2, const void *V, double gamma, double cshift, double *dV,
                   hipStream_t st) {
  typedef C2<T> V2;
  typedef typename std::conditional<std::is_same<T, double>::value, double, float>::type VT;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  V2 *b1 = reinterpret_cast<V2 *>(box1);
  V2 *b2 = reinterpret_cast<V2 *>(box2);
  hipLaunchKernelGGL((cpass_a_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st,
                     reinterpret_cast<const V2 *>(Ak1), lda1, band0, s->d_box, s->d_plane, tw, b1);
  hipLaunchKernelGGL((cpass_a_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st,
                     reinterpret_cast<const V2 *>(Yk), ldy, band0, s->d_box, s->d_plane, tw, b2);
  hipLaunchKernelGGL((cpass_b_inv_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st, b2, tw,
                     s->zocc);
  hipLaunchKernelGGL((cpass_b_adj_kernel<T, VT, N>), dim3(N, nb), dim3(kCT), 0, st, b1, b2,
                     reinterpret_cast<const VT *>(V), tw, s->zocc);
  const int64_t nbox = (int64_t)N * N * N;
  hipLaunchKernelGGL(dv_reduce_kernel<T>, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, st,
                     nbox, nb, (const V2 *)b2, gamma / (double)nbox, dV);
  const T scale = (T)(1.0 / (double)nbox);
  hipLaunchKernelGGL((cpass_c_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st, b1, tw, s->d_box,
                     s->d_plane, s->d_kin, band0, reinterpret_cast<const V2 *>(Ak1), lda1,
                     accumulate ? reinterpret_cast<const V2 *>(Ak) : (const V2 *)nullptr, ldak,
                     reinterpret_cast<V2 *>(Ak), ldak, (T)gamma, (T)cshift, (T)-1, scale,
                     (const V2 *)nullptr, (int64_t)0, (const double *)nullptr,
                     PlanesOut{nullptr, 0, 0});
  CHEBFI_HIP(hipGetLastError());
}

template <typename T, int N>
void density_cubic(const abi_system_s *s, const void *Psi, int64_t ld, int band0, int nb,
                   void *box, const double *w, double *rho, hipStream_t st) {
  typedef C2<T> V2;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  V2 *bx = reinterpret_cast<V2 *>(box);
  hipLaunchKernelGGL((cpass_a_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st,
                     reinterpret_cast<const V2 *>(Psi), ld, band0, s->d_box, s->d_plane, tw, bx);
  hipLaunchKernelGGL((cpass_b_inv_kernel<T, N>), dim3(N, nb), dim3(kCT), 0, st, bx, tw,
                     s->zocc);
  const int64_t nbox = (int64_t)N * N * N;
  hipLaunchKernelGGL(rho_accum_kernel<T>, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, st,
                     nbox, nb, band0, (const V2 *)bx, w, 1.0 / (double)nbox, rho);
  CHEBFI_HIP(hipGetLastError());
}

// Edges with compile-time specialised passes (cubic boxes).
#define CHEBFI_CUBIC_SIZES(X) \
  X(12) X(15) X(16) X(18) X(20) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(45) X(48) X(64)

template <typename T>
bool try_cubic_adjoint(const abi_system_s *s, const void *Ak1, int64_t lda1, const void *Yk,
                       int64_t ldy, void *Ak, int64_t ldak, bool accumulate, int band0, int nb,
                       void *box1, void *box2, const void *V, double gamma, double cshift,
                       double *dV, hipStream_t st) {
  if (s->n1 != s->n2 || s->n1 != s->n3) return false;
  if (s->generic_fft) return false;
#define CHEBFI_CASE(N_)                                                                      \
  case N_:                                                                                   \
    adjoint_cubic<T, N_>(s, Ak1, lda1, Yk, ldy, Ak, ldak, accumulate, band0, nb, box1, box2, \
                         V, gamma, cshift, dV, st);                                          \
    return true;
  switch (s->n1) {
    CHEBFI_CUBIC_SIZES(CHEBFI_CASE)
    default:
      return false;
  }
#undef CHEBFI_CASE
}

template <typename T>
bool try_cubic_density(const abi_system_s *s, const void *Psi, int64_t ld, int band0, int nb,
                       void *box, const double *w, double *rho, hipStream_t st) {
  if (s->n1 != s->n2 || s->n1 != s->n3) return false;
  if (s->generic_fft) return false;
#define CHEBFI_CASE(N_)                                                       \
  case N_:                                                                    \
    density_cubic<T, N_>(s, Psi, ld, band0, nb, box, w, rho, st);             \
    return true;
  switch (s->n1) {
    CHEBFI_CUBIC_SIZES(CHEBFI_CASE)
    default:
      return false;
  }
#undef CHEBFI_CASE
}

template <typename T>
bool try_cubic(const abi_system_s *s, const void *Yk, int64_t ldk, const void *Yprev, int64_t ldp,
               void *Out, int64_t ldo, int band0, int nb, void *box, const void *V, double alpha,
               double cshift, double beta, hipStream_t st, Profiler *prof, double bA, double bB,
               double bC, const void *E, int64_t lde, PlanesOut po) {
  if (s->n1 != s->n2 || s->n1 != s->n3) return false;
  if (s->generic_fft) return false;
#define CHEBFI_CUBIC(N_)                                                                     \
  case N_:                                                                                   \
    launch_cubic<T, N_>(s, Yk, ldk, Yprev, ldp, Out, ldo, band0, nb, box, V, alpha, cshift,  \
                        beta, st, prof, bA, bB, bC, E, lde, po);                             \
    return true;
  switch (s->n1) {
    CHEBFI_CUBIC(12)
    CHEBFI_CUBIC(15)
    CHEBFI_CUBIC(16)
    CHEBFI_CUBIC(18)
    CHEBFI_CUBIC(20)
    CHEBFI_CUBIC(24)
    CHEBFI_CUBIC(25)
    CHEBFI_CUBIC(27)
    CHEBFI_CUBIC(30)
    CHEBFI_CUBIC(32)
    CHEBFI_CUBIC(36)
    CHEBFI_CUBIC(40)
    CHEBFI_CUBIC(45)
    CHEBFI_CUBIC(48)
    CHEBFI_CUBIC(64)
    default:
      return false;
  }
#undef CHEBFI_CUBIC
}

template <typename F> void set_lds(F kernel, size_t bytes) {
  CHEBFI_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

template <typename T>
void launch_local_potential(const abi_system_s *s, const void *Yk, int64_t ldk, const void *Yprev,
                            int64_t ldp, void *Out, int64_t ldo, int band0, int nb, void *box,
                            const void *V, double alpha, double cshift, double beta,
                            hipStream_t st, Profiler *prof, const void *E, int64_t lde,
                            void *ypl, int64_t ldpl, int64_t pspl) {
  using V2 = C2<T>;
  const BoxPlan &plan = s->plan;
  const PlanesOut po{std::is_same<T, float>::value ? (unsigned short *)ypl : nullptr, ldpl, pspl};
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  const int tA = std::max(stage_threads(plan.d[0], n2), stage_threads(plan.d[1], n1));
  const int tB = stage_threads(plan.d[2], n1);
  CHEBFI_REQUIRE(tA <= 512 && tB <= 512, ABI_ERR_GRID, "FFT plane too large for one workgroup");
  const size_t ldsA = sizeof(V2) * (size_t)(n2 * (n1 + 1) + n1 + n2);
  const size_t ldsB = sizeof(V2) * (size_t)(n3 * (n1 + 1) + n3);
  set_lds(pass_a_kernel<T>, ldsA);
  set_lds(pass_c_kernel<T>, ldsA);
  if (std::is_same<T, double>::value)
    set_lds(pass_b_kernel<T, double>, ldsB);
  else
    set_lds(pass_b_kernel<T, float>, ldsB);
  V2 *bx = reinterpret_cast<V2 *>(box);
  // algorithmic HBM bytes of each pass (sphere rows, box planes, V once)
  const double es = (double)sizeof(V2), nbx = (double)n1 * n2 * n3, np = (double)s->npw;
  const double bytesA = nb * (np + nbx) * es;
  const double bytesB = nb * 2.0 * nbx * es + nbx * (double)sizeof(T);
  const double bytesC = nb * (nbx + np * ((Yprev ? 3.0 : 2.0) + (E ? 1.0 : 0.0))) * es;
  if (try_cubic<T>(s, Yk, ldk, Yprev, ldp, Out, ldo, band0, nb, box, V, alpha, cshift, beta, st,
                   prof, bytesA, bytesB, bytesC, E, lde, po))
    return;
  int tok = prof ? prof->begin(PROF_FFT_A, bytesA, st) : -1;
  hipLaunchKernelGGL(pass_a_kernel<T>, dim3(n3, nb), dim3(tA), ldsA, st,
                     reinterpret_cast<const V2 *>(Yk), ldk, band0, s->d_box, s->d_plane, plan, tw,
                     bx);
  CHEBFI_HIP(hipGetLastError());
  if (prof) prof->end(tok, st);
  tok = prof ? prof->begin(PROF_FFT_B, bytesB, st) : -1;
  if (std::is_same<T, double>::value)
    hipLaunchKernelGGL((pass_b_kernel<T, double>), dim3(n2, nb), dim3(tB), ldsB, st, bx,
                       reinterpret_cast<const double *>(V), plan, tw);
  else
    hipLaunchKernelGGL((pass_b_kernel<T, float>), dim3(n2, nb), dim3(tB), ldsB, st, bx,
                       reinterpret_cast<const float *>(V), plan, tw);
  CHEBFI_HIP(hipGetLastError());
  if (prof) prof->end(tok, st);
  tok = prof ? prof->begin(PROF_FFT_C, bytesC, st) : -1;
  const T scale = (T)(1.0 / ((double)n1 * (double)n2 * (double)n3));
  hipLaunchKernelGGL(pass_c_kernel<T>, dim3(n3, nb), dim3(tA), ldsA, st, bx, plan, tw, s->d_box,
                     s->d_plane, s->d_kin, band0, reinterpret_cast<const V2 *>(Yk), ldk,
                     reinterpret_cast<const V2 *>(Yprev), ldp, reinterpret_cast<V2 *>(Out), ldo,
                     (T)alpha, (T)cshift, (T)beta, scale, reinterpret_cast<const V2 *>(E), lde,
                     s->coef_dev, po);
  CHEBFI_HIP(hipGetLastError());
  if (prof) prof->end(tok, st);
}

template <typename T>
void launch_adjoint_local(const abi_system_s *s, const void *Ak1, int64_t lda1, const void *Yk,
                          int64_t ldy, void *Ak, int64_t ldak, bool accumulate, int band0, int nb,
                          void *box1, void *box2, const void *V, double gamma, double cshift,
                          double *dV, hipStream_t st) {
  using V2 = C2<T>;
  if (try_cubic_adjoint<T>(s, Ak1, lda1, Yk, ldy, Ak, ldak, accumulate, band0, nb, box1, box2, V,
                           gamma, cshift, dV, st))
    return;
  const BoxPlan &plan = s->plan;
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  const int tA = std::max(stage_threads(plan.d[0], n2), stage_threads(plan.d[1], n1));
  const int tB = stage_threads(plan.d[2], n1);
  CHEBFI_REQUIRE(tA <= 512 && tB <= 512, ABI_ERR_GRID, "FFT plane too large for one workgroup");
  const size_t ldsA = sizeof(V2) * (size_t)(n2 * (n1 + 1) + n1 + n2);
  const size_t ldsB = sizeof(V2) * (size_t)(n3 * (n1 + 1) + n3);
  set_lds(pass_a_kernel<T>, ldsA);
  set_lds(pass_c_kernel<T>, ldsA);
  set_lds(pass_b_inv_kernel<T>, ldsB);
  set_lds(pass_b_adj_kernel<T>, ldsB);
  V2 *b1 = reinterpret_cast<V2 *>(box1);
  V2 *b2 = reinterpret_cast<V2 *>(box2);
  hipLaunchKernelGGL(pass_a_kernel<T>, dim3(n3, nb), dim3(tA), ldsA, st,
                     reinterpret_cast<const V2 *>(Ak1), lda1, band0, s->d_box, s->d_plane, plan, tw,
                     b1);
  hipLaunchKernelGGL(pass_a_kernel<T>, dim3(n3, nb), dim3(tA), ldsA, st,
                     reinterpret_cast<const V2 *>(Yk), ldy, band0, s->d_box, s->d_plane, plan, tw,
                     b2);
  hipLaunchKernelGGL(pass_b_inv_kernel<T>, dim3(n2, nb), dim3(tB), ldsB, st, b2, plan, tw);
  hipLaunchKernelGGL(pass_b_adj_kernel<T>, dim3(n2, nb), dim3(tB), ldsB, st, b1, b2,
                     reinterpret_cast<const T *>(V), plan, tw);
  const int64_t nbox = (int64_t)n1 * n2 * n3;
  hipLaunchKernelGGL(dv_reduce_kernel<T>, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, st,
                     nbox, nb, (const V2 *)b2, gamma / (double)nbox, dV);
  const T scale = (T)(1.0 / (double)nbox);
  // Ak = gamma (local + (kin - c) Ak1) + Ak   (beta = -1 adds the previous content)
  hipLaunchKernelGGL(pass_c_kernel<T>, dim3(n3, nb), dim3(tA), ldsA, st, b1, plan, tw, s->d_box,
                     s->d_plane, s->d_kin, band0, reinterpret_cast<const V2 *>(Ak1), lda1,
                     accumulate ? reinterpret_cast<const V2 *>(Ak) : (const V2 *)nullptr, ldak,
                     reinterpret_cast<V2 *>(Ak), ldak, (T)gamma, (T)cshift, (T)-1, scale,
                     (const V2 *)nullptr, (int64_t)0, (const double *)nullptr,
                     PlanesOut{nullptr, 0, 0});
  CHEBFI_HIP(hipGetLastError());
}

template <typename T>
void launch_density(const abi_system_s *s, const void *Psi, int64_t ld, int band0, int nb,
                    void *box, const double *w, double *rho, hipStream_t st) {
  using V2 = C2<T>;
  if (try_cubic_density<T>(s, Psi, ld, band0, nb, box, w, rho, st)) return;
  const BoxPlan &plan = s->plan;
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  const int tA = std::max(stage_threads(plan.d[0], n2), stage_threads(plan.d[1], n1));
  const int tB = stage_threads(plan.d[2], n1);
  CHEBFI_REQUIRE(tA <= 512 && tB <= 512, ABI_ERR_GRID, "FFT plane too large for one workgroup");
  const size_t ldsA = sizeof(V2) * (size_t)(n2 * (n1 + 1) + n1 + n2);
  const size_t ldsB = sizeof(V2) * (size_t)(n3 * (n1 + 1) + n3);
  set_lds(pass_a_kernel<T>, ldsA);
  set_lds(pass_b_inv_kernel<T>, ldsB);
  V2 *bx = reinterpret_cast<V2 *>(box);
  hipLaunchKernelGGL(pass_a_kernel<T>, dim3(n3, nb), dim3(tA), ldsA, st,
                     reinterpret_cast<const V2 *>(Psi), ld, band0, s->d_box, s->d_plane, plan, tw,
                     bx);
  hipLaunchKernelGGL(pass_b_inv_kernel<T>, dim3(n2, nb), dim3(tB), ldsB, st, bx, plan, tw);
  const int64_t nbox = (int64_t)n1 * n2 * n3;
  hipLaunchKernelGGL(rho_accum_kernel<T>, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, st,
                     nbox, nb, band0, (const V2 *)bx, w, 1.0 / (double)nbox, rho);
  CHEBFI_HIP(hipGetLastError());
}

template void launch_density<double>(const abi_system_s *, const void *, int64_t, int, int, void *,
                                     const double *, double *, hipStream_t);
template void launch_density<float>(const abi_system_s *, const void *, int64_t, int, int, void *,
                                    const double *, double *, hipStream_t);

template void launch_adjoint_local<double>(const abi_system_s *, const void *, int64_t, const void *,
                                           int64_t, void *, int64_t, bool, int, int, void *,
                                           void *, const void *, double, double, double *,
                                           hipStream_t);
template void launch_adjoint_local<float>(const abi_system_s *, const void *, int64_t, const void *,
                                           int64_t, void *, int64_t, bool, int, int, void *,
                                           void *, const void *, double, double, double *,
                                           hipStream_t);

template void launch_local_potential<double>(const abi_system_s *, const void *, int64_t,
                                             const void *, int64_t, void *, int64_t, int, int,
                                             void *, const void *, double, double, double,
                                             hipStream_t, Profiler *, const void *, int64_t,
                                             void *, int64_t, int64_t);
template void launch_local_potential<float>(const abi_system_s *, const void *, int64_t,
                                             const void *, int64_t, void *, int64_t, int, int,
                                             void *, const void *, double, double, double,
                                             hipStream_t, Profiler *, const void *, int64_t,
                                             void *, int64_t, int64_t);

int fft_stage_threads(const Plan1D &pl, int npen) { return stage_need(pl, npen); }

}  // namespace chebfi
