// Batched Chebyshev filter over many independent systems (cells and k-points
// of uneven plane-wave counts and FFT boxes) in one set of launches.
//
// The paper batches the bands of one system into one FFT call (section "Batch
// processing"); here the batch spans systems as well.  One filter step of
// every system is six launches (the passes once per group of boxes), each a
// flat, grid-stride ("persistent") loop over the work items of all systems:
//   K1 proj   (system, band tile, projector tile, chunk): partial sums of C = P^H Y_k;
//   K1r       (system, 8 bands, projector tile): C' = alpha D C per atom;
//   K1b expand (system, plane-wave tile, band tile): E = P C';
//   K2 pass A (system, band, i3 group):     sphere planes -> inverse xy FFT -> box;
//   K3 pass B (system, band, i2 group):     z FFT, * V, z FFT;
//   K4 pass C (system, band, i3 group):     forward xy FFT -> gather, kinetic term,
//                                           + E, three-term recurrence.
// The nonlocal products are small here (a few to a few hundred projectors):
// plain FMA kernels tiled over bands and over projectors (32 each), so that P
// is read once per tile of 32 bands.  Per-system tables,
// per-step pointers and coefficients are read from device descriptors, so the
// 4 x degree launches are captured once into a HIP graph and replayed.
#include <algorithm>
#include <cstring>

#include "cplx.h"
#include "fft_dev.h"
#include "internal.h"
#include "kernels.h"

namespace chebfi {

namespace {

// cubic edges with specialised batched passes
#define CHEBFI_BATCH_SIZES(X) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(45) X(48) X(64)

// item -> system by a scan of the prefix offsets off[0..nsys]
__device__ __forceinline__ int find_sys(const int64_t *off, int nsys, int64_t item) {
  int s = 0;
  while (s + 1 < nsys && item >= off[s + 1]) ++s;
  return s;
}

// The descriptors' pointers are read from memory, so the compiler cannot tell
// that they address global memory and would use flat accesses, which also
// count as LDS operations (every LDS wait would then wait for them too);
// pointers of this type make them global accesses.
template <typename T>
using gptr = T __attribute__((address_space(1))) *;
template <typename T>
__device__ __forceinline__ C2<T> gload(gptr<const C2<T>> p) {
  C2<T> v;
  v.x = p->x;
  v.y = p->y;
  return v;
}
template <typename T>
__device__ __forceinline__ void gstore(gptr<C2<T>> p, C2<T> v) {
  p->x = v.x;
  p->y = v.y;
}

template <typename T>
__device__ __forceinline__ C2<T> wave_sum(C2<T> v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

// K1: partial sums of C = P^H Y_k over one chunk of kBatchKC plane waves for a
// tile of kBatchBT bands and a tile of kBatchPT projectors of one system.  The
// chunk streams through LDS in pieces of KC, so each element of P is read once
// per band tile instead of once per band; a thread holds 2 projectors x 2
// bands, sums a piece in the block's precision and adds the piece sums in FP64.
// The next piece is loaded into registers while the current one is multiplied.
template <typename T>
__global__ __launch_bounds__(256) void bproj_tile_kernel(const BatchSys *__restrict__ sys,
                                                         const BatchStep *__restrict__ step,
                                                         const int64_t *__restrict__ off,
                                                         int nsys) {
  constexpr int KC = sizeof(T) == 4 ? 64 : 32;
  constexpr int NJ = kBatchPT, NB = kBatchBT;
  static_assert(NJ == NB && KC * NJ % 256 == 0, "one element of P and of Y per (thread, q)");
  constexpr int QP = KC * NJ / 256;
  __shared__ C2<T> ps[KC][NJ + 1];
  __shared__ C2<T> ys[KC][NB + 1];
  const int t = threadIdx.x;
  const int j0 = t & 15, bq = t >> 4;  // projectors j0, j0 + 16; bands bq, bq + 16
  const int64_t total = off[nsys];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(off, nsys, item);
    const BatchSys &d = sys[s];
    const BatchStep &st = step[s];
    const int64_t npw = d.npw;
    const int64_t nch = (npw + kBatchKC - 1) / kBatchKC;
    const int64_t loc = item - off[s];  // ((band tile) x npt + projector tile) x nch + chunk
    const int64_t tp = loc / nch, ch = loc - tp * nch;
    const int64_t bt = tp / d.npt, pj = tp - bt * d.npt;
    const int64_t b0 = bt * NB;
    const int nb = d.nband - b0 < NB ? (int)(d.nband - b0) : NB;
    const int np = d.nproj - (int)pj * NJ < NJ ? d.nproj - (int)pj * NJ : NJ;
    const gptr<const C2<T>> P = (gptr<const C2<T>>)d.P + pj * NJ * npw;
    const gptr<const C2<T>> y = (gptr<const C2<T>>)st.yk + b0 * st.ldk;
    const int64_t kend = (ch + 1) * kBatchKC < npw ? (ch + 1) * kBatchKC : npw;
    // this thread's elements of a piece: e = t + 256 q, element k = e % KC of
    // projector (or band) e / KC; the next piece is fetched into registers
    // while the current one is multiplied
    C2<T> pn[QP], yn[QP];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int q = 0; q < QP; ++q) {
        const int e = t + 256 * q, k = e % KC, r = e / KC;
        C2<T> a{0, 0}, b{0, 0};
        if (k0 + k < kend) {
          if (r < np) a = gload<T>(P + k0 + k + (int64_t)r * npw);
          if (r < nb) b = gload<T>(y + (int64_t)r * st.ldk + k0 + k);
        }
        pn[q] = a;
        yn[q] = b;
      }
    };
    // with at most 16 projectors in the tile the second projector of a thread
    // is zero: only the first one is multiplied
    const bool two = np > 16;
    double2 tot[2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
    fetch(ch * kBatchKC);
    for (int64_t k0 = ch * kBatchKC; k0 < kend; k0 += KC) {
#pragma unroll
      for (int q = 0; q < QP; ++q) {
        const int e = t + 256 * q, k = e % KC, r = e / KC;
        ps[k][r] = pn[q];
        ys[k][r] = yn[q];
      }
      __syncthreads();
      if (k0 + KC < kend) fetch(k0 + KC);
      C2<T> acc[2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
      auto madd = [&](int u, int v, C2<T> p, C2<T> q) {  // acc += conj(p) q
        acc[u][v].x = fma(p.x, q.x, acc[u][v].x);
        acc[u][v].x = fma(p.y, q.y, acc[u][v].x);
        acc[u][v].y = fma(p.x, q.y, acc[u][v].y);
        acc[u][v].y = fma(-p.y, q.x, acc[u][v].y);
      };
      if (two) {
#pragma unroll 8
        for (int k = 0; k < KC; ++k) {
          const C2<T> p0 = ps[k][j0], p1 = ps[k][j0 + 16];
          const C2<T> y0 = ys[k][bq], y1 = ys[k][bq + 16];
          madd(0, 0, p0, y0);
          madd(0, 1, p0, y1);
          madd(1, 0, p1, y0);
          madd(1, 1, p1, y1);
        }
      } else {
#pragma unroll 8
        for (int k = 0; k < KC; ++k) {
          const C2<T> p0 = ps[k][j0];
          const C2<T> y0 = ys[k][bq], y1 = ys[k][bq + 16];
          madd(0, 0, p0, y0);
          madd(0, 1, p0, y1);
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          tot[u][v].x += (double)acc[u][v].x;
          tot[u][v].y += (double)acc[u][v].y;
        }
      __syncthreads();
    }
    double2 *part = d.Cpart + (tp * nch + ch) * (NJ * NB);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) part[(j0 + 16 * u) * NB + bq + 16 * v] = tot[u][v];
  }
}

// K1r: C' = alpha D C for kBatchBR bands and one projector tile: the chunk
// sums added in a fixed order (FP64), then the per-atom 4 x 4 D (a tile holds
// whole atoms).
template <typename T>
__global__ __launch_bounds__(256) void bproj_reduce_kernel(const BatchSys *__restrict__ sys,
                                                           const BatchStep *__restrict__ step,
                                                           const int64_t *__restrict__ off,
                                                           int nsys) {
  constexpr int NJ = kBatchPT, NB = kBatchBT, NR = kBatchBR;
  __shared__ double2 cs[NJ][NR];
  const int t = threadIdx.x;
  const int64_t total = off[nsys];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(off, nsys, item);
    const BatchSys &d = sys[s];
    const BatchStep &st = step[s];
    const int64_t loc = item - off[s];  // (band group) x npt + projector tile
    const int64_t bg = loc / d.npt, pj = loc - bg * d.npt;
    const int64_t b0 = bg * NR;  // first band of the item
    const int64_t bt = b0 / NB, bl = b0 - bt * NB;
    const int nb = d.nband - b0 < NR ? (int)(d.nband - b0) : NR;
    const int np = d.nproj - (int)pj * NJ < NJ ? d.nproj - (int)pj * NJ : NJ;
    const int j0 = (int)pj * NJ;
    const int64_t nch = (d.npw + kBatchKC - 1) / kBatchKC;
    const double2 *part = d.Cpart + (bt * d.npt + pj) * nch * (NJ * NB);
    for (int e = t; e < NJ * NR; e += 256) {
      const int j = e / NR, b = e % NR;
      double2 v{0, 0};
      for (int64_t c = 0; c < nch; ++c) {
        const double2 p = part[c * (NJ * NB) + j * NB + bl + b];
        v.x += p.x;
        v.y += p.y;
      }
      cs[j][b] = v;
    }
    __syncthreads();
    C2<T> *cp = reinterpret_cast<C2<T> *>(d.Cp);
    for (int e = t; e < np * nb; e += 256) {
      const int j = e % np, b = e / np, R = j >> 2, i = j & 3;  // local atom R of the tile
      const double2 *Dm = d.D + 16 * (j0 / 4 + R) + 4 * i;
      double2 v{0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q) v = cadd(v, cmul(Dm[q], cs[4 * R + q][b]));
      cp[(b0 + b) * d.nproj + j0 + j] = C2<T>{(T)(st.alpha * v.x), (T)(st.alpha * v.y)};
    }
    __syncthreads();
  }
}

// K1b: E = P C' for kBatchEP plane waves x kBatchBT bands of one system (E:
// npw x nband, ld npw; pass C adds it).  A thread owns one plane wave and
// keeps its kBatchBT outputs in registers over all projector tiles: per
// projector one P element from global memory and the C' row from LDS (the
// same address in every lane), four FMAs per band, so E is written once.
// Projectors come four per atom, so a tile's count is a multiple of four and
// the loop over them runs in unrolled steps of four.
template <typename T>
__global__ __launch_bounds__(kBatchEP) void bexpand_kernel(const BatchSys *__restrict__ sys,
                                                           const int64_t *__restrict__ off,
                                                           int nsys) {
  constexpr int NJ = kBatchPT, NB = kBatchBT;
  // a system has four projectors per atom, so with tiles of a multiple of four
  // every tile's count is one too and the steps of four stay inside the tile
  static_assert(NJ % 4 == 0, "projector tiles hold whole atoms");
  __shared__ C2<T> cs[NJ][NB];
  const int t = threadIdx.x;
  const int64_t total = off[nsys];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(off, nsys, item);
    const BatchSys &d = sys[s];
    const int64_t nbt = (d.nband + NB - 1) / NB;
    const int64_t loc = item - off[s];
    const int64_t pt = loc / nbt, bt = loc - pt * nbt;  // band tiles fastest
    const int64_t b0 = bt * NB;
    const int nb = d.nband - b0 < NB ? (int)(d.nband - b0) : NB;
    const int64_t npw = d.npw;
    const int64_t g = pt * kBatchEP + t;
    const gptr<const C2<T>> cp = (gptr<const C2<T>>)d.Cp;
    C2<T> v[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) v[b] = C2<T>{0, 0};
    for (int pj = 0; pj < d.npt; ++pj) {
      const int j0 = pj * NJ;
      const int np = d.nproj - j0 < NJ ? d.nproj - j0 : NJ;
      for (int e = t; e < NJ * NB; e += kBatchEP) {
        const int j = e / NB, b = e % NB;
        C2<T> c{0, 0};
        if (j < np && b < nb) c = gload<T>(cp + (b0 + b) * d.nproj + j0 + j);
        cs[j][b] = c;
      }
      __syncthreads();
      if (g < npw) {
        const gptr<const C2<T>> P = (gptr<const C2<T>>)d.P + (int64_t)j0 * npw + g;
        for (int j = 0; j < np; j += 4) {
          C2<T> pr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) pr[q] = gload<T>(P + (int64_t)(j + q) * npw);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              const C2<T> c = cs[j + q][b];
              v[b].x = fma(pr[q].x, c.x, v[b].x);
              v[b].x = fma(-pr[q].y, c.y, v[b].x);
              v[b].y = fma(pr[q].x, c.y, v[b].y);
              v[b].y = fma(pr[q].y, c.x, v[b].y);
            }
        }
      }
      __syncthreads();
    }
    if (g < npw) {
      const gptr<C2<T>> E = (gptr<C2<T>>)d.E + b0 * npw + g;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b < nb) gstore<T>(E + (int64_t)b * npw, v[b]);
    }
  }
}

// K2: pass A over (system, band, i3).
template <typename T>
__global__ __launch_bounds__(512) void bpass_a_kernel(const BatchSys *__restrict__ sys,
                                                      const BatchStep *__restrict__ step,
                                                      const int64_t *__restrict__ off, int nsys) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  const int64_t total = off[nsys];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(off, nsys, item);
    const BatchSys &d = sys[s];
    const BatchStep &st = step[s];
    const int n1 = d.plan.d[0].n, n2 = d.plan.d[1].n, n3 = d.plan.d[2].n;
    const int nxy = n1 * n2, L1 = n1 + 1;  // LDS plane rows padded to n1 + 1
    const int64_t loc = item - off[s];
    const int64_t b = loc / n3;
    const int i3 = (int)(loc - b * n3);
    C2<T> *tw1 = buf + n2 * L1;
    C2<T> *tw2 = tw1 + n1;
    load_twiddles<T>(tw1, d.tw, n1);
    load_twiddles<T>(tw2, d.tw + kMaxN, n2);
    for (int i = threadIdx.x; i < n2 * L1; i += blockDim.x) buf[i] = C2<T>{0, 0};
    __syncthreads();
    const int s0 = d.plane[i3], s1 = d.plane[i3 + 1];
    const C2<T> *xb = reinterpret_cast<const C2<T> *>(st.yk) + b * st.ldk;
    const int offp = i3 * nxy;
    for (int idx = s0 + threadIdx.x; idx < s1; idx += blockDim.x) {
      const int e = d.box_index[idx] - offp;
      buf[e + e / n1] = xb[idx];
    }
    __syncthreads();
    lds_fft<T>(buf, d.plan.d[0], 1, n2, L1, tw1, +1);
    lds_fft<T>(buf, d.plan.d[1], L1, n1, 1, tw2, +1);
    C2<T> *dst = reinterpret_cast<C2<T> *>(d.box) + b * (int64_t)nxy * n3 + offp;
    for (int i = threadIdx.x; i < nxy; i += blockDim.x) dst[i] = buf[i + i / n1];
    __syncthreads();
  }
}

// K3: pass B over (system, band, i2).
template <typename T>
__global__ __launch_bounds__(512) void bpass_b_kernel(const BatchSys *__restrict__ sys,
                                                      const int64_t *__restrict__ off, int nsys) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  const int64_t total = off[nsys];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(off, nsys, item);
    const BatchSys &d = sys[s];
    const int n1 = d.plan.d[0].n, n2 = d.plan.d[1].n, n3 = d.plan.d[2].n;
    const int nxz = n1 * n3, L1 = n1 + 1;  // LDS slab rows padded to n1 + 1
    const int64_t loc = item - off[s];
    const int64_t b = loc / n2;
    const int i2 = (int)(loc - b * n2);
    C2<T> *tw3 = buf + n3 * L1;
    load_twiddles<T>(tw3, d.tw + 2 * kMaxN, n3);
    C2<T> *src = reinterpret_cast<C2<T> *>(d.box) + b * (int64_t)n1 * n2 * n3;
    const T *V = reinterpret_cast<const T *>(d.V);
    for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
      const int i1 = i % n1, i3 = i / n1;
      buf[i3 * L1 + i1] = src[i1 + n1 * (i2 + n2 * i3)];
    }
    __syncthreads();
    lds_fft<T>(buf, d.plan.d[2], L1, n1, 1, tw3, +1);
    for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
      const int i1 = i % n1, i3 = i / n1;
      buf[i3 * L1 + i1] = cscale(buf[i3 * L1 + i1], V[i1 + n1 * (i2 + n2 * i3)]);
    }
    __syncthreads();
    lds_fft<T>(buf, d.plan.d[2], L1, n1, 1, tw3, -1);
    for (int i = threadIdx.x; i < nxz; i += blockDim.x) {
      const int i1 = i % n1, i3 = i / n1;
      src[i1 + n1 * (i2 + n2 * i3)] = buf[i3 * L1 + i1];
    }
    __syncthreads();
  }
}

// K4: pass C over (system, band, i3) with the nonlocal expansion and the
// recurrence: out = alpha (local + (kin - c) y_k) + P C' - beta y_prev.
template <typename T>
__global__ __launch_bounds__(512) void bpass_c_kernel(const BatchSys *__restrict__ sys,
                                                      const BatchStep *__restrict__ step,
                                                      const int64_t *__restrict__ off, int nsys) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T> *buf = reinterpret_cast<C2<T> *>(smem_raw);
  const int64_t total = off[nsys];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(off, nsys, item);
    const BatchSys &d = sys[s];
    const BatchStep &st = step[s];
    const int n1 = d.plan.d[0].n, n2 = d.plan.d[1].n, n3 = d.plan.d[2].n;
    const int nxy = n1 * n2, L1 = n1 + 1;  // LDS plane rows padded to n1 + 1
    const int64_t loc = item - off[s];
    const int64_t b = loc / n3;
    const int i3 = (int)(loc - b * n3);
    const int np = d.nproj;
    C2<T> *tw1 = buf + n2 * L1;
    C2<T> *tw2 = tw1 + n1;
    load_twiddles<T>(tw1, d.tw, n1);
    load_twiddles<T>(tw2, d.tw + kMaxN, n2);
    const int offp = i3 * nxy;
    const C2<T> *src = reinterpret_cast<const C2<T> *>(d.box) + b * (int64_t)nxy * n3 + offp;
    for (int i = threadIdx.x; i < nxy; i += blockDim.x) buf[i + i / n1] = src[i];
    __syncthreads();
    lds_fft<T>(buf, d.plan.d[1], L1, n1, 1, tw2, -1);
    lds_fft<T>(buf, d.plan.d[0], 1, n2, L1, tw1, -1);
    const int s0 = d.plane[i3], s1 = d.plane[i3 + 1];
    const C2<T> *yk = reinterpret_cast<const C2<T> *>(st.yk) + b * st.ldk;
    const C2<T> *yp =
        st.yprev ? reinterpret_cast<const C2<T> *>(st.yprev) + b * st.ldp : nullptr;
    C2<T> *out = reinterpret_cast<C2<T> *>(st.out) + b * st.ldo;
    const C2<T> *E = np > 0 ? reinterpret_cast<const C2<T> *>(d.E) + b * d.npw : nullptr;
    const T alpha = (T)st.alpha, cshift = (T)st.cshift, beta = (T)st.beta;
    const T scale = (T)(1.0 / ((double)nxy * n3));
    for (int idx = s0 + threadIdx.x; idx < s1; idx += blockDim.x) {
      const int e = d.box_index[idx] - offp;
      const C2<T> lc = cscale(buf[e + e / n1], scale);
      const C2<T> x = yk[idx];
      const T kd = (T)d.kin[idx] - cshift;
      const C2<T> h = cadd(lc, cscale(x, kd));
      const C2<T> nl = E ? E[idx] : C2<T>{0, 0};
      C2<T> o{alpha * h.x + nl.x, alpha * h.y + nl.y};
      if (yp) {
        const C2<T> p = yp[idx];
        o.x -= beta * p.x;
        o.y -= beta * p.y;
      }
      out[idx] = o;
    }
    __syncthreads();
  }
}

// ---- specialised passes for the systems of one cubic edge N ----------------
// Same three passes as above over the items of the systems listed in gsys,
// with N, the radix sequence and the plane strides known at compile time (the
// cubic building blocks).  An item is NPL consecutive planes (pass B: x-z
// slabs) of one band, stacked in LDS N cld<N>() elements apart, so that a
// workgroup keeps about as much box data in flight on small boxes as one 64^2
// plane; G = ceil(N / NPL) items per band (the last may hold fewer planes).

// item -> (system, band, plane group) inside one edge group
__device__ __forceinline__ int group_item(const int32_t *gsys, const int64_t *goff, int gns,
                                          int64_t item, int G, int64_t *b, int *grp) {
  const int q = find_sys(goff, gns, item);
  const int64_t loc = item - goff[q];
  *b = loc / G;
  *grp = (int)(loc - *b * G);
  return gsys[q];
}

template <typename T, int N>
__global__ __launch_bounds__(kCT) void bcpass_a_kernel(const BatchSys *__restrict__ sys,
                                                       const BatchStep *__restrict__ step,
                                                       const int32_t *__restrict__ gsys,
                                                       const int64_t *__restrict__ goff, int gns) {
  constexpr int NXY = N * N, LD = cld<N>(), PL = N * LD;
  constexpr int NPL = cplanes_per_item<T, N>(), G = (N + NPL - 1) / NPL;
  __shared__ C2<T> buf[NPL * PL];
  __shared__ C2<T> tw[N];
  const int64_t total = goff[gns];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    int64_t b;
    int g;
    const int s = group_item(gsys, goff, gns, item, G, &b, &g);
    const int i30 = g * NPL, np3 = N - i30 < NPL ? N - i30 : NPL;
    const BatchSys &d = sys[s];
    const BatchStep &st = step[s];
    // planes with no sphere points stay unwritten: pass B reads them as zeros
    const int s0 = d.plane[i30], s1 = d.plane[i30 + np3];
    if (s0 == s1) continue;
    for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(d.tw[i]);
    for (int i = threadIdx.x; i < NPL * PL; i += kCT) buf[i] = C2<T>{0, 0};
    __syncthreads();
    // the sphere points of planes i30 .. i30 + np3 - 1 are contiguous; element
    // e of the group (plane p, row r, column c) sits at (e / N) LD + e % N = p PL + r LD + c
    const C2<T> *xb = reinterpret_cast<const C2<T> *>(st.yk) + b * st.ldk;
    const int off = i30 * NXY;
    for (int idx = s0 + threadIdx.x; idx < s1; idx += kCT) {
      const int e = d.box_index[idx] - off;
      buf[(e / N) * LD + e % N] = xb[idx];
    }
    __syncthreads();
    cfft<T, N, 0, 1, NPL * N, 1, LD, +1>(buf, tw);         // x: every row of every plane
    // y: pencil pa = (plane p, column i1), element i2; the last stage writes the box
    C2<T> *dst = reinterpret_cast<C2<T> *>(d.box) + b * (int64_t)NXY * N + off;
    auto ldm = [&](int pa, int e) { return buf[(pa / N) * PL + pa % N + e * LD]; };
    auto stm = [&](int pa, int e, C2<T> v) { buf[(pa / N) * PL + pa % N + e * LD] = v; };
    auto stg = [&](int pa, int e, C2<T> v) {
      if (pa / N < np3) dst[(pa / N) * NXY + pa % N + e * N] = v;
    };
    cfft_io<T, N, 0, 1, NPL * N, +1, true, false>(tw, ldm, stg, ldm, stm);
    __syncthreads();
  }
}

// Waves per SIMD asked of the batched pass B: six (three workgroups of kCT
// threads per CU instead of two) for the complex64 edges where that measured
// faster (at 24 and 45 the compiler spills a few registers to fit, and the
// pass is still faster), else the least a workgroup of kCT threads needs.
template <typename T, int N>
constexpr int bcpass_b_waves() {
  return sizeof(T) == 4 && (N == 24 || N == 40 || N == 45) ? 6 : kCT / 256;
}

template <typename T, int N>
__global__ __launch_bounds__(kCT) __attribute__((amdgpu_waves_per_eu(bcpass_b_waves<T, N>())))
void bcpass_b_kernel(const BatchSys *__restrict__ sys, const int32_t *__restrict__ gsys,
                     const int64_t *__restrict__ goff, int gns) {
  constexpr int LD = cld<N>(), PL = N * LD;
  constexpr int NPL = cplanes_per_item<T, N>(), G = (N + NPL - 1) / NPL;
  __shared__ C2<T> buf[NPL * PL];
  __shared__ C2<T> tw[N];
  const int64_t total = goff[gns];
  if ((int64_t)blockIdx.x >= total) return;
  // the twiddles depend on N only (the same for every system of the group)
  for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(sys[gsys[0]].tw[2 * kMaxN + i]);
  __syncthreads();
  constexpr int64_t ZS = (int64_t)N * N;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    int64_t b;
    int g;
    const int s = group_item(gsys, goff, gns, item, G, &b, &g);
    const int i20 = g * NPL, np2 = N - i20 < NPL ? N - i20 : NPL;
    const BatchSys &d = sys[s];
    // slabs i20 .. i20 + np2 - 1: for each i3 their rows are one contiguous run
    // of np2 N elements in the box; pencil pa = p N + i1 is the position along
    // it, element i3; the forward z transform reads the box and applies V in
    // its last stage, the inverse's last stage writes the box
    C2<T> *src = reinterpret_cast<C2<T> *>(d.box) + b * (int64_t)N * N * N + (int64_t)i20 * N;
    const T *V = reinterpret_cast<const T *>(d.V) + (int64_t)i20 * N;
    const int run = np2 * N;
    auto ldm = [&](int pa, int e) { return buf[(pa / N) * PL + pa % N + e * LD]; };
    auto stm = [&](int pa, int e, C2<T> v) { buf[(pa / N) * PL + pa % N + e * LD] = v; };
    // z-planes without sphere points: zero on input (pass A leaves them
    // unwritten) and not written on output (pass C does not read them)
    const uint64_t zocc = d.zocc;
    auto occ = [&](int e) { return ((zocc >> e) & 1ull) != 0; };
    auto ldg = [&](int pa, int e) {
      return (pa < run && occ(e)) ? src[pa + e * ZS] : C2<T>{0, 0};
    };
    auto stv = [&](int pa, int e, C2<T> v) {
      buf[(pa / N) * PL + pa % N + e * LD] = pa < run ? cscale(v, V[pa + e * ZS]) : v;
    };
    auto stg = [&](int pa, int e, C2<T> v) {
      if (pa < run && occ(e)) src[pa + e * ZS] = v;
    };
    cfft_io<T, N, 0, 1, NPL * N, +1, false, true>(tw, ldg, stv, ldm, stm);
    cfft_io<T, N, 0, 1, NPL * N, -1, true, false>(tw, ldm, stg, ldm, stm);
    __syncthreads();
  }
}

// Waves per SIMD asked of the batched pass C: eight (a 64-VGPR budget, four
// workgroups of kCT threads per CU, as the LDS allows) where the compiler
// fits it without spilling (complex64, every edge but 36), else the least a
// workgroup of kCT threads needs.
template <typename T, int N>
constexpr int bcpass_c_waves() {
  return sizeof(T) == 4 && N != 36 ? 8 : kCT / 256;
}

template <typename T, int N>
__global__ __launch_bounds__(kCT) __attribute__((amdgpu_waves_per_eu(bcpass_c_waves<T, N>())))
void bcpass_c_kernel(const BatchSys *__restrict__ sys, const BatchStep *__restrict__ step,
                     const int32_t *__restrict__ gsys, const int64_t *__restrict__ goff,
                     int gns) {
  constexpr int NXY = N * N, LD = cld<N>(), PL = N * LD;
  constexpr int NPL = cplanes_per_item<T, N>(), G = (N + NPL - 1) / NPL;
  __shared__ C2<T> buf[NPL * PL];
  __shared__ C2<T> tw[N];
  const int64_t total = goff[gns];
  if ((int64_t)blockIdx.x >= total) return;
  // the twiddles depend on N only (the same for every system of the group)
  for (int i = threadIdx.x; i < N; i += kCT) tw[i] = to_c2<T>(sys[gsys[0]].tw[i]);
  __syncthreads();
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    int64_t b;
    int g;
    const int s = group_item(gsys, goff, gns, item, G, &b, &g);
    const int i30 = g * NPL, np3 = N - i30 < NPL ? N - i30 : NPL;
    const BatchSys &d = sys[s];
    const BatchStep &st = step[s];
    const int np = d.nproj;
    // no sphere points in these planes: nothing to gather (pass B left them
    // unwritten; in an item that also holds an occupied plane, such a plane's
    // values stay within its own 2-D transform and are never gathered)
    const int s0 = d.plane[i30], s1 = d.plane[i30 + np3];
    if (s0 == s1) continue;
    const int off = i30 * NXY;
    const C2<T> *src = reinterpret_cast<const C2<T> *>(d.box) + b * (int64_t)NXY * N + off;
    {  // y: pencil pa = (plane p, column i1), element i2; the first stage reads the box
      auto ldm = [&](int pa, int e) { return buf[(pa / N) * PL + pa % N + e * LD]; };
      auto stm = [&](int pa, int e, C2<T> v) { buf[(pa / N) * PL + pa % N + e * LD] = v; };
      auto ldg = [&](int pa, int e) {
        return pa / N < np3 ? src[(pa / N) * NXY + pa % N + e * N] : C2<T>{0, 0};
      };
      cfft_io<T, N, 0, 1, NPL * N, -1, false, true>(tw, ldg, stm, ldm, stm);
    }
    cfft<T, N, 0, 1, NPL * N, 1, LD, -1>(buf, tw);         // x: every row of every plane
    const C2<T> *yk = reinterpret_cast<const C2<T> *>(st.yk) + b * st.ldk;
    const C2<T> *yp =
        st.yprev ? reinterpret_cast<const C2<T> *>(st.yprev) + b * st.ldp : nullptr;
    C2<T> *out = reinterpret_cast<C2<T> *>(st.out) + b * st.ldo;
    const C2<T> *E = np > 0 ? reinterpret_cast<const C2<T> *>(d.E) + b * d.npw : nullptr;
    const T alpha = (T)st.alpha, cshift = (T)st.cshift, beta = (T)st.beta;
    const T scale = (T)(1.0 / ((double)NXY * N));
    for (int idx = s0 + threadIdx.x; idx < s1; idx += kCT) {
      const int e = d.box_index[idx] - off;
      const C2<T> lc = cscale(buf[(e / N) * LD + e % N], scale);
      const C2<T> x = yk[idx];
      const T kd = (T)d.kin[idx] - cshift;
      const C2<T> h = cadd(lc, cscale(x, kd));
      const C2<T> nl = E ? E[idx] : C2<T>{0, 0};
      C2<T> o{alpha * h.x + nl.x, alpha * h.y + nl.y};
      if (yp) {
        const C2<T> p = yp[idx];
        o.x -= beta * p.x;
        o.y -= beta * p.y;
      }
      out[idx] = o;
    }
    __syncthreads();
  }
}

template <typename F> void set_lds_b(F kernel, size_t bytes) {
  CHEBFI_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

// Host side: launches of one filter step for all systems.  With a side
// stream the projector products (which only pass C needs, as E) run there,
// beside passes A and B: they read the step's input, written by the previous
// step's pass C before the fork, and write E, C' and their partial sums, which
// nothing else reads before the join.
template <typename T>
void batch_step(const BatchLaunch &L, int j, hipStream_t st, hipStream_t side, hipEvent_t fork,
                hipEvent_t join) {
  const BatchStep *stp = L.d_steps + (size_t)j * L.nsys;
  const int64_t *offP = L.d_off;
  const int64_t *offA = L.d_off + (L.nsys + 1);
  const int64_t *offB = L.d_off + 2 * (L.nsys + 1);
  const int64_t *offE = L.d_off + 3 * (L.nsys + 1);
  const int64_t *offR = L.d_off + 4 * (L.nsys + 1);
  auto grid = [&](int64_t items) {
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(items, L.max_wgs)));
  };
  const bool fork_proj = L.any_proj && side != nullptr;
  if (L.any_proj) {
    hipStream_t sp = st;
    if (fork_proj) {
      CHEBFI_HIP(hipEventRecord(fork, st));
      CHEBFI_HIP(hipStreamWaitEvent(side, fork, 0));
      sp = side;
    }
    hipLaunchKernelGGL(bproj_tile_kernel<T>, grid(L.items_p), dim3(256), 0, sp, L.d_sys, stp,
                       offP, L.nsys);
    CHEBFI_HIP(hipGetLastError());
    hipLaunchKernelGGL(bproj_reduce_kernel<T>, grid(L.items_r), dim3(256), 0, sp, L.d_sys, stp,
                       offR, L.nsys);
    CHEBFI_HIP(hipGetLastError());
    hipLaunchKernelGGL(bexpand_kernel<T>, grid(L.items_e), dim3(kBatchEP), 0, sp, L.d_sys, offE,
                       L.nsys);
    CHEBFI_HIP(hipGetLastError());
    if (fork_proj) CHEBFI_HIP(hipEventRecord(join, side));
  }
  const size_t e = sizeof(C2<T>);
  // systems on cubic boxes with specialised passes: one launch per edge and pass
  auto cubic = [&](int pass) {
    for (int gi = 0; gi < L.ngroups; ++gi) {
      const BatchGroup &G = L.groups[gi];
      const dim3 gr = grid(G.items);
#define CHEBFI_CASE(N_)                                                                       \
  case N_:                                                                                    \
    if (pass == 0)                                                                            \
      hipLaunchKernelGGL((bcpass_a_kernel<T, N_>), gr, dim3(kCT), 0, st, L.d_sys, stp, G.gsys, \
                         G.goff, G.nsys);                                                     \
    else if (pass == 1)                                                                       \
      hipLaunchKernelGGL((bcpass_b_kernel<T, N_>), gr, dim3(kCT), 0, st, L.d_sys, G.gsys,      \
                         G.goff, G.nsys);                                                     \
    else                                                                                      \
      hipLaunchKernelGGL((bcpass_c_kernel<T, N_>), gr, dim3(kCT), 0, st, L.d_sys, stp, G.gsys, \
                         G.goff, G.nsys);                                                     \
    break;
      switch (G.n) {
        CHEBFI_BATCH_SIZES(CHEBFI_CASE)
        default:
          break;
      }
#undef CHEBFI_CASE
      CHEBFI_HIP(hipGetLastError());
    }
  };
  cubic(0);
  if (L.items_a > 0) {
    hipLaunchKernelGGL(bpass_a_kernel<T>, grid(L.items_a), dim3(L.fft_threads), e * L.lds_a, st,
                       L.d_sys, stp, offA, L.nsys);
    CHEBFI_HIP(hipGetLastError());
  }
  cubic(1);
  if (L.items_b > 0) {
    hipLaunchKernelGGL(bpass_b_kernel<T>, grid(L.items_b), dim3(L.fft_threads), e * L.lds_b, st,
                       L.d_sys, offB, L.nsys);
    CHEBFI_HIP(hipGetLastError());
  }
  if (fork_proj) CHEBFI_HIP(hipStreamWaitEvent(st, join, 0));
  cubic(2);
  if (L.items_a > 0) {
    hipLaunchKernelGGL(bpass_c_kernel<T>, grid(L.items_a), dim3(L.fft_threads), e * L.lds_c, st,
                       L.d_sys, stp, offA, L.nsys);
    CHEBFI_HIP(hipGetLastError());
  }
}

int batch_item_planes(int n, bool fp32) {
  // (the host side of cplanes_per_item)
  const int per = 34000 / (n * (n + 1) * (fp32 ? 8 : 16));
  return per > 1 ? per : 1;
}

bool batch_edge_specialised(int n) {
  switch (n) {
#define CHEBFI_CASE(N_) case N_:
    CHEBFI_BATCH_SIZES(CHEBFI_CASE)
#undef CHEBFI_CASE
    return true;
    default:
      return false;
  }
}

template <typename T>
void batch_prepare(const BatchLaunch &L) {
  const size_t e = sizeof(C2<T>);
  set_lds_b(bpass_a_kernel<T>, e * L.lds_a);
  set_lds_b(bpass_b_kernel<T>, e * L.lds_b);
  set_lds_b(bpass_c_kernel<T>, e * L.lds_c);
}

template void batch_step<float>(const BatchLaunch &, int, hipStream_t, hipStream_t, hipEvent_t,
                                hipEvent_t);
template void batch_step<double>(const BatchLaunch &, int, hipStream_t, hipStream_t, hipEvent_t,
                                 hipEvent_t);
template void batch_prepare<float>(const BatchLaunch &);
template void batch_prepare<double>(const BatchLaunch &);

}  // namespace chebfi
