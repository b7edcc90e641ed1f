// Device building blocks of the LDS-resident FFTs: radix-2/3/4/5/6/8 DFTs in
// registers, one Stockham stage over a set of pencils held in LDS, a 1D FFT
// from a radix plan, twiddle loading; and the host rule for the thread count
// of a stage.  Shared by the single-system passes and the batched passes.
#pragma once

#include "cplx.h"
#include "internal.h"

namespace chebfi {
namespace {

// butterflies per thread in one runtime-size stage of radix R: at most 20
// complex values held per thread (radix 2: 10, 3: 6, 4: 5, 5: 4), which takes
// every plane up to 96 x 96 in 512 threads
constexpr int kStageValues = 20;
__host__ __device__ constexpr int max_butterflies(int r) { return kStageValues / r; }

// Radix-R DFT in registers; sgn = -1 forward (e^{-}), +1 inverse (e^{+}).
template <typename T, int R> struct Dft;

template <typename T> struct Dft<T, 2> {
  static __device__ __forceinline__ void run(C2<T> *x, int) {
    C2<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <typename T> struct Dft<T, 4> {
  static __device__ __forceinline__ void run(C2<T> *x, int sgn) {
    C2<T> s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    C2<T> s13 = cadd(x[1], x[3]), d13 = cmul_i(csub(x[1], x[3]), sgn);
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, d13);
    x[3] = csub(d02, d13);
  }
};

template <typename T> struct Dft<T, 3> {
  static __device__ __forceinline__ void run(C2<T> *x, int sgn) {
    const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
    C2<T> t1 = cadd(x[1], x[2]);
    C2<T> t2 = cmul_i(cscale(csub(x[1], x[2]), h), sgn);
    C2<T> m = csub(x[0], cscale(t1, (T)0.5));
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, t2);
    x[2] = csub(m, t2);
  }
};

template <typename T> struct Dft<T, 5> {
  static __device__ __forceinline__ void run(C2<T> *x, int sgn) {
    const T c1 = (T)0.30901699437494742410;   // cos(2 pi / 5)
    const T c2 = (T)-0.80901699437494742410;  // cos(4 pi / 5)
    const T s1 = (T)0.95105651629515357212;   // sin(2 pi / 5)
    const T s2 = (T)0.58778525229247312917;   // sin(4 pi / 5)
    C2<T> t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    C2<T> t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
    C2<T> a1 = cadd(x[0], cadd(cscale(t1, c1), cscale(t2, c2)));
    C2<T> a2 = cadd(x[0], cadd(cscale(t1, c2), cscale(t2, c1)));
    C2<T> b1 = cmul_i(cadd(cscale(t3, s1), cscale(t4, s2)), sgn);
    C2<T> b2 = cmul_i(csub(cscale(t3, s2), cscale(t4, s1)), sgn);
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(a1, b1);
    x[4] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[3] = csub(a2, b2);
  }
};

template <typename T> struct Dft<T, 6> {
  // even/odd split: two radix-3 DFTs combined with w6^k = e^{sgn i pi k/3}
  static __device__ __forceinline__ void run(C2<T> *x, int sgn) {
    C2<T> e[3] = {x[0], x[2], x[4]}, o[3] = {x[1], x[3], x[5]};
    Dft<T, 3>::run(e, sgn);
    Dft<T, 3>::run(o, sgn);
    const T h = (T)0.86602540378443864676;
    const C2<T> w1{(T)0.5, (T)sgn * h}, w2{(T)-0.5, (T)sgn * h};
    const C2<T> t1 = cmul(o[1], w1), t2 = cmul(o[2], w2);
    x[0] = cadd(e[0], o[0]);
    x[3] = csub(e[0], o[0]);
    x[1] = cadd(e[1], t1);
    x[4] = csub(e[1], t1);
    x[2] = cadd(e[2], t2);
    x[5] = csub(e[2], t2);
  }
};

template <typename T> struct Dft<T, 9> {
  // 3 x 3: radix-3 DFTs of x[n2], x[n2+3], x[n2+6], twiddles w9^(n2 k1), then
  // radix-3 DFTs across n2 (output k1 + 3 k2), w9 = e^{sgn 2 pi i / 9}
  static __device__ __forceinline__ void run(C2<T> *x, int sgn) {
    C2<T> a[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
      a[n2][0] = x[n2];
      a[n2][1] = x[n2 + 3];
      a[n2][2] = x[n2 + 6];
      Dft<T, 3>::run(a[n2], sgn);
    }
    const T c1 = (T)0.76604444311897803520, s1 = (T)0.64278760968653932632;   // 2 pi / 9
    const T c2 = (T)0.17364817766693034885, s2 = (T)0.98480775301220805936;   // 4 pi / 9
    const T c4 = (T)-0.93969262078590838405, s4 = (T)0.34202014332566873304;  // 8 pi / 9
    a[1][1] = cmul(a[1][1], C2<T>{c1, (T)sgn * s1});
    a[1][2] = cmul(a[1][2], C2<T>{c2, (T)sgn * s2});
    a[2][1] = cmul(a[2][1], C2<T>{c2, (T)sgn * s2});
    a[2][2] = cmul(a[2][2], C2<T>{c4, (T)sgn * s4});
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      C2<T> b[3] = {a[0][k1], a[1][k1], a[2][k1]};
      Dft<T, 3>::run(b, sgn);
      x[k1] = b[0];
      x[k1 + 3] = b[1];
      x[k1 + 6] = b[2];
    }
  }
};

template <typename T> struct Dft<T, 8> {
  // even/odd split: two radix-4 DFTs combined with w8^k = e^{sgn i pi k/4}
  static __device__ __forceinline__ void run(C2<T> *x, int sgn) {
    C2<T> e[4] = {x[0], x[2], x[4], x[6]}, o[4] = {x[1], x[3], x[5], x[7]};
    Dft<T, 4>::run(e, sgn);
    Dft<T, 4>::run(o, sgn);
    const T c = (T)0.70710678118654752440;
    const C2<T> t1{c * (o[1].x - sgn * o[1].y), c * (o[1].y + sgn * o[1].x)};
    const C2<T> t2 = cmul_i(o[2], sgn);
    const C2<T> t3{c * (-o[3].x - sgn * o[3].y), c * (-o[3].y + sgn * o[3].x)};
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], t1);
    x[5] = csub(e[1], t1);
    x[2] = cadd(e[2], t2);
    x[6] = csub(e[2], t2);
    x[3] = cadd(e[3], t3);
    x[7] = csub(e[3], t3);
  }
};

// One Stockham stage of radix R over `npen` pencils of length n held in LDS.
// Element e of pencil q sits at buf[q*pstride + e*estride].  p is the product
// of the radices already applied.
template <typename T, int R>
__device__ void stage(C2<T> *buf, int n, int estride, int npen, int pstride, int p,
                      const C2<T> *tw, int sgn) {
  const int nbf = n / R;
  const int total = npen * nbf;
  const int m = n / (p * R);
  constexpr int MB = max_butterflies(R);
  C2<T> y[MB][R];
  int dst[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) {
    const int i = threadIdx.x + c * blockDim.x;
    dst[c] = -1;
    if (i < total) {
      // consecutive lanes take consecutive pencils: with an odd pencil stride
      // (padded planes) or a unit one their accesses spread over all LDS banks
      const int pen = i % npen, bf = i / npen;
      const int base = pen * pstride;
      C2<T> x[R];
#pragma unroll
      for (int t = 0; t < R; ++t) x[t] = buf[base + (bf + t * nbf) * estride];
      const int k = bf % p;
#pragma unroll
      for (int t = 1; t < R; ++t) {
        C2<T> w = tw[t * k * m];
        if (sgn > 0) w.y = -w.y;
        x[t] = cmul(x[t], w);
      }
      Dft<T, R>::run(x, sgn);
#pragma unroll
      for (int t = 0; t < R; ++t) y[c][t] = x[t];
      dst[c] = base + ((bf - k) * R + k) * estride;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < MB; ++c) {
    if (dst[c] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[dst[c] + t * p * estride] = y[c][t];
    }
  }
  __syncthreads();
}

template <typename T>
__device__ void lds_fft(C2<T> *buf, const Plan1D &pl, int estride, int npen, int pstride,
                        const C2<T> *tw, int sgn) {
  int p = 1;
  for (int s = 0; s < pl.nstage; ++s) {
    const int r = pl.radix[s];
    if (r == 4)
      stage<T, 4>(buf, pl.n, estride, npen, pstride, p, tw, sgn);
    else if (r == 2)
      stage<T, 2>(buf, pl.n, estride, npen, pstride, p, tw, sgn);
    else if (r == 3)
      stage<T, 3>(buf, pl.n, estride, npen, pstride, p, tw, sgn);
    else
      stage<T, 5>(buf, pl.n, estride, npen, pstride, p, tw, sgn);
    p *= r;
  }
}

template <typename T>
__device__ void load_twiddles(C2<T> *dst, const double2 *src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = to_c2<T>(src[i]);
}


// Smallest multiple of 64 threads with at most max_butterflies(r) butterflies
// per thread in every stage of the plan over npen pencils.
inline int stage_need(const Plan1D &pl, int npen) {
  int need = 64;
  for (int s = 0; s < pl.nstage; ++s) {
    const int total = npen * (pl.n / pl.radix[s]);
    const int mb = max_butterflies(pl.radix[s]);
    const int t = (total + mb - 1) / mb;
    if (t > need) need = t;
  }
  return (need + 63) / 64 * 64;
}

// Threads of the runtime-size passes: 512 (the most a pass may use); the
// extra waves per CU hide the latency of the plane loads and stores.
inline int stage_threads(const Plan1D &pl, int npen) {
  const int need = stage_need(pl, npen);
  return need > 512 ? need : 512;
}

// ---- compile-time specialised passes for cubic boxes ------------------------
// Same three passes as above with the box edge N, the radix sequence, the
// pencil strides and the thread count known at compile time, so that all
// index arithmetic reduces to constant multiplies and shifts.  A plane sits in
// LDS with a row stride of N + 1 elements, and the lanes of a wave take
// consecutive pencils in both directions: pencils along a row are then an odd
// stride apart, which spreads a wave's accesses over all LDS banks.
template <int N> struct CPlan;
#define CHEBFI_CPLAN(N_, NS_, R0_, R1_, R2_)                              \
  template <> struct CPlan<N_> {                                          \
    static constexpr int ns = NS_;                                        \
    static constexpr int r[3] = {R0_, R1_, R2_};                          \
  };
CHEBFI_CPLAN(12, 2, 4, 3, 1)
CHEBFI_CPLAN(15, 2, 5, 3, 1)
CHEBFI_CPLAN(16, 2, 4, 4, 1)
CHEBFI_CPLAN(18, 2, 6, 3, 1)
CHEBFI_CPLAN(20, 2, 5, 4, 1)
CHEBFI_CPLAN(24, 2, 8, 3, 1)
CHEBFI_CPLAN(25, 2, 5, 5, 1)
CHEBFI_CPLAN(27, 2, 3, 9, 1)
CHEBFI_CPLAN(30, 2, 6, 5, 1)
CHEBFI_CPLAN(32, 2, 8, 4, 1)
CHEBFI_CPLAN(36, 2, 6, 6, 1)
CHEBFI_CPLAN(40, 2, 8, 5, 1)
CHEBFI_CPLAN(45, 2, 5, 9, 1)
CHEBFI_CPLAN(48, 2, 8, 6, 1)
CHEBFI_CPLAN(64, 2, 8, 8, 1)
#undef CHEBFI_CPLAN

constexpr int kCT = 512;  // threads of the specialised passes (16 waves per CU per 4 planes)

// LDS row pitch of an N x N plane in the specialised passes: odd, so that the
// lanes of a wave walking consecutive pencils across rows (8-byte elements,
// row stride 2 cld dwords) meet every bank pair once: N + 1 for even N, N + 2
// for odd N (an even pitch such as 46 for N = 45 reaches only 16 banks).
template <int N>
constexpr int cld() {
  return N % 2 ? N + 2 : N + 1;
}

// NG groups of NPEN pencils (group g's pencils start at g * GS): several
// planes of one LDS buffer transformed by one pass over all their pencils.
template <typename T, int N, int R, int P, int NPEN, int ES, int PS, int SGN, int NG = 1,
          int GS = 0>
__device__ __forceinline__ void cstage(C2<T> *buf, const C2<T> *tw) {
  constexpr int NBF = N / R;
  constexpr int NP = NG * NPEN;
  constexpr int TOTAL = NP * NBF;
  constexpr int M = N / (P * R);
  constexpr int MAXB = (TOTAL + kCT - 1) / kCT;
  C2<T> y[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int i = threadIdx.x + c * kCT;
    dst[c] = -1;
    if (TOTAL % kCT == 0 || i < TOTAL) {
      const int pa = i % NP, bf = i / NP;
      const int base = NG == 1 ? pa * PS : (pa / NPEN) * GS + (pa % NPEN) * PS;
      C2<T> x[R];
#pragma unroll
      for (int t = 0; t < R; ++t) x[t] = buf[base + (bf + t * NBF) * ES];
      const int k = bf % P;
      if (P > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          C2<T> w = tw[t * k * M];
          if (SGN > 0) w.y = -w.y;
          x[t] = cmul(x[t], w);
        }
      }
      Dft<T, R>::run(x, SGN);
#pragma unroll
      for (int t = 0; t < R; ++t) y[c][t] = x[t];
      dst[c] = base + ((bf - k) * R + k) * ES;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    if (TOTAL % kCT == 0 || dst[c] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[dst[c] + t * P * ES] = y[c][t];
    }
  }
  __syncthreads();
}

template <typename T, int N, int S, int P, int NPEN, int ES, int PS, int SGN, int NG = 1,
          int GS = 0>
__device__ __forceinline__ void cfft(C2<T> *buf, const C2<T> *tw) {
  if constexpr (S < CPlan<N>::ns) {
    constexpr int R = CPlan<N>::r[S];
    cstage<T, N, R, P, NPEN, ES, PS, SGN, NG, GS>(buf, tw);
    cfft<T, N, S + 1, P * R, NPEN, ES, PS, SGN, NG, GS>(buf, tw);
  }
}

// One stage of the same Stockham FFT over NPEN pencils with its inputs taken
// from ld(pencil, element) and its outputs given to st(pencil, element,
// value): the first stage of a transform can read straight from global memory
// and the last one write straight to it (or fuse a pointwise product into its
// store), saving a pass of the plane through LDS.  SYNC_MID: a barrier
// between the reads and the writes (needed when both are the same LDS plane).
template <typename T, int N, int R, int P, int NPEN, int SGN, bool SYNC_MID, class Ld, class St>
__device__ __forceinline__ void cstage_io(const C2<T> *tw, Ld ld, St st) {
  constexpr int NBF = N / R;
  constexpr int TOTAL = NPEN * NBF;
  constexpr int M = N / (P * R);
  constexpr int MAXB = (TOTAL + kCT - 1) / kCT;
  C2<T> y[MAXB][R];
  int eo[MAXB], pp[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int i = threadIdx.x + c * kCT;
    eo[c] = -1;
    pp[c] = 0;
    if (TOTAL % kCT == 0 || i < TOTAL) {
      const int pa = i % NPEN, bf = i / NPEN;
      C2<T> x[R];
#pragma unroll
      for (int t = 0; t < R; ++t) x[t] = ld(pa, bf + t * NBF);
      const int k = bf % P;
      if (P > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          C2<T> w = tw[t * k * M];
          if (SGN > 0) w.y = -w.y;
          x[t] = cmul(x[t], w);
        }
      }
      Dft<T, R>::run(x, SGN);
#pragma unroll
      for (int t = 0; t < R; ++t) y[c][t] = x[t];
      eo[c] = (bf - k) * R + k;
      pp[c] = pa;
    }
  }
  if (SYNC_MID) __syncthreads();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    if (TOTAL % kCT == 0 || eo[c] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) st(pp[c], eo[c] + t * P, y[c][t]);
    }
  }
}

// A whole transform of NPEN pencils: the first stage reads through ld0 (from
// LDS if IN_LDS, else from global memory), the last one writes through stl
// (into LDS if OUT_LDS), the stages between through the LDS accessors ldm /
// stm.  A barrier follows every stage whose output is in LDS.
template <typename T, int N, int S, int P, int NPEN, int SGN, bool IN_LDS, bool OUT_LDS, class Ld0,
          class StL, class LdM, class StM>
__device__ __forceinline__ void cfft_io(const C2<T> *tw, Ld0 ld0, StL stl, LdM ldm, StM stm) {
  if constexpr (S < CPlan<N>::ns) {
    constexpr int R = CPlan<N>::r[S];
    constexpr bool first = S == 0, last = S + 1 == CPlan<N>::ns;
    constexpr bool rd = first ? IN_LDS : true, wr = last ? OUT_LDS : true;
    if constexpr (first && last)
      cstage_io<T, N, R, P, NPEN, SGN, rd && wr>(tw, ld0, stl);
    else if constexpr (first)
      cstage_io<T, N, R, P, NPEN, SGN, rd && wr>(tw, ld0, stm);
    else if constexpr (last)
      cstage_io<T, N, R, P, NPEN, SGN, rd && wr>(tw, ldm, stl);
    else
      cstage_io<T, N, R, P, NPEN, SGN, true>(tw, ldm, stm);
    if constexpr (wr) __syncthreads();
    cfft_io<T, N, S + 1, P * R, NPEN, SGN, IN_LDS, OUT_LDS>(tw, ld0, stl, ldm, stm);
  }
}

// Planes (or slabs) of one band that a batched pass keeps in LDS together:
// about 34 KB of LDS per workgroup, so that four workgroups of kCT threads per
// CU hold as much box data in flight as the 64^3 passes do.
template <typename T, int N>
constexpr int cplanes_per_item() {
  return 34000 / (N * cld<N>() * (int)sizeof(C2<T>)) > 1
             ? 34000 / (N * cld<N>() * (int)sizeof(C2<T>))
             : 1;
}


}  // namespace
}  // namespace chebfi
