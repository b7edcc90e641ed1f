// extern "C" entry points of the library (declared in include/chebfi.h).
//
// Each call validates its arguments, converts failures to status codes with a
// thread-local message, and enqueues kernels on the caller's stream.  The
// order of operations follows arXiv 2604.11139: the matrix-free H application
// (section "Main computational kernels"), the Chebyshev filter loop of
// Algorithm "Parallel Chebyshev filtering of degree k" and the S-ortho / RR
// algorithms of section "Parallel implementation design".  The drivers of the
// H / S applications, the generalised filter step and Rayleigh-Ritz live in
// driver.cpp, block LOBPCG in lobpcg.cpp; the batched filter's host side and
// the eigensolver and SCF loops are here.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>

#include "cplx.h"
#include "driver.h"
#include "kernels.h"

namespace chebfi {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

thread_local ScratchArena *g_scratch_arena = nullptr;

void *ScratchArena::take(DevBuf *b, size_t need) {
  for (const Lent &l : lent)
    if (l.buf == b && b->bytes >= need) return b->ptr;  // already lent, large enough
  const size_t start = (used + 255) / 256 * 256;
  CHEBFI_REQUIRE(start <= size && need <= size - start, ABI_ERR_NOMEM,
                 "no-allocation call: its work buffers need more than the " +
                     std::to_string(size >> 20) + " MiB scratch array");
  bool seen = false;
  for (const Lent &l : lent) seen = seen || l.buf == b;
  if (!seen) lent.push_back(Lent{b, b->ptr, b->bytes});
  used = start + need;
  b->ptr = base + start;
  b->bytes = need;
  return b->ptr;
}

namespace {
std::atomic<uint64_t> g_devbuf_gen{0};
}  // namespace

uint64_t devbuf_generation() { return g_devbuf_gen.load(); }

void *DevBuf::get(size_t need) {
  if (need == 0) need = 256;
  if (g_scratch_arena) return g_scratch_arena->take(this, need);
  if (bytes >= need) return ptr;
  release();
  ++g_devbuf_gen;
  hipError_t e = hipMalloc(&ptr, need);
  if (e != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    throw Error{ABI_ERR_NOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed"};
  }
  bytes = need;
  return ptr;
}

void DevBuf::release() {
  if (ptr) {
    ++g_devbuf_gen;
    (void)hipFree(ptr);
  }
  ptr = nullptr;
  bytes = 0;
}

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  CHEBFI_HIP(hipEventCreate(&e));
  return e;
}

int Profiler::begin(int cls, double w, hipStream_t st) {
  if (!on) return -1;
  // H-application classes: filter only
  if ((cls <= PROF_DAPPLY || cls == PROF_SPLIT) && !in_filter) return -1;
  Rec r{cls, take(), take(), w};
  CHEBFI_HIP(hipEventRecord(r.a, st));
  pending.push_back(r);
  return (int)pending.size() - 1;
}

void Profiler::end(int token, hipStream_t st) {
  if (!on || token < 0) return;
  CHEBFI_HIP(hipEventRecord(pending[token].b, st));
}

void Profiler::collect() {
  for (Rec &r : pending) {
    CHEBFI_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    CHEBFI_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    total_ms[r.cls] += ms;
    work[r.cls] += r.work;
    count[r.cls] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}

Profiler::~Profiler() {
  for (Rec &r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace chebfi

using namespace chebfi;

namespace {

template <typename F> abi_status guarded(F &&f) {
  try {
    f();
    return ABI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return ABI_ERR_NOMEM;
  } catch (...) {
    set_error("unexpected exception");
    return ABI_ERR_DEVICE;
  }
}

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

void check_desc(const abi_system_desc *d) {
  CHEBFI_REQUIRE(d != nullptr, ABI_ERR_ARG, "desc is NULL");
  CHEBFI_REQUIRE(d->abi_version == 1 || d->abi_version == 2, ABI_ERR_ARG,
                 "abi_version must be 1 or 2");
  CHEBFI_REQUIRE(d->ecut > 0.0 && std::isfinite(d->ecut), ABI_ERR_ARG, "ecut must be > 0");
  for (int c = 0; c < 3; ++c) {
    const int n = d->ngrid[c];
    CHEBFI_REQUIRE(n >= 2 && n <= kMaxN, ABI_ERR_GRID, "FFT box edge must be in [2, 96]");
    Plan1D p;
    CHEBFI_REQUIRE(make_plan(n, &p), ABI_ERR_GRID, "FFT box edge must be {2,3,5}-smooth");
  }
  CHEBFI_REQUIRE(d->natom >= 0, ABI_ERR_ARG, "natom < 0");
  if (d->natom > 0) {
    CHEBFI_REQUIRE(d->tau_cart && d->dij, ABI_ERR_ARG, "tau_cart/dij are NULL");
    CHEBFI_REQUIRE(d->rc > 0.0, ABI_ERR_ARG, "rc must be > 0");
  }
  CHEBFI_REQUIRE(d->precision == ABI_PREC_FP64 || d->precision == ABI_PREC_MIXED, ABI_ERR_ARG,
                 "unknown precision");
  double B[9];
  reciprocal(d->lattice, B);
  for (double b : B) CHEBFI_REQUIRE(std::isfinite(b), ABI_ERR_ARG, "singular lattice");
}


void free_graph_entry(abi_system_s::FilterGraph &f) {
  if (f.exec) (void)hipGraphExecDestroy(f.exec);
  if (f.graph) (void)hipGraphDestroy(f.graph);
  f = abi_system_s::FilterGraph{};
}

void free_filter_graph(abi_system_s *s) {
  for (auto &f : s->fg) free_graph_entry(f);
  s->fg_next = 0;
}

void free_tables(abi_system_s *s) {
  free_filter_graph(s);
  if (s->coef_copied) (void)hipEventSynchronize(s->coef_copied);
  if (s->coef_copied) (void)hipEventDestroy(s->coef_copied);
  s->coef_copied = nullptr;
  if (s->h_coef) (void)hipHostFree(s->h_coef);
  s->h_coef = nullptr;
  s->h_coef_n = 0;
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  s->cap_stream = nullptr;
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  if (s->ev_half) (void)hipEventDestroy(s->ev_half);
  s->ev_half = nullptr;
  if (s->aux) (void)hipStreamDestroy(s->aux);
  s->ev_fork = s->ev_join = nullptr;
  s->aux = nullptr;
  void *ptrs[] = {s->d_kin, s->d_box, s->d_plane, s->d_P, s->d_D, s->d_V, s->d_tw,
                  s->d_Pf,  s->d_Vf,  s->d_PA,    s->d_PB, s->d_Q, s->d_B, s->d_K};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  s->d_Q = s->d_B = s->d_K = nullptr;
  s->has_S = false;
  s->d_kin = nullptr;
  s->d_box = nullptr;
  s->d_plane = nullptr;
  s->d_P = nullptr;
  s->d_D = nullptr;
  s->d_V = nullptr;
  s->d_tw = nullptr;
  s->d_Pf = nullptr;
  s->d_Vf = nullptr;
  s->d_PA = nullptr;
  s->d_PB = nullptr;
}

// bf16 round-to-nearest-even of a float and its value (host side)
uint16_t bf16_rn_host(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_val_host(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void check_block(const abi_system_s *s, const void *p, int64_t nband, int64_t ld, int32_t dtype) {
  CHEBFI_REQUIRE(s != nullptr, ABI_ERR_ARG, "system handle is NULL");
  CHEBFI_REQUIRE(p != nullptr, ABI_ERR_ARG, "block pointer is NULL");
  CHEBFI_REQUIRE(nband > 0, ABI_ERR_ARG, "nband must be > 0");
  CHEBFI_REQUIRE(ld >= s->npw, ABI_ERR_ARG, "ld must be >= npw");
  CHEBFI_REQUIRE(dtype == ABI_C128 || dtype == ABI_C64, ABI_ERR_ARG, "unknown dtype");
  CHEBFI_REQUIRE(dtype == ABI_C128 || s->precision == ABI_PREC_MIXED, ABI_ERR_STATE,
                 "complex64 blocks need a handle built with ABI_PREC_MIXED");
}


}  // namespace

// ---- batched filter (host side) --------------------------------------------------
struct abi_batch_s {
  std::vector<abi_system_s *> sys;
  int precision = ABI_PREC_FP64;
  hipStream_t cap = nullptr;  // capture stream of the graphs
  // the projector products' stream beside the FFT passes, and its fork / join
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = true;
  chebfi::DevBuf d_tab, work;   // device tables [systems | steps | offsets], workspace
  void *h_tab = nullptr;        // pinned staging copy of the tables
  size_t h_tab_bytes = 0;
  hipEvent_t tab_copied = nullptr;  // the last table upload has left h_tab
  std::vector<chebfi::BatchSys> hsys;
  std::vector<chebfi::BatchStep> hsteps;
  std::vector<int64_t> hoff;
  int fft_threads = 512, proj_threads = 256, radix_desc = 0, fft_min_threads = 64;
  bool use_graph = true;
  // the captured graph and what it was captured for
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> g_nband;
  int g_degree = -1, g_dtype = -1, g_fft = 0, g_proj = 0;
  bool g_overlap = false;
  const void *g_sys = nullptr, *g_steps = nullptr, *g_off = nullptr;
};

namespace chebfi {
namespace {

BoxPlan ordered_plan(const BoxPlan &p, bool descending) {
  BoxPlan q = p;
  if (descending)
    for (int d = 0; d < 3; ++d) std::reverse(q.d[d].radix, q.d[d].radix + q.d[d].nstage);
  return q;
}

template <typename T>
void batch_run(abi_batch_s *B, const BatchLaunch &L, int degree, int32_t dtype,
               const std::vector<int64_t> &nb, hipStream_t st) {
  batch_prepare<T>(L);
  hipStream_t side = B->overlap ? B->side : nullptr;
  if (!B->use_graph) {
    for (int j = 0; j < degree; ++j) batch_step<T>(L, j, st, side, B->ev_fork, B->ev_join);
    return;
  }
  const bool same = B->gexec && B->g_nband == nb && B->g_degree == degree && B->g_dtype == dtype &&
                    B->g_fft == L.fft_threads && B->g_proj == L.proj_threads &&
                    B->g_sys == L.d_sys && B->g_steps == L.d_steps && B->g_off == L.d_off &&
                    B->g_overlap == B->overlap;
  if (!same) {
    if (B->gexec) {
      CHEBFI_HIP(hipGraphExecDestroy(B->gexec));
      B->gexec = nullptr;
    }
    hipGraph_t g = nullptr;
    CHEBFI_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    try {
      for (int j = 0; j < degree; ++j) batch_step<T>(L, j, B->cap, side, B->ev_fork, B->ev_join);
    } catch (...) {
      (void)hipStreamEndCapture(B->cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    CHEBFI_HIP(hipStreamEndCapture(B->cap, &g));
    const hipError_t e = hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CHEBFI_HIP(e);
    B->g_nband = nb;
    B->g_degree = degree;
    B->g_dtype = dtype;
    B->g_fft = L.fft_threads;
    B->g_proj = L.proj_threads;
    B->g_sys = L.d_sys;
    B->g_steps = L.d_steps;
    B->g_off = L.d_off;
    B->g_overlap = B->overlap;
  }
  CHEBFI_HIP(hipGraphLaunch(B->gexec, st));
}

}  // namespace

void batch_filter(abi_batch_s *B, const void *const *X, void *const *Y, const int64_t *nband,
                  const int64_t *ld, int32_t dtype, int32_t degree, const double *a,
                  const double *b, const double *a0, hipStream_t st) {
  CHEBFI_REQUIRE(B != nullptr, ABI_ERR_ARG, "batch is NULL");
  CHEBFI_REQUIRE(X && Y && nband && ld && a && b && a0, ABI_ERR_ARG, "NULL argument array");
  CHEBFI_REQUIRE(degree >= 1, ABI_ERR_ARG, "degree must be >= 1");
  const int nsys = (int)B->sys.size();
  const bool fp32 = (dtype == ABI_C64);
  for (int i = 0; i < nsys; ++i) {
    check_block(B->sys[i], X[i], nband[i], ld[i], dtype);
    CHEBFI_REQUIRE(Y[i] != nullptr && Y[i] != X[i], ABI_ERR_ARG, "Y must be a separate block");
    CHEBFI_REQUIRE(std::isfinite(a[i]) && std::isfinite(b[i]) && std::isfinite(a0[i]),
                   ABI_ERR_ARG, "bounds must be finite");
    CHEBFI_REQUIRE(b[i] > a[i], ABI_ERR_ARG, "need b > a");
    CHEBFI_REQUIRE(a0[i] <= a[i], ABI_ERR_ARG, "need a0 <= a");
  }
  const size_t esz = elem_bytes(dtype);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  // workspace: boxes, C', E = P C', two iterate slots per system
  std::vector<size_t> o_box(nsys), o_cp(nsys), o_e(nsys), o_part(nsys), o_slot(nsys);
  size_t tot = 0;
  int min_threads = 64;
  size_t lds_a = 0, lds_b = 0;
  bool any_proj = false;
  for (int i = 0; i < nsys; ++i) {
    const abi_system_s *s = B->sys[i];
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    o_box[i] = tot;
    tot += al(esz * (size_t)nbox * nband[i]);
    o_cp[i] = tot;
    tot += al(esz * (size_t)std::max(s->nproj, 1) * nband[i]);
    o_e[i] = tot;
    if (s->nproj > 0) tot += al(esz * (size_t)s->npw * nband[i]);
    o_part[i] = tot;
    if (s->nproj > 0)
      tot += al(sizeof(double2) * (size_t)((nband[i] + kBatchBT - 1) / kBatchBT) *
                (size_t)((s->nproj + kBatchPT - 1) / kBatchPT) *
                (size_t)((s->npw + kBatchKC - 1) / kBatchKC) * kBatchPT * kBatchBT);
    o_slot[i] = tot;
    if (degree >= 2) tot += 2 * al(esz * (size_t)s->npw * nband[i]);
    min_threads = std::max({min_threads, fft_stage_threads(s->plan.d[0], s->n2),
                            fft_stage_threads(s->plan.d[1], s->n1),
                            fft_stage_threads(s->plan.d[2], s->n1)});
    lds_a = std::max(lds_a, (size_t)(s->n2 * (s->n1 + 1) + s->n1 + s->n2));
    lds_b = std::max(lds_b, (size_t)(s->n3 * (s->n1 + 1) + s->n3));
    any_proj = any_proj || s->nproj > 0;
  }
  CHEBFI_REQUIRE(min_threads <= 512, ABI_ERR_GRID, "FFT plane too large for one workgroup");
  B->fft_min_threads = min_threads;
  if (B->fft_threads < min_threads) B->fft_threads = min_threads <= 256 ? 256 : 512;
  char *ws = (char *)B->work.get(tot);
  // per-system descriptors and item offsets
  B->hoff.assign(5 * (size_t)(nsys + 1), 0);
  int64_t *offP = B->hoff.data(), *offA = offP + (nsys + 1), *offB = offA + (nsys + 1);
  int64_t *offE = offB + (nsys + 1), *offR = offE + (nsys + 1);
  for (int i = 0; i < nsys; ++i) {
    const abi_system_s *s = B->sys[i];
    BatchSys &d = B->hsys[i];
    d.plan = ordered_plan(s->plan, B->radix_desc != 0);
    d.npw = s->npw;
    d.nproj = s->nproj;
    d.npt = (s->nproj + kBatchPT - 1) / kBatchPT;
    d.box_index = s->d_box;
    d.plane = s->d_plane;
    d.zocc = s->zocc;
    d.kin = s->d_kin;
    d.V = fp32 ? (const void *)s->d_Vf : (const void *)s->d_V;
    d.tw = reinterpret_cast<const double2 *>(s->d_tw);
    d.P = fp32 ? (const void *)s->d_Pf : (const void *)s->d_P;
    d.D = reinterpret_cast<const double2 *>(s->d_D);
    d.nband = nband[i];
    d.box = ws + o_box[i];
    d.Cp = ws + o_cp[i];
    d.E = ws + o_e[i];
    d.Cpart = (double2 *)(ws + o_part[i]);
    // projector products in tiles of kBatchBT bands (x kBatchPT projectors x
    // kBatchKC-wave chunks for the projection, x kBatchEP plane waves for the
    // expansion)
    const int64_t nbt = s->nproj > 0 ? (nband[i] + kBatchBT - 1) / kBatchBT : 0;
    offP[i + 1] = offP[i] + nbt * d.npt * ((s->npw + kBatchKC - 1) / kBatchKC);
    offR[i + 1] = offR[i] + (s->nproj > 0 ? (nband[i] + kBatchBR - 1) / kBatchBR * d.npt : 0);
    offE[i + 1] = offE[i] + nbt * ((s->npw + kBatchEP - 1) / kBatchEP);
    // systems on cubic boxes with specialised passes go to their edge group and
    // contribute no items to the runtime-size passes
    const bool grouped = s->n1 == s->n2 && s->n1 == s->n3 && batch_edge_specialised(s->n1) &&
                         !s->generic_fft;
    offA[i + 1] = offA[i] + (grouped ? 0 : nband[i] * s->n3);
    offB[i + 1] = offB[i] + (grouped ? 0 : nband[i] * s->n2);
  }
  // edge groups: system lists and item offsets (appended to the device table)
  std::vector<int> gedge;
  std::vector<std::vector<int32_t>> glist;
  for (int i = 0; i < nsys; ++i) {
    const abi_system_s *s = B->sys[i];
    if (offA[i + 1] != offA[i] || !(s->n1 == s->n2 && s->n1 == s->n3)) continue;
    if (!batch_edge_specialised(s->n1) || s->generic_fft) continue;
    size_t g = 0;
    while (g < gedge.size() && gedge[g] != s->n1) ++g;
    if (g == gedge.size()) {
      gedge.push_back(s->n1);
      glist.emplace_back();
    }
    glist[g].push_back(i);
  }
  CHEBFI_REQUIRE((int)gedge.size() <= kBatchMaxGroups, ABI_ERR_ARG, "too many box sizes");
  std::vector<int32_t> hgsys;
  std::vector<int64_t> hgoff;
  std::vector<size_t> gsys_at, goff_at;
  for (size_t g = 0; g < gedge.size(); ++g) {
    gsys_at.push_back(hgsys.size());
    goff_at.push_back(hgoff.size());
    hgoff.push_back(0);
    const int npl = batch_item_planes(gedge[g], fp32);
    for (int32_t i : glist[g]) {
      hgsys.push_back(i);
      hgoff.push_back(hgoff.back() + nband[i] * ((gedge[g] + npl - 1) / npl));
    }
  }
  // step table: Y_0 = X, Y_m = Y, Y_j (0 < j < m) in slot j % 2 (the update of
  // step j reads Y_{j-2} and writes Y_j element by element in the same thread)
  B->hsteps.assign((size_t)degree * nsys, BatchStep{});
  for (int i = 0; i < nsys; ++i) {
    const abi_system_s *s = B->sys[i];
    const double e = (b[i] - a[i]) / 2.0, c = (b[i] + a[i]) / 2.0, s1 = e / (a0[i] - c);
    const int64_t npw = s->npw;
    auto iter = [&](int j, int64_t *ldj) -> void * {
      if (j == 0) {
        *ldj = ld[i];
        return const_cast<void *>(X[i]);
      }
      if (j == degree) {
        *ldj = ld[i];
        return Y[i];
      }
      *ldj = npw;
      return ws + o_slot[i] + (size_t)(j % 2) * al(esz * (size_t)npw * nband[i]);
    };
    double sk = s1;
    for (int j = 1; j <= degree; ++j) {
      BatchStep &p = B->hsteps[(size_t)(j - 1) * nsys + i];
      p.yk = iter(j - 1, &p.ldk);
      p.out = iter(j, &p.ldo);
      p.cshift = c;
      if (j == 1) {
        p.alpha = s1 / e;
        p.beta = 0.0;
        p.yprev = nullptr;
        p.ldp = 0;
      } else {
        const double sk1 = 1.0 / (2.0 / s1 - sk);
        p.alpha = 2.0 * sk1 / e;
        p.beta = sk * sk1;
        sk = sk1;
        p.yprev = iter(j - 2, &p.ldp);
      }
    }
  }
  // one upload of the tables from a pinned staging buffer, ordered on the
  // caller's stream after the previous filter of this batch
  const size_t t_sys = al(sizeof(BatchSys) * (size_t)nsys);
  const size_t t_steps = al(sizeof(BatchStep) * B->hsteps.size());
  const size_t t_off = al(sizeof(int64_t) * B->hoff.size());
  const size_t t_gsys = al(sizeof(int32_t) * std::max<size_t>(hgsys.size(), 1));
  const size_t t_goff = al(sizeof(int64_t) * std::max<size_t>(hgoff.size(), 1));
  const size_t t_all = t_sys + t_steps + t_off + t_gsys + t_goff;
  if (B->tab_copied) CHEBFI_HIP(hipEventSynchronize(B->tab_copied));
  if (B->h_tab_bytes < t_all) {
    if (B->h_tab) CHEBFI_HIP(hipHostFree(B->h_tab));
    B->h_tab = nullptr;
    B->h_tab_bytes = 0;
    CHEBFI_HIP(hipHostMalloc(&B->h_tab, t_all, hipHostMallocDefault));
    B->h_tab_bytes = t_all;
  }
  if (!B->tab_copied) CHEBFI_HIP(hipEventCreateWithFlags(&B->tab_copied, hipEventDisableTiming));
  char *ht = (char *)B->h_tab;
  std::memcpy(ht, B->hsys.data(), sizeof(BatchSys) * (size_t)nsys);
  std::memcpy(ht + t_sys, B->hsteps.data(), sizeof(BatchStep) * B->hsteps.size());
  std::memcpy(ht + t_sys + t_steps, B->hoff.data(), sizeof(int64_t) * B->hoff.size());
  if (!hgsys.empty())
    std::memcpy(ht + t_sys + t_steps + t_off, hgsys.data(), sizeof(int32_t) * hgsys.size());
  if (!hgoff.empty())
    std::memcpy(ht + t_sys + t_steps + t_off + t_gsys, hgoff.data(),
                sizeof(int64_t) * hgoff.size());
  char *dt = (char *)B->d_tab.get(t_all);
  CHEBFI_HIP(hipMemcpyAsync(dt, ht, t_all, hipMemcpyHostToDevice, st));
  CHEBFI_HIP(hipEventRecord(B->tab_copied, st));
  void *dsys = dt, *dsteps = dt + t_sys, *doff = dt + t_sys + t_steps;
  BatchLaunch L;
  L.nsys = nsys;
  L.d_sys = (const BatchSys *)dsys;
  L.d_steps = (const BatchStep *)dsteps;
  L.d_off = (const int64_t *)doff;
  L.items_p = offP[nsys];
  L.items_e = offE[nsys];
  L.items_r = offR[nsys];
  L.items_a = offA[nsys];
  L.items_b = offB[nsys];
  L.max_wgs = 2048;
  L.ngroups = (int)gedge.size();
  for (size_t g = 0; g < gedge.size(); ++g) {
    BatchGroup &G = L.groups[g];
    G.n = gedge[g];
    G.nsys = (int)glist[g].size();
    G.gsys = (const int32_t *)(dt + t_sys + t_steps + t_off) + gsys_at[g];
    G.goff = (const int64_t *)(dt + t_sys + t_steps + t_off + t_gsys) + goff_at[g];
    G.items = hgoff[goff_at[g] + G.nsys];
  }
  L.fft_threads = B->fft_threads;
  L.proj_threads = B->proj_threads;
  L.lds_a = lds_a;
  L.lds_b = lds_b;
  L.lds_c = lds_a;
  L.any_proj = any_proj;
  std::vector<int64_t> nb(nband, nband + nsys);
  if (fp32)
    batch_run<float>(B, L, degree, dtype, nb, st);
  else
    batch_run<double>(B, L, degree, dtype, nb, st);
}

}  // namespace chebfi

extern "C" {

const char *abi_last_error(void) { return g_last_error.c_str(); }

abi_status abi_gsphere_count(const abi_system_desc *desc, int64_t *npw) {
  return guarded([&] {
    check_desc(desc);
    CHEBFI_REQUIRE(npw != nullptr, ABI_ERR_ARG, "npw is NULL");
    Sphere sp;
    std::string err;
    abi_status st = build_sphere(desc, &sp, &err);
    if (st != ABI_OK) throw Error{st, err};
    *npw = (int64_t)sp.kinetic.size();
  });
}

abi_status abi_gsphere_build(const abi_system_desc *desc, int64_t npw, int32_t *miller,
                             int32_t *box_index, double *kinetic) {
  return guarded([&] {
    check_desc(desc);
    Sphere sp;
    std::string err;
    abi_status st = build_sphere(desc, &sp, &err);
    if (st != ABI_OK) throw Error{st, err};
    CHEBFI_REQUIRE(npw == (int64_t)sp.kinetic.size(), ABI_ERR_ARG, "npw does not match the basis");
    if (miller) std::memcpy(miller, sp.miller.data(), sizeof(int32_t) * 3 * npw);
    if (box_index) std::memcpy(box_index, sp.box_index.data(), sizeof(int32_t) * npw);
    if (kinetic) std::memcpy(kinetic, sp.kinetic.data(), sizeof(double) * npw);
  });
}

abi_status abi_set_system(const abi_system_desc *desc, void *stream, abi_system *out) {
  abi_system_s *s = nullptr;
  abi_status rc = guarded([&] {
    check_desc(desc);
    CHEBFI_REQUIRE(out != nullptr, ABI_ERR_ARG, "out is NULL");
    CHEBFI_REQUIRE(desc->vloc != nullptr, ABI_ERR_ARG, "vloc is NULL");
    s = new abi_system_s();
    CHEBFI_HIP(hipGetDevice(&s->device));
    s->scratch = scratch_for_device(s->device);
    s->n1 = desc->ngrid[0];
    s->n2 = desc->ngrid[1];
    s->n3 = desc->ngrid[2];
    s->natom = desc->natom;
    s->nproj = 4 * desc->natom;
    s->precision = desc->precision;
    for (int i = 0; i < 9; ++i) s->lattice[i] = desc->lattice[i];
    {
      const double *a = desc->lattice;
      s->omega = std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                           a[2] * (a[3] * a[7] - a[4] * a[6]));
    }
    std::string err;
    abi_status st = build_sphere(desc, &s->sphere, &err);
    if (st != ABI_OK) throw Error{st, err};
    s->npw = (int64_t)s->sphere.kinetic.size();
    CHEBFI_REQUIRE(s->npw > 0, ABI_ERR_ARG, "empty basis");
    for (int c = 0; c < 3; ++c) make_plan(desc->ngrid[c], &s->plan.d[c]);
    const int64_t nxy = (int64_t)s->n1 * s->n2;
    const int64_t nbox = nxy * s->n3;
    std::vector<int32_t> plane(s->n3 + 1, 0);
    {
      int64_t idx = 0;
      for (int i3 = 0; i3 <= s->n3; ++i3) {
        while (idx < s->npw && s->sphere.box_index[idx] < (int64_t)i3 * nxy) ++idx;
        plane[i3] = (int32_t)idx;
      }
      plane[s->n3] = (int32_t)s->npw;
    }
    s->zocc = ~0ull;
    if (s->n3 <= 64) {
      s->zocc = 0;
      for (int i3 = 0; i3 < s->n3; ++i3)
        if (plane[i3] < plane[i3 + 1]) s->zocc |= 1ull << i3;
    }
    std::vector<double> tw(3 * kMaxN * 2, 0.0);
    for (int c = 0; c < 3; ++c) {
      const int n = desc->ngrid[c];
      for (int j = 0; j < n; ++j) {
        const double ang = 2.0 * M_PI * (double)j / (double)n;
        tw[2 * (c * kMaxN + j)] = std::cos(ang);
        tw[2 * (c * kMaxN + j) + 1] = -std::sin(ang);
      }
    }
    std::vector<double> P;
    build_projectors(desc, s->sphere, &P);
    s->d_kin = upload(s->sphere.kinetic.data(), s->npw);
    s->d_box = upload(s->sphere.box_index.data(), s->npw);
    s->d_plane = upload(plane.data(), plane.size());
    s->d_P = upload(P.data(), P.size());
    s->d_D = upload(desc->dij, (size_t)desc->natom * 32);
    s->d_V = upload(desc->vloc, (size_t)nbox);
    s->d_tw = upload(tw.data(), tw.size());
    if (s->precision == ABI_PREC_MIXED) {
      std::vector<float> Pf(P.size()), Vf((size_t)nbox);
      for (size_t i = 0; i < P.size(); ++i) Pf[i] = (float)P[i];
      for (int64_t i = 0; i < nbox; ++i) Vf[i] = (float)desc->vloc[i];
      s->d_Pf = upload(Pf.data(), Pf.size());
      s->d_Vf = upload(Vf.data(), Vf.size());
      // split-BF16 planes in the two k-contiguous layouts the projector GEMMs read
      const int64_t npw = s->npw, np = s->nproj;
      s->ldPA = (npw + 63) / 64 * 64;
      s->ldPB = (np + 31) / 32 * 32;  // zero planes up to the 32-wide K slices
      const size_t szA = (size_t)np * s->ldPA, szB = (size_t)npw * s->ldPB;
      std::vector<uint16_t> PA(4 * szA, 0), PB(4 * szB, 0);
      for (int64_t j = 0; j < np; ++j)
        for (int64_t g = 0; g < npw; ++g) {
          const size_t src = 2 * ((size_t)j * npw + g);
          for (int part = 0; part < 2; ++part) {
            const float x = Pf[src + part];
            const uint16_t hi = bf16_rn_host(x);
            const uint16_t lo = bf16_rn_host(x - bf16_val_host(hi));
            PA[(size_t)part * szA + j * s->ldPA + g] = hi;
            PA[(size_t)(2 + part) * szA + j * s->ldPA + g] = lo;
            PB[(size_t)part * szB + g * s->ldPB + j] = hi;
            PB[(size_t)(2 + part) * szB + g * s->ldPB + j] = lo;
          }
        }
      s->d_PA = upload(PA.data(), PA.size());
      s->d_PB = upload(PB.data(), PB.size());
      // tile variants of the split-BF16 products (abi_set_tuning, abi_autotune):
      // both default to the direct-to-LDS 128 x 128 tile with eight waves and the
      // scheduled fragment reads (the projection splits the block into planes as
      // it reads its fragments; the expansion's workgroups run through several
      // tiles)
      s->pl_proj = 14;
      s->pl_expand = 15;
    }
    // bands per FFT batch: keep the box buffer near 128 MiB
    const int64_t fb = (int64_t)((128ll << 20) / (sizeof(double2) * nbox));
    s->fft_batch = (int)std::max<int64_t>(1, std::min<int64_t>(fb, 4096));
    // FFT passes beside the projection GEMM on a second stream (default priority)
    CHEBFI_HIP(hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking));
    CHEBFI_HIP(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    CHEBFI_HIP(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    CHEBFI_HIP(hipEventCreateWithFlags(&s->ev_half, hipEventDisableTiming));
    s->overlap = 0;
    if (desc->abi_version >= 2 && desc->qij != nullptr) setup_overlap(s, desc->qij, S(stream));
    CHEBFI_HIP(hipStreamSynchronize(S(stream)));
    *out = s;
  });
  if (rc != ABI_OK && s) {
    free_tables(s);
    delete s;
  }
  return rc;
}

abi_status abi_system_info(abi_system s, int64_t *npw, int32_t *nproj, int32_t ngrid[3]) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr, ABI_ERR_ARG, "system handle is NULL");
    if (npw) *npw = s->npw;
    if (nproj) *nproj = s->nproj;
    if (ngrid) {
      ngrid[0] = s->n1;
      ngrid[1] = s->n2;
      ngrid[2] = s->n3;
    }
  });
}

abi_status abi_get_gsphere(abi_system s, int32_t *miller, int32_t *box_index) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr, ABI_ERR_ARG, "system handle is NULL");
    if (miller) std::memcpy(miller, s->sphere.miller.data(), sizeof(int32_t) * 3 * s->npw);
    if (box_index) std::memcpy(box_index, s->sphere.box_index.data(), sizeof(int32_t) * s->npw);
  });
}

abi_status abi_get_projectors(abi_system s, void *P_out, void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr && P_out != nullptr, ABI_ERR_ARG, "NULL argument");
    const size_t bytes = sizeof(double2) * (size_t)s->npw * (size_t)std::max(s->nproj, 0);
    if (bytes)
      CHEBFI_HIP(hipMemcpyAsync(P_out, s->d_P, bytes, hipMemcpyDeviceToDevice, S(stream)));
    CHEBFI_HIP(hipStreamSynchronize(S(stream)));
  });
}

abi_status abi_destroy(abi_system s) {
  return guarded([&] {
    if (!s) return;
    (void)hipDeviceSynchronize();
    free_tables(s);
    delete s;
  });
}

abi_status abi_apply_H(abi_system s, const void *X, void *HX, int64_t nband, int64_t ld,
                       int32_t dtype, void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(HX != nullptr, ABI_ERR_ARG, "HX is NULL");
    CHEBFI_REQUIRE(HX != X, ABI_ERR_ARG, "X and HX must not overlap");
    apply_core(s, X, ld, nullptr, 0, HX, ld, nband, 1.0, 0.0, 0.0, S(stream), dtype);
  });
}

abi_status abi_apply_H_noalloc(abi_system s, const void *X, void *HX, int64_t nband, int64_t ld,
                               int32_t dtype, void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(HX != nullptr, ABI_ERR_ARG, "HX is NULL");
    CHEBFI_REQUIRE(HX != X, ABI_ERR_ARG, "X and HX must not overlap");
    CHEBFI_REQUIRE(!s->prof.on, ABI_ERR_STATE,
                   "timing creates events: turn it off for the no-allocation call");
    CHEBFI_REQUIRE(s->scratch != nullptr, ABI_ERR_STATE, "no scratch array on this device");
    ScratchArena arena;
    arena.base = (char *)s->scratch;
    arena.size = scratch_bytes();
    const bool fp32 = dtype == ABI_C64;
    if (!fp32 && s->nproj > 0) {
      // the FP64 path runs the FFT passes before the projector products: keep
      // room for the split-K parts and C' behind the box batch
      const int64_t splits = nband == 1 ? 1 : zgemm_splits(s->nproj, nband, s->npw);
      arena.reserve = sizeof(double2) * (size_t)s->nproj * nband * (splits + 1) + 512;
    }
    const int overlap = s->overlap;
    s->overlap = 0;  // one stream: the second one's events are not needed
    try {
      ArenaScope scope(&arena);
      apply_core(s, X, ld, nullptr, 0, HX, ld, nband, 1.0, 0.0, 0.0, S(stream), dtype);
    } catch (...) {
      s->overlap = overlap;
      throw;
    }
    s->overlap = overlap;
  });
}

namespace chebfi {
namespace {

// The filter; HX (ld ld, or NULL) is H X given by the caller, which turns the
// first step into Y_1 = (s1/e)(HX - c X).
void cheb_filter_impl(abi_system s, const void *X, const void *HX, void *Y, int64_t nband,
                      int64_t ld, int32_t dtype, int32_t degree, double a, double b, double a0,
                      hipStream_t st) {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(Y != nullptr && Y != X, ABI_ERR_ARG, "Y must be a separate block");
    CHEBFI_REQUIRE(HX == nullptr || (HX != Y && HX != X), ABI_ERR_ARG,
                   "HX must not alias X or Y");
    CHEBFI_REQUIRE(HX == nullptr || !s->has_S, ABI_ERR_STATE,
                   "a given H X serves the filter on H only (S = I)");
    CHEBFI_REQUIRE(degree >= 1, ABI_ERR_ARG, "degree must be >= 1");
    CHEBFI_REQUIRE(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0), ABI_ERR_ARG,
                   "bounds must be finite");
    CHEBFI_REQUIRE(b > a, ABI_ERR_ARG, "need b > a");
    CHEBFI_REQUIRE(a0 <= a, ABI_ERR_ARG, "need a0 <= a");
    const int64_t npw = s->npw;
    const double e = (b - a) / 2.0, c = (b + a) / 2.0;
    const double s1 = e / (a0 - c);
    // Y_j lives in bufs[(degree - j) % 3] so that Y_degree lands in Y.
    void *bufs[3] = {Y, nullptr, nullptr};
    int64_t lds[3] = {ld, npw, npw};
    const size_t eb = elem_bytes(dtype);
    if (degree >= 2) bufs[1] = s->blk1.get(eb * (size_t)npw * nband);
    if (degree >= 3) bufs[2] = s->blk2.get(eb * (size_t)npw * nband);
    auto slot = [&](int j) { return (degree - j) % 3; };
    struct Scope {
      Profiler &p;
      explicit Scope(Profiler &q) : p(q) { p.in_filter = true; }
      ~Scope() { p.in_filter = false; }
    } scope(s->prof);
    if (s->has_S) {
      // polynomial of S^-1 H; C_j = P^H Y_j rides along in Cs[j % 3]
      const size_t nc = (size_t)s->nproj * nband;
      double2 *cbase = (double2 *)s->gen_c.get(3 * sizeof(double2) * nc);
      double2 *Cs[3] = {cbase, cbase + nc, cbase + 2 * nc};
      project_c128(s, X, ld, nband, Cs[0], st, dtype);
      auto step = [&](const void *yk, int64_t ldk, const void *yp, int64_t ldp, void *out,
                      int64_t ldo, double al, double be, int j) {
        const double2 *cm1 = yp ? Cs[(j + 2) % 3] : nullptr;
        gen_step(s, yk, ldk, yp, ldp, out, ldo, nband, al, c, be, Cs[j % 3], cm1,
                 Cs[(j + 1) % 3], st, dtype);
      };
      step(X, ld, nullptr, 0, bufs[slot(1)], lds[slot(1)], s1 / e, 0.0, 0);
      double sk = s1;
      for (int j = 1; j < degree; ++j) {
        const double sk1 = 1.0 / (2.0 / s1 - sk);
        const void *yp = (j == 1) ? X : bufs[slot(j - 1)];
        const int64_t ldp = (j == 1) ? ld : lds[slot(j - 1)];
        step(bufs[slot(j)], lds[slot(j)], yp, ldp, bufs[slot(j + 1)], lds[slot(j + 1)],
             2.0 * sk1 / e, sk * sk1, j);
        sk = sk1;
      }
      return;
    }
    // (alpha, cshift, beta) of steps 1 .. degree
    std::vector<double> cf(3 * (size_t)degree);
    {
      cf[0] = s1 / e;
      cf[1] = c;
      cf[2] = 0.0;
      double sk = s1;
      for (int j = 1; j < degree; ++j) {
        const double sk1 = 1.0 / (2.0 / s1 - sk);
        cf[3 * j] = 2.0 * sk1 / e;
        cf[3 * j + 1] = c;
        cf[3 * j + 2] = sk * sk1;
        sk = sk1;
      }
    }
    // The launches of the filter on stream q; with dc (device copy of cf) the
    // kernels take each step's coefficients from it (same values, same bits).
    auto run = [&](hipStream_t q, const double *dc) {
      struct CoefScope {
        abi_system_s *s;
        ~CoefScope() {
          s->coef_dev = nullptr;
          s->pl_chain = false;
          s->pl_have = nullptr;
        }
      } scope_c{s};
      // each step's last FFT pass writes the bf16 planes of its output for the
      // next step's projection (variants that read planes)
      s->pl_chain = true;
      s->pl_have = nullptr;
      // Y_1 = (s1/e)(H - c) X
      s->coef_dev = dc;
      if (HX)
        launch_cheb_first(npw, nband, X, ld, HX, ld, cf[0], c, bufs[slot(1)], lds[slot(1)], q,
                          dtype == ABI_C64, dc);
      else
        apply_core(s, X, ld, nullptr, 0, bufs[slot(1)], lds[slot(1)], nband, cf[0], c, 0.0, q,
                   dtype);
      for (int j = 1; j < degree; ++j) {
        const void *yk = bufs[slot(j)];
        const int64_t ldk = lds[slot(j)];
        const void *yp = (j == 1) ? X : bufs[slot(j - 1)];
        const int64_t ldp = (j == 1) ? ld : lds[slot(j - 1)];
        s->coef_dev = dc ? dc + 3 * j : nullptr;
        apply_core(s, yk, ldk, yp, ldp, bufs[slot(j + 1)], lds[slot(j + 1)], nband, cf[3 * j], c,
                   cf[3 * j + 2], q, dtype);
      }
    };
    // captured form: not with the second stream, the profiler's events, or inside a
    // no-allocation call
    const bool graph = s->filter_graph && !(s->overlap && s->nproj > 0 && s->aux) &&
                       !s->prof.on && g_scratch_arena == nullptr;
    if (!graph) {
      run(st, nullptr);
      return;
    }
    // upload the coefficients through pinned memory (the previous upload is
    // complete before the staging buffer is rewritten)
    const size_t nc = cf.size();
    if (!s->coef_copied)
      CHEBFI_HIP(hipEventCreateWithFlags(&s->coef_copied, hipEventDisableTiming));
    else
      CHEBFI_HIP(hipEventSynchronize(s->coef_copied));
    if (s->h_coef_n < nc) {
      if (s->h_coef) CHEBFI_HIP(hipHostFree(s->h_coef));
      s->h_coef = nullptr;
      s->h_coef_n = 0;
      CHEBFI_HIP(hipHostMalloc((void **)&s->h_coef, sizeof(double) * nc, hipHostMallocDefault));
      s->h_coef_n = nc;
    }
    std::memcpy(s->h_coef, cf.data(), sizeof(double) * nc);
    double *dc = (double *)s->coef.get(sizeof(double) * nc);
    CHEBFI_HIP(hipMemcpyAsync(dc, s->h_coef, sizeof(double) * nc, hipMemcpyHostToDevice, st));
    CHEBFI_HIP(hipEventRecord(s->coef_copied, st));
    const uint64_t key[16] = {(uint64_t)(uintptr_t)X,  (uint64_t)(uintptr_t)HX,
                              (uint64_t)(uintptr_t)Y,  (uint64_t)nband,
                              (uint64_t)ld,            (uint64_t)dtype,
                              (uint64_t)degree,        (uint64_t)s->pl_proj,
                              (uint64_t)s->pl_expand,  (uint64_t)s->fft_batch,
                              (uint64_t)s->generic_fft, (uint64_t)s->mixed_gemm,
                              (uint64_t)s->overlap,    (uint64_t)(uintptr_t)dc,
                              devbuf_generation(),     1};
    for (auto &f : s->fg) {
      if (f.exec && std::memcmp(key, f.key, sizeof(key)) == 0) {
        CHEBFI_HIP(hipGraphLaunch(f.exec, st));
        return;
      }
    }
    // first call with these arguments: run eagerly (this also sizes every work
    // buffer), then record the same launches on the capture stream
    run(st, dc);
    abi_system_s::FilterGraph &slotg = s->fg[s->fg_next];
    s->fg_next = (s->fg_next + 1) % abi_system_s::kFilterGraphs;
    free_graph_entry(slotg);
    if (!s->cap_stream) CHEBFI_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    CHEBFI_HIP(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      run(s->cap_stream, dc);
    } catch (...) {
      (void)hipStreamEndCapture(s->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      s->filter_graph = 0;  // (the result is in Y already; later calls run eagerly)
      return;
    }
    CHEBFI_HIP(hipStreamEndCapture(s->cap_stream, &g));
    slotg.graph = g;
    CHEBFI_HIP(hipGraphInstantiate(&slotg.exec, slotg.graph, nullptr, nullptr, 0));
    std::memcpy(slotg.key, key, sizeof(key));
    slotg.key[14] = devbuf_generation();  // (unchanged unless the recording allocated)
}

}  // namespace
}  // namespace chebfi

abi_status abi_cheb_filter(abi_system s, const void *X, void *Y, int64_t nband, int64_t ld,
                           int32_t dtype, int32_t degree, double a, double b, double a0,
                           void *stream) {
  return guarded([&] {
    cheb_filter_impl(s, X, nullptr, Y, nband, ld, dtype, degree, a, b, a0, S(stream));
  });
}

abi_status abi_cheb_filter_hx(abi_system s, const void *X, const void *HX, void *Y,
                              int64_t nband, int64_t ld, int32_t dtype, int32_t degree, double a,
                              double b, double a0, void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(HX != nullptr, ABI_ERR_ARG, "HX is NULL");
    cheb_filter_impl(s, X, HX, Y, nband, ld, dtype, degree, a, b, a0, S(stream));
  });
}

abi_status abi_spectral_bounds(abi_system s, const void *X, int64_t nband, int64_t ld,
                               int32_t dtype, const void *v0, int32_t nlanczos, double *out,
                               void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(v0 != nullptr && out != nullptr, ABI_ERR_ARG, "NULL argument");
    CHEBFI_REQUIRE(nlanczos >= 1 && nlanczos <= 64, ABI_ERR_ARG, "nlanczos must be in [1, 64]");
    hipStream_t st = S(stream);
    const int64_t npw = s->npw;
    void *HX = s->blk3.get(elem_bytes(dtype) * (size_t)npw * nband);
    // scalars: [0..2] out, [8..8+64) alpha, [80..80+64) beta, rq after 160
    double *scal = (double *)s->scal.get(sizeof(double) * (size_t)(160 + nband));
    double *alpha = scal + 8, *beta = scal + 80, *rq = scal + 160;
    apply_core(s, X, ld, nullptr, 0, HX, npw, nband, 1.0, 0.0, 0.0, st, dtype);
    if (s->has_S) {
      // generalised quotients Re(x^H H x) / Re(x^H S x)
      void *SX = s->blk5.get(elem_bytes(dtype) * (size_t)npw * nband);
      apply_S(s, X, ld, SX, npw, nband, st, dtype);
      launch_rayleigh_quotients(npw, nband, X, ld, HX, npw, rq, st, dtype == ABI_C64, SX, npw);
    } else {
      launch_rayleigh_quotients(npw, nband, X, ld, HX, npw, rq, st, dtype == ABI_C64);
    }
    launch_minmax(nband, rq, scal, st);
    // Lanczos basis V (npw x (nl+1)), residual w, projections h
    const int nl = nlanczos;
    double2 *V = (double2 *)s->blk2.get(sizeof(double2) * (size_t)npw * (nl + 2));
    double2 *w = V + (size_t)npw * (nl + 1);
    double2 *h = (double2 *)s->small4.get(sizeof(double2) * 128);
    int k = nl;
    int add_last = 1;
    if (s->has_S) {
      // Lanczos on S^-1 H in the S inner product: SV holds S v_j beside v_j
      double2 *SV = (double2 *)s->blk6.get(sizeof(double2) * (size_t)npw * (nl + 3));
      double2 *u = SV + (size_t)npw * (nl + 1);
      double2 *sw = u + npw;
      apply_S(s, v0, npw, sw, npw, 1, st);
      launch_dot_re(npw, v0, sw, scal + 4, st);
      launch_sqrt_scalar(scal + 4, scal + 3, st);
      launch_scale_inv(npw, scal + 3, v0, V, st);
      launch_scale_inv(npw, scal + 3, sw, SV, st);
      for (int j = 0; j < nl; ++j) {
        double2 *vj = V + (size_t)j * npw;
        apply_core(s, vj, npw, nullptr, 0, u, npw, 1, 1.0, 0.0, 0.0, st);
        apply_Sinv(s, u, npw, w, npw, 1, st);
        if (j > 0) launch_axpy_dev(npw, beta + (j - 1), -1.0, V + (size_t)(j - 1) * npw, w, st);
        launch_dot_re(npw, SV + (size_t)j * npw, w, alpha + j, st);
        launch_axpy_dev(npw, alpha + j, -1.0, vj, w, st);
        launch_multi_dot(npw, j + 1, SV, npw, w, h, st);
        launch_multi_axpy(npw, j + 1, V, npw, h, w, st);
        apply_S(s, w, npw, sw, npw, 1, st);
        launch_dot_re(npw, w, sw, scal + 4, st);
        launch_sqrt_scalar(scal + 4, beta + j, st);
        double ab[2];
        CHEBFI_HIP(hipMemcpyAsync(&ab[0], alpha + j, sizeof(double), hipMemcpyDeviceToHost, st));
        CHEBFI_HIP(hipMemcpyAsync(&ab[1], beta + j, sizeof(double), hipMemcpyDeviceToHost, st));
        CHEBFI_HIP(hipStreamSynchronize(st));
        if (ab[1] <= 1e-12 * std::max(1.0, std::fabs(ab[0]))) {
          k = j + 1;
          add_last = 0;
          break;
        }
        launch_scale_inv(npw, beta + j, w, V + (size_t)(j + 1) * npw, st);
        launch_scale_inv(npw, beta + j, sw, SV + (size_t)(j + 1) * npw, st);
      }
    } else {
      launch_norm(npw, v0, scal + 3, st);
      launch_scale_inv(npw, scal + 3, v0, V, st);
      for (int j = 0; j < nl; ++j) {
        apply_core(s, V + (size_t)j * npw, npw, nullptr, 0, w, npw, 1, 1.0, 0.0, 0.0, st);
        if (j > 0) launch_axpy_dev(npw, beta + (j - 1), -1.0, V + (size_t)(j - 1) * npw, w, st);
        launch_dot_re(npw, V + (size_t)j * npw, w, alpha + j, st);
        launch_axpy_dev(npw, alpha + j, -1.0, V + (size_t)j * npw, w, st);
        launch_multi_dot(npw, j + 1, V, npw, w, h, st);
        launch_multi_axpy(npw, j + 1, V, npw, h, w, st);
        launch_norm(npw, w, beta + j, st);
        double ab[2];
        CHEBFI_HIP(hipMemcpyAsync(&ab[0], alpha + j, sizeof(double), hipMemcpyDeviceToHost, st));
        CHEBFI_HIP(hipMemcpyAsync(&ab[1], beta + j, sizeof(double), hipMemcpyDeviceToHost, st));
        CHEBFI_HIP(hipStreamSynchronize(st));
        if (ab[1] <= 1e-12 * std::max(1.0, std::fabs(ab[0]))) {
          k = j + 1;
          add_last = 0;
          break;
        }
        launch_scale_inv(npw, beta + j, w, V + (size_t)(j + 1) * npw, st);
      }
    }
    launch_tridiag_bound(k, alpha, beta, add_last, scal, st);
    double host[3];
    CHEBFI_HIP(hipMemcpyAsync(host, scal, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
    CHEBFI_HIP(hipStreamSynchronize(st));
    out[0] = host[0];
    out[1] = host[1];
    out[2] = host[2];
  });
}

abi_status abi_rayleigh_ritz(abi_system s, void *Y, void *HPsi, int64_t nband, int64_t ld,
                             int32_t dtype, double *eval, double *resnorm, void *coef,
                             int32_t *flags, void *stream) {
  return guarded([&] {
    check_block(s, Y, nband, ld, dtype);
    CHEBFI_REQUIRE(eval != nullptr, ABI_ERR_ARG, "eval is NULL");
    CHEBFI_REQUIRE(HPsi != Y, ABI_ERR_ARG, "HPsi must not alias Y");
    hipStream_t st = S(stream);
    const int64_t npw = s->npw, M = nband;
    const bool want_low = flags && (*flags & ABI_RR_LOWPREC) && dtype == ABI_C64 &&
                          s->mixed_gemm == 0 && !s->has_S && s->precision == ABI_PREC_MIXED;
    int32_t out_flags = 0;
    bool done = false;
    if (want_low) {
      const int passes = rr_lowprec(s, Y, ld, HPsi, ld, M, eval, resnorm, coef, st);
      done = passes > 0;
      out_flags = !done ? ABI_RR_FELL_BACK
                        : passes == 2 ? (ABI_RR_LOWPREC | ABI_RR_TWO_PASS) : ABI_RR_LOWPREC;
    }
    if (done) {
    } else if (dtype == ABI_C128) {
      rr_core(s, (double2 *)Y, ld, (double2 *)HPsi, ld, M, eval, resnorm, coef, st);
    } else {
      // promote the complex64 block, run the FP64 Rayleigh-Ritz, round back
      double2 *Y2 = (double2 *)s->blk4.get(sizeof(double2) * (size_t)npw * M);
      double2 *H2 = (double2 *)s->blk3.get(sizeof(double2) * (size_t)npw * M);
      launch_c64_to_c128(npw, M, Y, ld, Y2, npw, st);
      rr_core(s, Y2, npw, H2, npw, M, eval, resnorm, coef, st);
      launch_c128_to_c64(npw, M, Y2, npw, Y, ld, st);
      if (HPsi) launch_c128_to_c64(npw, M, H2, npw, HPsi, ld, st);
      CHEBFI_HIP(hipStreamSynchronize(st));
    }
    if (flags) *flags = out_flags;
  });
}

abi_status abi_chebfi_solve(abi_system s, void *X, int64_t nband, int64_t ld, int32_t dtype,
                            const void *v0, int32_t degree, int32_t max_cycles, int32_t nconv,
                            double tol, int32_t refine_degree, double *eval, double *resnorm,
                            int32_t *info, void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(v0 != nullptr && eval != nullptr, ABI_ERR_ARG, "v0 or eval is NULL");
    CHEBFI_REQUIRE(degree >= 1 && max_cycles >= 1, ABI_ERR_ARG,
                   "degree and max_cycles must be >= 1");
    CHEBFI_REQUIRE(nconv >= 1 && nconv <= nband, ABI_ERR_ARG, "need 1 <= nconv <= nband");
    CHEBFI_REQUIRE(tol > 0.0 && std::isfinite(tol), ABI_ERR_ARG, "tol must be positive");
    CHEBFI_REQUIRE(refine_degree >= 0, ABI_ERR_ARG, "refine_degree must be >= 0");
    CHEBFI_REQUIRE(refine_degree == 0 || dtype == ABI_C64, ABI_ERR_ARG,
                   "the FP64 refinement applies to complex64 blocks");
    auto call = [](abi_status rc) {
      if (rc != ABI_OK) throw Error{rc, g_last_error};
    };
    hipStream_t st = S(stream);
    const int64_t npw = s->npw;
    std::vector<double> res((size_t)nband, 0.0);
    auto worst = [&]() {
      double m = 0.0;
      for (int i = 0; i < nconv; ++i) m = std::max(m, res[i]);
      return m;
    };
    // one cycle: bounds of A, filter A -> B, Rayleigh-Ritz in place on B.  From the
    // second cycle on, A holds Ritz vectors, whose Rayleigh quotients are their Ritz
    // values (the last Rayleigh-Ritz step's eval), and H is fixed, so the first
    // cycle's Lanczos upper bound still holds: the bounds need no H application.
    // The Rayleigh-Ritz step also returns H Psi (HB), which the next cycle's
    // filter takes as its first step (abi_cheb_filter_hx): a cycle then applies H
    // degree times in all, the one of the Rayleigh-Ritz included.
    bool have_ritz = false, have_h = false;
    double b_upper = 0.0;
    auto cycle = [&](void *A, void *Bk, void *HA, void *HB, int64_t l, int32_t dt, int32_t m) {
      double bd[3] = {0.0, 0.0, 0.0};
      bool reuse = false;
      if (have_ritz) {
        bd[0] = *std::max_element(eval, eval + nband);
        bd[2] = *std::min_element(eval, eval + nband);
        bd[1] = b_upper;
        reuse = bd[1] > bd[0];
      }
      if (!reuse) {
        call(abi_spectral_bounds(s, A, nband, l, dt, v0, 10, bd, stream));
        b_upper = bd[1];
      }
      if (have_h)
        call(abi_cheb_filter_hx(s, A, HA, Bk, nband, l, dt, m, bd[0], bd[1], bd[2], stream));
      else
        call(abi_cheb_filter(s, A, Bk, nband, l, dt, m, bd[0], bd[1], bd[2], stream));
      // the mixed cycles ahead of an FP64 refinement use the split-BF16
      // Rayleigh-Ritz (the refinement's FP64 cycles win the accuracy back)
      int32_t flags = (dt == ABI_C64 && refine_degree > 0) ? ABI_RR_LOWPREC : 0;
      call(abi_rayleigh_ritz(s, Bk, HB, nband, l, dt, eval, res.data(), nullptr, &flags,
                             stream));
      have_ritz = true;
      have_h = HB != nullptr;
      return (flags & ABI_RR_LOWPREC) != 0;
    };
    const bool refine = refine_degree > 0;
    // the mixed cycles hand over to the FP64 refinement when they stall (a cycle
    // that improves the worst residual by less than 10%) or after half the budget
    const int first_budget = refine ? std::max(1, max_cycles / 2) : max_cycles;
    void *bufA = X;
    void *bufB = s->solve1.get(elem_bytes(dtype) * (size_t)ld * nband);
    // (with S != I the filter has no H X form: H Psi is not kept)
    void *hA = s->has_S ? nullptr : s->solve4.get(elem_bytes(dtype) * (size_t)ld * nband);
    void *hB = s->has_S ? nullptr : s->solve5.get(elem_bytes(dtype) * (size_t)ld * nband);
    int cycles = 0, rcycles = 0, converged = 0;
    double prev = HUGE_VAL;
    while (cycles < first_budget) {
      const bool low = cycle(bufA, bufB, hA, hB, ld, dtype, degree);
      std::swap(bufA, bufB);
      std::swap(hA, hB);
      ++cycles;
      const double cur = worst();
      if (cur <= tol) {
        // residuals of the split-BF16 Rayleigh-Ritz are not final: refine
        converged = low ? 0 : 1;
        break;
      }
      if (refine && cur > 0.9 * prev) break;
      prev = cur;
    }
    if (bufA != X) launch_copy_block(npw, nband, bufA, ld, X, ld, st, dtype == ABI_C64);
    if (refine && !converged) {
      void *A = s->solve2.get(sizeof(double2) * (size_t)npw * nband);
      void *Bk = s->solve3.get(sizeof(double2) * (size_t)npw * nband);
      launch_c64_to_c128(npw, nband, X, ld, A, npw, st);
      // H Psi of the last mixed cycle is complex64: the first FP64 cycle applies H
      have_h = false;
      void *rA = s->has_S ? nullptr : s->solve4.get(sizeof(double2) * (size_t)npw * nband);
      void *rB = s->has_S ? nullptr : s->solve5.get(sizeof(double2) * (size_t)npw * nband);
      while (cycles + rcycles < max_cycles) {
        cycle(A, Bk, rA, rB, npw, ABI_C128, refine_degree);
        std::swap(A, Bk);
        std::swap(rA, rB);
        ++rcycles;
        if (worst() <= tol) {
          converged = 1;
          break;
        }
      }
      launch_c128_to_c64(npw, nband, A, npw, X, ld, st);
    }
    CHEBFI_HIP(hipStreamSynchronize(st));
    if (resnorm) std::memcpy(resnorm, res.data(), sizeof(double) * (size_t)nband);
    if (info) {
      info[0] = cycles;
      info[1] = rcycles;
      info[2] = converged;
      info[3] = 0;
    }
  });
}

abi_status abi_apply_S(abi_system s, const void *X, void *SX, int64_t nband, int64_t ld,
                       int32_t dtype, void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(SX != nullptr && SX != X, ABI_ERR_ARG, "SX must be a separate block");
    apply_S(s, X, ld, SX, ld, nband, S(stream), dtype);
  });
}

abi_status abi_apply_Sinv(abi_system s, const void *X, void *Y, int64_t nband, int64_t ld,
                          int32_t dtype, void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(Y != nullptr && Y != X, ABI_ERR_ARG, "Y must be a separate block");
    apply_Sinv(s, X, ld, Y, ld, nband, S(stream), dtype);
  });
}

abi_status abi_overlap_info(abi_system s, int32_t *has_overlap, double *s_min) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr, ABI_ERR_ARG, "system handle is NULL");
    if (has_overlap) *has_overlap = s->has_S ? 1 : 0;
    if (s_min) *s_min = s->s_min;
  });
}

abi_status abi_lobpcg_solve(abi_system s, void *X, int64_t nband, int64_t ld, int32_t dtype,
                            int32_t nblocks, int32_t nline, int32_t max_passes, int32_t nconv,
                            double tol, double *eval, double *resnorm, int32_t *info,
                            void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(dtype == ABI_C128, ABI_ERR_ARG, "LOBPCG runs on complex128 blocks");
    CHEBFI_REQUIRE(eval != nullptr, ABI_ERR_ARG, "eval is NULL");
    CHEBFI_REQUIRE(nblocks >= 1 && nband % nblocks == 0, ABI_ERR_ARG,
                   "nblocks must divide nband");
    CHEBFI_REQUIRE(nline >= 1 && max_passes >= 1, ABI_ERR_ARG,
                   "nline and max_passes must be >= 1");
    CHEBFI_REQUIRE(nconv >= 1 && nconv <= nband, ABI_ERR_ARG, "need 1 <= nconv <= nband");
    CHEBFI_REQUIRE(tol >= 0.0 && std::isfinite(tol), ABI_ERR_ARG, "tol must be >= 0");
    hipStream_t st = S(stream);
    std::vector<double> res((size_t)nband, 0.0);
    std::vector<int> steps((size_t)nblocks, 0);
    int passes = 0, total = 0, converged = 0;
    while (passes < max_passes) {
      lobpcg_pass_core(s, (double2 *)X, ld, nband, nblocks, nline, tol, eval, res.data(),
                       steps.data(), st);
      ++passes;
      for (int v : steps) total += v;
      double worst = 0.0;
      for (int i = 0; i < nconv; ++i) worst = std::max(worst, res[i]);
      if (worst <= tol) {
        converged = 1;
        break;
      }
    }
    if (resnorm) std::memcpy(resnorm, res.data(), sizeof(double) * (size_t)nband);
    if (info) {
      info[0] = passes;
      info[1] = total;
      info[2] = converged;
      info[3] = 0;
    }
  });
}

abi_status abi_get_potential(abi_system s, double *vloc, void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr && vloc != nullptr, ABI_ERR_ARG, "NULL argument");
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    CHEBFI_HIP(hipMemcpyAsync(vloc, s->d_V, sizeof(double) * nbox, hipMemcpyDeviceToDevice,
                              S(stream)));
  });
}

abi_status abi_update_potential(abi_system s, const double *vloc, const void *dij, void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr, ABI_ERR_ARG, "system handle is NULL");
    hipStream_t st = S(stream);
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    if (vloc) {
      CHEBFI_HIP(hipMemcpyAsync(s->d_V, vloc, sizeof(double) * nbox, hipMemcpyDeviceToDevice, st));
      if (s->d_Vf) launch_d2f(nbox, s->d_V, s->d_Vf, st);
    }
    if (dij && s->natom > 0)
      CHEBFI_HIP(hipMemcpyAsync(s->d_D, dij, sizeof(double2) * 16 * (size_t)s->natom,
                                hipMemcpyDeviceToDevice, st));
  });
}

abi_status abi_filter_backward(abi_system s, const void *X, const void *W, int64_t nband,
                               int64_t ld, int32_t dtype, int32_t degree, double a, double b,
                               double a0, int32_t ckpt_every, double *dV, void *dD, void *dX,
                               void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(s == nullptr || !s->has_S, ABI_ERR_STATE,
                   "the filter adjoint is provided for S = I only");
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(W != nullptr, ABI_ERR_ARG, "W is NULL");
    CHEBFI_REQUIRE(dV != nullptr, ABI_ERR_ARG, "dV is NULL");
    CHEBFI_REQUIRE(dD != nullptr || s->natom == 0, ABI_ERR_ARG, "dD is NULL");
    CHEBFI_REQUIRE(degree >= 1, ABI_ERR_ARG, "degree must be >= 1");
    CHEBFI_REQUIRE(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0), ABI_ERR_ARG,
                   "bounds must be finite");
    CHEBFI_REQUIRE(b > a, ABI_ERR_ARG, "need b > a");
    CHEBFI_REQUIRE(a0 <= a, ABI_ERR_ARG, "need a0 <= a");
    CHEBFI_REQUIRE(ckpt_every >= 0, ABI_ERR_ARG, "ckpt_every must be >= 0");
    hipStream_t st = S(stream);
    const bool fp32 = (dtype == ABI_C64);
    const int64_t npw = s->npw;
    const int nproj = s->nproj, natom = s->natom;
    const int m = degree;
    // recurrence coefficients
    const double e = (b - a) / 2.0, c = (b + a) / 2.0, s1 = e / (a0 - c);
    std::vector<double> gam(m), del(m, 0.0);
    {
      double sk = s1;
      gam[0] = s1 / e;
      for (int k = 1; k < m; ++k) {
        const double sk1 = 1.0 / (2.0 / s1 - sk);
        gam[k] = 2.0 * sk1 / e;
        del[k] = sk * sk1;
        sk = sk1;
      }
    }
    const int cseg = (ckpt_every > 0) ? std::min(ckpt_every, m) : m;
    std::vector<int> starts;  // segment starts 0, cseg, 2 cseg, ... < m
    for (int s0 = 0; s0 < m; s0 += cseg) starts.push_back(s0);
    const int nck = (int)starts.size() - 1;  // checkpoint pairs (Y_{s-1}, Y_s), s > 0
    const size_t esz = elem_bytes(dtype);
    const size_t blk = esz * (size_t)npw * nband;
    // blocks: the checkpoint pairs, the recomputed iterates Y_{s0+1} ..
    // Y_{s0+cseg-1} of a segment (Y_{s0} is its checkpoint or X) and three
    // adjoint iterates
    const int nblocks = 2 * nck + (cseg - 1) + 3;
    char *base = (char *)s->adj.get(blk * (size_t)nblocks);
    auto block = [&](int i) { return (void *)(base + blk * (size_t)i); };
    auto ck_prev = [&](int j) { return block(2 * (j - 1)); };  // Y_{s_j - 1}
    auto ck_cur = [&](int j) { return block(2 * (j - 1) + 1); };  // Y_{s_j}
    auto seg = [&](int i) { return block(2 * nck + i - 1); };  // Y_{s0 + i}, i >= 1
    const int ab = 2 * nck + cseg - 1;
    void *abuf[3] = {block(ab), block(ab + 1), block(ab + 2)};
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    // small accumulators: dV (nbox), dD (natom*16 complex), CA, CY (nproj*nband), C'
    const size_t small_bytes = sizeof(double) * (size_t)nbox + sizeof(double2) * 16 * (size_t)natom +
                               3 * sizeof(double2) * (size_t)std::max(nproj, 1) * nband + 1024;
    char *sb = (char *)s->adjsmall.get(small_bytes);
    double *dV_acc = (double *)sb;
    double2 *dD_acc = (double2 *)(sb + ((sizeof(double) * nbox + 255) / 256 * 256));
    double2 *CA = dD_acc + 16 * (size_t)natom;
    double2 *CY = CA + (size_t)std::max(nproj, 1) * nband;
    double2 *Cp = CY + (size_t)std::max(nproj, 1) * nband;
    launch_fill_zero(nbox, dV_acc, st);
    launch_fill_zero(32 * (int64_t)natom, (double *)dD_acc, st);

    // raw projections P^H Y_k kept from the steps that apply H to Y_k (the reverse step
    // needs them for dD); kept only where the step projects with the same kernel and
    // split count as the reverse step (not the one-band FP64 step, not the FP32-MFMA
    // tuning forms), so the gradients do not change
    const bool keep_c = nproj > 0 && (fp32 ? s->mixed_gemm == 0 : nband > 1);
    char *cst = keep_c ? (char *)s->adjc.get(esz * (size_t)nproj * nband * m) : nullptr;
    auto cslot = [&](int k) { return (void *)(cst + esz * (size_t)nproj * nband * k); };
    std::vector<char> have_c(m, 0);
    auto step_fwd = [&](int j, const void *ym1, int64_t ld1, const void *ym2, int64_t ld2,
                        void *dst) {  // Y_j from Y_{j-1} (and Y_{j-2})
      void *craw = keep_c ? cslot(j - 1) : nullptr;
      if (j == 1)
        apply_core(s, ym1, ld1, nullptr, 0, dst, npw, nband, gam[0], c, 0.0, st, dtype, craw);
      else
        apply_core(s, ym1, ld1, ym2, ld2, dst, npw, nband, gam[j - 1], c, del[j - 1], st, dtype,
                   craw);
      if (keep_c) have_c[j - 1] = 1;
    };
    // raw projections out = P^H Z (nproj x nband, contiguous), in the block's precision
    const bool planes = fp32 && s->mixed_gemm == 0;
    auto project = [&](const void *Z, int64_t ldz, void *out) {
      if (planes) {
        const int splits = mixed_proj_splits(s, nband);
        void *part = s->cpart.get(sizeof(float2) * (size_t)splits * nproj * nband);
        mixed_project(s, Z, ldz, nband, part, splits, st);
        launch_sum_parts(nproj, nband, part, splits, out, st, true);
      } else {
        const int splits = zgemm_splits(nproj, nband, npw);
        void *part = s->cpart.get(esz * (size_t)splits * nproj * nband);
        proj_gemm(nproj, nband, npw, fp32 ? (const void *)s->d_Pf : (const void *)s->d_P, Z, ldz,
                  part, splits, st, fp32);
        launch_sum_parts(nproj, nband, part, splits, out, st, fp32);
      }
    };
    // forward sweep: keep the checkpoint pairs
    {
      const int jmax = nck > 0 ? starts.back() : 0;
      const void *p1 = X;  // Y_{j-1}
      int64_t l1 = ld;
      const void *p2 = nullptr;  // Y_{j-2}
      int64_t l2 = npw;
      for (int j = 1; j <= jmax; ++j) {
        // slots that must receive Y_j (two when checkpoints are one step apart)
        std::vector<void *> slots;
        for (int q = 1; q <= nck; ++q) {
          if (j == starts[q] - 1) slots.push_back(ck_prev(q));
          if (j == starts[q]) slots.push_back(ck_cur(q));
        }
        void *dst = slots.empty() ? abuf[j % 3] : slots[0];
        step_fwd(j, p1, l1, p2, l2, dst);
        for (size_t t = 1; t < slots.size(); ++t)
          launch_copy_block(npw, nband, dst, npw, slots[t], npw, st, fp32);
        p2 = p1;
        l2 = l1;
        p1 = dst;
        l1 = npw;
      }
    }
    // reverse sweep, one segment at a time
    const int fb = (int)std::min<int64_t>(s->fft_batch * (fp32 ? 2 : 1), nband);
    void *box1 = s->box.get(esz * (size_t)nbox * fb);
    void *box2 = s->box2.get(esz * (size_t)nbox * fb);
    for (int q = (int)starts.size() - 1; q >= 0; --q) {
      const int s0 = starts[q];
      const int s1e = std::min(s0 + cseg, m);  // iterates Y_{s0} .. Y_{s1e-1}
      const void *ys = (q == 0) ? X : (const void *)ck_cur(q);
      const int64_t lys = (q == 0) ? ld : npw;
      const void *ysm1 = (q == 0) ? nullptr : (const void *)ck_prev(q);
      auto yk = [&](int k, int64_t *ldk) -> const void * {
        if (k == s0) {
          *ldk = lys;
          return ys;
        }
        *ldk = npw;
        return seg(k - s0);
      };
      for (int j = s0 + 1; j < s1e; ++j) {
        int64_t l1, l2 = npw;
        const void *p1 = yk(j - 1, &l1);
        const void *p2 = nullptr;
        if (j - 2 >= s0)
          p2 = yk(j - 2, &l2);
        else if (j >= 2)
          p2 = ysm1;
        step_fwd(j, p1, l1, p2, l2, seg(j - s0));
      }
      for (int k = s1e - 1; k >= s0; --k) {
        int64_t ldy;
        const void *Yk = yk(k, &ldy);
        const void *Ak1 = (k + 1 == m) ? W : (const void *)abuf[(k + 1) % 3];
        const int64_t lda1 = (k + 1 == m) ? ld : npw;
        void *Ak = abuf[k % 3];
        const bool acc = (k + 1 < m);
        // the adjoint local part runs beside the projections, as in the forward step
        const bool side = s->overlap && nproj > 0 && s->aux;
        hipStream_t fst = side ? s->aux : st;
        if (side) {
          CHEBFI_HIP(hipEventRecord(s->ev_fork, st));
          CHEBFI_HIP(hipStreamWaitEvent(s->aux, s->ev_fork, 0));
        }
        for (int64_t b0 = 0; b0 < nband; b0 += fb) {
          const int nb = (int)std::min<int64_t>(fb, nband - b0);
          if (fp32)
            launch_adjoint_local<float>(s, Ak1, lda1, Yk, ldy, Ak, npw, acc, (int)b0, nb, box1,
                                        box2, s->d_Vf, gam[k], c, dV_acc, fst);
          else
            launch_adjoint_local<double>(s, Ak1, lda1, Yk, ldy, Ak, npw, acc, (int)b0, nb, box1,
                                         box2, s->d_V, gam[k], c, dV_acc, fst);
        }
        if (side) CHEBFI_HIP(hipEventRecord(s->ev_join, s->aux));
        if (nproj > 0) {
          project(Ak1, lda1, CA);
          const void *cy = CY;
          if (have_c[k])
            cy = cslot(k);
          else
            project(Yk, ldy, CY);
          launch_dd_accum(natom, nband, CA, cy, gam[k], dD_acc, st, fp32);
          launch_dapply(natom, nband, CA, 1, s->d_D, gam[k], Cp, st, fp32);
        }
        if (side) CHEBFI_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
        if (nproj > 0) {
          if (planes)
            mixed_expand(s, Cp, Ak, npw, nband, st, true);
          else
            expand_gemm(npw, nband, nproj, fp32 ? (const void *)s->d_Pf : (const void *)s->d_P,
                        Cp, Ak, npw, st, fp32);
        }
        if (k >= 1)
          launch_scale_neg(npw, nband, Ak1, lda1, del[k], abuf[(k + 2) % 3], npw, st, fp32);
      }
    }
    CHEBFI_HIP(hipMemcpyAsync(dV, dV_acc, sizeof(double) * nbox, hipMemcpyDeviceToDevice, st));
    if (natom > 0)
      CHEBFI_HIP(hipMemcpyAsync(dD, dD_acc, sizeof(double2) * 16 * (size_t)natom,
                                hipMemcpyDeviceToDevice, st));
    if (dX) launch_copy_block(npw, nband, abuf[0], npw, dX, ld, st, fp32);
  });
}

abi_status abi_density(abi_system s, const void *Psi, int64_t nband, int64_t ld, int32_t dtype,
                       const double *weights, double *rho, void *stream) {
  return guarded([&] {
    check_block(s, Psi, nband, ld, dtype);
    CHEBFI_REQUIRE(rho != nullptr, ABI_ERR_ARG, "rho is NULL");
    hipStream_t st = S(stream);
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    launch_fill_zero(nbox, rho, st);
    const size_t es = elem_bytes(dtype);
    const int fb = (int)std::min<int64_t>(s->fft_batch * (dtype == ABI_C64 ? 2 : 1), nband);
    void *box = s->box.get(es * (size_t)nbox * fb);
    for (int64_t b0 = 0; b0 < nband; b0 += fb) {
      const int nb = (int)std::min<int64_t>(fb, nband - b0);
      if (dtype == ABI_C64)
        launch_density<float>(s, Psi, ld, (int)b0, nb, box, weights, rho, st);
      else
        launch_density<double>(s, Psi, ld, (int)b0, nb, box, weights, rho, st);
    }
  });
}

abi_status abi_density_add(abi_system s, const void *Psi, int64_t nband, int64_t ld,
                           int32_t dtype, const double *weights, double *rho, void *stream) {
  return guarded([&] {
    check_block(s, Psi, nband, ld, dtype);
    CHEBFI_REQUIRE(rho != nullptr, ABI_ERR_ARG, "rho is NULL");
    hipStream_t st = S(stream);
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    const size_t es = elem_bytes(dtype);
    const int fb = (int)std::min<int64_t>(s->fft_batch * (dtype == ABI_C64 ? 2 : 1), nband);
    void *box = s->box.get(es * (size_t)nbox * fb);
    for (int64_t b0 = 0; b0 < nband; b0 += fb) {
      const int nb = (int)std::min<int64_t>(fb, nband - b0);
      if (dtype == ABI_C64)
        launch_density<float>(s, Psi, ld, (int)b0, nb, box, weights, rho, st);
      else
        launch_density<double>(s, Psi, ld, (int)b0, nb, box, weights, rho, st);
    }
  });
}

abi_status abi_occupations(int64_t n, const double *eval, double nelec, double kT, double occ_max,
                           double *f, double *mu) {
  return guarded([&] {
    CHEBFI_REQUIRE(n >= 1 && eval != nullptr && f != nullptr, ABI_ERR_ARG, "NULL argument");
    CHEBFI_REQUIRE(kT > 0.0 && occ_max > 0.0, ABI_ERR_ARG, "kT and occ_max must be > 0");
    CHEBFI_REQUIRE(nelec >= 0.0 && nelec <= occ_max * (double)n, ABI_ERR_ARG,
                   "nelec must be in [0, occ_max n]");
    double emin = eval[0], emax = eval[0];
    for (int64_t i = 0; i < n; ++i) {
      CHEBFI_REQUIRE(std::isfinite(eval[i]), ABI_ERR_ARG, "eigenvalues must be finite");
      emin = std::min(emin, eval[i]);
      emax = std::max(emax, eval[i]);
    }
    auto occ = [&](double e, double m) {
      const double x = std::max(-700.0, std::min(700.0, (e - m) / kT));
      return occ_max / (1.0 + std::exp(x));
    };
    auto total = [&](double m) {
      double t = 0.0;
      for (int64_t i = 0; i < n; ++i) t += occ(eval[i], m);
      return t;
    };
    double lo = emin - 50.0 * kT - 1.0, hi = emax + 50.0 * kT + 1.0;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (total(mid) < nelec)
        lo = mid;
      else
        hi = mid;
    }
    const double m = 0.5 * (lo + hi);
    for (int64_t i = 0; i < n; ++i) f[i] = occ(eval[i], m);
    if (mu) *mu = m;
  });
}

abi_status abi_scf_potential(abi_system s, const double *rho, const double *vion, double *vout,
                             void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr && rho && vion && vout, ABI_ERR_ARG, "NULL argument");
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    void *box = s->scf_box.get(sizeof(double2) * (size_t)nbox);
    launch_scf_potential(s, rho, vion, vout, box, S(stream));
  });
}

abi_status abi_scf_solve(abi_system s, void *X, int64_t nband, int64_t ld, int32_t dtype,
                         const void *v0, const double *vion, double nelec, double kT,
                         double alpha, double q0, int32_t degree, int32_t cycles_per_iter,
                         int32_t max_iter, double tol, double *eval, double *rho_out,
                         double *dv_out, int32_t *info, void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    CHEBFI_REQUIRE(v0 && vion && eval, ABI_ERR_ARG, "v0, vion or eval is NULL");
    CHEBFI_REQUIRE(alpha > 0.0 && alpha <= 1.0, ABI_ERR_ARG, "alpha must be in (0, 1]");
    CHEBFI_REQUIRE(q0 >= 0.0 && std::isfinite(q0), ABI_ERR_ARG, "q0 must be >= 0");
    CHEBFI_REQUIRE(degree >= 1 && cycles_per_iter >= 1 && max_iter >= 1, ABI_ERR_ARG,
                   "degree, cycles_per_iter and max_iter must be >= 1");
    CHEBFI_REQUIRE(tol > 0.0 && std::isfinite(tol), ABI_ERR_ARG, "tol must be positive");
    auto call = [](abi_status rc) {
      if (rc != ABI_OK) throw Error{rc, g_last_error};
    };
    hipStream_t st = S(stream);
    const int64_t nbox = (int64_t)s->n1 * s->n2 * s->n3;
    double *rho = (double *)s->scf_rho.get(sizeof(double) * (size_t)nbox);
    double *vbuf = (double *)s->scf_v.get(sizeof(double) * (size_t)(2 * nbox + 8));
    double *vout = vbuf, *vnext = vbuf + nbox, *dv_dev = vbuf + 2 * nbox;
    double *w_dev = (double *)s->scf_w.get(sizeof(double) * (size_t)nband);
    std::vector<double> f((size_t)nband);
    int iters = 0, converged = 0;
    double dv = HUGE_VAL;
    while (iters < max_iter) {
      // solve at the current potential: cycles_per_iter cycles of bounds, filter, RR
      call(abi_chebfi_solve(s, X, nband, ld, dtype, v0, degree, cycles_per_iter, (int32_t)nband,
                            1e-300, 0, eval, nullptr, nullptr, stream));
      call(abi_occupations(nband, eval, nelec, kT, 2.0, f.data(), nullptr));
      CHEBFI_HIP(hipMemcpyAsync(w_dev, f.data(), sizeof(double) * (size_t)nband,
                                hipMemcpyHostToDevice, st));
      call(abi_density(s, X, nband, ld, dtype, w_dev, rho, stream));
      call(abi_scf_potential(s, rho, vion, vout, stream));
      launch_mix(s, s->d_V, vout, alpha, q0, vnext, dv_dev,
                 s->scf_box.get(sizeof(double2) * (size_t)nbox), st);
      CHEBFI_HIP(hipMemcpyAsync(&dv, dv_dev, sizeof(double), hipMemcpyDeviceToHost, st));
      CHEBFI_HIP(hipStreamSynchronize(st));
      ++iters;
      if (dv <= tol) {
        converged = 1;
        break;
      }
      call(abi_update_potential(s, vnext, nullptr, stream));
    }
    if (rho_out)
      CHEBFI_HIP(hipMemcpyAsync(rho_out, rho, sizeof(double) * (size_t)nbox,
                                hipMemcpyDeviceToDevice, st));
    CHEBFI_HIP(hipStreamSynchronize(st));
    if (dv_out) *dv_out = dv;
    if (info) {
      info[0] = iters;
      info[1] = converged;
      info[2] = 0;
      info[3] = 0;
    }
  });
}

abi_status abi_set_tuning(abi_system s, int32_t param, int32_t value) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr, ABI_ERR_ARG, "system handle is NULL");
    const bool mixed = s->precision == ABI_PREC_MIXED;
    switch (param) {
      case ABI_TUNE_PROJ:
        CHEBFI_REQUIRE(mixed, ABI_ERR_STATE, "split-BF16 variants need a mixed handle");
        CHEBFI_REQUIRE(value >= 0 && value <= 16, ABI_ERR_ARG, "projection variant out of range");
        s->pl_proj = value;
        break;
      case ABI_TUNE_EXPAND:
        CHEBFI_REQUIRE(mixed, ABI_ERR_STATE, "split-BF16 variants need a mixed handle");
        CHEBFI_REQUIRE(value >= 0 && value <= 15, ABI_ERR_ARG, "expansion variant out of range");
        s->pl_expand = value;
        break;
      case ABI_TUNE_FFT_BATCH:
        CHEBFI_REQUIRE(value >= 1 && value <= 4096, ABI_ERR_ARG, "FFT batch out of range");
        s->fft_batch = value;
        break;
      case ABI_TUNE_OVERLAP:
        CHEBFI_REQUIRE(value == 0 || value == 1, ABI_ERR_ARG, "overlap is 0 or 1");
        s->overlap = value;
        break;
      case ABI_TUNE_GENERIC_FFT:
        CHEBFI_REQUIRE(value == 0 || value == 1, ABI_ERR_ARG, "generic FFT is 0 or 1");
        s->generic_fft = value;
        break;
      case ABI_TUNE_MIXED_GEMM:
        CHEBFI_REQUIRE(mixed, ABI_ERR_STATE, "projector product forms need a mixed handle");
        CHEBFI_REQUIRE(value >= 0 && value <= 2, ABI_ERR_ARG, "projector product form is 0..2");
        s->mixed_gemm = value;
        break;
      case ABI_TUNE_FILTER_GRAPH:
        CHEBFI_REQUIRE(value == 0 || value == 1, ABI_ERR_ARG, "filter graph is 0 or 1");
        s->filter_graph = value;
        if (!value) free_filter_graph(s);
        break;
      default:
        CHEBFI_REQUIRE(false, ABI_ERR_ARG, "unknown tuning parameter");
    }
  });
}

abi_status abi_get_tuning(abi_system s, int32_t param, int32_t *value) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr && value != nullptr, ABI_ERR_ARG, "NULL argument");
    switch (param) {
      case ABI_TUNE_PROJ: *value = s->pl_proj; break;
      case ABI_TUNE_EXPAND: *value = s->pl_expand; break;
      case ABI_TUNE_FFT_BATCH: *value = s->fft_batch; break;
      case ABI_TUNE_OVERLAP: *value = s->overlap; break;
      case ABI_TUNE_GENERIC_FFT: *value = s->generic_fft; break;
      case ABI_TUNE_MIXED_GEMM: *value = s->mixed_gemm; break;
      case ABI_TUNE_FILTER_GRAPH: *value = s->filter_graph; break;
      default: CHEBFI_REQUIRE(false, ABI_ERR_ARG, "unknown tuning parameter");
    }
  });
}

// ---- autotuner --------------------------------------------------------------
}  // extern "C": the cache helpers below return C++ types

namespace {

struct TuneChoice {
  int proj = 0, expand = 0, fft_batch = 1, overlap = 0;
  double ms = 0.0;  // one H application with this choice
};

std::string tune_key(const abi_system_s *s, int64_t nband, int32_t dtype) {
  hipDeviceProp_t prop;
  CHEBFI_HIP(hipGetDeviceProperties(&prop, s->device));
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  std::ostringstream k;
  k << arch << " cus=" << prop.multiProcessorCount << " npw=" << s->npw << " nproj=" << s->nproj
    << " nband=" << nband << " box=" << s->n1 << "x" << s->n2 << "x" << s->n3
    << (dtype == ABI_C64 ? " c64" : " c128");
  return k.str();
}

// The cache is a JSON object written by this library, one entry per line:
//   "<key>": {"proj": P, "expand": E, "fft_batch": F, "overlap": O, "ms_per_apply": T}
std::map<std::string, std::string> cache_read(const std::string &path) {
  std::map<std::string, std::string> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    const size_t b = a == std::string::npos ? a : line.find("\": {", a + 1);
    if (a == std::string::npos || b == std::string::npos) continue;
    std::string body = line.substr(b + 3);
    while (!body.empty() && (body.back() == ',' || body.back() == ' ')) body.pop_back();
    out[line.substr(a + 1, b - a - 1)] = body;
  }
  return out;
}

bool cache_parse(const std::string &body, TuneChoice *c) {
  return std::sscanf(body.c_str(),
                     "{\"proj\": %d, \"expand\": %d, \"fft_batch\": %d, \"overlap\": %d, "
                     "\"ms_per_apply\": %lf}",
                     &c->proj, &c->expand, &c->fft_batch, &c->overlap, &c->ms) == 5;
}

void cache_write(const std::string &path, const std::string &key, const TuneChoice &c) {
  auto all = cache_read(path);
  char body[256];
  std::snprintf(body, sizeof body,
                "{\"proj\": %d, \"expand\": %d, \"fft_batch\": %d, \"overlap\": %d, "
                "\"ms_per_apply\": %.4f}",
                c.proj, c.expand, c.fft_batch, c.overlap, c.ms);
  all[key] = body;
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    CHEBFI_REQUIRE(f.good(), ABI_ERR_ARG, "cannot write the autotune cache " + tmp);
    f << "{\n";
    size_t i = 0;
    for (const auto &kv : all)
      f << " \"" << kv.first << "\": " << kv.second << (++i < all.size() ? ",\n" : "\n");
    f << "}\n";
  }
  CHEBFI_REQUIRE(std::rename(tmp.c_str(), path.c_str()) == 0, ABI_ERR_ARG,
                 "cannot replace the autotune cache " + path);
}

}  // namespace

extern "C" {

abi_status abi_autotune(abi_system s, const void *X, int64_t nband, int64_t ld, int32_t dtype,
                        const char *cache_path, int32_t *from_cache, void *stream) {
  return guarded([&] {
    check_block(s, X, nband, ld, dtype);
    hipStream_t st = S(stream);
    if (from_cache) *from_cache = 0;
    std::string path = cache_path ? cache_path : "";
    if (path.empty())
      if (const char *e = std::getenv("ABI_AUTOTUNE_CACHE")) path = e;
    const std::string key = tune_key(s, nband, dtype);
    const bool split_bf16 = dtype == ABI_C64 && s->mixed_gemm == 0 && s->nproj > 0;
    auto apply = [&](const TuneChoice &c) {
      if (split_bf16) {
        s->pl_proj = c.proj;
        s->pl_expand = c.expand;
      }
      s->fft_batch = c.fft_batch;
      s->overlap = c.overlap;
    };
    if (!path.empty()) {
      const auto all = cache_read(path);
      const auto it = all.find(key);
      TuneChoice c;
      if (it != all.end() && cache_parse(it->second, &c) && c.fft_batch >= 1 &&
          c.fft_batch <= 4096 && (c.overlap == 0 || c.overlap == 1) &&
          (!split_bf16 || (c.proj >= 0 && c.proj <= 16 && c.expand >= 0 && c.expand <= 15))) {
        apply(c);
        if (from_cache) *from_cache = 1;
        return;
      }
    }
    // time one filter step per candidate (best of five after a warm-up): H
    // applied with the recurrence's previous block read as in the filter (X
    // itself stands in for it; the values do not matter here), so that the last
    // FFT pass moves the bytes it moves inside a filter.  One coordinate at a
    // time from the current choice; a candidate replaces the current one only if
    // it is more than 1% faster (the timings of one choice vary by about that
    // much from run to run)
    void *HX = s->tune_out.get(elem_bytes(dtype) * (size_t)s->npw * nband);
    const bool prof = s->prof.on;
    s->prof.on = false;
    hipEvent_t e0, e1;
    CHEBFI_HIP(hipEventCreate(&e0));
    CHEBFI_HIP(hipEventCreate(&e1));
    // a chained-planes projection is timed as inside a filter (planes present)
    struct ChainScope {
      abi_system_s *s;
      ~ChainScope() {
        s->pl_chain = false;
        s->pl_assume = false;
        s->pl_have = nullptr;
      }
    } chain_scope{s};
    auto timed = [&](const TuneChoice &c) {
      apply(c);
      s->pl_chain = s->pl_assume = split_bf16 && c.proj >= 15;
      apply_core(s, X, ld, X, ld, HX, s->npw, nband, 1.0, 0.0, 1.0, st, dtype);
      float best = 1e30f;
      for (int r = 0; r < 5; ++r) {
        CHEBFI_HIP(hipEventRecord(e0, st));
        apply_core(s, X, ld, X, ld, HX, s->npw, nband, 1.0, 0.0, 1.0, st, dtype);
        CHEBFI_HIP(hipEventRecord(e1, st));
        CHEBFI_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        CHEBFI_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
      }
      return (double)best;
    };
    TuneChoice cur;
    cur.proj = s->pl_proj;
    cur.expand = s->pl_expand;
    cur.fft_batch = s->fft_batch;
    cur.overlap = s->overlap;
    try {
      cur.ms = timed(cur);
      auto sweep = [&](int TuneChoice::*field, const std::vector<int> &vals) {
        for (int v : vals) {
          if (v == cur.*field) continue;
          TuneChoice c = cur;
          c.*field = v;
          const double ms = timed(c);
          if (ms < 0.99 * cur.ms) {
            cur = c;
            cur.ms = ms;
          }
        }
      };
      if (split_bf16) {
        sweep(&TuneChoice::proj, {14, 15, 11, 4});
        sweep(&TuneChoice::expand, {15, 13, 9, 6});
      }
      const int fb = cur.fft_batch;
      sweep(&TuneChoice::fft_batch,
            {std::max(1, fb / 2), std::min(4096, 2 * fb)});
      if (s->nproj > 0 && !(nband == 1 && dtype == ABI_C128)) sweep(&TuneChoice::overlap, {0, 1});
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      s->prof.on = prof;
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->prof.on = prof;
    apply(cur);
    if (!path.empty()) cache_write(path, key, cur);
  });
}

abi_status abi_profile_enable(abi_system s, int32_t on) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr, ABI_ERR_ARG, "system handle is NULL");
    s->prof.collect();
    for (int c = 0; c < PROF_NCLASS; ++c) {
      s->prof.total_ms[c] = 0;
      s->prof.work[c] = 0;
      s->prof.count[c] = 0;
    }
    s->prof.on = (on != 0);
  });
}

abi_status abi_profile_read(abi_system s, int32_t nclass, double *total_ms, double *work,
                            int64_t *count) {
  return guarded([&] {
    CHEBFI_REQUIRE(s != nullptr && total_ms && work && count, ABI_ERR_ARG, "NULL argument");
    s->prof.collect();
    for (int c = 0; c < nclass; ++c) {
      const bool ok = c < PROF_NCLASS;
      total_ms[c] = ok ? s->prof.total_ms[c] : 0.0;
      work[c] = ok ? s->prof.work[c] : 0.0;
      count[c] = ok ? s->prof.count[c] : 0;
    }
  });
}

abi_status abi_zpotrf_upper(int64_t m, void *A, int64_t lda, void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(m >= 1 && A != nullptr && lda >= m, ABI_ERR_ARG, "bad matrix arguments");
    hipStream_t st = S(stream);
    int *info = nullptr;
    CHEBFI_HIP(hipMalloc(&info, sizeof(int)));
    zpotrf_upper(m, A, lda, info, nullptr, st);
    int h = 0;
    CHEBFI_HIP(hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, st));
    CHEBFI_HIP(hipStreamSynchronize(st));
    (void)hipFree(info);
    if (h != 0) throw Error{ABI_ERR_NOT_HPD, "not positive definite at pivot " + std::to_string(h)};
  });
}

abi_status abi_zheev(int64_t m, void *A, int64_t lda, double *w, void *Z, int64_t ldz,
                     void *stream) {
  return guarded([&] {
    CHEBFI_REQUIRE(m >= 1 && A && w && Z && lda >= m && ldz >= m, ABI_ERR_ARG,
                   "bad matrix arguments");
    hipStream_t st = S(stream);
    void *work = nullptr;
    CHEBFI_HIP(hipMalloc(&work, zheev_work_bytes(m)));
    try {
      zheev(m, A, lda, w, Z, ldz, work, st);
      CHEBFI_HIP(hipStreamSynchronize(st));
    } catch (...) {
      (void)hipFree(work);
      throw;
    }
    (void)hipFree(work);
  });
}

// ---- batching -----------------------------------------------------------------

abi_status abi_set_system_batch(const abi_system_desc *descs, int32_t nsys, void *stream,
                                abi_batch *out) {
  abi_batch_s *B = nullptr;
  abi_status rc = guarded([&] {
    CHEBFI_REQUIRE(descs != nullptr && out != nullptr, ABI_ERR_ARG, "descs or out is NULL");
    CHEBFI_REQUIRE(nsys >= 1 && nsys <= kBatchMaxSys, ABI_ERR_ARG, "nsys out of range");
    for (int i = 0; i < nsys; ++i) {
      CHEBFI_REQUIRE(descs[i].natom >= 0 && descs[i].natom <= kBatchMaxAtoms, ABI_ERR_ARG,
                     "a batched system has more than 256 atoms");
      CHEBFI_REQUIRE(descs[i].precision == descs[0].precision, ABI_ERR_ARG,
                     "all systems of a batch need the same precision");
      CHEBFI_REQUIRE(descs[i].abi_version < 2 || descs[i].qij == nullptr, ABI_ERR_ARG,
                     "the batched filter takes systems with S = I (no Q)");
    }
    B = new abi_batch_s();
    B->precision = descs[0].precision;
    for (int i = 0; i < nsys; ++i) {
      abi_system h = nullptr;
      const abi_status st = abi_set_system(&descs[i], stream, &h);
      if (st != ABI_OK) throw Error{st, "system " + std::to_string(i) + ": " + g_last_error};
      B->sys.push_back(h);
    }
    B->hsys.resize(nsys);
    CHEBFI_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    CHEBFI_HIP(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    CHEBFI_HIP(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
    CHEBFI_HIP(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
  });
  if (rc != ABI_OK) {
    if (B) {
      for (abi_system h : B->sys) (void)abi_destroy(h);
      if (B->cap) (void)hipStreamDestroy(B->cap);
      if (B->side) (void)hipStreamDestroy(B->side);
      if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
      if (B->ev_join) (void)hipEventDestroy(B->ev_join);
      delete B;
    }
    return rc;
  }
  *out = B;
  return ABI_OK;
}

abi_status abi_batch_system(abi_batch B, int32_t i, abi_system *out) {
  return guarded([&] {
    CHEBFI_REQUIRE(B != nullptr && out != nullptr, ABI_ERR_ARG, "batch or out is NULL");
    CHEBFI_REQUIRE(i >= 0 && i < (int32_t)B->sys.size(), ABI_ERR_ARG, "system index out of range");
    *out = B->sys[i];
  });
}

abi_status abi_batch_use_graph(abi_batch B, int32_t on) {
  return guarded([&] {
    CHEBFI_REQUIRE(B != nullptr, ABI_ERR_ARG, "batch is NULL");
    B->use_graph = (on != 0);
  });
}

abi_status abi_batch_use_overlap(abi_batch B, int32_t on) {
  return guarded([&] {
    CHEBFI_REQUIRE(B != nullptr, ABI_ERR_ARG, "batch is NULL");
    B->overlap = (on != 0);
  });
}

abi_status abi_cheb_filter_batch(abi_batch B, const void *const *X, void *const *Y,
                                 const int64_t *nband, const int64_t *ld, int32_t dtype,
                                 int32_t degree, const double *a, const double *b,
                                 const double *a0, void *stream) {
  return guarded([&] {
    batch_filter(B, X, Y, nband, ld, dtype, degree, a, b, a0, S(stream));
  });
}

abi_status abi_batch_autotune(abi_batch B, const void *const *X, void *const *Y,
                              const int64_t *nband, const int64_t *ld, int32_t dtype,
                              int32_t degree, const double *a, const double *b, const double *a0,
                              int32_t *choice, void *stream) {
  return guarded([&] {
    hipStream_t st = S(stream);
    batch_filter(B, X, Y, nband, ld, dtype, degree, a, b, a0, st);  // validates, warms up
    const bool graph = B->use_graph;
    B->use_graph = false;
    hipEvent_t e0, e1;
    CHEBFI_HIP(hipEventCreate(&e0));
    CHEBFI_HIP(hipEventCreate(&e1));
    float best = -1.f;
    int bf = B->fft_threads, bp = B->proj_threads, br = B->radix_desc, tried = 0;
    try {
      // (the projector products are tiled kernels of a fixed 256 threads)
      for (int rd = 0; rd < 2; ++rd)
        for (int ft : {256, 512}) {
          if (ft < B->fft_min_threads) continue;
          for (int pt : {256}) {
            B->fft_threads = ft;
            B->proj_threads = pt;
            B->radix_desc = rd;
            batch_filter(B, X, Y, nband, ld, dtype, degree, a, b, a0, st);  // warm-up
            // best of three filters: with the projector products on the second
            // stream an eager filter now and then takes much longer than the
            // others (about one in four, seen on the 16-cell batch), which a
            // sum would charge to the variant
            float ms = 1e30f;
            for (int r = 0; r < 3; ++r) {
              CHEBFI_HIP(hipEventRecord(e0, st));
              batch_filter(B, X, Y, nband, ld, dtype, degree, a, b, a0, st);
              CHEBFI_HIP(hipEventRecord(e1, st));
              CHEBFI_HIP(hipEventSynchronize(e1));
              float one = 0.f;
              CHEBFI_HIP(hipEventElapsedTime(&one, e0, e1));
              ms = std::min(ms, one);
            }
            ++tried;
            if (best < 0.f || ms < best) {
              best = ms;
              bf = ft;
              bp = pt;
              br = rd;
            }
          }
        }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      B->use_graph = graph;
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B->fft_threads = bf;
    B->proj_threads = bp;
    B->radix_desc = br;
    B->use_graph = graph;
    batch_filter(B, X, Y, nband, ld, dtype, degree, a, b, a0, st);
    CHEBFI_HIP(hipStreamSynchronize(st));
    if (choice) {
      choice[0] = bf;
      choice[1] = bp;
      choice[2] = br;
      choice[3] = tried;
    }
  });
}

abi_status abi_destroy_batch(abi_batch B) {
  return guarded([&] {
    if (!B) return;
    (void)hipDeviceSynchronize();
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    if (B->side) (void)hipStreamDestroy(B->side);
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    if (B->ev_join) (void)hipEventDestroy(B->ev_join);
    if (B->tab_copied) (void)hipEventDestroy(B->tab_copied);
    if (B->h_tab) (void)hipHostFree(B->h_tab);
    for (abi_system h : B->sys) (void)abi_destroy(h);
    delete B;
  });
}

}  // extern "C"
