// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chebfi.h"

namespace chebfi {

// ---- errors ---------------------------------------------------------------
void set_error(const std::string &msg);

struct Error {
  abi_status code;
  std::string msg;
};

#define CHEBFI_HIP(call)                                                        \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      throw ::chebfi::Error{ABI_ERR_DEVICE, std::string(#call) + ": " +        \
                                                hipGetErrorString(e_)};         \
  } while (0)

#define CHEBFI_REQUIRE(cond, code, msg)                                         \
  do {                                                                          \
    if (!(cond)) throw ::chebfi::Error{(code), (msg)};                          \
  } while (0)

// ---- device buffers -------------------------------------------------------
// A grow-only device allocation owned by the handle.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  void *get(size_t need);  // (re)allocates when too small; contents not kept
  void release();
  ~DevBuf() { release(); }
};
// Counts device-buffer (re)allocations and releases in the process: a captured
// graph is replayed only while it is unchanged (its buffers are all alive).
uint64_t devbuf_generation();

// Work-buffer arena of a no-allocation call.  While one is installed on the
// calling thread, DevBuf::get hands out 256-byte aligned pieces of it (the
// device scratch array) instead of allocating, and fails with ABI_ERR_NOMEM
// when the pieces do not fit.  The DevBufs it lends pieces to get their own
// buffers back when the arena is removed.  `reserve` bytes are kept free by
// the FFT passes, which size their box batch to what is left.
struct ScratchArena {
  char *base = nullptr;
  size_t size = 0, used = 0, reserve = 0;
  struct Lent {
    DevBuf *buf;
    void *ptr;
    size_t bytes;
  };
  std::vector<Lent> lent;
  void *take(DevBuf *b, size_t need);
  size_t remaining() const { return size - used; }
};
extern thread_local ScratchArena *g_scratch_arena;

// Installs an arena for the lifetime of the object and restores the lent
// DevBufs when it ends (also on an error).
struct ArenaScope {
  ScratchArena *arena;
  explicit ArenaScope(ScratchArena *a) : arena(a) { g_scratch_arena = a; }
  ~ArenaScope() {
    for (auto it = arena->lent.rbegin(); it != arena->lent.rend(); ++it) {
      it->buf->ptr = it->ptr;
      it->buf->bytes = it->bytes;
    }
    arena->lent.clear();
    g_scratch_arena = nullptr;
  }
};

// Device address of this library's scratch array on device `dev` (which must
// be current), looked up once per device; scratch_bytes() is its size.
void *scratch_for_device(int dev);
size_t scratch_bytes();

// ---- FFT plan -------------------------------------------------------------
constexpr int kMaxN = 96;       // largest box edge handled by the LDS passes (an FP64
                                // 96 x 97 plane with its twiddles: 152 KB of LDS)
constexpr int kMaxStages = 6;   // radix stages per 1D transform

struct Plan1D {
  int n = 0;
  int nstage = 0;
  int radix[kMaxStages] = {0};
};

bool make_plan(int n, Plan1D *p);  // false if n is not {2,3,5}-smooth

// All 1D plans of a box, passed by value to the FFT kernels.
struct BoxPlan {
  Plan1D d[3];
};

// ---- host setup (system.cpp) ----------------------------------------------
struct Sphere {
  std::vector<int32_t> miller;     // npw*3
  std::vector<int32_t> box_index;  // npw
  std::vector<double> kinetic;     // npw
  std::vector<double> qcart;       // npw*3, k+G
  std::vector<double> gcart;       // npw*3, G
};

abi_status build_sphere(const abi_system_desc *d, Sphere *out, std::string *err);

// ---- per-kernel-class timing (HIP events on the launch stream) ---------------
enum ProfClass {
  PROF_PROJ = 0,     // C = P^H X (projection GEMM, split along plane waves)
  PROF_EXPAND = 1,   // Out += P C' (expansion GEMM)
  PROF_FFT_A = 2,    // sphere -> inverse xy FFT
  PROF_FFT_B = 3,    // z FFT, * V, z FFT
  PROF_FFT_C = 4,    // forward xy FFT -> sphere + recurrence combine
  PROF_DAPPLY = 5,   // split-K sum + D application
  PROF_GRAM = 6,     // Y^H Y and Y^H (H Y)
  PROF_CHOL = 7,     // Cholesky + triangular inverse + reduction to U^-H H_s U^-1
  PROF_EIG = 8,      // Hermitian eigensolver
  PROF_ROT = 9,      // Psi = Y W, H Psi = (H Y) W
  PROF_SPLIT = 10,   // complex64 block -> bf16 hi/lo planes (split-BF16 products)
  PROF_NCLASS = 11
};

struct Profiler {
  bool on = false;
  bool in_filter = false;  // H-application classes are timed inside the filter only
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double work;  // algorithmic flops or bytes of the bracketed launch
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[PROF_NCLASS] = {0};
  double work[PROF_NCLASS] = {0};
  int64_t count[PROF_NCLASS] = {0};
  hipEvent_t take();
  // Brackets one launch: begin() before, end() after (no-ops when off).
  int begin(int cls, double work, hipStream_t st);
  void end(int token, hipStream_t st);
  void collect();  // waits for pending events and accumulates them
  ~Profiler();
};
void reciprocal(const double lattice[9], double B[9]);
void build_projectors(const abi_system_desc *d, const Sphere &s, std::vector<double> *P);

// ---- batched filter over many systems ---------------------------------------
constexpr int kBatchPT = 32;       // projectors per tile of the batched projector products
                                   // (8 atoms: no atom's 4 projectors straddle two tiles)
constexpr int kBatchMaxAtoms = 256; // atoms per system in the batched path
constexpr int kBatchBT = 32;       // bands per tile of the batched projector products
constexpr int kBatchEP = 256;      // plane waves per tile of the batched expansion
constexpr int kBatchKC = 256;      // plane waves per partial sum of the batched projection
constexpr int kBatchBR = 8;        // bands per item of the partial-sum reduction
constexpr int kBatchMaxSys = 1024;

// Per-system device descriptor of the batched passes (plain data).
struct BatchSys {
  BoxPlan plan;               // radix order chosen for the batch
  int64_t npw = 0;
  int nproj = 0;
  int npt = 0;                // projector tiles of kBatchPT
  const int32_t *box_index = nullptr;
  const int32_t *plane = nullptr;
  uint64_t zocc = ~0ull;      // bit i3: z-plane i3 holds sphere points
  const double *kin = nullptr;
  const void *V = nullptr;    // float (complex64 blocks) or double
  const double2 *tw = nullptr;
  const void *P = nullptr;    // npw x nproj complex float or double, column-major
  const double2 *D = nullptr;
  int64_t nband = 0;
  void *box = nullptr;        // nband boxes
  void *Cp = nullptr;         // nproj x nband
  void *E = nullptr;          // npw x nband (ld npw): P C' of the current step
  double2 *Cpart = nullptr;   // per band tile, projector tile, plane-wave chunk: P^H Y_k partials
};

// Per (filter step, system): Out = alpha (H - cshift) Y_k - beta Y_prev.
struct BatchStep {
  const void *yk = nullptr;
  int64_t ldk = 0;
  const void *yprev = nullptr;  // NULL on the first step
  int64_t ldp = 0;
  void *out = nullptr;
  int64_t ldo = 0;
  double alpha = 0, cshift = 0, beta = 0;
};

// Systems of one cubic edge n with specialised passes: their indices and the
// prefix offsets of their items (bands x n per system).
struct BatchGroup {
  int n = 0, nsys = 0;
  const int32_t *gsys = nullptr;
  const int64_t *goff = nullptr;
  int64_t items = 0;
};
constexpr int kBatchMaxGroups = 16;

// What one batched step launches (device pointers and launch shapes).
struct BatchLaunch {
  int nsys = 0;
  const BatchSys *d_sys = nullptr;
  const BatchStep *d_steps = nullptr;  // degree x nsys
  // prefix offsets: band tiles x plane-wave chunks, bands*n3, bands*n2,
  // plane-wave tiles x band tiles, band tiles
  const int64_t *d_off = nullptr;
  int64_t items_p = 0, items_a = 0, items_b = 0, items_e = 0, items_r = 0;
  int max_wgs = 2048;
  int fft_threads = 256, proj_threads = 256;
  size_t lds_a = 0, lds_b = 0, lds_c = 0;  // dynamic LDS of the passes, in elements
  bool any_proj = false;
  int ngroups = 0;  // edge groups with specialised passes (their items are not in items_a/b)
  BatchGroup groups[kBatchMaxGroups];
};

}  // namespace chebfi

// ---- the handle -----------------------------------------------------------
struct abi_system_s {
  int device = 0;
  int n1 = 0, n2 = 0, n3 = 0;
  int64_t npw = 0;
  int natom = 0, nproj = 0;
  int precision = ABI_PREC_FP64;
  double lattice[9] = {0};  // rows a1, a2, a3 (bohr)
  double omega = 0.0;       // cell volume (bohr^3)
  chebfi::Sphere sphere;
  chebfi::BoxPlan plan;

  // device tables
  double *d_kin = nullptr;         // npw
  int32_t *d_box = nullptr;        // npw, box index of each sphere point
  int32_t *d_plane = nullptr;      // n3+1 sphere ranges per i3 plane
  uint64_t zocc = ~0ull;           // bit i3: z-plane i3 holds sphere points (n3 <= 64)
  double *d_P = nullptr;           // npw x nproj complex (interleaved), ld = npw
  double *d_D = nullptr;           // natom*16 complex, row-major per atom
  double *d_V = nullptr;           // n1*n2*n3
  double *d_tw = nullptr;          // 3 * kMaxN complex twiddles exp(-2 pi i j/n_d)
  // mixed-precision copies (ABI_PREC_MIXED handles only)
  float *d_Pf = nullptr;           // npw x nproj complex float
  float *d_Vf = nullptr;           // n1*n2*n3 float
  // split-BF16 planes of P (Re hi, Im hi, Re lo, Im lo), k-contiguous rows:
  uint16_t *d_PA = nullptr;        // rows = projectors, k = plane waves (stride ldPA)
  uint16_t *d_PB = nullptr;        // rows = plane waves, k = projectors (stride ldPB)
  int64_t ldPA = 0, ldPB = 0;
  // overlap S = I + sum_R P_R Q_R P_R^H (descriptions with Q): Q per atom, the
  // projector Gram B = P^H P and the Woodbury kernel K with S^-1 = I - P K P^H
  // (nproj x nproj complex, ld nproj); s_min is the smallest eigenvalue of S
  bool has_S = false;
  double *d_Q = nullptr;           // natom*16 complex, row-major per atom
  double *d_B = nullptr, *d_K = nullptr;
  double s_min = 1.0;
  int mixed_gemm = 0;              // 0: split-BF16 MFMA, 1: FP32 MFMA projector products
  int generic_fft = 0;             // 1: runtime-size FFT passes also for cubic boxes
  int pl_proj = 0, pl_expand = 0;  // tile variants of the split-BF16 products
  // Chained planes (projection variants 15, 16, inside one filter run): the last
  // FFT pass of a step also writes the bf16 planes of its output into `planes`,
  // so that the next step's projection needs no split pass.  pl_have: the block
  // whose planes `planes` holds (null: none); pl_assume: treat them as present
  // (the autotuner's timing of a chained step).
  bool pl_chain = false, pl_assume = false;
  const void *pl_have = nullptr;

  // work buffers
  chebfi::DevBuf box, cpart, cprime, blk1, blk2, blk3, small1, small2, small3, small4, small5, scal;
  chebfi::DevBuf eig1, eig2, eig3, blk4, box2, adj, adjsmall, adjc, planes, cplanes;
  chebfi::DevBuf solve1, solve2, solve3, solve4, solve5;  // blocks of the multi-cycle driver
  chebfi::DevBuf expout;  // projector part P C' of the mixed H application
  chebfi::DevBuf tune_out;  // output block of the autotuner's timed H applications
  chebfi::DevBuf rr_planes;  // split-BF16 Rayleigh-Ritz: planes of the equilibrated block
  chebfi::DevBuf gen_c, gen_e, gen_f, gen_ff, blk5, blk6;  // overlap path
  chebfi::DevBuf lob_z, lob_hz, lob_sz, lob_t1, lob_t2, lob_t3, lob_psi, lob_hp, lob_sp, lob_c,
      lob_g, lob_v;  // block LOBPCG
  chebfi::DevBuf scf_rho, scf_v, scf_box, scf_w;  // SCF step

  void *scratch = nullptr;  // this device's scratch array (no-allocation calls)
  int fft_batch = 0;  // bands per FFT batch (box buffer holds this many boxes)
  // second stream: with overlap = 1 (CHEBFI_OVERLAP=1) the FFT passes of an H
  // application run on it beside the projection GEMM (they are independent until
  // the expansion).  Off by default: the GEMM workgroups hold 128 KB of LDS, so an
  // FFT workgroup cannot share a CU with one and the two only time-slice the chip.
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_half = nullptr;
  int overlap = 0;
  chebfi::Profiler prof;

  // Captured filter: abi_cheb_filter records its launches once into a HIP graph
  // (on cap_stream) and replays it on the caller's stream while the arguments,
  // the launch choices and the work buffers (devbuf_generation) are unchanged;
  // the coefficients of each step are read from `coef` (uploaded from h_coef
  // before each replay), through coef_dev while the launches are recorded.
  int filter_graph = 0;
  hipStream_t cap_stream = nullptr;
  struct FilterGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t key[16] = {0};
  };
  static constexpr int kFilterGraphs = 4;  // (a loop alternating two block pairs keeps both)
  FilterGraph fg[kFilterGraphs];
  int fg_next = 0;
  chebfi::DevBuf coef;
  double *h_coef = nullptr;
  size_t h_coef_n = 0;
  hipEvent_t coef_copied = nullptr;
  const double *coef_dev = nullptr;
};
