// libpipesafe: host driver and C ABI of the gfx950 BiCGSafe-family solvers.
//
// Iteration schedules (one enqueue per iteration; every kernel reads the
// device stop flag, so iterations enqueued past the stop are no-ops and the
// host only polls the flag once per batch of iterations):
//
//   p-BiCGSafe (Algorithm 4), iteration i:
//     stream A:  As_i = A s_i                      (sparse product)
//     stream B:  9 inner products + finish        (concurrent with A s_i: the
//                                                  one-GPU form of hiding the
//                                                  global reduction, Section 3)
//     stream A:  join; pass A (ten updates); A w_i + pass B (l, g, s) epilogue
//   p-BiCGSafe, fused-dot schedule (option): pass A and the epilogue of A w_i
//     also write block partial sums of the next iteration's nine inner
//     products, so stream B only folds them and runs the finish, concurrently
//     with A s_{i+1}; the separate inner-product pass disappears.
//   ssBiCGSafe2 (Algorithm 3): s_i = A r_i; 9 inner products + finish;
//     p, u; w_i = A u_i + epilogue (t, z, y, x, r).  One stream: the inner
//     products need s_i.
//   p-BiCGSafe-rr (Algorithm 5): p-BiCGSafe, except every m-th iteration
//     (0 < i < M) runs the replacement step with products A o, A u, A x,
//     A t, A y, A r (A s_i, unused there, is skipped).
//   p-BiCGStab: pass 1; [A z_i || (q,y),(y,y) + omega]; pass 2;
//     [A w_{i+1} || 5 inner products + stop test + beta, alpha].
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "pipesafe.h"
#include "device_common.hpp"
#include "dots.hpp"
#include "layout.hpp"
#include "solve_one.hpp"
#include "spmv.hpp"
#include "updates.hpp"

using namespace ps;

namespace {

constexpr int kSlotTmp = PS_V_COUNT;  // internal scratch vector
constexpr int kNumSlots = PS_V_COUNT + 1;
constexpr int kMaxDotGrid = 512;  // partial-sum blocks: two per CU
// Automatic choices (options overlap = -1, schedule = -1), from measurements on
// 4k..2M-row stencils and band matrices: a second stream pays once one sparse
// product streams at least kOverlapMinBytes (below that the cross-stream waits
// cost more than they hide); the fused schedules pay on the sliced layout at
// every size, and on CSR below kFusedMinRows rows, but not on large CSR
// matrices with uneven rows, whose gather-bound product gains little from the
// skipped pass and pays for the extra reads in its epilogue.
constexpr int64_t kOverlapMinBytes = 128ll << 20;
constexpr int64_t kFusedMinRows = 1 << 18;
// schedule 4 (the whole solve in one workgroup per system): its largest
// workgroup (1024 threads leave 128 registers per lane, and the epilogue's
// accumulators then spill: 58.4 against 43.3 us per iteration on 4096 rows),
// the threads the chip holds at once (two 64-lane waves per SIMD at the
// kernel's 176 registers: 8 waves on each of 256 CUs), and the rows per system
// it accepts at all
constexpr int kOneGroupThreads = 512;
constexpr int64_t kOneGroupResident = 256 * 8 * 64;
constexpr int64_t kOneGroupMaxRows = 1 << 20;
// the automatic schedule's choice (auto_schedule): one system, a batch's largest
constexpr int64_t kOneGroupAutoRows = 1024, kOneGroupBatchAutoRows = 1600;
// p-BiCGSafe's update passes stream the vectors they do not hand to the next
// kernel past the cache once an iteration moves at least kStreamMinBytes (well
// above the 256 MiB last-level cache; below it the cache still holds part of
// the previous iteration's vectors and the hint costs a little).
constexpr int64_t kStreamMinBytes = 512ll << 20;
// p-BiCGStab's passes and ssBiCGSafe2's epilogue stream from a larger
// iteration: the hints cost 2-3% at 112^3 (~550 MiB by the same count) and save
// 18% (p-BiCGStab) and 4.6% (ssBiCGSafe2) at 128^3 (~825 MiB)
constexpr int64_t kOtherStreamMinBytes = 640ll << 20;
constexpr double kSellMaxPadding = 1.10;  // sliced ELLPACK if its slots <= 1.10 nnz
constexpr int64_t kSellUnroll7MinRows = 1 << 20;  // seven slots per step from here (sell_launch)
// ... or <= 1.5 nnz for systems the automatic schedule solves in one workgroup
// each (schedule 4 needs the sliced layout; it reads a row's entries once, or
// from cache, so their padding costs it little): a batch of 4096 systems of
// 8^2..16^2 rows has 1.25 slots per entry
constexpr double kSellMaxPaddingSmall = 1.5;
constexpr int kSellRowsPerLane = 1;       // 64-row slices
constexpr double kTuneMaxPadding = 1.5;   // the autotuner tries the sliced layout up to this
// fused schedules: the finish adds the partial lists itself (no fold kernel)
// when they hold at most this many workgroups' pairs
constexpr int kDirectFinishMax = 4096;

struct Timer {
  hipEvent_t a, b;
  int cls;
  int iter;  // iteration the launch belongs to (-1: set-up)
  bool aux;  // enqueued on the second (reduction) stream
};

// Everything a captured batch of iterations depends on.
struct GraphKey {
  int variant, maxit, rr_m, rr_M, overlap, count, phase, schedule, precision;
  double tol;
  hipStream_t stream;
  bool operator==(const GraphKey &o) const {
    return variant == o.variant && maxit == o.maxit && rr_m == o.rr_m && rr_M == o.rr_M &&
           overlap == o.overlap && count == o.count && phase == o.phase &&
           schedule == o.schedule && precision == o.precision && tol == o.tol &&
           stream == o.stream;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
  int sweep_flip;  // parity of the full sweeps the batch performs
};

}  // namespace

// Static workspace of ps_solve_dev_static (callers that cannot allocate): the
// scalar and control blocks, inner-product partial sums and the residual
// history of one solve.  Each GPU the library runs on holds its own copy for
// the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (static_workspace()).
constexpr size_t kScratchDoubles = (size_t)1 << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

struct ps_matrix {
  int device = -1;
  int64_t n = 0, nnz = 0;
  int *rowptr = nullptr, *col = nullptr, *blk = nullptr;
  unsigned char *rord = nullptr;  // CSR, multi-lane shapes: rows of each block longest first
  short *col16 = nullptr;         // CSR column - first row of its row block (index_bits 16)
  unsigned short *pos = nullptr;  // CSR gather order: each entry's place in its block's row order
  bool gather_sort = false;       // CSR: blocks stored in column order (pos != nullptr)
  double *val = nullptr;
  int nblk = 0;             // workgroups of one sparse product
  int shape = 1;            // SpMV shape: 0..4 = (IPT, LPR) (4,1) (8,1) (16,4) (16,8) (16,16)
  int format = PS_FMT_CSR;  // device layout of the matrix
  int *scol = nullptr, *soff = nullptr;  // sliced ELLPACK arrays (format PS_FMT_SELL)
  short *scol16 = nullptr;               // sliced ELLPACK column - row (index_bits 16)
  int index_bits = 32;                   // stored column index (either layout): 32 or 16
  double *sval = nullptr;
  int64_t slots = 0;
  int nslice = 0;
  int sell_rpl = 1;                      // rows per lane of the sliced layout (1 or 2)
  int sell_width = 0;                    // the sliced layout's widest slice (entries per row)
  int stream_override = -1;              // streaming update passes: -1 automatic, 0, 1
  // the values rounded to FP32 (mixed-precision solves), made on first use
  float *val32 = nullptr, *sval32 = nullptr;
  bool f32_ok = true;                    // every value rounds to a finite FP32 number
  bool pzu32 = false;                    // the p, u, z slots hold FP32 numbers (precision 3)
  size_t ld = 0;            // doubles between consecutive vector slots (256-byte multiple)
  double *vec = nullptr;    // kNumSlots * ld doubles
  double *sc = nullptr;     // SC_COUNT doubles
  int *ctl = nullptr;       // C_COUNT ints
  double *partials = nullptr;
  int dot_grid = 0;
  // fused-dot schedule: pass A partials [5][ga], epilogue partials [4][nblk],
  // folded partials [9][gfold], all (a, b, c) triples, in one allocation
  double *fpart = nullptr;
  int ga = 0, gfold = 0;
  // batched solves (nsys > 1): the caller's rows map to padded rows (each
  // system padded to a multiple of 512), one control/scalar block and history
  // row per system, inner-product partials per 512-row workgroup
  int nsys = 1;
  int64_t n_orig = 0;            // rows of the caller's concatenation (= n for one system)
  int64_t max_sys_rows = 0;      // rows of the largest system (= n for one system)
  int *chunk_sys = nullptr;      // device: system of each 256-row chunk (nullptr: one system)
  int *first_blk = nullptr;      // device: first 512-row workgroup of each system, [nsys+1]
  int *first_pblk = nullptr;     // device: first sparse-product workgroup of each system
  int *sys_end = nullptr;        // device: end of each system's own rows, [nsys]
  int *row_map = nullptr;        // device: padded row of each caller row
  double *stage = nullptr;       // device: n_orig doubles for host input/output
  double *bpart = nullptr;       // device: [9][n/512] partial triples
  int64_t hist_stride = 0;       // history entries per system
  double *hist = nullptr;
  int64_t hist_cap = 0;
  int *pinned = nullptr;    // 2 * C_COUNT ints of pinned host memory
  hipStream_t own = nullptr, aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_batch[2] = {nullptr, nullptr};
  std::atomic<int> busy{0};
  // kernel timing
  int prof_mask = 0;
  int cur_iter = -1;        // iteration being enqueued (for kernel timing)
  int sweep = 0;            // direction of the next full-sweep kernel (0 forward, 1 backward)
  std::vector<GraphEntry> graphs;  // instantiated batches of iterations
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<Timer> timers;
  double prof_ms[PS_K_COUNT] = {};
  int64_t prof_cnt[PS_K_COUNT] = {};
  int64_t prof_aux[PS_K_COUNT] = {};     // of those, launches on the second stream

  double *slot(int s) const { return vec + (size_t)s * ld; }
  int *running() const { return ctl + (size_t)nsys * C_COUNT; }
  int nblk512() const { return (int)(n / 512); }
  template <class VT, class IT>
  CsrDev<VT, IT> csr() const {
    CsrDev<VT, IT> A{};
    A.rowptr = rowptr;
    if constexpr (sizeof(IT) == 4) A.col = col;
    else A.col = col16;
    if constexpr (sizeof(VT) == 8) A.val = val;
    else A.val = val32;
    A.blk = blk;
    A.rord = rord;
    A.pos = pos;
    A.nblk = nblk;
    return A;
  }
  template <class VT, class IT>
  SellDev<VT, IT> sell() const {
    SellDev<VT, IT> S{};
    if constexpr (sizeof(IT) == 4) S.col = scol;
    else S.col = scol16;
    if constexpr (sizeof(VT) == 8) S.val = sval;
    else S.val = sval32;
    S.off = soff;
    S.n = (int)n;
    S.nblk = nblk;
    return S;
  }
};

namespace {

#define PS_HIP(...)                                                                   \
  do {                                                                                \
    hipError_t e_ = (__VA_ARGS__);                                                    \
    if (e_ != hipSuccess) {                                                           \
      std::fprintf(stderr, "pipesafe: %s failed: %s\n", #__VA_ARGS__, hipGetErrorString(e_)); \
      return PS_EHIP;                                                                 \
    }                                                                                 \
  } while (0)

struct BusyGuard {
  std::atomic<int> &flag;
  bool ok;
  explicit BusyGuard(std::atomic<int> &f) : flag(f) {
    int expect = 0;
    ok = flag.compare_exchange_strong(expect, 1);
  }
  ~BusyGuard() {
    if (ok) flag.store(0);
  }
};

int next_event(ps_matrix *M, hipEvent_t *ev) {
  if (M->ev_used == M->ev_pool.size()) {
    hipEvent_t e;
    PS_HIP(hipEventCreate(&e));
    M->ev_pool.push_back(e);
  }
  *ev = M->ev_pool[M->ev_used++];
  return PS_OK;
}

// Launch `kernel` on `s`; when class `cls` is profiled, the runtime records a
// pair of events at the start and the end of the kernel's execution itself
// (hipExtLaunchKernelGGL), so the timing excludes the dispatch around it.
template <typename Kernel, typename... Args>
int launch(ps_matrix *M, hipStream_t s, int cls, Kernel kernel, dim3 grid, size_t shmem,
           Args... args) {
  if (grid.x == 0) return PS_OK;
  const bool prof = (M->prof_mask >> cls) & 1;
  if (!prof) {
    hipLaunchKernelGGL(kernel, grid, dim3(kBlock), shmem, s, args...);
    return PS_OK;
  }
  hipEvent_t a = nullptr, b = nullptr;
  if (next_event(M, &a) || next_event(M, &b)) return PS_EHIP;
  hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), (uint32_t)shmem, s, a, b, 0u, args...);
  M->timers.push_back(Timer{a, b, cls, M->cur_iter, s == M->aux && s != nullptr});
  return PS_OK;
}

#define PS_TRY(...)                 \
  do {                              \
    int rc_ = (__VA_ARGS__);        \
    if (rc_ != PS_OK) return rc_;   \
  } while (0)

// The device address of `scratch` on device `dev` (which must be current),
// looked up once per device and kept.
constexpr int kMaxDevices = 64;
double *g_scratch_addr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int static_workspace(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return PS_ENODEV;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *addr = nullptr;
    PS_HIP(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
    if (!addr) return PS_EHIP;
    g_scratch_addr[dev] = (double *)addr;
  }
  *out = g_scratch_addr[dev];
  return PS_OK;
}

dim3 pair_grid(int64_t n) { return dim3((unsigned)((n + 2 * kBlock - 1) / (2 * kBlock))); }
dim3 elem_grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

// Direction of the next full sweep over the rows: consecutive sweeps alternate
// (see sweep_block).
// fold slices of the separate inner-product pass's partial lists
int dot_slices(const ps_matrix *M) { return (M->dot_grid + kBlock - 1) / kBlock; }

int next_rev(ps_matrix *M) {
  const int r = M->sweep;
  M->sweep ^= 1;
  return r;
}

template <int IPT, int LPR, class Epi>
int spmv_launch(ps_matrix *M, hipStream_t s, int cls, const double *x, Epi epi, Stop stop,
                int rev, bool f32) {
  const size_t lds = (size_t)IPT * kBlock * sizeof(double);
  const dim3 g(M->nblk);
  if (M->index_bits == 16)
    return f32 ? launch(M, s, cls, k_spmv<IPT, LPR, float, short, Epi>, g, lds,
                        M->template csr<float, short>(), x, epi, stop, rev)
               : launch(M, s, cls, k_spmv<IPT, LPR, double, short, Epi>, g, lds,
                        M->template csr<double, short>(), x, epi, stop, rev);
  return f32 ? launch(M, s, cls, k_spmv<IPT, LPR, float, int, Epi>, g, lds,
                      M->template csr<float, int>(), x, epi, stop, rev)
             : launch(M, s, cls, k_spmv<IPT, LPR, double, int, Epi>, g, lds,
                      M->template csr<double, int>(), x, epi, stop, rev);
}

// A product whose epilogue forms partial sums of inner products gives each
// workgroup M->sell_chunks row blocks (one system only: a batch's workgroups
// must not cross systems), so that its partial lists are short.
template <class VT, class IT, class Epi>
int sell_launch(ps_matrix *M, hipStream_t s, int cls, const double *x, Epi epi, Stop stop,
                int rev) {
  const SellDev<VT, IT> S = M->template sell<VT, IT>();
  const dim3 g(M->nblk);
  if (M->sell_rpl == 2) return launch(M, s, cls, k_sell<2, VT, IT, Epi>, g, 0, S, x, epi, stop, rev);
  // batches whose slices hold at most five entries per row (five-point stencils)
  // load five slots per step instead of eight (the 512-system stencil batch:
  // 464.1 -> 441.1 ms; one 1024^2 stencil: 67.1 -> 68.2 us per iteration, so
  // single systems keep eight)
  if (M->nsys > 1 && M->sell_width <= kSellUnrollNarrow)
    return launch(M, s, cls, k_sell<1, VT, IT, Epi, kSellUnrollNarrow>, g, 0, S, x, epi, stop, rev);
  // large systems whose slices hold exactly seven entries per row (seven-point
  // stencils): seven slots per step, none loaded in vain.  Measured on one box,
  // schedule 3, us per iteration with eight / seven: 128^3 127.3 / 126.2, 112^3
  // 90.3 / 90.0, but 96^3 62.8 / 64.6, 64^3 32.8 / 33.3, 32^3 19.9 / 20.1
  if (M->sell_width == kSellUnroll7 && M->n >= kSellUnroll7MinRows)
    return launch(M, s, cls, k_sell<1, VT, IT, Epi, kSellUnroll7>, g, 0, S, x, epi, stop, rev);
  return launch(M, s, cls, k_sell<1, VT, IT, Epi>, g, 0, S, x, epi, stop, rev);
}

// One sparse product with epilogue `epi`; `stop_word` (C_DONE, C_HALT or -1)
// names the control word that makes it a no-op (per system).  f32: read the
// values rounded to FP32 (mixed-precision solves) instead of the FP64 ones.
template <class Epi>
int spmv(ps_matrix *M, hipStream_t s, int cls, const double *x, Epi epi, int stop_word,
         bool f32 = false) {
  const int rev = next_rev(M);
  const Stop stop{M->ctl, stop_word, M->chunk_sys};
  if (M->format == PS_FMT_SELL) {
    if (M->index_bits == 16)
      return f32 ? sell_launch<float, short>(M, s, cls, x, epi, stop, rev)
                 : sell_launch<double, short>(M, s, cls, x, epi, stop, rev);
    return f32 ? sell_launch<float, int>(M, s, cls, x, epi, stop, rev)
               : sell_launch<double, int>(M, s, cls, x, epi, stop, rev);
  }
  switch (M->shape) {
    case 0: return spmv_launch<4, 1>(M, s, cls, x, epi, stop, rev, f32);
    case 1: return spmv_launch<8, 1>(M, s, cls, x, epi, stop, rev, f32);
    case 2: return spmv_launch<16, 4>(M, s, cls, x, epi, stop, rev, f32);
    case 3: return spmv_launch<16, 8>(M, s, cls, x, epi, stop, rev, f32);
    default: return spmv_launch<16, 16>(M, s, cls, x, epi, stop, rev, f32);
  }
}

template <class Prod, class Fin>
int dots(ps_matrix *M, hipStream_t s, std::initializer_list<const double *> in, int maxit,
         double tol, int flags, double *hist) {
  DotArgs A{};
  int j = 0;
  for (const double *p : in) A.v[j++] = p;
  A.n = M->n;
  A.partials = M->partials;
  A.ctl = M->ctl;
  A.sc = M->sc;
  A.hist = hist;
  A.maxit = maxit;
  A.tol = tol;
  A.flags = flags;
  A.running = M->running();
  if (M->nsys > 1) {
    A.partials = M->bpart;
    PS_TRY(launch(M, s, PS_K_DOTS, k_dots_batch<Prod>, dim3(M->nblk512()), 0, A,
                  (const int *)M->chunk_sys));
    return launch(M, s, PS_K_DOTS_FINISH, k_dots_finish_batch<Prod::ND, Fin>, dim3(M->nsys), 0, A,
                  (const int *)M->first_blk, M->nblk512(), M->hist_stride);
  }
  PS_TRY(launch(M, s, PS_K_DOTS, k_dots<Prod>, dim3(M->dot_grid), 0, A));
  // the [ND][dot_grid] partials folded by a few workgroups, the last of which
  // finishes; the folded slices go after the partials
  const FoldLists lists{M->partials, M->partials, M->dot_grid, M->dot_grid, 0u, 0x876543210ull};
  A.partials = M->partials + kPart * 9 * (size_t)M->dot_grid;
  return launch(M, s, PS_K_DOTS_FINISH, k_fold_finish<Prod::ND, Fin>, dim3(dot_slices(M)), 0,
                lists, A);
}

// ------------------------------------------------------------------ set-up

int zero_slots(ps_matrix *M, hipStream_t s, std::initializer_list<int> slots) {
  for (int sl : slots)
    PS_TRY(launch(M, s, PS_K_OTHER, k_zero, elem_grid(M->n), 0, M->slot(sl), (int64_t)M->ld, 1,
                  M->n));
  return PS_OK;
}

struct Plan {
  int variant;
  int maxit;
  double tol;
  int rr_m, rr_M;
  int norm_ref;
  bool resume;
  int i0;
  hipStream_t A, B;
  bool overlap;
  bool fused;     // fused-dot schedule (p-BiCGSafe): schedule 1 or 2
  bool fused2;    // schedules 2, 3: every update but w_i in the epilogue of A w_i
  bool fused3;    // schedule 3: the reduction folded and finished inside A s_i, one stream
  bool one;       // schedule 4: the whole solve in one workgroup (k_solve_one)
  bool fallback;  // replace an initial guess that is worse than zero
  bool scale;     // first scale the guess to its least residual (x0_fallback = 2)
  bool stream_nt; // streaming (nontemporal) loads and stores in the update passes
  int precision;  // 0 FP64; 1 FP32 values in every product; 2 FP32 in the Krylov products
  bool kry32;     // the Krylov products read the FP32 values
  bool res32;     // the residual statements (r = b - A x) read the FP32 values
  bool vec32;     // p, u, z held as FP32 numbers (precision 3, p-BiCGSafe(-rr))
};

// r_0 = b - A x_0, r0* = r_0 and the zero vectors of each algorithm (x_0 and b
// are already in their slots).
int enqueue_setup(ps_matrix *M, const Plan &P) {
  hipStream_t s = P.A;
  double *X = M->slot(PS_V_X), *R = M->slot(PS_V_R), *RS = M->slot(PS_V_RS),
         *Bv = M->slot(PS_V_B);
  if (P.variant == PS_PBICGSTAB) {
    PS_TRY(zero_slots(M, s, {PS_V_P, PS_V_S, PS_V_Z, PS_V_V, PS_V_Q, PS_V_Y, PS_V_U, PS_V_L,
                             PS_V_G, PS_V_O, PS_V_AS}));
  } else {
    PS_TRY(zero_slots(M, s, {PS_V_Y, PS_V_T, PS_V_P, PS_V_U, PS_V_Z, PS_V_W, PS_V_L, PS_V_G,
                             PS_V_Q, PS_V_O, PS_V_AS, PS_V_V}));
  }
  if (P.scale) {
    // c = (A x0, b) / (A x0, A x0), x0 = c x0 (a residual statement: FP64 values
    // unless every product reads the rounded ones)
    double *Ax = M->slot(kSlotTmp);
    PS_TRY(spmv(M, s, PS_K_OTHER, X, EpiStore{Ax}, -1, P.res32));
    PS_TRY(dots<ProdScale, FinScale>(M, s, {Ax, Bv}, P.maxit, P.tol, 0, M->hist));
    PS_TRY(launch(M, s, PS_K_OTHER, k_scale_x, elem_grid(M->n), 0, X, (const double *)M->sc,
                  (const int *)M->chunk_sys, M->n));
  }
  PS_TRY(spmv(M, s, PS_K_OTHER, X, EpiResidual{Bv, R, RS}, -1, P.res32));
  if (P.fallback) {
    PS_TRY(dots<ProdFallback, FinFallback>(M, s, {R, Bv}, P.maxit, P.tol, 0, M->hist));
    PS_TRY(launch(M, s, PS_K_OTHER, k_fallback, elem_grid(M->n), 0, X, R, RS, (const double *)Bv,
                  (const double *)M->sc, (const int *)M->chunk_sys, M->n));
  }
  if (P.variant == PS_PBICGSAFE || P.variant == PS_PBICGSAFE_RR) {
    // s_0 = A r_0 (its definition s_i := A r_i; Algorithm 4 uses s_0 without forming it)
    PS_TRY(spmv(M, s, PS_K_OTHER, R, EpiStore{M->slot(PS_V_S)}, -1, P.kry32));
  }
  if (P.norm_ref == 1) {
    PS_TRY(dots<ProdNorm, FinNormRef>(M, s, {Bv}, P.maxit, P.tol, 0, M->hist));
  }
  if (P.variant == PS_PBICGSTAB) {
    double *W = M->slot(PS_V_W), *T = M->slot(PS_V_T);
    PS_TRY(spmv(M, s, PS_K_OTHER, R, EpiStore{W}, -1, P.kry32));  // w_0 = A r_0
    PS_TRY(spmv(M, s, PS_K_OTHER, W, EpiStore{T}, -1, P.kry32));  // t_0 = A w_0
    PS_TRY(dots<ProdStab3, FinStabSetup>(M, s, {RS, R, W}, P.maxit, P.tol,
                                         P.norm_ref == 0 ? DF_SET_REF : 0, M->hist));
  }
  return PS_OK;
}

// fork: stream B waits for everything enqueued on A so far
int fork(ps_matrix *M, const Plan &P) {
  if (!P.overlap) return PS_OK;
  PS_HIP(hipEventRecord(M->ev_fork, P.A));
  PS_HIP(hipStreamWaitEvent(P.B, M->ev_fork, 0));
  return PS_OK;
}
// join: stream A waits for everything enqueued on B so far
int join(ps_matrix *M, const Plan &P) {
  if (!P.overlap) return PS_OK;
  PS_HIP(hipEventRecord(M->ev_join, P.B));
  PS_HIP(hipStreamWaitEvent(P.A, M->ev_join, 0));
  return PS_OK;
}

// ------------------------------------------------------------ iterations

int iter_safe_dots(ps_matrix *M, const Plan &P, hipStream_t s, int i) {
  const int flags = (i == 0 && !P.resume && P.norm_ref == 0) ? DF_SET_REF : 0;
  double *S = M->slot(PS_V_S), *Y = M->slot(PS_V_Y), *R = M->slot(PS_V_R),
         *RS = M->slot(PS_V_RS), *T = M->slot(PS_V_T);
  if (i == 0)
    return dots<ProdSafe9<true>, FinSafe>(M, s, {S, Y, R, RS, T}, P.maxit, P.tol, flags, M->hist);
  return dots<ProdSafe9<false>, FinSafe>(M, s, {S, Y, R, RS, T}, P.maxit, P.tol, flags, M->hist);
}

// Fused-dot schedule: the reduction phase of iteration i from the partial sums
// that pass A and the epilogue of A w_{i-1} wrote.
int fused_finish(ps_matrix *M, const Plan &P, hipStream_t s) {
  // schedule 1: pass A's [5][ga] then the epilogue's [4][nblk]; schedule 2: the
  // epilogue's [5][nblk] then [4][nblk]; the folded [9][gfold] after the largest
  const int ga = P.fused2 ? M->nblk : M->ga;
  double *pa = M->fpart, *pb = pa + kPart * 5 * (size_t)ga;
  double *pf = M->fpart + kPart * (5 * (size_t)std::max(M->ga, M->nblk) + 4 * (size_t)M->nblk);
  DotArgs D{};
  D.n = M->n;
  D.ctl = M->ctl;
  D.sc = M->sc;
  D.hist = M->hist;
  D.maxit = P.maxit;
  D.tol = P.tol;
  D.flags = 0;
  D.running = M->running();
  if (M->nsys > 1)  // per system, over its ranges of both lists
    return launch(M, s, PS_K_DOTS_FINISH, k_dots_finish_batch_direct<FinSafe>, dim3(M->nsys), 0,
                  D, (const double *)pa, ga,
                  (const int *)(P.fused2 ? M->first_pblk : M->first_blk), (const double *)pb,
                  M->nblk, (const int *)M->first_pblk, M->hist_stride);
  if (ga + M->nblk <= kDirectFinishMax)  // short lists: no fold
    return launch(M, s, PS_K_DOTS_FINISH, k_dots_finish_direct<FinSafe>, dim3(1), 0, D,
                  (const double *)pa, ga, (const double *)pb, M->nblk);
  PS_TRY(launch(M, s, PS_K_DOTS, k_fold_partials, dim3(M->gfold), 0, (const double *)pa, ga,
                (const double *)pb, M->nblk, pf, (const int *)M->ctl));
  D.partials = pf;
  return launch(M, s, PS_K_DOTS_FINISH, k_dots_finish<9, FinSafe>, dim3(1), 0, D, M->gfold);
}

// p-BiCGSafe-rr: iteration i is a replacement step (Algorithm 5)
bool replacement(const Plan &P, int i) {
  return P.variant == PS_PBICGSAFE_RR && P.rr_m > 0 && (i % P.rr_m) == 0 && i > 0 && i < P.rr_M;
}
bool after_replacement(const Plan &P, int i) { return i > 0 && replacement(P, i - 1); }
// schedule 3: iteration j's reduction phase is folded and finished inside its
// product A s_j, from the partial sums the previous fused epilogue left -- the
// iterations whose inner products schedule 2 takes from those sums
bool fold_in_product(const Plan &P, int j) {
  return P.fused3 && j > P.i0 && !replacement(P, j) && !after_replacement(P, j);
}

int iter_pbicgsafe(ps_matrix *M, const Plan &P, int i) {
  hipStream_t A = P.A;
  double *X = M->slot(PS_V_X), *R = M->slot(PS_V_R), *S = M->slot(PS_V_S), *Y = M->slot(PS_V_Y),
         *T = M->slot(PS_V_T), *Pp = M->slot(PS_V_P), *U = M->slot(PS_V_U), *Z = M->slot(PS_V_Z),
         *W = M->slot(PS_V_W), *L = M->slot(PS_V_L), *G = M->slot(PS_V_G), *Q = M->slot(PS_V_Q),
         *O = M->slot(PS_V_O), *As = M->slot(PS_V_AS), *Bv = M->slot(PS_V_B);
  const bool replace = replacement(P, i);
  if (!replace) {
    if (fold_in_product(P, i)) {
      // schedule 3, one stream: A s_i, whose first workgroups fold the previous
      // epilogue's partial sums and finish the reduction phase; the stop word is
      // C_DONE, as nothing else runs beside it
      double *pa = M->fpart, *pb = pa + kPart * 5 * (size_t)M->nblk;
      DotArgs D{};
      D.n = M->n;
      D.partials = M->fpart + kPart * (5 * (size_t)std::max(M->ga, M->nblk) + 4 * (size_t)M->nblk);
      D.ctl = M->ctl;
      D.sc = M->sc;
      D.hist = M->hist;
      D.maxit = P.maxit;
      D.tol = P.tol;
      D.flags = 0;
      D.running = M->running();
      const FoldLists lists{pa, pb, M->nblk, M->nblk, kSafeFromB, kSafeRows};
      PS_TRY(spmv(M, A, PS_K_SPMV, S, EpiStoreFold<9, FinSafe>{As, lists, M->gfold, D}, C_DONE,
                  P.kry32));
    } else {
      PS_TRY(fork(M, P));
      // the reduction phase on the second stream, enqueued first so that its few
      // workgroups are dispatched ahead of the product's thousands; the partial
      // sums come from the previous iteration's passes, which the first
      // iteration and the one after a replacement step do not have
      if (P.fused && i > P.i0 && !after_replacement(P, i))
        PS_TRY(fused_finish(M, P, P.B));
      else PS_TRY(iter_safe_dots(M, P, P.B, i));
      PS_TRY(spmv(M, A, PS_K_SPMV, S, EpiStore{As}, C_HALT, P.kry32));  // As_i, concurrently
      PS_TRY(join(M, P));
    }
    if (!P.fused) {
      PassAArgs pa{X, R, Pp, U, T, Y, Z, W, S, As, L, G, M->sc, M->ctl, M->n, next_rev(M),
                   nullptr, nullptr};
      pa.chunk_sys = M->chunk_sys;
      const dim3 g = pair_grid(M->n);
      if (P.vec32)
        PS_TRY(P.stream_nt
                   ? launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<false, true, float>, g, 0, pa)
                   : launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<false, false, float>, g, 0, pa));
      else
        PS_TRY(P.stream_nt
                   ? launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<false, true>, g, 0, pa)
                   : launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<false, false>, g, 0, pa));
      PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, W, EpiPBiCGSafeB{As, L, G, S, M->sc}, C_DONE, P.kry32));
      return PS_OK;
    }
    if (P.fused2) {
      // only w_i before the product; everything else in its epilogue, which also
      // forms the nine partial sums of iteration i+1
      PassWArgs pw{As, L, G, W, M->sc, M->ctl, M->n, next_rev(M), M->chunk_sys};
      PS_TRY(launch(M, A, PS_K_UPDATE, k_pass_w, pair_grid(M->n), 0, pw));
      double *part = M->fpart, *RS = M->slot(PS_V_RS);
      if (P.vec32 && P.stream_nt)
        PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, W,
                    EpiPBiCGSafeAll<true, float>{R, Pp, U, S, T, Y, Z, X, L, G, As, W, RS, M->sc,
                                                 part},
                    C_DONE, P.kry32));
      else if (P.vec32)
        PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, W,
                    EpiPBiCGSafeAll<false, float>{R, Pp, U, S, T, Y, Z, X, L, G, As, W, RS, M->sc,
                                                  part},
                    C_DONE, P.kry32));
      else if (P.stream_nt)
        PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, W,
                    EpiPBiCGSafeAll<true>{R, Pp, U, S, T, Y, Z, X, L, G, As, W, RS, M->sc, part},
                    C_DONE, P.kry32));
      else
        PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, W,
                    EpiPBiCGSafeAll<false>{R, Pp, U, S, T, Y, Z, X, L, G, As, W, RS, M->sc, part},
                    C_DONE, P.kry32));
      return PS_OK;
    }
    double *pa_part = M->fpart, *pb_part = pa_part + kPart * 5 * (size_t)M->ga;
    PassAArgs pa{X, R, Pp, U, T, Y, Z, W, S, As, L, G, M->sc, M->ctl, M->n, next_rev(M),
                 M->slot(PS_V_RS), pa_part};
    pa.chunk_sys = M->chunk_sys;
    if (P.vec32)
      PS_TRY(P.stream_nt
                 ? launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<true, true, float>, pair_grid(M->n),
                          0, pa)
                 : launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<true, false, float>, pair_grid(M->n),
                          0, pa));
    if (P.stream_nt) {
      if (!P.vec32)
        PS_TRY(launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<true, true>, pair_grid(M->n), 0, pa));
      PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, W,
                  EpiPBiCGSafeBDots<true>{As, L, G, S, Y, R, M->slot(PS_V_RS), M->sc, pb_part},
                  C_DONE, P.kry32));
    } else {
      if (!P.vec32)
        PS_TRY(launch(M, A, PS_K_UPDATE, k_passA_pbicgsafe<true, false>, pair_grid(M->n), 0, pa));
      PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, W,
                  EpiPBiCGSafeBDots<false>{As, L, G, S, Y, R, M->slot(PS_V_RS), M->sc, pb_part},
                  C_DONE, P.kry32));
    }
    return PS_OK;
  }
  // replacement step (Algorithm 5): true values of q, w, r, l, g, s
  PS_TRY(iter_safe_dots(M, P, A, i));
  // (p, u held in FP32: u also widened into the scratch slot for the product)
  double *Uw = P.vec32 ? M->slot(kSlotTmp) : U;
  PouArgs po{R, S, T, Y, Pp, U, O, Uw, M->sc, M->ctl, M->n, next_rev(M)};
  po.chunk_sys = M->chunk_sys;
  PS_TRY(launch(M, A, PS_K_OTHER, P.vec32 ? k_pou32 : k_pou, pair_grid(M->n), 0, po));
  PS_TRY(spmv(M, A, PS_K_SPMV, O, EpiStore{Q}, C_DONE, P.kry32));   // q_i = A o_i
  PS_TRY(spmv(M, A, PS_K_SPMV, Uw, EpiStore{W}, C_DONE, P.kry32));  // w_i = A u_i
  TzyxArgs tz{O, W, R, U, S, Pp, T, Z, Y, X, M->sc, M->ctl, M->n, next_rev(M)};
  tz.chunk_sys = M->chunk_sys;
  PS_TRY(launch(M, A, PS_K_OTHER, P.vec32 ? k_tzyx32 : k_tzyx, pair_grid(M->n), 0, tz));
  PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, X, EpiResidual{Bv, R, nullptr}, C_DONE, P.res32));  // b - A x_{i+1}
  PS_TRY(spmv(M, A, PS_K_SPMV, T, EpiStore{L}, C_DONE, P.kry32));  // l_i = A t_i
  PS_TRY(spmv(M, A, PS_K_SPMV, Y, EpiStore{G}, C_DONE, P.kry32));  // g_{i+1} = A y_{i+1}
  PS_TRY(spmv(M, A, PS_K_SPMV, R, EpiStore{S}, C_DONE, P.kry32));  // s_{i+1} = A r_{i+1}
  return PS_OK;
}

int iter_ssbicgsafe2(ps_matrix *M, const Plan &P, int i) {
  hipStream_t A = P.A;
  double *X = M->slot(PS_V_X), *R = M->slot(PS_V_R), *S = M->slot(PS_V_S), *Y = M->slot(PS_V_Y),
         *T = M->slot(PS_V_T), *Pp = M->slot(PS_V_P), *U = M->slot(PS_V_U), *Z = M->slot(PS_V_Z);
  PS_TRY(spmv(M, A, PS_K_SPMV, R, EpiStore{S}, C_DONE, P.kry32));  // s_i = A r_i
  PS_TRY(iter_safe_dots(M, P, A, i));
  PouArgs po{R, S, T, Y, Pp, U, nullptr, nullptr, M->sc, M->ctl, M->n, next_rev(M)};
  po.chunk_sys = M->chunk_sys;
  PS_TRY(launch(M, A, PS_K_UPDATE, k_pu, pair_grid(M->n), 0, po));
  if (P.stream_nt)
    PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, U, EpiSsBiCGSafe2B<true>{S, U, Pp, T, Z, Y, X, R, M->sc},
                C_DONE, P.kry32));
  else
    PS_TRY(spmv(M, A, PS_K_SPMV_FUSED, U, EpiSsBiCGSafe2B<false>{S, U, Pp, T, Z, Y, X, R, M->sc},
                C_DONE, P.kry32));
  return PS_OK;
}

int iter_pbicgstab(ps_matrix *M, const Plan &P, int /*i*/) {
  hipStream_t A = P.A;
  double *X = M->slot(PS_V_X), *R = M->slot(PS_V_R), *RS = M->slot(PS_V_RS),
         *S = M->slot(PS_V_S), *Y = M->slot(PS_V_Y), *T = M->slot(PS_V_T), *Pp = M->slot(PS_V_P),
         *Z = M->slot(PS_V_Z), *W = M->slot(PS_V_W), *Q = M->slot(PS_V_Q), *V = M->slot(PS_V_V);
  Stab1Args s1{R, W, T, V, Pp, S, Z, Q, Y, M->sc, M->ctl, M->n, next_rev(M)};
  s1.chunk_sys = M->chunk_sys;
  if (P.fused3) {
    // one stream: each pass also forms the partial sums of the inner products of
    // the vectors it writes, and the product after it folds them and runs the
    // phase's finish (omega after pass 1; beta, alpha and the stop test after
    // pass 2).  The products keep their C_HALT stop word, so that a product whose
    // own prologue stops the solve still completes its rows, as before.
    double *p1 = M->fpart, *p2 = p1 + kPart * 4 * (size_t)M->ga;  // [4][ga], [3][ga]
    double *pf = M->fpart + kPart * (5 * (size_t)std::max(M->ga, M->nblk) + 4 * (size_t)M->nblk);
    const int gf = (M->ga + kBlock - 1) / kBlock;
    DotArgs D{};
    D.n = M->n;
    D.ctl = M->ctl;
    D.sc = M->sc;
    D.hist = M->hist;
    D.maxit = P.maxit;
    D.tol = P.tol;
    D.flags = 0;
    D.running = M->running();
    s1.rs = RS;
    s1.part = p1;
    PS_TRY(P.stream_nt ? launch(M, A, PS_K_UPDATE, k_stab_pass1<true, true>, pair_grid(M->n), 0, s1)
                       : launch(M, A, PS_K_UPDATE, k_stab_pass1<true, false>, pair_grid(M->n), 0,
                                s1));
    D.partials = pf;  // [2][gf]: (q, y), (y, y), rows 0 and 1 of pass 1's list
    const FoldLists l1{p1, p1, M->ga, M->ga, 0u, 0x10ull};
    PS_TRY(spmv(M, A, PS_K_SPMV, Z, EpiStoreFold<2, FinStabOmega>{V, l1, gf, D}, C_HALT,
                P.kry32));  // v_i = A z_i
    Stab2Args s2{Pp, Q, Y, T, V, X, R, W, M->sc, M->ctl, M->n, next_rev(M)};
    s2.rs = RS;
    s2.part = p2;
    PS_TRY(P.stream_nt ? launch(M, A, PS_K_UPDATE, k_stab_pass2<true, true>, pair_grid(M->n), 0, s2)
                       : launch(M, A, PS_K_UPDATE, k_stab_pass2<true, false>, pair_grid(M->n), 0,
                                s2));
    // [5][gf] in FinStabBetaAlpha's order: (r0*, r), (r0*, w) from pass 2's rows 0, 1;
    // (r0*, s), (r0*, z) from pass 1's rows 2, 3; (r, r) from pass 2's row 2
    D.partials = pf + kPart * 2 * (size_t)gf;
    const FoldLists l2{p2, p1, M->ga, M->ga, 0xCu, 0x23210ull};
    PS_TRY(spmv(M, A, PS_K_SPMV, W, EpiStoreFold<5, FinStabBetaAlpha>{T, l2, gf, D}, C_HALT,
                P.kry32));  // t_{i+1} = A w_{i+1}
    return PS_OK;
  }
  PS_TRY(P.stream_nt ? launch(M, A, PS_K_UPDATE, k_stab_pass1<false, true>, pair_grid(M->n), 0, s1)
                     : launch(M, A, PS_K_UPDATE, k_stab_pass1<false, false>, pair_grid(M->n), 0, s1));
  PS_TRY(fork(M, P));
  // each reduction phase enqueued ahead of the product it overlaps
  PS_TRY(dots<ProdStab2, FinStabOmega>(M, P.B, {Q, Y}, P.maxit, P.tol, 0, M->hist));
  PS_TRY(spmv(M, A, PS_K_SPMV, Z, EpiStore{V}, C_HALT, P.kry32));  // v_i = A z_i
  PS_TRY(join(M, P));
  Stab2Args s2{Pp, Q, Y, T, V, X, R, W, M->sc, M->ctl, M->n, next_rev(M)};
  s2.chunk_sys = M->chunk_sys;
  PS_TRY(P.stream_nt ? launch(M, A, PS_K_UPDATE, k_stab_pass2<false, true>, pair_grid(M->n), 0, s2)
                     : launch(M, A, PS_K_UPDATE, k_stab_pass2<false, false>, pair_grid(M->n), 0, s2));
  PS_TRY(fork(M, P));
  PS_TRY(dots<ProdStab5, FinStabBetaAlpha>(M, P.B, {RS, R, W, S, Z}, P.maxit, P.tol, 0,
                                           M->hist));
  PS_TRY(spmv(M, A, PS_K_SPMV, W, EpiStore{T}, C_HALT, P.kry32));  // t_{i+1} = A w_{i+1}
  PS_TRY(join(M, P));
  return PS_OK;
}

int enqueue_iteration(ps_matrix *M, const Plan &P, int i) {
  switch (P.variant) {
    case PS_SSBICGSAFE2: return iter_ssbicgsafe2(M, P, i);
    case PS_PBICGSTAB: return iter_pbicgstab(M, P, i);
    default: return iter_pbicgsafe(M, P, i);
  }
}

// An iteration whose launches are the same as every other such iteration's
// (all arguments fixed; the iteration index lives on the device): not the
// first iteration of the BiCGSafe forms, not a replacement step, and with a
// fused schedule not the iteration after one.
bool is_standard(const Plan &P, int i) {
  if (P.variant == PS_PBICGSTAB) return true;
  if (i == 0) return false;
  if (P.fused && i == P.i0) return false;  // its inner products come from their own pass
  if (replacement(P, i)) return false;
  if (P.fused && after_replacement(P, i)) return false;  // so do this one's
  return true;
}

void clear_graphs(ps_matrix *M) {
  for (GraphEntry &g : M->graphs) (void)hipGraphExecDestroy(g.exec);
  M->graphs.clear();
}

// The instantiated graph of `count` standard iterations that starts in the
// current sweep phase, captured from the launch sequence on first use.
int get_graph(ps_matrix *M, const Plan &P, int count, int probe_i, GraphEntry **out) {
  const GraphKey key{P.variant, P.maxit,   P.rr_m,           P.rr_M, P.overlap ? 1 : 0,
                     count,     M->sweep,
                     (P.fused ? 1 : 0) | (P.stream_nt ? 2 : 0) | (P.fused2 ? 4 : 0) |
                         (P.fused3 ? 8 : 0),
                     P.precision, P.tol,   P.A};
  for (GraphEntry &g : M->graphs)
    if (g.key == key) {
      *out = &g;
      return PS_OK;
    }
  const int phase = M->sweep;
  hipGraph_t graph = nullptr;
  PS_HIP(hipStreamBeginCapture(P.A, hipStreamCaptureModeThreadLocal));
  int rc = PS_OK;
  for (int k = 0; k < count && rc == PS_OK; ++k) rc = enqueue_iteration(M, P, probe_i);
  const hipError_t e = hipStreamEndCapture(P.A, &graph);
  const int flip = M->sweep ^ phase;
  M->sweep = phase;  // nothing ran yet
  if (rc != PS_OK || e != hipSuccess || graph == nullptr) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return PS_EHIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    (void)hipGetLastError();
    return PS_EHIP;
  }
  if (M->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(M->graphs.front().exec);
    M->graphs.erase(M->graphs.begin());
  }
  M->graphs.push_back(GraphEntry{key, exec, flip});
  *out = &M->graphs.back();
  return PS_OK;
}

// Iterations past this index are never needed: the finish at the last one stops.
int last_iteration(const Plan &P) { return P.variant == PS_PBICGSTAB ? P.maxit - 1 : P.maxit; }

// Iterations per host check (and per cached graph).  Measured: longer batches
// spread the graph launch and the check over more iterations, but the check
// runs one batch behind, so up to two batches of no-op iterations follow the
// stop; 16 was best for the 2M-row systems (~165 us per iteration), 8 for
// small ones (~25 us per iteration).
int auto_batch(const ps_matrix *M) {
  const double bytes = 24.0 * (double)M->nnz + 300.0 * (double)M->n;
  const double us = bytes / 5.0e6 + 20.0;  // rough time of one iteration
  return us >= 100.0 ? 16 : 8;
}

int ensure_hist(ps_matrix *M, int64_t need) {
  if (need <= M->hist_cap) return PS_OK;
  if (M->hist) {
    PS_HIP(hipDeviceSynchronize());
    clear_graphs(M);  // captured launches hold the old history pointer
    PS_HIP(hipFree(M->hist));
    M->hist = nullptr;
  }
  int64_t cap = std::max<int64_t>(need, 1024);
  PS_HIP(hipMalloc(&M->hist, cap * sizeof(double)));
  M->hist_cap = cap;
  return PS_OK;
}

// The matrix values rounded to FP32 (nearest, ties to even), made on the
// device from the FP64 values at the first mixed-precision solve and kept.
int ensure_f32(ps_matrix *M, hipStream_t s) {
  const bool csr = M->format == PS_FMT_CSR;
  float *&dst = csr ? M->val32 : M->sval32;
  if (dst) return PS_OK;
  const int64_t cnt = csr ? M->nnz : M->slots;
  PS_HIP(hipMalloc(&dst, std::max<int64_t>(cnt, 1) * sizeof(float)));
  if (cnt > 0)
    PS_TRY(launch(M, s, PS_K_OTHER, k_round_f32, elem_grid(cnt), 0,
                  (const double *)(csr ? M->val : M->sval), dst, cnt));
  return PS_OK;
}

// Sum the timed launches of iterations before the stop; launches of the
// stopping iteration and of iterations enqueued after it may be no-ops and are
// left out.
int collect_profile(ps_matrix *M, int stop_iter) {
  for (int c = 0; c < PS_K_COUNT; ++c) {
    M->prof_ms[c] = 0.0;
    M->prof_cnt[c] = 0;
    M->prof_aux[c] = 0;
  }
  for (const Timer &t : M->timers) {
    if (t.iter < 0 || t.iter >= stop_iter) continue;
    float ms = 0.f;
    PS_HIP(hipEventElapsedTime(&ms, t.a, t.b));
    M->prof_ms[t.cls] += ms;
    M->prof_cnt[t.cls] += 1;
    M->prof_aux[t.cls] += t.aux ? 1 : 0;
  }
  M->timers.clear();
  M->ev_used = 0;
  return PS_OK;
}

int64_t matrix_bytes(const ps_matrix *M) {
  return M->format == PS_FMT_CSR
             ? (8 + M->index_bits / 8 + (M->gather_sort ? 2 : 0)) * M->nnz + 4 * (M->n + 1)
             : (8 + M->index_bits / 8) * M->slots + 4 * ((int64_t)M->nslice + 1);
}
bool auto_overlap(const ps_matrix *M) { return matrix_bytes(M) + 16 * M->n >= kOverlapMinBytes; }
// The automatic p-BiCGSafe(-rr) schedule, from measurements with the triple
// inner-product accumulators (microseconds per iteration, schedules 0 / 2 / 3):
//  - one system, sliced layout: the single-stream fused epilogue (3) -- stencils
//    of 24^3 .. 128^3 rows: 24.6 / 19.8 / 18.4, 42.9 / 37.0 / 33.3 (64^3),
//    78.2 / 74.0 / 63.4 (96^3), 151.5 / 140.0 / 128.5 (128^3); schedule 2
//    beats 1 by 4-7% and 0 by 6-20%;
//  - one system, CSR: 3 below kFusedMinRows rows (banded 2*10^4 and 2*10^5
//    rows: 35.2 / 30.1 / 28.5 and 71.8 / 72.1 / 61.0), else the separate pass
//    (0; 10^6 uneven rows: 219 / 249 / 238 -- the gather-bound products gain
//    nothing from the skipped pass and pay for the extra epilogue reads);
//  - batches: 2 (the 512-system stencil batch: 17% more solves/s than 0, 4%
//    more than 1; schedule 3 is single-system only), or 4 (one workgroup per
//    system) on the sliced layout when no system has more than
//    kOneGroupBatchAutoRows rows (stencil batches, ms for 2 / 4: 512 systems
//    of 8^2..16^2 rows 1.58 / 0.57, 4096 of them 5.16 / 1.66; 512 of
//    24^2..32^2 4.11 / 2.25, 2048 10.37 / 7.52; 512 of 30^2..40^2 5.95 / 4.24;
//    of 40^2..64^2: 512 15.6 / 14.7, 1024 29.1 / 34.9, 2048 56.9 / 71.5);
//  - one sliced system of at most kOneGroupAutoRows rows: the whole solve in
//    one workgroup (4; 3 / 4, stencils, whose rows the workgroup keeps in
//    registers: 36 rows 15.3 / 5.1, 256 rows 16.1 / 5.7, 576 rows 17.6 / 10.0,
//    1024 rows 17.6 / 11.5; wider rows, read from memory every iteration: 1024
//    rows 17.7 / 17.4; 1296 rows 17.9 / 21.0, 4096 rows 17.9 / 43.3 -- a
//    single CU's bandwidth caps it beyond about a thousand rows).
//    p-BiCGSafe only: the other methods fall back to 3.
int auto_schedule(const ps_matrix *M) {
  if (M->nsys > 1)
    return M->format == PS_FMT_SELL && M->sell_rpl == 1 && M->max_sys_rows <= kOneGroupBatchAutoRows
               ? 4
               : 2;
  if (M->format == PS_FMT_SELL)
    return M->n <= kOneGroupAutoRows && M->sell_rpl == 1 ? 4 : 3;
  return M->n < kFusedMinRows ? 3 : 0;
}
// two sparse products and the update passes' 34 vector reads and writes
bool streaming(const ps_matrix *M, int32_t variant = PS_PBICGSAFE) {
  if (M->stream_override >= 0) return M->stream_override != 0;
  const bool safe = variant == PS_PBICGSAFE || variant == PS_PBICGSAFE_RR;
  return 2 * matrix_bytes(M) + 272 * M->n >= (safe ? kStreamMinBytes : kOtherStreamMinBytes);
}

// Put p, u, z in FP32 (to32) or FP64 storage, converting the slots that hold the
// other one (through the scratch slot).
int convert_pzu(ps_matrix *M, hipStream_t s, bool to32) {
  if (M->pzu32 == to32) return PS_OK;
  double *tmp = M->slot(kSlotTmp);
  for (int v : {PS_V_P, PS_V_U, PS_V_Z}) {
    double *x = M->slot(v);
    if (to32) {
      PS_TRY(launch(M, s, PS_K_OTHER, k_copy, elem_grid(M->n), 0, tmp, (const double *)x, M->n));
      PS_TRY(launch(M, s, PS_K_OTHER, k_narrow, elem_grid(M->n), 0, reinterpret_cast<float *>(x),
                    (const double *)tmp, M->n));
    } else {
      PS_TRY(launch(M, s, PS_K_OTHER, k_widen, elem_grid(M->n), 0, tmp,
                    reinterpret_cast<const float *>(x), M->n));
      PS_TRY(launch(M, s, PS_K_OTHER, k_copy, elem_grid(M->n), 0, x, (const double *)tmp, M->n));
    }
  }
  M->pzu32 = to32;
  return PS_OK;
}

// Where one solve's scalar and control blocks, inner-product partial sums and
// history lie in a workspace of `total` doubles (ps_solve_dev_static); every
// region starts on a 256-byte boundary.
struct WorkspaceLayout {
  size_t sc, ctl, partials, fpart, hist, total;
};
size_t round32(size_t v) { return (v + 31) / 32 * 32; }
WorkspaceLayout workspace_layout(const ps_matrix *M, int32_t maxit) {
  WorkspaceLayout L;
  size_t at = 0;
  L.sc = at;
  at += round32((size_t)M->nsys * SC_COUNT);
  L.ctl = at;
  at += round32((((size_t)M->nsys + 1) * C_COUNT * sizeof(int) + sizeof(double) - 1) / sizeof(double));
  L.partials = at;
  at += round32(kPart * 9 * ((size_t)M->dot_grid + dot_slices(M)));
  L.fpart = at;
  at += round32(kPart * (5 * (size_t)std::max(M->ga, M->nblk) + 4 * (size_t)M->nblk +
                         9 * (size_t)M->gfold));
  L.hist = at;
  at += round32((size_t)maxit + 2);
  L.total = at;
  return L;
}

// For the duration of one solve, the handle's scalar and control blocks,
// partial sums and history are those of a workspace (restored on return).
struct WorkspaceSwap {
  ps_matrix *M = nullptr;
  double *sc = nullptr, *partials = nullptr, *fpart = nullptr, *hist = nullptr;
  int *ctl = nullptr;
  int64_t hist_cap = 0;
  void apply(ps_matrix *M_, double *ws, const WorkspaceLayout &L) {
    M = M_;
    sc = M->sc;
    partials = M->partials;
    fpart = M->fpart;
    hist = M->hist;
    ctl = M->ctl;
    hist_cap = M->hist_cap;
    M->sc = ws + L.sc;
    M->ctl = reinterpret_cast<int *>(ws + L.ctl);
    M->partials = ws + L.partials;
    M->fpart = ws + L.fpart;
    M->hist = ws + L.hist;
    M->hist_cap = (int64_t)(L.total - L.hist);
  }
  ~WorkspaceSwap() {
    if (!M) return;
    M->sc = sc;
    M->ctl = ctl;
    M->partials = partials;
    M->fpart = fpart;
    M->hist = hist;
    M->hist_cap = hist_cap;
  }
};

// One solve of every system of the handle.  iters, status: int32[nsys];
// hist: NULL or double[nsys][maxit+1]; b, x0, x: double[n_orig] (the caller's
// row order), on the device or the host.  ws: NULL, or a device workspace laid
// out by workspace_layout that replaces the handle's own blocks for this solve
// (then nothing is allocated: no graphs, no profiling, no history growth).
// k_solve_one, one workgroup of nt threads (64, 128, 256 or 512) per system;
// k_solve_tiny when every system has at most 2 nt rows and no slice more than
// kTinySlots entries per row
template <class IT, int NT>
void launch_one_it(ps_matrix *M, hipStream_t s, const OneArgs &a) {
  const SellDev<double, IT> S = M->template sell<double, IT>();
  const bool tiny = M->sell_width <= kTinySlots;
  if (tiny && M->max_sys_rows <= NT)
    hipLaunchKernelGGL((k_solve_tiny<IT, NT, 1>), dim3(M->nsys), dim3(NT), 0, s, S, a);
  else if (tiny && M->max_sys_rows <= 2 * NT)
    hipLaunchKernelGGL((k_solve_tiny<IT, NT, 2>), dim3(M->nsys), dim3(NT), 0, s, S, a);
  else
    hipLaunchKernelGGL((k_solve_one<IT, NT>), dim3(M->nsys), dim3(NT), 0, s, S, a);
}
template <int NT>
int launch_one_nt(ps_matrix *M, hipStream_t s, const OneArgs &a) {
  if (M->index_bits == 16) launch_one_it<short, NT>(M, s, a);
  else launch_one_it<int, NT>(M, s, a);
  PS_HIP(hipGetLastError());
  return PS_OK;
}
int launch_one(ps_matrix *M, hipStream_t s, int nt, const OneArgs &a) {
  switch (nt) {
    case 64: return launch_one_nt<64>(M, s, a);
    case 128: return launch_one_nt<128>(M, s, a);
    case 256: return launch_one_nt<256>(M, s, a);
    case 512: return launch_one_nt<512>(M, s, a);
  }
  return PS_EINVAL;
}

// schedule 4 runs p-BiCGSafe in FP64 on the sliced layout (one row per lane),
// from x_0 (no resume), without profiling, on systems of at most
// kOneGroupMaxRows rows each
bool one_group_ok(const ps_matrix *M, int32_t variant, const ps_options &o) {
  return variant == PS_PBICGSAFE && M->format == PS_FMT_SELL && M->sell_rpl == 1 &&
         o.precision == PS_PREC_FP64 && !o.resume && !o.profile &&
         M->max_sys_rows <= kOneGroupMaxRows;
}

int solve_impl(ps_matrix *M, const double *b, const double *x0, bool on_device, double tol,
               int32_t maxit, int32_t variant, const ps_options *opt, double *x, int32_t *iters,
               double *hist, int32_t *status, double *ws = nullptr) {
  if (!M) return PS_EINVAL;
  if (variant < PS_SSBICGSAFE2 || variant > PS_PBICGSTAB) return PS_EINVAL;
  if (maxit < 0 || !(tol >= 0.0) || !iters || !status || !x) return PS_EINVAL;
  ps_options o;
  ps_default_options(&o);
  if (opt) o = *opt;
  const bool batch = M->nsys > 1;
  if (!o.resume && !b) return PS_EINVAL;
  if (o.norm_ref != 0 && o.norm_ref != 1) return PS_EINVAL;
  if (o.x0_fallback < 0 || o.x0_fallback > 2) return PS_EINVAL;
  if (o.resume && (batch || o.resume_iter < 0 || o.resume_iter > maxit)) return PS_EINVAL;
  const bool safe_pipelined = variant == PS_PBICGSAFE || variant == PS_PBICGSAFE_RR;
  // schedule 3 folds in the product's first gfold workgroups: never more than the
  // product has with the layouts built here (gfold = nblk / 256, rounded up)
  if (o.schedule < -1 || o.schedule > 4 ||
      (o.schedule >= 1 && !safe_pipelined && !(o.schedule == 3 && variant == PS_PBICGSTAB)) ||
      (o.schedule == 3 && (batch || M->gfold > M->nblk)) ||
      (o.schedule == 4 && !one_group_ok(M, variant, o)))
    return PS_EINVAL;
  if (o.precision < PS_PREC_FP64 || o.precision > PS_PREC_FP32_VECTORS ||
      (o.precision != PS_PREC_FP64 && !M->f32_ok) ||
      (o.precision == PS_PREC_FP32_VECTORS && !safe_pipelined))
    return PS_EINVAL;
  if (ws && (batch || o.resume || o.profile || o.graph)) return PS_EINVAL;
  BusyGuard guard(M->busy);
  if (!guard.ok) return PS_EBUSY;
  PS_HIP(hipSetDevice(M->device));
  WorkspaceSwap swap;
  if (ws) swap.apply(M, ws, workspace_layout(M, maxit));

  Plan P;
  P.variant = variant;
  P.maxit = maxit;
  P.tol = tol;
  P.rr_m = o.rr_m;
  P.rr_M = o.rr_M > 0 ? o.rr_M : maxit;
  P.norm_ref = o.norm_ref;
  P.resume = o.resume != 0;
  P.i0 = P.resume ? o.resume_iter : 0;
  // device-buffer solves follow the caller's stream (NULL = the null stream, which
  // orders them after the caller's pending work); host-buffer solves default to
  // the library's own stream
  P.A = (on_device || o.stream) ? (hipStream_t)o.stream : M->own;
  bool use_graph = o.graph != 0 && o.profile == 0;
  if (use_graph && P.A == nullptr) {
    // the null stream cannot be captured: run on the library's stream, after
    // the work already queued on the null stream
    PS_HIP(hipEventRecord(M->ev_fork, nullptr));
    PS_HIP(hipStreamWaitEvent(M->own, M->ev_fork, 0));
    P.A = M->own;
  }
  // a second stream pays only when the product it hides behind is long
  const bool want_overlap = o.overlap > 0 || (o.overlap < 0 && auto_overlap(M));
  P.overlap = want_overlap && variant != PS_SSBICGSAFE2;
  P.B = P.overlap ? M->aux : P.A;
  P.fallback = o.x0_fallback != 0 && x0 != nullptr && !P.resume;
  P.scale = o.x0_fallback == 2 && x0 != nullptr && !P.resume;
  int sched = o.schedule >= 0 ? o.schedule : auto_schedule(M);
  if (sched == 4 && !one_group_ok(M, variant, o)) sched = batch ? 2 : 3;  // automatic
  P.one = sched == 4;
  P.fused = safe_pipelined && sched >= 1;
  P.fused2 = P.fused && sched >= 2;
  // p-BiCGStab: schedule 3 or the separate passes; automatically 3 for one system
  // (microseconds per iteration, 0 / 3: 128^3 stencil 166.7 / 148.9, 96^3 77.8 /
  // 61.7, 2*10^5-row band 74.7 / 59.8, 10^6-row band 243.8 / 229.2)
  const bool stab3 = o.schedule == 3 || (o.schedule < 0 && !batch);
  P.fused3 = variant == PS_PBICGSTAB ? stab3 : sched == 3 && safe_pipelined;
  P.stream_nt = streaming(M, variant);
  P.precision = o.precision;
  P.kry32 = o.precision != PS_PREC_FP64;
  P.res32 = o.precision == PS_PREC_FP32_MATRIX;
  P.vec32 = o.precision == PS_PREC_FP32_VECTORS;
  M->prof_mask = o.profile;
  M->cur_iter = -1;
  M->sweep = 0;
  M->timers.clear();
  M->ev_used = 0;
  if (P.kry32) PS_TRY(ensure_f32(M, P.A));
  // the storage of p, u, z: a resumed solve converts the loaded state; a fresh
  // set-up zeroes them (zero bits are zero in either type)
  if (P.resume) PS_TRY(convert_pzu(M, P.A, P.vec32));
  M->pzu32 = P.vec32;
  M->hist_stride = (int64_t)maxit + 2;
  PS_TRY(ensure_hist(M, M->hist_stride * M->nsys));

  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (ws)  // a workspace holds the previous call's scalars: start from zero
    PS_TRY(launch(M, P.A, PS_K_OTHER, k_zero, elem_grid((int64_t)M->nsys * SC_COUNT), 0, M->sc,
                  (int64_t)0, 1, (int64_t)M->nsys * SC_COUNT));
  PS_TRY(launch(M, P.A, PS_K_OTHER, k_init_ctl, elem_grid((int64_t)M->nsys * C_COUNT + 1), 0,
                M->ctl, P.i0, M->nsys));
  if (!P.resume) {
    if (!batch) {
      const size_t vbytes = (size_t)M->n * sizeof(double);
      PS_HIP(hipMemcpyAsync(M->slot(PS_V_B), b, vbytes, kind, P.A));
      if (x0) PS_HIP(hipMemcpyAsync(M->slot(PS_V_X), x0, vbytes, kind, P.A));
      else PS_TRY(zero_slots(M, P.A, {PS_V_X}));
    } else {
      // padded rows keep b = x = 0 (empty rows: they stay zero in every vector)
      PS_TRY(zero_slots(M, P.A, {PS_V_B, PS_V_X}));
      const size_t obytes = (size_t)M->n_orig * sizeof(double);
      const double *src = b;
      if (!on_device) {
        PS_HIP(hipMemcpyAsync(M->stage, b, obytes, hipMemcpyHostToDevice, P.A));
        src = M->stage;
      }
      PS_TRY(launch(M, P.A, PS_K_OTHER, k_scatter, elem_grid(M->n_orig), 0, M->slot(PS_V_B), src,
                    (const int *)M->row_map, M->n_orig));
      if (x0) {
        src = x0;
        if (!on_device) {
          PS_HIP(hipMemcpyAsync(M->stage, x0, obytes, hipMemcpyHostToDevice, P.A));
          src = M->stage;
        }
        PS_TRY(launch(M, P.A, PS_K_OTHER, k_scatter, elem_grid(M->n_orig), 0, M->slot(PS_V_X),
                      src, (const int *)M->row_map, M->n_orig));
      }
    }
    PS_TRY(enqueue_setup(M, P));
  }

  const int last = last_iteration(P);
  const int K = o.batch_iters > 0 ? o.batch_iters : auto_batch(M);
  int nbatch = 0;
  bool stopped = false;
  if (P.one) {
    // one workgroup per system
    OneArgs a{M->slot(PS_V_X), M->slot(PS_V_R), M->slot(PS_V_S), M->slot(PS_V_Y),
              M->slot(PS_V_T), M->slot(PS_V_P), M->slot(PS_V_U), M->slot(PS_V_Z),
              M->slot(PS_V_W), M->slot(PS_V_L), M->slot(PS_V_G), M->slot(PS_V_AS),
              M->slot(PS_V_RS), M->sc, M->ctl, M->hist, M->hist_stride, M->running(),
              M->nsys > 1 ? M->first_blk : nullptr, M->nsys > 1 ? M->sys_end : nullptr,
              (int)M->n, P.maxit, P.tol, P.norm_ref == 0 ? DF_SET_REF : 0};
    // (never profiled, so launched directly, with its own block size).  The
    // workgroup: 512 threads, fewer when the systems have fewer rows or when so
    // many systems run that smaller workgroups let more of them be resident at
    // once; 64 at the least
    int nt = kOneGroupThreads;
    while (nt > 64 && (nt / 2 >= M->max_sys_rows || (int64_t)M->nsys * nt > kOneGroupResident))
      nt /= 2;
    PS_TRY(launch_one(M, P.A, nt, a));
    stopped = true;  // the loop below has nothing left to launch
  }
  for (int i = P.i0; i <= last && !stopped;) {
    const int end = std::min(last, i + K - 1);
    bool launched = false;
    if (use_graph && end - i + 1 == K) {
      bool uniform = true;
      for (int j = i; j <= end; ++j) uniform = uniform && is_standard(P, j);
      GraphEntry *g = nullptr;
      if (uniform && get_graph(M, P, K, i, &g) == PS_OK) {
        PS_HIP(hipGraphLaunch(g->exec, P.A));
        M->sweep ^= g->sweep_flip;
        i = end + 1;
        launched = true;
      } else if (uniform) {
        use_graph = false;  // capture not possible here: launch directly from now on
      }
    }
    if (!launched) {
      for (; i <= end; ++i) {
        M->cur_iter = i;
        PS_TRY(enqueue_iteration(M, P, i));
      }
    }
    PS_HIP(hipGetLastError());
    // the count of systems still running, read one batch behind
    const int cur = nbatch & 1;
    PS_HIP(hipMemcpyAsync(M->pinned + cur * C_COUNT, M->running(), sizeof(int),
                          hipMemcpyDeviceToHost, P.A));
    PS_HIP(hipEventRecord(M->ev_batch[cur], P.A));
    if (nbatch > 0) {
      PS_HIP(hipEventSynchronize(M->ev_batch[cur ^ 1]));
      if (M->pinned[(cur ^ 1) * C_COUNT] == 0) stopped = true;
    }
    ++nbatch;
  }
  PS_HIP(hipStreamSynchronize(P.A));
  if (P.overlap) PS_HIP(hipStreamSynchronize(P.B));

  // the control blocks (one system: on the stack, so that a solve into a
  // workspace allocates nothing)
  int c_one[C_COUNT];
  std::vector<int> c_many;
  int *c = c_one;
  if (M->nsys > 1) {
    c_many.resize((size_t)M->nsys * C_COUNT);
    c = c_many.data();
  }
  PS_HIP(hipMemcpy(c, M->ctl, (size_t)M->nsys * C_COUNT * sizeof(int), hipMemcpyDeviceToHost));
  int it_max = 0;
  for (int k = 0; k < M->nsys; ++k) {
    const int *ck = c + (size_t)k * C_COUNT;
    int st = ck[C_STATUS], it = ck[C_ITERS];
    if (!ck[C_DONE]) {  // cannot happen: the finish at the last iteration always stops
      st = PS_MAXIT;
      it = maxit;
    }
    iters[k] = it;
    status[k] = st;
    it_max = std::max(it_max, it);
  }
  if (hist) {
    if (!batch) {
      PS_HIP(hipMemcpy(hist, M->hist, (size_t)(iters[0] + 1) * sizeof(double),
                       hipMemcpyDeviceToHost));
    } else {
      PS_HIP(hipMemcpy2D(hist, (size_t)(maxit + 1) * sizeof(double), M->hist,
                         (size_t)M->hist_stride * sizeof(double), (size_t)(maxit + 1) * sizeof(double),
                         (size_t)M->nsys, hipMemcpyDeviceToHost));
    }
  }
  if (!batch) {
    PS_HIP(hipMemcpy(x, M->slot(PS_V_X), (size_t)M->n * sizeof(double),
                     on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  } else {
    double *dst = on_device ? x : M->stage;
    hipLaunchKernelGGL(k_gather, elem_grid(M->n_orig), dim3(kBlock), 0, P.A, dst,
                       (const double *)M->slot(PS_V_X), (const int *)M->row_map, M->n_orig);
    PS_HIP(hipGetLastError());
    PS_HIP(hipStreamSynchronize(P.A));
    if (!on_device)
      PS_HIP(hipMemcpy(x, M->stage, (size_t)M->n_orig * sizeof(double), hipMemcpyDeviceToHost));
  }
  if (M->prof_mask) PS_TRY(collect_profile(M, it_max));
  return PS_OK;
}

void free_matrix(ps_matrix *M) {
  if (!M) return;
  if (M->device >= 0) (void)hipSetDevice(M->device);
  (void)hipDeviceSynchronize();
  clear_graphs(M);
  (void)hipFree(M->rowptr);
  (void)hipFree(M->col);
  (void)hipFree(M->col16);
  (void)hipFree(M->pos);
  (void)hipFree(M->val);
  (void)hipFree(M->blk);
  (void)hipFree(M->rord);
  (void)hipFree(M->scol);
  (void)hipFree(M->scol16);
  (void)hipFree(M->sval);
  (void)hipFree(M->val32);
  (void)hipFree(M->sval32);
  (void)hipFree(M->soff);
  (void)hipFree(M->vec);
  (void)hipFree(M->sc);
  (void)hipFree(M->ctl);
  (void)hipFree(M->partials);
  (void)hipFree(M->fpart);
  (void)hipFree(M->chunk_sys);
  (void)hipFree(M->first_blk);
  (void)hipFree(M->first_pblk);
  (void)hipFree(M->sys_end);
  (void)hipFree(M->row_map);
  (void)hipFree(M->stage);
  (void)hipFree(M->bpart);
  (void)hipFree(M->hist);
  if (M->pinned) (void)hipHostFree(M->pinned);
  for (hipEvent_t e : M->ev_pool) (void)hipEventDestroy(e);
  if (M->ev_fork) (void)hipEventDestroy(M->ev_fork);
  if (M->ev_join) (void)hipEventDestroy(M->ev_join);
  for (hipEvent_t e : M->ev_batch)
    if (e) (void)hipEventDestroy(e);
  if (M->own) (void)hipStreamDestroy(M->own);
  if (M->aux) (void)hipStreamDestroy(M->aux);
  delete M;
}

// Host description of a batch: the systems padded to 512-row multiples
// (layout.hpp).
using BatchLayout = psl::BatchPadding;
static_assert(psl::kRowsPerBlock == kBlock && psl::kSliceRows == kWave &&
                  psl::kPad16 == kSellPad16 && psl::kBatchAlign == 2 * kBlock,
              "host layouts and kernels must agree");

// CSR checks shared by the create entry points
bool valid_csr(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                      const double *val) {
  if (n < 1 || n >= INT32_MAX - 1 || nnz < 0 || nnz >= INT32_MAX || !rowptr) return false;
  if (nnz > 0 && (!col || !val)) return false;
  if (rowptr[0] != 0 || rowptr[n] != nnz) return false;
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return false;
  for (int64_t k = 0; k < nnz; ++k)
    if (col[k] < 0 || col[k] >= n || !std::isfinite(val[k])) return false;
  return true;
}

int create_impl(ps_matrix **out, int64_t n, int64_t nnz, const int64_t *rowptr,
                const int32_t *col, const double *val, const BatchLayout *bl,
                const ps_layout *lay);

// every field -1 (automatic) or a value the field allows
bool valid_layout(const ps_layout *l) {
  if (!l) return true;
  return (l->format == -1 || l->format == PS_FMT_CSR || l->format == PS_FMT_SELL) &&
         (l->sell_rows_per_lane == -1 || l->sell_rows_per_lane == 1 ||
          l->sell_rows_per_lane == 2) &&
         (l->spmv_shape >= -1 && l->spmv_shape <= 4) &&
         (l->index_bits == -1 || l->index_bits == 16 || l->index_bits == 32) &&
         (l->gather_sort >= -1 && l->gather_sort <= 1);
}

int create_batch_impl(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n,
                      int64_t nnz, const int64_t *rowptr, const int32_t *col, const double *val,
                      const ps_layout *lay);

}  // namespace

// ======================================================================= C ABI

extern "C" {

void ps_default_options(ps_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->rr_m = 100;
  opt->rr_M = 0;
  opt->norm_ref = 0;
  opt->batch_iters = 0;
  opt->overlap = -1;
  opt->profile = 0;
  opt->resume = 0;
  opt->resume_iter = 0;
  opt->graph = 1;
  opt->schedule = -1;
  opt->x0_fallback = 0;
  opt->precision = PS_PREC_FP64;
  opt->stream = nullptr;
}

int ps_create(ps_matrix **out, int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
              const double *val) {
  return ps_create_ex(out, n, nnz, rowptr, col, val, nullptr);
}

int ps_create_ex(ps_matrix **out, int64_t n, int64_t nnz, const int64_t *rowptr,
                 const int32_t *col, const double *val, const ps_layout *layout) {
  if (!out) return PS_EINVAL;
  *out = nullptr;
  if (!valid_csr(n, nnz, rowptr, col, val) || !valid_layout(layout)) return PS_EINVAL;
  return create_impl(out, n, nnz, rowptr, col, val, nullptr, layout);
}

int ps_create_batch(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n, int64_t nnz,
                    const int64_t *rowptr, const int32_t *col, const double *val) {
  return create_batch_impl(out, nsys, sys_ptr, n, nnz, rowptr, col, val, nullptr);
}

int ps_create_batch_ex(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n,
                       int64_t nnz, const int64_t *rowptr, const int32_t *col, const double *val,
                       const ps_layout *layout) {
  return create_batch_impl(out, nsys, sys_ptr, n, nnz, rowptr, col, val, layout);
}

}  // extern "C"

namespace {

int create_batch_impl(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n,
                      int64_t nnz, const int64_t *rowptr, const int32_t *col, const double *val,
                      const ps_layout *lay) {
  if (!out) return PS_EINVAL;
  *out = nullptr;
  if (nsys < 1 || !sys_ptr || !valid_csr(n, nnz, rowptr, col, val) || !valid_layout(lay))
    return PS_EINVAL;
  if (sys_ptr[0] != 0 || sys_ptr[nsys] != n) return PS_EINVAL;
  for (int32_t k = 0; k < nsys; ++k)
    if (sys_ptr[k + 1] <= sys_ptr[k]) return PS_EINVAL;
  // every row of a system references columns of that system only
  for (int32_t k = 0; k < nsys; ++k)
    for (int64_t r = sys_ptr[k]; r < sys_ptr[k + 1]; ++r)
      for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
        if (col[e] < sys_ptr[k] || col[e] >= sys_ptr[k + 1]) return PS_EINVAL;
  if (nsys == 1) return create_impl(out, n, nnz, rowptr, col, val, nullptr, lay);
  // pad each system to a multiple of 512 rows with empty rows
  BatchLayout bl;
  if (!psl::pad_batch(nsys, sys_ptr, n, rowptr, col, bl)) return PS_EINVAL;
  return create_impl(out, bl.n_pad, nnz, bl.rowptr.data(), bl.col.data(), val, &bl, lay);
}

int create_impl(ps_matrix **out, int64_t n, int64_t nnz, const int64_t *rowptr,
                const int32_t *col, const double *val, const BatchLayout *bl,
                const ps_layout *lay) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return PS_ENODEV;
  int dev = 0;
  PS_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  PS_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PS_ENODEV;

  ps_matrix *M = new ps_matrix();
  M->device = dev;
  M->n = n;
  M->nnz = nnz;
  for (int64_t k = 0; k < nnz && M->f32_ok; ++k) M->f32_ok = std::isfinite((float)val[k]);
  // SpMV shape from the mean row length: short rows one lane each with the
  // smallest per-thread budget that holds kBlock average rows; longer rows get
  // 4, 8 or 16 lanes each (4 up to a mean of 40: measured best on power-law
  // band matrices with means 18-31, equal to 8 lanes at 40)
  const double mean = (double)nnz / (double)n;
  M->shape = mean * 1.1 <= 4.0 ? 0 : (mean * 1.1 <= 8.0 ? 1 : (mean <= 40.0 ? 2 : (mean <= 64.0 ? 3 : 4)));
  if (const char *e = std::getenv("PIPESAFE_SPMV_SHAPE")) {  // tuning override
    const int v = std::atoi(e);
    if (v >= 0 && v <= 4) M->shape = v;
  }
  if (lay && lay->spmv_shape >= 0) M->shape = lay->spmv_shape;
  static const int kIpt[] = {4, 8, 16, 16, 16};
  // sliced ELLPACK when padding every slice to its longest row costs little
  M->sell_rpl = kSellRowsPerLane;
  if (const char *e = std::getenv("PIPESAFE_SELL_RPL")) {  // tuning override
    const int v = std::atoi(e);
    if (v == 1 || v == 2) M->sell_rpl = v;
  }
  if (lay && lay->sell_rows_per_lane > 0) M->sell_rpl = lay->sell_rows_per_lane;
  const int64_t SH = (int64_t)kWave * M->sell_rpl;  // rows per slice
  const int64_t slots = psl::sell_slots(n, rowptr, M->sell_rpl);
  int64_t sys_rows = n;  // rows of the largest system
  if (bl) {
    sys_rows = 0;
    for (int k = 0; k < bl->nsys; ++k)
      sys_rows = std::max<int64_t>(sys_rows, bl->sys_end[k] - bl->pstart[k]);
  }
  const bool one_group = M->sell_rpl == 1 && sys_rows <= (bl ? kOneGroupBatchAutoRows : kOneGroupAutoRows);
  const double max_pad = one_group ? kSellMaxPaddingSmall : kSellMaxPadding;
  M->format = (double)slots <= max_pad * (double)nnz + SH ? PS_FMT_SELL : PS_FMT_CSR;
  if (const char *e = std::getenv("PIPESAFE_FORMAT")) {  // tuning override
    const int v = std::atoi(e);
    if (v == PS_FMT_CSR || v == PS_FMT_SELL) M->format = v;
  }
  if (lay && lay->format >= 0) M->format = lay->format;
  if (slots >= INT32_MAX) M->format = PS_FMT_CSR;
  // 16-bit column offsets where every entry fits (unless 32-bit columns are asked for)
  bool want16 = true;
  if (const char *e = std::getenv("PIPESAFE_INDEX")) {  // tuning override: 32
    if (std::atoi(e) == 32) want16 = false;
  }
  if (lay && lay->index_bits == 32) want16 = false;
  psl::CsrLayout C;   // the layout's host arrays (layout.hpp)
  psl::SellLayout SL;
  if (M->format == PS_FMT_CSR) {
    const int budget = kIpt[M->shape] * kBlock;
    const std::vector<int64_t> cuts =
        bl ? std::vector<int64_t>(bl->pstart.begin() + 1, bl->pstart.end()) : std::vector<int64_t>();
    // multi-lane shapes sum each block's rows longest first (stable) when the
    // rows are uneven (longest above twice the mean): power-law band rows
    // 7-13% faster per product, uniform rows 3% slower (the extra index load)
    int64_t maxlen = 0;
    for (int64_t i = 0; i < n; ++i) maxlen = std::max<int64_t>(maxlen, rowptr[i + 1] - rowptr[i]);
    bool order = M->shape >= 2 && (double)maxlen > 2.0 * mean;
    if (const char *e = std::getenv("PIPESAFE_CSR_ORDER")) order = order && std::atoi(e) != 0;
    // gather order: each short-row block's entries sorted by column (stable),
    // when a typical block's columns span more than the L1 holds of x (4096
    // doubles): a wave's gathers then touch a few cache lines instead of up to 64
    // (1M-row band, +-5000: product 120 -> 100 us; a +-250 band, whose gathers
    // already hit L1, 87 -> 97 us, hence the condition)
    bool gsort = psl::csr_wide_blocks(psl::row_blocks(n, rowptr, budget, cuts), rowptr, col,
                                      budget, 4096);
    if (const char *e = std::getenv("PIPESAFE_CSR_SORT")) gsort = std::atoi(e) != 0;
    if (lay && lay->gather_sort >= 0) gsort = lay->gather_sort != 0;
    psl::build_csr(n, rowptr, col, val, budget, cuts, order, gsort, want16, C);
    M->nblk = (int)C.blk.size() - 1;
    M->gather_sort = gsort;
    M->index_bits = C.index_bits;
  } else {
    psl::build_sell(n, rowptr, col, val, M->sell_rpl, want16, SL);
    M->nslice = (int)SL.nslice;
    M->slots = SL.slots;
    M->nblk = (int)((n + kBlock * M->sell_rpl - 1) / (kBlock * M->sell_rpl));
    M->index_bits = SL.index_bits;
  }
  const std::vector<int> &blk = C.blk, &rp32 = C.rowptr, &scol = SL.col, &soff = SL.off;
  const std::vector<unsigned char> &rord = C.rord;
  const std::vector<unsigned short> &gpos = C.pos;
  const std::vector<short> &col16 = C.col16, &scol16 = SL.col16;
  const std::vector<double> &sval = SL.val;
  const int32_t *ccol = C.col;  // the CSR arrays as uploaded
  const double *cval = C.val;
  M->ld = ((size_t)n + 31) / 32 * 32;
  // batches: each system's first sparse-product workgroup (blocks never cross
  // systems: the sliced layout's 256*RPL rows divide the 512-row padding, and
  // CSR row blocks are cut at every system start)
  std::vector<int> pfirst;
  if (bl) {
    pfirst.resize((size_t)bl->nsys + 1);
    for (int k = 0; k <= bl->nsys; ++k) {
      const int64_t r = bl->pstart[k];
      if (M->format == PS_FMT_SELL) {
        pfirst[k] = (int)(r / ((int64_t)kBlock * M->sell_rpl));
      } else {
        pfirst[k] = (int)(std::lower_bound(blk.begin(), blk.end(), (int)r) - blk.begin());
      }
    }
  }
  int max_dot_grid = kMaxDotGrid;
  if (const char *e = std::getenv("PIPESAFE_DOT_GRID")) {  // tuning override
    const int v = std::atoi(e);
    if (v >= 1 && v <= 8192) max_dot_grid = v;
  }
  M->dot_grid = (int)std::max<int64_t>(1, std::min<int64_t>(max_dot_grid, (n / 2 + kBlock - 1) / kBlock));
  if (const char *e = std::getenv("PIPESAFE_STREAM")) {  // tuning override: 0 or 1
    if (e[0] == '0' || e[0] == '1') M->stream_override = e[0] - '0';
  }

  auto fail = [&](int code) {
    free_matrix(M);
    return code;
  };
#define PS_CREATE_HIP(call)                 \
  do {                                      \
    if ((call) != hipSuccess) return fail(PS_ENOMEM); \
  } while (0)
  if (M->format == PS_FMT_CSR) {
    PS_CREATE_HIP(hipMalloc(&M->rowptr, (n + 1) * sizeof(int)));
    if (!gpos.empty())
      PS_CREATE_HIP(hipMalloc(&M->pos, gpos.size() * sizeof(unsigned short)));
    if (M->index_bits == 16)
      PS_CREATE_HIP(hipMalloc(&M->col16, std::max<int64_t>(nnz, 1) * sizeof(short)));
    else
      PS_CREATE_HIP(hipMalloc(&M->col, std::max<int64_t>(nnz, 1) * sizeof(int)));
    PS_CREATE_HIP(hipMalloc(&M->val, std::max<int64_t>(nnz, 1) * sizeof(double)));
    PS_CREATE_HIP(hipMalloc(&M->blk, blk.size() * sizeof(int)));
    if (!rord.empty()) PS_CREATE_HIP(hipMalloc(&M->rord, rord.size()));
  } else {
    if (M->index_bits == 16)
      PS_CREATE_HIP(hipMalloc(&M->scol16, std::max<int64_t>(slots, 1) * sizeof(short)));
    else
      PS_CREATE_HIP(hipMalloc(&M->scol, std::max<int64_t>(slots, 1) * sizeof(int)));
    PS_CREATE_HIP(hipMalloc(&M->sval, std::max<int64_t>(slots, 1) * sizeof(double)));
    PS_CREATE_HIP(hipMalloc(&M->soff, soff.size() * sizeof(int)));
    for (size_t q = 0; q + 1 < soff.size(); ++q)
      M->sell_width = std::max(M->sell_width, (soff[q + 1] - soff[q]) / (kWave * M->sell_rpl));
  }
  PS_CREATE_HIP(hipMalloc(&M->vec, (size_t)kNumSlots * M->ld * sizeof(double)));
  const int nsys = bl ? bl->nsys : 1;
  M->nsys = nsys;
  M->n_orig = bl ? bl->n_orig : n;
  M->max_sys_rows = n;
  if (bl) {
    M->max_sys_rows = 0;
    for (int k = 0; k < nsys; ++k)
      M->max_sys_rows = std::max<int64_t>(M->max_sys_rows,
                                          bl->sys_end[k] - 512 * (int64_t)bl->first_blk[k]);
  }
  PS_CREATE_HIP(hipMalloc(&M->sc, (size_t)nsys * SC_COUNT * sizeof(double)));
  PS_CREATE_HIP(hipMalloc(&M->ctl, ((size_t)nsys + 1) * C_COUNT * sizeof(int)));
  if (bl) {
    PS_CREATE_HIP(hipMalloc(&M->chunk_sys, bl->chunk_sys.size() * sizeof(int)));
    PS_CREATE_HIP(hipMalloc(&M->first_blk, bl->first_blk.size() * sizeof(int)));
    PS_CREATE_HIP(hipMalloc(&M->first_pblk, pfirst.size() * sizeof(int)));
    PS_CREATE_HIP(hipMalloc(&M->sys_end, bl->sys_end.size() * sizeof(int)));
    PS_CREATE_HIP(hipMalloc(&M->row_map, bl->row_map.size() * sizeof(int)));
    PS_CREATE_HIP(hipMalloc(&M->stage, (size_t)bl->n_orig * sizeof(double)));
    PS_CREATE_HIP(hipMalloc(&M->bpart, kPart * 9 * (size_t)(n / 512) * sizeof(double)));
  }
  PS_CREATE_HIP(hipMalloc(&M->partials,
                          kPart * 9 * ((size_t)M->dot_grid + dot_slices(M)) * sizeof(double)));
  M->ga = (int)pair_grid(n).x;
  M->gfold = (std::max(M->ga, M->nblk) + kFoldPerThread * kBlock - 1) / (kFoldPerThread * kBlock);
  PS_CREATE_HIP(hipMalloc(&M->fpart, kPart * (5 * (size_t)std::max(M->ga, M->nblk) +
                                          4 * (size_t)M->nblk + 9 * (size_t)M->gfold) *
                                         sizeof(double)));
  PS_CREATE_HIP(hipHostMalloc(&M->pinned, 2 * C_COUNT * sizeof(int), hipHostMallocDefault));
#undef PS_CREATE_HIP
  auto chk = [&](hipError_t e) { return e == hipSuccess; };
  const bool csr = M->format == PS_FMT_CSR;
  if ((csr && !chk(hipMemcpy(M->rowptr, rp32.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice))) ||
      (csr && nnz > 0 && M->index_bits == 32 &&
       !chk(hipMemcpy(M->col, ccol, nnz * sizeof(int), hipMemcpyHostToDevice))) ||
      (csr && !gpos.empty() &&
       !chk(hipMemcpy(M->pos, gpos.data(), gpos.size() * sizeof(unsigned short),
                      hipMemcpyHostToDevice))) ||
      (csr && nnz > 0 && M->index_bits == 16 &&
       !chk(hipMemcpy(M->col16, col16.data(), nnz * sizeof(short), hipMemcpyHostToDevice))) ||
      (csr && nnz > 0 && !chk(hipMemcpy(M->val, cval, nnz * sizeof(double), hipMemcpyHostToDevice))) ||
      (csr && !chk(hipMemcpy(M->blk, blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice))) ||
      (csr && !rord.empty() &&
       !chk(hipMemcpy(M->rord, rord.data(), rord.size(), hipMemcpyHostToDevice))) ||
      (!csr && slots > 0 && M->index_bits == 32 &&
       !chk(hipMemcpy(M->scol, scol.data(), slots * sizeof(int), hipMemcpyHostToDevice))) ||
      (!csr && slots > 0 && M->index_bits == 16 &&
       !chk(hipMemcpy(M->scol16, scol16.data(), slots * sizeof(short), hipMemcpyHostToDevice))) ||
      (!csr && slots > 0 && !chk(hipMemcpy(M->sval, sval.data(), slots * sizeof(double), hipMemcpyHostToDevice))) ||
      (!csr && !chk(hipMemcpy(M->soff, soff.data(), soff.size() * sizeof(int), hipMemcpyHostToDevice))) ||
      !chk(hipMemset(M->vec, 0, (size_t)kNumSlots * M->ld * sizeof(double))) ||
      !chk(hipMemset(M->sc, 0, (size_t)nsys * SC_COUNT * sizeof(double))) ||
      !chk(hipMemset(M->ctl, 0, ((size_t)nsys + 1) * C_COUNT * sizeof(int))) ||
      (bl && !chk(hipMemcpy(M->chunk_sys, bl->chunk_sys.data(), bl->chunk_sys.size() * sizeof(int),
                            hipMemcpyHostToDevice))) ||
      (bl && !chk(hipMemcpy(M->first_blk, bl->first_blk.data(), bl->first_blk.size() * sizeof(int),
                            hipMemcpyHostToDevice))) ||
      (bl && !chk(hipMemcpy(M->first_pblk, pfirst.data(), pfirst.size() * sizeof(int),
                            hipMemcpyHostToDevice))) ||
      (bl && !chk(hipMemcpy(M->sys_end, bl->sys_end.data(), bl->sys_end.size() * sizeof(int),
                            hipMemcpyHostToDevice))) ||
      (bl && !chk(hipMemcpy(M->row_map, bl->row_map.data(), bl->row_map.size() * sizeof(int),
                            hipMemcpyHostToDevice))) ||
      !chk(hipStreamCreateWithFlags(&M->own, hipStreamNonBlocking)) ||
      !chk(hipStreamCreateWithFlags(&M->aux, hipStreamNonBlocking)) ||
      !chk(hipEventCreateWithFlags(&M->ev_fork, hipEventDisableTiming)) ||
      !chk(hipEventCreateWithFlags(&M->ev_join, hipEventDisableTiming)) ||
      !chk(hipEventCreateWithFlags(&M->ev_batch[0], hipEventDisableTiming)) ||
      !chk(hipEventCreateWithFlags(&M->ev_batch[1], hipEventDisableTiming)))
    return fail(PS_EHIP);
  if (ensure_hist(M, 10002) != PS_OK) return fail(PS_ENOMEM);
  *out = M;
  return PS_OK;
}

}  // namespace

extern "C" {

int ps_solve(ps_matrix *A, const double *b, const double *x0, double tol, int32_t maxit,
             int32_t variant, const ps_options *opt, double *x, int32_t *iters, double *hist,
             int32_t *status) {
  if (A && A->nsys > 1) return PS_EINVAL;  // batches return per-system results: ps_solve_batch
  return solve_impl(A, b, x0, false, tol, maxit, variant, opt, x, iters, hist, status);
}

int ps_solve_dev(ps_matrix *A, const double *b_dev, const double *x0_dev, double tol, int32_t maxit,
                 int32_t variant, const ps_options *opt, double *x_dev, int32_t *iters,
                 double *hist, int32_t *status) {
  if (A && A->nsys > 1) return PS_EINVAL;
  return solve_impl(A, b_dev, x0_dev, true, tol, maxit, variant, opt, x_dev, iters, hist, status);
}

int ps_solve_batch(ps_matrix *A, const double *b, const double *x0, double tol, int32_t maxit,
                   int32_t variant, const ps_options *opt, double *x, int32_t *iters, double *hist,
                   int32_t *status) {
  return solve_impl(A, b, x0, false, tol, maxit, variant, opt, x, iters, hist, status);
}

int ps_solve_batch_dev(ps_matrix *A, const double *b_dev, const double *x0_dev, double tol,
                       int32_t maxit, int32_t variant, const ps_options *opt, double *x_dev,
                       int32_t *iters, double *hist, int32_t *status) {
  return solve_impl(A, b_dev, x0_dev, true, tol, maxit, variant, opt, x_dev, iters, hist, status);
}

int ps_solve_dev_static(ps_matrix *A, const double *b_dev, const double *x0_dev, double tol,
                        int32_t maxit, int32_t variant, const ps_options *opt, double *x_dev,
                        int32_t *iters, double *hist, int32_t *status) {
  if (!A || A->nsys > 1 || maxit < 0) return PS_EINVAL;
  ps_options o;
  ps_default_options(&o);
  if (opt) o = *opt;
  if (o.resume || o.profile) return PS_EINVAL;
  o.graph = 0;  // instantiating a graph allocates
  // the FP32 copy of the values is made (allocated) by the first mixed-precision ps_solve*
  if (o.precision != PS_PREC_FP64 &&
      (A->format == PS_FMT_CSR ? A->val32 == nullptr : A->sval32 == nullptr))
    return PS_EINVAL;
  if (workspace_layout(A, maxit).total > kScratchDoubles) return PS_ETOOBIG;
  PS_HIP(hipSetDevice(A->device));
  double *ws = nullptr;
  PS_TRY(static_workspace(A->device, &ws));
  return solve_impl(A, b_dev, x0_dev, true, tol, maxit, variant, &o, x_dev, iters, hist, status,
                    ws);
}

int ps_spmv_dev(ps_matrix *A, const double *x_dev, double *y_dev, void *stream) {
  if (!A || !x_dev || !y_dev || A->nsys > 1) return PS_EINVAL;
  BusyGuard guard(A->busy);
  if (!guard.ok) return PS_EBUSY;
  PS_HIP(hipSetDevice(A->device));
  hipStream_t s = (hipStream_t)stream;
  A->prof_mask = 0;
  PS_TRY(spmv(A, s, PS_K_SPMV, x_dev, EpiStore{y_dev}, -1));
  PS_HIP(hipGetLastError());
  PS_HIP(hipStreamSynchronize(s));
  return PS_OK;
}

// the state vectors are FP64 at the interface; p, u, z of a precision-3 solve
// are converted (exactly) on the way in and out
bool pzu_slot(int which) { return which == PS_V_P || which == PS_V_U || which == PS_V_Z; }

int ps_get_state(ps_matrix *A, int32_t which, double *host_out) {
  if (!A || !host_out || which < 0 || which >= PS_V_COUNT || A->nsys > 1) return PS_EINVAL;
  BusyGuard guard(A->busy);
  if (!guard.ok) return PS_EBUSY;
  PS_HIP(hipSetDevice(A->device));
  const double *src = A->slot(which);
  if (A->pzu32 && pzu_slot(which)) {
    double *tmp = A->slot(kSlotTmp);
    hipLaunchKernelGGL(k_widen, elem_grid(A->n), dim3(kBlock), 0, A->own, tmp,
                       reinterpret_cast<const float *>(src), A->n);
    PS_HIP(hipGetLastError());
    PS_HIP(hipStreamSynchronize(A->own));
    src = tmp;
  }
  PS_HIP(hipMemcpy(host_out, src, A->n * sizeof(double), hipMemcpyDeviceToHost));
  return PS_OK;
}

int ps_set_state(ps_matrix *A, int32_t which, const double *host_in) {
  if (!A || !host_in || which < 0 || which >= PS_V_COUNT || A->nsys > 1) return PS_EINVAL;
  BusyGuard guard(A->busy);
  if (!guard.ok) return PS_EBUSY;
  PS_HIP(hipSetDevice(A->device));
  if (A->pzu32 && pzu_slot(which)) {
    // the other two of p, u, z back to FP64 first: the slots share one storage state
    PS_TRY(convert_pzu(A, A->own, false));
    PS_HIP(hipStreamSynchronize(A->own));
  }
  PS_HIP(hipMemcpy(A->slot(which), host_in, A->n * sizeof(double), hipMemcpyHostToDevice));
  return PS_OK;
}

int ps_get_scalars(ps_matrix *A, double *host_out) {
  if (!A || !host_out || A->nsys > 1) return PS_EINVAL;
  PS_HIP(hipSetDevice(A->device));
  PS_HIP(hipMemcpy(host_out, A->sc, PS_S_COUNT * sizeof(double), hipMemcpyDeviceToHost));
  return PS_OK;
}

int ps_set_scalars(ps_matrix *A, const double *host_in) {
  if (!A || !host_in || A->nsys > 1) return PS_EINVAL;
  PS_HIP(hipSetDevice(A->device));
  PS_HIP(hipMemcpy(A->sc, host_in, PS_S_COUNT * sizeof(double), hipMemcpyHostToDevice));
  return PS_OK;
}

int ps_matrix_info(ps_matrix *A, ps_info *info) {
  if (!A || !info) return PS_EINVAL;
  info->format = A->format;
  info->spmv_shape = A->format == PS_FMT_CSR ? A->shape : -1;
  info->n = A->n_orig;
  info->nnz = A->nnz;
  info->slots = A->format == PS_FMT_CSR ? A->nnz : A->slots;
  info->spmv_blocks = A->nblk;
  info->dot_grid = A->dot_grid;
  info->matrix_bytes = matrix_bytes(A);
  info->auto_overlap = auto_overlap(A) ? 1 : 0;
  info->auto_schedule = auto_schedule(A);
  info->nsys = A->nsys;
  info->streaming = streaming(A) ? 1 : 0;
  info->index_bits = A->index_bits;
  info->gather_sort = A->format == PS_FMT_CSR && A->gather_sort ? 1 : 0;
  info->n_padded = A->n;
  return PS_OK;
}

int ps_kernel_stats(ps_matrix *A, int32_t cls, double *total_ms, int64_t *launches) {
  if (!A || cls < 0 || cls >= PS_K_COUNT || !total_ms || !launches) return PS_EINVAL;
  *total_ms = A->prof_ms[cls];
  *launches = A->prof_cnt[cls];
  return PS_OK;
}

int ps_kernel_streams(ps_matrix *A, int32_t cls, int64_t *aux_launches) {
  if (!A || cls < 0 || cls >= PS_K_COUNT || !aux_launches) return PS_EINVAL;
  *aux_launches = A->prof_aux[cls];
  return PS_OK;
}

int ps_stream_copy(void *dst, const void *src, int64_t bytes, void *stream) {
  if (!dst || !src || bytes < 0 || (bytes % 16) != 0) return PS_EINVAL;
  if (((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return PS_EINVAL;
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return PS_OK;
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = (unsigned)std::min<int64_t>((n16 + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kBlock), 0, s, (double2 *)dst,
                     (const double2 *)src, n16);
  PS_HIP(hipGetLastError());
  PS_HIP(hipStreamSynchronize(s));
  return PS_OK;
}

int ps_destroy(ps_matrix *A) {
  free_matrix(A);
  return PS_OK;
}

const char *ps_strerror(int code) {
  switch (code) {
    case PS_OK: return "ok / converged";
    case PS_MAXIT: return "stopped at the iteration limit";
    case PS_BREAKDOWN: return "breakdown: a coefficient denominator was zero or not finite";
    case PS_NONFINITE: return "an inner product was not finite";
    case PS_EINVAL: return "invalid argument";
    case PS_ENOMEM: return "out of memory";
    case PS_EHIP: return "HIP runtime error";
    case PS_EBUSY: return "handle in use by another thread";
    case PS_ENODEV: return "no usable gfx950 device";
    case PS_ETOOBIG: return "the solve does not fit the static workspace of ps_solve_dev_static";
    default: return "unknown code";
  }
}

const char *ps_version(void) { return "pipesafe 0.1 (gfx950)"; }


// ------------------------------------------------------------------ autotuner
// Every layout, launch shape and schedule gives the same results, so the
// tuner chooses by measured time alone.

int ps_autotune_layout(ps_matrix **out, int32_t nsys, const int64_t *sys_ptr, int64_t n,
                       int64_t nnz, const int64_t *rowptr, const int32_t *col, const double *val,
                       int32_t reps, ps_tune_report *report) {
  if (!out) return PS_EINVAL;
  *out = nullptr;
  if (reps < 1 || reps > 100000 || nsys < 1 || (nsys > 1 && !sys_ptr)) return PS_EINVAL;
  if (!valid_csr(n, nnz, rowptr, col, val)) return PS_EINVAL;
  // the sliced forms only where padding every slice to its longest row keeps the
  // stored slots within kTuneMaxPadding of the nonzeros
  auto sell_ok = [&](int rpl) {
    const int64_t SH = (int64_t)kWave * rpl;
    int64_t slots = 0;
    for (int64_t r0 = 0; r0 < n; r0 += SH) {
      int64_t w = 0;
      for (int64_t r = r0; r < std::min<int64_t>(n, r0 + SH); ++r)
        w = std::max<int64_t>(w, rowptr[r + 1] - rowptr[r]);
      slots += w * SH;
    }
    return (double)slots <= kTuneMaxPadding * (double)nnz + (double)SH;
  };
  std::vector<ps_layout> cand;
  for (int rpl = 1; rpl <= 2; ++rpl)
    if (sell_ok(rpl)) {
      cand.push_back(ps_layout{PS_FMT_SELL, rpl, -1, -1, -1});
      cand.push_back(ps_layout{PS_FMT_SELL, rpl, -1, 32, -1});
    }
  for (int gs = 0; gs <= 1; ++gs)
    for (int sh = 0; sh <= 4; ++sh) cand.push_back(ps_layout{PS_FMT_CSR, -1, sh, -1, gs});
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->best = -1;
  }
  // b = 1 and x on the device, in the caller's row order
  double *ones = nullptr, *x = nullptr;
  auto release = [&]() {
    (void)hipFree(ones);
    (void)hipFree(x);
  };
  {
    const std::vector<double> h((size_t)std::max<int64_t>(n, 1), 1.0);
    if (hipMalloc(&ones, h.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&x, h.size() * sizeof(double)) != hipSuccess ||
        hipMemcpy(ones, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess) {
      release();
      return PS_EHIP;
    }
  }
  ps_options o;
  ps_default_options(&o);
  std::vector<int32_t> it((size_t)nsys), st((size_t)nsys);
  ps_matrix *best = nullptr;
  double best_us = 0.0;
  for (const ps_layout &l : cand) {
    ps_matrix *M = nullptr;
    const int rc = nsys > 1 ? ps_create_batch_ex(&M, nsys, sys_ptr, n, nnz, rowptr, col, val, &l)
                            : ps_create_ex(&M, n, nnz, rowptr, col, val, &l);
    if (rc != PS_OK) {
      if (best) free_matrix(best);
      release();
      return rc;
    }
    // a 16-bit request that does not fit gives the 32-bit layout: measured already
    if (l.format == PS_FMT_SELL && l.index_bits == -1 && M->index_bits == 32) {
      free_matrix(M);
      continue;
    }
    // time `reps` iterations of p-BiCGSafe with the automatic options (the
    // schedule, and with it the products' epilogues and the passes, depends on
    // the layout): once to capture the graphs, once timed
    double us = 0.0;
    {
      int err = PS_OK;
      for (int rep = 0; rep < 2 && err == PS_OK; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        err = ps_solve_batch_dev(M, ones, nullptr, 0.0, reps, PS_PBICGSAFE, &o, x, it.data(),
                                 nullptr, st.data());
        const auto t1 = std::chrono::steady_clock::now();
        us = std::chrono::duration<double, std::micro>(t1 - t0).count() / reps;
      }
      if (err != PS_OK) {
        free_matrix(M);
        if (best) free_matrix(best);
        release();
        return err;
      }
    }
    if (report && report->count < PS_TUNE_MAX) {
      ps_tune_entry &e = report->entry[report->count];
      e.layout = ps_layout{M->format, M->format == PS_FMT_SELL ? M->sell_rpl : -1,
                           M->format == PS_FMT_CSR ? M->shape : -1, M->index_bits,
                           M->format == PS_FMT_CSR ? (M->gather_sort ? 1 : 0) : -1};
      e.schedule = e.overlap = e.streaming = e.batch_iters = -1;
      e.us = us;
      if (!best || us < best_us) report->best = report->count;
      report->count++;
    }
    if (!best || us < best_us) {
      if (best) free_matrix(best);
      best = M;
      best_us = us;
    } else {
      free_matrix(M);
    }
  }
  release();
  *out = best;
  return PS_OK;
}

int ps_tune_options(ps_matrix *A, const double *b_dev, int32_t variant, int32_t iters,
                    ps_options *opt, ps_tune_report *report) {
  if (!A || !b_dev || !opt || iters < 1 || iters > 100000) return PS_EINVAL;
  if (variant < PS_SSBICGSAFE2 || variant > PS_PBICGSTAB) return PS_EINVAL;
  const ps_options base = *opt;
  std::vector<int> scheds = {0}, overlaps = {0, 1}, streams = {-1}, batches = {8, 16, 32};
  const bool safe_pipelined = variant == PS_PBICGSAFE || variant == PS_PBICGSAFE_RR;
  if (safe_pipelined) scheds = {0, 1, 2};
  // one stream (3): one system, p-BiCGSafe(-rr) or p-BiCGStab; one workgroup per
  // system (4): where the base options allow it
  if (A->nsys == 1 && (safe_pipelined || variant == PS_PBICGSTAB) && A->gfold <= A->nblk)
    scheds.push_back(3);
  ps_options one = base;
  one.resume = 0;
  one.profile = 0;
  if (one_group_ok(A, variant, one)) scheds.push_back(4);
  if (variant == PS_SSBICGSAFE2) overlaps = {0};  // a single stream either way
  if (safe_pipelined) streams = {0, 1};
  double *x = nullptr;
  PS_HIP(hipSetDevice(A->device));
  PS_HIP(hipMalloc(&x, std::max<int64_t>(A->n_orig, 1) * sizeof(double)));
  std::vector<int32_t> it((size_t)A->nsys), st((size_t)A->nsys);
  const int saved_stream = A->stream_override;
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->best = -1;
  }
  int rc = PS_OK;
  double best_us = -1.0;
  ps_options best = base;
  int best_stream = saved_stream;
  const std::vector<int> one_ov = {0}, one_sm = {-1}, one_bi = {8};
  for (int sc : scheds)
    // schedules 3 and 4 use one stream; 4 launches once per solve, so that the
    // streaming and graph-batch choices do nothing there
    for (int ov : sc >= 3 ? one_ov : overlaps)
      for (int sm : sc == 4 ? one_sm : streams)
        for (int bi : sc == 4 ? one_bi : batches) {
          ps_options o = base;
          o.schedule = sc;
          o.overlap = ov;
          o.batch_iters = bi;
          o.graph = 1;
          o.profile = 0;
          o.resume = 0;
          A->stream_override = sm;
          double us = 0.0;
          for (int rep = 0; rep < 2 && rc == PS_OK; ++rep) {  // the first captures the graphs
            const auto t0 = std::chrono::steady_clock::now();
            rc = ps_solve_batch_dev(A, b_dev, nullptr, 0.0, iters, variant, &o, x, it.data(),
                                    nullptr, st.data());
            const auto t1 = std::chrono::steady_clock::now();
            us = std::chrono::duration<double, std::micro>(t1 - t0).count() / iters;
          }
          if (rc != PS_OK) break;
          if (report && report->count < PS_TUNE_MAX) {
            ps_tune_entry &e = report->entry[report->count];
            e.layout = ps_layout{-1, -1, -1, -1, -1};
            e.schedule = sc;
            e.overlap = ov;
            e.streaming = sm < 0 ? (streaming(A) ? 1 : 0) : sm;
            e.batch_iters = bi;
            e.us = us;
            if (best_us < 0.0 || us < best_us) report->best = report->count;
            report->count++;
          }
          if (best_us < 0.0 || us < best_us) {
            best_us = us;
            best = o;
            best_stream = sm;
          }
        }
  (void)hipFree(x);
  if (rc != PS_OK) {
    A->stream_override = saved_stream;
    return rc;
  }
  opt->schedule = variant != PS_SSBICGSAFE2 ? best.schedule : base.schedule;
  opt->overlap = best.overlap;
  opt->batch_iters = best.batch_iters;
  A->stream_override = best_stream;
  return PS_OK;
}

}  // extern "C"
