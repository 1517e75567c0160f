// CSR sparse matrix-vector product y = A x with a fused per-row epilogue.
//
// Rows are cut at creation time into row blocks of at most kBlock rows whose
// nonzeros fit an LDS budget.  A block streams its contiguous slice of
// (val, col) with coalesced loads, forms val*x[col] into LDS, and then sums
// each row (see LPR below) and hands the row sum to the epilogue, which
// updates the row's entries of other vectors (the update passes that the
// paper's algorithms place right after each product).  A row longer than the
// budget gets a block of its own, which splits it over all threads.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "dots.hpp"

namespace ps {

// An epilogue may carry a prologue: work that some workgroups of the product do
// before their rows (EpiStoreFold).
template <class E, class = void>
struct has_prologue : std::false_type {};
template <class E>
struct has_prologue<E, std::void_t<decltype(&E::prologue)>> : std::true_type {};

// VT: the stored type of the values, double or float (the matrix rounded to
// FP32 for the mixed-precision solves); a float value is widened exactly, so
// every product and sum below is the same FP64 arithmetic either way.
// IT: the stored column index, int (the column) or short (the column minus
// the first row of the entry's row block, when every entry fits: 10 instead
// of 12 bytes per FP64 nonzero).
template <class VT, class IT = int>
struct CsrDev {
  const int *rowptr;   // int32[n+1]
  const IT *col;       // IT[nnz]
  const VT *val;       // VT[nnz]
  const int *blk;      // int32[nblk+1] first row of each row block
  // multi-lane shapes: the order in which a block's rows are summed, longest
  // first (uint8[n], block-local indices), so that the rows a wave sums in one
  // round have similar lengths; nullptr = storage order
  const unsigned char *rord;
  // gather order: a block's nonzeros stored sorted by column (so that a wave's
  // gathers touch few cache lines), with each one's position in the block's
  // row order (uint16[nnz]) for the product's slot; nullptr = row order
  const unsigned short *pos;
  int nblk;
};

// IPT: nonzeros per thread of a short-row block (the block's LDS budget is
// IPT * kBlock products).  Every load a thread needs for the products -- and,
// with one lane per row, its row bounds and the epilogue's operands -- is
// issued before the first dependent gather, so a block waits for about three
// memory latencies in total instead of two per nonzero.
//
// LPR: lanes per row when the rows are summed.  Each row's rounded products
// are added with two-sum accumulators (hi, lo) and rounded once, so the value
// does not depend on the order of the additions: with LPR = 1 a lane adds its
// row in storage order; with LPR > 1 the group's lanes take every LPR-th
// product (alternately into two accumulators) and their pairs are combined
// across the group, which keeps lanes busy on long, uneven rows.
//
// `st` names the control word that turns the launch (for a batch: the row
// block's system) into a no-op: C_DONE for products that follow a finish in
// stream order, C_HALT for products that may run concurrently with one.  The
// epilogue reads the scalars of the row block's system.  `rev` = 1 walks the
// row blocks from the last to the first (see sweep_block).
//
// An epilogue with kDots > 0 also accumulates per-row terms of inner products
// (compensated triples, see dots.hpp) and writes the block's partial sums for row
// block b; all lanes of the block take part in that reduction.
template <int IPT, int LPR, class VT, class IT, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmv(CsrDev<VT, IT> A, const double *__restrict__ x,
                                                 Epi epi_all, Stop st, int rev) {
  extern __shared__ double prod[];
  const int b = sweep_block(xcd_block(blockIdx.x, A.nblk), A.nblk, rev);
  const int r0 = A.blk[b], r1 = A.blk[b + 1];
  const int sys = system_of(st.chunk_sys, r0);
  if (st.stopped(sys)) return;
  const Epi epi = epi_all.at(sys);
  if constexpr (has_prologue<Epi>::value) {
    __shared__ double pro[kLeanLds];
    epi.prologue(pro);
  }
  constexpr int ND = Epi::kDots;
  TD dacc[ND > 0 ? ND : 1];
#pragma unroll
  for (int j = 0; j < (ND > 0 ? ND : 1); ++j) dacc[j] = TD{0.0, 0.0, 0.0};
  auto put = [&](int row, double ax, const typename Epi::In &in) {
    if constexpr (ND > 0) epi.store(row, ax, in, dacc);
    else epi.store(row, ax, in);
  };
  const int r = r0 + threadIdx.x;
  int ra = 0, re = 0;
  typename Epi::In ein{};
  if (LPR == 1 && r < r1) {
    ra = A.rowptr[r];
    re = A.rowptr[r + 1];
    ein = epi.load(r);
  }
  // LPR > 1: the row sums are staged in LDS and thread k finishes row r0 + k, so
  // the epilogue's loads (issued here, before the products) and stores are
  // coalesced whatever order the rows are summed in
  if constexpr (LPR > 1) {
    if (r < r1) ein = epi.load(r);
  }
  const int k0 = A.rowptr[r0], k1 = A.rowptr[r1];
  const int nz = k1 - k0;
  if (nz > IPT * kBlock) {
    // one long row: strided pair sums, then a fixed-order block combination
    DD acc[1] = {DD{0.0, 0.0}};
    constexpr int kU = 4;  // nonzeros per lane in flight
    for (int k = k0 + threadIdx.x; k < k1; k += kU * kBlock) {
      // loads from a clamped slot (this row's first) instead of a guarded branch, and
      // values widened only at the product: with FP32 values a branch around each
      // load would hold its conversion and make every load wait for itself
      IT cc[kU];
      VT vv[kU];
      double xx[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int kk = k + u * kBlock < k1 ? k + u * kBlock : k0;
        cc[u] = A.col[kk];
        vv[u] = A.val[kk];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) xx[u] = x[sizeof(IT) == 4 ? (int)cc[u] : r0 + (int)cc[u]];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (k + u * kBlock < k1) sum_acc(acc[0], (double)vv[u] * xx[u]);
    }
    const DD t = block_sum_dd<1>(acc, prod);
    if (threadIdx.x == 0) put(r0, t.hi + t.lo, epi.load(r0));
  } else {
    int c[IPT], ps[IPT];
    VT v[IPT];  // widened at the product
    double xv[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) ps[i] = threadIdx.x + i * kBlock;
    if constexpr (sizeof(VT) == 8 && sizeof(IT) == 4) {
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const int k = threadIdx.x + i * kBlock;
        c[i] = 0;
        v[i] = 0.0;
        if (k < nz) {
          c[i] = A.col[k0 + k];
          v[i] = A.val[k0 + k];
          if (A.pos) ps[i] = A.pos[k0 + k];
        }
      }
    } else {
      // FP32 values or 16-bit columns: a guarded load would be widened or offset
      // inside its branch and wait for itself there, so unused slots load the
      // block's first slot instead (a line lane 0 loads anyway; their products
      // are never stored), and columns are formed after all loads are issued
      IT cr[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        cr[i] = IT(0);
        v[i] = VT(0);
      }
      if (nz > 0) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const int k = threadIdx.x + i * kBlock;
          const int kk = k0 + (k < nz ? k : 0);
          cr[i] = A.col[kk];
          v[i] = A.val[kk];
          if (A.pos) ps[i] = A.pos[kk];
        }
      }
#pragma unroll
      for (int i = 0; i < IPT; ++i)
        c[i] = sizeof(IT) == 4 ? (int)cr[i] : (nz > 0 ? r0 + (int)cr[i] : 0);
    }
    // every gather unconditional (unused slots read x[0]), so that all IPT are
    // in flight together instead of one memory latency each
#pragma unroll
    for (int i = 0; i < IPT; ++i) xv[i] = x[c[i]];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int k = threadIdx.x + i * kBlock;
      if (k < nz) prod[ps[i]] = (double)v[i] * xv[i];
    }
    __syncthreads();
    if constexpr (LPR == 1) {
      if (r < r1) {
        DD acc{0.0, 0.0};
        for (int k = ra - k0; k < re - k0; ++k) sum_acc(acc, prod[k]);
        put(r, acc.hi + acc.lo, ein);
      }
    } else {
      // a block's <= kBlock rows take at most LPR rounds of kBlock / LPR groups;
      // lane j of a group keeps the sum of its round-j row
      constexpr int kGroups = kBlock / LPR;
      static_assert(kGroups * LPR == kBlock, "rounds of groups cover a block");
      const int g = threadIdx.x / LPR, j = threadIdx.x % LPR;
      double mine = 0.0;
      int mine_at = -1;
      for (int t = 0, base = 0; base < r1 - r0; ++t, base += kGroups) {  // same trip count
        const int li = base + g;
        const int rr = li < r1 - r0 ? r0 + (A.rord ? (int)A.rord[r0 + li] : li) : r1;
        DD acc{0.0, 0.0};
        if (rr < r1) {
          // two accumulators per lane (every 2 LPR-th product each), so that two
          // additions are in flight: 1M-row band product 99.5 -> 96.9 us
          const int a = A.rowptr[rr] - k0, e = A.rowptr[rr + 1] - k0;
          DD acc2{0.0, 0.0};
          int k = a + j;
          for (; k + LPR < e; k += 2 * LPR) {
            sum_acc(acc, prod[k]);
            sum_acc(acc2, prod[k + LPR]);
          }
          if (k < e) sum_acc(acc, prod[k]);
          dd_add(acc, acc2.hi, acc2.lo);
        }
        group_sum_dd<LPR>(acc);
        if (rr < r1 && j == t) {
          mine = acc.hi + acc.lo;
          mine_at = rr - r0;
        }
      }
      __syncthreads();  // every product has been read: the row sums go where they were
      if (mine_at >= 0) prod[mine_at] = mine;
      __syncthreads();
      if (r < r1) put(r, prod[threadIdx.x], ein);
    }
  }
  if constexpr (ND > 0) {
    __shared__ double red[kTdSlots * ND * kPart];
    const TD t = block_sum_td<ND>(dacc, red);
    if (threadIdx.x < ND) {
      td_store(epi.part, threadIdx.x * A.nblk + b, t);
    }
  }
}

// Sliced ELLPACK form of the same matrix, for matrices whose rows have nearly
// equal lengths (stencils): rows are cut into slices of SH = 64 * RPL
// consecutive rows (one wavefront, RPL rows per lane); slice s holds its
// rows' nonzeros column by column, width w_s = its longest row, so entry j of
// row q of the slice sits at off[s] + j * SH + q.  Each row keeps its CSR
// order; shorter rows are padded, and padding is skipped.  The column/value
// loads (RPL consecutive entries per lane) and the gather of x are contiguous
// across the lanes of a wave, and no LDS staging is needed.
//
// IT: the stored column index.  int: the column itself, -1 = padding.  short:
// the column minus the row (when every entry lies within 32767 of its row's
// diagonal, as in stencils), kSellPad16 = padding -- 10 instead of 12 bytes
// per FP64 slot.
constexpr short kSellPad16 = -32768;

template <class VT, class IT>
struct SellDev {
  const IT *col;      // IT[slots] (see above)
  const VT *val;      // VT[slots] (double, or float: see CsrDev)
  const int *off;     // int32[nslice+1] first slot of each slice
  int n;
  int nblk;           // ceil(n / (kBlock * RPL)) row blocks of kWavesPerBlock slices
};

// Slots per row loaded ahead of their gathers per step: 8, or 5 for batches of
// five-point stencils, 7 for large seven-point ones (see sell_launch).
constexpr int kSellUnroll = 8;
constexpr int kSellUnrollNarrow = 5;
constexpr int kSellUnroll7 = 7;

template <int RPL, class VT, class IT>
__device__ __forceinline__ void sell_load(const SellDev<VT, IT> &S, int kk, IT (&c)[RPL],
                                          VT (&v)[RPL]) {
  if constexpr (RPL == 2) {
    if constexpr (sizeof(IT) == 4) {
      const int2 cc = *reinterpret_cast<const int2 *>(S.col + kk);
      c[0] = cc.x;
      c[1] = cc.y;
    } else {
      const short2 cc = *reinterpret_cast<const short2 *>(S.col + kk);
      c[0] = cc.x;
      c[1] = cc.y;
    }
    if constexpr (sizeof(VT) == 8) {
      const double2 vv = *reinterpret_cast<const double2 *>(S.val + kk);
      v[0] = vv.x;
      v[1] = vv.y;
    } else {
      const float2 vv = *reinterpret_cast<const float2 *>(S.val + kk);
      v[0] = vv.x;
      v[1] = vv.y;
    }
  } else {
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      c[u] = S.col[kk + u];
      v[u] = S.val[kk + u];
    }
  }
}

template <int RPL, class VT, class IT, class Epi, int SU = kSellUnroll>
__global__ __launch_bounds__(kBlock) void k_sell(SellDev<VT, IT> S, const double *__restrict__ x,
                                                 Epi epi_all, Stop st, int rev) {
  constexpr int ND = Epi::kDots;
  constexpr int SH = kWave * RPL;
  TD dacc[ND > 0 ? ND : 1];
#pragma unroll
  for (int j = 0; j < (ND > 0 ? ND : 1); ++j) dacc[j] = TD{0.0, 0.0, 0.0};
  const int b = sweep_block(xcd_block(blockIdx.x, S.nblk), S.nblk, rev);
  const int sys = system_of(st.chunk_sys, (int64_t)b * kBlock * RPL);
  if (st.stopped(sys)) return;
  const Epi epi = epi_all.at(sys);
  if constexpr (has_prologue<Epi>::value) {
    __shared__ double pro[kLeanLds];
    epi.prologue(pro);
  }
  const int lane = threadIdx.x % kWave;
  const int sl = b * kWavesPerBlock + threadIdx.x / kWave;
  const int r0 = sl * SH + lane * RPL;  // the lane's first row
  if (r0 < S.n) {
    typename Epi::In in[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (r0 + u < S.n) in[u] = epi.load(r0 + u);
    const int end = S.off[sl + 1];
    DD acc[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) acc[u] = DD{0.0, 0.0};
    for (int k = S.off[sl] + lane * RPL; k < end; k += SU * SH) {
      int c[SU][RPL];
      VT v[SU][RPL];  // widened at the product: a conversion next to its load
                               // would make each load wait for itself
      if constexpr (sizeof(IT) == 4) {
#pragma unroll
        for (int t = 0; t < SU; ++t) {
          const int kk = k + t * SH;
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            c[t][u] = -1;
            v[t][u] = VT(0);
          }
          if (kk < end) sell_load<RPL, VT, IT>(S, kk, c[t], v[t]);
        }
      } else {
        // 16-bit offsets: loads from a clamped slot (this step's first, which is in
        // range) instead of a guarded branch, columns formed after all loads are
        // issued, so that no load waits for itself
        IT d[SU][RPL];
#pragma unroll
        for (int t = 0; t < SU; ++t) {
          const int kk = k + t * SH < end ? k + t * SH : k;
          sell_load<RPL, VT, IT>(S, kk, d[t], v[t]);
        }
        // schedule all the step's loads (an index and a value per slot and row)
        // before the column arithmetic, which would otherwise be interleaved with
        // them and make later loads wait for earlier ones (128^3: 143.7 -> 140.3 us
        // per iteration)
        __builtin_amdgcn_sched_group_barrier(0x020, 2 * SU * RPL, 0);  // VMEM reads
        __builtin_amdgcn_sched_group_barrier(0x002, 64, 0);                     // then VALU
#pragma unroll
        for (int t = 0; t < SU; ++t)
#pragma unroll
          for (int u = 0; u < RPL; ++u)
            c[t][u] = (k + t * SH < end && d[t][u] != kSellPad16) ? r0 + u + (int)d[t][u] : -1;
      }
      // unconditional gathers (padding reads x[0]): all of them in flight at once
      double xv[SU][RPL];
#pragma unroll
      for (int t = 0; t < SU; ++t)
#pragma unroll
        for (int u = 0; u < RPL; ++u) xv[t][u] = x[c[t][u] < 0 ? 0 : c[t][u]];
#pragma unroll
      for (int t = 0; t < SU; ++t)
#pragma unroll
        for (int u = 0; u < RPL; ++u)
          if (c[t][u] >= 0) sum_acc(acc[u], (double)v[t][u] * xv[t][u]);
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      if (r0 + u < S.n) {
        if constexpr (ND > 0) epi.store(r0 + u, acc[u].hi + acc[u].lo, in[u], dacc);
        else epi.store(r0 + u, acc[u].hi + acc[u].lo, in[u]);
      }
    }
  }
  if constexpr (ND > 0) {
    __shared__ double red[kTdSlots * ND * kPart];
    const TD t = block_sum_td<ND>(dacc, red);
    if (threadIdx.x < ND) {
      td_store(epi.part, threadIdx.x * S.nblk + b, t);
    }
  }
}

// ------------------------------------------------------------------ epilogues
// load(r) fetches the row's operands before the products; store(r, ax, in)
// finishes the row once its sum A x is known.

// y = A x
struct EpiStore {
  static constexpr int kDots = 0;
  __device__ __forceinline__ EpiStore at(int) const { return *this; }
  double *y;
  struct In {};
  __device__ __forceinline__ In load(int) const { return In{}; }
  __device__ __forceinline__ void store(int r, double ax, const In &) const { y[r] = ax; }
};

// y = A x, with a prologue for the single-stream schedule (schedule 3): the
// product's first gf workgroups fold the partial sums of a reduction phase's ND
// inner products that earlier kernels left (lists) into [ND][gf]
// (fin.partials), and the last of them to finish adds those and runs the
// phase's finish Fin (fold_then_finish) -- the reduction phase inside the
// product it is hidden behind, with no second stream and no launch of its own.
// Rows are stored as by EpiStore; no workgroup of the product reads what the
// prologue writes.
template <int ND, class Fin>
struct EpiStoreFold {
  static constexpr int kDots = 0;
  __device__ __forceinline__ EpiStoreFold at(int) const { return *this; }
  double *y;
  FoldLists lists;
  int gf;      // fold slices (workgroups taking part)
  DotArgs fin; // the finish: fin.partials = the [ND][gf] folded triples
  struct In {};
  __device__ __forceinline__ In load(int) const { return In{}; }
  __device__ __forceinline__ void store(int r, double ax, const In &) const { y[r] = ax; }
  __device__ __forceinline__ void prologue(double *lds) const {
    if ((int)blockIdx.x < gf) fold_then_finish<ND, Fin>(lists, fin, gf, (int)blockIdx.x, lds);
  }
};

// r = b - A x (and optionally r0* = r): the initial residual of every
// algorithm, and the true residual of a replacement step (Algorithm 5)
struct EpiResidual {
  static constexpr int kDots = 0;
  __device__ __forceinline__ EpiResidual at(int) const { return *this; }
  const double *b;
  double *r;
  double *rs;  // may be null
  struct In {
    double b;
  };
  __device__ __forceinline__ In load(int row) const { return In{b[row]}; }
  __device__ __forceinline__ void store(int row, double ax, const In &in) const {
    const double v = in.b - ax;
    r[row] = v;
    if (rs) rs[row] = v;
  }
};

// p-BiCGSafe, the product A w_i and the three recurrences that follow it in
// Algorithm 4: l_i = q_i - A w_i (Eq. (l)), g_{i+1} = zeta A s_i + eta g_i -
// alpha A w_i (Eq. (g)), s_{i+1} = s_i - alpha q_i - g_{i+1} (Eq. (sip1)),
// with q_i = As_i + beta l_{i-1} (Eq. (q)) formed here from the old l, as in
// pass A, instead of being stored there.  A w_i itself is never stored.
struct EpiPBiCGSafeB {
  static constexpr int kDots = 0;
  // the scalars of system `sys`
  __device__ __forceinline__ EpiPBiCGSafeB at(int sys) const {
    EpiPBiCGSafeB e = *this;
    e.sc += (size_t)sys * SC_COUNT;
    return e;
  }
  const double *As;
  double *l, *g, *s;
  const double *sc;
  struct In {
    double l, As, g, s;
  };
  __device__ __forceinline__ In load(int r) const { return In{l[r], As[r], g[r], s[r]}; }
  __device__ __forceinline__ void store(int r, double aw, const In &in) const {
    const double al = sc[PS_S_ALPHA], be = sc[PS_S_BETA], ze = sc[PS_S_ZETA], et = sc[PS_S_ETA];
    const double q = in.As + be * in.l;
    l[r] = q - aw;
    const double gn = ze * in.As + et * in.g - al * aw;
    g[r] = gn;
    s[r] = in.s - al * q - gn;
  }
};

// ssBiCGSafe2, the product w_i = A u_i and the updates after it (Algorithm 3):
// o_i = s_i + beta t_{i-1} (recomputed, not stored), t_i = o_i - w_i,
// z_i = zeta r_i + eta z_{i-1} - alpha u_i, y_{i+1} = zeta s_i + eta y_i - alpha w_i,
// x_{i+1} = x_i + alpha p_i + z_i, r_{i+1} = r_i - alpha o_i - y_{i+1}.
// NT: x and z, which no other kernel of the iteration touches, stream past the
// cache (cd3d 128^3: 141.3 -> 134.8 us per iteration).
template <bool NT>
struct EpiSsBiCGSafe2B {
  static constexpr int kDots = 0;
  // the scalars of system `sys`
  __device__ __forceinline__ EpiSsBiCGSafe2B at(int sys) const {
    EpiSsBiCGSafe2B e = *this;
    e.sc += (size_t)sys * SC_COUNT;
    return e;
  }
  const double *s, *u, *p;
  double *t, *z, *y, *x, *r;
  const double *sc;
  struct In {
    double s, t, r, z, u, y, x, p;
  };
  __device__ __forceinline__ static double ld(const double *a, int k) {
    if constexpr (NT) return __builtin_nontemporal_load(a + k);
    else return a[k];
  }
  __device__ __forceinline__ static void st(double *a, int k, double v) {
    if constexpr (NT) __builtin_nontemporal_store(v, a + k);
    else a[k] = v;
  }
  __device__ __forceinline__ In load(int row) const {
    return In{s[row], t[row], r[row], ld(z, row), u[row], y[row], ld(x, row), p[row]};
  }
  __device__ __forceinline__ void store(int row, double wv, const In &in) const {
    const double al = sc[PS_S_ALPHA], be = sc[PS_S_BETA], ze = sc[PS_S_ZETA], et = sc[PS_S_ETA];
    const double o = in.s + be * in.t;
    t[row] = o - wv;
    const double zn = ze * in.r + et * in.z - al * in.u;
    st(z, row, zn);
    const double yn = ze * in.s + et * in.y - al * wv;
    y[row] = yn;
    st(x, row, in.x + al * in.p + zn);
    r[row] = in.r - al * o - yn;
  }
};

// EpiPBiCGSafeB, plus the partial sums of the four inner products of the next
// iteration that involve s_{i+1}: a = (s,s), c = (s,y), d = (s,r), g = (r0*,s),
// with y_{i+1} and r_{i+1} from the pass A that precedes this product.
// part: [4][nblk] (a, b, c) triples.  NT: l and g (next read by the next pass A)
// and As (dead after this product) stream past the cache.
template <bool NT>
struct EpiPBiCGSafeBDots {
  static constexpr int kDots = 4;
  // the scalars of system `sys`
  __device__ __forceinline__ EpiPBiCGSafeBDots at(int sys) const {
    EpiPBiCGSafeBDots e = *this;
    e.sc += (size_t)sys * SC_COUNT;
    return e;
  }
  const double *As;
  double *l, *g, *s;
  const double *y, *r, *rs;
  const double *sc;
  double *part;
  struct In {
    double l, As, g, s, y, r, rs;
  };
  __device__ __forceinline__ In load(int k) const {
    if constexpr (NT)
      return In{__builtin_nontemporal_load(l + k), __builtin_nontemporal_load(As + k),
                __builtin_nontemporal_load(g + k), s[k], y[k], r[k], rs[k]};
    else
      return In{l[k], As[k], g[k], s[k], y[k], r[k], rs[k]};
  }
  __device__ __forceinline__ void store(int k, double aw, const In &in, TD (&acc)[4]) const {
    const double al = sc[PS_S_ALPHA], be = sc[PS_S_BETA], ze = sc[PS_S_ZETA], et = sc[PS_S_ETA];
    const double q = in.As + be * in.l;
    const double ln = q - aw;
    const double gn = ze * in.As + et * in.g - al * aw;
    if constexpr (NT) {
      __builtin_nontemporal_store(ln, l + k);
      __builtin_nontemporal_store(gn, g + k);
    } else {
      l[k] = ln;
      g[k] = gn;
    }
    const double sn = in.s - al * q - gn;
    s[k] = sn;
    td_fma(acc[0], sn, sn);
    td_fma(acc[1], sn, in.y);
    td_fma(acc[2], sn, in.r);
    td_fma(acc[3], in.rs, sn);
  }
};

// p-BiCGSafe, fused-epilogue schedule: with w_i already formed for every row
// (k_pass_w, Eqs. (q), (w)), the epilogue of A w_i makes all the other updates
// of iteration i (Algorithm 4): the search directions p_i, u_i and q_i (Eq. (q),
// formed again from the operands pass w read), the residual updates t_i, z_i,
// y_{i+1}, x_{i+1}, r_{i+1}, then the recurrences Eqs. (l), (g), (sip1) with A w_i
// -- and the partial sums of all nine inner products of iteration i+1, written
// as [5][nblk] triples of (b, e, f, h, rho) followed by [4][nblk] triples of
// (a, c, d, g): the layout k_fold_partials takes.  NT: p, u, t, z, x, y, r (next
// read by the next such epilogue) and As (dead here) stream past the cache; l,
// g, w and s, read by the next w pass and product, do not.  ZT: the stored type
// of p, u, z (float: precision 3).
template <bool NT, class ZT = double>
struct EpiPBiCGSafeAll {
  static constexpr int kDots = 9;
  __device__ __forceinline__ EpiPBiCGSafeAll at(int sys) const {
    EpiPBiCGSafeAll e = *this;
    e.sc += (size_t)sys * SC_COUNT;
    return e;
  }
  // p, u, z of stored type ZT (float: held as FP32 numbers, widened on load,
  // rounded to nearest when formed)
  __device__ __forceinline__ static double ldz(const double *a, int k) {
    if constexpr (sizeof(ZT) == 8) return ld(a, k);
    const float *f = reinterpret_cast<const float *>(a);
    if constexpr (NT) return (double)__builtin_nontemporal_load(f + k);
    else return (double)f[k];
  }
  __device__ __forceinline__ static void stz(double *a, int k, double v) {
    if constexpr (sizeof(ZT) == 8) {
      st(a, k, v);
    } else {
      float *f = reinterpret_cast<float *>(a);
      if constexpr (NT) __builtin_nontemporal_store((float)v, f + k);
      else f[k] = (float)v;
    }
  }
  __device__ __forceinline__ static double held(double v) {
    if constexpr (sizeof(ZT) == 8) return v;
    else return (double)(float)v;
  }
  double *r, *p, *u, *s, *t, *y, *z, *x, *l, *g;
  const double *As, *w, *rs;
  const double *sc;
  double *part;
  struct In {
    double r, p, u, s, t, y, As, l, g, z, x, rs, w;
  };
  __device__ __forceinline__ static double ld(const double *a, int k) {
    if constexpr (NT) return __builtin_nontemporal_load(a + k);
    else return a[k];
  }
  __device__ __forceinline__ static void st(double *a, int k, double v) {
    if constexpr (NT) __builtin_nontemporal_store(v, a + k);
    else a[k] = v;
  }
  __device__ __forceinline__ In load(int k) const {
    return In{ld(r, k), ldz(p, k), ldz(u, k), s[k], ld(t, k), ld(y, k), ld(As, k),
              l[k],     g[k],      ldz(z, k), ld(x, k), rs[k], w[k]};
  }
  // the row's new entries, from its operands and A w_i (aw)
  struct Out {
    double p, u, t, z, y, x, r, l, g, s;
  };
  __device__ __forceinline__ static Out next(const In &in, double aw, double al, double be,
                                             double ze, double et) {
    const double o = in.s + be * in.t;
    const double pn = held(in.r + be * (in.p - in.u));
    const double un = held(ze * o + et * (in.y + be * in.u));
    const double q = in.As + be * in.l;
    const double tn = o - in.w;
    const double zn = held(ze * in.r + et * in.z - al * un);
    const double yn = ze * in.s + et * in.y - al * in.w;
    const double xn = in.x + al * pn + zn;
    const double rn = in.r - al * o - yn;
    const double ln = q - aw;
    const double gn = ze * in.As + et * in.g - al * aw;
    const double sn = in.s - al * q - gn;
    return Out{pn, un, tn, zn, yn, xn, rn, ln, gn, sn};
  }
  // the row's terms of the nine inner products of iteration i+1
  __device__ __forceinline__ static void dots(const Out &o, double rs, TD (&acc)[9]) {
    td_fma(acc[0], o.y, o.y);
    td_fma(acc[1], o.y, o.r);
    td_fma(acc[2], rs, o.r);
    td_fma(acc[3], rs, o.t);
    td_fma(acc[4], o.r, o.r);
    td_fma(acc[5], o.s, o.s);
    td_fma(acc[6], o.s, o.y);
    td_fma(acc[7], o.s, o.r);
    td_fma(acc[8], rs, o.s);
  }
  __device__ __forceinline__ void store(int k, double aw, const In &in, TD (&acc)[9]) const {
    const Out o = next(in, aw, sc[PS_S_ALPHA], sc[PS_S_BETA], sc[PS_S_ZETA], sc[PS_S_ETA]);
    stz(p, k, o.p);
    stz(u, k, o.u);
    st(t, k, o.t);
    stz(z, k, o.z);
    st(y, k, o.y);
    st(x, k, o.x);
    st(r, k, o.r);
    l[k] = o.l;
    g[k] = o.g;
    s[k] = o.s;
    dots(o, in.rs, acc);
  }
};

}  // namespace ps
