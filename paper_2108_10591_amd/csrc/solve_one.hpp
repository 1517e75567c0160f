// p-BiCGSafe (Algorithm 4) in one workgroup per system: the whole solve of a
// small system on the sliced layout, for systems whose iterations are a few
// microseconds of launch and drain with almost no work (schedule 4).
//
// The workgroup's NT threads own the rows r0 + t, r0 + t + NT, ... of their
// system (a batch's padding rows excluded) in every phase, so A s_i and w_i,
// which are row-local once the row's sum is known, need no barrier between
// them; a barrier separates the phases that gather (A s_i reads every s, A w_i
// every w).  Each iteration is the single-stream fused schedule's: the
// reduction phase from the nine inner products that the previous iteration's
// epilogue accumulated (the first from the vectors themselves), A s_i with
// w_i, and A w_i with every other update.
// Every per-row expression is the one the separate kernels use (sell_row adds
// a row's slots in slot order, as k_sell does; w_next and EpiPBiCGSafeAll are
// the pass's and the epilogue's), and the inner products are exact sums
// rounded once, so the results are the multi-kernel solve's bit for bit.
//
// The scalar and control blocks live in LDS during the solve (thread 0 forms
// the scalars; every wave reads them after a barrier) and are written back to
// the system's blocks when it stops, which the finish does at i = maxit at the
// latest.  Coherence of the vectors inside the workgroup: its waves share one
// CU, so a global store is visible to every wave of it after a barrier.
#pragma once

#include "dots.hpp"
#include "spmv.hpp"
#include "updates.hpp"

namespace ps {

// Block-wide triple sums for NT threads: on return thread k (< K) holds the
// block total of a[k].  Four DPP steps give every lane its 16-lane row's total;
// the NT/16 row totals of each product go through LDS, where 4K threads add a
// quarter of them each and a last quad step adds the four quarters.
// lds: K * (NT / 16) * kPart doubles.
template <int K, int NT>
__device__ __forceinline__ TD block_sum_td_rows(TD (&a)[K], double *lds) {
  constexpr int R = NT / 16;
  static_assert(4 * K <= kWave && R % 4 == 0, "block shape");
#pragma unroll
  for (int k = 0; k < K; ++k) {
    td_step<0xB1>(a[k]);   // quad_perm [1,0,3,2]
    td_step<0x4E>(a[k]);   // quad_perm [2,3,0,1]
    td_step<0x141>(a[k]);  // row_half_mirror: 8-lane totals
    td_step<0x140>(a[k]);  // row_mirror: 16-lane totals
  }
  if ((threadIdx.x & 15) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) td_store(lds, k * R + threadIdx.x / 16, a[k]);
  }
  __syncthreads();
  TD r{0.0, 0.0, 0.0};
  if (threadIdx.x < 4 * K) {
    const int base = (threadIdx.x / 4) * R + (threadIdx.x & 3) * (R / 4);
    r = td_load(lds, base);
    for (int j = 1; j < R / 4; ++j) td_add(r, td_load(lds, base + j));
  }
  if (threadIdx.x < kWave) {
    td_step<0xB1>(r);
    td_step<0x4E>(r);
  }
  __syncthreads();
  if (threadIdx.x < 4 * K && (threadIdx.x & 3) == 0) td_store(lds, threadIdx.x / 4, r);
  __syncthreads();
  TD out{0.0, 0.0, 0.0};
  if (threadIdx.x < K) out = td_load(lds, threadIdx.x);
  __syncthreads();
  return out;
}

// Row `row` of a sliced matrix (row < n): its slots summed in slot order with
// a compensated accumulator and rounded once, as k_sell sums them; SU slots'
// indices and values are loaded, then their gathers issued, per step.
template <class IT, int SU>
__device__ __forceinline__ double sell_row(const SellDev<double, IT> &S,
                                           const double *__restrict__ x, int row) {
  const int sl = row / kWave;
  const int beg = S.off[sl] + row % kWave, end = S.off[sl + 1];
  DD acc{0.0, 0.0};
  for (int k0 = beg; k0 < end; k0 += SU * kWave) {
    int c[SU];
    double v[SU];
#pragma unroll
    for (int j = 0; j < SU; ++j) {
      const int k = k0 + j * kWave;
      const bool in = k < end;
      const IT d = S.col[in ? k : k0];
      v[j] = S.val[in ? k : k0];
      if constexpr (sizeof(IT) == 4) c[j] = in ? (int)d : -1;
      else c[j] = (in && d != kSellPad16) ? row + (int)d : -1;
    }
    double xv[SU];
#pragma unroll
    for (int j = 0; j < SU; ++j) xv[j] = x[c[j] < 0 ? 0 : c[j]];
#pragma unroll
    for (int j = 0; j < SU; ++j)
      if (c[j] >= 0) sum_acc(acc, v[j] * xv[j]);
  }
  return acc.hi + acc.lo;
}

struct OneArgs {
  double *x, *r, *s, *y, *t, *p, *u, *z, *w, *l, *g, *As;
  const double *rs;
  double *sc;    // scalar blocks, [systems][SC_COUNT]
  int *ctl;      // control blocks, [systems][C_COUNT]
  double *hist;  // residual histories, hist_stride entries per system
  int64_t hist_stride;
  int *running;
  // batches: first 512-row block of each system, [systems + 1], and the end of its own
  // rows, [systems] (its padding rows are empty and stay zero in every vector, so they
  // are skipped); one system: nullptr
  const int *first_blk, *sys_end;
  int n, maxit;
  double tol;
  int first_flags;  // DotFlags of the first reduction phase (DF_SET_REF: rho_0 is the reference)
};

template <class IT, int NT>
__global__ __launch_bounds__(NT) void k_solve_one(SellDev<double, IT> S, OneArgs O) {
  constexpr int SU = 8;   // slots per row loaded ahead of their gathers: A s_i
  constexpr int SUW = 8;  // and A w_i, whose epilogue holds more registers
  __shared__ double lds[9 * (NT / 16) * kPart];
  __shared__ double d9[9];
  __shared__ double scl[SC_COUNT];  // the system's scalars during the solve
  __shared__ int cl[C_COUNT];       // and its control block
  const int sys = blockIdx.x;
  const int r0 = O.first_blk ? O.first_blk[sys] * 512 : 0;
  const int r1 = O.first_blk ? O.sys_end[sys] : O.n;
  double *gsc = O.sc + (size_t)sys * SC_COUNT;
  int *gctl = O.ctl + (size_t)sys * C_COUNT;
  if (threadIdx.x < SC_COUNT) scl[threadIdx.x] = gsc[threadIdx.x];
  if (threadIdx.x < C_COUNT) cl[threadIdx.x] = gctl[threadIdx.x];
  __syncthreads();
  if (cl[C_DONE]) return;  // stopped in the set-up
  DotArgs D{};
  D.v[0] = O.s;
  D.v[1] = O.y;
  D.v[2] = O.r;
  D.v[3] = O.rs;
  D.v[4] = O.t;
  D.ctl = cl;
  D.sc = scl;
  D.hist = O.hist + (size_t)sys * O.hist_stride;
  D.maxit = O.maxit;
  D.tol = O.tol;
  D.flags = O.first_flags;
  D.running = O.running;
  const EpiPBiCGSafeAll<false> E{O.r, O.p, O.u, O.s, O.t, O.y, O.z, O.x, O.l, O.g,
                                 O.As, O.w, O.rs, scl, nullptr};
  // the first reduction phase from the vectors (y_0 = t_{-1} = 0), in ProdSafe9's order
  bool first = true;
  TD acc[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) acc[j] = TD{0.0, 0.0, 0.0};
  for (int k = r0 + threadIdx.x; k < r1; k += NT) {
    double a[5];
    load_in<ProdSafe9<true>::MASK>(D, k, a);
    ProdSafe9<true>::acc(a, acc);
  }
  for (;;) {
    // reduction phase: the nine inner products rounded once, then the finish
    const TD tot = block_sum_td_rows<9, NT>(acc, lds);
    if (threadIdx.x < 9) d9[threadIdx.x] = td_round(tot);
    __syncthreads();
    if (threadIdx.x == 0) {
      const FinPre pre = fin_preload(D);
      // the epilogue accumulates (y,y), (y,r), (r0*,r), (r0*,t), (r,r), then the four
      // products with s_{i+1}: placed in ProdSafe9's order as the fold places them
      double d[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int row = (int)((kSafeRows >> (4 * j)) & 15u);
        d[j] = d9[first ? j : ((kSafeFromB >> j) & 1u) ? 5 + row : row];
      }
      FinSafe::run(D, pre, d);
      if (cl[C_DONE]) atomicSub(D.running, 1);
    }
    D.flags = 0;
    first = false;
    __syncthreads();
    if (cl[C_DONE]) break;
    const double be = scl[PS_S_BETA], ze = scl[PS_S_ZETA], et = scl[PS_S_ETA];
    // A s_i and w_i (Eqs. (q), (w)), row by row
    for (int k = r0 + threadIdx.x; k < r1; k += NT) {
      const double l = O.l[k], g = O.g[k], w = O.w[k];
      const double as = sell_row<IT, SU>(S, O.s, k);
      O.As[k] = as;
      O.w[k] = w_next(as, l, g, w, be, ze, et);
    }
    __syncthreads();  // every w_i before A w_i
    // A w_i with every other update, and the next iteration's inner products
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] = TD{0.0, 0.0, 0.0};
    for (int k = r0 + threadIdx.x; k < r1; k += NT) {
      const auto in = E.load(k);
      E.store(k, sell_row<IT, SUW>(S, O.w, k), in, acc);
    }
    __syncthreads();  // every s_{i+1} before the next A s
  }
  if (threadIdx.x < SC_COUNT) gsc[threadIdx.x] = scl[threadIdx.x];
  if (threadIdx.x < C_COUNT) gctl[threadIdx.x] = cl[threadIdx.x];
}

// The same solve when every system has at most R * NT rows (R = 1 or 2) and the
// layout's slices at most kTinySlots entries per row: thread t owns rows
// r0 + t + q NT (q < R) for the whole solve and keeps those rows' entries and
// their vector entries in registers; s and w, the vectors the products gather,
// also live in LDS (sv, wv), so an iteration touches global memory only for the
// history.  The arithmetic is k_solve_one's (each row's slots summed in slot
// order, w_next, the epilogue's next() and dots()), so are the results.  The
// vectors are written back when the system stops.
constexpr int kTinySlots = 8;

template <class IT, int NT, int R>
__global__ __launch_bounds__(NT) void k_solve_tiny(SellDev<double, IT> S, OneArgs O) {
  using E = EpiPBiCGSafeAll<false>;
  __shared__ double lds[9 * (NT / 16) * kPart];
  __shared__ double d9[9];
  __shared__ double scl[SC_COUNT];
  __shared__ int cl[C_COUNT];
  __shared__ double sv[R * NT], wv[R * NT];  // s and w of the system's rows
  const int sys = blockIdx.x;
  const int r0 = O.first_blk ? O.first_blk[sys] * 512 : 0;
  const int r1 = O.first_blk ? O.sys_end[sys] : O.n;
  double *gsc = O.sc + (size_t)sys * SC_COUNT;
  int *gctl = O.ctl + (size_t)sys * C_COUNT;
  if (threadIdx.x < SC_COUNT) scl[threadIdx.x] = gsc[threadIdx.x];
  if (threadIdx.x < C_COUNT) cl[threadIdx.x] = gctl[threadIdx.x];
  __syncthreads();
  if (cl[C_DONE]) return;  // stopped in the set-up
  DotArgs D{};
  D.ctl = cl;
  D.sc = scl;
  D.hist = O.hist + (size_t)sys * O.hist_stride;
  D.maxit = O.maxit;
  D.tol = O.tol;
  D.flags = O.first_flags;
  D.running = O.running;
  // the rows' entries in slot order: columns as indices into sv / wv (-1: padding)
  int cc[R][kTinySlots];
  double vv[R][kTinySlots];
  E::In st[R];
  bool mine[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = r0 + threadIdx.x + q * NT;
    mine[q] = k < r1;
    st[q] = E::In{};
#pragma unroll
    for (int j = 0; j < kTinySlots; ++j) {
      cc[q][j] = -1;
      vv[q][j] = 0.0;
    }
    if (mine[q]) {
      const int sl = k / kWave;
      const int beg = S.off[sl] + k % kWave, end = S.off[sl + 1];
#pragma unroll
      for (int j = 0; j < kTinySlots; ++j) {
        const int kk = beg + j * kWave;
        if (kk < end) {
          const IT d = S.col[kk];
          vv[q][j] = S.val[kk];
          if constexpr (sizeof(IT) == 4) cc[q][j] = d < 0 ? -1 : (int)d - r0;
          else cc[q][j] = d == kSellPad16 ? -1 : k + (int)d - r0;
        }
      }
      st[q] = E::In{O.r[k], O.p[k], O.u[k], O.s[k], O.t[k], O.y[k], O.As[k],
                    O.l[k], O.g[k], O.z[k], O.x[k], O.rs[k], O.w[k]};
    }
    sv[threadIdx.x + q * NT] = st[q].s;
  }
  // the first reduction phase from the vectors (y_0 = t_{-1} = 0), in ProdSafe9's order
  bool first = true;
  TD acc[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) acc[j] = TD{0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (mine[q]) {
      const double a[5] = {st[q].s, st[q].y, st[q].r, st[q].rs, st[q].t};
      ProdSafe9<true>::acc(a, acc);
    }
  for (;;) {
    const TD tot = block_sum_td_rows<9, NT>(acc, lds);  // (its barriers also publish sv)
    if (threadIdx.x < 9) d9[threadIdx.x] = td_round(tot);
    __syncthreads();
    if (threadIdx.x == 0) {
      const FinPre pre = fin_preload(D);
      double d[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int row = (int)((kSafeRows >> (4 * j)) & 15u);
        d[j] = d9[first ? j : ((kSafeFromB >> j) & 1u) ? 5 + row : row];
      }
      FinSafe::run(D, pre, d);
      if (cl[C_DONE]) atomicSub(D.running, 1);
    }
    D.flags = 0;
    first = false;
    __syncthreads();
    if (cl[C_DONE]) break;
    const double al = scl[PS_S_ALPHA], be = scl[PS_S_BETA], ze = scl[PS_S_ZETA],
                 et = scl[PS_S_ETA];
    // A s_i and w_i (Eqs. (q), (w))
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (mine[q]) {
        DD a{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < kTinySlots; ++j)
          if (cc[q][j] >= 0) sum_acc(a, vv[q][j] * sv[cc[q][j]]);
        st[q].As = a.hi + a.lo;
        st[q].w = w_next(st[q].As, st[q].l, st[q].g, st[q].w, be, ze, et);
      }
      wv[threadIdx.x + q * NT] = st[q].w;
    }
    __syncthreads();  // every w_i before A w_i
    // A w_i with every other update, and the next iteration's inner products
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] = TD{0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (mine[q]) {
        DD a{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < kTinySlots; ++j)
          if (cc[q][j] >= 0) sum_acc(a, vv[q][j] * wv[cc[q][j]]);
        const E::Out o = E::next(st[q], a.hi + a.lo, al, be, ze, et);
        st[q].p = o.p;
        st[q].u = o.u;
        st[q].t = o.t;
        st[q].z = o.z;
        st[q].y = o.y;
        st[q].x = o.x;
        st[q].r = o.r;
        st[q].l = o.l;
        st[q].g = o.g;
        st[q].s = o.s;
        E::dots(o, st[q].rs, acc);
      }
      // (this iteration's reads of sv all came before the barrier above)
      sv[threadIdx.x + q * NT] = st[q].s;
    }
    __syncthreads();  // every s_{i+1} before the next A s
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = r0 + threadIdx.x + q * NT;
    if (mine[q]) {
      O.r[k] = st[q].r;
      O.p[k] = st[q].p;
      O.u[k] = st[q].u;
      O.s[k] = st[q].s;
      O.t[k] = st[q].t;
      O.y[k] = st[q].y;
      O.As[k] = st[q].As;
      O.l[k] = st[q].l;
      O.g[k] = st[q].g;
      O.z[k] = st[q].z;
      O.x[k] = st[q].x;
      O.w[k] = st[q].w;
    }
  }
  if (threadIdx.x < SC_COUNT) gsc[threadIdx.x] = scl[threadIdx.x];
  if (threadIdx.x < C_COUNT) gctl[threadIdx.x] = cl[threadIdx.x];
}

}  // namespace ps
