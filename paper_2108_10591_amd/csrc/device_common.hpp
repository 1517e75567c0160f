// Device-side building blocks shared by the solver kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pipesafe.h"

namespace ps {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// int32 control block on the device
enum Ctl : int {
  C_DONE = 0,     // nonzero once the solve has stopped; every later kernel is a no-op
  C_STATUS = 1,   // ps_status once done
  C_ITERS = 2,    // iteration index at the stop
  C_HALT = 4,     // set by the first main-stream kernel that sees C_DONE; read by the
                  // sparse products that may run concurrently with a finish
  C_ITER = 5,     // index of the iteration whose reduction phase runs next; advanced
                  // by the finish, so replayed launches need no per-iteration argument
  C_FOLDS = 6,    // fold slices completed in the current product (single-stream
                  // schedule); back to 0 once the last one has finished the phase
  C_COUNT = 16
};

// double scalar block on the device: the public ps_scalar slots, then private ones
enum Sc : int {
  SC_DOTS = 16,      // raw inner products of the last reduction phase (up to 9)
  SC_SCALE = 28,     // least-residual factor c of the initial guess (x0_fallback = 2)
  SC_SCALE_OK = 29,  // 1: c could be formed; 0: the scaled guess is zero
  SC_FALLBACK = 30,  // 1: the initial guess was worse than zero and has been replaced
  SC_COUNT = 32
};

__device__ __forceinline__ bool bad_den(double d) { return d == 0.0 || !isfinite(d); }

// Batched solves: independent systems share every launch.  Each system's rows
// are padded to a multiple of 512, so a workgroup of 256 rows (products) or
// 512 rows (streaming passes) belongs to one system; chunk_sys[row / 256]
// names it.  Every system has its own control block (C_COUNT ints) and scalar
// block (SC_COUNT doubles).  chunk_sys = nullptr: one system.
__device__ __forceinline__ int system_of(const int *chunk_sys, int64_t row) {
  return chunk_sys ? chunk_sys[row >> 8] : 0;
}

// The control word that turns a sparse product into a no-op (see k_spmv).
struct Stop {
  const int *ctl;        // control blocks, [systems][C_COUNT]
  int word;              // C_DONE, C_HALT, or -1 (never stop)
  const int *chunk_sys;  // system of each 256-row chunk, or nullptr
  __device__ __forceinline__ bool stopped(int sys) const {
    return word >= 0 && ctl[(size_t)sys * C_COUNT + word] != 0;
  }
};

// Sweep direction.  Consecutive streaming kernels of an iteration walk the
// rows in alternating directions, so each one starts on the rows the previous
// one touched last -- the lines most likely still held in the 256 MB
// memory-side Infinity Cache (MALL) -- instead of the ones it evicted first.
// Per-row arithmetic is unchanged, so results do not depend on the direction.
__device__ __forceinline__ int sweep_block(int b, int nb, int rev) { return rev ? nb - 1 - b : b; }

// Row-block index for workgroup `b`: consecutive workgroups are dispatched
// round-robin over the 8 XCDs, so give each XCD a contiguous range of row
// blocks; its L2 then holds the x entries its rows gather.  The streaming
// passes use the same mapping, so that a vector entry is written through the
// L2 of the XCD whose product reads it next (cd3d 128^3: p-BiCGSafe 154.7 ->
// 147.4 us per iteration with the separate inner-product pass, 128.7 -> 127.4
// with the single-stream schedule).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, rem = nb % kXcd;
  const int xcd = b % kXcd, k = b / kXcd;
  // XCD x owns q (+1 if x < rem) consecutive blocks
  const int start = xcd * q + (xcd < rem ? xcd : rem);
  return start + k;
}

// Stop the solve: record status and iteration index.
__device__ __forceinline__ void set_stop(int *ctl, int status, int iters) {
  ctl[C_STATUS] = status;
  ctl[C_ITERS] = iters;
  ctl[C_DONE] = 1;
}

// hist[i] = sqrt(rho)/sqrt(rhoref) and the stop test ||r_i|| <= tol ||r_ref||
// (Algorithms 3-5; the test is taken before the coefficients are formed).
// Returns true if the solve stops here.
__device__ __forceinline__ bool stop_test(double rho, double rhoref, int *ctl, double *hist,
                                          int i, int maxit, double tol) {
  const double ref = sqrt(rhoref);
  const double nr = sqrt(rho);
  hist[i] = ref > 0.0 ? nr / ref : 0.0;
  if (nr <= tol * ref) {
    set_stop(ctl, PS_CONVERGED, i);
    return true;
  }
  if (i >= maxit) {
    set_stop(ctl, PS_MAXIT, i);
    return true;
  }
  return false;
}

// ------------------------------------------------------- compensated sums
// pair accumulator for the sparse products' row sums: hi + lo carries a sum
// to about twice double precision
struct DD {
  double hi, lo;
};

// a += b for two pairs
__device__ __forceinline__ void dd_add(DD &a, double bhi, double blo) {
  const double t = a.hi + bhi;
  const double z = t - a.hi;
  const double es = (a.hi - (t - z)) + (bhi - z);
  a.hi = t;
  a.lo = a.lo + (blo + es);
}

// (hi, lo) += v: Knuth's two-sum; the rounding error of the addition goes to lo
__device__ __forceinline__ void sum_acc(DD &a, double v) {
  const double t = a.hi + v;
  const double z = t - a.hi;
  const double e = (a.hi - (t - z)) + (v - z);
  a.hi = t;
  a.lo = a.lo + e;
}

// ------------------------------------------------- inner-product accumulators
// Triple accumulator for inner products: a + b + c carries a sum to about
// three times double precision.  Each product is split exactly into its
// rounded value and error (one FMA); a collects the rounded sum, b the exact
// errors of a's additions plus the products' errors (themselves summed with
// exact error terms), and c the errors of b's additions.  Only c rounds, at
// about u^3 of the terms' magnitudes, so the final rounding of a + b + c gives
// the inner product rounded once from its exact value except when that value
// lies within that distance of a rounding boundary -- whatever the order in
// which the grid adds the terms.
struct TD {
  double a, b, c;
};
constexpr int kPart = 3;  // doubles per stored partial sum (a, b, c)
// (two_sum, td_fma, td_add and td_round also compile for the host, where the
// tests check them against exact rational arithmetic)

// s + e = x + y exactly (Knuth's two-sum)
__host__ __device__ __forceinline__ void two_sum(double x, double y, double &s, double &e) {
  s = x + y;
  const double z = s - x;
  e = (x - (s - z)) + (y - z);
}

// T += x*y
__host__ __device__ __forceinline__ void td_fma(TD &T, double x, double y) {
  const double p = x * y;
  const double ep = __builtin_fma(x, y, -p);  // x*y = p + ep exactly
  double e1, e2, e3;
  two_sum(T.a, p, T.a, e1);
  two_sum(T.b, e1, T.b, e2);
  two_sum(T.b, ep, T.b, e3);
  T.c = T.c + (e2 + e3);
}

// T += U
__host__ __device__ __forceinline__ void td_add(TD &T, const TD &U) {
  double e1, e2, e3;
  two_sum(T.a, U.a, T.a, e1);
  two_sum(T.b, U.b, T.b, e2);
  two_sum(T.b, e1, T.b, e3);
  T.c = T.c + (U.c + (e2 + e3));
}

// partial sum number k of a list of triples
__device__ __forceinline__ TD td_load(const double *p, int64_t k) {
  return TD{p[k * kPart], p[k * kPart + 1], p[k * kPart + 2]};
}
__device__ __forceinline__ void td_store(double *p, int64_t k, const TD &T) {
  p[k * kPart] = T.a;
  p[k * kPart + 1] = T.b;
  p[k * kPart + 2] = T.c;
}

// The one rounding of a + b + c to the nearest double (ties to even): the
// three are brought to t + w + werr exactly by error-free additions, t + w is
// rounded, and a remainder of exactly half a unit that werr pushes past the
// midpoint moves the result one unit away.
__host__ __device__ __forceinline__ double td_round(const TD &T) {
  double s1, e1, t, e0, w, werr, r, rl;
  two_sum(T.b, T.c, s1, e1);
  two_sum(T.a, s1, t, e0);
  two_sum(e0, e1, w, werr);
  two_sum(t, w, r, rl);
  if (rl != 0.0 && werr != 0.0 && ((rl < 0.0) == (werr < 0.0))) {
    const double y = 2.0 * rl;
    const double x = r + y;
    if (x - r == y) r = x;
  }
  return r;
}

// Lane permutations of a double within rows of 16 lanes (DPP), and a lane read.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ void dd_step(DD &a) {
  const double h = dpp_f64<CTRL>(a.hi);
  const double l = dpp_f64<CTRL>(a.lo);
  dd_add(a, h, l);
}

// Pair sum over a wavefront, the same value in every lane.  Within each row of
// 16 lanes: partner at lane^1 and lane^2 (quad permutes), then the other quad
// of the half-row and the other half of the row (mirrors); then the four row
// totals (lanes 0, 16, 32, 48) in row order.
__device__ __forceinline__ DD wave_sum_dd(DD a) {
  dd_step<0xB1>(a);   // quad_perm [1,0,3,2]
  dd_step<0x4E>(a);   // quad_perm [2,3,0,1]
  dd_step<0x141>(a);  // row_half_mirror
  dd_step<0x140>(a);  // row_mirror
  DD t{readlane_f64(a.hi, 0), readlane_f64(a.lo, 0)};
#pragma unroll
  for (int r = 1; r < 4; ++r) dd_add(t, readlane_f64(a.hi, 16 * r), readlane_f64(a.lo, 16 * r));
  return t;
}

// Block-wide pair sums: on return thread k (< K) holds the block total of a[k].
template <int K>
__device__ __forceinline__ DD block_sum_dd(DD (&a)[K], double *lds) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) a[k] = wave_sum_dd(a[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      lds[(wid * K + k) * 2] = a[k].hi;
      lds[(wid * K + k) * 2 + 1] = a[k].lo;
    }
  }
  __syncthreads();
  DD r{0.0, 0.0};
  if (threadIdx.x < K) {
    r.hi = lds[threadIdx.x * 2];
    r.lo = lds[threadIdx.x * 2 + 1];
    for (int w = 1; w < kWavesPerBlock; ++w)
      dd_add(r, lds[(w * K + threadIdx.x) * 2], lds[(w * K + threadIdx.x) * 2 + 1]);
  }
  __syncthreads();
  return r;
}

// Pair sum within aligned groups of LPR (1, 2, 4, 8 or 16) lanes; lane 0 of
// each group ends with the group total.
template <int LPR>
__device__ __forceinline__ void group_sum_dd(DD &a) {
  if constexpr (LPR >= 2) dd_step<0xB1>(a);   // quad_perm [1,0,3,2]
  if constexpr (LPR >= 4) dd_step<0x4E>(a);   // quad_perm [2,3,0,1]
  if constexpr (LPR >= 8) dd_step<0x141>(a);  // row_half_mirror
  if constexpr (LPR >= 16) dd_step<0x140>(a); // row_mirror
}

template <int CTRL>
__device__ __forceinline__ void td_step(TD &T) {
  const TD U{dpp_f64<CTRL>(T.a), dpp_f64<CTRL>(T.b), dpp_f64<CTRL>(T.c)};
  td_add(T, U);
}

// Block-wide triple sums: on return thread k (< K) holds the block total of
// a[k].  The lanes of each quad are added first (two DPP steps, every lane
// taking part); the block's kBlock/4 quad totals of each product then go
// through LDS, where 4K threads add 16 each in index order and a last quad
// step adds those four.  A full wavefront butterfly would make every lane
// run all six steps for every product -- six times the additions the sums
// need, which for nine products costs more issue time than the kernels'
// memory traffic.  lds: kTdSlots * K * kPart doubles.
constexpr int kTdSlots = kBlock / 4;
template <int K>
__device__ __forceinline__ TD block_sum_td(TD (&a)[K], double *lds) {
  static_assert(4 * K <= kWave, "the last quad step runs in the first wavefront");
#pragma unroll
  for (int k = 0; k < K; ++k) {
    td_step<0xB1>(a[k]);  // quad_perm [1,0,3,2]
    td_step<0x4E>(a[k]);  // quad_perm [2,3,0,1]: every lane holds its quad's total
  }
  if ((threadIdx.x & 3) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) td_store(lds, k * kTdSlots + threadIdx.x / 4, a[k]);
  }
  __syncthreads();
  TD r{0.0, 0.0, 0.0};
  if (threadIdx.x < 4 * K) {
    const int base = (threadIdx.x / 4) * kTdSlots + (threadIdx.x & 3) * (kTdSlots / 4);
    r = td_load(lds, base);
    for (int j = 1; j < kTdSlots / 4; ++j) td_add(r, td_load(lds, base + j));
  }
  if (threadIdx.x < kWave) {  // the first wavefront: quarters 4k .. 4k+3 -> lane 4k
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

}  // namespace ps
