// Multi-inner-product kernels and their finish.
//
// One pass over the input vectors forms every inner product of a reduction
// phase at once: each thread keeps one accumulator per product over a fixed
// grid-stride set of entries, the block combines them with wavefront
// shuffles and LDS, and each block writes its partial sums.  A one-block
// finish kernel, next in the same stream, adds the partials in block order --
// so the result is bit-for-bit reproducible -- and computes the phase's scalar
// coefficients and the stop test on the device.  No host round trip.
//
// Why two kernels rather than a last-arriving-block finish: on this part each
// XCD has its own write-back L2, so a block that publishes partials to a block
// on another XCD needs a device-scope release (a full L2 write-back) per
// block; one kernel boundary gives the same visibility once.  The finish is a
// small launch on the reduction's own stream, hidden behind the concurrent
// sparse product.
//
// Accumulators are unevaluated triples (a, b, c) (TD in device_common.hpp):
// each product is split exactly into its rounded value and rounding error (one
// FMA), each addition into its rounded sum and exact error (Knuth's two-sum),
// and the errors are carried one level down, twice.  a + b + c is rounded once
// at the end.  Only the third level rounds, near u^3 of the terms, so the
// result is the inner product rounded once from its exact value whenever that
// value is not within that distance of a rounding boundary: it does not depend
// on how the grid splits the sum, even where the terms cancel to 1e-12 of
// their magnitude (near-orthogonal r0* and r late in a long solve), where a
// pair accumulator's u^2 error can already move the rounding.
#pragma once

#include "device_common.hpp"

namespace ps {

struct DotArgs {
  const double *v[5];  // input vectors
  int64_t n;
  double *partials;    // [ND][gridDim.x] (a, b, c) triples
  int *ctl;
  double *sc;
  double *hist;
  int maxit;
  double tol;
  int flags;           // finish-specific flags
  int *running;        // systems still running; a finish that stops its system decrements it
};

enum DotFlags : int {
  DF_SET_REF = 1,      // take rho of this phase as the stop-test reference (||r_0||^2)
};

// ---------------------------------------------------------------- products

// the nine inner products of Algorithms 3-5 over (s, y, r, r0*, t_{i-1}):
// a=(s,s) b=(y,y) c=(s,y) d=(s,r) e=(y,r) f=(r0*,r) g=(r0*,s) h=(r0*,t) rho=(r,r).
// FIRST: i = 0, where only a, d, f, g, rho are formed (y_0 = t_{-1} = 0).
template <bool FIRST>
struct ProdSafe9 {
  static constexpr unsigned MASK = FIRST ? 0b01101u : 0b11111u;  // s, (y), r, r0*, (t)
  static constexpr int ND = 9;
  __device__ __forceinline__ static void acc(const double (&in)[5], TD (&a)[ND]) {
    const double s = in[0], r = in[2], rs = in[3];
    td_fma(a[0], s, s);
    td_fma(a[3], s, r);
    td_fma(a[5], rs, r);
    td_fma(a[6], rs, s);
    td_fma(a[8], r, r);
    if (!FIRST) {
      const double y = in[1], t = in[4];
      td_fma(a[1], y, y);
      td_fma(a[2], s, y);
      td_fma(a[4], y, r);
      td_fma(a[7], rs, t);
    }
  }
};

// p-BiCGStab phase 1: (q, y), (y, y)
struct ProdStab2 {
  static constexpr unsigned MASK = 0b11u;  // q, y
  static constexpr int ND = 2;
  __device__ __forceinline__ static void acc(const double (&in)[5], TD (&a)[ND]) {
    td_fma(a[0], in[0], in[1]);
    td_fma(a[1], in[1], in[1]);
  }
};

// p-BiCGStab phase 2: (r0*, r), (r0*, w), (r0*, s), (r0*, z), (r, r)
// inputs: v = {r0*, r, w, s, z}
struct ProdStab5 {
  static constexpr unsigned MASK = 0b11111u;
  static constexpr int ND = 5;
  __device__ __forceinline__ static void acc(const double (&in)[5], TD (&a)[ND]) {
    const double rs = in[0], r = in[1];
    td_fma(a[0], rs, r);
    td_fma(a[1], rs, in[2]);
    td_fma(a[2], rs, in[3]);
    td_fma(a[3], rs, in[4]);
    td_fma(a[4], r, r);
  }
};

// p-BiCGStab set-up: (r0*, r0), (r0*, w0), (r0, r0); inputs v = {r0*, r, w}
struct ProdStab3 {
  static constexpr unsigned MASK = 0b111u;
  static constexpr int ND = 3;
  __device__ __forceinline__ static void acc(const double (&in)[5], TD (&a)[ND]) {
    td_fma(a[0], in[0], in[1]);
    td_fma(a[1], in[0], in[2]);
    td_fma(a[2], in[1], in[1]);
  }
};

// (r0, r0) and (b, b) of an initial guess x0 (inputs v = {r0, b})
struct ProdFallback {
  static constexpr unsigned MASK = 0b11u;
  static constexpr int ND = 2;
  __device__ __forceinline__ static void acc(const double (&in)[5], TD (&a)[ND]) {
    td_fma(a[0], in[0], in[0]);
    td_fma(a[1], in[1], in[1]);
  }
};

// (A x0, b) and (A x0, A x0) of an initial guess (inputs v = {A x0, b})
struct ProdScale {
  static constexpr unsigned MASK = 0b11u;
  static constexpr int ND = 2;
  __device__ __forceinline__ static void acc(const double (&in)[5], TD (&a)[ND]) {
    td_fma(a[0], in[0], in[1]);
    td_fma(a[1], in[0], in[0]);
  }
};

// (v, v): the squared norm of b for the ||b|| stop-test scale
struct ProdNorm {
  static constexpr unsigned MASK = 0b1u;
  static constexpr int ND = 1;
  __device__ __forceinline__ static void acc(const double (&in)[5], TD (&a)[ND]) {
    td_fma(a[0], in[0], in[0]);
  }
};

// load entry k (or the pair k, k+1, 16-byte aligned) of the inputs in MASK
template <unsigned MASK>
__device__ __forceinline__ void load_in(const DotArgs &A, int64_t k, double (&a)[5]) {
#pragma unroll
  for (int j = 0; j < 5; ++j)
    if ((MASK >> j) & 1u) a[j] = A.v[j][k];
}
template <unsigned MASK>
__device__ __forceinline__ void load_in2(const DotArgs &A, int64_t k, double (&a)[5],
                                         double (&b)[5]) {
#pragma unroll
  for (int j = 0; j < 5; ++j)
    if ((MASK >> j) & 1u) {
      const double2 v = *reinterpret_cast<const double2 *>(A.v[j] + k);
      a[j] = v.x;
      b[j] = v.y;
    }
}

// ---------------------------------------------------------------- finishes
// Run by one thread with the phase's final inner products.  The scalars a
// finish reads (left by earlier phases) are loaded by that thread at the start
// of the kernel, before the partial sums, so the coefficient formulas do not
// wait for a memory round trip each after the sums.
struct FinPre {
  int i;  // index of the iteration whose phase this is (C_ITER)
  double rhoref, alpha, zeta, omega, f;
};
__device__ __forceinline__ FinPre fin_preload(const DotArgs &A) {
  FinPre p;
  p.i = A.ctl[C_ITER];
  p.rhoref = A.sc[PS_S_RHOREF];
  p.alpha = A.sc[PS_S_ALPHA];
  p.zeta = A.sc[PS_S_ZETA];
  p.omega = A.sc[PS_S_OMEGA];
  p.f = A.sc[PS_S_F];
  return p;
}

// The outcome of the BiCGSafe reduction phase of iteration i (Algorithms 3-5;
// the stop test first, reading R5; a zero or non-finite denominator is a
// breakdown, reading R10): the history entry, the status if the solve stops
// here (else -1), and otherwise beta, alpha, zeta, eta.  It writes nothing, so
// every caller that needs the coefficients can form them itself.
struct SafeStep {
  double hist;  // ||r_i|| / ||r_ref||, NaN if an inner product is not finite
  int status;   // ps_status when the solve stops at i, else -1
  double alpha, beta, zeta, eta;
};
__device__ __forceinline__ SafeStep safe_step(const double (&d)[9], int i, double rhoref,
                                              double alpha_prev, double zeta_prev, double f_prev,
                                              int maxit, double tol) {
  SafeStep s{0.0, -1, 0.0, 0.0, 0.0, 0.0};
  const double a = d[0], b = d[1], c = d[2], dd = d[3], e = d[4], f = d[5], g = d[6], h = d[7],
               rho = d[8];
  bool finite = true;
  for (int j = 0; j < 9; ++j) finite = finite && isfinite(d[j]);
  if (!finite) {
    s.hist = NAN;
    s.status = PS_NONFINITE;
    return s;
  }
  const double ref = sqrt(rhoref);
  const double nr = sqrt(rho);
  s.hist = ref > 0.0 ? nr / ref : 0.0;
  if (nr <= tol * ref) {
    s.status = PS_CONVERGED;
    return s;
  }
  if (i >= maxit) {
    s.status = PS_MAXIT;
    return s;
  }
  double beta, alpha, zeta, eta;
  if (i == 0) {
    if (bad_den(g) || bad_den(a)) {
      s.status = PS_BREAKDOWN;
      return s;
    }
    beta = 0.0;
    alpha = f / g;
    zeta = dd / a;
    eta = 0.0;
  } else {
    const double den_beta = zeta_prev * f_prev;
    if (bad_den(den_beta)) {
      s.status = PS_BREAKDOWN;
      return s;
    }
    beta = (alpha_prev * f) / den_beta;
    const double den_alpha = g + beta * h;
    const double den_ze = a * b - c * c;
    if (bad_den(den_alpha) || bad_den(den_ze)) {
      s.status = PS_BREAKDOWN;
      return s;
    }
    alpha = f / den_alpha;
    zeta = (b * dd - c * e) / den_ze;
    eta = (a * e - c * dd) / den_ze;
  }
  if (!isfinite(beta) || !isfinite(alpha) || !isfinite(zeta) || !isfinite(eta)) {
    s.status = PS_BREAKDOWN;
    return s;
  }
  s.alpha = alpha;
  s.beta = beta;
  s.zeta = zeta;
  s.eta = eta;
  return s;
}

// Algorithms 3-5: stop test first, then beta, alpha, zeta, eta, stored in the
// scalar block.
struct FinSafe {
  __device__ static void run(const DotArgs &A, const FinPre &P, const double (&d)[9]) {
    double *sc = A.sc;
    const int i = P.i;
    const double rho = d[8];
    for (int j = 0; j < 9; ++j) sc[SC_DOTS + j] = d[j];
    sc[PS_S_RHO] = rho;
    const bool set_ref = (A.flags & DF_SET_REF) != 0;
    const SafeStep st =
        safe_step(d, i, set_ref ? rho : P.rhoref, P.alpha, P.zeta, P.f, A.maxit, A.tol);
    A.hist[i] = st.hist;
    if (set_ref && st.status != PS_NONFINITE) sc[PS_S_RHOREF] = rho;
    if (st.status >= 0) {
      set_stop(A.ctl, st.status, i);
      return;
    }
    sc[PS_S_ALPHA] = st.alpha;
    sc[PS_S_BETA] = st.beta;
    sc[PS_S_ZETA] = st.zeta;
    sc[PS_S_ETA] = st.eta;
    sc[PS_S_F] = d[5];
    A.ctl[C_ITER] = i + 1;
  }
};

// p-BiCGStab phase 1: omega_i = (q, y)/(y, y); (y, y) = 0 gives omega = 0.
struct FinStabOmega {
  __device__ static void run(const DotArgs &A, const FinPre &P, const double (&d)[2]) {
    double *sc = A.sc;
    const int i = P.i;
    sc[SC_DOTS + 0] = d[0];
    sc[SC_DOTS + 1] = d[1];
    if (!isfinite(d[0]) || !isfinite(d[1])) {
      set_stop(A.ctl, PS_NONFINITE, i);
      return;
    }
    const double om = d[1] == 0.0 ? 0.0 : d[0] / d[1];
    if (!isfinite(om)) {
      set_stop(A.ctl, PS_BREAKDOWN, i);
      return;
    }
    sc[PS_S_OMEGA] = om;
  }
};

// p-BiCGStab phase 2 of iteration i: beta_i and alpha_{i+1}, then the stop
// test of iteration i+1 on rho_{i+1}.  A coefficient that cannot be formed is
// a breakdown only if the solve does not stop there.
struct FinStabBetaAlpha {
  __device__ static void run(const DotArgs &A, const FinPre &P, const double (&d)[5]) {
    double *sc = A.sc;
    const double f = d[0], gw = d[1], gs = d[2], gz = d[3], rho = d[4];
    for (int j = 0; j < 5; ++j) sc[SC_DOTS + j] = d[j];
    const int i1 = P.i + 1;
    const double al = P.alpha, om = P.omega;  // omega: this iteration's phase 1
    double beta = 0.0, alpha = 0.0;
    bool pend = false;
    const double den_beta = om * P.f;
    if (bad_den(den_beta)) {
      pend = true;
    } else {
      beta = (al * f) / den_beta;
      const double den_alpha = gw + beta * gs - beta * om * gz;
      if (bad_den(den_alpha)) pend = true;
      else alpha = f / den_alpha;
      if (!isfinite(beta) || !isfinite(alpha)) pend = true;
    }
    sc[PS_S_ALPHA] = alpha;
    sc[PS_S_BETA] = beta;
    sc[PS_S_F] = f;
    sc[PS_S_GW] = gw;
    sc[PS_S_GS] = gs;
    sc[PS_S_GZ] = gz;
    sc[PS_S_RHO] = rho;
    sc[PS_S_PENDING] = pend ? 1.0 : 0.0;
    if (!isfinite(f) || !isfinite(gw) || !isfinite(gs) || !isfinite(gz) || !isfinite(rho)) {
      A.hist[i1] = NAN;
      set_stop(A.ctl, PS_NONFINITE, i1);
      return;
    }
    if (stop_test(rho, P.rhoref, A.ctl, A.hist, i1, A.maxit, A.tol)) return;
    if (pend) {
      set_stop(A.ctl, PS_BREAKDOWN, i1);
      return;
    }
    A.ctl[C_ITER] = i1;
  }
};

// p-BiCGStab set-up: alpha_0 = (r0*, r0)/(r0*, w0), then the stop test at i = 0.
struct FinStabSetup {
  __device__ static void run(const DotArgs &A, const FinPre &P, const double (&d)[3]) {
    double *sc = A.sc;
    const double f = d[0], gw = d[1], rho = d[2];
    for (int j = 0; j < 3; ++j) sc[SC_DOTS + j] = d[j];
    const bool pend = bad_den(gw) || !isfinite(f / gw);
    sc[PS_S_ALPHA] = pend ? 0.0 : f / gw;
    sc[PS_S_BETA] = 0.0;
    sc[PS_S_OMEGA] = 0.0;
    sc[PS_S_F] = f;
    sc[PS_S_GW] = gw;
    sc[PS_S_GS] = 0.0;
    sc[PS_S_GZ] = 0.0;
    sc[PS_S_RHO] = rho;
    sc[PS_S_PENDING] = pend ? 1.0 : 0.0;
    if (A.flags & DF_SET_REF) sc[PS_S_RHOREF] = rho;
    if (!isfinite(f) || !isfinite(gw) || !isfinite(rho)) {
      A.hist[0] = NAN;
      set_stop(A.ctl, PS_NONFINITE, 0);
      return;
    }
    const double rhoref = (A.flags & DF_SET_REF) ? rho : P.rhoref;
    if (stop_test(rho, rhoref, A.ctl, A.hist, 0, A.maxit, A.tol)) return;
    if (pend) set_stop(A.ctl, PS_BREAKDOWN, 0);
  }
};

// Keep an initial guess only if ||b - A x0|| <= ||b|| (a non-finite residual
// does not qualify); otherwise the set-up continues from x0 = 0.
struct FinFallback {
  __device__ static void run(const DotArgs &A, const FinPre &, const double (&d)[2]) {
    A.sc[SC_FALLBACK] = (d[0] <= d[1]) ? 0.0 : 1.0;
  }
};

// The multiple c x0 of an initial guess with the least residual ||b - c A x0||:
// c = (A x0, b) / (A x0, A x0); when that cannot be formed (A x0 = 0, or a
// non-finite value) the scaled guess is zero.
struct FinScale {
  __device__ static void run(const DotArgs &A, const FinPre &, const double (&d)[2]) {
    const double c = d[0] / d[1];
    const bool ok = d[1] != 0.0 && isfinite(c);
    A.sc[SC_SCALE] = ok ? c : 0.0;
    A.sc[SC_SCALE_OK] = ok ? 1.0 : 0.0;
  }
};

// ||b||^2 as the stop-test reference
struct FinNormRef {
  __device__ static void run(const DotArgs &A, const FinPre &, const double (&d)[1]) { A.sc[PS_S_RHOREF] = d[0]; }
};

// ---------------------------------------------------------------- the kernel

template <class Prod>
__global__ __launch_bounds__(kBlock) void k_dots(DotArgs A) {
  constexpr int ND = Prod::ND;
  __shared__ double lds[kTdSlots * 9 * kPart];
  if (A.ctl[C_DONE]) return;
  TD acc[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = TD{0.0, 0.0, 0.0};
  // a pair of entries (16-byte loads) per thread per grid-stride step
  double a0[5], a1[5];
  const int64_t npair = A.n / 2;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < npair; p += stride) {
    load_in2<Prod::MASK>(A, 2 * p, a0, a1);
    Prod::acc(a0, acc);
    Prod::acc(a1, acc);
  }
  if ((A.n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    load_in<Prod::MASK>(A, A.n - 1, a0);
    Prod::acc(a0, acc);
  }
  const TD s = block_sum_td<ND>(acc, lds);
  const int G = gridDim.x;
  if (threadIdx.x < ND) {
    td_store(A.partials, threadIdx.x * G + blockIdx.x, s);
  }
}

// One block: add the G partial triples of each product in block order, round
// once, and run the phase's finish.  Every thread of the block calls it; lds
// holds kTdSlots * ND * kPart doubles.
template <int ND, class Fin>
__device__ __forceinline__ void finish_block(const DotArgs &A, int G, double *lds) {
  __shared__ double fin[ND];
  FinPre pre{};
  if (threadIdx.x == 0) pre = fin_preload(A);
  TD tot[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) tot[j] = TD{0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < G; b += kBlock) {
#pragma unroll
    for (int j = 0; j < ND; ++j)
      td_add(tot[j], td_load(A.partials, j * G + b));
  }
  const TD s = block_sum_td<ND>(tot, lds);
  if (threadIdx.x < ND) fin[threadIdx.x] = td_round(s);  // the one final rounding
  __syncthreads();
  if (threadIdx.x == 0) {
    double d[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) d[j] = fin[j];
    Fin::run(A, pre, d);
    if (A.ctl[C_DONE]) atomicSub(A.running, 1);
  }
}

template <int ND, class Fin>
__global__ __launch_bounds__(kBlock) void k_dots_finish(DotArgs A, int G) {
  __shared__ double lds[kTdSlots * 9 * kPart];
  if (A.ctl[C_DONE]) return;
  finish_block<ND, Fin>(A, G, lds);
}

// The fused schedules' finish when the partial lists are short: add pass A's
// (or the fused epilogue's) [5][ga] triples of (b, e, f, h, rho) and the
// epilogue's [4][gb] triples of (a, c, d, g) directly, without k_fold_partials --
// one launch fewer per iteration on small systems.
template <class Fin>
__global__ __launch_bounds__(kBlock) void k_dots_finish_direct(DotArgs A,
                                                               const double *__restrict__ pa,
                                                               int ga,
                                                               const double *__restrict__ pb,
                                                               int gb) {
  __shared__ double lds[kTdSlots * 9 * kPart];
  __shared__ double fin[9];
  if (A.ctl[C_DONE]) return;
  FinPre pre{};
  if (threadIdx.x == 0) pre = fin_preload(A);
  constexpr int kA[5] = {1, 4, 5, 7, 8};
  constexpr int kB[4] = {0, 2, 3, 6};
  TD tot[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) tot[j] = TD{0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < ga; b += kBlock) {
#pragma unroll
    for (int j = 0; j < 5; ++j) td_add(tot[kA[j]], td_load(pa, j * ga + b));
  }
  for (int b = threadIdx.x; b < gb; b += kBlock) {
#pragma unroll
    for (int j = 0; j < 4; ++j) td_add(tot[kB[j]], td_load(pb, j * gb + b));
  }
  const TD s = block_sum_td<9>(tot, lds);
  if (threadIdx.x < 9) fin[threadIdx.x] = td_round(s);  // the one final rounding
  __syncthreads();
  if (threadIdx.x == 0) {
    double d[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) d[j] = fin[j];
    Fin::run(A, pre, d);
    if (A.ctl[C_DONE]) atomicSub(A.running, 1);
  }
}

// ------------------------------------------------------- batched solves
// Every system is padded to a multiple of 512 rows, so workgroup b (rows
// 512 b .. 512 b + 511, one pair per lane) lies in one system; it writes its
// partial sums, or nothing once its system has stopped.
template <class Prod>
__global__ __launch_bounds__(kBlock) void k_dots_batch(DotArgs A, const int *__restrict__ chunk_sys) {
  constexpr int ND = Prod::ND;
  __shared__ double lds[kTdSlots * 9 * kPart];
  const int sys = chunk_sys[2 * blockIdx.x];
  if (A.ctl[(size_t)sys * C_COUNT + C_DONE]) return;
  TD acc[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = TD{0.0, 0.0, 0.0};
  double a0[5], a1[5];
  load_in2<Prod::MASK>(A, 2 * ((int64_t)blockIdx.x * kBlock + threadIdx.x), a0, a1);
  Prod::acc(a0, acc);
  Prod::acc(a1, acc);
  const TD s = block_sum_td<ND>(acc, lds);
  const int G = gridDim.x;
  if (threadIdx.x < ND) {
    td_store(A.partials, threadIdx.x * G + blockIdx.x, s);
  }
}

// One workgroup per system: add the partials of the system's workgroups
// first_blk[k] .. first_blk[k+1]-1 (G in all) in order, round once, and run
// the phase's finish on the system's control and scalar blocks and history.
template <int ND, class Fin>
__global__ __launch_bounds__(kBlock) void k_dots_finish_batch(DotArgs A, const int *__restrict__ first_blk,
                                                              int G, int64_t hist_stride) {
  __shared__ double lds[kTdSlots * 9 * kPart];
  __shared__ double fin[9];
  const int k = blockIdx.x;
  DotArgs Ak = A;
  Ak.ctl += (size_t)k * C_COUNT;
  Ak.sc += (size_t)k * SC_COUNT;
  Ak.hist += k * hist_stride;
  if (Ak.ctl[C_DONE]) return;
  FinPre pre{};
  if (threadIdx.x == 0) pre = fin_preload(Ak);
  TD tot[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) tot[j] = TD{0.0, 0.0, 0.0};
  for (int b = first_blk[k] + threadIdx.x; b < first_blk[k + 1]; b += kBlock) {
#pragma unroll
    for (int j = 0; j < ND; ++j)
      td_add(tot[j], td_load(A.partials, j * G + b));
  }
  const TD s = block_sum_td<ND>(tot, lds);
  if (threadIdx.x < ND) fin[threadIdx.x] = td_round(s);
  __syncthreads();
  if (threadIdx.x == 0) {
    double d[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) d[j] = fin[j];
    Fin::run(Ak, pre, d);
    if (Ak.ctl[C_DONE]) atomicSub(A.running, 1);
  }
}

// Batched fused schedules: per system k (one workgroup each), add its range of
// the [5][ga] triples of (b, e, f, h, rho) -- workgroups a_first[k] ..
// a_first[k+1]-1 -- and of the [4][gb] triples of (a, c, d, g) -- b_first[k] ..
// b_first[k+1]-1 -- and run the system's finish.
template <class Fin>
__global__ __launch_bounds__(kBlock) void k_dots_finish_batch_direct(
    DotArgs A, const double *__restrict__ pa, int ga, const int *__restrict__ a_first,
    const double *__restrict__ pb, int gb, const int *__restrict__ b_first, int64_t hist_stride) {
  __shared__ double lds[kTdSlots * 9 * kPart];
  __shared__ double fin[9];
  const int k = blockIdx.x;
  DotArgs Ak = A;
  Ak.ctl += (size_t)k * C_COUNT;
  Ak.sc += (size_t)k * SC_COUNT;
  Ak.hist += k * hist_stride;
  if (Ak.ctl[C_DONE]) return;
  FinPre pre{};
  if (threadIdx.x == 0) pre = fin_preload(Ak);
  constexpr int kA[5] = {1, 4, 5, 7, 8};
  constexpr int kB[4] = {0, 2, 3, 6};
  TD tot[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) tot[j] = TD{0.0, 0.0, 0.0};
  for (int b = a_first[k] + threadIdx.x; b < a_first[k + 1]; b += kBlock) {
#pragma unroll
    for (int j = 0; j < 5; ++j) td_add(tot[kA[j]], td_load(pa, j * ga + b));
  }
  for (int b = b_first[k] + threadIdx.x; b < b_first[k + 1]; b += kBlock) {
#pragma unroll
    for (int j = 0; j < 4; ++j) td_add(tot[kB[j]], td_load(pb, j * gb + b));
  }
  const TD s = block_sum_td<9>(tot, lds);
  if (threadIdx.x < 9) fin[threadIdx.x] = td_round(s);
  __syncthreads();
  if (threadIdx.x == 0) {
    double d[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) d[j] = fin[j];
    Fin::run(Ak, pre, d);
    if (Ak.ctl[C_DONE]) atomicSub(A.running, 1);
  }
}

constexpr int kFoldPerThread = 1;

// Fused-dot schedule: the nine inner products of iteration i arrive as block
// partial sums from the two passes of iteration i-1 -- pass A: [5][ga] triples of
// (b, e, f, h, rho), the epilogue of A w_{i-1}: [4][gb] triples of (a, c, d, g).
// This kernel folds them into [9][gridDim.x] triples in the layout k_dots
// writes (block k takes entries k*kFoldPerThread*kBlock .. of every list,
// kFoldPerThread per thread), so the same one-block finish follows.
// Slice `slice` of the fold: entries slice*kFoldPerThread*kBlock .. of every list,
// added into out[j * G + slice] (G slices in all).  All threads of the block take part.
__device__ __forceinline__ void fold_slice(const double *__restrict__ pa, int ga,
                                           const double *__restrict__ pb, int gb,
                                           double *__restrict__ out, int G, int slice,
                                           double *lds) {
  constexpr int kA[5] = {1, 4, 5, 7, 8};
  constexpr int kB[4] = {0, 2, 3, 6};
  TD t[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) t[j] = TD{0.0, 0.0, 0.0};
  // kFoldPerThread entries of every list per thread, kBlock apart
#pragma unroll
  for (int q = 0; q < kFoldPerThread; ++q) {
    const int idx = (slice * kFoldPerThread + q) * kBlock + threadIdx.x;
    if (idx < ga) {
#pragma unroll
      for (int j = 0; j < 5; ++j) td_add(t[kA[j]], td_load(pa, j * ga + idx));
    }
    if (idx < gb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) td_add(t[kB[j]], td_load(pb, j * gb + idx));
    }
  }
  const TD s = block_sum_td<9>(t, lds);
  if (threadIdx.x < 9) td_store(out, threadIdx.x * G + slice, s);
}

__global__ __launch_bounds__(kBlock) void k_fold_partials(const double *__restrict__ pa, int ga,
                                                          const double *__restrict__ pb, int gb,
                                                          double *__restrict__ out,
                                                          const int *__restrict__ ctl) {
  __shared__ double lds[kTdSlots * 9 * kPart];
  if (ctl[C_DONE]) return;
  fold_slice(pa, ga, pb, gb, out, gridDim.x, blockIdx.x, lds);
}

// Lean sums of a reduction phase's ND products for use inside a sparse product
// (the single-stream schedule), where the fold and finish must stay short and
// use few registers: one triple accumulator per thread, no per-product register
// arrays.  kPer threads work for each product (thread t for product t / kPer)
// and add their entries sequentially; those partials go through LDS, where lane
// 4j + q of wavefront 0 adds a quarter of product j's, and two quad steps add
// the four quarters.  The order differs from block_sum_td's, which the triple
// accumulators make immaterial: the final rounding gives each product rounded
// once from its exact value either way (see TD).
template <int ND>
struct Lean {
  static_assert(ND >= 1 && 4 * ND <= kWave, "the quarters of every product in one wavefront");
  static constexpr int kPer = ((kBlock / ND) & ~3) < 64 ? ((kBlock / ND) & ~3) : 64;
};
constexpr int kLeanLds = kBlock * kPart;  // doubles of LDS the lean sums use (ND * kPer <= kBlock)

// Thread (j, s) = (t / kPer, t % kPer) holds a partial of product j; on return
// lane 4j of wavefront 0 (j < ND) holds product j's total.  Every thread calls it.
template <int ND>
__device__ __forceinline__ TD lean_sum(const TD &acc, double *lds) {
  constexpr int P = Lean<ND>::kPer;
  const int t = threadIdx.x;
  if (t < ND * P) td_store(lds, t, acc);
  __syncthreads();
  TD r{0.0, 0.0, 0.0};
  if (t < 4 * ND) {
    const int base = (t >> 2) * P + (t & 3) * (P / 4);
    r = td_load(lds, base);
    for (int k = 1; k < P / 4; ++k) td_add(r, td_load(lds, base + k));
  }
  if (t < kWave) {  // the lanes past 4 ND add zeros
    td_step<0xB1>(r);  // quad_perm [1,0,3,2]
    td_step<0x4E>(r);  // quad_perm [2,3,0,1]
  }
  __syncthreads();  // lds free again
  return r;
}

// The partial lists a fold reads: product j comes from list pb if bit j of
// from_b is set, else from pa, at row (rows >> 4j) & 15 of that list; each row
// of pa holds ga triples, each of pb gb.
struct FoldLists {
  const double *pa, *pb;
  int ga, gb;
  unsigned from_b;
  unsigned long long rows;
};

// Slice `slice` of the fold (kBlock entries of every list) into out[j * G + slice].
template <int ND>
__device__ __forceinline__ void fold_lean(const FoldLists &L, double *__restrict__ out, int G,
                                          int slice, double *lds) {
  static_assert(kFoldPerThread == 1, "a slice is kBlock entries of every list");
  constexpr int P = Lean<ND>::kPer;
  const int t = threadIdx.x;
  TD acc{0.0, 0.0, 0.0};
  if (t < ND * P) {
    const int j = t / P, s = t % P;
    const bool from_b = (L.from_b >> j) & 1u;
    const int len = from_b ? L.gb : L.ga;
    const double *src = (from_b ? L.pb : L.pa) + (size_t)((L.rows >> (4 * j)) & 15u) * len * kPart;
    for (int e = s; e < kBlock; e += P) {
      const int idx = slice * kBlock + e;
      if (idx < len) td_add(acc, td_load(src, idx));
    }
  }
  const TD r = lean_sum<ND>(acc, lds);
  if (t < 4 * ND && (t & 3) == 0) td_store(out, (int64_t)(t >> 2) * G + slice, r);
}

// The G folded triples of each product, rounded once into fin[0 .. ND-1].
template <int ND>
__device__ __forceinline__ void finish_lean(const double *__restrict__ partials, int G,
                                            double *lds, double *fin) {
  constexpr int P = Lean<ND>::kPer;
  const int t = threadIdx.x;
  TD acc{0.0, 0.0, 0.0};
  if (t < ND * P) {
    const int j = t / P, s = t % P;
    for (int b = s; b < G; b += P) td_add(acc, td_load(partials, (int64_t)j * G + b));
  }
  const TD r = lean_sum<ND>(acc, lds);
  if (t < 4 * ND && (t & 3) == 0) fin[t >> 2] = td_round(r);  // the one final rounding
}

// Fold and finish inside another kernel (the single-stream schedule): workgroup
// `slice` (< G) folds its slice of the lists into F.partials ([ND][G]); the
// workgroup that completes the last slice -- counted in the control word
// C_FOLDS, which it resets for the next phase -- then adds the G slices and
// runs Fin, as k_fold_partials and k_dots_finish would (with the lean sums).
// No workgroup waits for another: the others go on with their own work.  A
// release fence before the count and an acquire fence after the last count
// make every slice visible to the last workgroup, whichever XCD and L2 wrote
// it.  Every thread of the block calls it; lds holds kLeanLds doubles.
template <int ND, class Fin>
__device__ __forceinline__ void fold_then_finish(const FoldLists &L, const DotArgs &F, int G,
                                                 int slice, double *lds) {
  __shared__ int last;
  __shared__ double fin[ND];
  if (F.ctl[C_DONE]) return;  // the same answer in every fold workgroup (nothing else runs)
  fold_lean<ND>(L, F.partials, G, slice, lds);
  __syncthreads();  // the slice's stores (lanes 0, 4, ..) are done
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int before = atomicAdd(&F.ctl[C_FOLDS], 1);
    last = before == G - 1;
    if (last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      atomicExch(&F.ctl[C_FOLDS], 0);
    }
  }
  __syncthreads();
  if (!last) return;
  FinPre pre{};
  if (threadIdx.x == 0) pre = fin_preload(F);
  finish_lean<ND>(F.partials, G, lds, fin);
  __syncthreads();
  if (threadIdx.x == 0) {
    double d[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) d[j] = fin[j];
    Fin::run(F, pre, d);
    if (F.ctl[C_DONE]) atomicSub(F.running, 1);
  }
}

// The fold and finish as a kernel of their own, over G = gridDim.x slices: the
// finish of the separate inner-product pass (its [ND][dot grid] triples, G =
// the dot grid / kBlock rounded up), where the lean sums of a few workgroups
// take less time than k_dots_finish's one-workgroup sum (ssBiCGSafe2, whose
// reduction phase is on the main stream: 128^3 134.7 -> 132.7 us per
// iteration, 96^3 70.4 -> 68.4).
template <int ND, class Fin>
__global__ __launch_bounds__(kBlock) void k_fold_finish(FoldLists L, DotArgs F) {
  __shared__ double lds[kLeanLds];
  fold_then_finish<ND, Fin>(L, F, (int)gridDim.x, (int)blockIdx.x, lds);
}

// The lists of the BiCGSafe schedules: the fused epilogue's [5][ga] triples of
// (b, e, f, h, rho) and [4][gb] of (a, c, d, g), in the order of ProdSafe9
constexpr unsigned kSafeFromB = 0x4Du;                   // products 0, 2, 3, 6 from pb
constexpr unsigned long long kSafeRows = 0x433212100ull;  // rows 0,0,1,2,1,2,3,3,4

}  // namespace ps
