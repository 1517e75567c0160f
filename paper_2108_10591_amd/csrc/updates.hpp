// Fused, row-local vector-update passes.  Each kernel streams every vector it
// needs once (two entries per thread, 16-byte loads and stores) and applies a
// whole block of the algorithm's update statements per entry, in the
// algorithm's order, so no intermediate vector makes an HBM round trip.
#pragma once

#include "device_common.hpp"

namespace ps {

template <int W>
__device__ __forceinline__ void ldv(const double *__restrict__ p, int64_t k, double (&o)[W]) {
  if constexpr (W == 2) {
    const double2 v = *reinterpret_cast<const double2 *>(p + k);
    o[0] = v.x;
    o[1] = v.y;
  } else {
    o[0] = p[k];
  }
}

template <int W>
__device__ __forceinline__ void stv(double *__restrict__ p, int64_t k, const double (&o)[W]) {
  if constexpr (W == 2) {
    *reinterpret_cast<double2 *>(p + k) = make_double2(o[0], o[1]);
  } else {
    p[k] = o[0];
  }
}

// Streaming (nontemporal) forms, for vectors that no kernel reads again before
// the next iteration's pass: on systems whose iteration traffic is well above
// the last-level cache, keeping their lines only evicts the ones that are
// read again soon (the matrix, the SpMV inputs, the epilogue's operands).
typedef double d2v __attribute__((ext_vector_type(2)));

template <int W, bool NT>
__device__ __forceinline__ void ldv_s(const double *__restrict__ p, int64_t k, double (&o)[W]) {
  if constexpr (!NT) {
    ldv<W>(p, k, o);
  } else if constexpr (W == 2) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p + k));
    o[0] = v.x;
    o[1] = v.y;
  } else {
    o[0] = __builtin_nontemporal_load(p + k);
  }
}

template <int W, bool NT>
__device__ __forceinline__ void stv_s(double *__restrict__ p, int64_t k, const double (&o)[W]) {
  if constexpr (!NT) {
    stv<W>(p, k, o);
  } else if constexpr (W == 2) {
    const d2v v = {o[0], o[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<d2v *>(p + k));
  } else {
    __builtin_nontemporal_store(o[0], p + k);
  }
}

// Vectors held as FP32 numbers (precision 3: p, u, z): loaded and widened
// exactly, rounded to the nearest FP32 number (ties to even) when stored.  ZT is
// the stored type, double or float; the arithmetic is FP64 either way.
typedef float f2v __attribute__((ext_vector_type(2)));

template <int W, bool NT, class ZT>
__device__ __forceinline__ void ldz(const double *__restrict__ p, int64_t k, double (&o)[W]) {
  if constexpr (sizeof(ZT) == 8) {
    ldv_s<W, NT>(p, k, o);
  } else {
    const float *q = reinterpret_cast<const float *>(p);
    if constexpr (W == 2) {
      const f2v v = NT ? __builtin_nontemporal_load(reinterpret_cast<const f2v *>(q + k))
                       : *reinterpret_cast<const f2v *>(q + k);
      o[0] = (double)v.x;
      o[1] = (double)v.y;
    } else {
      o[0] = (double)(NT ? __builtin_nontemporal_load(q + k) : q[k]);
    }
  }
}

template <int W, bool NT, class ZT>
__device__ __forceinline__ void stz(double *__restrict__ p, int64_t k, const double (&o)[W]) {
  if constexpr (sizeof(ZT) == 8) {
    stv_s<W, NT>(p, k, o);
  } else {
    float *q = reinterpret_cast<float *>(p);
    if constexpr (W == 2) {
      const f2v v = {(float)o[0], (float)o[1]};
      if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<f2v *>(q + k));
      else *reinterpret_cast<f2v *>(q + k) = v;
    } else {
      if constexpr (NT) __builtin_nontemporal_store((float)o[0], q + k);
      else q[k] = (float)o[0];
    }
  }
}

// the value a vector of stored type ZT holds for v: v itself, or the FP32 number
// nearest to it
template <class ZT>
__device__ __forceinline__ double held(double v) {
  if constexpr (sizeof(ZT) == 8) return v;
  else return (double)(float)v;
}

// A kernel that follows a reduction phase: if that phase stopped the solve
// (of the workgroup's system), note it in C_HALT (read by the sparse products
// of later iterations, which may run concurrently with a finish and so must
// not read C_DONE) and return.  Every workgroup that sees the stop writes the
// same value.
__device__ __forceinline__ bool halted_after_finish(int *ctl) {
  if (ctl[C_DONE]) {
    if (threadIdx.x == 0) ctl[C_HALT] = 1;
    return true;
  }
  return false;
}

// The arguments with the scalar and control blocks of the system that the
// workgroup's 512 rows belong to (batched solves; chunk_sys = nullptr: one
// system).
// The pair block (512 rows) this workgroup of a streaming pass takes: the
// products' XCD-aware order (xcd_block), walked in the sweep direction.
__device__ __forceinline__ int pass_block(int rev) {
  return sweep_block(xcd_block((int)blockIdx.x, (int)gridDim.x), (int)gridDim.x, rev);
}

template <class Args>
__device__ __forceinline__ Args bind_system(Args P) {
  if (P.chunk_sys) {
    const int sys = P.chunk_sys[2 * pass_block(P.rev)];
    P.sc += (size_t)sys * SC_COUNT;
    P.ctl += (size_t)sys * C_COUNT;
  }
  return P;
}

// Entry index of this thread (two entries per thread), blocks taken in the
// sweep direction `rev`.
__device__ __forceinline__ int64_t pair_index(int rev) {
  const int b = pass_block(rev);
  return 2 * ((int64_t)b * kBlock + threadIdx.x);
}

#define PS_DISPATCH_PAIRS(n, body)            \
  do {                                        \
    const int64_t k_ = pair_index(P.rev);     \
    if (k_ + 1 < (n)) {                       \
      body<2>(P, k_);                         \
    } else if (k_ < (n)) {                    \
      body<1>(P, k_);                         \
    }                                         \
  } while (0)

// ------------------------------------------------ p-BiCGSafe, Algorithm 4
// The ten updates between the reduction phase and the product A w_i:
//   p_i = r_i + beta (p_{i-1} - u_{i-1})         o_i = s_i + beta t_{i-1}
//   u_i = zeta o_i + eta (y_i + beta u_{i-1})    q_i = As_i + beta l_{i-1}       (Eq. (q))
//   w_i = zeta q_i + eta (g_i + beta w_{i-1})    (Eq. (w))
//   t_i = o_i - w_i                              z_i = zeta r_i + eta z_{i-1} - alpha u_i
//   y_{i+1} = zeta s_i + eta y_i - alpha w_i     x_{i+1} = x_i + alpha p_i + z_i
//   r_{i+1} = r_i - alpha o_i - y_{i+1}
// o_i and q_i stay in registers: the epilogue of A w_i forms q_i again from
// the same operands (As_i, l_{i-1}), which it reads anyway.
struct PassAArgs {
  double *x, *r, *p, *u, *t, *y, *z, *w;
  const double *s, *As, *l, *g;
  const double *sc;
  int *ctl;
  int64_t n;
  int rev;  // sweep direction
  // fused inner products (k_passA_pbicgsafe<true, NT> only): r0* and the
  // [5][gridDim.x] (a, b, c) partial sums of the next iteration's
  // b = (y,y), e = (y,r), f = (r0*,r), h = (r0*,t), rho = (r,r)
  const double *rs;
  double *part;
  const int *chunk_sys;  // system of each 256-row chunk (batched solves), or nullptr
};

template <int W, bool DOTS, bool NT, class ZT>
__device__ __forceinline__ void passA_body(const PassAArgs &P, int64_t k, TD (&acc)[5]) {
  const double al = P.sc[PS_S_ALPHA], be = P.sc[PS_S_BETA], ze = P.sc[PS_S_ZETA],
               et = P.sc[PS_S_ETA];
  double r[W], p[W], u[W], s[W], t[W], y[W], As[W], l[W], g[W], w[W], z[W], x[W], q[W];
  ldv<W>(P.r, k, r);
  ldz<W, NT, ZT>(P.p, k, p);
  ldz<W, NT, ZT>(P.u, k, u);
  ldv<W>(P.s, k, s);
  ldv_s<W, NT>(P.t, k, t);
  ldv<W>(P.y, k, y);
  ldv<W>(P.As, k, As);
  ldv<W>(P.l, k, l);
  ldv<W>(P.g, k, g);
  ldv<W>(P.w, k, w);
  ldz<W, NT, ZT>(P.z, k, z);
  ldv_s<W, NT>(P.x, k, x);
#pragma unroll
  for (int j = 0; j < W; ++j) {
    // directions and Eqs. (q), (w); then the residuals and the iterate
    const double o = s[j] + be * t[j];
    p[j] = held<ZT>(r[j] + be * (p[j] - u[j]));
    u[j] = held<ZT>(ze * o + et * (y[j] + be * u[j]));
    q[j] = As[j] + be * l[j];
    w[j] = ze * q[j] + et * (g[j] + be * w[j]);
    t[j] = o - w[j];
    z[j] = held<ZT>(ze * r[j] + et * z[j] - al * u[j]);
    y[j] = ze * s[j] + et * y[j] - al * w[j];
    x[j] = x[j] + al * p[j] + z[j];
    r[j] = r[j] - al * o - y[j];
  }
  if constexpr (DOTS) {
    double rs[W];
    ldv<W>(P.rs, k, rs);
#pragma unroll
    for (int j = 0; j < W; ++j) {
      td_fma(acc[0], y[j], y[j]);
      td_fma(acc[1], y[j], r[j]);
      td_fma(acc[2], rs[j], r[j]);
      td_fma(acc[3], rs[j], t[j]);
      td_fma(acc[4], r[j], r[j]);
    }
  }
  stz<W, NT, ZT>(P.p, k, p);
  stz<W, NT, ZT>(P.u, k, u);
  stv<W>(P.w, k, w);
  stv_s<W, NT>(P.t, k, t);
  stz<W, NT, ZT>(P.z, k, z);
  stv<W>(P.y, k, y);
  stv_s<W, NT>(P.x, k, x);
  stv<W>(P.r, k, r);
}

// NT: p, u, t, z, x (read and written here, next read by the next pass A)
// stream past the cache.  ZT: the stored type of p, u, z.
template <bool DOTS, bool NT, class ZT = double>
__global__ __launch_bounds__(kBlock) void k_passA_pbicgsafe(PassAArgs P_) {
  const PassAArgs P = bind_system(P_);
  if (halted_after_finish(P.ctl)) return;
  TD acc[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) acc[j] = TD{0.0, 0.0, 0.0};
  const int b = pass_block(P.rev);
  const int64_t k = 2 * ((int64_t)b * kBlock + threadIdx.x);
  if (k + 1 < P.n) passA_body<2, DOTS, NT, ZT>(P, k, acc);
  else if (k < P.n) passA_body<1, DOTS, NT, ZT>(P, k, acc);
  if constexpr (DOTS) {
    __shared__ double red[kTdSlots * 5 * kPart];
    const TD t = block_sum_td<5>(acc, red);
    const int G = gridDim.x;
    if (threadIdx.x < 5) {
      td_store(P.part, threadIdx.x * G + b, t);
    }
  }
}

// ---------------------------------- p-BiCGSafe, fused-epilogue schedule: only
// w_i = zeta q_i + eta (g_i + beta w_{i-1}), q_i = As_i + beta l_{i-1} (Eqs. (q),
// (w)) has to exist for every row before the product A w_i; this pass forms it
// alone, and the product's epilogue (EpiPBiCGSafeAll) makes every other update
// of the iteration.
struct PassWArgs {
  const double *As, *l, *g;
  double *w;
  const double *sc;
  int *ctl;
  int64_t n;
  int rev;               // sweep direction
  const int *chunk_sys;  // system of each 256-row chunk (batched solves), or nullptr
};

// w_i from A s_i, l_{i-1}, g_{i-1}, w_{i-1} (Eqs. (q), (w): q_i = A s_i + beta l_{i-1})
__device__ __forceinline__ double w_next(double As, double l, double g, double w, double be,
                                         double ze, double et) {
  const double q = As + be * l;
  return ze * q + et * (g + be * w);
}

template <int W>
__device__ __forceinline__ void passW_body(const PassWArgs &P, int64_t k) {
  const double be = P.sc[PS_S_BETA], ze = P.sc[PS_S_ZETA], et = P.sc[PS_S_ETA];
  double As[W], l[W], g[W], w[W];
  ldv<W>(P.As, k, As);
  ldv<W>(P.l, k, l);
  ldv<W>(P.g, k, g);
  ldv<W>(P.w, k, w);
#pragma unroll
  for (int j = 0; j < W; ++j) w[j] = w_next(As[j], l[j], g[j], w[j], be, ze, et);
  stv<W>(P.w, k, w);
}

__global__ __launch_bounds__(kBlock) void k_pass_w(PassWArgs P_) {
  const PassWArgs P = bind_system(P_);
  if (halted_after_finish(P.ctl)) return;
  const int b = pass_block(P.rev);
  const int64_t k = 2 * ((int64_t)b * kBlock + threadIdx.x);
  if (k + 1 < P.n) passW_body<2>(P, k);
  else if (k < P.n) passW_body<1>(P, k);
}

// ---------------------------------- ssBiCGSafe2 (Algorithm 3) and the
// replacement step of Algorithm 5: p_i, o_i, u_i before the product A u_i.
struct PouArgs {
  const double *r, *s, *t, *y;
  double *p, *u;
  double *o;  // stored only when a later kernel needs A o_i (replacement step)
  double *u_wide;  // p, u held in FP32 (k_pou<float>): u widened, for the product A u_i
  const double *sc;
  int *ctl;
  int64_t n;
  int rev;  // sweep direction
  const int *chunk_sys;  // system of each 256-row chunk (batched solves), or nullptr
};

template <int W, bool STORE_O, class ZT = double>
__device__ __forceinline__ void pou_body(const PouArgs &P, int64_t k) {
  const double be = P.sc[PS_S_BETA], ze = P.sc[PS_S_ZETA], et = P.sc[PS_S_ETA];
  double r[W], p[W], u[W], s[W], t[W], y[W], o[W];
  ldv<W>(P.r, k, r);
  ldz<W, false, ZT>(P.p, k, p);
  ldz<W, false, ZT>(P.u, k, u);
  ldv<W>(P.s, k, s);
  ldv<W>(P.t, k, t);
  ldv<W>(P.y, k, y);
#pragma unroll
  for (int j = 0; j < W; ++j) {
    o[j] = s[j] + be * t[j];
    p[j] = held<ZT>(r[j] + be * (p[j] - u[j]));
    u[j] = held<ZT>(ze * o[j] + et * (y[j] + be * u[j]));
  }
  stz<W, false, ZT>(P.p, k, p);
  stz<W, false, ZT>(P.u, k, u);
  if (STORE_O) stv<W>(P.o, k, o);
  if constexpr (sizeof(ZT) == 4) stv<W>(P.u_wide, k, u);
}

template <int W>
__device__ __forceinline__ void pou_body_noo(const PouArgs &P, int64_t k) {
  pou_body<W, false>(P, k);
}
template <int W>
__device__ __forceinline__ void pou_body_o(const PouArgs &P, int64_t k) {
  pou_body<W, true>(P, k);
}
template <int W>
__device__ __forceinline__ void pou_body_o32(const PouArgs &P, int64_t k) {
  pou_body<W, true, float>(P, k);
}

__global__ __launch_bounds__(kBlock) void k_pu(PouArgs P_) {
  const PouArgs P = bind_system(P_);
  if (halted_after_finish(P.ctl)) return;
  PS_DISPATCH_PAIRS(P.n, pou_body_noo);
}

__global__ __launch_bounds__(kBlock) void k_pou(PouArgs P_) {
  const PouArgs P = bind_system(P_);
  if (halted_after_finish(P.ctl)) return;
  PS_DISPATCH_PAIRS(P.n, pou_body_o);
}

// k_pou with p, u held in FP32 (and u also written widened to P.u_wide)
__global__ __launch_bounds__(kBlock) void k_pou32(PouArgs P_) {
  const PouArgs P = bind_system(P_);
  if (halted_after_finish(P.ctl)) return;
  PS_DISPATCH_PAIRS(P.n, pou_body_o32);
}

// replacement step of Algorithm 5, after q_i = A o_i and w_i = A u_i:
//   t_i = o_i - w_i, z_i = zeta r_i + eta z_{i-1} - alpha u_i,
//   y_{i+1} = zeta s_i + eta y_i - alpha w_i, x_{i+1} = x_i + alpha p_i + z_i
struct TzyxArgs {
  const double *o, *w, *r, *u, *s, *p;
  double *t, *z, *y, *x;
  const double *sc;
  int *ctl;
  int64_t n;
  int rev;  // sweep direction
  const int *chunk_sys;  // system of each 256-row chunk (batched solves), or nullptr
};

template <int W, class ZT = double>
__device__ __forceinline__ void tzyx_body(const TzyxArgs &P, int64_t k) {
  const double al = P.sc[PS_S_ALPHA], ze = P.sc[PS_S_ZETA], et = P.sc[PS_S_ETA];
  double o[W], w[W], r[W], u[W], s[W], p[W], t[W], z[W], y[W], x[W];
  ldv<W>(P.o, k, o);
  ldv<W>(P.w, k, w);
  ldv<W>(P.r, k, r);
  ldz<W, false, ZT>(P.u, k, u);
  ldv<W>(P.s, k, s);
  ldz<W, false, ZT>(P.p, k, p);
  ldz<W, false, ZT>(P.z, k, z);
  ldv<W>(P.y, k, y);
  ldv<W>(P.x, k, x);
#pragma unroll
  for (int j = 0; j < W; ++j) {
    t[j] = o[j] - w[j];
    z[j] = held<ZT>(ze * r[j] + et * z[j] - al * u[j]);
    y[j] = ze * s[j] + et * y[j] - al * w[j];
    x[j] = x[j] + al * p[j] + z[j];
  }
  stv<W>(P.t, k, t);
  stz<W, false, ZT>(P.z, k, z);
  stv<W>(P.y, k, y);
  stv<W>(P.x, k, x);
}
template <int W>
__device__ __forceinline__ void tzyx_body32(const TzyxArgs &P, int64_t k) {
  tzyx_body<W, float>(P, k);
}

__global__ __launch_bounds__(kBlock) void k_tzyx(TzyxArgs P_) {
  const TzyxArgs P = bind_system(P_);
  if (P.ctl[C_DONE]) return;
  PS_DISPATCH_PAIRS(P.n, tzyx_body);
}

// k_tzyx with u, p, z held in FP32
__global__ __launch_bounds__(kBlock) void k_tzyx32(TzyxArgs P_) {
  const TzyxArgs P = bind_system(P_);
  if (P.ctl[C_DONE]) return;
  PS_DISPATCH_PAIRS(P.n, tzyx_body32);
}

// conversions of a vector slot between FP64 and FP32 storage (through a scratch
// slot: the FP32 numbers occupy the first half of the slot's bytes)
__global__ __launch_bounds__(kBlock) void k_narrow(float *__restrict__ dst,
                                                   const double *__restrict__ src, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[k] = (float)src[k];
}
__global__ __launch_bounds__(kBlock) void k_widen(double *__restrict__ dst,
                                                  const float *__restrict__ src, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[k] = (double)src[k];
}

// --------------------------------------------------- pipelined BiCGStab
// pass 1 of iteration i (after the stop test on rho_i):
//   p_i = r_i + beta (p - omega s),  s_i = w_i + beta (s - omega z),
//   z_i = t_i + beta (z - omega v),  q_i = r_i - alpha s_i,  y_i = w_i - alpha z_i
// With DOTS (the single-stream schedule) it also forms the block partial sums
// of the inner products whose vectors it has just written: [4][gridDim.x]
// triples of (q, y), (y, y) -- phase 1 -- and (r0*, s), (r0*, z) -- two of
// phase 2's, whose s and z nothing changes before that phase.
// NT: p, s, q, y (next read by pass 2 or the next pass 1) stream past the
// cache, so that it keeps the matrix, which both products read, and z, w, v, t,
// r (cd3d 128^3: 144.0 -> 117.7 us per iteration with the single-stream
// schedule); pass 2 streams p, q, y and x.
struct Stab1Args {
  const double *r, *w, *t, *v;
  double *p, *s, *z, *q, *y;
  const double *sc;
  int *ctl;
  int64_t n;
  int rev;  // sweep direction
  const int *chunk_sys;  // system of each 256-row chunk (batched solves), or nullptr
  const double *rs;      // r0* (DOTS)
  double *part;          // partial sums (DOTS)
};

template <int W, bool DOTS, bool NT>
__device__ __forceinline__ void stab1_body(const Stab1Args &P, int64_t k, TD (&acc)[4]) {
  const double al = P.sc[PS_S_ALPHA], be = P.sc[PS_S_BETA], om = P.sc[PS_S_OMEGA];
  double r[W], w[W], t[W], v[W], p[W], s[W], z[W], q[W], y[W];
  ldv<W>(P.r, k, r);
  ldv<W>(P.w, k, w);
  ldv<W>(P.t, k, t);
  ldv<W>(P.v, k, v);
  ldv_s<W, NT>(P.p, k, p);
  ldv_s<W, NT>(P.s, k, s);
  ldv<W>(P.z, k, z);
#pragma unroll
  for (int j = 0; j < W; ++j) {
    p[j] = r[j] + be * (p[j] - om * s[j]);
    s[j] = w[j] + be * (s[j] - om * z[j]);
    z[j] = t[j] + be * (z[j] - om * v[j]);
    q[j] = r[j] - al * s[j];
    y[j] = w[j] - al * z[j];
  }
  if constexpr (DOTS) {
    double rs[W];
    ldv<W>(P.rs, k, rs);
#pragma unroll
    for (int j = 0; j < W; ++j) {
      td_fma(acc[0], q[j], y[j]);
      td_fma(acc[1], y[j], y[j]);
      td_fma(acc[2], rs[j], s[j]);
      td_fma(acc[3], rs[j], z[j]);
    }
  }
  stv_s<W, NT>(P.p, k, p);
  stv_s<W, NT>(P.s, k, s);
  stv<W>(P.z, k, z);
  stv_s<W, NT>(P.q, k, q);
  stv_s<W, NT>(P.y, k, y);
}

// The partial sums of a pass's block: [ND][gridDim.x] triples, block b's at
// column b.
template <int ND>
__device__ __forceinline__ void store_pass_partials(TD (&acc)[ND], double *part, int b) {
  __shared__ double red[kTdSlots * ND * kPart];
  const TD t = block_sum_td<ND>(acc, red);
  if (threadIdx.x < ND) td_store(part, (int64_t)threadIdx.x * gridDim.x + b, t);
}

template <bool DOTS, bool NT>
__global__ __launch_bounds__(kBlock) void k_stab_pass1(Stab1Args P_) {
  const Stab1Args P = bind_system(P_);
  if (halted_after_finish(P.ctl)) return;
  TD acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = TD{0.0, 0.0, 0.0};
  const int b = pass_block(P.rev);
  const int64_t k = 2 * ((int64_t)b * kBlock + threadIdx.x);
  if (k + 1 < P.n) stab1_body<2, DOTS, NT>(P, k, acc);
  else if (k < P.n) stab1_body<1, DOTS, NT>(P, k, acc);
  if constexpr (DOTS) store_pass_partials<4>(acc, P.part, b);
}

// pass 2 of iteration i (after omega_i):
//   x_{i+1} = x_i + alpha p_i + omega q_i,  r_{i+1} = q_i - omega y_i,
//   w_{i+1} = y_i - omega (t_i - alpha v_i)
// With DOTS also [3][gridDim.x] partial triples of (r0*, r), (r0*, w), (r, r)
// of the new r and w (the rest of phase 2).
struct Stab2Args {
  const double *p, *q, *y, *t, *v;
  double *x, *r, *w;
  const double *sc;
  int *ctl;
  int64_t n;
  int rev;  // sweep direction
  const int *chunk_sys;  // system of each 256-row chunk (batched solves), or nullptr
  const double *rs;      // r0* (DOTS)
  double *part;          // partial sums (DOTS)
};

template <int W, bool DOTS, bool NT>
__device__ __forceinline__ void stab2_body(const Stab2Args &P, int64_t k, TD (&acc)[3]) {
  const double al = P.sc[PS_S_ALPHA], om = P.sc[PS_S_OMEGA];
  double p[W], q[W], y[W], t[W], v[W], x[W], r[W], w[W];
  ldv_s<W, NT>(P.p, k, p);
  ldv_s<W, NT>(P.q, k, q);
  ldv_s<W, NT>(P.y, k, y);
  ldv<W>(P.t, k, t);
  ldv<W>(P.v, k, v);
  ldv_s<W, NT>(P.x, k, x);
#pragma unroll
  for (int j = 0; j < W; ++j) {
    x[j] = x[j] + al * p[j] + om * q[j];
    r[j] = q[j] - om * y[j];
    w[j] = y[j] - om * (t[j] - al * v[j]);
  }
  if constexpr (DOTS) {
    double rs[W];
    ldv<W>(P.rs, k, rs);
#pragma unroll
    for (int j = 0; j < W; ++j) {
      td_fma(acc[0], rs[j], r[j]);
      td_fma(acc[1], rs[j], w[j]);
      td_fma(acc[2], r[j], r[j]);
    }
  }
  stv_s<W, NT>(P.x, k, x);
  stv<W>(P.r, k, r);
  stv<W>(P.w, k, w);
}

template <bool DOTS, bool NT>
__global__ __launch_bounds__(kBlock) void k_stab_pass2(Stab2Args P_) {
  const Stab2Args P = bind_system(P_);
  if (halted_after_finish(P.ctl)) return;
  TD acc[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) acc[j] = TD{0.0, 0.0, 0.0};
  const int b = pass_block(P.rev);
  const int64_t k = 2 * ((int64_t)b * kBlock + threadIdx.x);
  if (k + 1 < P.n) stab2_body<2, DOTS, NT>(P, k, acc);
  else if (k < P.n) stab2_body<1, DOTS, NT>(P, k, acc);
  if constexpr (DOTS) store_pass_partials<3>(acc, P.part, b);
}

// ------------------------------------------------------------ bookkeeping

// zero-fill of `count` vectors of length n laid out `ld` doubles apart
__global__ __launch_bounds__(kBlock) void k_zero(double *base, int64_t ld, int count, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  for (int c = 0; c < count; ++c) base[c * ld + k] = 0.0;
}

// dst = src rounded to the nearest FP32 number (ties to even: the default
// rounding mode of the conversion)
__global__ __launch_bounds__(kBlock) void k_round_f32(const double *__restrict__ src,
                                                      float *__restrict__ dst, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[k] = (float)src[k];
}

__global__ __launch_bounds__(kBlock) void k_copy(double *__restrict__ dst,
                                                 const double *__restrict__ src, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[k] = src[k];
}

// plain streaming copy, 16 bytes per thread per step (bandwidth calibration)
__global__ __launch_bounds__(kBlock) void k_stream_copy(double2 *__restrict__ dst,
                                                        const double2 *__restrict__ src,
                                                        int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n16; k += stride)
    dst[k] = src[k];
}

// x0 fallback: where the system's guess was rejected, x = 0 and r = r0* = b
__global__ __launch_bounds__(kBlock) void k_fallback(double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ rs, const double *__restrict__ b,
                                                     const double *__restrict__ sc,
                                                     const int *__restrict__ chunk_sys, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int sys = system_of(chunk_sys, k);
  if (sc[(size_t)sys * SC_COUNT + SC_FALLBACK] != 0.0) {
    x[k] = 0.0;
    r[k] = b[k];
    rs[k] = b[k];
  }
}

// x0 = c x0 with each system's least-residual factor (FinScale), or 0
__global__ __launch_bounds__(kBlock) void k_scale_x(double *__restrict__ x,
                                                    const double *__restrict__ sc,
                                                    const int *__restrict__ chunk_sys, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const double *s = sc + (size_t)system_of(chunk_sys, k) * SC_COUNT;
  x[k] = s[SC_SCALE_OK] != 0.0 ? s[SC_SCALE] * x[k] : 0.0;
}

// control blocks of `nsys` systems, then the count of systems still running
__global__ __launch_bounds__(kBlock) void k_init_ctl(int *ctl, int first_iter, int nsys) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t words = (int64_t)nsys * C_COUNT;
  if (k < words) {
    const int w = (int)(k % C_COUNT);
    ctl[k] = (w == C_STATUS) ? -1 : (w == C_ITER ? first_iter : 0);
  } else if (k == words) {
    ctl[k] = nsys;
  }
}

// batched solves: dst[map[i]] = src[i] (map: row i of the caller's
// concatenation -> its padded row), and the inverse gather
__global__ __launch_bounds__(kBlock) void k_scatter(double *__restrict__ dst,
                                                    const double *__restrict__ src,
                                                    const int *__restrict__ map, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[map[k]] = src[k];
}
__global__ __launch_bounds__(kBlock) void k_gather(double *__restrict__ dst,
                                                   const double *__restrict__ src,
                                                   const int *__restrict__ map, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[k] = src[map[k]];
}

}  // namespace ps
