// CSR sparse matrix-vector product y = A x with a fused per-row epilogue.
//
// Rows are cut at creation time into row blocks of at most kBlock rows whose
// nonzeros fit an LDS budget.  A block streams its contiguous slice of
// (val, col) with coalesced loads, forms val*x[col] into LDS, and then one
// thread per row adds its row's products in storage order and hands the row
// sum to the epilogue, which updates the row's entries of other vectors (the
// update passes that the paper's algorithms place right after each product).
// A row longer than the budget gets a block of its own, which splits it over
// all threads and combines the pieces with a fixed-order block reduction.
#pragma once

#include "device_common.hpp"

namespace ps {

struct CsrDev {
  const int *rowptr;   // int32[n+1]
  const int *col;      // int32[nnz]
  const double *val;   // double[nnz]
  const int *blk;      // int32[nblk+1] first row of each row block
  int nblk;
  int budget;          // max nonzeros of a short-row block (LDS doubles)
};

// Row-block index for workgroup `b`: consecutive workgroups are dispatched
// round-robin over the 8 XCDs, so give each XCD a contiguous range of row
// blocks; its L2 then holds the x entries its rows gather.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, rem = nb % kXcd;
  const int xcd = b % kXcd, k = b / kXcd;
  // XCD x owns q (+1 if x < rem) consecutive blocks
  const int start = xcd * q + (xcd < rem ? xcd : rem);
  return start + k;
}

// `stop` (may be null) points at the control word that turns the launch into a
// no-op: C_DONE for products that follow a finish in stream order, C_HALT for
// products that may run concurrently with one.
template <class Epi>
__global__ __launch_bounds__(kBlock) void k_spmv(CsrDev A, const double *__restrict__ x, Epi epi,
                                                 const int *__restrict__ stop) {
  if (stop != nullptr && *stop) return;
  extern __shared__ double prod[];
  const int b = xcd_block(blockIdx.x, A.nblk);
  const int r0 = A.blk[b], r1 = A.blk[b + 1];
  const int k0 = A.rowptr[r0], k1 = A.rowptr[r1];
  const int nz = k1 - k0;
  if (nz <= A.budget) {
    for (int k = threadIdx.x; k < nz; k += kBlock) prod[k] = A.val[k0 + k] * x[A.col[k0 + k]];
    __syncthreads();
    const int r = r0 + threadIdx.x;
    if (r < r1) {
      const int a = A.rowptr[r] - k0, e = A.rowptr[r + 1] - k0;
      double acc = 0.0;
      for (int k = a; k < e; ++k) acc += prod[k];
      epi(r, acc);
    }
  } else {
    // one long row: strided partial sums, then a fixed-order block reduction
    double acc = 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += kBlock) acc += A.val[k] * x[A.col[k]];
    acc = block_sum_1(acc, prod);
    if (threadIdx.x == 0) epi(r0, acc);
  }
}

// ------------------------------------------------------------------ epilogues

// y = A x
struct EpiStore {
  double *y;
  __device__ __forceinline__ void operator()(int r, double ax) const { y[r] = ax; }
};

// r = b - A x (and optionally r0* = r): the initial residual of every
// algorithm, and the true residual of a replacement step (Algorithm 5)
struct EpiResidual {
  const double *b;
  double *r;
  double *rs;  // may be null
  __device__ __forceinline__ void operator()(int row, double ax) const {
    const double v = b[row] - ax;
    r[row] = v;
    if (rs) rs[row] = v;
  }
};

// p-BiCGSafe, the product A w_i and the three recurrences that follow it in
// Algorithm 4: l_i = q_i - A w_i (Eq. (l)), g_{i+1} = zeta A s_i + eta g_i -
// alpha A w_i (Eq. (g)), s_{i+1} = s_i - alpha q_i - g_{i+1} (Eq. (sip1)).
// A w_i itself is never stored.
struct EpiPBiCGSafeB {
  const double *q, *As;
  double *l, *g, *s;
  const double *sc;
  __device__ __forceinline__ void operator()(int r, double aw) const {
    const double al = sc[PS_S_ALPHA], ze = sc[PS_S_ZETA], et = sc[PS_S_ETA];
    const double qr = q[r];
    l[r] = qr - aw;
    const double gn = ze * As[r] + et * g[r] - al * aw;
    g[r] = gn;
    s[r] = s[r] - al * qr - gn;
  }
};

// ssBiCGSafe2, the product w_i = A u_i and the updates after it (Algorithm 3):
// o_i = s_i + beta t_{i-1} (recomputed, not stored), t_i = o_i - w_i,
// z_i = zeta r_i + eta z_{i-1} - alpha u_i, y_{i+1} = zeta s_i + eta y_i - alpha w_i,
// x_{i+1} = x_i + alpha p_i + z_i, r_{i+1} = r_i - alpha o_i - y_{i+1}.
struct EpiSsBiCGSafe2B {
  const double *s, *u, *p;
  double *t, *z, *y, *x, *r;
  const double *sc;
  __device__ __forceinline__ void operator()(int row, double wv) const {
    const double al = sc[PS_S_ALPHA], be = sc[PS_S_BETA], ze = sc[PS_S_ZETA], et = sc[PS_S_ETA];
    const double sr = s[row], rr = r[row];
    const double o = sr + be * t[row];
    t[row] = o - wv;
    const double zn = ze * rr + et * z[row] - al * u[row];
    z[row] = zn;
    const double yn = ze * sr + et * y[row] - al * wv;
    y[row] = yn;
    x[row] = x[row] + al * p[row] + zn;
    r[row] = rr - al * o - yn;
  }
};

}  // namespace ps
