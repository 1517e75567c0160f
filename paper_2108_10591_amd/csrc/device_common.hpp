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
  C_COUNT = 16
};

// double scalar block on the device: the public ps_scalar slots, then private ones
enum Sc : int {
  SC_DOTS = 16,   // raw inner products of the last reduction phase (up to 9)
  SC_COUNT = 32
};

// Sum over a wavefront by an xor butterfly; every lane ends with the same
// bit pattern because each lane adds the same operands in the same order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sums of K values in a fixed order.  On return thread k (< K)
// holds the block total of v[k].  `lds` must hold kWavesPerBlock * K doubles.
template <int K>
__device__ __forceinline__ double block_sum_k(double (&v)[K], double *lds) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[wid * K + k] = v[k];
  }
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < K) {
    s = lds[threadIdx.x];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) s += lds[w * K + threadIdx.x];
  }
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_sum_1(double v, double *lds) {
  double a[1] = {v};
  double s = block_sum_k<1>(a, lds);
  if (threadIdx.x == 0) lds[0] = s;
  __syncthreads();
  s = lds[0];
  __syncthreads();
  return s;
}

__device__ __forceinline__ bool bad_den(double d) { return d == 0.0 || !isfinite(d); }

// Sweep direction.  Consecutive streaming kernels of an iteration walk the
// rows in alternating directions, so each one starts on the rows the previous
// one touched last -- the lines most likely still held in the 256 MB
// memory-side Infinity Cache (MALL) -- instead of the ones it evicted first.
// Per-row arithmetic is unchanged, so results do not depend on the direction.
__device__ __forceinline__ int sweep_block(int b, int nb, int rev) { return rev ? nb - 1 - b : b; }

// Stop the solve: record status and iteration index.
__device__ __forceinline__ void set_stop(int *ctl, int status, int iters) {
  ctl[C_STATUS] = status;
  ctl[C_ITERS] = iters;
  ctl[C_DONE] = 1;
}

// hist[i] = sqrt(rho)/sqrt(rhoref) and the stop test ||r_i|| <= tol ||r_ref||
// (Algorithms 3-5; the test is taken before the coefficients are formed).
// Returns true if the solve stops here.
__device__ __forceinline__ bool stop_test(double rho, const double *sc, int *ctl, double *hist,
                                          int i, int maxit, double tol) {
  const double ref = sqrt(sc[PS_S_RHOREF]);
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

}  // namespace ps
