// Kernels of the warm-start network: a small U-Net over NHWC images whose
// activations, weights and gradients are stored in bfloat16 and whose 3x3
// convolutions run on the matrix cores (v_mfma_f32_16x16x32_bf16: bf16
// products, fp32 accumulation).
//
// Storage: a tensor "view" is (base, ld, off): pixel q (n*H*W + y*W + x),
// channel c lives at base[q*ld + off + c], so a convolution can read or write
// a channel slice of a wider buffer (the skip concatenations cost nothing).
// Channel counts and offsets are multiples of 16, so 8 consecutive channels
// are one 16-byte load.
//
// bf16 <-> fp32 conversions are written out (round to nearest even), so the
// rounding points are explicit and the same as the CPU reference's.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ws {

constexpr int kBlock = 256;
constexpr int kWave = 64;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);  // NaN
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

struct View {
  uint16_t *p;
  int ld, off;
};
struct CView {
  const uint16_t *p;
  int ld, off;
};

// ------------------------------------------------------ 3x3 convolution
// out[q, co] = sum_{tap, ci} in[q + d(tap), ci] * w[co][tap*Ci + ci]  (+ bias, ReLU)
// with d(tap) = (tap/3 - 1, tap%3 - 1) rows/columns, zero outside the image;
// `flip` negates d (the data gradient of a convolution is this with the
// weights rearranged as [ci][tap*Co + co]).  An implicit GEMM: M = pixels,
// N = output channels, K = 9 * input channels (padded to Kp, a multiple of
// 32, with zero weights).  Each wavefront computes 16 consecutive pixels x
// all NT*16 output channels; per K step of 32 every lane loads 8 channels of
// one tap of its pixel (16 bytes) and 8 weights per output tile.
struct ConvArgs {
  CView in;
  const uint16_t *w;   // [Co][Kp]
  const float *bias;   // [Co] or nullptr
  View out;
  int N, H, W, Ci, Co, Kp;
  int relu, flip;
};

template <int NT>
__global__ __launch_bounds__(kBlock) void k_conv3x3(ConvArgs a) {
  const int lane = threadIdx.x % kWave;
  const int64_t npx = (int64_t)a.N * a.H * a.W;
  const int64_t q0 = ((int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * 16;
  if (q0 >= npx) return;  // whole wavefront past the end
  const int row = lane % 16, kq = lane / 16;
  // the pixel this lane loads for the A operand
  const int64_t qa = q0 + row;
  const bool qa_ok = qa < npx;
  int n = 0, y = 0, x = 0;
  if (qa_ok) {
    n = (int)(qa / ((int64_t)a.H * a.W));
    const int r = (int)(qa % ((int64_t)a.H * a.W));
    y = r / a.W;
    x = r % a.W;
  }
  const int K = 9 * a.Ci;
  f32x4 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < a.Kp; k0 += 32) {
    const int k = k0 + 8 * kq;
    uint4 av = make_uint4(0, 0, 0, 0);
    if (qa_ok && k < K) {
      const int tap = k / a.Ci, c = k % a.Ci;
      int dy = tap / 3 - 1, dx = tap % 3 - 1;
      if (a.flip) {
        dy = -dy;
        dx = -dx;
      }
      const int yy = y + dy, xx = x + dx;
      if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) {
        const int64_t qq = ((int64_t)n * a.H + yy) * a.W + xx;
        av = *reinterpret_cast<const uint4 *>(a.in.p + qq * a.in.ld + a.in.off + c);
      }
    }
    const bf16x8 A = __builtin_bit_cast(bf16x8, av);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const uint4 bv = *reinterpret_cast<const uint4 *>(a.w + (int64_t)(j * 16 + row) * a.Kp + k);
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, bv), acc[j], 0, 0, 0);
    }
  }
  // lane holds D[m = 4*kq + i][n = row] of each tile: pixel q0 + 4*kq + i, channel j*16 + row
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int co = j * 16 + row;
    const float b = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t q = q0 + 4 * kq + i;
      if (q < npx) {
        float v = acc[j][i] + b;
        if (a.relu) v = v > 0.f ? v : 0.f;
        a.out.p[q * a.out.ld + a.out.off + co] = f2bf(v);
      }
    }
  }
}

// ------------------------------------------------ 3x3 weight gradient
// dw[co][tap*Ci + ci] = sum_q g[q, co] * in[q + d(tap), ci], for one tap per
// blockIdx.y and a share of the pixels per blockIdx.x: the block stages 64
// pixels of g (as [Co][64]) and of the shifted input (as [Ci][64]) in LDS,
// transposed so that each MFMA operand lane reads 8 consecutive pixels, and
// its 4 wavefronts split the (Co/16) x (Ci/16) output tiles.  Each block
// writes its fp32 partial sums; k_sum_partials adds them in block order.
struct WGradArgs {
  CView in, g;
  float *part;  // [gridDim.x][Co][9*Ci]
  int N, H, W, Ci, Co;
};

constexpr int kWgTilesPerWave = 8;  // (Co/16)*(Ci/16)/4 <= 8 for every layer
constexpr int kWgChunk = 64;

__global__ __launch_bounds__(kBlock) void k_conv3x3_wgrad(WGradArgs a) {
  __shared__ __align__(16) uint16_t sg[64 * kWgChunk];   // [Co <= 64][64 px]
  __shared__ __align__(16) uint16_t sx[128 * kWgChunk];  // [Ci <= 128][64 px]
  const int tap = blockIdx.y;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int row = lane % 16, kq = lane / 16;
  const int tco = a.Co / 16, tci = a.Ci / 16, ntile = tco * tci;
  f32x4 acc[kWgTilesPerWave];
#pragma unroll
  for (int t = 0; t < kWgTilesPerWave; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t hw = (int64_t)a.H * a.W, npx = (int64_t)a.N * hw;
  const int64_t nchunk = (npx + kWgChunk - 1) / kWgChunk;
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t qbase = ch * kWgChunk;
    // stage g: 64 px x Co channels, 8 channels per load
    for (int e = threadIdx.x; e < kWgChunk * (a.Co / 8); e += kBlock) {
      const int p = e / (a.Co / 8), c8 = (e % (a.Co / 8)) * 8;
      const int64_t q = qbase + p;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (q < npx) v = *reinterpret_cast<const uint4 *>(a.g.p + q * a.g.ld + a.g.off + c8);
      const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
      for (int u = 0; u < 8; ++u) sg[(c8 + u) * kWgChunk + p] = h[u];
    }
    // stage the input shifted by the tap
    for (int e = threadIdx.x; e < kWgChunk * (a.Ci / 8); e += kBlock) {
      const int p = e / (a.Ci / 8), c8 = (e % (a.Ci / 8)) * 8;
      const int64_t q = qbase + p;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (q < npx) {
        const int n = (int)(q / hw);
        const int r = (int)(q % hw);
        const int yy = r / a.W + dy, xx = r % a.W + dx;
        if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
          v = *reinterpret_cast<const uint4 *>(a.in.p + (((int64_t)n * a.H + yy) * a.W + xx) * a.in.ld +
                                               a.in.off + c8);
      }
      const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
      for (int u = 0; u < 8; ++u) sx[(c8 + u) * kWgChunk + p] = h[u];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kWgTilesPerWave; ++t) {
      const int tile = wave + 4 * t;
      if (tile < ntile) {
        const int cot = tile / tci, cit = tile % tci;
#pragma unroll
        for (int kk = 0; kk < kWgChunk; kk += 32) {
          const uint4 av = *reinterpret_cast<const uint4 *>(&sg[(cot * 16 + row) * kWgChunk + kk + 8 * kq]);
          const uint4 bv = *reinterpret_cast<const uint4 *>(&sx[(cit * 16 + row) * kWgChunk + kk + 8 * kq]);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                           __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // D[m = co][n = ci]: lane holds co = cot*16 + 4*kq + i, ci = cit*16 + row
  float *part = a.part + (int64_t)blockIdx.x * a.Co * 9 * a.Ci;
#pragma unroll
  for (int t = 0; t < kWgTilesPerWave; ++t) {
    const int tile = wave + 4 * t;
    if (tile < ntile) {
      const int cot = tile / tci, cit = tile % tci;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = cot * 16 + 4 * kq + i, ci = cit * 16 + row;
        part[(int64_t)co * 9 * a.Ci + tap * a.Ci + ci] = acc[t][i];
      }
    }
  }
}

// dst[e] = sum over p < np of part[p*len + e], in order (fp32)
__global__ __launch_bounds__(kBlock) void k_sum_partials(const float *__restrict__ part, int np, int64_t len,
                                                         float *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  float s = 0.f;
  for (int p = 0; p < np; ++p) s += part[(int64_t)p * len + e];
  dst[e] = s;
}

// column sums of a bf16 view: part[b][c] = sum of channel c over block b's pixels
__global__ __launch_bounds__(kBlock) void k_colsum(CView g, int64_t npx, int C, float *__restrict__ part) {
  // thread t handles channel t % C over pixels t / C, t / C + kBlock / C, ...
  const int per = kBlock / C;
  const int c = threadIdx.x % C, j = threadIdx.x / C;
  __shared__ float red[kBlock];
  float s = 0.f;
  if (j < per) {
    for (int64_t q = (int64_t)blockIdx.x * per + j; q < npx; q += (int64_t)gridDim.x * per)
      s += bf2f(g.p[q * g.ld + g.off + c]);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < C) {
    float t = 0.f;
    for (int k = 0; k < per; ++k) t += red[k * C + threadIdx.x];
    part[(int64_t)blockIdx.x * C + threadIdx.x] = t;
  }
}

// ------------------------------------------------------ elementwise
// ReLU backward in place: g = g * (act > 0)
__global__ __launch_bounds__(kBlock) void k_relu_mask(View g, CView act, int64_t npx, int C) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= npx * C) return;
  const int64_t q = e / C;
  const int c = (int)(e % C);
  if (!(bf2f(act.p[q * act.ld + act.off + c]) > 0.f)) g.p[q * g.ld + g.off + c] = 0;
}

// 2x2 average pooling (H, W even): out (N, H/2, W/2, C)
__global__ __launch_bounds__(kBlock) void k_pool2(CView in, View out, int N, int H, int W, int C) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (e >= (int64_t)N * Ho * Wo * C) return;
  const int c = (int)(e % C);
  const int64_t qo = e / C;
  const int n = (int)(qo / ((int64_t)Ho * Wo));
  const int r = (int)(qo % ((int64_t)Ho * Wo));
  const int y = r / Wo, x = r % Wo;
  float s = 0.f;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t qi = ((int64_t)n * H + 2 * y + u / 2) * W + 2 * x + u % 2;
    s += bf2f(in.p[qi * in.ld + in.off + c]);
  }
  out.p[qo * out.ld + out.off + c] = f2bf(0.25f * s);
}

// its gradient, added to what the fine view already holds: fine += 0.25 coarse
__global__ __launch_bounds__(kBlock) void k_pool2_bwd_add(CView coarse, View fine, int N, int H, int W, int C) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)N * H * W * C) return;
  const int c = (int)(e % C);
  const int64_t q = e / C;
  const int n = (int)(q / ((int64_t)H * W));
  const int r = (int)(q % ((int64_t)H * W));
  const int y = r / W, x = r % W;
  const int64_t qc = ((int64_t)n * (H / 2) + y / 2) * (W / 2) + x / 2;
  const float v = bf2f(fine.p[q * fine.ld + fine.off + c]) + 0.25f * bf2f(coarse.p[qc * coarse.ld + coarse.off + c]);
  fine.p[q * fine.ld + fine.off + c] = f2bf(v);
}

// nearest 2x upsampling: out (N, 2H, 2W, C) from in (N, H, W, C)
__global__ __launch_bounds__(kBlock) void k_up2(CView in, View out, int N, int H, int W, int C) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int Ho = 2 * H, Wo = 2 * W;
  if (e >= (int64_t)N * Ho * Wo * C) return;
  const int c = (int)(e % C);
  const int64_t q = e / C;
  const int n = (int)(q / ((int64_t)Ho * Wo));
  const int r = (int)(q % ((int64_t)Ho * Wo));
  const int y = r / Wo, x = r % Wo;
  const int64_t qi = ((int64_t)n * H + y / 2) * W + x / 2;
  out.p[q * out.ld + out.off + c] = in.p[qi * in.ld + in.off + c];
}

// its gradient: coarse = sum of the 4 fine values
__global__ __launch_bounds__(kBlock) void k_up2_bwd(CView fine, View coarse, int N, int H, int W, int C) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)N * H * W * C) return;
  const int c = (int)(e % C);
  const int64_t q = e / C;
  const int n = (int)(q / ((int64_t)H * W));
  const int r = (int)(q % ((int64_t)H * W));
  const int y = r / W, x = r % W;
  float s = 0.f;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t qf = ((int64_t)n * 2 * H + 2 * y + u / 2) * (2 * W) + 2 * x + u % 2;
    s += bf2f(fine.p[qf * fine.ld + fine.off + c]);
  }
  coarse.p[q * coarse.ld + coarse.off + c] = f2bf(s);
}

// network input: fp32 (npx, cin) -> bf16 view, channels cin..ld-1 zero
__global__ __launch_bounds__(kBlock) void k_input(const float *__restrict__ x, int cin, View out, int64_t npx) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= npx * out.ld) return;
  const int64_t q = e / out.ld;
  const int c = (int)(e % out.ld);
  out.p[e] = c < cin ? f2bf(x[q * cin + c]) : (uint16_t)0;
}

// ------------------------------------------------------ 1x1 output head
// y[q] = sum_c w[c] h[q, c] + b   (fp32 weights and output)
__global__ __launch_bounds__(kBlock) void k_head(CView h, const float *__restrict__ w, int C, int64_t npx,
                                                 float *__restrict__ y) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= npx) return;
  float s = 0.f;
  for (int c = 0; c < C; ++c) s += w[c] * bf2f(h.p[q * h.ld + h.off + c]);
  y[q] = s + w[C];
}

// loss: d[q] = 2 (y - t) / npx (the gradient of the mean squared error);
// part[b] = the block's sum of (y - t)^2 in fp64
__global__ __launch_bounds__(kBlock) void k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                                int64_t npx, float *__restrict__ d, double *__restrict__ part) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < npx; q += (int64_t)gridDim.x * kBlock) {
    const float e = y[q] - t[q];
    d[q] = 2.f * e / (float)npx;
    s += (double)e * (double)e;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k /= 2) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// head backward: dh[q, c] = w[c] dy[q] (bf16); part[b][c] = sum_q h[q,c] dy[q], part[b][C] = sum_q dy[q]
__global__ __launch_bounds__(kBlock) void k_head_bwd(CView h, const float *__restrict__ w, int C, int64_t npx,
                                                     const float *__restrict__ dy, View dh,
                                                     float *__restrict__ part) {
  __shared__ float red[kBlock][17];
  float acc[17];
  for (int c = 0; c <= C; ++c) acc[c] = 0.f;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < npx; q += (int64_t)gridDim.x * kBlock) {
    const float g = dy[q];
    for (int c = 0; c < C; ++c) {
      acc[c] += bf2f(h.p[q * h.ld + h.off + c]) * g;
      dh.p[q * dh.ld + dh.off + c] = f2bf(w[c] * g);
    }
    acc[C] += g;
  }
  for (int c = 0; c <= C; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  if (threadIdx.x <= C) {
    float s = 0.f;
    for (int k = 0; k < kBlock; ++k) s += red[k][threadIdx.x];
    part[(int64_t)blockIdx.x * (C + 1) + threadIdx.x] = s;
  }
}

// ------------------------------------------------------ parameters
// Adam on the fp32 master parameters (bias-corrected first and second moments)
__global__ __launch_bounds__(kBlock) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                                 float *__restrict__ m, float *__restrict__ v, int64_t n,
                                                 float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// bf16 weight layouts of one 3x3 layer from its fp32 master weights
// W[co][tap][ci]: forward wf[co][Kp] (k = tap*Ci + ci, zero past 9*Ci) and,
// for the data gradient, wb[ci][Kpb] (k = tap*Co + co, zero past 9*Co)
__global__ __launch_bounds__(kBlock) void k_pack_weights(const float *__restrict__ W, int Ci, int Co, int Kp,
                                                         int Kpb, uint16_t *__restrict__ wf,
                                                         uint16_t *__restrict__ wb) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nf = (int64_t)Co * Kp, nb = (int64_t)Ci * Kpb;
  if (e < nf) {
    const int co = (int)(e / Kp), k = (int)(e % Kp);
    wf[e] = k < 9 * Ci ? f2bf(W[(int64_t)co * 9 * Ci + k]) : (uint16_t)0;
  } else if (e < nf + nb) {
    const int64_t e2 = e - nf;
    const int ci = (int)(e2 / Kpb), k = (int)(e2 % Kpb);
    uint16_t v = 0;
    if (k < 9 * Co) {
      const int tap = k / Co, co = k % Co;
      v = f2bf(W[(int64_t)co * 9 * Ci + tap * Ci + ci]);
    }
    wb[e2] = v;
  }
}

}  // namespace ws
