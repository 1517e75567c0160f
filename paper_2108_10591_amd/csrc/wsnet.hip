// wsnet: host driver and C ABI of the warm-start U-Net (see include/wsnet.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wsnet.h"
#include "wsnet_kernels.hpp"

using namespace ws;

namespace {

constexpr int kLayers = 10;        // 3x3 layers
constexpr int kMaxBatch = 64;
constexpr int kWgradBlocks = 64;   // pixel shares of the weight gradient
constexpr int kColBlocks = 256;
constexpr int kHeadBlocks = 256;
constexpr int kLossBlocks = 256;

#define WS_HIP(...)                                                                   \
  do {                                                                                \
    hipError_t e_ = (__VA_ARGS__);                                                    \
    if (e_ != hipSuccess) {                                                           \
      std::fprintf(stderr, "wsnet: %s failed: %s\n", #__VA_ARGS__, hipGetErrorString(e_)); \
      return -3;                                                                      \
    }                                                                                 \
  } while (0)
#define WS_TRY(...)               \
  do {                            \
    int rc_ = (__VA_ARGS__);      \
    if (rc_ != 0) return rc_;     \
  } while (0)

struct Layer {
  int Ci, Co, Kp, Kpb, level;  // level: the layer runs at H >> level
  int64_t w_off, b_off;        // into the fp32 parameter vector
  uint16_t *wf, *wb;           // packed bf16 weights
};

// activation / gradient buffers of one batch capacity
struct Buf {
  uint16_t *p = nullptr;
  int C = 0, level = 0;
};

int64_t up32(int64_t k) { return (k + 31) / 32 * 32; }

}  // namespace

struct ws_net {
  int H = 0, W = 0, cin = 0, c = 0, cin_pad = 16;
  Layer L[kLayers];
  int64_t nparams = 0, head_off = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wbuf = nullptr;
  float *part = nullptr;     // weight-gradient partial sums
  float *hpart = nullptr;    // column / head partial sums
  double *lpart = nullptr;   // loss partial sums
  int64_t step = 0;
  int nmax = 0;              // batch capacity of the buffers below
  Buf X, A0, C0, P1, A1, C1, P2, A2, C2, P3, BT, D2, D1, D0;
  Buf dD0, dC0, dD1, dC1, dD2, dC2, dBT, dP3, dA2, dP2, dA1, dP1, dA0;
  float *out = nullptr, *dout = nullptr;
  float *bx = nullptr, *bt = nullptr;  // gathered mini-batch inputs and targets
  int *idx = nullptr;
  std::vector<void *> allocs;
};

namespace {

int64_t npx_at(const ws_net *N, int n, int level) {
  return (int64_t)n * (N->H >> level) * (N->W >> level);
}

int alloc(ws_net *N, void **p, size_t bytes) {
  if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) return -2;
  N->allocs.push_back(*p);
  return 0;
}

int ensure_batch(ws_net *N, int n) {
  if (n <= N->nmax) return 0;
  // free the previous batch buffers (everything allocated after the parameters)
  WS_HIP(hipDeviceSynchronize());
  while (N->allocs.size() > 1) {
    (void)hipFree(N->allocs.back());
    N->allocs.pop_back();
  }
  const int c = N->c;
  auto mk = [&](Buf &b, int C, int level) {
    b.C = C;
    b.level = level;
    return alloc(N, (void **)&b.p, (size_t)npx_at(N, n, level) * C * sizeof(uint16_t));
  };
  WS_TRY(mk(N->X, N->cin_pad, 0));
  WS_TRY(mk(N->A0, c, 0));
  WS_TRY(mk(N->C0, 3 * c, 0));
  WS_TRY(mk(N->P1, c, 1));
  WS_TRY(mk(N->A1, 2 * c, 1));
  WS_TRY(mk(N->C1, 6 * c, 1));
  WS_TRY(mk(N->P2, 2 * c, 2));
  WS_TRY(mk(N->A2, 4 * c, 2));
  WS_TRY(mk(N->C2, 8 * c, 2));
  WS_TRY(mk(N->P3, 4 * c, 3));
  WS_TRY(mk(N->BT, 4 * c, 3));
  WS_TRY(mk(N->D2, 4 * c, 2));
  WS_TRY(mk(N->D1, 2 * c, 1));
  WS_TRY(mk(N->D0, c, 0));
  WS_TRY(mk(N->dD0, c, 0));
  WS_TRY(mk(N->dC0, 3 * c, 0));
  WS_TRY(mk(N->dD1, 2 * c, 1));
  WS_TRY(mk(N->dC1, 6 * c, 1));
  WS_TRY(mk(N->dD2, 4 * c, 2));
  WS_TRY(mk(N->dC2, 8 * c, 2));
  WS_TRY(mk(N->dBT, 4 * c, 3));
  WS_TRY(mk(N->dP3, 4 * c, 3));
  WS_TRY(mk(N->dA2, 4 * c, 2));
  WS_TRY(mk(N->dP2, 2 * c, 2));
  WS_TRY(mk(N->dA1, 2 * c, 1));
  WS_TRY(mk(N->dP1, c, 1));
  WS_TRY(mk(N->dA0, c, 0));
  WS_TRY(alloc(N, (void **)&N->out, (size_t)npx_at(N, n, 0) * sizeof(float)));
  WS_TRY(alloc(N, (void **)&N->dout, (size_t)npx_at(N, n, 0) * sizeof(float)));
  WS_TRY(alloc(N, (void **)&N->bx, (size_t)npx_at(N, n, 0) * N->cin * sizeof(float)));
  WS_TRY(alloc(N, (void **)&N->bt, (size_t)npx_at(N, n, 0) * sizeof(float)));
  WS_TRY(alloc(N, (void **)&N->idx, (size_t)n * sizeof(int)));
  N->nmax = n;
  return 0;
}

CView cv(const Buf &b, int off = 0) { return CView{b.p, b.C, off}; }
View vw(const Buf &b, int off = 0) { return View{b.p, b.C, off}; }

unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int NT>
void conv_launch(const ConvArgs &a, hipStream_t s) {
  const int64_t npx = (int64_t)a.N * a.H * a.W;
  const int64_t waves = (npx + 15) / 16;
  hipLaunchKernelGGL(k_conv3x3<NT>, dim3((unsigned)((waves + 3) / 4)), dim3(kBlock), 0, s, a);
}

// one 3x3 convolution (forward: weights wf; data gradient: weights wb, flip)
int conv(ws_net *N, const Layer &l, CView in, View out, int n, bool data_grad, hipStream_t s) {
  ConvArgs a{};
  a.in = in;
  a.out = out;
  a.N = n;
  a.H = N->H >> l.level;
  a.W = N->W >> l.level;
  if (!data_grad) {
    a.w = l.wf;
    a.bias = N->params + l.b_off;
    a.Ci = l.Ci;
    a.Co = l.Co;
    a.Kp = l.Kp;
    a.relu = 1;
    a.flip = 0;
  } else {
    a.w = l.wb;
    a.bias = nullptr;
    a.Ci = l.Co;
    a.Co = l.Ci;
    a.Kp = l.Kpb;
    a.relu = 0;
    a.flip = 1;
  }
  switch (a.Co / 16) {
    case 1: conv_launch<1>(a, s); break;
    case 2: conv_launch<2>(a, s); break;
    case 3: conv_launch<3>(a, s); break;
    case 4: conv_launch<4>(a, s); break;
    case 6: conv_launch<6>(a, s); break;
    case 8: conv_launch<8>(a, s); break;
    default: return -1;
  }
  WS_HIP(hipGetLastError());
  return 0;
}

// weight and bias gradients of one 3x3 layer
int wgrad(ws_net *N, const Layer &l, CView in, CView g, int n, hipStream_t s) {
  WGradArgs a{in, g, N->part, n, N->H >> l.level, N->W >> l.level, l.Ci, l.Co};
  hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(kWgradBlocks, 9), dim3(kBlock), 0, s, a);
  const int64_t len = (int64_t)l.Co * 9 * l.Ci;
  hipLaunchKernelGGL(k_sum_partials, dim3(blocks(len)), dim3(kBlock), 0, s, (const float *)N->part,
                     kWgradBlocks, len, N->grads + l.w_off);
  hipLaunchKernelGGL(k_colsum, dim3(kColBlocks), dim3(kBlock), 0, s, g, npx_at(N, n, l.level), l.Co,
                     N->hpart);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, (const float *)N->hpart, kColBlocks,
                     (int64_t)l.Co, N->grads + l.b_off);
  WS_HIP(hipGetLastError());
  return 0;
}

int relu_mask(ws_net *N, View g, CView act, int C, int n, int level, hipStream_t s) {
  const int64_t e = npx_at(N, n, level) * C;
  hipLaunchKernelGGL(k_relu_mask, dim3(blocks(e)), dim3(kBlock), 0, s, g, act, npx_at(N, n, level), C);
  WS_HIP(hipGetLastError());
  return 0;
}

int pool(ws_net *N, CView in, View out, int C, int n, int level, hipStream_t s) {
  const int H = N->H >> level, W = N->W >> level;
  hipLaunchKernelGGL(k_pool2, dim3(blocks((int64_t)n * (H / 2) * (W / 2) * C)), dim3(kBlock), 0, s, in, out,
                     n, H, W, C);
  WS_HIP(hipGetLastError());
  return 0;
}
int pool_bwd_add(ws_net *N, CView coarse, View fine, int C, int n, int level, hipStream_t s) {
  const int H = N->H >> level, W = N->W >> level;
  hipLaunchKernelGGL(k_pool2_bwd_add, dim3(blocks((int64_t)n * H * W * C)), dim3(kBlock), 0, s, coarse,
                     fine, n, H, W, C);
  WS_HIP(hipGetLastError());
  return 0;
}
// coarse level `level` -> fine level `level - 1`
int up(ws_net *N, CView in, View out, int C, int n, int level, hipStream_t s) {
  const int H = N->H >> level, W = N->W >> level;
  hipLaunchKernelGGL(k_up2, dim3(blocks((int64_t)n * 4 * H * W * C)), dim3(kBlock), 0, s, in, out, n, H,
                     W, C);
  WS_HIP(hipGetLastError());
  return 0;
}
int up_bwd(ws_net *N, CView fine, View coarse, int C, int n, int level, hipStream_t s) {
  const int H = N->H >> level, W = N->W >> level;
  hipLaunchKernelGGL(k_up2_bwd, dim3(blocks((int64_t)n * H * W * C)), dim3(kBlock), 0, s, fine, coarse, n,
                     H, W, C);
  WS_HIP(hipGetLastError());
  return 0;
}

int pack_weights(ws_net *N, hipStream_t s) {
  for (int i = 0; i < kLayers; ++i) {
    const Layer &l = N->L[i];
    const int64_t e = (int64_t)l.Co * l.Kp + (int64_t)l.Ci * l.Kpb;
    hipLaunchKernelGGL(k_pack_weights, dim3(blocks(e)), dim3(kBlock), 0, s,
                       (const float *)(N->params + l.w_off), l.Ci, l.Co, l.Kp, l.Kpb, l.wf, l.wb);
  }
  WS_HIP(hipGetLastError());
  return 0;
}

// forward pass of n samples whose fp32 inputs are at x; network output at N->out
int forward(ws_net *N, const float *x, int n, hipStream_t s) {
  const int c = N->c;
  Layer *L = N->L;
  const int64_t np0 = npx_at(N, n, 0);
  hipLaunchKernelGGL(k_input, dim3(blocks(np0 * N->cin_pad)), dim3(kBlock), 0, s, x, N->cin, vw(N->X),
                     np0);
  WS_TRY(conv(N, L[0], cv(N->X), vw(N->A0), n, false, s));
  WS_TRY(conv(N, L[1], cv(N->A0), vw(N->C0, 2 * c), n, false, s));           // s0
  WS_TRY(pool(N, cv(N->C0, 2 * c), vw(N->P1), c, n, 0, s));
  WS_TRY(conv(N, L[2], cv(N->P1), vw(N->A1), n, false, s));
  WS_TRY(conv(N, L[3], cv(N->A1), vw(N->C1, 4 * c), n, false, s));           // s1
  WS_TRY(pool(N, cv(N->C1, 4 * c), vw(N->P2), 2 * c, n, 1, s));
  WS_TRY(conv(N, L[4], cv(N->P2), vw(N->A2), n, false, s));
  WS_TRY(conv(N, L[5], cv(N->A2), vw(N->C2, 4 * c), n, false, s));           // s2
  WS_TRY(pool(N, cv(N->C2, 4 * c), vw(N->P3), 4 * c, n, 2, s));
  WS_TRY(conv(N, L[6], cv(N->P3), vw(N->BT), n, false, s));
  WS_TRY(up(N, cv(N->BT), vw(N->C2, 0), 4 * c, n, 3, s));
  WS_TRY(conv(N, L[7], cv(N->C2), vw(N->D2), n, false, s));
  WS_TRY(up(N, cv(N->D2), vw(N->C1, 0), 4 * c, n, 2, s));
  WS_TRY(conv(N, L[8], cv(N->C1), vw(N->D1), n, false, s));
  WS_TRY(up(N, cv(N->D1), vw(N->C0, 0), 2 * c, n, 1, s));
  WS_TRY(conv(N, L[9], cv(N->C0), vw(N->D0), n, false, s));
  hipLaunchKernelGGL(k_head, dim3(blocks(np0)), dim3(kBlock), 0, s, cv(N->D0),
                     (const float *)(N->params + N->head_off), c, np0, N->out);
  WS_HIP(hipGetLastError());
  return 0;
}

// loss of N->out against t and every parameter gradient into N->grads
int backward(ws_net *N, const float *t, int n, hipStream_t s) {
  const int c = N->c;
  Layer *L = N->L;
  const int64_t np0 = npx_at(N, n, 0);
  hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kBlock), 0, s, (const float *)N->out, t, np0, N->dout,
                     N->lpart);
  hipLaunchKernelGGL(k_head_bwd, dim3(kHeadBlocks), dim3(kBlock), 0, s, cv(N->D0),
                     (const float *)(N->params + N->head_off), c, np0, (const float *)N->dout, vw(N->dD0),
                     N->hpart);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, (const float *)N->hpart, kHeadBlocks,
                     (int64_t)(c + 1), N->grads + N->head_off);
  WS_HIP(hipGetLastError());
  // level 0 decoder
  WS_TRY(relu_mask(N, vw(N->dD0), cv(N->D0), c, n, 0, s));
  WS_TRY(wgrad(N, L[9], cv(N->C0), cv(N->dD0), n, s));
  WS_TRY(conv(N, L[9], cv(N->dD0), vw(N->dC0), n, true, s));
  WS_TRY(up_bwd(N, cv(N->dC0, 0), vw(N->dD1), 2 * c, n, 1, s));
  WS_TRY(relu_mask(N, vw(N->dD1), cv(N->D1), 2 * c, n, 1, s));
  WS_TRY(wgrad(N, L[8], cv(N->C1), cv(N->dD1), n, s));
  WS_TRY(conv(N, L[8], cv(N->dD1), vw(N->dC1), n, true, s));
  WS_TRY(up_bwd(N, cv(N->dC1, 0), vw(N->dD2), 4 * c, n, 2, s));
  WS_TRY(relu_mask(N, vw(N->dD2), cv(N->D2), 4 * c, n, 2, s));
  WS_TRY(wgrad(N, L[7], cv(N->C2), cv(N->dD2), n, s));
  WS_TRY(conv(N, L[7], cv(N->dD2), vw(N->dC2), n, true, s));
  WS_TRY(up_bwd(N, cv(N->dC2, 0), vw(N->dBT), 4 * c, n, 3, s));
  WS_TRY(relu_mask(N, vw(N->dBT), cv(N->BT), 4 * c, n, 3, s));
  WS_TRY(wgrad(N, L[6], cv(N->P3), cv(N->dBT), n, s));
  WS_TRY(conv(N, L[6], cv(N->dBT), vw(N->dP3), n, true, s));
  // encoder, level 2
  WS_TRY(pool_bwd_add(N, cv(N->dP3), vw(N->dC2, 4 * c), 4 * c, n, 2, s));
  WS_TRY(relu_mask(N, vw(N->dC2, 4 * c), cv(N->C2, 4 * c), 4 * c, n, 2, s));
  WS_TRY(wgrad(N, L[5], cv(N->A2), cv(N->dC2, 4 * c), n, s));
  WS_TRY(conv(N, L[5], cv(N->dC2, 4 * c), vw(N->dA2), n, true, s));
  WS_TRY(relu_mask(N, vw(N->dA2), cv(N->A2), 4 * c, n, 2, s));
  WS_TRY(wgrad(N, L[4], cv(N->P2), cv(N->dA2), n, s));
  WS_TRY(conv(N, L[4], cv(N->dA2), vw(N->dP2), n, true, s));
  // level 1
  WS_TRY(pool_bwd_add(N, cv(N->dP2), vw(N->dC1, 4 * c), 2 * c, n, 1, s));
  WS_TRY(relu_mask(N, vw(N->dC1, 4 * c), cv(N->C1, 4 * c), 2 * c, n, 1, s));
  WS_TRY(wgrad(N, L[3], cv(N->A1), cv(N->dC1, 4 * c), n, s));
  WS_TRY(conv(N, L[3], cv(N->dC1, 4 * c), vw(N->dA1), n, true, s));
  WS_TRY(relu_mask(N, vw(N->dA1), cv(N->A1), 2 * c, n, 1, s));
  WS_TRY(wgrad(N, L[2], cv(N->P1), cv(N->dA1), n, s));
  WS_TRY(conv(N, L[2], cv(N->dA1), vw(N->dP1), n, true, s));
  // level 0
  WS_TRY(pool_bwd_add(N, cv(N->dP1), vw(N->dC0, 2 * c), c, n, 0, s));
  WS_TRY(relu_mask(N, vw(N->dC0, 2 * c), cv(N->C0, 2 * c), c, n, 0, s));
  WS_TRY(wgrad(N, L[1], cv(N->A0), cv(N->dC0, 2 * c), n, s));
  WS_TRY(conv(N, L[1], cv(N->dC0, 2 * c), vw(N->dA0), n, true, s));
  WS_TRY(relu_mask(N, vw(N->dA0), cv(N->A0), c, n, 0, s));
  WS_TRY(wgrad(N, L[0], cv(N->X), cv(N->dA0), n, s));
  return 0;
}

int read_loss(ws_net *N, int n, hipStream_t s, double *loss) {
  double part[kLossBlocks];
  WS_HIP(hipMemcpyAsync(part, N->lpart, sizeof(part), hipMemcpyDeviceToHost, s));
  WS_HIP(hipStreamSynchronize(s));
  double sum = 0.0;
  for (double p : part) sum += p;
  *loss = sum / (double)npx_at(N, n, 0);
  return 0;
}

int adam(ws_net *N, float lr, hipStream_t s) {
  N->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)N->step), c2 = 1.f - std::pow(b2, (float)N->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(N->nparams)), dim3(kBlock), 0, s, N->params,
                     (const float *)N->grads, N->m, N->v, N->nparams, lr, b1, b2, 1e-8f, c1, c2);
  WS_HIP(hipGetLastError());
  return pack_weights(N, s);
}

// gather samples idx[0..n) of (x, t) into the batch buffers
__global__ __launch_bounds__(kBlock) void k_gather_batch(const float *__restrict__ x, const float *__restrict__ t,
                                                         const int *__restrict__ idx, int n, int64_t px,
                                                         int cin, float *__restrict__ bx,
                                                         float *__restrict__ bt) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)n * px) return;
  const int j = (int)(e / px);
  const int64_t q = e % px;
  const int64_t src = (int64_t)idx[j] * px + q;
  for (int c = 0; c < cin; ++c) bx[e * cin + c] = x[src * cin + c];
  bt[e] = t[src];
}

__global__ __launch_bounds__(kBlock) void k_scale(const float *__restrict__ a, float s, int64_t n,
                                                  float *__restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) b[e] = s * a[e];
}

uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int ws_create(ws_net **out, int32_t H, int32_t W, int32_t cin, int32_t c, uint64_t seed) {
  if (!out) return -1;
  *out = nullptr;
  if (H < 8 || W < 8 || H % 8 || W % 8 || cin < 1 || cin > 16 || c != 16) return -1;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return -5;
  int dev = 0;
  WS_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  WS_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return -5;
  ws_net *N = new ws_net();
  N->H = H;
  N->W = W;
  N->cin = cin;
  N->c = c;
  // (Ci, Co, level) of the ten 3x3 layers
  const int spec[kLayers][3] = {{16, c, 0},         {c, c, 0},         {c, 2 * c, 1},
                                {2 * c, 2 * c, 1},  {2 * c, 4 * c, 2}, {4 * c, 4 * c, 2},
                                {4 * c, 4 * c, 3},  {8 * c, 4 * c, 2}, {6 * c, 2 * c, 1},
                                {3 * c, c, 0}};
  int64_t off = 0, wtot = 0;
  for (int i = 0; i < kLayers; ++i) {
    Layer &l = N->L[i];
    l.Ci = spec[i][0];
    l.Co = spec[i][1];
    l.level = spec[i][2];
    l.Kp = (int)up32(9 * l.Ci);
    l.Kpb = (int)up32(9 * l.Co);
    l.w_off = off;
    off += (int64_t)l.Co * 9 * l.Ci;
    l.b_off = off;
    off += l.Co;
    wtot += (int64_t)l.Co * l.Kp + (int64_t)l.Ci * l.Kpb;
  }
  N->head_off = off;
  off += c + 1;
  N->nparams = off;
  auto fail = [&](int code) {
    ws_destroy(N);
    return code;
  };
  // the parameter block stays first in `allocs` (ensure_batch frees the rest)
  size_t pbytes = 4 * (size_t)N->nparams * sizeof(float) + (size_t)wtot * sizeof(uint16_t) +
                  (size_t)kWgradBlocks * 64 * 9 * 128 * sizeof(float) +
                  (size_t)std::max(kColBlocks * 128, kHeadBlocks * 17) * sizeof(float) +
                  kLossBlocks * sizeof(double) + 1024;
  char *base = nullptr;
  if (alloc(N, (void **)&base, pbytes)) return fail(-2);
  auto carve = [&](size_t bytes) {
    char *p = base;
    base += (bytes + 255) / 256 * 256;
    return (void *)p;
  };
  N->params = (float *)carve(N->nparams * sizeof(float));
  N->grads = (float *)carve(N->nparams * sizeof(float));
  N->m = (float *)carve(N->nparams * sizeof(float));
  N->v = (float *)carve(N->nparams * sizeof(float));
  N->part = (float *)carve((size_t)kWgradBlocks * 64 * 9 * 128 * sizeof(float));
  N->hpart = (float *)carve((size_t)std::max(kColBlocks * 128, kHeadBlocks * 17) * sizeof(float));
  N->lpart = (double *)carve(kLossBlocks * sizeof(double));
  for (int i = 0; i < kLayers; ++i) {
    Layer &l = N->L[i];
    l.wf = (uint16_t *)carve((size_t)l.Co * l.Kp * sizeof(uint16_t));
    l.wb = (uint16_t *)carve((size_t)l.Ci * l.Kpb * sizeof(uint16_t));
  }
  (void)pbytes;
  // He-uniform initial weights, zero biases, small head
  std::vector<float> p((size_t)N->nparams, 0.f);
  uint64_t st = seed;
  auto uni = [&]() { return (float)((splitmix(st) >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f; };
  for (int i = 0; i < kLayers; ++i) {
    const Layer &l = N->L[i];
    const int ci_true = i == 0 ? cin : l.Ci;
    const float a = std::sqrt(6.f / (9.f * ci_true));
    for (int co = 0; co < l.Co; ++co)
      for (int tap = 0; tap < 9; ++tap)
        for (int ci = 0; ci < l.Ci; ++ci)
          p[l.w_off + ((int64_t)co * 9 + tap) * l.Ci + ci] = ci < ci_true ? a * uni() : 0.f;
  }
  for (int k = 0; k < c; ++k) p[N->head_off + k] = 0.1f * uni();
  if (ws_set_params(N, p.data()) != 0) return fail(-3);
  *out = N;
  return 0;
}

int ws_destroy(ws_net *N) {
  if (!N) return 0;
  (void)hipDeviceSynchronize();
  for (void *p : N->allocs) (void)hipFree(p);
  delete N;
  return 0;
}

int64_t ws_num_params(const ws_net *N) { return N ? N->nparams : -1; }

int ws_get_params(ws_net *N, float *host) {
  if (!N || !host) return -1;
  WS_HIP(hipMemcpy(host, N->params, N->nparams * sizeof(float), hipMemcpyDeviceToHost));
  return 0;
}

int ws_set_params(ws_net *N, const float *host) {
  if (!N || !host) return -1;
  WS_HIP(hipMemcpy(N->params, host, N->nparams * sizeof(float), hipMemcpyHostToDevice));
  WS_HIP(hipMemset(N->m, 0, N->nparams * sizeof(float)));
  WS_HIP(hipMemset(N->v, 0, N->nparams * sizeof(float)));
  N->step = 0;
  WS_TRY(pack_weights(N, nullptr));
  WS_HIP(hipDeviceSynchronize());
  return 0;
}

int ws_forward(ws_net *N, const float *x, float *y, int32_t count, float scale, void *stream) {
  if (!N || !x || !y || count < 0) return -1;
  hipStream_t s = (hipStream_t)stream;
  WS_TRY(ensure_batch(N, kMaxBatch));
  const int64_t px = (int64_t)N->H * N->W;
  for (int64_t i = 0; i < count; i += kMaxBatch) {
    const int n = (int)std::min<int64_t>(kMaxBatch, count - i);
    WS_TRY(forward(N, x + i * px * N->cin, n, s));
    hipLaunchKernelGGL(k_scale, dim3(blocks(n * px)), dim3(kBlock), 0, s, (const float *)N->out, scale,
                       n * px, y + i * px);
    WS_HIP(hipGetLastError());
  }
  WS_HIP(hipStreamSynchronize(s));
  return 0;
}

int ws_gradients(ws_net *N, const float *x, const float *t, int32_t count, float *grad, double *loss) {
  if (!N || !x || !t || !grad || !loss || count < 1 || count > kMaxBatch) return -1;
  WS_TRY(ensure_batch(N, kMaxBatch));
  WS_TRY(forward(N, x, count, nullptr));
  WS_TRY(backward(N, t, count, nullptr));
  WS_TRY(read_loss(N, count, nullptr, loss));
  WS_HIP(hipMemcpy(grad, N->grads, N->nparams * sizeof(float), hipMemcpyDeviceToHost));
  return 0;
}

int ws_train(ws_net *N, const float *x, const float *t, int64_t count, int32_t batch, int32_t epochs,
             float lr, uint64_t seed, double *loss_hist) {
  if (!N || !x || !t || count < 1 || batch < 1 || batch > kMaxBatch || epochs < 0 || !(lr > 0.f))
    return -1;
  WS_TRY(ensure_batch(N, kMaxBatch));
  hipStream_t s = nullptr;
  const int64_t px = (int64_t)N->H * N->W;
  std::vector<int> order((size_t)count);
  for (int64_t i = 0; i < count; ++i) order[i] = (int)i;
  uint64_t st = seed;
  const int64_t steps_per_epoch = (count + batch - 1) / batch;
  const double total = (double)steps_per_epoch * epochs;
  int64_t k = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t i = count - 1; i > 0; --i) std::swap(order[i], order[splitmix(st) % (uint64_t)(i + 1)]);
    double sum = 0.0;
    for (int64_t b0 = 0; b0 < count; b0 += batch, ++k) {
      const int n = (int)std::min<int64_t>(batch, count - b0);
      WS_HIP(hipMemcpyAsync(N->idx, order.data() + b0, n * sizeof(int), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_gather_batch, dim3(blocks(n * px)), dim3(kBlock), 0, s, x, t,
                         (const int *)N->idx, n, px, N->cin, N->bx, N->bt);
      WS_HIP(hipGetLastError());
      WS_TRY(forward(N, N->bx, n, s));
      WS_TRY(backward(N, N->bt, n, s));
      const float rate = (float)(lr * (0.55 + 0.45 * std::cos(M_PI * (double)k / total)));
      WS_TRY(adam(N, rate, s));
      double l = 0.0;
      WS_TRY(read_loss(N, n, s, &l));
      sum += l;
    }
    if (loss_hist) loss_hist[e] = sum / (double)steps_per_epoch;
  }
  WS_HIP(hipStreamSynchronize(s));
  return 0;
}

}  // extern "C"
