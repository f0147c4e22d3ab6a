// Host orchestration of the learned surrogate detector behind include/seg_nn.h:
// parameter table, workspace carve-up, forward, loss and backward passes, and
// the RMSProp update. Every arithmetic step runs in the kernels of k_nn.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "nn_internal.h"
#include "seg_nn.h"

namespace {

using namespace seg::nn;

// ---- parameter table: (rows, cols) of each weight matrix, bias = rows
struct PDef {
  int rows, cols;
};
enum PId { T1, T2, T3, E1A, E1B, E2A, E2B, E3A, E3B, U2, D2A, D2B, U1, D1A, D1B, FO, NPAR };
const PDef kP[NPAR] = {
    {32, 5},          // t1: temporal, 1 -> 32, kernel 5, stride 5
    {32, 160},        // t2: 32 -> 32, kernel 5, stride 2, pad 2
    {32, 160},        // t3: 32 -> 32, kernel 5 (length 5 -> 1)
    {32, 32 * 9},     // e1a
    {32, 32 * 9},     // e1b
    {64, 32 * 9},     // e2a
    {64, 64 * 9},     // e2b
    {128, 64 * 9},    // e3a
    {128, 128 * 9},   // e3b
    {64 * 4, 128},    // u2: transposed 2x2, 128 -> 64 (rows = co*4 + a*2 + b)
    {64, 128 * 9},    // d2a (concat 64 + 64)
    {64, 64 * 9},     // d2b
    {32 * 4, 64},     // u1: transposed 2x2, 64 -> 32
    {32, 64 * 9},     // d1a (concat 32 + 32)
    {32, 32 * 9},     // d1b
    {1, 32},          // output 1x1
};
// The summary-image network (paper's input, Sec. III-C): no temporal
// layers, and the first convolution reads the two channels (S, T).
const PDef kPst[NPAR] = {
    {0, 0}, {0, 0}, {0, 0},
    {32, 2 * 9},      // e1a: (S, T) -> 32
    {32, 32 * 9}, {64, 32 * 9}, {64, 64 * 9}, {128, 64 * 9}, {128, 128 * 9}, {64 * 4, 128},
    {64, 128 * 9}, {64, 64 * 9}, {32 * 4, 64}, {32, 64 * 9}, {32, 32 * 9}, {1, 32},
};
int bias_len(const PDef* P, int id) { return (id == U2 || id == U1) ? P[id].rows / 4 : P[id].rows; }

struct POff {
  size_t w[NPAR], b[NPAR], total;
};
POff param_offsets(const PDef* P) {
  POff o{};
  size_t at = 0;
  for (int i = 0; i < NPAR; ++i) {
    o.w[i] = at;
    at += (size_t)P[i].rows * P[i].cols;
    o.b[i] = at;
    at += bias_len(P, i);
  }
  o.total = at;
  return o;
}

constexpr int L = 50;
constexpr int SPLITS = 32;   // split-K for weight gradients (K = pixels)

struct Buf {
  size_t off, bytes;
};

struct Plan {
  int B, H, W;
  long long N, N2, N4;  // pixels at full, half and quarter resolution (times batch)
  // activations (FP32)
  Buf x0, a1, a2, a3, e1a, cat1, p1, e2a, cat2, p2, e3a, b3, z2, d2a, d2, z1, d1a, d1, logit, prob;
  Buf arg1, arg2;  // pool argmax (u8)
  // gradients of the activations (FP32)
  Buf ga1, ga2, ga3, ge1a, gcat1, gp1, ge2a, gcat2, gp2, ge3a, gb3, gz2, gd2a, gd2, gz1, gd1a, gd1, glogit;
  Buf col, dcol, splitk, lossp;
  Buf wb, grad, vel;   // BF16 weights, FP32 gradients, RMSProp state
  Buf wr;              // 3 x 3 convolution weights reordered for the direct kernel
  size_t wr_off[NPAR]; // element offset of each 3 x 3 layer in wr
  size_t total;
};

Plan make_plan(int B, int H, int W, bool st) {
  Plan p{};
  p.B = B;
  p.H = H;
  p.W = W;
  p.N = (long long)B * H * W;
  p.N2 = p.N / 4;
  p.N4 = p.N / 16;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    Buf b{at, bytes};
    at = (at + bytes + 255) & ~size_t(255);
    return b;
  };
  const size_t f = 4;
  const long long N = p.N, N2 = p.N2, N4 = p.N4;
  const long long tn = st ? 0 : 1;   // temporal activations (frames input only)
  p.x0 = take(f * (st ? 2 : L) * N);
  p.a1 = take(f * 32 * 10 * N * tn);
  p.a2 = take(f * 32 * 5 * N * tn);
  p.a3 = take(f * 32 * N * tn);
  p.e1a = take(f * 32 * N);
  p.cat1 = take(f * 64 * N);
  p.p1 = take(f * 32 * N2);
  p.e2a = take(f * 64 * N2);
  p.cat2 = take(f * 128 * N2);
  p.p2 = take(f * 64 * N4);
  p.e3a = take(f * 128 * N4);
  p.b3 = take(f * 128 * N4);
  p.z2 = take(f * 256 * N4);
  p.d2a = take(f * 64 * N2);
  p.d2 = take(f * 64 * N2);
  p.z1 = take(f * 128 * N2);
  p.d1a = take(f * 32 * N);
  p.d1 = take(f * 32 * N);
  p.logit = take(f * N);
  p.prob = take(f * N);
  p.arg1 = take(32 * N2);
  p.arg2 = take(64 * N4);
  p.ga1 = take(f * 32 * 10 * N * tn);
  p.ga2 = take(f * 32 * 5 * N * tn);
  p.ga3 = take(f * 32 * N * tn);
  p.ge1a = take(f * 32 * N);
  p.gcat1 = take(f * 64 * N);
  p.gp1 = take(f * 32 * N2);
  p.ge2a = take(f * 64 * N2);
  p.gcat2 = take(f * 128 * N2);
  p.gp2 = take(f * 64 * N4);
  p.ge3a = take(f * 128 * N4);
  p.gb3 = take(f * 128 * N4);
  p.gz2 = take(f * 256 * N4);
  p.gd2a = take(f * 64 * N2);
  p.gd2 = take(f * 64 * N2);
  p.gz1 = take(f * 128 * N2);
  p.gd1a = take(f * 32 * N);
  p.gd1 = take(f * 32 * N);
  p.glogit = take(f * N);
  // largest im2col: 160 rows x 5N (t2) vs 576 rows x N (d1a) vs 1152 x N2 ...
  long long colmax = 160 * 5 * N;
  colmax = std::max(colmax, 5LL * 10 * N);
  colmax = std::max(colmax, 576LL * N);
  colmax = std::max(colmax, 1152LL * N2);
  colmax = std::max(colmax, 1152LL * N4);
  p.col = take(2 * colmax);
  p.dcol = take(f * colmax);
  p.splitk = take(f * (size_t)SPLITS * 256 * 1152);
  p.lossp = take(f * ((N + 255) / 256 + 1));
  const POff po = param_offsets(st ? kPst : kP);
  p.wb = take(2 * po.total);
  {
    const PDef* P = st ? kPst : kP;
    size_t at_wr = 0;
    for (int i = 0; i < NPAR; ++i) {
      p.wr_off[i] = at_wr;
      if (P[i].rows > 0 && P[i].cols % 9 == 0 && i >= E1A && i != U2 && i != U1 && i != FO)
        at_wr += (conv3_reordered_size(P[i].rows, P[i].cols / 9) + 7) / 8 * 8;
    }
    p.wr = take(2 * at_wr);
  }
  p.grad = take(f * po.total);
  p.vel = take(f * po.total);
  p.total = at;
  return p;
}

}  // namespace

struct seg_nn {
  Plan plan;
  POff po;
  const PDef* P;   // parameter table of the input mode
  bool st;         // input: summary-image patches (S, T) instead of frames
  char* ws;
  float* params;   // caller's FP32 master weights
  int device;
  int batch;       // batch of the last forward
};

namespace {

template <class T>
T* at(seg_nn* n, const Buf& b) {
  return reinterpret_cast<T*>(n->ws + b.off);
}
const uint16_t* wbf(seg_nn* n, int id) { return at<uint16_t>(n, n->plan.wb) + n->po.w[id]; }
const float* bias(seg_nn* n, int id) { return n->params + n->po.b[id]; }

// refreshes the reordered copy of every 3 x 3 convolution's BF16 weights
void reorder_conv3(seg_nn* n, hipStream_t st) {
  for (int id = E1A; id < NPAR; ++id)
    if (id != U2 && id != U1 && id != FO)
      conv3_reorder(wbf(n, id), at<uint16_t>(n, n->plan.wr) + n->plan.wr_off[id], n->P[id].rows,
                    n->P[id].cols / 9, st);
}
float* gw(seg_nn* n, int id) { return at<float>(n, n->plan.grad) + n->po.w[id]; }
float* gb(seg_nn* n, int id) { return at<float>(n, n->plan.grad) + n->po.b[id]; }

hipError_t gemm_wx(seg_nn* n, int id, const void* X, bool x_bf16, long long ncols, float* Y, hipStream_t st) {
  // Y [rows][ncols] = W [rows][cols] X [cols][ncols]
  GemmOp g{};
  g.A = wbf(n, id);
  g.sam = n->P[id].cols;
  g.sak = 1;
  g.a_bf16 = true;
  g.B = X;
  g.sbk = ncols;
  g.sbn = 1;
  g.b_bf16 = x_bf16;
  g.C = Y;
  g.M = n->P[id].rows;
  g.N = (int)ncols;
  g.K = n->P[id].cols;
  g.splits = 1;
  return gemm(g, st);
}

hipError_t gemm_wtdy(seg_nn* n, int id, const float* dY, long long ncols, float* dX, hipStream_t st) {
  // dX [cols][ncols] = W^T [cols][rows] dY [rows][ncols]
  GemmOp g{};
  g.A = wbf(n, id);
  g.sam = 1;
  g.sak = n->P[id].cols;
  g.a_bf16 = true;
  g.B = dY;
  g.sbk = ncols;
  g.sbn = 1;
  g.b_bf16 = false;
  g.C = dX;
  g.M = n->P[id].cols;
  g.N = (int)ncols;
  g.K = n->P[id].rows;
  g.splits = 1;
  return gemm(g, st);
}

hipError_t gemm_dw(seg_nn* n, int id, const float* dY, const void* X, bool x_bf16, long long ncols, hipStream_t st) {
  // dW [rows][cols] = dY [rows][ncols] X^T [ncols][cols]   (X stored [cols][ncols])
  GemmOp g{};
  g.A = dY;
  g.sam = ncols;
  g.sak = 1;
  g.a_bf16 = false;
  g.B = X;
  g.sbk = 1;
  g.sbn = ncols;
  g.b_bf16 = x_bf16;
  g.C = gw(n, id);
  g.M = n->P[id].rows;
  g.N = n->P[id].cols;
  g.K = (int)ncols;
  g.splits = SPLITS;
  g.scratch = at<float>(n, n->plan.splitk);
  return gemm(g, st);
}

// 3x3 convolution + bias (+ ReLU): X [Ci][Bn H W] -> Y [Co][Bn H W]
hipError_t conv3(seg_nn* n, int id, const float* X, int Bn, int H, int W, float* Y, bool relu, hipStream_t st) {
  const int Ci = n->P[id].cols / 9;
  const long long N = (long long)Bn * H * W;
  hipError_t e = hipSuccess;
  const uint16_t* wr = at<uint16_t>(n, n->plan.wr) + n->plan.wr_off[id];
  if (!conv3_implicit(wbf(n, id), wr, X, Y, n->P[id].rows, Ci, Bn, H, W, bias(n, id), relu, st)) {
    uint16_t* col = at<uint16_t>(n, n->plan.col);
    im2col3(X, col, Ci, Bn, H, W, st);
    e = gemm_wx(n, id, col, true, N, Y, st);
    bias_act(Y, bias(n, id), n->P[id].rows, N, relu, st);
  }
  return e;
}

// backward of conv3: dY (modified in place by the ReLU mask), weight and bias
// gradients, input gradient into dX (accumulated when acc)
hipError_t conv3_bwd(seg_nn* n, int id, const float* X, const float* Y, float* dY, int Bn, int H, int W,
                     float* dX, bool acc, bool relu, hipStream_t st) {
  const int Ci = n->P[id].cols / 9, Co = n->P[id].rows;
  const long long N = (long long)Bn * H * W;
  if (relu) relu_bwd(dY, Y, (long long)Co * N, st);
  bias_grad(dY, gb(n, id), Co, N, st);
  uint16_t* col = at<uint16_t>(n, n->plan.col);
  im2col3(X, col, Ci, Bn, H, W, st);
  hipError_t e = gemm_dw(n, id, dY, col, true, N, st);
  if (e != hipSuccess) return e;
  if (!dX) return hipSuccess;
  float* dcol = at<float>(n, n->plan.dcol);
  e = gemm_wtdy(n, id, dY, N, dcol, st);
  col2im3(dcol, dX, Ci, Bn, H, W, acc, st);
  return e;
}

hipError_t forward(seg_nn* n, const uint16_t* frames, const float* stin, int Bn, hipStream_t st) {
  const Plan& p = n->plan;
  const int H = p.H, W = p.W;
  const long long HW = (long long)H * W;
  const long long N = Bn * HW, N2 = N / 4, N4 = N / 16;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  float* x0 = at<float>(n, p.x0);
  uint16_t* col = at<uint16_t>(n, p.col);
  const float* unet_in = nullptr;   // input of the first 3x3 convolution
  if (n->st) {
    st_norm(stin, x0, Bn, HW, st);
    unet_in = x0;
  } else {
    tnorm(frames, x0, Bn, L, HW, st);
    // temporal convolutions
    float* a1 = at<float>(n, p.a1);
    im2col1(x0, col, 1, L, 10, 5, 5, 0, N, st);
    chk(gemm_wx(n, T1, col, true, 10 * N, a1, st));
    bias_act(a1, bias(n, T1), 32, 10 * N, true, st);
    float* a2 = at<float>(n, p.a2);
    im2col1(a1, col, 32, 10, 5, 5, 2, 2, N, st);
    chk(gemm_wx(n, T2, col, true, 5 * N, a2, st));
    bias_act(a2, bias(n, T2), 32, 5 * N, true, st);
    float* a3 = at<float>(n, p.a3);
    chk(gemm_wx(n, T3, a2, false, N, a3, st));     // a2 viewed as [160][N]
    bias_act(a3, bias(n, T3), 32, N, true, st);
    unet_in = a3;
  }
  // U-Net encoder
  float* e1a = at<float>(n, p.e1a);
  float* cat1 = at<float>(n, p.cat1);
  float* s1 = cat1 + 32 * N;
  chk(conv3(n, E1A, unet_in, Bn, H, W, e1a, true, st));
  chk(conv3(n, E1B, e1a, Bn, H, W, s1, true, st));
  float* p1 = at<float>(n, p.p1);
  pool(s1, p1, at<uint8_t>(n, p.arg1), 32 * Bn, H, W, st);
  float* e2a = at<float>(n, p.e2a);
  float* cat2 = at<float>(n, p.cat2);
  float* s2 = cat2 + 64 * N2;
  chk(conv3(n, E2A, p1, Bn, H / 2, W / 2, e2a, true, st));
  chk(conv3(n, E2B, e2a, Bn, H / 2, W / 2, s2, true, st));
  float* p2 = at<float>(n, p.p2);
  pool(s2, p2, at<uint8_t>(n, p.arg2), 64 * Bn, H / 2, W / 2, st);
  float* e3a = at<float>(n, p.e3a);
  float* b3 = at<float>(n, p.b3);
  chk(conv3(n, E3A, p2, Bn, H / 4, W / 4, e3a, true, st));
  chk(conv3(n, E3B, e3a, Bn, H / 4, W / 4, b3, true, st));
  // decoder
  float* z2 = at<float>(n, p.z2);
  if (!up_direct(wbf(n, U2), b3, bias(n, U2), cat2, 64, 128, Bn, H / 4, W / 4, st)) {
    chk(gemm_wx(n, U2, b3, false, N4, z2, st));
    up_scatter(z2, bias(n, U2), cat2, 64, Bn, H / 4, W / 4, st);
  }
  float* d2a = at<float>(n, p.d2a);
  float* d2 = at<float>(n, p.d2);
  chk(conv3(n, D2A, cat2, Bn, H / 2, W / 2, d2a, true, st));
  chk(conv3(n, D2B, d2a, Bn, H / 2, W / 2, d2, true, st));
  float* z1 = at<float>(n, p.z1);
  if (!up_direct(wbf(n, U1), d2, bias(n, U1), cat1, 32, 64, Bn, H / 2, W / 2, st)) {
    chk(gemm_wx(n, U1, d2, false, N2, z1, st));
    up_scatter(z1, bias(n, U1), cat1, 32, Bn, H / 2, W / 2, st);
  }
  float* d1a = at<float>(n, p.d1a);
  float* d1 = at<float>(n, p.d1);
  chk(conv3(n, D1A, cat1, Bn, H, W, d1a, true, st));
  chk(conv3(n, D1B, d1a, Bn, H, W, d1, true, st));
  float* logit = at<float>(n, p.logit);
  if (!conv1_out(wbf(n, FO), d1, bias(n, FO), logit, n->P[FO].cols, N, st)) {
    chk(gemm_wx(n, FO, d1, false, N, logit, st));
    bias_act(logit, bias(n, FO), 1, N, false, st);
  }
  chk(hipGetLastError());
  return e;
}

// Forward pass for inference: the U-Net's activations are kept as BF16 in
// channel blocks of 16 (half the bytes of every layer's reads and writes, 16
// bytes per load). Every consumer of an activation takes it rounded to BF16
// (the convolutions' staging, the transposed convolutions, the output layer;
// a maximum commutes with the rounding) and every product sums in the same
// order, so the logits are the same as forward()'s. The 2 x 2 poolings and
// the output layer with its sigmoid run in the epilogues of the convolutions
// before them; the probabilities go to `prob`. Returns false, with nothing
// left that forward() does not redo, when a layer's shape does not fit the
// BF16 kernels (H not a multiple of 4 or W of 64); *err gets launch errors.
bool forward_infer(seg_nn* n, const uint16_t* frames, const float* stin, int Bn, float* prob, hipStream_t st,
                   hipError_t* err) {
  const Plan& p = n->plan;
  const int H = p.H, W = p.W;
  const long long HW = (long long)H * W;
  const long long N = Bn * HW, N2 = N / 4;
  if (H % 4 || W % 64) return false;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  float* x0 = at<float>(n, p.x0);
  const void* unet_in = nullptr;
  bool unet_bf16 = false;   // the U-Net's input: FP32 planar, or BF16 in channel blocks
  if (n->st) {
    st_norm(stin, x0, Bn, HW, st);
    unet_in = x0;
  } else {
    // the frame normalisation runs inside the first temporal convolution;
    // the other two gather their im2col as they load it, with bias and ReLU
    // in the product's epilogue; a1, a2 and a3 are stored as BF16 (their
    // consumers round them to BF16), a3 in channel blocks for the U-Net
    uint16_t* a1 = at<uint16_t>(n, p.a1);
    uint16_t* a2 = at<uint16_t>(n, p.a2);
    uint16_t* a3 = at<uint16_t>(n, p.a3);
    if (!(tconv1_h(frames, L, wbf(n, T1), n->P[T1].rows, n->P[T1].cols, bias(n, T1), a1, Bn, HW, st) &&
          tconv(wbf(n, T2), 32, a1, true, 32, 10, 5, 5, 2, 2, N, bias(n, T2), true, a2, 1, st) &&
          tconv(wbf(n, T3), 32, a2, true, 32, 5, 1, 5, 1, 0, N, bias(n, T3), true, a3, 2, st)))
      return false;
    unet_in = a3;
    unet_bf16 = true;
  }
  auto h = [&](const Buf& b) { return at<uint16_t>(n, b); };
  auto conv = [&](int id, const void* X, bool x_bf16, uint16_t* Y, int hh, int ww, int mode, const ConvEpi& ep) {
    return conv3_h(wbf(n, id), at<uint16_t>(n, p.wr) + p.wr_off[id], X, x_bf16, Y, n->P[id].rows, n->P[id].cols / 9,
                   Bn, hh, ww, bias(n, id), true, mode, ep, st);
  };
  // activations in the FP32 buffers' memory, as BF16 in channel blocks
  uint16_t *e1a = h(p.e1a), *cat1 = h(p.cat1), *s1 = cat1 + 32 * N, *p1 = h(p.p1);
  uint16_t *e2a = h(p.e2a), *cat2 = h(p.cat2), *s2 = cat2 + 64 * N2, *p2 = h(p.p2);
  uint16_t *e3a = h(p.e3a), *b3 = h(p.b3), *d2a = h(p.d2a), *d2 = h(p.d2), *d1a = h(p.d1a);
  const ConvEpi none;
  ConvEpi pool1, pool2, out;
  pool1.pool = p1;
  pool2.pool = p2;
  out.wo = wbf(n, FO);
  out.bo = bias(n, FO);
  out.z = at<float>(n, p.logit);
  out.prob = prob;
  // the pooling after e1b and e2b and the output layer after d1b run in
  // those convolutions' epilogues
  // the first two convolutions in one kernel where they fit it (summary
  // U-Net: 2 input channels), else one after the other
  const bool first2 =
      !unet_bf16 &&
      conv3_first2_h(wbf(n, E1A), bias(n, E1A), n->P[E1A].rows, n->P[E1A].cols / 9, static_cast<const float*>(unet_in),
                     at<uint16_t>(n, p.wr) + p.wr_off[E1B], bias(n, E1B), n->P[E1B].rows, n->P[E1B].cols / 9, s1, p1,
                     Bn, H, W, st);
  const bool ok = n->P[FO].cols == 32 &&
                  (first2 || (conv(E1A, unet_in, unet_bf16, e1a, H, W, CONV_STORE, none) &&
                              conv(E1B, e1a, true, s1, H, W, CONV_POOL, pool1))) &&
                  conv(E2A, p1, true, e2a, H / 2, W / 2, CONV_STORE, none) &&
                  conv(E2B, e2a, true, s2, H / 2, W / 2, CONV_POOL, pool2) &&
                  conv(E3A, p2, true, e3a, H / 4, W / 4, CONV_STORE, none) &&
                  conv(E3B, e3a, true, b3, H / 4, W / 4, CONV_STORE, none) &&
                  up2_h(wbf(n, U2), b3, bias(n, U2), cat2, 64, 128, Bn, H / 4, W / 4, st) &&
                  conv(D2A, cat2, true, d2a, H / 2, W / 2, CONV_STORE, none) &&
                  conv(D2B, d2a, true, d2, H / 2, W / 2, CONV_STORE, none) &&
                  up2_h(wbf(n, U1), d2, bias(n, U1), cat1, 32, 64, Bn, H / 2, W / 2, st) &&
                  conv(D1A, cat1, true, d1a, H, W, CONV_STORE, none) &&
                  conv(D1B, d1a, true, nullptr, H, W, CONV_OUT, out);
  chk(hipGetLastError());
  *err = e;
  return ok;
}

hipError_t backward(seg_nn* n, int Bn, hipStream_t st) {
  const Plan& p = n->plan;
  const int H = p.H, W = p.W;
  const long long N = (long long)Bn * H * W, N2 = N / 4, N4 = N / 16;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  float* gl = at<float>(n, p.glogit);
  float* d1 = at<float>(n, p.d1);
  float* gd1 = at<float>(n, p.gd1);
  // output 1x1
  bias_grad(gl, gb(n, FO), 1, N, st);
  chk(gemm_dw(n, FO, gl, d1, false, N, st));
  chk(gemm_wtdy(n, FO, gl, N, gd1, st));
  // d1b, d1a
  float* d1a = at<float>(n, p.d1a);
  float* gd1a = at<float>(n, p.gd1a);
  float* cat1 = at<float>(n, p.cat1);
  float* gcat1 = at<float>(n, p.gcat1);
  chk(conv3_bwd(n, D1B, d1a, d1, gd1, Bn, H, W, gd1a, false, true, st));
  chk(conv3_bwd(n, D1A, cat1, d1a, gd1a, Bn, H, W, gcat1, false, true, st));
  // u1: channels 0..31 of cat1 came from the transposed convolution
  float* gz1 = at<float>(n, p.gz1);
  float* d2 = at<float>(n, p.d2);
  float* gd2 = at<float>(n, p.gd2);
  bias_grad(gcat1, gb(n, U1), 32, N, st);
  up_gather(gcat1, gz1, 32, Bn, H / 2, W / 2, st);
  chk(gemm_dw(n, U1, gz1, d2, false, N2, st));
  chk(gemm_wtdy(n, U1, gz1, N2, gd2, st));
  // d2b, d2a
  float* d2a = at<float>(n, p.d2a);
  float* gd2a = at<float>(n, p.gd2a);
  float* cat2 = at<float>(n, p.cat2);
  float* gcat2 = at<float>(n, p.gcat2);
  chk(conv3_bwd(n, D2B, d2a, d2, gd2, Bn, H / 2, W / 2, gd2a, false, true, st));
  chk(conv3_bwd(n, D2A, cat2, d2a, gd2a, Bn, H / 2, W / 2, gcat2, false, true, st));
  // u2: channels 0..63 of cat2
  float* gz2 = at<float>(n, p.gz2);
  float* b3 = at<float>(n, p.b3);
  float* gb3 = at<float>(n, p.gb3);
  bias_grad(gcat2, gb(n, U2), 64, N2, st);
  up_gather(gcat2, gz2, 64, Bn, H / 4, W / 4, st);
  chk(gemm_dw(n, U2, gz2, b3, false, N4, st));
  chk(gemm_wtdy(n, U2, gz2, N4, gb3, st));
  // bottleneck
  float* e3a = at<float>(n, p.e3a);
  float* ge3a = at<float>(n, p.ge3a);
  float* p2 = at<float>(n, p.p2);
  float* gp2 = at<float>(n, p.gp2);
  chk(conv3_bwd(n, E3B, e3a, b3, gb3, Bn, H / 4, W / 4, ge3a, false, true, st));
  chk(conv3_bwd(n, E3A, p2, e3a, ge3a, Bn, H / 4, W / 4, gp2, false, true, st));
  // skip 2 = channels 64..127 of cat2: its gradient is the concat part plus the pool path
  float* gs2 = gcat2 + 64 * N2;
  pool_bwd(gp2, at<uint8_t>(n, p.arg2), gs2, 64 * Bn, H / 2, W / 2, true, st);
  float* e2a = at<float>(n, p.e2a);
  float* ge2a = at<float>(n, p.ge2a);
  float* p1 = at<float>(n, p.p1);
  float* gp1 = at<float>(n, p.gp1);
  chk(conv3_bwd(n, E2B, e2a, cat2 + 64 * N2, gs2, Bn, H / 2, W / 2, ge2a, false, true, st));
  chk(conv3_bwd(n, E2A, p1, e2a, ge2a, Bn, H / 2, W / 2, gp1, false, true, st));
  float* gs1 = gcat1 + 32 * N;
  pool_bwd(gp1, at<uint8_t>(n, p.arg1), gs1, 32 * Bn, H, W, true, st);
  float* e1a = at<float>(n, p.e1a);
  float* ge1a = at<float>(n, p.ge1a);
  float* a3 = at<float>(n, p.a3);
  float* ga3 = at<float>(n, p.ga3);
  chk(conv3_bwd(n, E1B, e1a, cat1 + 32 * N, gs1, Bn, H, W, ge1a, false, true, st));
  if (n->st) {   // the input needs no gradient
    chk(conv3_bwd(n, E1A, at<float>(n, p.x0), e1a, ge1a, Bn, H, W, nullptr, false, true, st));
    chk(hipGetLastError());
    return e;
  }
  chk(conv3_bwd(n, E1A, a3, e1a, ge1a, Bn, H, W, ga3, false, true, st));
  // temporal convolutions
  float* a2 = at<float>(n, p.a2);
  float* ga2 = at<float>(n, p.ga2);
  relu_bwd(ga3, a3, 32 * N, st);
  bias_grad(ga3, gb(n, T3), 32, N, st);
  chk(gemm_dw(n, T3, ga3, a2, false, N, st));
  chk(gemm_wtdy(n, T3, ga3, N, ga2, st));
  float* a1 = at<float>(n, p.a1);
  float* ga1 = at<float>(n, p.ga1);
  uint16_t* col = at<uint16_t>(n, p.col);
  float* dcol = at<float>(n, p.dcol);
  relu_bwd(ga2, a2, 32 * 5 * N, st);
  bias_grad(ga2, gb(n, T2), 32, 5 * N, st);
  im2col1(a1, col, 32, 10, 5, 5, 2, 2, N, st);
  chk(gemm_dw(n, T2, ga2, col, true, 5 * N, st));
  chk(gemm_wtdy(n, T2, ga2, 5 * N, dcol, st));
  col2im1(dcol, ga1, 32, 10, 5, 5, 2, 2, N, st);
  relu_bwd(ga1, a1, 32 * 10 * N, st);
  bias_grad(ga1, gb(n, T1), 32, 10 * N, st);
  im2col1(at<float>(n, p.x0), col, 1, L, 10, 5, 5, 0, N, st);
  chk(gemm_dw(n, T1, ga1, col, true, 10 * N, st));
  chk(hipGetLastError());
  return e;
}

int enter(seg_nn* n) {
  if (!n) return SEG_E_INVAL;
  return hipSetDevice(n->device) == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

}  // namespace

extern "C" {

int seg_nn_param_count(size_t* n) {
  if (!n) return SEG_E_INVAL;
  *n = param_offsets(kP).total;
  return SEG_OK;
}

int seg_nn_st_param_count(size_t* n) {
  if (!n) return SEG_E_INVAL;
  *n = param_offsets(kPst).total;
  return SEG_OK;
}

static int layout_of(const PDef* P, uint32_t index, uint32_t* rows, uint32_t* cols, size_t* w_offset,
                     size_t* b_offset) {
  if (index >= (uint32_t)NPAR) return SEG_E_INVAL;
  const POff o = param_offsets(P);
  if (rows) *rows = (uint32_t)P[index].rows;
  if (cols) *cols = (uint32_t)P[index].cols;
  if (w_offset) *w_offset = o.w[index];
  if (b_offset) *b_offset = o.b[index];
  return SEG_OK;
}

int seg_nn_param_layout(uint32_t index, uint32_t* rows, uint32_t* cols, size_t* w_offset, size_t* b_offset) {
  return layout_of(kP, index, rows, cols, w_offset, b_offset);
}

int seg_nn_st_param_layout(uint32_t index, uint32_t* rows, uint32_t* cols, size_t* w_offset, size_t* b_offset) {
  return layout_of(kPst, index, rows, cols, w_offset, b_offset);
}

static int ws_bytes(uint32_t batch, uint32_t height, uint32_t width, bool st, size_t* bytes) {
  if (!bytes || batch < 1 || height < 4 || width < 4 || height % 4 || width % 4) return SEG_E_INVAL;
  if ((long long)batch * height * width * 576 >= (1LL << 31)) return SEG_E_INVAL;
  *bytes = make_plan((int)batch, (int)height, (int)width, st).total;
  return SEG_OK;
}

int seg_nn_workspace_bytes(uint32_t batch, uint32_t height, uint32_t width, size_t* bytes) {
  return ws_bytes(batch, height, width, false, bytes);
}

int seg_nn_st_workspace_bytes(uint32_t batch, uint32_t height, uint32_t width, size_t* bytes) {
  return ws_bytes(batch, height, width, true, bytes);
}

static int create(uint32_t batch, uint32_t height, uint32_t width, bool st, float* dev_params, void* dev_workspace,
                  size_t bytes, seg_nn** out) {
  if (!out || !dev_params || !dev_workspace) return SEG_E_INVAL;
  *out = nullptr;
  size_t need = 0;
  int e = ws_bytes(batch, height, width, st, &need);
  if (e) return e;
  if (bytes < need) return SEG_E_CAPACITY;
  if (reinterpret_cast<uintptr_t>(dev_workspace) & 255) return SEG_E_INVAL;
  seg_nn* n = new (std::nothrow) seg_nn();
  if (!n) return SEG_E_INVAL;
  n->plan = make_plan((int)batch, (int)height, (int)width, st);
  n->P = st ? kPst : kP;
  n->st = st;
  n->po = param_offsets(n->P);
  n->ws = static_cast<char*>(dev_workspace);
  n->params = dev_params;
  n->batch = 0;
  if (hipGetDevice(&n->device) != hipSuccess) {
    delete n;
    return SEG_E_DEVICE;
  }
  *out = n;
  return SEG_OK;
}

int seg_nn_create(uint32_t batch, uint32_t height, uint32_t width, float* dev_params, void* dev_workspace,
                  size_t bytes, seg_nn** out) {
  return create(batch, height, width, false, dev_params, dev_workspace, bytes, out);
}

int seg_nn_st_create(uint32_t batch, uint32_t height, uint32_t width, float* dev_params, void* dev_workspace,
                     size_t bytes, seg_nn** out) {
  return create(batch, height, width, true, dev_params, dev_workspace, bytes, out);
}

int seg_nn_sync_weights(seg_nn* n, void* stream) {
  int e = enter(n);
  if (e) return e;
  hipStream_t st = static_cast<hipStream_t>(stream);
  to_bf16_copy(n->params, at<uint16_t>(n, n->plan.wb), (long long)n->po.total, st);
  reorder_conv3(n, st);
  if (hipMemsetAsync(at<float>(n, n->plan.vel), 0, n->po.total * 4, st) != hipSuccess) return SEG_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

static int run_forward(seg_nn* n, const uint16_t* frames, const float* stin, uint32_t batch, float* dev_prob,
                       void* stream) {
  int e = enter(n);
  if (e) return e;
  if ((n->st ? (const void*)stin : (const void*)frames) == nullptr || batch < 1 || (int)batch > n->plan.B)
    return SEG_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t fe = hipSuccess;
  float* prob = dev_prob ? dev_prob : at<float>(n, n->plan.prob);
  if (!forward_infer(n, frames, stin, (int)batch, prob, st, &fe)) {
    fe = forward(n, frames, stin, (int)batch, st);
    const long long N = (long long)batch * n->plan.H * n->plan.W;
    bce(at<float>(n, n->plan.logit), nullptr, nullptr, prob, nullptr, N, st);
  }
  if (fe != hipSuccess) return SEG_E_DEVICE;
  n->batch = (int)batch;
  return hipGetLastError() == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

static int run_backward(seg_nn* n, const uint16_t* frames, const float* stin, const float* dev_labels,
                        uint32_t batch, float* dev_grad, float* host_loss, void* stream) {
  int e = enter(n);
  if (e) return e;
  if ((n->st ? (const void*)stin : (const void*)frames) == nullptr || !dev_labels || batch < 1 ||
      (int)batch > n->plan.B)
    return SEG_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (forward(n, frames, stin, (int)batch, st) != hipSuccess) return SEG_E_DEVICE;
  const long long N = (long long)batch * n->plan.H * n->plan.W;
  float* part = at<float>(n, n->plan.lossp);
  bce(at<float>(n, n->plan.logit), dev_labels, at<float>(n, n->plan.glogit), at<float>(n, n->plan.prob), part, N,
      st);
  if (backward(n, (int)batch, st) != hipSuccess) return SEG_E_DEVICE;
  n->batch = (int)batch;
  if (dev_grad &&
      hipMemcpyAsync(dev_grad, at<float>(n, n->plan.grad), n->po.total * 4, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return SEG_E_DEVICE;
  if (host_loss) {
    const long long nb = (N + 255) / 256;
    std::vector<float> h(nb);
    if (hipMemcpyAsync(h.data(), part, nb * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SEG_E_DEVICE;
    double s = 0.0;
    for (long long i = 0; i < nb; ++i) s += h[i];
    *host_loss = (float)(s / (double)N);
  }
  return hipGetLastError() == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

int seg_nn_forward(seg_nn* n, const uint16_t* dev_frames, uint32_t batch, float* dev_prob, void* stream) {
  if (n && n->st) return SEG_E_STATE;
  return run_forward(n, dev_frames, nullptr, batch, dev_prob, stream);
}

int seg_nn_backward(seg_nn* n, const uint16_t* dev_frames, const float* dev_labels, uint32_t batch,
                    float* dev_grad, float* host_loss, void* stream) {
  if (n && n->st) return SEG_E_STATE;
  return run_backward(n, dev_frames, nullptr, dev_labels, batch, dev_grad, host_loss, stream);
}

int seg_nn_st_forward(seg_nn* n, const float* dev_st, uint32_t batch, float* dev_prob, void* stream) {
  if (n && !n->st) return SEG_E_STATE;
  return run_forward(n, nullptr, dev_st, batch, dev_prob, stream);
}

int seg_nn_st_backward(seg_nn* n, const float* dev_st, const float* dev_labels, uint32_t batch, float* dev_grad,
                       float* host_loss, void* stream) {
  if (n && !n->st) return SEG_E_STATE;
  return run_backward(n, nullptr, dev_st, dev_labels, batch, dev_grad, host_loss, stream);
}

int seg_nn_st_patch_count(uint32_t height, uint32_t width, uint32_t* n) {
  if (!n || height < 64 || width < 64) return SEG_E_INVAL;
  *n = (uint32_t)(st_origins((int)height) * st_origins((int)width));
  return SEG_OK;
}

int seg_nn_st_patches(const float* dev_S, const float* dev_T, uint32_t height, uint32_t width, float* dev_out,
                      void* stream) {
  if (!dev_S || !dev_T || !dev_out || height < 64 || width < 64) return SEG_E_INVAL;
  st_patches(dev_S, dev_T, (int)height, (int)width, dev_out, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

int seg_nn_st_merge(const float* dev_prob, uint32_t height, uint32_t width, float* dev_out, void* stream) {
  if (!dev_prob || !dev_out || height < 64 || width < 64) return SEG_E_INVAL;
  st_merge(dev_prob, (int)height, (int)width, dev_out, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

int seg_nn_input(const seg_nn* n, uint32_t* input) {
  if (!n || !input) return SEG_E_INVAL;
  *input = n->st ? SEG_NN_INPUT_SUMMARIES : SEG_NN_INPUT_FRAMES;
  return SEG_OK;
}

int seg_nn_step(seg_nn* n, float lr, float rho, float eps, void* stream) {
  int e = enter(n);
  if (e) return e;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rmsprop(n->params, at<float>(n, n->plan.grad), at<float>(n, n->plan.vel), at<uint16_t>(n, n->plan.wb),
          (long long)n->po.total, lr, rho, eps, st);
  reorder_conv3(n, st);
  return hipGetLastError() == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

int seg_nn_logits(seg_nn* n, float* dev_out, void* stream) {
  int e = enter(n);
  if (e) return e;
  if (!dev_out || n->batch < 1) return SEG_E_STATE;
  const long long N = (long long)n->batch * n->plan.H * n->plan.W;
  return hipMemcpyAsync(dev_out, at<float>(n, n->plan.logit), N * 4, hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEG_OK
             : SEG_E_DEVICE;
}

int seg_nn_gemm_test(const float* A, int a_trans, const float* B, int b_trans, float* C, int M, int N, int K,
                     int splits, float* scratch, void* stream) {
  // C [M][N] = op(A) op(B) with A stored [M][K] (or [K][M] when a_trans) and
  // B stored [K][N] (or [N][K] when b_trans); operands rounded to BF16
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return SEG_E_INVAL;
  GemmOp g{};
  g.A = A;
  g.sam = a_trans ? 1 : K;
  g.sak = a_trans ? M : 1;
  g.B = B;
  g.sbk = b_trans ? 1 : N;
  g.sbn = b_trans ? K : 1;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.splits = splits;
  g.scratch = scratch;
  return gemm(g, static_cast<hipStream_t>(stream)) == hipSuccess ? SEG_OK : SEG_E_DEVICE;
}

int seg_nn_shape(const seg_nn* n, uint32_t* batch, uint32_t* height, uint32_t* width) {
  if (!n) return SEG_E_INVAL;
  if (batch) *batch = (uint32_t)n->plan.B;
  if (height) *height = (uint32_t)n->plan.H;
  if (width) *width = (uint32_t)n->plan.W;
  return SEG_OK;
}

int seg_nn_destroy(seg_nn* n) {
  delete n;
  return SEG_OK;
}

}  // extern "C"
