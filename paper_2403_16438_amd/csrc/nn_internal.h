// Internal declarations of the surrogate detector's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace seg {
namespace nn {

// C (+)= op(A) op(B), operands FP32 or BF16 (given by the flags), FP32 out,
// row-major C with ldc = N. splits > 1 splits K over blocks; the partials go
// to `scratch` (splits * M * N floats) and are summed in order.
struct GemmOp {
  const void* A;
  long long sam, sak;
  bool a_bf16;
  const void* B;
  long long sbk, sbn;
  bool b_bf16;
  float* C;
  int M, N, K;
  int splits;
  float* scratch;
  bool accumulate;
};
hipError_t gemm(const GemmOp& g, hipStream_t st);

void im2col3(const float* X, uint16_t* col, int C, int Bn, int H, int W, hipStream_t st);
// Y [Co][Bn H W] = W [Co][Ci 9] (BF16) times the 3 x 3 im2col of X, plus bias
// and ReLU, without an im2col matrix: a direct convolution over LDS halo
// tiles (Wr: the weights reordered by conv3_reorder), else the product that
// gathers the im2col inside; false (nothing launched) when neither applies
// (W % 8 or Ci 9 % 8 not 0), and the caller takes the im2col + GEMM path.
bool conv3_implicit(const uint16_t* Wb, const uint16_t* Wr, const float* X, float* Y, int Co, int Ci, int Bn,
                    int H, int W, const float* bias, bool relu, hipStream_t st);
// Transposed 2 x 2 convolution, stride 2, with its bias, written straight to
// channels 0 .. Co - 1 of Y [.][Bn][2 h][2 w]:
// Y[co][b][2 y + a][2 x + e] = bias[co] + sum_c W[4 co + 2 a + e][c] X[c][b][y][x]
// (BF16 operands, FP32 accumulation). False (nothing launched) when Bn h w or
// Ci is not a multiple of 8 or W, X are not 16-byte aligned.
bool up_direct(const uint16_t* Wb, const float* X, const float* bias, float* Y, int Co, int Ci, int Bn, int h,
               int w, hipStream_t st);
// Y [N] = bias[0] + W [1][C] X [C][N] (BF16 operands, FP32 accumulation);
// always launched (returns true).
bool conv1_out(const uint16_t* Wb, const float* X, const float* bias, float* Y, int C, long long N, hipStream_t st);
// BF16 activations (inference) are kept in channel blocks of 16: element
// (c, b, y, x) of [C][Bn][H][W] (C a multiple of 16) at
// ((c / 16) Bn H W + (b H + y) W + x) 16 + c % 16.
// Epilogues of conv3_h:
//   CONV_STORE  Y only;
//   CONV_POOL   Y and its 2 x 2 max pooling ep.pool [C][Bn][H / 2][W / 2]
//               (blocked), the values k_pool would take;
//   CONV_OUT    not Y but the 1 x 1 output layer on it (Co = 32): logits
//               ep.z [Bn H W] = ep.bo[0] + sum_c ep.wo[c] Y[c] (as conv1_out)
//               and ep.prob = 1 / (1 + exp(-z)) (as bce).
enum { CONV_STORE = 0, CONV_POOL = 1, CONV_OUT = 2 };
struct ConvEpi {
  uint16_t* pool = nullptr;
  const uint16_t* wo = nullptr;
  const float* bo = nullptr;
  float* z = nullptr;
  float* prob = nullptr;
};
// The halo-tile convolution with X FP32 planar or BF16 blocked (x_bf16) and
// Y BF16 blocked, the BF16 rounding of what conv3_implicit stores, with the
// epilogue `mode`; false (nothing launched) when the shape or the epilogue
// does not fit the halo tiles.
bool conv3_h(const uint16_t* Wb, const uint16_t* Wr, const void* X, bool x_bf16, uint16_t* Y, int Co, int Ci, int Bn,
             int H, int W, const float* bias, bool relu, int mode, const ConvEpi& ep, hipStream_t st);
// A temporal convolution as one product without an im2col matrix:
// Y [Co][Tout Np] = W [Co][C KT] (BF16) times the 1-D im2col of BF16
// X [C][Tin][Np] that im2col1 would write (rounded), plus bias and ReLU,
// stored as FP32 (y_bf16 = 0), as BF16 row-major (1) or, with one output
// sample, as BF16 in channel blocks of 16 (2, Co a multiple of 16); the same
// MFMA sums as im2col1 + gemm + bias_act. False (nothing launched) unless
// x_bf16, Co <= 32, Np is a multiple of 8 and W, X, Y are 16-byte aligned.
bool tconv(const uint16_t* Wb, int Co, const void* X, bool x_bf16, int C, int Tin, int Tout, int KT, int S, int P,
           long long Np, const float* bias, bool relu, void* Y, int y_bf16, hipStream_t st);
// The first two 3 x 3 convolutions of the summary U-Net in one pass: e1a
// (W1 [32][2 9], bias b1, ReLU) on the planar FP32 input X [2][Bn][H][W],
// kept in LDS, then e1b (W2r: its conv3_reorder copy, bias b2, ReLU) with
// the 2 x 2 pooling: Y and Yp as conv3_h's CONV_POOL writes them, the same
// values as conv3_h for e1a then for e1b. False (nothing launched) unless
// the layers are 2 -> 32 -> 32 channels, H is a multiple of 4 and W of 64.
bool conv3_first2_h(const uint16_t* W1, const float* b1, int Co1, int Ci1, const float* X, const uint16_t* W2r,
                    const float* b2, int Co2, int Ci2, uint16_t* Y, uint16_t* Yp, int Bn, int H, int W,
                    hipStream_t st);
// up_direct on BF16 blocked X and Y, each input pixel read once; false
// (nothing launched) unless Co is 32 or 64 and Ci 64 or 128.
bool up2_h(const uint16_t* Wb, const uint16_t* X, const float* bias, uint16_t* Y, int Co, int Ci, int Bn, int h, int w,
           hipStream_t st);
// Wr [ceil(Ci / 16)][Co][9][16] from W [Co][Ci 9] (zero past Ci)
void conv3_reorder(const uint16_t* Wb, uint16_t* Wr, int Co, int Ci, hipStream_t st);
size_t conv3_reordered_size(int Co, int Ci);
void col2im3(const float* dcol, float* dX, int C, int Bn, int H, int W, bool acc, hipStream_t st);
void tnorm(const uint16_t* frames, float* out, int Bn, int L, long long HW, hipStream_t st);
// tnorm and the first temporal convolution (W [32][5], stride 5, no padding,
// bias and ReLU) in one pass for inference, a1 [32][10][Bn HW] as BF16: the
// same values as tnorm, im2col1, gemm and bias_act rounded to BF16. False
// (nothing launched) unless L = 50, Co = 32, KT = 5, Bn HW is a multiple of
// 64 and a1 is 16-byte aligned.
bool tconv1_h(const uint16_t* frames, int L, const uint16_t* Wb, int Co, int KT, const float* bias, uint16_t* a1,
              int Bn, long long HW, hipStream_t st);
void im2col1(const float* in, uint16_t* col, int C, int Tin, int Tout, int KT, int S, int P, long long N,
             hipStream_t st);
void col2im1(const float* dcol, float* din, int C, int Tin, int Tout, int KT, int S, int P, long long N,
             hipStream_t st);
void bias_act(float* Y, const float* b, int C, long long N, bool relu, hipStream_t st);
void relu_bwd(float* dY, const float* Y, long long n, hipStream_t st);
void bias_grad(const float* dY, float* db, int C, long long N, hipStream_t st);
void pool(const float* X, float* Y, uint8_t* arg, int CB, int H, int W, hipStream_t st);
void pool_bwd(const float* dY, const uint8_t* arg, float* dX, int CB, int H, int W, bool acc, hipStream_t st);
void up_scatter(const float* Z, const float* b, float* Y, int Co, int Bn, int h, int w, hipStream_t st);
void up_gather(const float* dY, float* dZ, int Co, int Bn, int h, int w, hipStream_t st);
void bce(const float* z, const float* y, float* dz, float* prob, float* part, long long n, hipStream_t st);
void rmsprop(float* w, const float* g, float* v, uint16_t* wb, long long n, float lr, float rho, float eps,
             hipStream_t st);
void to_bf16_copy(const float* w, uint16_t* wb, long long n, hipStream_t st);

// summary-image input (S, T): st [Bn][2][HW] -> x [2][Bn HW] with channel 0
// the patch-standardised S and channel 1 T / sqrt(S + 25)
void st_norm(const float* st, float* x, int Bn, long long HW, hipStream_t stream);
// 64 x 64 patches at origins every 32 pixels, the last one flush with the edge
int st_origins(int n);
void st_patches(const float* S, const float* T, int H, int W, float* out, hipStream_t stream);
// tent-weighted mean of patch probabilities [n_patch][64][64] over the frame
void st_merge(const float* prob, int H, int W, float* out, hipStream_t stream);
// the same for n segments in one launch: S, T and out planes H W apart,
// patches [n][n_patch][2][64][64], probabilities [n][n_patch][64][64]
void st_patches_n(const float* S, const float* T, int H, int W, int n, float* out, hipStream_t stream);
void st_merge_n(const float* prob, int H, int W, int n, float* out, hipStream_t stream);

}  // namespace nn
}  // namespace seg
