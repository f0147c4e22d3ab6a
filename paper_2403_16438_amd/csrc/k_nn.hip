// Kernels of the learned surrogate detector (the spiking-pixel identifier of
// Sec. III-C: temporal convolutions feeding a 2-D U-Net). Activations are
// FP32 in a [channel][batch][row][col] layout, so a convolution is one GEMM
// whose output is already the next activation; matrix operands are rounded to
// BF16 (round to nearest even) and multiplied on MFMA with FP32 accumulation.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "nn_internal.h"

namespace seg {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Activations of the BF16 inference path are kept in channel blocks of 16:
// element (c, b, y, x) of a [C][Bn][H][W] tensor (C a multiple of 16) sits at
// ((c / 16) Bn H W + (b H + y) W + x) 16 + c % 16, so the 16 channels of one
// pixel are 32 contiguous bytes. A 16-byte load then brings 8 channels of one
// position, the depth order of an MFMA operand, where the planar layout took
// one 2-byte load per channel; a concatenation along channels is still two
// adjacent ranges of the buffer.
__device__ __forceinline__ long long cblk(int c, long long pix, long long npix) {
  return ((long long)(c >> 4) * npix + pix) * 16 + (c & 15);
}

template <class T>
__device__ __forceinline__ uint16_t ld_bf16(const T* p, long long i);
template <>
__device__ __forceinline__ uint16_t ld_bf16<uint16_t>(const uint16_t* p, long long i) {
  return p[i];
}
template <>
__device__ __forceinline__ uint16_t ld_bf16<float>(const float* p, long long i) {
  return to_bf16(p[i]);
}

// ---------------------------------------------------------------- GEMM
// C[m][n] (+)= sum_k A(m, k) B(k, n); A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn]. Block: 256 threads, 64 x 64 tile, K step 32.
// Split-K over gridDim.z writes partial tiles to C + z*M*ldc (summed later).
constexpr int GT = 64, GK = 32;

template <class TA, class TB>
__global__ __launch_bounds__(256) void k_gemm(const TA* __restrict__ A, long long sam, long long sak,
                                              const TB* __restrict__ B, long long sbk, long long sbn,
                                              float* __restrict__ C, long long ldc, int M, int N, int K,
                                              int kchunk, int accumulate) {
  __shared__ uint16_t As[GT][GK + 8];   // [m][k]
  __shared__ uint16_t Bs[GT][GK + 8];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  float* Cz = C + (long long)blockIdx.z * M * ldc;
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      int m, k;
      if (sak == 1) {
        m = e / GK;
        k = e % GK;
      } else {
        k = e / GT;
        m = e % GT;
      }
      const int gm = m0 + m, gk = k0 + k;
      As[m][k] = (gm < M && gk < kend) ? ld_bf16(A, gm * sam + gk * sak) : (uint16_t)0;
      int n, kb;
      if (sbn == 1) {
        kb = e / GT;
        n = e % GT;
      } else {
        n = e / GK;
        kb = e % GK;
      }
      const int gn = n0 + n, gkb = k0 + kb;
      Bs[n][kb] = (gn < N && gkb < kend) ? ld_bf16(B, gkb * sbk + gn * sbn) : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      const int kk = ks + (lane >> 5) * 8;
      bf16x8 a, b;
      const uint16_t* ap = &As[wm * 32 + (lane & 31)][kk];
      const uint16_t* bp = &Bs[wn * 32 + (lane & 31)][kk];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = __builtin_bit_cast(__bf16, ap[q]);
        b[q] = __builtin_bit_cast(__bf16, bp[q]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = n0 + wn * 32 + (lane & 31);
  if (col >= N) return;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm * 32 + 8 * g + 4 * (lane >> 5) + r;
      if (row < M) {
        float* c = Cz + (long long)row * ldc + col;
        *c = accumulate ? *c + acc[4 * g + r] : acc[4 * g + r];
      }
    }
}

// Contiguous BF16 operands (A [M][K] with K fastest, B [K][N] with N
// fastest, rows 16-byte aligned): each thread moves 16-byte groups of 8, and
// the next K step is loaded into registers while the current one runs on
// MFMA. Tile MT x NT (64 x 64, or 32 x 128 for M <= 32), 4 waves of 32 x 32.
// The B operand by MODE:
//   GV_BF16   B itself;
//   GV_IM2COL the 3 x 3 im2col matrix of the FP32 activations X [Ci][Bn][H][W]
//             (row k = c 9 + ky 3 + kx, column n = pixel), gathered from X as
//             it is loaded (W a multiple of 8, so a group of 8 pixels lies in
//             one row);
//   GV_UP     FP32 X [K][N] (row stride sbk) rounded to BF16 as it is loaded,
//             for the transposed 2 x 2 convolution: row 4 co + 2 a + e of the
//             product, plus bias[co], is stored to C at channel co, pixel
//             (2 y + a, 2 x + e) of an image of 2 H x 2 W (X's pixels H x W),
//             so the product lands directly in the concatenation buffer;
//   GV_TCONV  the 1-D temporal im2col of BF16 X [C][Tin][Np]: row
//             k = c KT + tap, column j Np + n holds
//             X[c][j S + tap - P][n] (zero outside 0 .. Tin - 1), what
//             im2col1 would write, gathered as it is loaded (Np a multiple
//             of 8, so a group of 8 columns lies in one j); C is stored as
//             FP32, or as BF16 bits when `out_h` (row-major when 1; when 2,
//             with rows as channels in blocks of 16, see cblk).
enum { GV_BF16 = 0, GV_IM2COL = 1, GV_UP = 2, GV_TCONV = 3 };
struct Im2col {
  const float* X;
  int Bn, H, W;
  // GV_TCONV
  const void* TX;
  int Tin, KT, S, P, out_h, xcd;
  long long Np;
};
// bias (may be null) and relu are applied to the stored values (not with
// accumulate), as bias_act does after an unfused product.
template <int MT, int MODE>
__global__ __launch_bounds__(256) void k_gemm_v(const uint16_t* __restrict__ A, long long sam,
                                                const uint16_t* __restrict__ B, long long sbk, Im2col ic,
                                                float* __restrict__ C, long long ldc, int M, int N, int K,
                                                int accumulate, const float* __restrict__ bias, int relu) {
  constexpr int NT = 4096 / MT;
  constexpr int NB = NT / 64;                   // 16-byte B groups per thread per K step
  __shared__ uint16_t As[MT][GK + 8];
  __shared__ uint16_t Bs[NT][GK + 8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = MT == 64 ? wv >> 1 : 0, wn = MT == 64 ? wv & 1 : wv;
  const int m0 = blockIdx.y * MT;
  int n0 = blockIdx.x * NT;
  if constexpr (MODE == GV_TCONV) {
    if (ic.xcd) {
      // The output samples j of one pixel range read overlapping input rows:
      // tile t = (pixel range, j) with j fastest, and the workgroups that the
      // dispatcher sends to one XCD (blockIdx.x mod 8) take one contiguous
      // run of tiles, so the re-reads hit that XCD's L2.
      const int T = gridDim.x, x = blockIdx.x, t = (x & 7) * (T >> 3) + (x >> 3);
      const int tout = (int)(N / ic.Np), j = t % tout;
      n0 = (int)(j * ic.Np) + (t / tout) * NT;
    }
  }
  // A: thread -> (row am, k group ak); B: thread -> (k row bk, n group bn + 64 j)
  const int am = tid >> 2, ak = (tid & 3) * 8;
  const bool a_on = am < MT;
  const int bk = tid >> 3, bn = (tid & 7) * 8;
  uint4 ra = make_uint4(0, 0, 0, 0), rb[NB];
  // MODE 1: a thread's pixel groups are fixed, so their image, row and
  // column are found once
  int py[NB], px[NB];
  long long poff[NB];
  if constexpr (MODE == GV_TCONV) {
    // a thread's column groups are fixed: sample j and pixel n found once
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int gn = n0 + bn + 64 * j;
      const long long jj = gn / ic.Np;
      py[j] = gn < N ? (int)jj * ic.S - ic.P : -(1 << 20);   // input sample of tap 0 (off-range groups load nothing)
      poff[j] = gn - jj * ic.Np;
    }
  }
  if constexpr (MODE == GV_IM2COL) {
    const int HW = ic.H * ic.W;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int gn = n0 + bn + 64 * j;
      const int b = gn / HW, yx = gn - b * HW;
      py[j] = gn < N ? yx / ic.W : -(1 << 20);      // off-range groups load nothing
      px[j] = yx - (yx / ic.W) * ic.W;
      poff[j] = (long long)b * HW;
    }
  }
  auto load = [&](int k0) {
    const int gm = m0 + am, gk = k0 + ak;
    if (MODE == GV_TCONV && (sam & 7)) {   // rows not 16-byte aligned (K of 5): element loads
      uint16_t v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (a_on && gm < M && gk + q < K) ? A[gm * sam + gk + q] : (uint16_t)0;
      ra = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16), v[4] | ((uint32_t)v[5] << 16),
                      v[6] | ((uint32_t)v[7] << 16));
    } else {
      ra = (a_on && gm < M && gk < K) ? *reinterpret_cast<const uint4*>(A + gm * sam + gk) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int gkb = k0 + bk, gn = n0 + bn + 64 * j;
      if constexpr (MODE == GV_BF16) {
        rb[j] = (gkb < K && gn < N) ? *reinterpret_cast<const uint4*>(B + gkb * sbk + gn) : make_uint4(0, 0, 0, 0);
      } else if constexpr (MODE == GV_UP) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gkb < K && gn < N) {
          const float4* src = reinterpret_cast<const float4*>(ic.X + (long long)gkb * sbk + gn);
          const float4 lo = src[0], hi = src[1];
          v = make_uint4(to_bf16(lo.x) | ((uint32_t)to_bf16(lo.y) << 16), to_bf16(lo.z) | ((uint32_t)to_bf16(lo.w) << 16),
                         to_bf16(hi.x) | ((uint32_t)to_bf16(hi.y) << 16), to_bf16(hi.z) | ((uint32_t)to_bf16(hi.w) << 16));
        }
        rb[j] = v;
      } else if constexpr (MODE == GV_TCONV) {
        uint4 v = make_uint4(0, 0, 0, 0);
        (void)gn;
        if (gkb < K) {
          const int c = gkb / ic.KT, tap = gkb - c * ic.KT;
          const int t = py[j] + tap;
          if (t >= 0 && t < ic.Tin) {
            const long long off = ((long long)c * ic.Tin + t) * ic.Np + poff[j];
            v = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(ic.TX) + off);
          }
        }
        rb[j] = v;
      } else {
        uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        (void)gn;
        if (gkb < K) {
          const int c = gkb / 9, kk = gkb - 9 * c, ky = kk / 3, kx = kk - 3 * ky;
          const int x0 = px[j], yy = py[j] + ky - 1;
          if (yy >= 0 && yy < ic.H) {
            const float* src = ic.X + (long long)c * ic.Bn * ic.H * ic.W + poff[j] + (long long)yy * ic.W;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int xx = x0 + q + kx - 1;
              v[q] = (xx >= 0 && xx < ic.W) ? to_bf16(src[xx]) : (uint16_t)0;
            }
          }
        }
        rb[j] = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                           v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16));
      }
    }
  };
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  load(0);
  for (int k0 = 0; k0 < K; k0 += GK) {
    if (a_on) *reinterpret_cast<uint4*>(&As[am][ak]) = ra;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint32_t w[4] = {rb[j].x, rb[j].y, rb[j].z, rb[j].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Bs[bn + 64 * j + 2 * q][bk] = (uint16_t)(w[q] & 0xffffu);
        Bs[bn + 64 * j + 2 * q + 1][bk] = (uint16_t)(w[q] >> 16);
      }
    }
    __syncthreads();
    if (k0 + GK < K) load(k0 + GK);
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      const int kk = ks + (lane >> 5) * 8;
      bf16x8 a, b;
      const uint16_t* ap = &As[wm * 32 + (lane & 31)][kk];
      const uint16_t* bp = &Bs[wn * 32 + (lane & 31)][kk];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = __builtin_bit_cast(__bf16, ap[q]);
        b[q] = __builtin_bit_cast(__bf16, bp[q]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  if constexpr (MODE == GV_TCONV) {
    if (ic.out_h) {
      // BF16 output: the tile goes through LDS so that each thread stores
      // 16 bytes of one row (8 columns; N is a multiple of 8)
      __shared__ __attribute__((aligned(16))) uint16_t Ts[MT][NT + 8];
      const int cl = wn * 32 + (lane & 31);
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rl = wm * 32 + 8 * g + 4 * (lane >> 5) + r, row = m0 + rl;
          float v = acc[4 * g + r];
          if (bias && row < M) {
            v += bias[row];
            if (relu) v = fmaxf(v, 0.f);
          }
          Ts[rl][cl] = to_bf16(v);
        }
      __syncthreads();
      if (ic.out_h == 2) {
        // channel blocks of 16 (M a multiple of 16, rows = channels, columns
        // = pixels): a thread gathers the 16 channels of one pixel from the
        // tile's column and stores them as 32 bytes
        for (int e = tid; e < (MT / 16) * NT; e += 256) {
          const int cb = e / NT, cl2 = e - cb * NT, gc = n0 + cl2, c0 = m0 + 16 * cb;
          uint32_t w[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) w[k] = Ts[16 * cb + 2 * k][cl2] | ((uint32_t)Ts[16 * cb + 2 * k + 1][cl2] << 16);
          if (c0 < M && gc < N) {
            uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<uint16_t*>(C) + cblk(c0, gc, N));
            dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
            dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
          }
        }
        return;
      }
      for (int e = tid; e < MT * (NT / 8); e += 256) {
        const int rl = e / (NT / 8), c8 = (e - rl * (NT / 8)) * 8, row = m0 + rl, gc = n0 + c8;
        if (row < M && gc < N)
          *reinterpret_cast<uint4*>(reinterpret_cast<uint16_t*>(C) + (long long)row * ldc + gc) =
              *reinterpret_cast<const uint4*>(&Ts[rl][c8]);
      }
      return;
    }
  }
  const int col = n0 + wn * 32 + (lane & 31);
  if (col >= N) return;
  if constexpr (MODE == GV_UP) {
    // row 4 co + 2 a + e of pixel (b, y, x) lands on (b, 2 y + a, 2 x + e) of channel co
    const int hw = ic.H * ic.W, b = col / hw, yx = col - b * hw, y = yx / ic.W, x = yx - y * ic.W;
    float* base = C + (long long)b * 4 * hw + (long long)(2 * y) * (2 * ic.W) + 2 * x;
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + 8 * g + 4 * (lane >> 5) + r;
        if (row < M) {
          const int co = row >> 2, a = (row >> 1) & 1, e = row & 1;
          base[(long long)co * ic.Bn * 4 * hw + a * 2 * ic.W + e] = acc[4 * g + r] + bias[co];
        }
      }
    return;
  }
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm * 32 + 8 * g + 4 * (lane >> 5) + r;
      if (row < M) {
        float* c = C + (long long)row * ldc + col;
        float v = accumulate ? *c + acc[4 * g + r] : acc[4 * g + r];
        if (bias) {
          v += bias[row];
          if (relu) v = fmaxf(v, 0.f);
        }
        *c = v;
      }
    }
}

// Direct 3 x 3 convolution (stride 1, zero padding 1) on MFMA, forward:
// Y[co][b][y][x] = bias[co] + sum_{c, ky, kx} W[co][9 c + 3 ky + kx] X[c][b][y + ky - 1][x + kx - 1],
// then ReLU when asked. A workgroup computes MT output channels x NT = 4096 / MT
// pixels, a block of BR rows x BC columns of one image (BC = min(W, 64)).
// Per chunk of 16 input channels it stages, as BF16 with the channel fastest,
// the input rows y0 - 1 .. y0 + BR and columns x0 - 1 .. x0 + BC (zero outside
// the image) and the chunk's weights, (ky, kx) then channel, copied with
// 16-byte loads from a reordered copy kept beside the BF16 weights. A depth
// step of 16 is then one (ky, kx) and 16 channels, and each lane's 8
// consecutive depth values are 16 contiguous bytes in both arrays: every input
// value is loaded and converted once per chunk instead of once per (ky, kx),
// and the nine offsets read it from LDS.
constexpr int HC = 16;                          // input channels per chunk
constexpr int HX = 6336;                        // largest halo tile: 6 x 66 x 16
// Convolution weights reordered for k_conv3_halo: Wr[chunk][co][ky 3 + kx][cl]
// = W[co][9 (16 chunk + cl) + ky 3 + kx] (0 past Ci), so that a chunk's
// weights of one output channel are 144 contiguous values.
__global__ void k_conv3_reorder(const uint16_t* __restrict__ Wb, uint16_t* __restrict__ Wr, int Co, int Ci) {
  const int nch = (Ci + HC - 1) / HC;
  const long long total = (long long)nch * Co * 9 * HC;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int cl = (int)(i % HC), kyx = (int)((i / HC) % 9), co = (int)((i / (9 * HC)) % Co),
            ch = (int)(i / ((long long)9 * HC * Co));
  const int c = ch * HC + cl;
  Wr[i] = c < Ci ? Wb[(long long)co * Ci * 9 + c * 9 + kyx] : (uint16_t)0;
}

// Tile of this workgroup: the dispatcher deals workgroups to the eight XCDs
// in turn, so each XCD takes a contiguous run of tiles (vertical neighbours
// within an image), whose shared halo rows are then read through one L2.
__device__ __forceinline__ int xcd_tile() {
  const int T = (int)gridDim.x, x = (int)blockIdx.x;
  return T % 8 ? x : (x & 7) * (T >> 3) + (x >> 3);
}

// the value of lane ^ 1 (the neighbouring column of a 32-pixel row block)
__device__ __forceinline__ uint32_t from_pair_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false);   // quad_perm 1, 0, 3, 2
}

// A 32 x 32 MFMA result gives lanes l and l + 32 (l < 32) channels
// 4 (l >> 5) + 0..3 (BF16 pairs a0, a1) and 8 + 4 (l >> 5) + 0..3 (b0, b1)
// of one pixel's 16-channel block. Swapping the upper half of the lanes of
// a with the lower half of b leaves each lane 8 consecutive channels, stored
// with one 16-byte store: channels 0..7 in lanes 0..31, 8..15 in 32..63.
__device__ __forceinline__ uint4 gather8(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1) {
  const auto s0 = __builtin_amdgcn_permlane32_swap(a0, b0, false, false);
  const auto s1 = __builtin_amdgcn_permlane32_swap(a1, b1, false, false);
  return make_uint4(s0[0], s1[0], s0[1], s1[1]);
}

// the value of lane + 32 (lanes 0..31)
__device__ __forceinline__ uint32_t from_upper_half(uint32_t v) {
  return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
}

// first maximum of a, b, c, d in that order, compared as BF16 values (the
// order and ties of k_pool's window scan)
__device__ __forceinline__ uint16_t max4_bf16(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
  uint16_t m = a;
  if (from_bf16(b) > from_bf16(m)) m = b;
  if (from_bf16(c) > from_bf16(m)) m = c;
  if (from_bf16(d) > from_bf16(m)) m = d;
  return m;
}

// TX: float (FP32, planar [Ci][Bn][H][W]) or uint16_t (BF16 bits, channel
// blocks of 16) input; TY: float (planar) or uint16_t (BF16, channel blocks)
// output. A BF16 output is the BF16 rounding of the FP32 value, which is what
// the next layer's staging (or the 1 x 1 output layer) makes of an FP32
// output, so the two give the same network outputs. EP (BF16 output only):
//   CONV_STORE  store the activations;
//   CONV_POOL   store them and their 2 x 2 max pooling (ep.pool, channel
//               blocks, H / 2 x W / 2), taken as k_pool takes it;
//   CONV_OUT    store nothing but the 1 x 1 output layer on them (Co = 32):
//               ep.z = ep.bo[0] + sum_c ep.wo[c] Y[c] in channel order (as
//               conv1_out) and ep.prob = 1 / (1 + exp(-z)) (as bce).
// With CONV_POOL each wave's two 32-pixel blocks are vertically adjacent
// rows, so a 2 x 2 window lies in one lane and its neighbour.
template <int MT, int NTW, typename TX, typename TY, int EP>
__global__ __launch_bounds__(256) void k_conv3_halo(const uint16_t* __restrict__ Wr, const TX* __restrict__ X,
                                                    const float* __restrict__ bias, int relu,
                                                    TY* __restrict__ Y, int Co, int Ci, int Bn, int H, int W,
                                                    int BC, ConvEpi ep) {
  constexpr bool XH = sizeof(TX) == 2, YH = sizeof(TY) == 2;
  static_assert(EP == CONV_STORE || (YH && NTW == 2), "fused epilogues take BF16 outputs and row pairs");
  constexpr int NT = 4096 / MT * NTW;   // pixels: NTW 32-pixel blocks per wave
  __shared__ __attribute__((aligned(16))) uint16_t Xs[HX];
  __shared__ __attribute__((aligned(16))) uint16_t Ws[MT][9 * HC + 8];
  __shared__ float Osh[33];   // CONV_OUT: the output layer's weights and bias
  const int BR = NT / BC, TC = BC + 2, TR = BR + 2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = MT == 64 ? wv >> 1 : 0, wn = MT == 64 ? wv & 1 : wv;
  const int bx = (W + BC - 1) / BC, by = (H + BR - 1) / BR;
  const int blk = xcd_tile(), b = blk / (bx * by), rem = blk - b * bx * by;
  const int y0 = (rem / bx) * BR, x0 = (rem % bx) * BC;
  const int co0 = blockIdx.y * MT;
  const long long HW = (long long)H * W;
  // this lane's pixels (one per 32-pixel block of the wave) and their place
  // in the halo tile: with whole 32-pixel blocks per tile row the wave's two
  // blocks are rows 2 (wn / nbr) and 2 (wn / nbr) + 1 of column block
  // wn % nbr; otherwise blocks follow the tile in raster order
  const int nbr = BC & 31 ? 0 : BC >> 5;
  int pr[NTW], pc[NTW];
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    if (NTW == 2 && nbr) {
      pr[t] = 2 * (wn / nbr) + t;
      pc[t] = (wn % nbr) * 32 + (lane & 31);
    } else {
      const int pl = (wn * NTW + t) * 32 + (lane & 31);
      pr[t] = pl / BC;
      pc[t] = pl - pr[t] * BC;
    }
  }
  const int kg = (lane >> 5) * 8;
  f32x16 acc[NTW];
#pragma unroll
  for (int t = 0; t < NTW; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
  // Staging: a thread takes items of 8 channels of a tile position (BF16
  // input: one 16-byte load; FP32 input: 8 loads, each coalesced over the
  // positions) and stores each as 16 bytes to LDS, plus 16-byte groups of the
  // reordered weights. Every load is issued unconditionally (positions
  // outside the image or channels past Ci read a valid address and are then
  // replaced by zero), so a thread's loads go out together and wait once:
  // guarded loads were issued one at a time, each waiting for the previous.
  // The next chunk's loads are issued before the current chunk's MFMAs and
  // converted only when stored.
  const int np = TR * TC;
  constexpr int XI = MT == 64 ? 1 + NTW : 2 + NTW;     // input items per thread: 2 np <= 256 XI
  constexpr int WI = (MT * 18 + 255) / 256;
  float xv[XI][8];   // FP32 input
  uint4 xq[XI];      // BF16 input
  uint4 wv4[WI];
  uint32_t okx[XI], okw = 0;   // which loaded values are real (the rest become zero)
  // per item, fixed over the chunks: its channel-0 address (position
  // clamped into the image, so always valid), its LDS offset, and whether it
  // is a real tile position inside the image. BF16 input: item e is
  // position e / 2, channels 8 (e % 2) .. + 7 of the chunk (consecutive
  // threads read consecutive 16 bytes); FP32: position e % np, channel group
  // e / np.
  const long long cs = XH ? (long long)Bn * HW * 16 : (long long)Bn * HW;   // chunk (BF16) or channel stride
  const TX* ib[XI];
  int ig[XI], so[XI];
  uint32_t iin = 0;
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int e = tid + 256 * j;
    const int g = XH ? (e & 1) : (e >= np ? 1 : 0), pos = XH ? e >> 1 : e - g * np;
    const int r = pos / TC, cc = pos - r * TC;
    const int y = y0 + r - 1, x = x0 + cc - 1;
    iin |= (uint32_t)(e < 2 * np && y >= 0 && y < H && x >= 0 && x < W) << j;
    const int yc = min(max(y, 0), H - 1), xc = min(max(x, 0), W - 1);
    const long long pix = (long long)b * HW + (long long)yc * W + xc;
    ib[j] = XH ? X + pix * 16 + 8 * g : X + pix;
    ig[j] = 8 * g;
    so[j] = pos * HC + 8 * g;
  }
  // weights: item j's row (clamped output channel) and 16-byte group
  const int wstep = Co * 9 * HC;
  int wo[WI];
#pragma unroll
  for (int j = 0; j < WI; ++j) {
    const int e = tid + 256 * j, m = e / 18, q = e - m * 18, co = co0 + m;
    okw |= (uint32_t)(e < MT * 18 && co < Co) << j;
    wo[j] = min(co0 + min(m, MT - 1), Co - 1) * 9 * HC + 8 * q;
  }
  const bool full = Ci % HC == 0;   // no chunk runs past the last channel (always so for BF16 input)
  auto load = [&](int c0) {
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      if constexpr (XH) {
        xq[j] = *reinterpret_cast<const uint4*>(ib[j] + (long long)(c0 / HC) * cs);
        okx[j] = (iin >> j & 1u) ? 0xffu : 0u;
      } else {
        const int cb = c0 + ig[j];
        if (full) {
          const TX* src = ib[j] + (long long)cb * cs;
#pragma unroll
          for (int q = 0; q < 8; ++q) xv[j][q] = src[(long long)q * cs];
          okx[j] = (iin >> j & 1u) ? 0xffu : 0u;
        } else {
          okx[j] = 0;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int c = cb + q;
            xv[j][q] = ib[j][(long long)min(c, Ci - 1) * cs];
            okx[j] |= (uint32_t)((iin >> j & 1u) && c < Ci) << q;
          }
        }
      }
    }
    const uint16_t* wsrc = Wr + (long long)(c0 / HC) * wstep;
#pragma unroll
    for (int j = 0; j < WI; ++j) wv4[j] = *reinterpret_cast<const uint4*>(wsrc + wo[j]);
  };
  load(0);
  // CONV_OUT: the output layer's weights go out with the first chunk and
  // reach LDS with it, instead of costing a memory round trip after the
  // last MFMA
  float oload = 0.f;
  if (EP == CONV_OUT && tid < 32) oload = from_bf16(ep.wo[tid]);
  else if (EP == CONV_OUT && tid == 32) oload = ep.bo[0];
  for (int c0 = 0; c0 < Ci; c0 += HC) {
    __syncthreads();
    if (EP == CONV_OUT && c0 == 0 && tid < 33) Osh[tid] = oload;
    // the loaded values are taken here whether or not they are used, so the
    // compiler keeps every load unconditional (and in flight together)
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      if constexpr (XH)
        asm volatile("" : "+v"(xq[j].x), "+v"(xq[j].y), "+v"(xq[j].z), "+v"(xq[j].w));
      else
        asm volatile("" : "+v"(xv[j][0]), "+v"(xv[j][1]), "+v"(xv[j][2]), "+v"(xv[j][3]), "+v"(xv[j][4]),
                          "+v"(xv[j][5]), "+v"(xv[j][6]), "+v"(xv[j][7]));
    }
#pragma unroll
    for (int j = 0; j < WI; ++j) asm volatile("" : "+v"(wv4[j].x), "+v"(wv4[j].y), "+v"(wv4[j].z), "+v"(wv4[j].w));
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      const int e = tid + 256 * j;
      if (e < 2 * np) {
        uint4 s;
        if constexpr (XH) {
          s = okx[j] ? xq[j] : make_uint4(0, 0, 0, 0);
        } else {
          uint16_t v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = (okx[j] >> q & 1u) ? to_bf16(xv[j][q]) : (uint16_t)0;
          s = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16), v[4] | ((uint32_t)v[5] << 16),
                         v[6] | ((uint32_t)v[7] << 16));
        }
        *reinterpret_cast<uint4*>(&Xs[so[j]]) = s;
      }
    }
#pragma unroll
    for (int j = 0; j < WI; ++j) {
      const int e = tid + 256 * j;
      if (e < MT * 18)
        *reinterpret_cast<uint4*>(&Ws[e / 18][8 * (e % 18)]) = (okw >> j & 1u) ? wv4[j] : make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    if (c0 + HC < Ci) load(c0 + HC);
#pragma unroll
    for (int kyx = 0; kyx < 9; ++kyx) {
      const int ky = kyx / 3, kx = kyx - 3 * ky;
      bf16x8 a;
      const uint16_t* ap = &Ws[wm * 32 + (lane & 31)][kyx * HC + kg];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = __builtin_bit_cast(__bf16, ap[q]);
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        bf16x8 bb;
        const uint16_t* bp = &Xs[((pr[t] + ky) * TC + pc[t] + kx) * HC + kg];
#pragma unroll
        for (int q = 0; q < 8; ++q) bb[q] = __builtin_bit_cast(__bf16, bp[q]);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[t], 0, 0, 0);
      }
    }
  }
  float bv[16];   // biases loaded together (clamped index), used where co < Co
#pragma unroll
  for (int k = 0; k < 16; ++k) bv[k] = bias[min(co0 + wm * 32 + 8 * (k >> 2) + 4 * (lane >> 5) + (k & 3), Co - 1)];
  if constexpr (!YH) {
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int y = y0 + pr[t], x = x0 + pc[t];
      if (y >= H || x >= W) continue;
      TY* yp = Y + (long long)b * HW + (long long)y * W + x;
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = co0 + wm * 32 + 8 * g + 4 * (lane >> 5) + r;
          if (co < Co) {
            float v = acc[t][4 * g + r] + bv[4 * g + r];
            if (relu) v = fmaxf(v, 0.f);
            yp[(long long)co * Bn * HW] = v;
          }
        }
    }
  } else {
    // BF16 values, two per word: word 2 g + (r >> 1) of block t holds
    // channels co0 + wm 32 + 8 g + 4 (lane >> 5) + r
    uint32_t hv[NTW][8];
#pragma unroll
    for (int t = 0; t < NTW; ++t)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        float v0 = acc[t][2 * k] + bv[2 * k], v1 = acc[t][2 * k + 1] + bv[2 * k + 1];
        if (relu) {
          v0 = fmaxf(v0, 0.f);
          v1 = fmaxf(v1, 0.f);
        }
        hv[t][k] = to_bf16(v0) | ((uint32_t)to_bf16(v1) << 16);
      }
    const long long npix = (long long)Bn * HW;
    const int cw = co0 + wm * 32 + 8 * (lane >> 5);   // first channel of this lane's 8 in block 0
    if constexpr (EP != CONV_OUT) {
      uint4 q[NTW][2];
#pragma unroll
      for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int gg = 0; gg < 2; ++gg)
          q[t][gg] = gather8(hv[t][4 * gg], hv[t][4 * gg + 1], hv[t][4 * gg + 2], hv[t][4 * gg + 3]);
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        const int y = y0 + pr[t], x = x0 + pc[t];
        if (y >= H || x >= W) continue;
        const long long pix = (long long)b * HW + (long long)y * W + x;
#pragma unroll
        for (int gg = 0; gg < 2; ++gg)
          if (cw + 16 * gg < Co) *reinterpret_cast<uint4*>(Y + cblk(cw + 16 * gg, pix, npix)) = q[t][gg];
      }
    }
    if constexpr (EP == CONV_POOL) {
      // window (y, x), (y, x + 1), (y + 1, x), (y + 1, x + 1) at even y, x:
      // this lane's block 0 and 1 values and its neighbour's
      uint32_t pw[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t a = hv[0][k], c = hv[1][k], bn = from_pair_lane(a), dn = from_pair_lane(c);
        pw[k] = max4_bf16((uint16_t)a, (uint16_t)bn, (uint16_t)c, (uint16_t)dn) |
                ((uint32_t)max4_bf16((uint16_t)(a >> 16), (uint16_t)(bn >> 16), (uint16_t)(c >> 16),
                                     (uint16_t)(dn >> 16))
                 << 16);
      }
      uint4 pq[2];
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) pq[gg] = gather8(pw[4 * gg], pw[4 * gg + 1], pw[4 * gg + 2], pw[4 * gg + 3]);
      const int y = y0 + pr[0], x = x0 + pc[0];
      if (!(x & 1) && y < H && x < W) {
        const int h2 = H / 2, w2 = W / 2;
        const long long pix = ((long long)b * h2 + y / 2) * w2 + x / 2, np2 = (long long)Bn * h2 * w2;
#pragma unroll
        for (int gg = 0; gg < 2; ++gg)
          if (cw + 16 * gg < Co) *reinterpret_cast<uint4*>(ep.pool + cblk(cw + 16 * gg, pix, np2)) = pq[gg];
      }
    }
    if constexpr (EP == CONV_OUT) {
      // channels 8 g + r here (lanes 0 .. 31) and 8 g + 4 + r in lane + 32
      float wf[32];
#pragma unroll
      for (int c = 0; c < 32; ++c) wf[c] = Osh[c];
      const float b0 = Osh[32];
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        uint32_t hi[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) hi[k] = from_upper_half(hv[t][k]);
        const int y = y0 + pr[t], x = x0 + pc[t];
        if ((lane >> 5) || y >= H || x >= W) continue;
        float s = 0.f;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            s = fmaf(wf[8 * g + r], from_bf16((uint16_t)(hv[t][2 * g + (r >> 1)] >> (16 * (r & 1)))), s);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            s = fmaf(wf[8 * g + 4 + r], from_bf16((uint16_t)(hi[2 * g + (r >> 1)] >> (16 * (r & 1)))), s);
        }
        const float z = s + b0;
        const long long pix = (long long)b * HW + (long long)y * W + x;
        ep.z[pix] = z;
        ep.prob[pix] = 1.f / (1.f + expf(-z));
      }
    }
  }
}

// 1 x 1 convolution to one output channel plus its bias, one pixel per
// thread (enough workgroups to fill the chip): Y[n] = bias + sum_c W[c]
// X[c][n], both operands rounded to BF16 as in the products, FP32
// accumulation in channel order.
__global__ void k_conv1_out(const uint16_t* __restrict__ Wb, const float* __restrict__ X,
                            const float* __restrict__ bias, float* __restrict__ Y, int C, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float s = 0.f;
#pragma unroll 8
  for (int c = 0; c < C; ++c) s = fmaf(from_bf16(Wb[c]), from_bf16(to_bf16(X[(long long)c * N + i])), s);
  Y[i] = s + bias[0];
}

// Direct 3 x 3 convolution of inputs with at most two channels (the summary
// U-Net's first layer, input S and T) to at most 32 output channels: the
// depth of the product is k = 9 c + 3 ky + kx (the weights' own order),
// 18 values padded to two MFMA steps of 16, instead of one 16-channel chunk
// per (ky, kx) with 14 channels of zeros. A workgroup computes 32 output
// channels x 256 pixels (4 rows x 64 columns when W >= 64); the halo tile
// holds both channels of a position as one BF16 pair. X is planar; a BF16 Y
// is stored in channel blocks of 16, an FP32 Y planar.
constexpr int C2_TX = 6 * 66;   // largest halo tile (positions)
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_conv3_c2(const uint16_t* __restrict__ Wb, const TX* __restrict__ X,
                                                  const float* __restrict__ bias, int relu, TY* __restrict__ Y,
                                                  int Co, int Ci, int Bn, int H, int W, int BC) {
  constexpr int NT = 256;
  __shared__ uint32_t Xs[C2_TX];          // (c0, c1) BF16 pairs
  __shared__ uint16_t Ws[32][32 + 8];
  const int BR = NT / BC, TC = BC + 2, TR = BR + 2, np = TR * TC;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int bx = (W + BC - 1) / BC, by = (H + BR - 1) / BR;
  const int blk = xcd_tile(), b = blk / (bx * by), rem = blk - b * bx * by;
  const int y0 = (rem / bx) * BR, x0 = (rem % bx) * BC;
  const long long HW = (long long)H * W;
  // halo tile: both channels of each position (zero outside the image),
  // and the weights [co][k], k = 9 c + tap (zero past 9 Ci). Every load is
  // issued, from a clamped address, before the first store.
  constexpr int NI = (C2_TX + 255) / 256;
  const long long cstr = Ci > 1 ? (long long)Bn * HW : 0;
  TX v0[NI], v1[NI];
  uint32_t in = 0;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int e = tid + 256 * i, r = e / TC, cc = e - r * TC, y = y0 + r - 1, x = x0 + cc - 1;
    in |= (uint32_t)(e < np && y >= 0 && y < H && x >= 0 && x < W) << i;
    const TX* src = X + (long long)b * HW + (long long)min(max(y, 0), H - 1) * W + min(max(x, 0), W - 1);
    v0[i] = src[0];
    v1[i] = src[cstr];
  }
  uint16_t wl[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 256 * i, co = e >> 5, k = e & 31;
    wl[i] = Wb[(long long)min(co, Co - 1) * 9 * Ci + min(k, 9 * Ci - 1)];
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int e = tid + 256 * i;
    if (e < np) {
      uint16_t h0 = 0, h1 = 0;
      if (in >> i & 1u) {
        h0 = ld_bf16(v0, i);
        h1 = Ci > 1 ? ld_bf16(v1, i) : (uint16_t)0;
      }
      Xs[e] = h0 | ((uint32_t)h1 << 16);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 256 * i, co = e >> 5, k = e & 31;
    Ws[co][k] = (co < Co && k < 9 * Ci) ? wl[i] : (uint16_t)0;
  }
  __syncthreads();
  const int kg = (lane >> 5) * 8;
  f32x16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    bf16x8 a;
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = __builtin_bit_cast(__bf16, Ws[lane & 31][16 * st + kg + q]);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int pl = (wv * 2 + t) * 32 + (lane & 31), pr = pl / BC, pc = pl - pr * BC;
      bf16x8 bb;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = 16 * st + kg + q, c = k / 9, tap = k - 9 * c, ky = tap / 3, kx = tap - 3 * ky;
        uint16_t v = 0;
        if (k < 9 * Ci) {
          const uint32_t pair = Xs[(pr + ky) * TC + pc + kx];
          v = (uint16_t)(c ? pair >> 16 : pair);
        }
        bb[q] = __builtin_bit_cast(__bf16, v);
      }
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[t], 0, 0, 0);
    }
  }
  float v[2][16];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      v[t][k] = acc[t][k] + bias[min(8 * (k >> 2) + 4 * (lane >> 5) + (k & 3), Co - 1)];
      if (relu) v[t][k] = fmaxf(v[t][k], 0.f);
    }
  if constexpr (sizeof(TY) == 2) {
    // channel blocks of 16 (Co a multiple of 16), 16 bytes per lane and store
    uint4 q[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) {
        uint32_t w4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          w4[k] = to_bf16(v[t][8 * gg + 2 * k]) | ((uint32_t)to_bf16(v[t][8 * gg + 2 * k + 1]) << 16);
        q[t][gg] = gather8(w4[0], w4[1], w4[2], w4[3]);
      }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int pl = (wv * 2 + t) * 32 + (lane & 31), pr = pl / BC, pc = pl - pr * BC;
      const int y = y0 + pr, x = x0 + pc;
      if (y >= H || x >= W) continue;
      const long long pix = (long long)b * HW + (long long)y * W + x;
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) {
        const int c = 16 * gg + 8 * (lane >> 5);
        if (c < Co) *reinterpret_cast<uint4*>(Y + cblk(c, pix, (long long)Bn * HW)) = q[t][gg];
      }
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int pl = (wv * 2 + t) * 32 + (lane & 31), pr = pl / BC, pc = pl - pr * BC;
    const int y = y0 + pr, x = x0 + pc;
    if (y >= H || x >= W) continue;
    const long long pix = (long long)b * HW + (long long)y * W + x;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int co = 8 * g + 4 * (lane >> 5);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (co + r < Co) Y[pix + (long long)(co + r) * Bn * HW] = v[t][4 * g + r];
    }
  }
}

// Transposed 2 x 2 convolution, stride 2, on BF16 activations in channel
// blocks of 16: Y[co][b][2 y + a][2 x + e] = bias[co] + sum_c
// W[4 co + 2 a + e][c] X[c][b][y][x], rounded to BF16. Two waves share a
// block of 32 input pixels, each computing half of the 4 Co rows of the
// product, so X is read from memory once and each output pixel written once:
// row tile i (32 rows) is tap a 2 + e = i / (Co / 32), output channels
// 32 (i % (Co / 32)) .. + 31, from the weights permuted into that order in
// LDS. The MFMA B operand, 8 channels of one pixel, is one 16-byte load of
// the blocked input. The depth steps run in channel order, as in k_gemm_v's
// GV_UP product, so the sums are the same.
template <int MI, int KS>   // MI = 4 Co / 32 row tiles, KS = Ci / 16 depth steps
__global__ __launch_bounds__(256) void k_up2_h(const uint16_t* __restrict__ Wb, const uint16_t* __restrict__ X,
                                               const float* __restrict__ bias, uint16_t* __restrict__ Y, int Bn,
                                               int h, int w) {
  constexpr int M = 32 * MI, K = 16 * KS, Co = M / 4, TPC = Co / 32, MH = MI / 2;   // row tiles per tap, per wave
  static_assert(Co % 32 == 0 && MI % 2 == 0, "whole 32-channel tiles per tap, split over two waves");
  __shared__ __attribute__((aligned(16))) uint16_t Ws[M][K + 8];
  __shared__ float Bs[Co];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, i0 = (wv & 1) * MH;
  // weights and biases: every load issued before the first store
  constexpr int NWL = M * (K / 8) / 256;
  static_assert(M * (K / 8) % 256 == 0 && Co <= 256, "whole staging rounds");
  uint4 wl[NWL];
#pragma unroll
  for (int j = 0; j < NWL; ++j) {
    const int e = tid + 256 * j, m = e / (K / 8), q = e - m * (K / 8), tap = m / Co, co = m - tap * Co;
    wl[j] = *reinterpret_cast<const uint4*>(Wb + (long long)(4 * co + tap) * K + 8 * q);
  }
  const float bl = bias[min(tid, Co - 1)];
#pragma unroll
  for (int j = 0; j < NWL; ++j) {
    const int e = tid + 256 * j, m = e / (K / 8), q = e - m * (K / 8);
    *reinterpret_cast<uint4*>(&Ws[m][8 * q]) = wl[j];
  }
  if (tid < Co) Bs[tid] = bl;
  __syncthreads();
  const long long hw = (long long)h * w, npix = (long long)Bn * hw;
  const long long nblk = (npix + 31) / 32;
  for (long long blk = (long long)blockIdx.x * 2 + (wv >> 1); blk < nblk; blk += (long long)gridDim.x * 2) {
    // the weight reads below are the same for every block: kept inside the
    // loop (not hoisted into registers for all blocks)
    asm volatile("" ::: "memory");
    const long long p = blk * 32 + (lane & 31), pl = p < npix ? p : npix - 1;
    uint4 bq[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
      bq[s] = *reinterpret_cast<const uint4*>(X + ((long long)s * npix + pl) * 16 + 8 * (lane >> 5));
    f32x16 acc[MH];
#pragma unroll
    for (int i = 0; i < MH; ++i)
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[i][k] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bf16x8 bb = __builtin_bit_cast(bf16x8, bq[s]);
#pragma unroll
      for (int i = 0; i < MH; ++i) {
        const bf16x8 a = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const uint4*>(&Ws[32 * (i0 + i) + (lane & 31)][16 * s + 8 * (lane >> 5)]));
        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[i], 0, 0, 0);
      }
    }
    const long long b = pl / hw;
    const int yx = (int)(pl - b * hw), y = yx / w, x = yx - y * w;
#pragma unroll
    for (int i = 0; i < MH; ++i) {
      const int tap = (i0 + i) / TPC, a = tap >> 1, e = tap & 1;
      const long long op = (b * 2 * h + 2 * y + a) * (2LL * w) + 2 * x + e;   // output pixel
      const int cb = 32 * ((i0 + i) % TPC);
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) {
        uint32_t w4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int c = cb + 8 * (2 * gg + (k >> 1)) + 4 * (lane >> 5) + 2 * (k & 1);   // channels c, c + 1
          w4[k] = to_bf16(acc[i][8 * gg + 2 * k] + Bs[c]) |
                  ((uint32_t)to_bf16(acc[i][8 * gg + 2 * k + 1] + Bs[c + 1]) << 16);
        }
        const uint4 q = gather8(w4[0], w4[1], w4[2], w4[3]);
        if (p < npix) *reinterpret_cast<uint4*>(Y + cblk(cb + 16 * gg + 8 * (lane >> 5), op, 4 * npix)) = q;
      }
    }
  }
}

// The U-Net's first two convolutions in one kernel (inference, 64-column
// tiles): e1a (2 -> 32 channels, k_conv3_c2's product: depth 9 c + tap in
// two MFMA steps) is computed on the halo tile of e1b (32 -> 32, with 2 x 2
// pooling) straight into LDS, so its activations never go to HBM. A
// workgroup stages the FP32 input (S and T, planar) on an 8 x 68 tile as
// BF16 pairs, computes e1a on the 6 x 66 halo positions of its 4 x 64 output
// block (13 blocks of 32 positions over the four waves; zero outside the
// image, e1b's padding), then runs e1b over both 16-channel halves of that
// tile as k_conv3_halo does (same weights copy, same order of the sums),
// with the CONV_POOL epilogue. Every value equals the two-kernel path's.
constexpr int E1_TR = 8, E1_TC = 68;              // input tile
constexpr int E1_HR = 6, E1_HC = 66, E1_NP = E1_HR * E1_HC;   // e1b halo positions
// e1a on the halo tile: 32 channels (64 bytes) per position, the four
// 16-byte groups of position p rotated by p / 4, so that 16 lanes reading the
// same group of 16 consecutive positions hit all 64 banks once
__device__ __forceinline__ int e1_at(int p, int grp) { return p * 32 + 8 * ((grp + (p >> 2)) & 3); }
__global__ __launch_bounds__(256) void k_conv3_first2(const uint16_t* __restrict__ W1, const float* __restrict__ b1,
                                                      const float* __restrict__ X, const uint16_t* __restrict__ W2r,
                                                      const float* __restrict__ b2, uint16_t* __restrict__ Y,
                                                      uint16_t* __restrict__ Yp, int Bn, int H, int W) {
  __shared__ uint32_t Xs2[E1_TR * E1_TC];                                   // (S, T) BF16 pairs
  __shared__ __attribute__((aligned(16))) uint16_t Ws1[32][32 + 8];        // e1a weights [co][k]
  __shared__ __attribute__((aligned(16))) uint16_t XsE[E1_NP * 32];        // e1a on the halo tile (e1_at)
  __shared__ __attribute__((aligned(16))) uint16_t Ws2[2][32][9 * HC + 8];  // e1b weights, both chunks
  __shared__ float Bs[64];                                                  // biases of e1a, e1b
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, h = lane >> 5;
  const int bx = W / 64, by = H / 4;
  const int blk = xcd_tile(), b = blk / (bx * by), rem = blk - b * bx * by;
  const int y0 = (rem / bx) * 4, x0 = (rem % bx) * 64;
  const long long HW = (long long)H * W, cs = (long long)Bn * HW;
  // every load first (clamped addresses, masked when stored)
  float v0[3], v1[3];
  uint32_t in = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = tid + 256 * j, r = e / E1_TC, cc = e - r * E1_TC, y = y0 + r - 2, x = x0 + cc - 2;
    in |= (uint32_t)(e < E1_TR * E1_TC && y >= 0 && y < H && x >= 0 && x < W) << j;
    const float* src = X + (long long)b * HW + (long long)min(max(y, 0), H - 1) * W + min(max(x, 0), W - 1);
    v0[j] = src[0];
    v1[j] = src[cs];
  }
  uint16_t w1[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = tid + 256 * j, co = min(e / 18, 31), k = e - (e / 18) * 18;
    w1[j] = W1[co * 18 + k];
  }
  uint4 w2[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) w2[j] = *reinterpret_cast<const uint4*>(W2r + 8 * min(tid + 256 * j, 2 * 32 * 18 - 1));
  const float bl = tid < 32 ? b1[tid] : tid < 64 ? b2[tid - 32] : 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = tid + 256 * j;
    if (e < E1_TR * E1_TC)
      Xs2[e] = (in >> j & 1u) ? to_bf16(v0[j]) | ((uint32_t)to_bf16(v1[j]) << 16) : 0u;
  }
  for (int e = tid; e < 32 * 32; e += 256) Ws1[e >> 5][e & 31] = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = tid + 256 * j;
    if (e < 32 * 18) Ws1[e / 18][e - (e / 18) * 18] = w1[j];
  }
  // 16-byte group e: chunk e / 576, co (e / 18) % 32, group e % 18
  auto put_w2 = [&](int e, uint4 v) {
    if (e < 2 * 32 * 18) *reinterpret_cast<uint4*>(&Ws2[e / 576][(e / 18) % 32][8 * (e % 18)]) = v;
  };
  put_w2(tid, w2[0]);
  put_w2(tid + 256, w2[1]);
  put_w2(tid + 512, w2[2]);
  put_w2(tid + 768, w2[3]);
  put_w2(tid + 1024, w2[4]);
  if (tid < 64) Bs[tid] = bl;
  __syncthreads();
  const int kg = h * 8;
  // e1a on the halo positions
  bf16x8 a1[2];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int q = 0; q < 8; ++q) a1[st][q] = __builtin_bit_cast(__bf16, Ws1[lane & 31][16 * st + kg + q]);
  float be[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) be[k] = Bs[8 * (k >> 2) + 4 * h + (k & 3)];
  for (int blk32 = wv; blk32 * 32 < E1_NP; blk32 += 4) {
    const int p = blk32 * 32 + (lane & 31), pq = min(p, E1_NP - 1), r = pq / E1_HC, cc = pq - r * E1_HC;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      bf16x8 bb;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = 16 * st + kg + q, c = k / 9, tap = k - 9 * c, ky = tap / 3, kx = tap - 3 * ky;
        uint16_t v = 0;
        if (k < 18) {
          const uint32_t pair = Xs2[(r + ky) * E1_TC + cc + kx];
          v = (uint16_t)(c ? pair >> 16 : pair);
        }
        bb[q] = __builtin_bit_cast(__bf16, v);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[st], bb, acc, 0, 0, 0);
    }
    const int y = y0 + r - 1, x = x0 + cc - 1;
    const bool inside = y >= 0 && y < H && x >= 0 && x < W;
    uint4 qv[2];
#pragma unroll
    for (int gg = 0; gg < 2; ++gg) {
      uint32_t w4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i0 = 8 * gg + 2 * k;
        const uint16_t lo = inside ? to_bf16(fmaxf(acc[i0] + be[i0], 0.f)) : (uint16_t)0;
        const uint16_t hi = inside ? to_bf16(fmaxf(acc[i0 + 1] + be[i0 + 1], 0.f)) : (uint16_t)0;
        w4[k] = lo | ((uint32_t)hi << 16);
      }
      qv[gg] = gather8(w4[0], w4[1], w4[2], w4[3]);
    }
    if (p < E1_NP) {
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) *reinterpret_cast<uint4*>(&XsE[e1_at(p, 2 * gg + h)]) = qv[gg];
    }
  }
  __syncthreads();
  // e1b: wave wv owns rows 2 (wv / 2) + t of column block wv % 2
  int pr[2], pc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    pr[t] = 2 * (wv >> 1) + t;
    pc[t] = (wv & 1) * 32 + (lane & 31);
  }
  f32x16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
#pragma unroll
  for (int ch = 0; ch < 2; ++ch)
#pragma unroll
    for (int kyx = 0; kyx < 9; ++kyx) {
      const int ky = kyx / 3, kx = kyx - 3 * ky;
      bf16x8 a;
      const uint16_t* ap = &Ws2[ch][lane & 31][kyx * HC + kg];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = __builtin_bit_cast(__bf16, ap[q]);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        bf16x8 bb;
        const uint16_t* bp = &XsE[e1_at((pr[t] + ky) * E1_HC + pc[t] + kx, 2 * ch + h)];
#pragma unroll
        for (int q = 0; q < 8; ++q) bb[q] = __builtin_bit_cast(__bf16, bp[q]);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[t], 0, 0, 0);
      }
    }
  // epilogue: e1b's bias and ReLU, BF16 activations and their 2 x 2 pooling
  uint32_t hv[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i0 = 2 * k, i1 = 2 * k + 1;
      const float f0 = fmaxf(acc[t][i0] + Bs[32 + 8 * (i0 >> 2) + 4 * h + (i0 & 3)], 0.f);
      const float f1 = fmaxf(acc[t][i1] + Bs[32 + 8 * (i1 >> 2) + 4 * h + (i1 & 3)], 0.f);
      hv[t][k] = to_bf16(f0) | ((uint32_t)to_bf16(f1) << 16);
    }
  const long long npix = (long long)Bn * HW;
  const int cw = 8 * h;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const long long pix = (long long)b * HW + (long long)(y0 + pr[t]) * W + x0 + pc[t];
#pragma unroll
    for (int gg = 0; gg < 2; ++gg)
      *reinterpret_cast<uint4*>(Y + cblk(cw + 16 * gg, pix, npix)) =
          gather8(hv[t][4 * gg], hv[t][4 * gg + 1], hv[t][4 * gg + 2], hv[t][4 * gg + 3]);
  }
  uint32_t pw[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t a = hv[0][k], c = hv[1][k], bn = from_pair_lane(a), dn = from_pair_lane(c);
    pw[k] = max4_bf16((uint16_t)a, (uint16_t)bn, (uint16_t)c, (uint16_t)dn) |
            ((uint32_t)max4_bf16((uint16_t)(a >> 16), (uint16_t)(bn >> 16), (uint16_t)(c >> 16), (uint16_t)(dn >> 16))
             << 16);
  }
  uint4 pq[2];
#pragma unroll
  for (int gg = 0; gg < 2; ++gg) pq[gg] = gather8(pw[4 * gg], pw[4 * gg + 1], pw[4 * gg + 2], pw[4 * gg + 3]);
  if (!(pc[0] & 1)) {
    const int h2 = H / 2, w2 = W / 2;
    const long long pix = ((long long)b * h2 + (y0 + pr[0]) / 2) * w2 + (x0 + pc[0]) / 2, np2 = (long long)Bn * h2 * w2;
#pragma unroll
    for (int gg = 0; gg < 2; ++gg) *reinterpret_cast<uint4*>(Yp + cblk(cw + 16 * gg, pix, np2)) = pq[gg];
  }
}

// sum the split-K partials in order: C[m][n] (+)= sum_z P[z][m][n]
__global__ void k_splitk_reduce(const float* __restrict__ P, float* __restrict__ C, long long MN, int Z,
                                int accumulate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float s = 0.f;
  for (int z = 0; z < Z; ++z) s += P[(long long)z * MN + i];
  C[i] = accumulate ? C[i] + s : s;
}

// ------------------------------------------------------- 3x3 convolutions
// col[(c*9 + ky*3 + kx)][b*HW + y*W + x] = X[c][b][y + ky - 1][x + kx - 1]
__global__ void k_im2col3(const float* __restrict__ X, uint16_t* __restrict__ col, int C, int Bn, int H, int W) {
  const long long N = (long long)Bn * H * W;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * C * 9) return;
  const long long p = i % N;
  const int r = (int)(i / N);
  const int c = r / 9, kk = r % 9, ky = kk / 3, kx = kk % 3;
  const int b = (int)(p / (H * W)), yx = (int)(p % (H * W)), y = yx / W, x = yx % W;
  const int yy = y + ky - 1, xx = x + kx - 1;
  const float v = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? X[((long long)c * Bn + b) * H * W + yy * W + xx] : 0.f;
  col[i] = to_bf16(v);
}

// The same, 8 consecutive pixels of one row per thread and one 16-byte
// store (W a multiple of 8).
__global__ void k_im2col3_v(const float* __restrict__ X, uint16_t* __restrict__ col, int C, int Bn, int H, int W) {
  const long long N = (long long)Bn * H * W, N8 = N / 8;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N8 * C * 9) return;
  const long long p = (i % N8) * 8;
  const int r = (int)(i / N8);
  const int c = r / 9, kk = r % 9, ky = kk / 3, kx = kk % 3;
  const int b = (int)(p / (H * W)), yx = (int)(p % (H * W)), y = yx / W, x0 = yx % W;
  const int yy = y + ky - 1;
  uint16_t v[8];
  const bool row_in = yy >= 0 && yy < H;
  const float* src = X + ((long long)c * Bn + b) * H * W + (long long)yy * W;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int xx = x0 + j + kx - 1;
    v[j] = to_bf16(row_in && xx >= 0 && xx < W ? src[xx] : 0.f);
  }
  uint4 pk;
  pk.x = v[0] | ((uint32_t)v[1] << 16);
  pk.y = v[2] | ((uint32_t)v[3] << 16);
  pk.z = v[4] | ((uint32_t)v[5] << 16);
  pk.w = v[6] | ((uint32_t)v[7] << 16);
  *reinterpret_cast<uint4*>(col + (long long)r * N + p) = pk;
}

// dX[c][b][y][x] (+)= sum_{ky,kx} dcol[c*9 + ky*3 + kx][b, y - ky + 1, x - kx + 1]
__global__ void k_col2im3(const float* __restrict__ dcol, float* __restrict__ dX, int C, int Bn, int H, int W,
                          int accumulate) {
  const long long N = (long long)Bn * H * W;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * C) return;
  const int c = (int)(i / N);
  const long long p = i % N;
  const int b = (int)(p / (H * W)), yx = (int)(p % (H * W)), y = yx / W, x = yx % W;
  float s = 0.f;
  for (int ky = 0; ky < 3; ++ky)
    for (int kx = 0; kx < 3; ++kx) {
      const int yy = y - ky + 1, xx = x - kx + 1;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        s += dcol[(long long)(c * 9 + ky * 3 + kx) * N + (long long)b * H * W + yy * W + xx];
    }
  dX[i] = accumulate ? dX[i] + s : s;
}

// -------------------------------------------------- temporal convolutions
// input normalisation per segment and pixel: (V - mean) / sqrt(mean + 25);
// out layout [t][b][p] (one channel), frames [b][t][p] with p over H*W
__global__ void k_tnorm(const uint16_t* __restrict__ frames, float* __restrict__ out, int Bn, int L, long long HW) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)Bn * HW) return;
  const int b = (int)(i / HW);
  const long long p = i % HW;
  const uint16_t* f = frames + (long long)b * L * HW + p;
  float s = 0.f;
  for (int t = 0; t < L; ++t) s += (float)f[(long long)t * HW];
  const float mean = s / L;
  const float inv = rsqrtf(mean + 25.f);
  for (int t = 0; t < L; ++t) out[((long long)t * Bn + b) * HW + p] = ((float)f[(long long)t * HW] - mean) * inv;
}

// The frame normalisation and the first temporal convolution (one input
// channel, 32 outputs, kernel 5, stride 5, no padding: 50 -> 10 samples) in
// one pass, for inference. A wave takes 64 pixels. Each lane loads its
// pixel's 50 frames and normalises them as k_tnorm does (sequential FP32 sum,
// mean, 1 / sqrt(mean + 25)), rounding to BF16 as im2col1 does; for output
// sample j the 5 values are the depth of one 32 x 32 x 16 MFMA, lanes
// 32..63 handing their pixels to lanes 0..31 for a second one, each followed
// by the all-zero step that the product kernels run for the rest of their
// 32-deep chunk, so the sums are those of im2col1 + gemm. Bias, ReLU and BF16
// rounding as bias_act and the BF16 store; a1 [32][10][Np] (row c, column
// j Np + n) is written through a per-wave LDS tile, 16 bytes per lane.
constexpr int T1_L = 50, T1_K = 5, T1_TO = 10;
__global__ __launch_bounds__(256) void k_tconv1_h(const uint16_t* __restrict__ frames, const uint16_t* __restrict__ Wb,
                                                  const float* __restrict__ bias, uint16_t* __restrict__ a1, int Bn,
                                                  long long HW) {
  __shared__ __attribute__((aligned(16))) uint16_t Ts[4][32][64 + 8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, h = lane >> 5;
  const long long Np = (long long)Bn * HW;
  const long long p0 = ((long long)blockIdx.x * 4 + wv) * 64;   // the wave's first pixel (Np % 64 == 0)
  if (p0 >= Np) return;   // whole waves; no workgroup barrier below
  const long long n = p0 + lane;
  const long long b = n / HW, p = n - b * HW;
  const uint16_t* f = frames + b * T1_L * HW + p;
  float v[T1_L];
#pragma unroll
  for (int t = 0; t < T1_L; ++t) v[t] = (float)f[(long long)t * HW];
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < T1_L; ++t) s += v[t];
  const float mean = s / T1_L;
  const float inv = rsqrtf(mean + 25.f);
  // weights: row lane & 31, depth 0..4 in lanes 0..31, zero elsewhere
  bf16x8 a, z;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = __builtin_bit_cast(__bf16, (h == 0 && q < T1_K) ? Wb[(lane & 31) * T1_K + q] : (uint16_t)0);
    z[q] = __builtin_bit_cast(__bf16, (uint16_t)0);
  }
  float bv[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) bv[k] = bias[8 * (k >> 2) + 4 * h + (k & 3)];
#pragma unroll
  for (int j = 0; j < T1_TO; ++j) {
    uint32_t w[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint16_t lo = to_bf16((v[5 * j + 2 * q] - mean) * inv);
      const uint16_t hi = 2 * q + 1 < T1_K ? to_bf16((v[5 * j + 2 * q + 1] - mean) * inv) : (uint16_t)0;
      w[q] = lo | ((uint32_t)hi << 16);
    }
    uint32_t u[3];   // lanes 0..31: the words of lane + 32 (pixels 32..63)
#pragma unroll
    for (int q = 0; q < 3; ++q) u[q] = from_upper_half(w[q]);
    f32x16 acc[2];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const uint32_t* src = blk ? u : w;
      const uint4 bq = h == 0 ? make_uint4(src[0], src[1], src[2], 0) : make_uint4(0, 0, 0, 0);
      f32x16 c;
#pragma unroll
      for (int i = 0; i < 16; ++i) c[i] = 0.f;
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, bq), c, 0, 0, 0);
      acc[blk] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(z, z, c, 0, 0, 0);
    }
    // tile [32 channels][64 pixels] of sample j, then 16-byte row pieces
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const float y = fmaxf(acc[blk][k] + bv[k], 0.f);
        Ts[wv][8 * (k >> 2) + 4 * h + (k & 3)][32 * blk + (lane & 31)] = to_bf16(y);
      }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = lane + 64 * i, row = e >> 3, c8 = (e & 7) * 8;
      *reinterpret_cast<uint4*>(a1 + (long long)row * T1_TO * Np + (long long)j * Np + p0 + c8) =
          *reinterpret_cast<const uint4*>(&Ts[wv][row][c8]);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  }
}

// 1-D im2col: in [C][Tin][N], kernel KT, stride S, pad P ->
// col[(c*KT + k)][(j*N + n)] = in[c][j*S + k - P][n], j < Tout
__global__ void k_im2col1(const float* __restrict__ in, uint16_t* __restrict__ col, int C, int Tin, int Tout,
                          int KT, int S, int P, long long N) {
  const long long total = (long long)C * KT * Tout * N;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long cols = (long long)Tout * N;
  const int r = (int)(i / cols);
  const long long q = i % cols;
  const int c = r / KT, k = r % KT;
  const int j = (int)(q / N);
  const long long n = q % N;
  const int t = j * S + k - P;
  col[i] = to_bf16((t >= 0 && t < Tin) ? in[((long long)c * Tin + t) * N + n] : 0.f);
}

// 1-D col2im: d_in[c][t][n] = sum over (j, k) with j*S + k - P = t of dcol[c*KT + k][j*N + n]
__global__ void k_col2im1(const float* __restrict__ dcol, float* __restrict__ din, int C, int Tin, int Tout,
                          int KT, int S, int P, long long N) {
  const long long total = (long long)C * Tin * N;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i / ((long long)Tin * N));
  const long long q = i % ((long long)Tin * N);
  const int t = (int)(q / N);
  const long long n = q % N;
  float s = 0.f;
  for (int k = 0; k < KT; ++k) {
    const int jt = t + P - k;
    if (jt < 0 || jt % S) continue;
    const int j = jt / S;
    if (j >= Tout) continue;
    s += dcol[(long long)(c * KT + k) * Tout * N + (long long)j * N + n];
  }
  din[i] = s;
}

// ------------------------------------------------------------ elementwise
__global__ void k_bias_act(float* __restrict__ Y, const float* __restrict__ bias, int C, long long N, int relu) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)C * N) return;
  float v = Y[i] + bias[i / N];
  Y[i] = relu ? fmaxf(v, 0.f) : v;
}

// dY *= [Y > 0] (ReLU backward through the stored output)
__global__ void k_relu_bwd(float* __restrict__ dY, const float* __restrict__ Y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(Y[i] > 0.f)) dY[i] = 0.f;
}

// db[c] (+)= sum_n dY[c][n], one block per channel, fixed order
__global__ void k_bias_grad(const float* __restrict__ dY, float* __restrict__ db, long long N, int accumulate) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (long long n = threadIdx.x; n < N; n += 256) s += dY[(long long)c * N + n];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = accumulate ? db[c] + sh[0] : sh[0];
}

// 2x2 max pool (H, W even): Y[c][b][i][j] = max over the 2x2 block; arg = 0..3
__global__ void k_pool(const float* __restrict__ X, float* __restrict__ Y, uint8_t* __restrict__ arg, int CB,
                       int H, int W) {
  const int h = H / 2, w = W / 2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)CB * h * w) return;
  const long long cb = i / (h * w);
  const int yx = (int)(i % (h * w)), y = yx / w, x = yx % w;
  const float* s = X + cb * H * W + (2 * y) * W + 2 * x;
  float best = s[0];
  int a = 0;
  if (s[1] > best) { best = s[1]; a = 1; }
  if (s[W] > best) { best = s[W]; a = 2; }
  if (s[W + 1] > best) { best = s[W + 1]; a = 3; }
  Y[i] = best;
  arg[i] = (uint8_t)a;
}

// dX (+)= dY routed to the argmax position
__global__ void k_pool_bwd(const float* __restrict__ dY, const uint8_t* __restrict__ arg, float* __restrict__ dX,
                           int CB, int H, int W, int accumulate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)CB * H * W) return;
  const long long cb = i / (H * W);
  const int yx = (int)(i % (H * W)), y = yx / W, x = yx % W;
  const int h = H / 2, w = W / 2;
  const long long o = cb * h * w + (y / 2) * w + (x / 2);
  const int a = (y & 1) * 2 + (x & 1);
  const float v = arg[o] == a ? dY[o] : 0.f;
  dX[i] = accumulate ? dX[i] + v : v;
}

// transposed 2x2 stride-2 convolution, scatter of Z[(co*4 + a*2 + b)][n*hw + i*w + j]
// to Y[co][n][2i + a][2j + b] plus bias
__global__ void k_up_scatter(const float* __restrict__ Z, const float* __restrict__ bias, float* __restrict__ Y,
                             int Co, int Bn, int h, int w) {
  const int H = 2 * h, W = 2 * w;
  const long long tot = (long long)Co * Bn * H * W;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const int co = (int)(i / ((long long)Bn * H * W));
  const long long q = i % ((long long)Bn * H * W);
  const int n = (int)(q / (H * W)), yx = (int)(q % (H * W)), y = yx / W, x = yx % W;
  const int a = y & 1, bb = x & 1;
  Y[i] = Z[(long long)(co * 4 + a * 2 + bb) * Bn * h * w + (long long)n * h * w + (y / 2) * w + x / 2] + bias[co];
}

// backward of the scatter: dZ[(co*4 + a*2 + b)][n*hw + i*w + j] = dY[co][n][2i + a][2j + b]
__global__ void k_up_gather(const float* __restrict__ dY, float* __restrict__ dZ, int Co, int Bn, int h, int w) {
  const long long tot = (long long)Co * 4 * Bn * h * w;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const long long hw = (long long)h * w;
  const int r = (int)(i / (Bn * hw));
  const long long q = i % (Bn * hw);
  const int co = r / 4, a = (r % 4) / 2, bb = r % 2;
  const int n = (int)(q / hw), ij = (int)(q % hw), y = ij / w, x = ij % w;
  dZ[i] = dY[(long long)co * Bn * 4 * hw + (long long)n * 4 * hw + (2 * y + a) * (2 * w) + 2 * x + bb];
}

// sigmoid + binary cross-entropy on logits z with targets y:
// loss_i = max(z, 0) - z y + log(1 + exp(-|z|)); dz = (sigmoid(z) - y) / n;
// prob = sigmoid(z); per-block loss partials (summed in order on the host)
__global__ void k_bce(const float* __restrict__ z, const float* __restrict__ y, float* __restrict__ dz,
                      float* __restrict__ prob, float* __restrict__ part, long long n) {
  __shared__ float sh[256];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < n) {
    const float zi = z[i];
    const float p = 1.f / (1.f + expf(-zi));
    if (prob) prob[i] = p;
    if (y) {
      const float yi = y[i];
      l = fmaxf(zi, 0.f) - zi * yi + log1pf(expf(-fabsf(zi)));
      if (dz) dz[i] = (p - yi) / (float)n;
    }
  }
  if (!part) return;
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// RMSProp on FP32 master weights, then refresh the BF16 copy
__global__ void k_rmsprop(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ v,
                          uint16_t* __restrict__ wb, long long n, float lr, float rho, float eps) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float vi = rho * v[i] + (1.f - rho) * gi * gi;
  v[i] = vi;
  const float wi = w[i] - lr * gi / (sqrtf(vi) + eps);
  w[i] = wi;
  wb[i] = to_bf16(wi);
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = to_bf16(w[i]);
}

// ---- summary-image input (S, T) -------------------------------------------

// One 1024-thread block per patch (the FP64 divisions and square roots of
// the pixels are the work): exact-enough FP64 mean and population deviation
// of S, then channel 0 = (S - mean) / max(sd, 1e-3), channel 1 = T / sqrt(S + 25).
constexpr int NORM_NT = 1024;
__global__ __launch_bounds__(NORM_NT) void k_st_norm(const float* __restrict__ stin, float* __restrict__ x, int Bn,
                                                     long long HW) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const float* S = stin + (size_t)b * 2 * HW;
  const float* T = S + HW;
  double s = 0.0, s2 = 0.0;
  for (long long i = tid; i < HW; i += NORM_NT) {
    const double v = S[i];
    s += v;
    s2 += v * v;
  }
  __shared__ double r1[NORM_NT], r2[NORM_NT];
  r1[tid] = s;
  r2[tid] = s2;
  __syncthreads();
  for (int o = NORM_NT / 2; o > 0; o >>= 1) {
    if (tid < o) {
      r1[tid] += r1[tid + o];
      r2[tid] += r2[tid + o];
    }
    __syncthreads();
  }
  const double m = r1[0] / (double)HW;
  const double sd = fmax(sqrt(fmax(r2[0] / (double)HW - m * m, 0.0)), 1e-3);
  for (long long i = tid; i < HW; i += NORM_NT) {
    x[(size_t)b * HW + i] = (float)(((double)S[i] - m) / sd);
    x[((size_t)Bn + b) * HW + i] = (float)((double)T[i] / sqrt(fmax((double)S[i], 0.0) + 25.0));
  }
}

__device__ __forceinline__ int st_count(int n) { return (n - 64 + 31) / 32 + 1; }
__device__ __forceinline__ int st_origin(int k, int n) { return min(32 * k, n - 64); }

// out [n_patch][2][64][64], patches in raster order of their origins
// grid y: segment (S, T planes H W apart; patches np 2 4096 apart)
__global__ void k_st_patches(const float* __restrict__ S, const float* __restrict__ T, int H, int W,
                             float* __restrict__ out) {
  const int nx = st_count(W);
  const long long total = (long long)st_count(H) * nx * 2 * 4096;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  S += (long long)blockIdx.y * H * W;
  T += (long long)blockIdx.y * H * W;
  out += (long long)blockIdx.y * total;
  const int k = (int)(i / 8192), r = (int)(i % 8192), c = r / 4096, y = (r % 4096) / 64, x = r % 64;
  const int oy = st_origin(k / nx, H), ox = st_origin(k % nx, W);
  out[i] = (c ? T : S)[(size_t)(oy + y) * W + ox + x];
}

// out(y, x) = sum_k w w prob_k / sum_k w w over the patches that hold the pixel
// grid y: segment (probabilities np 4096 apart, maps H W apart)
__global__ void k_st_merge(const float* __restrict__ prob, int H, int W, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)H * W) return;
  const int y = (int)(i / W), x = (int)(i % W);
  const int ny = st_count(H), nx = st_count(W);
  prob += (long long)blockIdx.y * ny * nx * 4096;
  out += (long long)blockIdx.y * H * W;
  double num = 0.0, den = 0.0;
  for (int ky = 0; ky < ny; ++ky) {
    const int oy = st_origin(ky, H);
    if (y < oy || y >= oy + 64) continue;
    const double wy = 1.0 - fabs((double)(y - oy) - 31.5) / 32.0;
    for (int kx = 0; kx < nx; ++kx) {
      const int ox = st_origin(kx, W);
      if (x < ox || x >= ox + 64) continue;
      const double w = wy * (1.0 - fabs((double)(x - ox) - 31.5) / 32.0);
      num += w * (double)prob[(size_t)(ky * nx + kx) * 4096 + (y - oy) * 64 + (x - ox)];
      den += w;
    }
  }
  out[i] = (float)(num / den);
}

inline dim3 grid1(long long n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t gemm(const GemmOp& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int splits = g.splits < 1 ? 1 : g.splits;
  int kchunk = (g.K + splits - 1) / splits;
  kchunk = (kchunk + GK - 1) / GK * GK;
  const int z = (g.K + kchunk - 1) / kchunk;
  dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, z > 0 ? z : 1);
  float* out = z > 1 ? g.scratch : g.C;
  const int acc = z > 1 ? 0 : g.accumulate;
  const bool vec = z == 1 && g.a_bf16 && g.b_bf16 && g.sak == 1 && g.sbn == 1 && g.K % 8 == 0 && g.sam % 8 == 0 &&
                   g.sbk % 8 == 0 && g.N % 8 == 0 && ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0;
  if (vec) {
    const Im2col none{nullptr, 0, 0, 0};
    if (g.M <= 32)
      hipLaunchKernelGGL((k_gemm_v<32, GV_BF16>), dim3((g.N + 127) / 128, (g.M + 31) / 32), dim3(256), 0, st,
                         (const uint16_t*)g.A, g.sam, (const uint16_t*)g.B, g.sbk, none, out, (long long)g.N, g.M,
                         g.N, g.K, acc, nullptr, 0);
    else
      hipLaunchKernelGGL((k_gemm_v<64, GV_BF16>), dim3((g.N + 63) / 64, (g.M + 63) / 64), dim3(256), 0, st,
                         (const uint16_t*)g.A, g.sam, (const uint16_t*)g.B, g.sbk, none, out, (long long)g.N, g.M,
                         g.N, g.K, acc, nullptr, 0);
  } else if (g.a_bf16 && g.b_bf16)
    hipLaunchKernelGGL((k_gemm<uint16_t, uint16_t>), grid, dim3(256), 0, st, (const uint16_t*)g.A, g.sam, g.sak,
                       (const uint16_t*)g.B, g.sbk, g.sbn, out, (long long)g.N, g.M, g.N, g.K, kchunk, acc);
  else if (g.a_bf16)
    hipLaunchKernelGGL((k_gemm<uint16_t, float>), grid, dim3(256), 0, st, (const uint16_t*)g.A, g.sam, g.sak,
                       (const float*)g.B, g.sbk, g.sbn, out, (long long)g.N, g.M, g.N, g.K, kchunk, acc);
  else if (g.b_bf16)
    hipLaunchKernelGGL((k_gemm<float, uint16_t>), grid, dim3(256), 0, st, (const float*)g.A, g.sam, g.sak,
                       (const uint16_t*)g.B, g.sbk, g.sbn, out, (long long)g.N, g.M, g.N, g.K, kchunk, acc);
  else
    hipLaunchKernelGGL((k_gemm<float, float>), grid, dim3(256), 0, st, (const float*)g.A, g.sam, g.sak,
                       (const float*)g.B, g.sbk, g.sbn, out, (long long)g.N, g.M, g.N, g.K, kchunk, acc);
  if (z > 1) {
    const long long MN = (long long)g.M * g.N;
    hipLaunchKernelGGL(k_splitk_reduce, grid1(MN), dim3(256), 0, st, g.scratch, g.C, MN, z, g.accumulate);
  }
  return hipGetLastError();
}

#define L1(kernel, n, ...) hipLaunchKernelGGL(kernel, grid1(n), dim3(256), 0, st, __VA_ARGS__)

void conv3_reorder(const uint16_t* Wb, uint16_t* Wr, int Co, int Ci, hipStream_t st) {
  L1(k_conv3_reorder, (long long)((Ci + HC - 1) / HC) * Co * 9 * HC, Wb, Wr, Co, Ci);
}
size_t conv3_reordered_size(int Co, int Ci) { return (size_t)((Ci + HC - 1) / HC) * Co * 9 * HC; }

namespace {
template <int MT, typename TX, typename TY>
void launch_halo(dim3 grid, int mode, const uint16_t* Wr, const TX* X, const float* bias, bool relu, TY* Y, int Co,
                 int Ci, int Bn, int H, int W, int BC, const ConvEpi& ep, hipStream_t st) {
  if constexpr (sizeof(TY) == 2) {
    if (mode == CONV_POOL) {
      hipLaunchKernelGGL((k_conv3_halo<MT, 2, TX, TY, CONV_POOL>), grid, dim3(256), 0, st, Wr, X, bias, (int)relu, Y,
                         Co, Ci, Bn, H, W, BC, ep);
      return;
    }
    if constexpr (MT == 32) {
      if (mode == CONV_OUT) {
        hipLaunchKernelGGL((k_conv3_halo<MT, 2, TX, TY, CONV_OUT>), grid, dim3(256), 0, st, Wr, X, bias, (int)relu,
                           Y, Co, Ci, Bn, H, W, BC, ep);
        return;
      }
    }
  }
  hipLaunchKernelGGL((k_conv3_halo<MT, 2, TX, TY, CONV_STORE>), grid, dim3(256), 0, st, Wr, X, bias, (int)relu, Y, Co,
                     Ci, Bn, H, W, BC, ep);
}

// shape check and launch of the halo-tile convolution; false (nothing
// launched) when the shape or the epilogue does not fit it
template <typename TX, typename TY>
bool conv3_halo(const uint16_t* Wb, const uint16_t* Wr, const TX* X, TY* Y, int Co, int Ci, int Bn, int H, int W,
                const float* bias, bool relu, int mode, const ConvEpi& ep, hipStream_t st) {
  constexpr bool XH = sizeof(TX) == 2, YH = sizeof(TY) == 2;
  if (!(Wr && W % 8 == 0 && bias && (long long)Bn * H * W <= 0x7fffffffLL && ((uintptr_t)Wr & 15) == 0))
    return false;
  // channel blocks of 16 (16-byte aligned) for BF16 activations; fused
  // epilogues only on them
  if ((XH && (Ci % 16 || ((uintptr_t)X & 15))) || (YH && (Co % 16 || ((uintptr_t)Y & 15))) ||
      (!YH && mode != CONV_STORE))
    return false;
  if (Ci <= 2 && Co <= 32) {   // first layer: the depth is 9 Ci, two MFMA steps
    if constexpr (XH) {
      return false;   // (a BF16 input has channel blocks of 16)
    } else {
      const int BC = W < 64 ? W : 64;
      if (mode != CONV_STORE || 256 % BC || (256 / BC + 2) * (BC + 2) > C2_TX) return false;
      const int BR = 256 / BC;
      const long long blocks = (long long)Bn * ((H + BR - 1) / BR) * ((W + BC - 1) / BC);
      hipLaunchKernelGGL((k_conv3_c2<TX, TY>), dim3((unsigned)blocks), dim3(256), 0, st, Wb, X, bias, (int)relu, Y,
                         Co, Ci, Bn, H, W, BC);
      return true;
    }
  }
  const int MT = Co <= 32 ? 32 : 64, NTW = 2, NT = 4096 / MT * NTW, BC = W < 64 ? W : 64;
  const int np = (NT / BC + 2) * (BC + 2);
  if (!(NT % BC == 0 && np * HC <= HX && 2 * np <= 256 * (MT == 64 ? 1 + NTW : 2 + NTW))) return false;
  const int BR = NT / BC;
  if (mode == CONV_POOL && (BC % 32 || BR % 2 || H % 2 || W % 2 || !ep.pool || ((uintptr_t)ep.pool & 15)))
    return false;
  if (mode == CONV_OUT && (Co != 32 || !ep.wo || !ep.bo || !ep.z || !ep.prob)) return false;
  const long long blocks = (long long)Bn * ((H + BR - 1) / BR) * ((W + BC - 1) / BC);
  const dim3 grid((unsigned)blocks, (Co + MT - 1) / MT);
  if (MT == 32)
    launch_halo<32>(grid, mode, Wr, X, bias, relu, Y, Co, Ci, Bn, H, W, BC, ep, st);
  else
    launch_halo<64>(grid, mode, Wr, X, bias, relu, Y, Co, Ci, Bn, H, W, BC, ep, st);
  return true;
}
}  // namespace

bool conv3_h(const uint16_t* Wb, const uint16_t* Wr, const void* X, bool x_bf16, uint16_t* Y, int Co, int Ci, int Bn,
             int H, int W, const float* bias, bool relu, int mode, const ConvEpi& ep, hipStream_t st) {
  return x_bf16 ? conv3_halo(Wb, Wr, static_cast<const uint16_t*>(X), Y, Co, Ci, Bn, H, W, bias, relu, mode, ep, st)
                : conv3_halo(Wb, Wr, static_cast<const float*>(X), Y, Co, Ci, Bn, H, W, bias, relu, mode, ep, st);
}

bool conv3_implicit(const uint16_t* Wb, const uint16_t* Wr, const float* X, float* Y, int Co, int Ci, int Bn,
                    int H, int W, const float* bias, bool relu, hipStream_t st) {
  // direct convolution over halo tiles where a block of whole 8-aligned
  // columns fits the tile
  if (conv3_halo(Wb, Wr, X, Y, Co, Ci, Bn, H, W, bias, relu, CONV_STORE, ConvEpi{}, st)) return true;
  const int K = Ci * 9;
  const long long N = (long long)Bn * H * W;
  if (W % 8 || K % 8 || ((uintptr_t)Wb & 15) || N > 0x7fffffffLL) return false;
  const Im2col ic{X, Bn, H, W};
  if (Co <= 32)
    hipLaunchKernelGGL((k_gemm_v<32, GV_IM2COL>), dim3((unsigned)((N + 127) / 128), (Co + 31) / 32), dim3(256), 0, st,
                       Wb, (long long)K, nullptr, 0LL, ic, Y, N, Co, (int)N, K, 0, bias, (int)relu);
  else
    hipLaunchKernelGGL((k_gemm_v<64, GV_IM2COL>), dim3((unsigned)((N + 63) / 64), (Co + 63) / 64), dim3(256), 0, st,
                       Wb, (long long)K, nullptr, 0LL, ic, Y, N, Co, (int)N, K, 0, bias, (int)relu);
  return true;
}

bool up_direct(const uint16_t* Wb, const float* X, const float* bias, float* Y, int Co, int Ci, int Bn, int h,
               int w, hipStream_t st) {
  const long long N = (long long)Bn * h * w;
  if (N % 8 || Ci % 8 || N > 0x7fffffffLL || ((uintptr_t)Wb & 15) || ((uintptr_t)X & 15)) return false;
  const Im2col ic{X, Bn, h, w};
  const int M = 4 * Co;
  hipLaunchKernelGGL((k_gemm_v<64, GV_UP>), dim3((unsigned)((N + 63) / 64), (M + 63) / 64), dim3(256), 0, st, Wb,
                     (long long)Ci, nullptr, N, ic, Y, 0LL, M, (int)N, Ci, 0, bias, 0);
  return true;
}

bool conv1_out(const uint16_t* Wb, const float* X, const float* bias, float* Y, int C, long long N, hipStream_t st) {
  L1(k_conv1_out, N, Wb, X, bias, Y, C, N);
  return true;
}
bool tconv(const uint16_t* Wb, int Co, const void* X, bool x_bf16, int C, int Tin, int Tout, int KT, int S, int P,
           long long Np, const float* bias, bool relu, void* Y, int y_bf16, hipStream_t st) {
  const long long N = (long long)Tout * Np;
  const int K = C * KT;
  if (!x_bf16 || Co > 32 || Np % 8 || N > 0x7fffffffLL || ((uintptr_t)Wb & 15) || ((uintptr_t)X & 15) ||
      ((uintptr_t)Y & 15) || (y_bf16 == 2 && (Co % 16 || Tout != 1)))
    return false;
  Im2col ic{};
  ic.TX = X;
  ic.Tin = Tin;
  ic.KT = KT;
  ic.S = S;
  ic.P = P;
  ic.out_h = y_bf16;
  ic.Np = Np;
  const long long tiles = (N + 127) / 128;
  ic.xcd = Tout > 1 && Np % 128 == 0 && tiles % 8 == 0;   // tile order of the kernel's GV_TCONV remap
  hipLaunchKernelGGL((k_gemm_v<32, GV_TCONV>), dim3((unsigned)tiles, 1), dim3(256), 0, st, Wb, (long long)K,
                     nullptr, 0LL, ic, static_cast<float*>(Y), N, Co, (int)N, K, 0, bias, (int)relu);
  return true;
}

bool conv3_first2_h(const uint16_t* W1, const float* b1, int Co1, int Ci1, const float* X, const uint16_t* W2r,
                    const float* b2, int Co2, int Ci2, uint16_t* Y, uint16_t* Yp, int Bn, int H, int W,
                    hipStream_t st) {
  if (Co1 != 32 || Ci1 != 2 || Co2 != 32 || Ci2 != 32 || H % 4 || W % 64 || !W1 || !b1 || !W2r || !b2 || !X ||
      ((uintptr_t)W2r & 15) || ((uintptr_t)Y & 15) || ((uintptr_t)Yp & 15) || (long long)Bn * H * W > 0x7fffffffLL)
    return false;
  const long long blocks = (long long)Bn * (H / 4) * (W / 64);
  hipLaunchKernelGGL(k_conv3_first2, dim3((unsigned)blocks), dim3(256), 0, st, W1, b1, X, W2r, b2, Y, Yp, Bn, H, W);
  return true;
}

bool up2_h(const uint16_t* Wb, const uint16_t* X, const float* bias, uint16_t* Y, int Co, int Ci, int Bn, int h, int w,
           hipStream_t st) {
  const long long npix = (long long)Bn * h * w;
  if (npix < 1 || 4 * npix > 0x7fffffffLL || ((uintptr_t)Wb & 15) || ((uintptr_t)X & 15) || ((uintptr_t)Y & 7))
    return false;
  const long long nblk = (npix + 31) / 32;
  const dim3 grid((unsigned)std::min<long long>((nblk + 1) / 2, 1024));
#define UP2(MI, KS)                                                                                     \
  if (4 * Co == 32 * MI && Ci == 16 * KS) {                                                              \
    hipLaunchKernelGGL((k_up2_h<MI, KS>), grid, dim3(256), 0, st, Wb, X, bias, Y, Bn, h, w);            \
    return true;                                                                                         \
  }
  UP2(4, 4)
  UP2(4, 8)
  UP2(8, 4)
  UP2(8, 8)
#undef UP2
  return false;
}
void im2col3(const float* X, uint16_t* col, int C, int Bn, int H, int W, hipStream_t st) {
  if (W % 8 == 0 && ((uintptr_t)col & 15) == 0)
    L1(k_im2col3_v, (long long)C * 9 * Bn * H * W / 8, X, col, C, Bn, H, W);
  else
    L1(k_im2col3, (long long)C * 9 * Bn * H * W, X, col, C, Bn, H, W);
}
void col2im3(const float* dcol, float* dX, int C, int Bn, int H, int W, bool acc, hipStream_t st) {
  L1(k_col2im3, (long long)C * Bn * H * W, dcol, dX, C, Bn, H, W, (int)acc);
}
void tnorm(const uint16_t* frames, float* out, int Bn, int L, long long HW, hipStream_t st) {
  L1(k_tnorm, (long long)Bn * HW, frames, out, Bn, L, HW);
}
bool tconv1_h(const uint16_t* frames, int L, const uint16_t* Wb, int Co, int KT, const float* bias, uint16_t* a1,
              int Bn, long long HW, hipStream_t st) {
  const long long Np = (long long)Bn * HW;
  if (L != T1_L || Co != 32 || KT != T1_K || Np % 64 || ((uintptr_t)a1 & 15)) return false;
  const long long waves = Np / 64;
  hipLaunchKernelGGL(k_tconv1_h, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, frames, Wb, bias, a1, Bn, HW);
  return true;
}
void im2col1(const float* in, uint16_t* col, int C, int Tin, int Tout, int KT, int S, int P, long long N,
             hipStream_t st) {
  L1(k_im2col1, (long long)C * KT * Tout * N, in, col, C, Tin, Tout, KT, S, P, N);
}
void col2im1(const float* dcol, float* din, int C, int Tin, int Tout, int KT, int S, int P, long long N,
             hipStream_t st) {
  L1(k_col2im1, (long long)C * Tin * N, dcol, din, C, Tin, Tout, KT, S, P, N);
}
void bias_act(float* Y, const float* b, int C, long long N, bool relu, hipStream_t st) {
  L1(k_bias_act, (long long)C * N, Y, b, C, N, (int)relu);
}
void relu_bwd(float* dY, const float* Y, long long n, hipStream_t st) { L1(k_relu_bwd, n, dY, Y, n); }
void bias_grad(const float* dY, float* db, int C, long long N, hipStream_t st) {
  hipLaunchKernelGGL(k_bias_grad, dim3(C), dim3(256), 0, st, dY, db, N, 0);
}
void pool(const float* X, float* Y, uint8_t* arg, int CB, int H, int W, hipStream_t st) {
  L1(k_pool, (long long)CB * (H / 2) * (W / 2), X, Y, arg, CB, H, W);
}
void pool_bwd(const float* dY, const uint8_t* arg, float* dX, int CB, int H, int W, bool acc, hipStream_t st) {
  L1(k_pool_bwd, (long long)CB * H * W, dY, arg, dX, CB, H, W, (int)acc);
}
void up_scatter(const float* Z, const float* b, float* Y, int Co, int Bn, int h, int w, hipStream_t st) {
  L1(k_up_scatter, (long long)Co * Bn * 4 * h * w, Z, b, Y, Co, Bn, h, w);
}
void up_gather(const float* dY, float* dZ, int Co, int Bn, int h, int w, hipStream_t st) {
  L1(k_up_gather, (long long)Co * 4 * Bn * h * w, dY, dZ, Co, Bn, h, w);
}
void bce(const float* z, const float* y, float* dz, float* prob, float* part, long long n, hipStream_t st) {
  L1(k_bce, n, z, y, dz, prob, part, n);
}
void rmsprop(float* w, const float* g, float* v, uint16_t* wb, long long n, float lr, float rho, float eps,
             hipStream_t st) {
  L1(k_rmsprop, n, w, g, v, wb, n, lr, rho, eps);
}
void to_bf16_copy(const float* w, uint16_t* wb, long long n, hipStream_t st) { L1(k_to_bf16, n, w, wb, n); }

void st_norm(const float* stin, float* x, int Bn, long long HW, hipStream_t stream) {
  hipLaunchKernelGGL(k_st_norm, dim3((unsigned)Bn), dim3(NORM_NT), 0, stream, stin, x, Bn, HW);
}
int st_origins(int n) { return (n - 64 + 31) / 32 + 1; }
void st_patches(const float* S, const float* T, int H, int W, float* out, hipStream_t st) {
  st_patches_n(S, T, H, W, 1, out, st);
}
void st_merge(const float* prob, int H, int W, float* out, hipStream_t st) { st_merge_n(prob, H, W, 1, out, st); }
void st_patches_n(const float* S, const float* T, int H, int W, int n, float* out, hipStream_t st) {
  const long long total = (long long)st_origins(H) * st_origins(W) * 2 * 4096;
  hipLaunchKernelGGL(k_st_patches, dim3(grid1(total).x, n), dim3(256), 0, st, S, T, H, W, out);
}
void st_merge_n(const float* prob, int H, int W, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_st_merge, dim3(grid1((long long)H * W).x, n), dim3(256), 0, st, prob, H, W, out);
}

}  // namespace nn
}  // namespace seg
