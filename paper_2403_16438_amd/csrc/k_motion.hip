// Rigid motion correction by patch-wise ZNCC (Sec. II).
//
// A frame F is compared with an integer template T: for every 21 x 21 tile
// p of F and every integer vector d with |dy|, |dx| <= R, the zero-mean
// normalised cross-correlation of F's tile with T's window at p + d. The
// per-vector sum over tiles picks the motion of the frame.
//
// With n = 441 pixels, ZNCC = (n C - sF sT) / (sqrt(vF) sqrt(vT)), where
//   C  = sum F T over the tile (the cross term),
//   sF = sum F, vF = n sum F^2 - sF^2 (per frame and tile),
//   sT = sum T, vT = n sum T^2 - sT^2 (per tile and vector, from integral
//        images of T and T^2: the table-based area sums).
// All of these are integers below 2^53, so FP64 holds them exactly; C is a
// contraction of the template windows (rows d) with the frame tiles
// (columns: frames) and runs on FP64 MFMA, whose products and partial sums
// of integers below 2^53 are exact in any order. Only the reciprocal square
// roots (one per frame and tile, one per tile and vector, from tables) and
// the final products round.
#include "seg_motion.h"

#include <mutex>

// Partial ZNCC sums of seg_mc_estimate_static, for callers that cannot
// allocate device memory: one copy per GPU, held until the process ends.
// Host code never passes this name to a kernel (on the host it is only a
// stand-in): the device address comes from mc_static_scratch below.
static __device__ __align__(256) double scratch[seg::kMcStaticDoubles];

namespace seg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kMaxTW = kPatch + 2 * kMcMaxRadius;
constexpr int kSThreads = 512;               // scoring workgroup: 8 waves
constexpr int kSWaves = kSThreads / 64;

// ---- template -------------------------------------------------------------

__global__ void k_mc_template(const uint16_t* __restrict__ f, int n, long long M, uint16_t* __restrict__ t) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= M) return;
  uint32_t s = 0;
  for (int i = 0; i < n; ++i) s += f[(size_t)i * M + x];
  t[x] = (uint16_t)((s + (uint32_t)n / 2) / (uint32_t)n);
}

// ---- integral images and window tables --------------------------------------

// ii1, ii2: [H+1][W+1], row 0 and column 0 zero. Pass 1: running sums along
// each row (one thread per row); pass 2: down each column.
__global__ void k_mc_rows(const uint16_t* __restrict__ t, int H, int W, unsigned long long* ii1,
                          unsigned long long* ii2) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y > H) return;
  const size_t row = (size_t)y * (W + 1);
  unsigned long long a = 0, b = 0;
  ii1[row] = 0;
  ii2[row] = 0;
  for (int x = 0; x < W; ++x) {
    if (y > 0) {
      const unsigned long long v = t[(size_t)(y - 1) * W + x];
      a += v;
      b += v * v;
    }
    ii1[row + x + 1] = a;
    ii2[row + x + 1] = b;
  }
}

__global__ void k_mc_cols(int H, int W, unsigned long long* ii1, unsigned long long* ii2) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x > W) return;
  unsigned long long a = 0, b = 0;
  for (int y = 0; y <= H; ++y) {
    const size_t i = (size_t)y * (W + 1) + x;
    a += ii1[i];
    b += ii2[i];
    ii1[i] = a;
    ii2[i] = b;
  }
}

__global__ void k_mc_windows(McGeom g, const unsigned long long* __restrict__ ii1,
                             const unsigned long long* __restrict__ ii2, double* sT, double* vT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.P * g.Vp) return;
  const int p = i / g.Vp, v = i % g.Vp;
  if (v >= g.V) {
    sT[i] = 0.0;
    vT[i] = 0.0;
    return;
  }
  const int side = 2 * g.R + 1;
  const int y0 = g.oy + (p / g.nx) * kPatch + v / side - g.R;
  const int x0 = g.ox + (p % g.nx) * kPatch + v % side - g.R;
  const size_t w1 = (size_t)g.W + 1;
  auto box = [&](const unsigned long long* ii) {
    return ii[(size_t)(y0 + kPatch) * w1 + x0 + kPatch] - ii[(size_t)y0 * w1 + x0 + kPatch] -
           ii[(size_t)(y0 + kPatch) * w1 + x0] + ii[(size_t)y0 * w1 + x0];
  };
  const long long s1 = (long long)box(ii1), s2 = (long long)box(ii2);
  const long long var = kPatchPix * s2 - s1 * s1;
  sT[i] = (double)s1;
  vT[i] = var > 0 ? 1.0 / sqrt((double)var) : 0.0;   // 0: zero variance, ZNCC 0
}

// ---- scores -------------------------------------------------------------------

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The cross terms of one tile for the NT vector tiles a wave owns: per step
// of depth 4, one frame value and NT template values from LDS (held as FP64,
// converted once when staged), then NT independent MFMAs. NT is a compile-time count, so the loads of a step are
// issued together and no lane mask guards the MFMAs.
template <int NT, int TPW>
__device__ __forceinline__ void corr_tiles(d4 (&acc)[TPW], const double* s_t, const double* fb,
                                           const int (&dbase)[TPW], int q, int TW) {
  int x = q, off = q;                       // pixel k = 4 kk + q at (k / 21, k % 21)
#pragma unroll 1
  for (int kk = 0; kk < kPatchK / 4; ++kk) {
    const double b = fb[4 * kk];
    double av[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) av[i] = s_t[dbase[i] + off];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], b, acc[i], 0, 0, 0);
    x += 4;
    off += 4;
    if (x >= kPatch) {
      x -= kPatch;
      off += TW - kPatch;
    }
  }
}

// One workgroup: kMcFrames frames x one slice of tiles. Wave w owns the
// 16-vector tiles w, w + 8, ... (TPW of them). FP64 MFMA 16x16x4: lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16) and holds
// D(4 j + l / 16, l % 16) in element j; here A rows are vectors, the depth is
// the tile's pixels, and B columns are frames.
template <int TPW>
__global__ __launch_bounds__(kSThreads) void k_mc_scores(McScoreArgs a) {
  const McGeom g = a.g;
  __shared__ double s_t[(kMaxTW + 1) * kMaxTW];     // template window, one extra zero row
  __shared__ double s_f[kMcFrames * kPatchK];       // frame tiles, zero padded
  __shared__ double s_sf[kMcFrames], s_rf[kMcFrames];
  const int slice = blockIdx.x % g.S, grp = blockIdx.x / g.S;
  const int f0 = grp * kMcFrames;
  const int nf = min(kMcFrames, a.n - f0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, q = lane >> 4;
  const int MT = g.Vp / 16, side = 2 * g.R + 1, TW = g.TW;
  // vector tiles of this wave: wave, wave + 8, ... below MT (wave-uniform)
  const int nt = min(TPW, max(0, (MT - wave + kSWaves - 1) / kSWaves));
  const long long M = (long long)g.H * g.W;

  int dbase[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int d = (wave + kSWaves * i) * 16 + col;
    dbase[i] = (wave + kSWaves * i < MT && d < g.V) ? (d / side) * TW + d % side : 0;
  }
  double score[TPW][4];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) score[i][j] = 0.0;

  const int p0 = slice * g.pps, p1 = min(g.P, p0 + g.pps);
  for (int p = p0; p < p1; ++p) {
    const int py = g.oy + (p / g.nx) * kPatch, px = g.ox + (p % g.nx) * kPatch;
    __syncthreads();
    for (int i = tid; i < (TW + 1) * TW; i += kSThreads) {
      const int r = i / TW, c = i % TW;
      s_t[i] = r < TW ? (double)a.tmpl[(size_t)(py - g.R + r) * g.W + px - g.R + c] : 0.0;
    }
    for (int i = tid; i < kMcFrames * kPatchK; i += kSThreads) {
      const int f = i / kPatchK, k = i % kPatchK;
      double v = 0.0;
      if (f < nf && k < kPatchPix)
        v = (double)a.frames[(size_t)(f0 + f) * M + (size_t)(py + k / kPatch) * g.W + px + k % kPatch];
      s_f[i] = v;
    }
    __syncthreads();
    // exact per-frame moments of the tile
#pragma unroll
    for (int j = 0; j < kMcFrames / kSWaves; ++j) {
      const int f = wave * (kMcFrames / kSWaves) + j;
      unsigned long long s = 0, s2 = 0;
      for (int k = lane; k < kPatchPix; k += 64) {
        const unsigned long long v = (unsigned long long)s_f[f * kPatchK + k];
        s += v;
        s2 += v * v;
      }
      s = wave_sum_u64(s);
      s2 = wave_sum_u64(s2);
      if (lane == 0) {
        const long long v = (long long)(kPatchPix * s2) - (long long)(s * s);
        s_sf[f] = (double)s;
        s_rf[f] = v > 0 ? 1.0 / sqrt((double)v) : 0.0;
      }
    }
    __syncthreads();

    d4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    const double* fb = s_f + col * kPatchK + q;
    switch (nt) {
      case 1: corr_tiles<1>(acc, s_t, fb, dbase, q, TW); break;
      case 2: if constexpr (TPW >= 2) corr_tiles<2>(acc, s_t, fb, dbase, q, TW); break;
      case 3: if constexpr (TPW >= 3) corr_tiles<3>(acc, s_t, fb, dbase, q, TW); break;
      case 4: if constexpr (TPW >= 4) corr_tiles<4>(acc, s_t, fb, dbase, q, TW); break;
      default: break;
    }
    const double rf = s_rf[col], sf = s_sf[col];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      if (i >= nt) break;
      const int t = wave + kSWaves * i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int d = t * 16 + 4 * j + q;
        const double st = a.sT[(size_t)p * g.Vp + d], rt = a.vT[(size_t)p * g.Vp + d];
        score[i][j] += ((double)kPatchPix * acc[i][j] - sf * st) * rf * rt;
      }
    }
  }
  if (col < nf) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      if (i >= nt) break;
      const int t = wave + kSWaves * i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int d = t * 16 + 4 * j + q;
        a.part[((size_t)slice * a.chunk + f0 + col) * g.Vp + d] = score[i][j];
      }
    }
  }
}

// ---- pick and apply -----------------------------------------------------------

// One wave per frame: lanes take vectors d = lane, lane + 64, ...; the slice
// sums are added in slice order; the first maximum wins.
__global__ __launch_bounds__(kThreads) void k_mc_pick(McGeom g, const double* __restrict__ part, int chunk,
                                                      int n, int32_t* motion, double* scores) {
  const int f = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (f >= n) return;
  double best = -1.0e300;
  int arg = 0x7fffffff;
  for (int d = lane; d < g.V; d += 64) {
    double s = 0.0;
    for (int sl = 0; sl < g.S; ++sl) s += part[((size_t)sl * chunk + f) * g.Vp + d];
    if (scores) scores[(size_t)f * g.V + d] = s;
    if (s > best) {
      best = s;
      arg = d;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oa = __shfl_xor(arg, o, 64);
    if (ob > best || (ob == best && oa < arg)) {
      best = ob;
      arg = oa;
    }
  }
  if (lane == 0) {
    const int side = 2 * g.R + 1;
    motion[2 * (size_t)f] = -(arg / side - g.R);
    motion[2 * (size_t)f + 1] = -(arg % side - g.R);
  }
}

// C(y, x) = F(y + my, x + mx) where that pixel is in the frame, else the
// template's T(y, x). Grid: x runs over the 8-pixel runs of a frame, y over
// frames (uniform motion per workgroup); each thread gathers one run and
// writes it with one 16-byte store. Frame widths that are not a multiple of
// 8 take the per-pixel kernel.
__global__ void k_mc_apply8(const uint16_t* __restrict__ in, int H, int W, const int32_t* __restrict__ motion,
                            const uint16_t* __restrict__ tmpl, uint16_t* __restrict__ out) {
  const int runs = W >> 3;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H * runs) return;
  const size_t f = blockIdx.y;
  const int y = i / runs, x0 = (i - y * runs) << 3;
  const int my = motion[2 * f], mx = motion[2 * f + 1];
  const size_t M = (size_t)H * W;
  const int sy = y + my;
  const uint16_t* trow = tmpl + (size_t)y * W + x0;
  uint16_t v[8];
  if (sy < 0 || sy >= H) {
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = trow[k];
  } else {
    const uint16_t* srow = in + f * M + (size_t)sy * W;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int sx = x0 + k + mx;
      v[k] = (sx >= 0 && sx < W) ? srow[sx] : trow[k];
    }
  }
  uint4 pk;
  pk.x = v[0] | ((uint32_t)v[1] << 16);
  pk.y = v[2] | ((uint32_t)v[3] << 16);
  pk.z = v[4] | ((uint32_t)v[5] << 16);
  pk.w = v[6] | ((uint32_t)v[7] << 16);
  *reinterpret_cast<uint4*>(out + f * M + (size_t)y * W + x0) = pk;
}

__global__ void k_mc_apply1(const uint16_t* __restrict__ in, int H, int W, const int32_t* __restrict__ motion,
                            const uint16_t* __restrict__ tmpl, uint16_t* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= H * W) return;
  const size_t f = blockIdx.y, M = (size_t)H * W;
  const int y = r / W, x = r % W;
  const int sy = y + motion[2 * f], sx = x + motion[2 * f + 1];
  const bool inside = sy >= 0 && sy < H && sx >= 0 && sx < W;
  out[f * M + r] = inside ? in[f * M + (size_t)sy * W + sx] : tmpl[r];
}

}  // namespace

hipError_t launch_mc_template(const uint16_t* frames, int n, long long M, uint16_t* tmpl, hipStream_t st) {
  hipLaunchKernelGGL(k_mc_template, dim3((unsigned)((M + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                     frames, n, M, tmpl);
  return hipGetLastError();
}

hipError_t launch_mc_tables(const McGeom& g, const uint16_t* tmpl, unsigned long long* ii, double* sT,
                            double* vT, hipStream_t st) {
  unsigned long long* ii2 = ii + (size_t)(g.H + 1) * (g.W + 1);
  hipLaunchKernelGGL(k_mc_rows, dim3((g.H + 1 + 63) / 64), dim3(64), 0, st, tmpl, g.H, g.W, ii, ii2);
  hipLaunchKernelGGL(k_mc_cols, dim3((g.W + 1 + 63) / 64), dim3(64), 0, st, g.H, g.W, ii, ii2);
  const int n = g.P * g.Vp;
  hipLaunchKernelGGL(k_mc_windows, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, g, ii, ii2, sT,
                     vT);
  return hipGetLastError();
}

hipError_t launch_mc_scores(const McScoreArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  const int groups = (a.n + kMcFrames - 1) / kMcFrames;
  const dim3 grid((unsigned)(groups * a.g.S)), block(kSThreads);
  const int tpw = (a.g.Vp / 16 + kSWaves - 1) / kSWaves;
  switch (tpw) {
    case 1: hipLaunchKernelGGL(k_mc_scores<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_mc_scores<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_mc_scores<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_mc_scores<4>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mc_pick(const McGeom& g, const double* part, int chunk, int n, int32_t* motion,
                          double* scores, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int per = kThreads / 64;
  hipLaunchKernelGGL(k_mc_pick, dim3((unsigned)((n + per - 1) / per)), dim3(kThreads), 0, st, g, part, chunk, n,
                     motion, scores);
  return hipGetLastError();
}

hipError_t launch_mc_apply(const uint16_t* in, long long n, int H, int W, const int32_t* motion,
                           const uint16_t* tmpl, uint16_t* out, hipStream_t st) {
  const bool vec = W % 8 == 0 && ((uintptr_t)out & 15) == 0;
  const long long per = vec ? (long long)H * (W / 8) : (long long)H * W;
  const unsigned bx = (unsigned)((per + kThreads - 1) / kThreads);
  for (long long f0 = 0; f0 < n; f0 += 65535) {
    const unsigned nf = (unsigned)(n - f0 < 65535 ? n - f0 : 65535);
    const size_t o = (size_t)f0 * H * W;
    if (vec)
      hipLaunchKernelGGL(k_mc_apply8, dim3(bx, nf), dim3(kThreads), 0, st, in + o, H, W, motion + 2 * f0, tmpl,
                         out + o);
    else
      hipLaunchKernelGGL(k_mc_apply1, dim3(bx, nf), dim3(kThreads), 0, st, in + o, H, W, motion + 2 * f0, tmpl,
                         out + o);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t mc_static_scratch(double** ptr) {
  static std::mutex mu;
  static double* cache[kMaxMcDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxMcDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> hold(mu);
  if (!cache[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    cache[dev] = static_cast<double*>(p);
  }
  *ptr = cache[dev];
  return hipSuccess;
}

}  // namespace seg
