// Streaming segment-summary kernel: one pass over the uint16 video computes,
// per 50-frame segment and pixel,
//   S_i  temporal mean (Eq. 1),
//   T_i  max minus median over time of the Gaussian-smoothed video (Eq. 2),
//   D_i  mean of max(0, median - smoothed value) (noise-scale term),
//   U_i, P_i  sums of reference-subtracted values and of their products with
//        the right, lower, lower-right and lower-left neighbours (pooled
//        co-moments of the correlation image).
//
// Work decomposition: one workgroup of 256 threads per (64 x 16 pixel tile,
// segment). Per frame the tile plus a 12-pixel halo (88 x 40) is staged in
// LDS as d = V - R, where R is a per-pixel integer reference (the median of
// the segment's first three frames). Subtracting R leaves T, D and the
// centred co-moments unchanged but keeps the smoothed values small, so the
// per-pixel window can be held in FP32 without losing the precision the
// event threshold needs. The separable smoothing accumulates in FP64
// (full-rate FMA on gfx950): a vertical pass over 88 columns into LDS, then
// a horizontal pass straight into each thread's window registers. Every
// thread owns 4 adjacent pixels of one tile row and keeps their 50 smoothed
// values in VGPRs (40) and a per-thread LDS slot (the chunk being filled);
// after the segment a compare-exchange network gives the
// median, the maximum and the 25 smallest values.
#include "seg_kernels.h"
#include "selnet_gen.h"

namespace seg {
namespace {

constexpr int L = kSegLen;
constexpr int RAD = kMaxRadius;
constexpr int NTAP = 2 * RAD + 1;
constexpr int TW = 64, TH = 16;
constexpr int DW = TW + 2 * RAD;     // 88 staged columns
constexpr int DH = TH + 2 * RAD;     // 40 staged rows
constexpr int NT = 256;
constexpr int NPX = 4;               // pixels per thread
constexpr int CH = 10;               // frames per unrolled chunk
constexpr int NCH = L / CH;          // 5 chunks per segment
constexpr int ROWS_PER_WAVE = DH / 4;
constexpr int XTRA = DW - 64;        // 24 columns loaded by a second lane pass
static_assert(L % CH == 0, "chunking");
static_assert(DH % 4 == 0, "rows per wave");

struct KParams {
  const uint16_t* src0;
  const uint16_t* src1;
  long long n0;
  int H, W;
  int seg0, nseg;
  float *T, *S, *D, *U, *P;
  long long plane;
  double w[NTAP];
};

struct BatchSlot {
  KParams p;
  int ntile;   // tiles per segment
  int item0;   // first work item of this slot
  int quad;    // quad loader usable (W % 4 == 0 and W >= 16)
  int pad;
};

struct BatchTable {
  int nslots;
  int total;   // work items over all slots
  int pad[2];
  BatchSlot slot[kMaxBatch];
};

__device__ __forceinline__ int reflect(int j, int n) {
  const int m = 2 * n;
  j %= m;
  if (j < 0) j += m;
  return j >= n ? m - 1 - j : j;
}

__device__ __forceinline__ int med3i(int a, int b, int c) {
  return max(min(a, b), min(max(a, b), c));
}

// LDS-only workgroup barrier: waits for this wave's LDS traffic, not for its
// outstanding global loads, so the next frame's prefetch stays in flight.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Vertical pass for one (column, 8-row) task: U rows 8h..8h+7 of column c,
// streaming the 32 staged rows once.
constexpr int VROWS = 8;
constexpr int NVT8 = DW * (TH / VROWS);   // 176 tasks, one round
static_assert(NVT8 <= NT, "one vertical round");

__device__ __forceinline__ void vtask8(int q, const float* __restrict__ Dl,
                                       float* __restrict__ Ul, const KParams& p) {
  const int c = q % DW;
  const int h = q / DW;
  const float* col = Dl + h * VROWS * DW + c;
  double acc[VROWS];
#pragma unroll
  for (int o = 0; o < VROWS; ++o) acc[o] = 0.0;
#pragma unroll
  for (int j = 0; j < NTAP + VROWS - 1; ++j) {
    const double x = (double)col[j * DW];
#pragma unroll
    for (int o = 0; o < VROWS; ++o)
      if (j - o >= 0 && j - o < NTAP) acc[o] = fma(p.w[j - o], x, acc[o]);
  }
  float* out = Ul + h * VROWS * DW + c;
#pragma unroll
  for (int o = 0; o < VROWS; ++o) out[o * DW] = (float)acc[o];
}

// Quad loader: the staged region (40 rows x 88 columns) as 880 groups of 4
// consecutive columns. With W % 4 == 0 and W >= 16, every group maps to 4
// contiguous source columns, ascending, or descending where the group lies in
// the reflected border, so one 8-byte load fetches it.
constexpr int QPR = DW / 4;          // 22 groups per row
constexpr int NQ = DH * QPR;         // 880
constexpr int KQ = (NQ + NT - 1) / NT;  // 4 groups per thread at most

struct QuadPlan {
  int off[KQ];    // element offset of the group's lowest source column
  int dst[KQ];    // first LDS index of the group
  int rev;        // bit k: group k is reversed
  int nk;         // groups this thread owns
};

__device__ __forceinline__ QuadPlan quad_plan(int tid, int ty0, int tx0, int H, int W) {
  QuadPlan qp;
  qp.rev = 0;
  qp.nk = 0;
#pragma unroll
  for (int k = 0; k < KQ; ++k) {
    const int q = tid + k * NT;
    const int qq = q < NQ ? q : 0;
    const int r = qq / QPR, c4 = qq - r * QPR;
    const int srow = reflect(ty0 - RAD + r, H);
    const int a = tx0 - RAD + 4 * c4;
    const int c0 = reflect(a, W), c3 = reflect(a + 3, W);
    qp.off[k] = srow * W + (c3 < c0 ? c3 : c0);
    qp.dst[k] = r * DW + 4 * c4;
    if (c3 < c0) qp.rev |= 1 << k;
    if (q < NQ) qp.nk = k + 1;
  }
  return qp;
}

__device__ __forceinline__ void unpack4(uint2 v, bool rev, int (&x)[4]) {
  const int a = (int)(v.x & 0xffffu), b = (int)(v.x >> 16), c = (int)(v.y & 0xffffu), d = (int)(v.y >> 16);
  x[0] = rev ? d : a;
  x[1] = rev ? c : b;
  x[2] = rev ? b : c;
  x[3] = rev ? a : d;
}

struct Smem {
  float Dl[DH * DW];
  float Rl[DH * DW];
  float Ul[TH * DW];
  float4 Wl[CH * NT];
};

// One (segment sl, tile) work item of one recording.
template <bool QUAD>
__device__ __forceinline__ void block_body(const KParams& p, int sl, int tile, Smem& sm) {
  float* Dl = sm.Dl;
  float* Rl = sm.Rl;
  float* Ul = sm.Ul;
  float4* Wl = sm.Wl;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tiles_x = (p.W + TW - 1) / TW;
  const int ty0 = (tile / tiles_x) * TH;
  const int tx0 = (tile % tiles_x) * TW;
  const long long M = (long long)p.H * p.W;

  const long long fbase = (long long)sl * L;
  auto frame = [&](int t) -> const uint16_t* {
    const long long f = fbase + t;
    return f < p.n0 ? p.src0 + f * M : p.src1 + (f - p.n0) * M;
  };

  // ---- staging geometry
  QuadPlan qp;
  int cx0 = 0, cx1 = 0;
  int rowoff[ROWS_PER_WAVE];
  if constexpr (QUAD) {
    qp = quad_plan(tid, ty0, tx0, p.H, p.W);
  } else {
    // wave wv loads rows wv, wv+4, ...; lane = column
    cx0 = reflect(tx0 - RAD + lane, p.W);
    cx1 = reflect(tx0 - RAD + 64 + (lane < XTRA ? lane : 0), p.W);
#pragma unroll
    for (int k = 0; k < ROWS_PER_WAVE; ++k)
      rowoff[k] = __builtin_amdgcn_readfirstlane(reflect(ty0 - RAD + wv + 4 * k, p.H) * p.W);
  }

  // ---- per-pixel reference: median of the segment's first three frames
  {
    const uint16_t* f0 = frame(0);
    const uint16_t* f1 = frame(1);
    const uint16_t* f2 = frame(2);
    if constexpr (QUAD) {
#pragma unroll
      for (int k = 0; k < KQ; ++k) {
        if (k < qp.nk) {
          int a[4], b[4], c[4];
          const bool rv = (qp.rev >> k) & 1;
          unpack4(*reinterpret_cast<const uint2*>(f0 + qp.off[k]), rv, a);
          unpack4(*reinterpret_cast<const uint2*>(f1 + qp.off[k]), rv, b);
          unpack4(*reinterpret_cast<const uint2*>(f2 + qp.off[k]), rv, c);
          *reinterpret_cast<float4*>(Rl + qp.dst[k]) =
              make_float4((float)med3i(a[0], b[0], c[0]), (float)med3i(a[1], b[1], c[1]),
                          (float)med3i(a[2], b[2], c[2]), (float)med3i(a[3], b[3], c[3]));
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < ROWS_PER_WAVE; ++k) {
        const int r = wv + 4 * k;
        const int o = rowoff[k];
        Rl[r * DW + lane] = (float)med3i(f0[o + cx0], f1[o + cx0], f2[o + cx0]);
        if (lane < XTRA)
          Rl[r * DW + 64 + lane] = (float)med3i(f0[o + cx1], f1[o + cx1], f2[o + cx1]);
      }
    }
  }
  __syncthreads();

  // ---- thread-owned pixels: tile row hy, columns hx0 .. hx0+3
  const int hy = tid >> 4;
  const int hx0 = (tid & 15) * NPX;
  const float* own = Dl + (hy + RAD) * DW + hx0 + RAD;

  // 40 of the 50 window values live in VGPRs (chunks 0..3); the chunk being
  // filled lives in a per-thread LDS slot, so the frame loop needs no
  // compile-time frame index. The chunk loop is unrolled, so a completed
  // chunk c moves once into its own registers win[c].
  float win[NCH - 1][CH][NPX];
  float Uacc[NPX], Pacc[5][NPX];
#pragma unroll
  for (int i = 0; i < NPX; ++i) {
    Uacc[i] = 0.f;
#pragma unroll
    for (int k = 0; k < 5; ++k) Pacc[k][i] = 0.f;
  }

  uint2 pf[KQ];   // next frame's raw groups (quad path)
  if constexpr (QUAD) {
    const uint16_t* fr = frame(0);
#pragma unroll
    for (int k = 0; k < KQ; ++k)
      if (k < qp.nk) pf[k] = *reinterpret_cast<const uint2*>(fr + qp.off[k]);
  }

#pragma unroll
  for (int c = 0; c < NCH; ++c) {
#pragma unroll 1
    for (int f = 0; f < CH; ++f) {
      const int t = c * CH + f;
      // (a) stage d = V - R for the tile and its halo
      if constexpr (QUAD) {
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
          if (k < qp.nk) {
            int x[4];
            unpack4(pf[k], (qp.rev >> k) & 1, x);
            const float4 r = *reinterpret_cast<const float4*>(Rl + qp.dst[k]);
            *reinterpret_cast<float4*>(Dl + qp.dst[k]) =
                make_float4((float)x[0] - r.x, (float)x[1] - r.y, (float)x[2] - r.z, (float)x[3] - r.w);
          }
        }
        // prefetch frame t + 1 while this frame is processed
        if (t + 1 < L) {
          const uint16_t* fr = frame(t + 1);
#pragma unroll
          for (int k = 0; k < KQ; ++k)
            if (k < qp.nk) pf[k] = *reinterpret_cast<const uint2*>(fr + qp.off[k]);
        }
      } else {
        const uint16_t* fr = frame(t);
#pragma unroll
        for (int k = 0; k < ROWS_PER_WAVE; ++k) {
          const int r = wv + 4 * k;
          const int o = rowoff[k];
          Dl[r * DW + lane] = (float)fr[o + cx0] - Rl[r * DW + lane];
          if (lane < XTRA) Dl[r * DW + 64 + lane] = (float)fr[o + cx1] - Rl[r * DW + 64 + lane];
        }
      }
      lds_barrier();
      // (b) co-moment sums of the raw (reference-subtracted) values
      {
        float a[NPX + 1], b[NPX + 2];
#pragma unroll
        for (int i = 0; i <= NPX; ++i) a[i] = own[i];
#pragma unroll
        for (int i = 0; i < NPX + 2; ++i) b[i] = own[DW - 1 + i];
#pragma unroll
        for (int i = 0; i < NPX; ++i) {
          const float d = a[i];
          Uacc[i] += d;
          Pacc[0][i] = fmaf(d, d, Pacc[0][i]);
          Pacc[1][i] = fmaf(d, a[i + 1], Pacc[1][i]);
          Pacc[2][i] = fmaf(d, b[i + 1], Pacc[2][i]);
          Pacc[3][i] = fmaf(d, b[i + 2], Pacc[3][i]);
          Pacc[4][i] = fmaf(d, b[i], Pacc[4][i]);
        }
      }
      // (c) vertical pass into Ul
      if (tid < NVT8) vtask8(tid, Dl, Ul, p);
      lds_barrier();
      // (d) horizontal pass into this thread's LDS chunk slot
      {
        const float* row = Ul + hy * DW + hx0;
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
#pragma unroll
        for (int j = 0; j < NTAP + 3; ++j) {
          const double x = (double)row[j];
          if (j < NTAP) b0 = fma(p.w[j], x, b0);
          if (j >= 1 && j < NTAP + 1) b1 = fma(p.w[j - 1], x, b1);
          if (j >= 2 && j < NTAP + 2) b2 = fma(p.w[j - 2], x, b2);
          if (j >= 3) b3 = fma(p.w[j - 3], x, b3);
        }
        Wl[f * NT + tid] = make_float4((float)b0, (float)b1, (float)b2, (float)b3);
      }
    }
    if (c < NCH - 1) {
#pragma unroll
      for (int f = 0; f < CH; ++f) {
        const float4 q = Wl[f * NT + tid];
        win[c][f][0] = q.x;
        win[c][f][1] = q.y;
        win[c][f][2] = q.z;
        win[c][f][3] = q.w;
      }
    }
  }

  // ---- per-pixel selection and outputs
  const int gy = ty0 + hy;
  const float* rref = Rl + (hy + RAD) * DW + hx0 + RAD;
  const long long obase = (long long)(p.seg0 + sl) * M + (long long)gy * p.W;
#pragma unroll
  for (int i = 0; i < NPX; ++i) {
    float v[L];
#pragma unroll
    for (int s = 0; s < NCH - 1; ++s)
#pragma unroll
      for (int f = 0; f < CH; ++f) v[s * CH + f] = win[s][f][i];
#pragma unroll
    for (int f = 0; f < CH; ++f) {
      const float4 q = Wl[f * NT + tid];
      v[(NCH - 1) * CH + f] = i == 0 ? q.x : i == 1 ? q.y : i == 2 ? q.z : q.w;
    }
    SELNET50(v);
    const double med = 0.5 * ((double)v[SELNET50_LO] + (double)v[SELNET50_HI]);
    double lo = 0.0;
#pragma unroll
    for (int k = 0; k <= SELNET50_LO; ++k) lo += (double)v[k];
    const double dsum = (double)(L / 2) * med - lo;
    const int gx = tx0 + hx0 + i;
    if (gy < p.H && gx < p.W) {
      const long long o = obase + gx;
      p.T[o] = (float)((double)v[SELNET50_MAX] - med);
      p.D[o] = (float)(dsum / (double)L);
      p.S[o] = (float)(((double)L * (double)rref[i] + (double)Uacc[i]) / (double)L);
      p.U[o] = Uacc[i];
#pragma unroll
      for (int k = 0; k < 5; ++k) p.P[k * p.plane + o] = Pacc[k][i];
    }
  }
}

template <bool QUAD>
__global__ __launch_bounds__(NT, 2) void k_block_stats(KParams p) {
  __shared__ Smem sm;
  const int tiles_x = (p.W + TW - 1) / TW;
  const int tiles_y = (p.H + TH - 1) / TH;
  const int ntile = tiles_x * tiles_y;
  const int nblk = ntile * p.nseg;
  // Blocks are dealt round-robin over the 8 XCDs; give every XCD a
  // contiguous range of (segment, tile) pairs so that neighbouring tiles of a
  // segment share their halo rows in one L2.
  const int per = (nblk + 7) / 8;
  const int logical = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (logical >= nblk) return;
  const int sl = logical / ntile;
  block_body<QUAD>(p, sl, logical - sl * ntile, sm);
}

// Serving: one persistent launch over the work items of several recordings
// described by a device-side slot table (so the launch can be captured once
// in a graph and replayed after the table is rewritten).
__global__ __launch_bounds__(NT, 2) void k_block_stats_batch(const BatchTable* __restrict__ tab) {
  __shared__ Smem sm;
  const int ns = tab->nslots;
  const int total = tab->total;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    int s = 0;
    while (s + 1 < ns && tab->slot[s + 1].item0 <= item) ++s;
    const BatchSlot& bs = tab->slot[s];
    const KParams p = bs.p;
    const int local = item - bs.item0;
    const int sl = local / bs.ntile;
    const int tile = local - sl * bs.ntile;
    if (bs.quad)
      block_body<true>(p, sl, tile, sm);
    else
      block_body<false>(p, sl, tile, sm);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_block_stats(const StreamLaunch& a, hipStream_t st) {
  KParams p;
  p.src0 = a.src0;
  p.src1 = a.src1;
  p.n0 = a.n0;
  p.H = a.H;
  p.W = a.W;
  p.seg0 = a.seg0;
  p.nseg = a.nseg;
  p.T = a.T;
  p.S = a.S;
  p.D = a.D;
  p.U = a.U;
  p.P = a.P;
  p.plane = a.plane;
  for (int k = 0; k < NTAP; ++k) p.w[k] = a.w[k];
  const int tiles = ((a.W + TW - 1) / TW) * ((a.H + TH - 1) / TH);
  const long long nblk = (long long)tiles * a.nseg;
  const long long per = (nblk + 7) / 8;
  if (a.W % 4 == 0 && a.W >= 16)
    hipLaunchKernelGGL(k_block_stats<true>, dim3((unsigned)(per * 8)), dim3(NT), 0, st, p);
  else
    hipLaunchKernelGGL(k_block_stats<false>, dim3((unsigned)(per * 8)), dim3(NT), 0, st, p);
  return hipGetLastError();
}

size_t batch_table_bytes() { return sizeof(BatchTable); }

// Fill the host copy of the slot table; returns the number of work items.
int fill_batch_table(void* host_table, const StreamLaunch* launches, int count) {
  BatchTable* t = static_cast<BatchTable*>(host_table);
  int items = 0, ns = 0;
  for (int k = 0; k < count; ++k) {
    const StreamLaunch& a = launches[k];
    if (a.nseg <= 0) continue;
    BatchSlot& b = t->slot[ns++];
    b.p.src0 = a.src0;
    b.p.src1 = a.src1;
    b.p.n0 = a.n0;
    b.p.H = a.H;
    b.p.W = a.W;
    b.p.seg0 = a.seg0;
    b.p.nseg = a.nseg;
    b.p.T = a.T;
    b.p.S = a.S;
    b.p.D = a.D;
    b.p.U = a.U;
    b.p.P = a.P;
    b.p.plane = a.plane;
    for (int j = 0; j < NTAP; ++j) b.p.w[j] = a.w[j];
    b.ntile = ((a.W + TW - 1) / TW) * ((a.H + TH - 1) / TH);
    b.item0 = items;
    b.quad = (a.W % 4 == 0 && a.W >= 16) ? 1 : 0;
    b.pad = 0;
    items += b.ntile * a.nseg;
  }
  t->nslots = ns;
  t->total = items;
  return items;
}

hipError_t launch_block_stats_batch(const void* dev_table, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_block_stats_batch, dim3(grid), dim3(NT), 0, st,
                     static_cast<const BatchTable*>(dev_table));
  return hipGetLastError();
}

}  // namespace seg
