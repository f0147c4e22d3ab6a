// Voltage trace extraction (Sec. II, third stage): the mean intensity of
// each footprint's region of interest in every frame.
//
// The masks of the footprints of one component are subsets of that
// component's pixels, and components are disjoint. A workgroup takes one
// component and a block of frames; every pixel that lies in at least one mask
// is read once per frame, and its mask bits (bit r: footprint r of the
// component) route it into up to kMaxRank integer sums. Sums are exact
// (uint16 values, 32-bit per lane, 64-bit across the wave); the mean is one
// correctly rounded FP64 division, stored as FP32.
#include "seg_kernels.h"
#include "seg_traces.h"

namespace seg {
namespace {

constexpr int kTraceThreads = 256;
constexpr int kTraceWaves = kTraceThreads / 64;
constexpr int kTraceFrames = 16;     // frames per workgroup
constexpr int kTraceLds = 4096;      // entries staged in LDS (larger components read HBM)
constexpr int kXcds = 8;             // MI355X dispatches workgroups to its 8 XCDs in turn

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Each wave takes kFramesPerWave consecutive frames at once: the gathers of
// one pixel in those frames are independent loads in flight together.
constexpr int kFramesPerWave = kTraceFrames / kTraceWaves;

template <int R>
__device__ __forceinline__ void trace_frames(const TraceArgs& a, const int4 c, const int* pix,
                                             const uint8_t* bits, int n, long long t0) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long tw = t0 + (long long)wave * kFramesPerWave;
  if (tw >= a.n_frames) return;
  const long long left = a.n_frames - tw;
  const int nf = left < kFramesPerWave ? (int)left : kFramesPerWave;
  const uint16_t* fr = a.frames + (size_t)tw * a.M;
  uint32_t acc[kFramesPerWave][R] = {};
  if (nf == kFramesPerWave) {
#pragma unroll 2
    for (int i = lane; i < n; i += 64) {
      const int p = pix[i];
      const uint32_t b = bits[i];
      uint32_t v[kFramesPerWave];
#pragma unroll
      for (int k = 0; k < kFramesPerWave; ++k) v[k] = fr[(size_t)k * a.M + p];
#pragma unroll
      for (int k = 0; k < kFramesPerWave; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[k][r] += (b >> r & 1u) ? v[k] : 0u;
    }
  } else {
    for (int i = lane; i < n; i += 64) {
      const int p = pix[i];
      const uint32_t b = bits[i];
#pragma unroll
      for (int k = 0; k < kFramesPerWave; ++k) {
        if (k >= nf) break;
        const uint32_t v = fr[(size_t)k * a.M + p];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[k][r] += (b >> r & 1u) ? v : 0u;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kFramesPerWave; ++k) {
    if (k >= nf) break;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r >= c.w) break;
      const unsigned long long s = wave_sum(acc[k][r]);
      if (lane == 0) {
        const int j = c.z + r;
        a.out[(size_t)j * a.ld + tw + k] = (float)((double)s / (double)a.count[j]);
      }
    }
  }
}

// One workgroup per (frame block, component), numbered so that each XCD
// takes a contiguous run of frame blocks with all their components: lines
// that two neighbouring components share are then fetched into one L2.
// R: accumulators per frame, at least the largest footprint count of a
// component in the launch.
template <int R>
__global__ __launch_bounds__(kTraceThreads) void k_traces(TraceArgs a, unsigned total) {
  __shared__ int s_pix[kTraceLds];
  __shared__ uint8_t s_bits[kTraceLds];
  const unsigned xcd = blockIdx.x % kXcds, q = blockIdx.x / kXcds;
  const unsigned per = total / kXcds, rem = total % kXcds;
  const unsigned u = xcd * per + (xcd < rem ? xcd : rem) + q;
  const unsigned fblk = u / (unsigned)a.ncomp;
  const int4 c = a.comp[u % (unsigned)a.ncomp];  // x, y: entry range; z: first footprint; w: footprints
  const long long t0 = (long long)fblk * kTraceFrames;
  const int n = c.y - c.x;
  if (n <= kTraceLds) {
    for (int i = threadIdx.x; i < n; i += kTraceThreads) {
      s_pix[i] = a.pix[c.x + i];
      s_bits[i] = a.bits[c.x + i];
    }
    __syncthreads();
    trace_frames<R>(a, c, s_pix, s_bits, n, t0);
  } else {
    trace_frames<R>(a, c, a.pix + c.x, a.bits + c.x, n, t0);
  }
}

}  // namespace

hipError_t launch_traces(const TraceArgs& a, hipStream_t st) {
  if (a.n_frames <= 0 || a.ncomp <= 0) return hipSuccess;
  // frames per launch: a multiple of the frame block with at most 2^31 - 1 workgroups
  const long long max_blocks = 0x7fffffffLL / a.ncomp;
  if (max_blocks < 1) return hipErrorInvalidValue;
  const long long chunk = max_blocks * kTraceFrames;
  for (long long f0 = 0; f0 < a.n_frames; f0 += chunk) {
    TraceArgs b = a;
    b.frames = a.frames + (size_t)f0 * a.M;
    b.out = a.out + f0;
    b.n_frames = a.n_frames - f0 < chunk ? a.n_frames - f0 : chunk;
    const long long total = (b.n_frames + kTraceFrames - 1) / kTraceFrames * a.ncomp;
    const dim3 grid((unsigned)total), block(kTraceThreads);
    if (a.max_fp <= 1)
      hipLaunchKernelGGL(k_traces<1>, grid, block, 0, st, b, (unsigned)total);
    else if (a.max_fp <= 2)
      hipLaunchKernelGGL(k_traces<2>, grid, block, 0, st, b, (unsigned)total);
    else if (a.max_fp <= 4)
      hipLaunchKernelGGL(k_traces<4>, grid, block, 0, st, b, (unsigned)total);
    else
      hipLaunchKernelGGL(k_traces<kMaxRank>, grid, block, 0, st, b, (unsigned)total);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace seg
