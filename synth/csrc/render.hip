// GPU renderer of the seeded synthetic videos (input generator only: none of
// the segmentation method's arithmetic).
//
//   lam(x, t) = flick(t) * [ B(x) (1 + drift t / T) + sum_j g_j(x) act_j(t) ]
//   V(x, t)   = clip(round(Poisson(lam) + read_noise * N(0, 1)), 0, 65535)
//
// The scene (B, g_j, act_j, flick) comes from the host simulator; only the
// noise differs from it. Random numbers: Philox4x32-10 (Salmon, Moraes, Dror
// and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) keyed by
// the seed, counter = (pixel, frame, stream word, 0). Normals by Box-Muller.
// Poisson: inversion of the CDF for lam < 30, the normal approximation
// round(lam + sqrt(lam) z) above (a generator choice, documented as such).
// Footprint values below 1e-6 of their peak are zero in the GPU copy of the
// scene, so each pixel only visits nearby neurons.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

struct u4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
  const uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}

__device__ __forceinline__ u4 philox4x32_10(u4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo(0xD2511F53u, c.x, hi0, lo0);
    mulhilo(0xCD9E8D57u, c.z, hi1, lo1);
    c = u4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// uniform in (0, 1]
__device__ __forceinline__ double uni(uint32_t v) { return ((double)v + 1.0) * (1.0 / 4294967296.0); }

constexpr int FR = 50;   // frames per thread: each footprint value is read once per 50 frames

__global__ __launch_bounds__(256) void k_render(const float* __restrict__ B, const float* __restrict__ G,
                                                const float* __restrict__ act, const float* __restrict__ flick,
                                                float drift, int N, int M, int t0, int nf, int T, uint32_t k0,
                                                uint32_t k1, float read_noise, uint16_t* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int f0 = blockIdx.y * FR;
  if (x >= M) return;
  const int nfr = min(FR, nf - f0);
  float sig[FR];
#pragma unroll
  for (int k = 0; k < FR; ++k) sig[k] = 0.f;
  for (int j = 0; j < N; ++j) {
    const float g = G[(long long)j * M + x];
    if (g != 0.f) {
      const float* a = act + (long long)j * T + t0 + f0;
#pragma unroll
      for (int k = 0; k < FR; ++k)
        if (k < nfr) sig[k] += g * a[k];
    }
  }
  const float b = B[x];
#pragma unroll
  for (int k = 0; k < FR; ++k) {
    if (k >= nfr) break;
    const int t = t0 + f0 + k;
    double lam = ((double)b * (1.0 + (double)drift * t / T) + (double)sig[k]) * (double)flick[t];
    if (lam < 0.0) lam = 0.0;
    const u4 r = philox4x32_10(u4{(uint32_t)x, (uint32_t)t, 0u, 0u}, k0, k1);
    const double rad = sqrt(-2.0 * log(uni(r.x)));
    const double ang = 6.283185307179586 * uni(r.y);
    const double z1 = rad * cos(ang), z2 = rad * sin(ang);
    double pois;
    if (lam < 30.0) {
      // inversion: smallest k with CDF(k) >= u
      const double u = uni(r.z);
      double p = exp(-lam), cdf = p;
      int kk = 0;
      while (cdf < u && kk < 1000) {
        ++kk;
        p *= lam / kk;
        cdf += p;
      }
      pois = (double)kk;
    } else {
      pois = rint(lam + sqrt(lam) * z1);
    }
    double v = rint(pois + (double)read_noise * z2);
    v = v < 0.0 ? 0.0 : (v > 65535.0 ? 65535.0 : v);
    out[(long long)(f0 + k) * M + x] = (uint16_t)v;
  }
}

}  // namespace

extern "C" int synth_render(const float* B, const float* G, const float* act, const float* flick,
                            float drift, int N, int H, int W, int t0, int nf, int T,
                            unsigned long long seed, float read_noise, uint16_t* out, void* stream) {
  if (!B || !flick || !out || H < 1 || W < 1 || nf < 0 || t0 < 0 || t0 + nf > T) return -1;
  if (N > 0 && (!G || !act)) return -1;
  if (nf == 0) return 0;
  const int M = H * W;
  dim3 grid((M + 255) / 256, (nf + FR - 1) / FR);
  hipLaunchKernelGGL(k_render, grid, dim3(256), 0, static_cast<hipStream_t>(stream), B, G, act, flick,
                     drift, N, M, t0, nf, T, (uint32_t)seed, (uint32_t)(seed >> 32), read_noise, out);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}
