// Per-component NMF P_c ~ F A (Eq. 3, Sec. III-D), FP64 arithmetic, one
// workgroup of 512 threads per component of the aggregate mask.
//   gather  P_c[m][i] = p_i(x_m) for the component's pixels x_m (raster
//           order), stored twice in FP32 (exact: the maps are FP32): pixel-
//           major for column sweeps and segment-major for pixel sweeps
//   SPA     successive projection on the nonzero columns (FP64 residual):
//           pick the column of largest residual norm (lowest index on ties),
//           stop below delta x the first pick's norm or at the rank cap,
//           project the residual onto the complement of the picked direction
//   init    F = picked columns scaled to max 1, A = 0, one HALS update of A
//   HALS    `sweeps` times: rows of A in order, then columns of F in order,
//           each clipped at 0; a row/column with zero Gram diagonal is kept.
//           The A update is independent per column and the F update per
//           pixel, so a thread owns a column (a pixel), keeps it in
//           registers through the sequential row (column) updates, and only
//           the N x N Gram matrices F^T F and A A^T need block reductions.
//   scale   each f_n to max 1, a_n inversely
// Every reduction has a fixed order, so results are bit-reproducible.
#include "seg_internal.h"

namespace seg {
namespace {

constexpr int NT = 512;
constexpr int NW = NT / 64;
constexpr int R8 = kMaxRank;
constexpr int NPAIR = R8 * (R8 + 1) / 2;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Block-wide sums of the N(N+1)/2 pair values each thread holds in s[];
// result symmetric in gram[n1 * R8 + n2]. Fixed reduction order.
__device__ void block_gram(double (&s)[NPAIR], int N, double* red, double* gram) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int k = 0;
#pragma unroll
  for (int n1 = 0; n1 < R8; ++n1)
#pragma unroll
    for (int n2 = n1; n2 < R8; ++n2, ++k) {
      if (n2 < N) {
        const double v = wave_sum(s[k]);
        if (lane == 0) red[w * NPAIR + k] = v;
      }
    }
  __syncthreads();
  if (threadIdx.x < NPAIR) {
    const int kk = threadIdx.x;
    int n1 = 0, rem = kk;
    while (rem >= R8 - n1) {
      rem -= R8 - n1;
      ++n1;
    }
    const int n2 = n1 + rem;
    if (n2 < N) {
      double v = 0.0;
      for (int ww = 0; ww < NW; ++ww) v += red[ww * NPAIR + kk];
      gram[n1 * R8 + n2] = v;
      gram[n2 * R8 + n1] = v;
    }
  }
  __syncthreads();
}

__device__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if (lane == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
  for (int ww = 1; ww < NW; ++ww) m = fmax(m, red[ww]);
  __syncthreads();
  return m;
}

// argmax with lowest index on ties
__device__ void block_argmax(double v, int idx, double* red, int* redi, double* best, int* bidx) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (lane == 0) {
    red[w] = v;
    redi[w] = idx;
  }
  __syncthreads();
  double b = red[0];
  int bi = redi[0];
  for (int ww = 1; ww < NW; ++ww)
    if (red[ww] > b || (red[ww] == b && redi[ww] < bi)) {
      b = red[ww];
      bi = redi[ww];
    }
  *best = b;
  *bidx = bi;
  __syncthreads();
}

__global__ __launch_bounds__(NT) void k_nmf(NmfArgs a) {
  __shared__ double red[NW * NPAIR];
  __shared__ int redi[NW];
  __shared__ double gram[R8 * R8];
  __shared__ int picks[R8];
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const int off = a.coff[c];
  const int Mc = a.coff[c + 1] - off;
  const int K = a.K;
  float* P = reinterpret_cast<float*>(a.P) + (long long)off * K;    // [Mc][K]
  float* PT = reinterpret_cast<float*>(a.PT) + (long long)off * K;  // [K][Mc]
  double* R = a.R + (long long)off * K;                              // [Mc][K]
  double* F = a.F + (long long)off * R8;                             // [Mc][R8]
  double* U = a.G + (long long)off * R8;                             // SPA direction
  double* A = a.A + (long long)c * R8 * a.Kmax;                      // [R8][Kmax]
  double* nz = a.Wk + (long long)c * (R8 + 2) * a.Kmax;              // [K] flags
  double* prj = nz + a.Kmax;                                         // [K]

  for (long long e = t; e < (long long)Mc * K; e += NT) {
    const int m = (int)(e / K), i = (int)(e - (long long)m * K);
    const float v = a.p[(long long)i * a.M + a.pix[off + m]];
    P[e] = v;
    PT[(long long)i * Mc + m] = v;
    R[e] = (double)v;
  }
  __syncthreads();

  // ---------------------------------------------------------------- SPA
  for (int i = t; i < K; i += NT) {
    float s = 0.f;
    for (int m = 0; m < Mc; ++m) s = fmaxf(s, P[(long long)m * K + i]);
    nz[i] = s > 0.f ? 1.0 : 0.0;
  }
  __syncthreads();
  int N = 0;
  double ref = 0.0;
  while (N < a.max_rank) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int i = t; i < K; i += NT) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int m = 0;
      for (; m + 4 <= Mc; m += 4) {
        const double r0 = R[(long long)m * K + i], r1 = R[(long long)(m + 1) * K + i];
        const double r2 = R[(long long)(m + 2) * K + i], r3 = R[(long long)(m + 3) * K + i];
        s0 += r0 * r0;
        s1 += r1 * r1;
        s2 += r2 * r2;
        s3 += r3 * r3;
      }
      for (; m < Mc; ++m) {
        const double r = R[(long long)m * K + i];
        s0 += r * r;
      }
      const double nv = nz[i] > 0.0 ? sqrt((s0 + s1) + (s2 + s3)) : -1.0;
      if (nv > bv) {
        bv = nv;
        bi = i;
      }
    }
    double best;
    int j;
    block_argmax(bv, bi, red, redi, &best, &j);
    if (best <= 0.0) break;
    if (N == 0) ref = best;
    else if (best < a.delta * ref) break;
    if (t == 0) picks[N] = j;
    ++N;
    for (int m = t; m < Mc; m += NT) U[(long long)m * R8] = R[(long long)m * K + j] / best;
    __syncthreads();
    for (int i = t; i < K; i += NT) {
      double s0 = 0.0, s1 = 0.0;
      int m = 0;
      for (; m + 2 <= Mc; m += 2) {
        s0 += U[(long long)m * R8] * R[(long long)m * K + i];
        s1 += U[(long long)(m + 1) * R8] * R[(long long)(m + 1) * K + i];
      }
      if (m < Mc) s0 += U[(long long)m * R8] * R[(long long)m * K + i];
      prj[i] = s0 + s1;
    }
    __syncthreads();
    for (long long e = t; e < (long long)Mc * K; e += NT) {
      const int m = (int)(e / K), i = (int)(e - (long long)m * K);
      R[e] -= U[(long long)m * R8] * prj[i];
    }
    __syncthreads();
  }
  __syncthreads();

  // ------------------------------------------------- initial footprints
  for (int n = 0; n < N; ++n) {
    const int col = picks[n];
    double mx = 0.0;
    for (int m = t; m < Mc; m += NT) mx = fmax(mx, (double)P[(long long)m * K + col]);
    const double best = block_max(mx, red);
    for (int m = t; m < Mc; m += NT) F[(long long)m * R8 + n] = (double)P[(long long)m * K + col] / best;
  }
  for (int i = t; i < K; i += NT)
    for (int n = 0; n < R8; ++n) A[(long long)n * a.Kmax + i] = 0.0;
  __syncthreads();

  for (int sweep = -1; sweep < a.sweeps; ++sweep) {
    // ---- A update. Gram F^T F:
    {
      double s[NPAIR];
#pragma unroll
      for (int k = 0; k < NPAIR; ++k) s[k] = 0.0;
      for (int m = t; m < Mc; m += NT) {
        double f[R8];
#pragma unroll
        for (int n = 0; n < R8; ++n) f[n] = n < N ? F[(long long)m * R8 + n] : 0.0;
        int k = 0;
#pragma unroll
        for (int n1 = 0; n1 < R8; ++n1)
#pragma unroll
          for (int n2 = n1; n2 < R8; ++n2, ++k) s[k] += f[n1] * f[n2];
      }
      block_gram(s, N, red, gram);
    }
    // per column i: F^T P[:, i], then the rows of A in order
    for (int i = t; i < K; i += NT) {
      double fp[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) fp[n] = 0.0;
#pragma unroll 4
      for (int m = 0; m < Mc; ++m) {
        const double pv = (double)P[(long long)m * K + i];
        const double* fm = F + (long long)m * R8;
#pragma unroll
        for (int n = 0; n < R8; ++n)
          if (n < N) fp[n] += fm[n] * pv;
      }
      double av[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) av[n] = n < N ? A[(long long)n * a.Kmax + i] : 0.0;
#pragma unroll
      for (int n = 0; n < R8; ++n) {
        if (n < N) {
          const double d = gram[n * R8 + n];
          if (d > 0.0) {
            double s = 0.0;
#pragma unroll
            for (int n2 = 0; n2 < R8; ++n2)
              if (n2 < N) s += gram[n * R8 + n2] * av[n2];
            av[n] = fmax(0.0, av[n] + (fp[n] - s) / d);
          }
        }
      }
#pragma unroll
      for (int n = 0; n < R8; ++n)
        if (n < N) A[(long long)n * a.Kmax + i] = av[n];
    }
    __syncthreads();
    if (sweep < 0) continue;
    // ---- F update. Gram A A^T:
    {
      double s[NPAIR];
#pragma unroll
      for (int k = 0; k < NPAIR; ++k) s[k] = 0.0;
      for (int i = t; i < K; i += NT) {
        double av[R8];
#pragma unroll
        for (int n = 0; n < R8; ++n) av[n] = n < N ? A[(long long)n * a.Kmax + i] : 0.0;
        int k = 0;
#pragma unroll
        for (int n1 = 0; n1 < R8; ++n1)
#pragma unroll
          for (int n2 = n1; n2 < R8; ++n2, ++k) s[k] += av[n1] * av[n2];
      }
      block_gram(s, N, red, gram);
    }
    // per pixel m: P[m, :] A^T, then the columns of F in order
    for (int m = t; m < Mc; m += NT) {
      double g[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) g[n] = 0.0;
#pragma unroll 4
      for (int i = 0; i < K; ++i) {
        const double pv = (double)PT[(long long)i * Mc + m];
#pragma unroll
        for (int n = 0; n < R8; ++n)
          if (n < N) g[n] += pv * A[(long long)n * a.Kmax + i];
      }
      double f[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) f[n] = n < N ? F[(long long)m * R8 + n] : 0.0;
#pragma unroll
      for (int n = 0; n < R8; ++n) {
        if (n < N) {
          const double d = gram[n * R8 + n];
          if (d > 0.0) {
            double s = 0.0;
#pragma unroll
            for (int n2 = 0; n2 < R8; ++n2)
              if (n2 < N) s += f[n2] * gram[n2 * R8 + n];
            f[n] = fmax(0.0, f[n] + (g[n] - s) / d);
          }
        }
      }
#pragma unroll
      for (int n = 0; n < R8; ++n)
        if (n < N) F[(long long)m * R8 + n] = f[n];
    }
    __syncthreads();
  }

  // ---------------------------------------------- scale to peak 1
  for (int n = 0; n < N; ++n) {
    double mx = 0.0;
    for (int m = t; m < Mc; m += NT) mx = fmax(mx, F[(long long)m * R8 + n]);
    const double best = block_max(mx, red);
    if (best > 0.0) {
      for (int m = t; m < Mc; m += NT) F[(long long)m * R8 + n] /= best;
      for (int i = t; i < K; i += NT) A[(long long)n * a.Kmax + i] *= best;
    }
    __syncthreads();
  }
  if (t == 0) a.N[c] = N;
}

}  // namespace

hipError_t launch_nmf(const NmfArgs& a, hipStream_t st) {
  if (a.ncomp <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nmf, dim3(a.ncomp), dim3(NT), 0, st, a);
  return hipGetLastError();
}

}  // namespace seg
