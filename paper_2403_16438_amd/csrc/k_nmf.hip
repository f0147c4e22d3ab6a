// Per-component NMF P_c ~ F A (Eq. 3, Sec. III-D), FP64 arithmetic, one
// workgroup of 1024 threads per component of the aggregate mask.
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
//           F and A live in LDS when they fit (dynamic size chosen by the
//           host), and the column sums F^T P are split over Q pixel ranges
//           reduced in a fixed order.
//   scale   each f_n to max 1, a_n inversely
// Every reduction has a fixed order, so results are bit-reproducible.
#include <algorithm>

#include "seg_kernels.h"

namespace seg {
namespace {

constexpr int NT = 1024;
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

template <bool LDS>
__global__ __launch_bounds__(NT) void k_nmf(NmfArgs a) {
  extern __shared__ double dyn[];
  __shared__ double red[NW * NPAIR];
  __shared__ int redi[NW];
  __shared__ double gram[R8 * R8];
  __shared__ int picks[R8];
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const int off = a.coff[c];
  const int Mc = a.coff[c + 1] - off;
  const int K = a.K;
  const int Q = a.Q;
  float* P = reinterpret_cast<float*>(a.P) + (long long)off * K;    // [Mc][K]
  float* PT = reinterpret_cast<float*>(a.PT) + (long long)off * K;  // [K][Mc]
  double* R = a.R + (long long)off * K;                              // [Mc][K]
  double* U = a.G + (long long)off * R8;                             // SPA direction
  double* nz = a.Wk + (long long)c * 2 * a.Kmax;                     // [K] flags
  double* prj = nz + a.Kmax;                                         // [K]
  // LDS carve-up: A [R8][K], partial column sums [Q][R8][K], F [Mc][R8];
  // without room in LDS, A and F live in the output arrays and Q = 1 (each
  // thread sums a whole column, no partial sums)
  // (the placement is a template parameter so that LDS accesses compile to
  // ds instructions rather than flat ones)
  double* A;
  double* part;
  double* F;
  int As;                                                            // row stride of A
  if constexpr (LDS) {
    A = dyn;
    part = dyn + R8 * K;
    F = dyn + (long long)R8 * K * (1 + Q);
    As = K;
  } else {
    A = a.A + (long long)c * R8 * a.Kmax;
    part = nullptr;
    F = a.F + (long long)off * R8;
    As = a.Kmax;
  }

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
    for (int n = 0; n < R8; ++n) A[(long long)n * As + i] = 0.0;
  __syncthreads();

  const int mq = (Mc + Q - 1) / Q;   // pixels per partition of the column sums
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
    // partial F^T P over pixel range q of column i (LDS placement); with
    // Q = 1 the column sums stay in registers below
    if constexpr (LDS) {
      for (int e = t; e < Q * K; e += NT) {
        const int q = e / K, i = e - q * K;
        const int m0 = q * mq, m1 = min(Mc, m0 + mq);
        double fp[R8];
#pragma unroll
        for (int n = 0; n < R8; ++n) fp[n] = 0.0;
#pragma unroll 8
        for (int m = m0; m < m1; ++m) {
          const double pv = (double)P[(long long)m * K + i];
          const double* fm = F + (long long)m * R8;
#pragma unroll
          for (int n = 0; n < R8; ++n)
            if (n < N) fp[n] += fm[n] * pv;
        }
#pragma unroll
        for (int n = 0; n < R8; ++n)
          if (n < N) part[((long long)q * R8 + n) * K + i] = fp[n];
      }
      __syncthreads();
    }
    // per column: sum the partitions in order, then the rows of A in order
    for (int i = t; i < K; i += NT) {
      double fp[R8], av[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) {
        fp[n] = 0.0;
        av[n] = n < N ? A[(long long)n * As + i] : 0.0;
      }
      if constexpr (LDS) {
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int n = 0; n < R8; ++n)
            if (n < N) fp[n] += part[((long long)q * R8 + n) * K + i];
      } else {
#pragma unroll 8
        for (int m = 0; m < Mc; ++m) {
          const double pv = (double)P[(long long)m * K + i];
          const double* fm = F + (long long)m * R8;
#pragma unroll
          for (int n = 0; n < R8; ++n)
            if (n < N) fp[n] += fm[n] * pv;
        }
      }
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
        if (n < N) A[(long long)n * As + i] = av[n];
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
        for (int n = 0; n < R8; ++n) av[n] = n < N ? A[(long long)n * As + i] : 0.0;
        int k = 0;
#pragma unroll
        for (int n1 = 0; n1 < R8; ++n1)
#pragma unroll
          for (int n2 = n1; n2 < R8; ++n2, ++k) s[k] += av[n1] * av[n2];
      }
      block_gram(s, N, red, gram);
    }
    // per pixel m: P[m, :] A^T, then the columns of F in order; each thread
    // carries two pixels (m and m + NT) to keep more loads in flight
    for (int m0 = t; m0 < Mc; m0 += 2 * NT) {
      const int m1 = m0 + NT;
      const bool two = m1 < Mc;
      double g0[R8], g1[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) {
        g0[n] = 0.0;
        g1[n] = 0.0;
      }
#pragma unroll 4
      for (int i = 0; i < K; ++i) {
        const double pv0 = (double)PT[(long long)i * Mc + m0];
        const double pv1 = two ? (double)PT[(long long)i * Mc + m1] : 0.0;
#pragma unroll
        for (int n = 0; n < R8; ++n)
          if (n < N) {
            const double av = A[(long long)n * As + i];
            g0[n] += pv0 * av;
            g1[n] += pv1 * av;
          }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = h ? m1 : m0;
        if (h && !two) break;
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
              f[n] = fmax(0.0, f[n] + ((h ? g1[n] : g0[n]) - s) / d);
            }
          }
        }
#pragma unroll
        for (int n = 0; n < R8; ++n)
          if (n < N) F[(long long)m * R8 + n] = f[n];
      }
    }
    __syncthreads();
  }

  // ---------------------------------------------- scale to peak 1, export
  double* Ag = a.A + (long long)c * R8 * a.Kmax;
  double* Fg = a.F + (long long)off * R8;
  for (int n = 0; n < N; ++n) {
    double mx = 0.0;
    for (int m = t; m < Mc; m += NT) mx = fmax(mx, F[(long long)m * R8 + n]);
    const double best = block_max(mx, red);
    const double sc = best > 0.0 ? best : 1.0;
    for (int m = t; m < Mc; m += NT) Fg[(long long)m * R8 + n] = F[(long long)m * R8 + n] / sc;
    for (int i = t; i < K; i += NT) Ag[(long long)n * a.Kmax + i] = A[(long long)n * As + i] * sc;
    __syncthreads();
  }
  if (t == 0) a.N[c] = N;
}

}  // namespace

void plan_nmf(NmfArgs& a, int max_mc) {
  int dev = 0, max_lds = 65536;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    max_lds = 65536;   // the smallest LDS of the targets, if the query fails
  const size_t budget = max_lds > 16384 ? (size_t)max_lds - 8192 : 0;  // static LDS ~5 KB
  const size_t K = (size_t)a.K;
  int Q = (int)std::max<size_t>(1, std::min<size_t>(16, NT / std::max<size_t>(1, K)));
  auto aq = [&](int q) { return (size_t)R8 * K * 8 * (1 + q); };
  while (Q > 1 && aq(Q) > budget) --Q;
  a.lds_A = aq(Q) <= budget;
  if (!a.lds_A) Q = 1;
  a.Q = Q;
  const size_t used = a.lds_A ? aq(Q) : 0;
  const size_t fbytes = (size_t)max_mc * R8 * 8;
  a.lds_F = a.lds_A && used + fbytes <= budget;
  if (!a.lds_F) {  // global placement (A, partial sums and F), one pixel range
    a.lds_A = false;
    a.Q = 1;
  }
  a.lds_bytes = a.lds_F ? used + fbytes : 0;
}

hipError_t launch_nmf(const NmfArgs& a, hipStream_t st) {
  if (a.ncomp <= 0) return hipSuccess;
  if (a.lds_A && a.lds_F) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_nmf<true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)a.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nmf<true>, dim3(a.ncomp), dim3(NT), a.lds_bytes, st, a);
  } else {
    hipLaunchKernelGGL(k_nmf<false>, dim3(a.ncomp), dim3(NT), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace seg
