// Per-component NMF P_c ~ F A (Eq. 3, Sec. III-D), FP64, one workgroup per
// component of the aggregate mask.
//   gather  P_c[m][i] = p_i(x_m) for the component's pixels x_m (raster order)
//   SPA     successive projection on the nonzero columns: pick the column of
//           largest residual norm (lowest index on ties), stop below delta x
//           the first pick's norm or at the rank cap, project the residual
//           onto the complement of the picked direction
//   init    F = picked columns scaled to max 1, A = 0, one HALS update of A
//   HALS    `sweeps` times: rows of A in order, then columns of F in order,
//           each clipped at 0; a row/column with zero Gram diagonal is kept
//   scale   each f_n to max 1, a_n inversely
// Reductions run in a fixed order per thread, so results are deterministic.
#include "seg_internal.h"

namespace seg {
namespace {

constexpr int NT = 256;
constexpr int R8 = kMaxRank;

__device__ void block_argmax(double v, int idx, double* sv, int* si, double* best, int* bidx) {
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = idx;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (t < off) {
      const double a = sv[t], b = sv[t + off];
      const int ia = si[t], ib = si[t + off];
      if (b > a || (b == a && ib < ia)) {
        sv[t] = b;
        si[t] = ib;
      }
    }
    __syncthreads();
  }
  *best = sv[0];
  *bidx = si[0];
  __syncthreads();
}

__global__ __launch_bounds__(NT) void k_nmf(NmfArgs a) {
  __shared__ double sv[NT];
  __shared__ int si[NT];
  __shared__ double gram[R8 * R8];
  __shared__ int picks[R8];
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const int off = a.coff[c];
  const int Mc = a.coff[c + 1] - off;
  const int K = a.K;
  double* P = a.P + (long long)off * K;     // [Mc][K]
  double* PT = a.PT + (long long)off * K;   // [K][Mc]
  double* R = a.R + (long long)off * K;     // [Mc][K]
  double* F = a.F + (long long)off * R8;    // [Mc][R8]
  double* G = a.G + (long long)off * R8;    // [Mc][R8]
  double* A = a.A + (long long)c * R8 * a.Kmax;          // [R8][K]
  double* FtP = a.Wk + (long long)c * (R8 + 2) * a.Kmax; // [R8][K]
  double* nrm = FtP + (long long)R8 * a.Kmax;           // [K]
  double* prj = nrm + a.Kmax;                            // [K]

  // gather
  for (long long e = t; e < (long long)Mc * K; e += NT) {
    const int m = (int)(e / K), i = (int)(e - (long long)m * K);
    const double v = (double)a.p[(long long)i * a.M + a.pix[off + m]];
    P[e] = v;
    R[e] = v;
    PT[(long long)i * Mc + m] = v;
  }
  __syncthreads();

  // SPA on the nonzero columns
  int N = 0;
  double ref = 0.0;
  for (int i = t; i < K; i += NT) {
    double s = 0.0;
    for (int m = 0; m < Mc; ++m) s += fabs(P[(long long)m * K + i]);
    prj[i] = s > 0.0 ? 1.0 : 0.0;   // nonzero-column flag until the first projection
  }
  __syncthreads();
  while (N < a.max_rank) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int i = t; i < K; i += NT) {
      double s = 0.0;
      for (int m = 0; m < Mc; ++m) {
        const double r = R[(long long)m * K + i];
        s += r * r;
      }
      const double nv = prj[i] > 0.0 ? sqrt(s) : -1.0;
      nrm[i] = nv;
      if (nv > bv) {
        bv = nv;
        bi = i;
      }
    }
    double best;
    int j;
    block_argmax(bv, bi, sv, si, &best, &j);
    if (best <= 0.0) break;
    if (N == 0) ref = best;
    else if (best < a.delta * ref) break;
    if (t == 0) picks[N] = j;
    ++N;
    // u = R[:, j] / ||R[:, j]||, coefficients v_i = u . R[:, i], R -= u v^T
    for (int m = t; m < Mc; m += NT) G[(long long)m * R8] = R[(long long)m * K + j] / best;
    __syncthreads();
    for (int i = t; i < K; i += NT) {
      double s = 0.0;
      for (int m = 0; m < Mc; ++m) s += G[(long long)m * R8] * R[(long long)m * K + i];
      nrm[i] = s;
    }
    __syncthreads();
    for (long long e = t; e < (long long)Mc * K; e += NT) {
      const int m = (int)(e / K), i = (int)(e - (long long)m * K);
      R[e] -= G[(long long)m * R8] * nrm[i];
    }
    __syncthreads();
  }
  __syncthreads();

  // initial footprints: picked raw columns scaled to max 1
  for (int n = 0; n < N; ++n) {
    double mx = 0.0;
    for (int m = t; m < Mc; m += NT) {
      const double v = P[(long long)m * K + picks[n]];
      F[(long long)m * R8 + n] = v;
      mx = fmax(mx, v);
    }
    double best;
    int dummy;
    block_argmax(mx, 0, sv, si, &best, &dummy);
    for (int m = t; m < Mc; m += NT) F[(long long)m * R8 + n] /= best;
  }
  for (int n = 0; n < N; ++n)
    for (int i = t; i < K; i += NT) A[(long long)n * a.Kmax + i] = 0.0;
  __syncthreads();

  for (int sweep = -1; sweep < a.sweeps; ++sweep) {
    // ---- A update: FtP = F^T P, FtF = F^T F
    for (int i = t; i < K; i += NT) {
      double s[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) s[n] = 0.0;
      for (int m = 0; m < Mc; ++m) {
        const double pv = P[(long long)m * K + i];
#pragma unroll
        for (int n = 0; n < R8; ++n)
          if (n < N) s[n] += F[(long long)m * R8 + n] * pv;
      }
#pragma unroll
      for (int n = 0; n < R8; ++n)
        if (n < N) FtP[(long long)n * a.Kmax + i] = s[n];
    }
    if (t < N * N) {
      const int n1 = t / N, n2 = t % N;
      double s = 0.0;
      for (int m = 0; m < Mc; ++m) s += F[(long long)m * R8 + n1] * F[(long long)m * R8 + n2];
      gram[n1 * R8 + n2] = s;
    }
    __syncthreads();
    for (int n = 0; n < N; ++n) {
      const double d = gram[n * R8 + n];
      if (d > 0.0) {
        for (int i = t; i < K; i += NT) {
          double s = 0.0;
          for (int n2 = 0; n2 < N; ++n2) s += gram[n * R8 + n2] * A[(long long)n2 * a.Kmax + i];
          const long long ai = (long long)n * a.Kmax + i;
          A[ai] = fmax(0.0, A[ai] + (FtP[ai] - s) / d);
        }
      }
      __syncthreads();
    }
    if (sweep < 0) continue;
    // ---- F update: PAt = P A^T, AAt = A A^T
    for (int m = t; m < Mc; m += NT) {
      double s[R8];
#pragma unroll
      for (int n = 0; n < R8; ++n) s[n] = 0.0;
      for (int i = 0; i < K; ++i) {
        const double pv = PT[(long long)i * Mc + m];
#pragma unroll
        for (int n = 0; n < R8; ++n)
          if (n < N) s[n] += pv * A[(long long)n * a.Kmax + i];
      }
#pragma unroll
      for (int n = 0; n < R8; ++n)
        if (n < N) G[(long long)m * R8 + n] = s[n];
    }
    if (t < N * N) {
      const int n1 = t / N, n2 = t % N;
      double s = 0.0;
      for (int i = 0; i < K; ++i) s += A[(long long)n1 * a.Kmax + i] * A[(long long)n2 * a.Kmax + i];
      gram[n1 * R8 + n2] = s;
    }
    __syncthreads();
    for (int n = 0; n < N; ++n) {
      const double d = gram[n * R8 + n];
      if (d > 0.0) {
        for (int m = t; m < Mc; m += NT) {
          double s = 0.0;
          for (int n2 = 0; n2 < N; ++n2) s += F[(long long)m * R8 + n2] * gram[n2 * R8 + n];
          const long long fi = (long long)m * R8 + n;
          F[fi] = fmax(0.0, F[fi] + (G[fi] - s) / d);
        }
      }
      __syncthreads();
    }
  }

  // scale footprints to peak 1
  for (int n = 0; n < N; ++n) {
    double mx = 0.0;
    for (int m = t; m < Mc; m += NT) mx = fmax(mx, F[(long long)m * R8 + n]);
    double best;
    int dummy;
    block_argmax(mx, 0, sv, si, &best, &dummy);
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
