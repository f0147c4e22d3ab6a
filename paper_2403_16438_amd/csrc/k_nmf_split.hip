// Per-component NMF P_c ~ F A (Eq. 3, Sec. III-D) with each component split
// over several workgroups that run at the same time (cooperative launch).
//
// Workgroup w of component c owns a contiguous range of the component's
// pixels (rows of P_c) and keeps those rows of P_c in LDS (FP32, exact) for
// the whole factorisation, with an odd row stride so that both the row-wise
// and the column-wise sweeps are free of bank conflicts. Everything that needs
// all pixels of the component is a sum (or max) over pixels, so each
// workgroup writes its partial over its own rows to an exchange slot in HBM,
// the component's workgroups meet at a barrier, and each one adds the slots
// of all workgroups in the same fixed order. They thus hold bit-identical
// totals and take identical decisions without further communication:
//   SPA     per step: partial squared column norms of the residual, then the
//           partial projections onto the picked direction (two exchanges);
//           the residual rows stay with their owner (HBM, owner-only)
//   init    partial maxima of the picked columns (one exchange)
//   HALS    per sweep one exchange of the partial F^T F and F^T P; every
//           workgroup then runs the same A update (A is small and is kept
//           whole in each workgroup's LDS), forms A A^T itself and updates
//           the F rows it owns from its LDS rows of P_c
//   scale   partial column maxima of F (one exchange)
// The arithmetic is the single-workgroup kernel's (same update order, FP64,
// clipping, zero-Gram rule); only the summation order over pixels differs.
//
// Barrier: a per-component arrival counter (agent-scope release/acquire).
// The launch is cooperative, so all workgroups are resident; the wait is
// still bounded by a wall-clock limit, after which the component is marked
// abandoned, every workgroup of it leaves, and the error flag is set.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "seg_kernels.h"

namespace seg {
namespace {

constexpr int CT = 1024;
constexpr int CW = CT / 64;   // 16 waves
constexpr int CV = CT - 64;   // waves 0..14 of the HALS product phases (wave 15: Gram)
constexpr int R8 = kMaxRank;

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// pair k of the upper triangle of an NR x NR matrix, row by row
template <int NR>
__device__ __forceinline__ void pair_of(int k, int& n1, int& n2) {
  n1 = 0;
  while (k >= NR - n1) {
    k -= NR - n1;
    ++n1;
  }
  n2 = n1 + k;
}

// Gram matrix X^T X of the first NR columns of X [len][R8] (LDS), by the 64
// lanes of one wave: lane (chunk q, column n1) of QG = 64 / NR row chunks
// sums its chunk for all n2 into part[(q NR + n1) R8 + n2] ...
template <int NR>
__device__ __forceinline__ void gram_part(const double* X, int len, int lane, double* part) {
  constexpr int QG = 64 / NR;
  if (lane >= QG * NR) return;
  const int q = lane / NR, n1 = lane - q * NR;
  const int span = (len + QG - 1) / QG, j1 = min(len, (q + 1) * span);
  double s0[NR], s1[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n) s0[n] = s1[n] = 0.0;
  int j = q * span;
  for (; j + 1 < j1; j += 2) {
    const double x0 = X[j * R8 + n1], x1 = X[(j + 1) * R8 + n1];
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      s0[n] = fma(x0, X[j * R8 + n], s0[n]);
      s1[n] = fma(x1, X[(j + 1) * R8 + n], s1[n]);
    }
  }
  if (j < j1) {
    const double x0 = X[j * R8 + n1];
#pragma unroll
    for (int n = 0; n < NR; ++n) s0[n] = fma(x0, X[j * R8 + n], s0[n]);
  }
#pragma unroll
  for (int n = 0; n < NR; ++n) part[(q * NR + n1) * R8 + n] = s0[n] + s1[n];
}

// ... and entry k = n1 NR + n2 of the total, all QG chunks added in order
// (chunks past the data hold zeros); the bound is a constant, so the loads
// are issued ahead of the dependent adds
template <int NR>
__device__ __forceinline__ double gram_total(int k, const double* part) {
  constexpr int QG = 64 / NR;
  const int n1 = k / NR, n2 = k - n1 * NR;
  double v = part[n1 * R8 + n2];
#pragma unroll 8
  for (int q = 1; q < QG; ++q) v += part[(q * NR + n1) * R8 + n2];
  return v;
}

// in-order sum x[0] + x[step] + ... + x[(n - 1) step], n <= 16, loads issued
// in groups of four ahead of the adds
__device__ __forceinline__ double chunk_sum(const double* x, size_t step, int n) {
  double v = x[0];
  int q = 1;
  for (; q + 3 < n; q += 4) {
    const double a = x[q * step], b = x[(q + 1) * step], c = x[(q + 2) * step], d = x[(q + 3) * step];
    v += a;
    v += b;
    v += c;
    v += d;
  }
  for (; q < n; ++q) v += x[q * step];
  return v;
}

__device__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if (lane == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
  for (int ww = 1; ww < CW; ++ww) m = fmax(m, red[ww]);
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
  for (int ww = 1; ww < CW; ++ww)
    if (red[ww] > b || (red[ww] == b && redi[ww] < bi)) {
      b = red[ww];
      bi = redi[ww];
    }
  *best = b;
  *bidx = bi;
  __syncthreads();
}

// Slot writes are agent-scope stores: they go through to the level where all
// XCDs see them, so the release at the meeting finds no dirty slot lines to
// write back from the L2.
__device__ __forceinline__ void put(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// All workgroups of one component meet here; `target` is the number of
// arrivals that completes this meeting. Returns false when the component was
// abandoned (time limit), uniformly for the whole workgroup.
__device__ bool meet(unsigned* arrivals, unsigned* abandoned, unsigned* error, unsigned target,
                     long long limit, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    // release the workgroup's slot writes, arrive, poll without acquiring
    // (an acquire per poll would invalidate the caches every time), then
    // acquire once
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abandoned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = 0;
        break;
      }
      if (wall_clock64() - t0 > limit) {
        __hip_atomic_store(abandoned, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = ok;
  }
  __syncthreads();
  return *flag != 0;
}

__global__ __launch_bounds__(CT) void k_nmf_split(NmfArgs a, NmfSplit s) {
  extern __shared__ double dyn[];
  __shared__ double red[CW];
  __shared__ int redi[CW];
  __shared__ double gF[R8 * R8], gA[R8 * R8];
  __shared__ double gpart[64 * R8];   // Gram chunk sums (64 lanes x R8)
  __shared__ int picks[R8];
  __shared__ int flag;
  const int g = blockIdx.x, t = threadIdx.x;
  const int c = s.wg_comp[g];
  const int w0 = s.wg_base[c], nw = s.wg_n[c], r = g - w0;
  const int off = a.coff[c], Mc = a.coff[c + 1] - off;
  const int mw = s.mw, lo = r * mw, ml = min(mw, Mc - lo);  // own rows [lo, lo + ml)
  const int K = a.K, Kp = s.Kp;
  // LDS: A [K][R8], F [mw][R8], P A^T [mw][R8], scratch [scr], P rows [mw][Kp] (float)
  double* A = dyn;
  double* F = A + (size_t)K * R8;
  double* GP = F + (size_t)mw * R8;
  double* scr = GP + (size_t)mw * R8;
  float* Pl = reinterpret_cast<float*>(scr + s.scr);
  double* R = a.R + (long long)(off + lo) * K;  // own residual rows [ml][K], HBM
  unsigned* arrivals = s.sync + c;
  unsigned* abandoned = s.sync + a.ncomp + c;
  unsigned* error = s.sync + 2 * a.ncomp;
  unsigned ex = 0;  // exchanges done
  auto slot = [&](int w, unsigned e) { return s.xbuf + ((size_t)(w0 + w) * 2 + (e & 1)) * s.XS; };
  // sum (or max) of element j over the component's slots of exchange e, in
  // slot order; sixteen loads are in flight at a time
  auto gather = [&](size_t j, unsigned e, bool take_max) {
    double v = 0.0;
    for (int wb = 0; wb < nw; wb += 16) {
      double x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = wb + q < nw ? slot(wb + q, e)[j] : 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (wb + q < nw) v = take_max ? fmax(v, x[q]) : v + x[q];
    }
    return v;
  };
  // two elements at once, twelve slots per round of memory latency
  auto gather2 = [&](size_t j0, size_t j1, unsigned e, double& v0, double& v1) {
    v0 = 0.0;
    v1 = 0.0;
    for (int wb = 0; wb < nw; wb += 12) {
      double x[12], y[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        const double* sp = slot(wb + q, e);
        x[q] = wb + q < nw ? sp[j0] : 0.0;
        y[q] = wb + q < nw ? sp[j1] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 12; ++q)
        if (wb + q < nw) {
          v0 += x[q];
          v1 += y[q];
        }
    }
  };
#define MEET() \
  if (!meet(arrivals, abandoned, error, (ex + 1) * (unsigned)nw, s.limit, &flag)) return

  // gather own rows: consecutive threads read consecutive pixels of a plane
  for (int e = t; e < ml * K; e += CT) {
    const int i = e / ml, m = e - i * ml;
    Pl[m * Kp + i] = a.p[(long long)i * a.M + a.pix[off + lo + m]];
  }
  __syncthreads();
  for (int e = t; e < ml * K; e += CT) {
    const int m = e / K, i = e - m * K;
    R[e] = (double)Pl[m * Kp + i];
  }
  __syncthreads();

  // ---------------------------------------------------------------- SPA
  double* vec = scr;      // [K] projections
  double* U = scr + K;    // [mw] own entries of the picked direction
  double* nz = A;         // [K] nonzero-column flags (A is free until HALS)
  int N = 0;
  double ref = 0.0;
  while (N < a.max_rank) {
    {
      double* xs = slot(r, ex);
      for (int i = t; i < K; i += CT) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int m = 0;
        for (; m + 4 <= ml; m += 4) {
          const double r0 = R[(long long)m * K + i], r1 = R[(long long)(m + 1) * K + i];
          const double r2 = R[(long long)(m + 2) * K + i], r3 = R[(long long)(m + 3) * K + i];
          s0 += r0 * r0;
          s1 += r1 * r1;
          s2 += r2 * r2;
          s3 += r3 * r3;
        }
        for (; m < ml; ++m) {
          const double v = R[(long long)m * K + i];
          s0 += v * v;
        }
        put(xs + i, (s0 + s1) + (s2 + s3));
      }
    }
    MEET();
    double bv = -1.0;
    int bi = INT_MAX;
    for (int i = t; i < K; i += CT) {
      const double sq = gather(i, ex, false);
      if (N == 0) nz[i] = sq > 0.0 ? 1.0 : 0.0;  // the residual is still P (>= 0)
      const double nv = nz[i] > 0.0 ? sqrt(sq) : -1.0;
      if (nv > bv) {
        bv = nv;
        bi = i;
      }
    }
    ++ex;
    double best;
    int j;
    block_argmax(bv, bi, red, redi, &best, &j);
    if (best <= 0.0) break;
    if (N == 0) ref = best;
    else if (best < a.delta * ref) break;
    if (t == 0) picks[N] = j;
    ++N;
    for (int m = t; m < ml; m += CT) U[m] = R[(long long)m * K + j] / best;
    __syncthreads();
    {
      double* xs = slot(r, ex);
      for (int i = t; i < K; i += CT) {
        double s0 = 0.0, s1 = 0.0;
        int m = 0;
        for (; m + 2 <= ml; m += 2) {
          s0 += U[m] * R[(long long)m * K + i];
          s1 += U[m + 1] * R[(long long)(m + 1) * K + i];
        }
        if (m < ml) s0 += U[m] * R[(long long)m * K + i];
        put(xs + i, s0 + s1);
      }
    }
    MEET();
    for (int i = t; i < K; i += CT) {
      vec[i] = gather(i, ex, false);
    }
    ++ex;
    __syncthreads();
    for (int e = t; e < ml * K; e += CT) {
      const int m = e / K, i = e - m * K;
      R[e] -= U[m] * vec[i];
    }
    __syncthreads();
  }
  __syncthreads();

  if (N > 0) {
    // ---------------------------------------------- initial footprints
    {
      double* xs = slot(r, ex);
      for (int n = 0; n < N; ++n) {
        const int col = picks[n];
        double mx = 0.0;
        for (int m = t; m < ml; m += CT) mx = fmax(mx, (double)Pl[m * Kp + col]);
        mx = block_max(mx, red);
        if (t == 0) put(xs + n, mx);
      }
    }
    MEET();
    for (int m = t; m < ml; m += CT)
      for (int n = 0; n < R8; ++n) {
        double v = 0.0;
        if (n < N) {
          v = (double)Pl[m * Kp + picks[n]] / gather(n, ex, true);
        }
        F[m * R8 + n] = v;
      }
    ++ex;
    for (int e = t; e < K * R8; e += CT) A[e] = 0.0;
    __syncthreads();

    // HALS, compiled per rank so that the sequential row/column updates run
    // without predication
    auto hals = [&](auto rank) -> bool {
      constexpr int NR = decltype(rank)::value;
      constexpr int NP = NR * (NR + 1) / 2;
      double* FtP = scr;                    // [NR][K] totals (after the meeting)
      for (int sweep = -1; sweep < a.sweeps; ++sweep) {
        // ---- partial F^T P and F^T F over own rows (FP64, fixed order),
        // written to this workgroup's slot. Waves 0..14: thread (row chunk
        // q, segment i) sums its rows for all NR columns of F. Wave 15: F^T
        // F, lane (row chunk q, column n1). Chunks are then added in order.
        double* xs = slot(r, ex);
        {
          const int QC = max(1, min(min(CV / K, 8), s.scr / (K * NR)));
          const int rows = (ml + QC - 1) / QC;
          if (t < CV) {
            for (int e = t; e < QC * K; e += CV) {
              const int q = e / K, i = e - q * K;
              const int m1 = min(ml, (q + 1) * rows);
              double s0[NR], s1[NR];
#pragma unroll
              for (int n = 0; n < NR; ++n) s0[n] = s1[n] = 0.0;
              int m = q * rows;
              for (; m + 1 < m1; m += 2) {
                const double p0 = (double)Pl[m * Kp + i], p1 = (double)Pl[(m + 1) * Kp + i];
#pragma unroll
                for (int n = 0; n < NR; ++n) {
                  s0[n] = fma(F[m * R8 + n], p0, s0[n]);
                  s1[n] = fma(F[(m + 1) * R8 + n], p1, s1[n]);
                }
              }
              if (m < m1) {
                const double p0 = (double)Pl[m * Kp + i];
#pragma unroll
                for (int n = 0; n < NR; ++n) s0[n] = fma(F[m * R8 + n], p0, s0[n]);
              }
#pragma unroll
              for (int n = 0; n < NR; ++n) {
                if (QC == 1) put(xs + n * K + i, s0[n] + s1[n]);
                else scr[(size_t)e * NR + n] = s0[n] + s1[n];
              }
            }
          } else {
            gram_part<NR>(F, ml, t - CV, gpart);
          }
          __syncthreads();
          if (QC > 1)
            for (int o = t; o < NR * K; o += CT) {
              const int n = o / K, i = o - n * K;
              put(xs + o, chunk_sum(scr + (size_t)i * NR + n, (size_t)K * NR, QC));
            }
          if (t < NR * NR) put(xs + R8 * K + (t / NR) * R8 + t % NR, gram_total<NR>(t, gpart));
        }
        if (!meet(arrivals, abandoned, error, (ex + 1) * (unsigned)nw, s.limit, &flag)) return false;
        // ---- totals over the component's workgroups (slot order) into LDS
        if (t < NP) {   // upper triangle, mirrored
          int n1, n2;
          pair_of<NR>(t, n1, n2);
          const double v = gather(R8 * K + n1 * R8 + n2, ex, false);
          gF[n1 * R8 + n2] = v;
          gF[n2 * R8 + n1] = v;
        }
        for (int e = t; e < NR * K; e += 2 * CT) {
          if (e + CT < NR * K) {
            double v0, v1;
            gather2(e, e + CT, ex, v0, v1);
            FtP[e] = v0;
            FtP[e + CT] = v1;
          } else {
            FtP[e] = gather(e, ex, false);
          }
        }
        ++ex;
        __syncthreads();
        // ---- the A update (rows of A in order), every workgroup alike
        for (int i = t; i < K; i += CT) {
          double av[NR];
#pragma unroll
          for (int n = 0; n < NR; ++n) av[n] = A[i * R8 + n];
#pragma unroll
          for (int n = 0; n < NR; ++n) {
            // from rank 6 on, hoisting all Gram reads would spill: keep them per row
            if constexpr (NR > 5) asm volatile("" ::: "memory");
            const double d = gF[n * R8 + n];
            if (d > 0.0) {
              double sg = 0.0;
#pragma unroll
              for (int n2 = 0; n2 < NR; ++n2) sg += gF[n * R8 + n2] * av[n2];
              av[n] = fmax(0.0, av[n] + (FtP[n * K + i] - sg) / d);
            }
          }
#pragma unroll
          for (int n = 0; n < NR; ++n) A[i * R8 + n] = av[n];
        }
        __syncthreads();
        if (sweep < 0) continue;
        // ---- P A^T of own rows and A A^T (FP64, fixed order). Waves
        // 0..14: thread (segment chunk q, own row m) sums its segments for
        // all NR rows of A. Wave 15: A A^T, lane (segment chunk q, row n1),
        // chunked by K and NR only, so identical in every workgroup. Chunks
        // are then added in order.
        {
          // at most 16 chunks: their in-order sum is a chain of dependent adds
          const int QK = max(1, min(min(CV / ml, 16), s.scr / (ml * NR)));
          const int seg = (K + QK - 1) / QK;
          if (t < CV) {
            for (int e = t; e < QK * ml; e += CV) {
              const int q = e / ml, m = e - q * ml;
              const int i1 = min(K, (q + 1) * seg);
              double s0[NR], s1[NR];
#pragma unroll
              for (int n = 0; n < NR; ++n) s0[n] = s1[n] = 0.0;
              int i = q * seg;
              for (; i + 1 < i1; i += 2) {
                const double p0 = (double)Pl[m * Kp + i], p1 = (double)Pl[m * Kp + i + 1];
#pragma unroll
                for (int n = 0; n < NR; ++n) {
                  s0[n] = fma(p0, A[i * R8 + n], s0[n]);
                  s1[n] = fma(p1, A[(i + 1) * R8 + n], s1[n]);
                }
              }
              if (i < i1) {
                const double p0 = (double)Pl[m * Kp + i];
#pragma unroll
                for (int n = 0; n < NR; ++n) s0[n] = fma(p0, A[i * R8 + n], s0[n]);
              }
#pragma unroll
              for (int n = 0; n < NR; ++n) scr[(size_t)e * NR + n] = s0[n] + s1[n];
            }
          } else {
            gram_part<NR>(A, K, t - CV, gpart);
          }
          __syncthreads();
          for (int e = t; e < ml * NR; e += CT) {   // P A^T: chunks in order
            GP[e] = chunk_sum(scr + e, (size_t)ml * NR, QK);
          }
          if (t < NR * NR) gA[(t / NR) * R8 + t % NR] = gram_total<NR>(t, gpart);
          __syncthreads();
        }
        // ---- the own F rows (columns of F in order)
        for (int m = t; m < ml; m += CT) {
          double gp[NR], f[NR];
#pragma unroll
          for (int n = 0; n < NR; ++n) {
            gp[n] = GP[m * NR + n];
            f[n] = F[m * R8 + n];
          }
#pragma unroll
          for (int n = 0; n < NR; ++n) {
            if constexpr (NR > 5) asm volatile("" ::: "memory");
            const double d = gA[n * R8 + n];
            if (d > 0.0) {
              double sg = 0.0;
#pragma unroll
              for (int n2 = 0; n2 < NR; ++n2) sg += f[n2] * gA[n2 * R8 + n];
              f[n] = fmax(0.0, f[n] + (gp[n] - sg) / d);
            }
          }
#pragma unroll
          for (int n = 0; n < NR; ++n) F[m * R8 + n] = f[n];
        }
        __syncthreads();
      }
      return true;
    };
    bool ok = true;
    switch (N) {
      case 1: ok = hals(std::integral_constant<int, 1>{}); break;
      case 2: ok = hals(std::integral_constant<int, 2>{}); break;
      case 3: ok = hals(std::integral_constant<int, 3>{}); break;
      case 4: ok = hals(std::integral_constant<int, 4>{}); break;
      case 5: ok = hals(std::integral_constant<int, 5>{}); break;
      case 6: ok = hals(std::integral_constant<int, 6>{}); break;
      case 7: ok = hals(std::integral_constant<int, 7>{}); break;
      default: ok = hals(std::integral_constant<int, 8>{}); break;
    }
    if (!ok) return;

    // ------------------------------------------ scale to peak 1, export
    {
      double* xs = slot(r, ex);
      for (int n = 0; n < N; ++n) {
        double mx = 0.0;
        for (int m = t; m < ml; m += CT) mx = fmax(mx, F[m * R8 + n]);
        mx = block_max(mx, red);
        if (t == 0) put(xs + n, mx);
      }
    }
    MEET();
    double* Fg = a.F + (long long)(off + lo) * R8;
    double* Ag = a.A + (long long)c * R8 * a.Kmax;
    for (int n = 0; n < N; ++n) {
      const double mx = gather(n, ex, true);
      const double sc = mx > 0.0 ? mx : 1.0;
      for (int m = t; m < ml; m += CT) Fg[(long long)m * R8 + n] = F[m * R8 + n] / sc;
      if (r == 0)
        for (int i = t; i < K; i += CT) Ag[(long long)n * a.Kmax + i] = A[i * R8 + n] * sc;
    }
    ++ex;
  }
#undef MEET
  if (r == 0 && t == 0) a.N[c] = N;
}

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Dynamic LDS of one workgroup: A [K][R8], F and P A^T [mw][R8], scratch
// (F^T P totals, the twelve P A^T parts, or the SPA vectors), P rows [mw][Kp].
size_t split_lds(int K, int mw, int* scr_out) {
  const int Kp = K | 1;
  const size_t scr = std::max<size_t>({(size_t)R8 * K, (size_t)12 * 16 * R8, (size_t)K + mw});
  if (scr_out) *scr_out = (int)scr;
  return 8 * ((size_t)K * R8 + 2 * (size_t)mw * R8 + scr) + 4 * (size_t)mw * Kp;
}

}  // namespace

bool plan_nmf_split(NmfSplit& s, const NmfArgs& a, const std::vector<int>& coff, size_t xbuf_bytes,
                    NmfSplitTables& tab) {
  int dev = 0, coop = 0, ncu = 0, max_lds = 0, clock_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
    return false;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || clock_khz <= 0)
    return false;
  const size_t budget = max_lds > 16384 ? (size_t)max_lds - 12288 : 0;  // static LDS ~1.3 KB, with room to spare
  const int K = a.K;
  const int ncomp = a.ncomp;
  if (K < 1 || ncomp < 1) return false;
  const int XS = ((R8 * K + R8 * R8) + 31) / 32 * 32;
  // exchange slots: two per workgroup of the largest launch, in xbuf
  const size_t slot_bytes = (size_t)2 * XS * 8;
  // Slice widths in order of preference (measured: 96 rows balance the
  // per-sweep exchange against the per-workgroup work; at most twelve
  // 16-row tiles). Components are packed, in order, into launches of at most
  // one workgroup per compute unit; each launch costs about the same (its
  // sweeps are latency bound), so the width with the fewest launches wins.
  const int widths[] = {96, 128, 160, 192, 64, 32};
  int best_mw = 0, best_groups = 0;
  for (const int mw : widths) {
    int scr = 0;
    if (split_lds(K, mw, &scr) > budget) continue;
    int groups = 1, in_group = 0, widest = 0;
    bool fits = true;
    for (int k = 0; k < ncomp && fits; ++k) {
      const int nwk = (coff[k + 1] - coff[k] + mw - 1) / mw;
      if (nwk > ncu) fits = false;
      else if (in_group + nwk > ncu) {
        ++groups;
        in_group = nwk;
      } else {
        in_group += nwk;
      }
      widest = std::max(widest, in_group);
    }
    fits = fits && (size_t)widest * slot_bytes <= xbuf_bytes;
    if (fits && (best_mw == 0 || groups < best_groups)) {
      best_mw = mw;
      best_groups = groups;
    }
  }
  if (best_mw == 0) return false;
  const int mw = best_mw;
  int scr = 0;
  size_t lds = split_lds(K, mw, &scr);
  // spare LDS (up to 2 R8 K more doubles) widens the scratch of the HALS
  // products' chunk partials, so more chunks run at once at higher ranks
  const size_t more = std::min<size_t>((budget - lds) / 8, (size_t)2 * R8 * K);
  scr += (int)more;
  lds += 8 * more;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_nmf_split, CT, lds) != hipSuccess || occ < 1)
    return false;
  s.mw = mw;
  s.Kp = K | 1;
  s.scr = scr;
  s.XS = XS;
  s.lds_bytes = lds;
  s.limit = (long long)clock_khz * 1000LL * 2;  // two seconds of wall clock
  tab.comp.clear();
  tab.base.assign((size_t)ncomp, 0);
  tab.n.assign((size_t)ncomp, 0);
  tab.groups.clear();
  int start = 0, in_group = 0;
  for (int k = 0; k < ncomp; ++k) {
    const int nwk = (coff[k + 1] - coff[k] + mw - 1) / mw;
    if (in_group + nwk > ncu) {
      tab.groups.push_back({start, in_group});
      start += in_group;
      in_group = 0;
    }
    tab.base[k] = in_group;              // first workgroup within its launch
    tab.n[k] = nwk;
    for (int j = 0; j < nwk; ++j) tab.comp.push_back(k);
    in_group += nwk;
  }
  tab.groups.push_back({start, in_group});
  s.G = (int)tab.comp.size();
  return true;
}

hipError_t launch_nmf_split(const NmfArgs& a, const NmfSplit& s, bool first, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (first) {   // the counters and flags of every component, once per plan
    const int nsync = 2 * a.ncomp + 1;
    hipLaunchKernelGGL(k_fill_u32, dim3((nsync + 255) / 256), dim3(256), 0, st, s.sync, nsync, 0u);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_nmf_split),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)s.lds_bytes);
  if (e != hipSuccess) return e;
  NmfArgs aa = a;
  NmfSplit ss = s;
  void* args[] = {&aa, &ss};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_nmf_split), dim3(s.G), dim3(CT), args,
                                    (unsigned)s.lds_bytes, st);
}

}  // namespace seg
