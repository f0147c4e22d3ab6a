// Per-component NMF P_c ~ F A (Eq. 3, Sec. III-D) with each component split
// over several workgroups that run at the same time (cooperative launch).
//
// Workgroup w of component c owns a contiguous range of the component's
// pixels (rows of P_c) and keeps those rows of P_c in LDS (FP32, exact) for
// the whole factorisation, with an odd row stride so that both the row-wise
// and the column-wise sweeps are free of bank conflicts. Everything that needs
// all pixels of the component is a sum (or max) over pixels, so each
// workgroup writes its partial over its own rows to an exchange slot in HBM,
// and each workgroup of the component waits for and adds the slots of all of
// them in the same fixed order. They thus hold bit-identical
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
// clipping, zero-Gram rule); only the summation order of the sums differs.
// A sweep has five workgroup barriers: after the F^T P partials, after the
// gather, after the A update, after the P A^T partials and after the F
// update; the Gram matrices are formed within one wave, which needs none.
//
// Exchange: every slot value travels as two 64-bit words (its high and low
// halves), each tagged in its upper 32 bits with the number of the exchange
// that wrote it, and written and read with relaxed agent-scope atomics. A
// word read with the expected tag therefore holds that exchange's half
// (single-copy atomicity of the word), so readers poll the slot words
// themselves: no arrival counter, no fences, and the values are exact. Two
// slots per workgroup alternate between exchanges; a workgroup can only
// overwrite a slot after every workgroup of its component has read it (it
// needs their next slots first), and the slots are cleared before each
// launch, so a stale word never carries the expected tag. The launch is
// cooperative, so all workgroups are resident; a wait is still bounded by a
// wall-clock limit, after which the component is marked abandoned, every
// workgroup of it leaves, and the error flag is set.
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

// X^T X of the first NR columns of X [len][R8] (LDS) by the 64 lanes of one
// wave: lane (chunk q, entry p of the upper triangle) sums its chunk of rows
// for entry p, the QG chunk partials go to part [QG][NP] (LDS), and lane p < NP
// adds the partials of entry p in chunk order. Returns that total in lanes
// p < NP (0 elsewhere). The wave needs no barrier: the LDS requests of a wave
// complete in order.
template <int NR>
__device__ __forceinline__ double gram_wave(const double* X, int len, int lane, double* part) {
  constexpr int NP = NR * (NR + 1) / 2;
  constexpr int QG = NP <= 4 ? 16 : NP <= 8 ? 8 : NP <= 16 ? 4 : NP <= 32 ? 2 : 1;
  if (lane < QG * NP) {
    const int q = lane / NP, p = lane - q * NP;
    int n1, n2;
    pair_of<NR>(p, n1, n2);
    const int span = (len + QG - 1) / QG, j1 = min(len, (q + 1) * span);
    double g0 = 0.0, g1 = 0.0;
    int j = q * span;
    for (; j + 1 < j1; j += 2) {
      g0 = fma(X[j * R8 + n1], X[j * R8 + n2], g0);
      g1 = fma(X[(j + 1) * R8 + n1], X[(j + 1) * R8 + n2], g1);
    }
    if (j < j1) g0 = fma(X[j * R8 + n1], X[j * R8 + n2], g0);
    part[q * NP + p] = g0 + g1;
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  double v = 0.0;
  if (lane < NP) {
    double x[QG];
#pragma unroll
    for (int q = 0; q < QG; ++q) x[q] = part[q * NP + lane];
    v = x[0];
#pragma unroll
    for (int q = 1; q < QG; ++q) v += x[q];
  }
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

using u64 = unsigned long long;

__device__ __forceinline__ void put_word(u64* p, unsigned tag, unsigned half) {
  __hip_atomic_store(p, ((u64)tag << 32) | half, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ u64 get_word(u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The same word read through this XCD's L2 (workgroup scope: past the L1,
// not past the L2). The planner places a component's workgroups on one XCD
// where it can, so a slot written there (the agent-scope store passes
// through that L2) is seen at L2 latency; a word written on another XCD may
// sit stale in this L2, so the waits below also read with agent scope every
// fourth poll. The tags make a stale word harmless: it is only waited on.
__device__ __forceinline__ u64 get_word_near(u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ bool tagged(u64 w, unsigned tag) { return (unsigned)(w >> 32) == tag; }

// Waits until both halves at p and p + xs carry `tag` and returns them;
// ok is false when the component was abandoned or the wall-clock limit
// passed (then it marks the component abandoned and sets the error flag).
struct Halves {
  u64 hi, lo;
  bool ok;
};
__device__ __forceinline__ Halves wait_words(u64* p, int xs, unsigned tag, unsigned* abandoned,
                                             unsigned* error, long long limit) {
  const long long t0 = wall_clock64();
  for (unsigned n = 0;; ++n) {
    __builtin_amdgcn_s_sleep(2);
    const bool far = (n & 3) == 3;
    const u64 hi = far ? get_word(p) : get_word_near(p), lo = far ? get_word(p + xs) : get_word_near(p + xs);
    if (tagged(hi, tag) && tagged(lo, tag)) return {hi, lo, true};
    if ((n & 15) == 15 && __hip_atomic_load(abandoned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return {0, 0, false};
    if (wall_clock64() - t0 > limit) {
      __hip_atomic_store(abandoned, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return {0, 0, false};
    }
  }
}

__global__ __launch_bounds__(CT) void k_nmf_split(NmfArgs a, NmfSplit s) {
  extern __shared__ double dyn[];
  __shared__ double red[CW];
  __shared__ int redi[CW];
  __shared__ double gF[R8 * R8], gA[R8 * R8];
  __shared__ double gpart[64 * R8];   // Gram chunk sums (64 lanes x R8)
  __shared__ int picks[R8];
  __shared__ int bad;
  const int g = blockIdx.x, t = threadIdx.x;
  const int c = s.wg_comp[g];
  const int w0 = s.wg_base[c], nw = s.wg_n[c], r = s.wg_rank[g];
  const int off = a.coff[c], Mc = a.coff[c + 1] - off;
  const int mw = s.mw, lo = r * mw, ml = min(mw, Mc - lo);  // own rows [lo, lo + ml)
  const int K = a.K, Kp = s.Kp, XS = s.XS;
  // LDS: A [K][R8], F [mw][R8], F^T P totals [R8][K], scratch [scr], P rows [mw][Kp] (float)
  double* A = dyn;
  double* F = A + (size_t)K * R8;
  double* FtP = F + (size_t)mw * R8;
  double* scr = FtP + (size_t)R8 * K;
  float* Pl = reinterpret_cast<float*>(scr + s.scr);
  double* R = a.R + (long long)(off + lo) * K;  // own residual rows [ml][K], HBM
  unsigned* abandoned = s.sync + c;
  unsigned* error = s.sync + a.ncomp;
  unsigned ex = 0;  // exchanges done
  bool dead = false;  // this thread gave up waiting (the workgroup leaves at the next check)
  if (t == 0) bad = 0;
  // slot of workgroup w for exchange e: XS high words, then XS low words
  auto slot = [&](int w, unsigned e) { return s.xbuf + ((size_t)(w0 + w) * 2 + (e & 1)) * 2 * XS; };
  // element j of this workgroup's slot for exchange e
  auto put = [&](unsigned e, size_t j, double v) {
    u64* p = slot(r, e) + j;
    const u64 b = (u64)__double_as_longlong(v);
    put_word(p, e + 1, (unsigned)(b >> 32));
    put_word(p + XS, e + 1, (unsigned)b);
  };
  // sum (or max) of element j over the component's slots of exchange e, in
  // slot order, waiting for each slot's words; twelve slots per round of
  // memory latency
  auto gather = [&](size_t j, unsigned e, bool take_max) {
    const unsigned tag = e + 1;
    double v = 0.0;
    if (dead) return v;
    for (int wb = 0; wb < nw; wb += 12) {
      u64 hi[12], lw[12];
      // all 24 loads go out before the first use (slots past the last are
      // read as the last one and not used)
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        u64* p = slot(min(wb + q, nw - 1), e) + j;
        hi[q] = get_word_near(p);
        lw[q] = get_word_near(p + XS);
      }
      asm volatile("" : "+v"(hi[0]), "+v"(hi[1]), "+v"(hi[2]), "+v"(hi[3]), "+v"(hi[4]), "+v"(hi[5]),
                        "+v"(hi[6]), "+v"(hi[7]), "+v"(hi[8]), "+v"(hi[9]), "+v"(hi[10]), "+v"(hi[11]),
                        "+v"(lw[0]), "+v"(lw[1]), "+v"(lw[2]), "+v"(lw[3]), "+v"(lw[4]), "+v"(lw[5]),
                        "+v"(lw[6]), "+v"(lw[7]), "+v"(lw[8]), "+v"(lw[9]), "+v"(lw[10]), "+v"(lw[11]));
#pragma unroll
      for (int q = 0; q < 12; ++q)
        if (wb + q < nw) {
          if (!tagged(hi[q], tag) || !tagged(lw[q], tag)) {
            const Halves h = dead ? Halves{0, 0, false}
                                  : wait_words(slot(wb + q, e) + j, XS, tag, abandoned, error, s.limit);
            if (!h.ok) {
              dead = true;
              bad = 1;
              return 0.0;
            }
            hi[q] = h.hi;
            lw[q] = h.lo;
          }
          const double x = __longlong_as_double((long long)((hi[q] << 32) | (lw[q] & 0xffffffffull)));
          v = take_max ? fmax(v, x) : v + x;
        }
    }
    return v;
  };
  __syncthreads();
// leave when any thread of the workgroup gave up waiting (read after a barrier)
#define LEAVE_IF_ABANDONED(ret) \
  __syncthreads();              \
  if (bad) return ret

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
    for (int i = t; i < K; i += CT) {
      {
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
        put(ex, i, (s0 + s1) + (s2 + s3));
      }
    }
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
    LEAVE_IF_ABANDONED();
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
    for (int i = t; i < K; i += CT) {
      {
        double s0 = 0.0, s1 = 0.0;
        int m = 0;
        for (; m + 2 <= ml; m += 2) {
          s0 += U[m] * R[(long long)m * K + i];
          s1 += U[m + 1] * R[(long long)(m + 1) * K + i];
        }
        if (m < ml) s0 += U[m] * R[(long long)m * K + i];
        put(ex, i, s0 + s1);
      }
    }
    for (int i = t; i < K; i += CT) {
      vec[i] = gather(i, ex, false);
    }
    ++ex;
    LEAVE_IF_ABANDONED();
    for (int e = t; e < ml * K; e += CT) {
      const int m = e / K, i = e - m * K;
      R[e] -= U[m] * vec[i];
    }
    __syncthreads();
  }
  __syncthreads();

  if (N > 0) {
    // ---------------------------------------------- initial footprints
    for (int n = 0; n < N; ++n) {
      const int col = picks[n];
      double mx = 0.0;
      for (int m = t; m < ml; m += CT) mx = fmax(mx, (double)Pl[m * Kp + col]);
      mx = block_max(mx, red);
      if (t == 0) put(ex, n, mx);
    }
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
    LEAVE_IF_ABANDONED();

    // HALS, compiled per rank so that the sequential row/column updates run
    // without predication
    auto hals = [&](auto rank) -> bool {
      constexpr int NR = decltype(rank)::value;
      constexpr int NP = NR * (NR + 1) / 2;
      for (int sweep = -1; sweep < a.sweeps; ++sweep) {
        // ---- partial F^T P and F^T F over own rows (FP64, fixed order),
        // written to this workgroup's slot. Waves 0..14: thread (row chunk
        // q, segment i) sums its rows for all NR columns of F; after the
        // barrier the chunks are added in order and written to the slot,
        // and the gather of the totals follows without another barrier.
        // Wave 15: F^T F, whole within the wave (gram_wave), straight to the
        // slot.
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
                if (QC == 1) put(ex, (size_t)n * K + i, s0[n] + s1[n]);
                else scr[(size_t)e * NR + n] = s0[n] + s1[n];
              }
            }
          } else {   // F^T F of the own rows, upper triangle
            const double v = gram_wave<NR>(F, ml, t - CV, gpart);
            if (t - CV < NP) {
              int n1, n2;
              pair_of<NR>(t - CV, n1, n2);
              put(ex, (size_t)R8 * K + n1 * R8 + n2, v);
            }
          }
          __syncthreads();
          if (QC > 1)
            for (int o = t; o < NR * K; o += CT) {
              const int n = o / K, i = o - n * K;
              put(ex, o, chunk_sum(scr + (size_t)i * NR + n, (size_t)K * NR, QC));
            }
        }
        // ---- totals over the component's workgroups (slot order) into LDS:
        // the NR K entries of F^T P, then the upper triangle of F^T F (mirrored)
        for (int e = t; e < NR * K + NP; e += CT) {
          if (e < NR * K) {
            FtP[e] = gather(e, ex, false);
          } else {
            int n1, n2;
            pair_of<NR>(e - NR * K, n1, n2);
            const double v = gather((size_t)R8 * K + n1 * R8 + n2, ex, false);
            gF[n1 * R8 + n2] = v;
            gF[n2 * R8 + n1] = v;
          }
        }
        ++ex;
        LEAVE_IF_ABANDONED(false);
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
        // all NR rows of A. Wave 15: A A^T whole within the wave, chunked by
        // K and NR only, so identical in every workgroup.
        // at most 16 chunks: their in-order sum is a chain of dependent adds
        const int QK = max(1, min(min(CV / ml, 16), s.scr / (ml * NR)));
        {
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
          } else {   // A A^T, upper triangle mirrored (every workgroup alike)
            const double v = gram_wave<NR>(A, K, t - CV, gpart);
            if (t - CV < NP) {
              int n1, n2;
              pair_of<NR>(t - CV, n1, n2);
              gA[n1 * R8 + n2] = v;
              gA[n2 * R8 + n1] = v;
            }
          }
          __syncthreads();
        }
        // ---- the own F rows (columns of F in order), each thread adding
        // its row's P A^T chunks in order first
        for (int m = t; m < ml; m += CT) {
          double gp[NR], f[NR];
#pragma unroll
          for (int n = 0; n < NR; ++n) {
            gp[n] = chunk_sum(scr + (size_t)m * NR + n, (size_t)ml * NR, QK);   // P A^T: chunks in order
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
    for (int n = 0; n < N; ++n) {
      double mx = 0.0;
      for (int m = t; m < ml; m += CT) mx = fmax(mx, F[m * R8 + n]);
      mx = block_max(mx, red);
      if (t == 0) put(ex, n, mx);
    }
    double* peak = scr;
    if (t < N) peak[t] = gather(t, ex, true);
    ++ex;
    LEAVE_IF_ABANDONED();
    double* Fg = a.F + (long long)(off + lo) * R8;
    double* Ag = a.A + (long long)c * R8 * a.Kmax;
    for (int n = 0; n < N; ++n) {
      const double sc = peak[n] > 0.0 ? peak[n] : 1.0;
      for (int m = t; m < ml; m += CT) Fg[(long long)m * R8 + n] = F[m * R8 + n] / sc;
      if (r == 0)
        for (int i = t; i < K; i += CT) Ag[(long long)n * a.Kmax + i] = A[i * R8 + n] * sc;
    }
  }
#undef LEAVE_IF_ABANDONED
  if (r == 0 && t == 0) a.N[c] = N;
}

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Dynamic LDS of one workgroup: A [K][R8], F and P A^T [mw][R8], scratch
// (F^T P totals, the chunk partials of the HALS products, the SPA vectors or
// the final column maxima), P rows [mw][Kp].
size_t split_lds(int K, int mw, int* scr_out) {
  const int Kp = K | 1;
  const size_t scr = std::max<size_t>({(size_t)12 * 16 * R8, (size_t)K + mw});
  if (scr_out) *scr_out = (int)scr;
  return 8 * ((size_t)K * R8 + (size_t)mw * R8 + (size_t)R8 * K + scr) + 4 * (size_t)mw * Kp;
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
  // exchange slots: two per workgroup of the largest launch, in xbuf, each
  // of XS high and XS low words
  const size_t slot_bytes = (size_t)2 * 2 * XS * 8;
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
  // spare LDS (up to 3 R8 K more doubles) widens the scratch of the HALS
  // products' chunk partials, so more chunks run at once at higher ranks
  const size_t more = std::min<size_t>((budget - lds) / 8, (size_t)3 * R8 * K);
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
  tab.rank.clear();
  tab.base.assign((size_t)ncomp, 0);
  tab.n.assign((size_t)ncomp, 0);
  tab.groups.clear();
  // components in order into launches; base[k] numbers a component's slots
  // within its launch
  std::vector<std::vector<int>> members(1);
  int start = 0, in_group = 0;
  for (int k = 0; k < ncomp; ++k) {
    const int nwk = (coff[k + 1] - coff[k] + mw - 1) / mw;
    if (in_group + nwk > ncu) {
      tab.groups.push_back({start, in_group});
      members.emplace_back();
      start += in_group;
      in_group = 0;
    }
    tab.base[k] = in_group;
    tab.n[k] = nwk;
    members.back().push_back(k);
    in_group += nwk;
  }
  tab.groups.push_back({start, in_group});
  // Workgroup g of a launch runs on XCD g mod 8 (the dispatcher deals
  // workgroups to the XCDs in turn). Each component gets workgroups of one
  // XCD where one has room (largest components first, into the XCD with the
  // most room), so its exchanges stay in that XCD's L2; the rest take what
  // is left.
  constexpr int NX = 8;
  tab.comp.assign((size_t)start + in_group, 0);
  tab.rank.assign((size_t)start + in_group, 0);
  for (size_t gi = 0; gi < tab.groups.size(); ++gi) {
    const int first = tab.groups[gi].first, G = tab.groups[gi].second;
    std::vector<std::vector<int>> free_g(NX);
    for (int g = G - 1; g >= 0; --g) free_g[g % NX].push_back(g);   // popped in increasing order
    std::vector<int> order = members[gi];
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tab.n[x] > tab.n[y]; });
    std::vector<int> spill;
    for (const int k : order) {
      int best = -1;
      for (int x = 0; x < NX; ++x)
        if ((int)free_g[x].size() >= tab.n[k] && (best < 0 || free_g[x].size() > free_g[best].size())) best = x;
      if (best < 0) {
        spill.push_back(k);
        continue;
      }
      for (int j = 0; j < tab.n[k]; ++j) {
        const int g = free_g[best].back();
        free_g[best].pop_back();
        tab.comp[first + g] = k;
        tab.rank[first + g] = j;
      }
    }
    for (const int k : spill)
      for (int j = 0, x = 0; j < tab.n[k]; ++j) {
        while (free_g[x].empty()) ++x;
        const int g = free_g[x].back();
        free_g[x].pop_back();
        tab.comp[first + g] = k;
        tab.rank[first + g] = j;
      }
  }
  s.G = (int)tab.comp.size();
  return true;
}

hipError_t launch_nmf_split(const NmfArgs& a, const NmfSplit& s, bool first, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (first) {   // the abandon flags of every component and the error flag, once per plan
    const int nsync = a.ncomp + 1;
    hipLaunchKernelGGL(k_fill_u32, dim3((nsync + 255) / 256), dim3(256), 0, st, s.sync, nsync, 0u);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {   // the slots of this launch carry no tag (tags start at 1)
    const long long words = (long long)s.G * 2 * 2 * s.XS * 2;   // 32-bit words
    if (words > INT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<unsigned*>(s.xbuf), (int)words, 0u);
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
