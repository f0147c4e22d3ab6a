// Footprint-reconstruction kernels before the NMF (Sec. III-D):
//   pointwise   noise scale sigma(x), mean image (Eq. 1 averaged), pooled
//               co-moments and the 8-neighbour correlation image
//   events      z_i = T_i / sigma, e_i = [z_i >= theta], p_i = max(0, z_i - theta),
//               event count per pixel (segment chunks on the grid's y axis,
//               integer atomics, so the count does not depend on the order)
//   regions     8-connected components of every e_i by union-find whose roots
//               are the minimum pixel index of each component; roots are
//               compacted into region ids; per region: area, first and second
//               moments, bounding box (integer atomics, order independent);
//               the keep decision tests area, eccentricity and solidity (convex
//               hull of the pixel-square corners, exact integer shoelace)
//   aggregate   b_i = kept regions, n_b = sum_i b_i, b = [n_b >= c_min],
//               components of b numbered 1..n by minimum raster index
#include <climits>

#include "seg_kernels.h"

// The region decisions repeat the reference arithmetic operation by operation
// in FP64; no multiply-add contraction anywhere in this file.
#pragma clang fp contract(off)

namespace seg {
namespace {

constexpr int BS = 256;        // threads per block
constexpr int PER = 4;         // elements per thread in the compaction scans
constexpr int CHUNK = BS * PER;

// Parent reads during the merge go to L2 (relaxed agent-scope atomic loads):
// other CUs lower parents concurrently and the L1 is not coherent.
__device__ __forceinline__ int ld_par(int* par, int x) {
  return __hip_atomic_load(&par[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int* par, int x) {
  int p = ld_par(par, x);
  while (p != x) {
    x = p;
    p = ld_par(par, x);
  }
  return x;
}

// Union by minimum index: the root of every tree is its smallest element, so
// after all unions each component's root is its minimum index.
__device__ void uf_unite(int* par, int a, int b) {
  while (true) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    const int hi = a > b ? a : b;
    const int lo = a > b ? b : a;
    const int old = atomicMin(&par[hi], lo);
    if (old == hi) return;
    a = old;
    b = lo;
  }
}

// ---------------------------------------------------------------- pointwise

__global__ void k_moments(FinalizeArgs a, double* __restrict__ C) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.M) return;
  const int yy = x / a.W, xx = x - yy * a.W;
  const int dy[5] = {0, 0, 1, 1, 1};
  const int dx[5] = {0, 1, 0, 1, -1};
  for (int o = 0; o < 5; ++o) {
    const int ny = yy + dy[o], nx = xx + dx[o];
    double acc = 0.0;
    if (a.have_moments && ny < a.H && nx >= 0 && nx < a.W) {
      const int y = ny * a.W + nx;
      // unrolled so that several segments' loads are in flight; the sum
      // still runs in segment order
#pragma unroll 8
      for (int i = 0; i < a.K; ++i) {
        const long long b = (long long)i * a.M;
        acc += (double)a.P[o * a.plane + b + x] -
               (double)a.U[b + x] * (double)a.U[b + y] / (double)kSegLen;
      }
    }
    C[(long long)o * a.M + x] = acc;
  }
}

__global__ void k_pointwise(FinalizeArgs a, const double* __restrict__ C) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.M) return;
  double sd = 0.0, ss = 0.0;
#pragma unroll 8
  for (int i = 0; i < a.K; ++i) {
    sd += (double)a.D[(long long)i * a.M + x];
    ss += (double)a.S[(long long)i * a.M + x];
  }
  a.sigma[x] = sqrt(2.0 * 3.14159265358979323846) * sd / (double)a.K;
  a.mean[x] = (float)(ss / (double)a.K);
  a.count[x] = 0;   // accumulated by k_events
  a.nb[x] = 0;      // accumulated by k_kept
  // correlation image: mean of rho over in-frame 8-neighbours
  const int yy = x / a.W, xx = x - yy * a.W;
  const int dy[4] = {0, 1, 1, 1};
  const int dx[4] = {1, 0, 1, -1};
  const double vx = C[x];
  double acc = 0.0;
  int cnt = 0;
  for (int o = 0; o < 4; ++o) {
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      const int ny = yy + sgn * dy[o], nx = xx + sgn * dx[o];
      if (ny < 0 || ny >= a.H || nx < 0 || nx >= a.W) continue;
      const int y = ny * a.W + nx;
      const double cov = sgn > 0 ? C[(long long)(o + 1) * a.M + x] : C[(long long)(o + 1) * a.M + y];
      const double d = vx * C[y];
      acc += d > 0.0 ? cov / sqrt(d) : 0.0;
      ++cnt;
    }
  }
  a.corr[x] = cnt ? (float)(acc / cnt) : 0.f;
}

// ------------------------------------------------------------------- events

constexpr int KCH = 8;   // segment chunks of the per-pixel loops (grid y)

__device__ __forceinline__ void seg_chunk(int K, int& i0, int& i1) {
  const int per = (K + KCH - 1) / KCH;
  i0 = min(K, (int)blockIdx.y * per);
  i1 = min(K, i0 + per);
}

__global__ void k_events(FinalizeArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.M) return;
  const double s = a.sigma[x];
  const bool ok = s >= a.sigma_floor;
  int cnt = 0, i0, i1;
  seg_chunk(a.K, i0, i1);
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    const long long g = (long long)i * a.M + x;
    bool e;
    if (a.prob_mode) {
      e = (double)a.p[g] >= a.theta;   // learned probability map
    } else {
      const double z = ok ? (double)a.T[g] / s : 0.0;
      e = z >= a.theta;
      a.p[g] = (float)fmax(0.0, z - a.theta);
    }
    a.lab[g] = e ? (int)g : -1;
    cnt += e;
  }
  if (cnt) atomicAdd(&a.count[x], cnt);
}

// ------------------------------------------------- connected components

// lab: [n_img][M] with -1 = background, else a parent index (global).
// The flatten takes four consecutive elements per thread, read with one
// 16-byte load where all four lie in the array: nearly all of them are
// background, so most waves are done after a single memory round trip for
// 256 elements instead of 64. The merge keeps one element per thread: with
// four, a thread's unions run one after another and the slowest waves get
// longer (80 -> 111 us over 200 segments of 256x256).
constexpr int CCL_PER = 4;
static_assert(CCL_PER == 4 && PER == 4, "label loads are four wide");

__device__ __forceinline__ void load_labels(const int* lab, long long g0, long long n, int v[CCL_PER]) {
  if (g0 + CCL_PER <= n) {
    const int4 q = *reinterpret_cast<const int4*>(lab + g0);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
#pragma unroll
    for (int k = 0; k < CCL_PER; ++k) v[k] = g0 + k < n ? lab[g0 + k] : -1;
  }
}

__device__ __forceinline__ void ccl_link(int* __restrict__ lab, long long g, int W, long long M) {
  const int x = (int)(g % M);
  const int yy = x / W, xx = x - yy * W;
  // neighbours earlier in raster order: W, NW, N, NE. Every foreground pixel
  // links its own, so links implied by a neighbour's are skipped: with W
  // set, W has linked NW and N (or N through NW), leaving NE when N is
  // clear; with N set, N has linked NW, and NE links N itself.
  const bool w = xx > 0 && lab[g - 1] >= 0;
  const long long up = g - W;
  const bool n_ = yy > 0 && lab[up] >= 0;
  const bool ne = yy > 0 && xx + 1 < W && lab[up + 1] >= 0;
  if (w) {
    uf_unite(lab, (int)g, (int)(g - 1));
    if (!n_ && ne) uf_unite(lab, (int)g, (int)(up + 1));
  } else if (n_) {
    uf_unite(lab, (int)g, (int)up);
  } else if (yy > 0) {
    if (xx > 0 && lab[up - 1] >= 0) uf_unite(lab, (int)g, (int)(up - 1));
    if (ne) uf_unite(lab, (int)g, (int)(up + 1));
  }
}

__global__ void k_ccl_merge(int* __restrict__ lab, int H, int W, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (lab[g] < 0) return;
  ccl_link(lab, g, W, (long long)H * W);
}

// After the merge the forest no longer changes, except that this kernel
// points pixels at their roots: any parent value a thread reads, the merged
// one or the root written here, leads to the same root. So the parents are
// read with ordinary loads, which the L1 serves when the lanes of a wave walk
// the same path (neighbouring pixels of a run share it).
__global__ void k_ccl_flatten(int* __restrict__ lab, long long n) {
  const long long g0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * CCL_PER;
  if (g0 >= n) return;
  int v[CCL_PER];
  load_labels(lab, g0, n, v);
#pragma unroll
  for (int k = 0; k < CCL_PER; ++k) {
    int p = v[k];
    if (p < 0) continue;
    int x = (int)(g0 + k);
    while (p != x) {
      x = p;
      p = lab[x];
    }
    lab[g0 + k] = x;
  }
}

// ------------------------------------------------------ compaction of roots

// Exclusive scan over a block of NTH threads (integer, so exact in any
// order): a shuffle scan within each wave, then the wave totals (sh holds
// NTH / 64 of them); two barriers. Returns the exclusive prefix, the block
// total in *total.
template <int NTH>
__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NTH / 64; ++k) {
    const int s = sh[k];
    before += k < w ? s : 0;
    all += s;
  }
  __syncthreads();   // sh is reused by the next call
  *total = all;
  return before + x - v;
}

constexpr int SCAN_NT = 1024;   // threads of the one-block scan of block sums

__global__ void k_count_roots(const int* __restrict__ lab, long long n, int* __restrict__ sums) {
  __shared__ int sh[BS / 64];
  const long long base = (long long)blockIdx.x * CHUNK + (long long)threadIdx.x * PER;
  int v[PER];
  load_labels(lab, base, n, v);
  int c = 0;
  for (int k = 0; k < PER; ++k) c += v[k] == (int)(base + k);
  int total;
  block_exclusive_scan<BS>(c, sh, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of nb block sums by one block; grand total to *total
__global__ __launch_bounds__(SCAN_NT) void k_scan_sums(int* __restrict__ sums, int nb, int* __restrict__ total) {
  __shared__ int sh[SCAN_NT / 64];
  int carry = 0;
  for (int base = 0; base < nb; base += SCAN_NT) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    int tot;
    const int ex = block_exclusive_scan<SCAN_NT>(v, sh, &tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// id[g] = rank of root g among all roots (only written at roots)
__global__ void k_assign_ids(const int* __restrict__ lab, long long n, const int* __restrict__ sums,
                             int* __restrict__ id) {
  __shared__ int sh[BS / 64];
  const long long base = (long long)blockIdx.x * CHUNK + (long long)threadIdx.x * PER;
  int v[PER];
  load_labels(lab, base, n, v);
  int flags[PER];
  int c = 0;
  for (int k = 0; k < PER; ++k) {
    flags[k] = v[k] == (int)(base + k);
    c += flags[k];
  }
  int total;
  int r = block_exclusive_scan<BS>(c, sh, &total) + sums[blockIdx.x];
  for (int k = 0; k < PER; ++k)
    if (flags[k]) id[base + k] = r++;
}

// ------------------------------------------------------------ region stats

__global__ void k_region_zero(FinalizeArgs a, int* __restrict__ root) {
  const int nreg = a.counters[1];
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < nreg;
       r += (long long)gridDim.x * blockDim.x) {
    a.reg_area[r] = 0;
    a.reg_sx[r] = 0;
    a.reg_sy[r] = 0;
    a.reg_sxx[r] = 0;
    a.reg_syy[r] = 0;
    a.reg_sxy[r] = 0;
    a.reg_box[4 * r + 0] = 0x7fffffff;
    a.reg_box[4 * r + 1] = -1;
    a.reg_box[4 * r + 2] = 0x7fffffff;
    a.reg_box[4 * r + 3] = -1;
    a.reg_keep[r] = 0;
    root[r] = -1;
  }
}

// Region moments and bounding boxes. Consecutive pixels of a wave that carry
// the same label form runs; each run is reduced with shuffles onto its first
// lane, which issues the atomics (integer, so the totals do not depend on
// the order).
__global__ void k_region_accum(FinalizeArgs a, long long n, int* __restrict__ root) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int l = g < n ? a.lab[g] : -1;
  // a wave without a labelled pixel contributes nothing (most waves: the
  // event regions are sparse); the wave leaves as a whole, so the shuffles
  // below always see all its lanes
  if (__ballot(l >= 0) == 0) return;
  unsigned cnt = 0, sx = 0, sy = 0;
  unsigned long long sxx = 0, syy = 0, sxy = 0;
  int x0 = INT_MAX, x1 = -1, y0 = INT_MAX, y1 = -1;
  if (l >= 0) {
    const int x = (int)(g % a.M);
    const unsigned yy = (unsigned)(x / a.W), xx = (unsigned)(x - (int)yy * a.W);
    cnt = 1;
    sx = xx;
    sy = yy;
    sxx = (unsigned long long)xx * xx;
    syy = (unsigned long long)yy * yy;
    sxy = (unsigned long long)xx * yy;
    x0 = x1 = (int)xx;
    y0 = y1 = (int)yy;
  }
  const int lp = __shfl_up(l, 1);
  const bool head = l >= 0 && (lane == 0 || lp != l);
  int key = head ? lane : -1;  // first lane of the run: inclusive max-scan of the heads
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(key, d);
    if (lane >= d) key = max(key, o);
  }
  if (l < 0) key = -2;
  for (int d = 1; d < 64; d <<= 1) {
    const int ko = __shfl_down(key, d);
    const unsigned c_ = __shfl_down(cnt, d), sx_ = __shfl_down(sx, d), sy_ = __shfl_down(sy, d);
    const unsigned long long sxx_ = __shfl_down(sxx, d), syy_ = __shfl_down(syy, d), sxy_ = __shfl_down(sxy, d);
    const int x0_ = __shfl_down(x0, d), x1_ = __shfl_down(x1, d);
    const int y0_ = __shfl_down(y0, d), y1_ = __shfl_down(y1, d);
    if (lane + d < 64 && ko == key) {
      cnt += c_;
      sx += sx_;
      sy += sy_;
      sxx += sxx_;
      syy += syy_;
      sxy += sxy_;
      x0 = min(x0, x0_);
      x1 = max(x1, x1_);
      y0 = min(y0, y0_);
      y1 = max(y1, y1_);
    }
  }
  if (l < 0) return;
  const int r = a.rid[l];
  if (head) {
    atomicAdd(&a.reg_area[r], cnt);
    atomicAdd(&a.reg_sx[r], sx);
    atomicAdd(&a.reg_sy[r], sy);
    atomicAdd(&a.reg_sxx[r], sxx);
    atomicAdd(&a.reg_syy[r], syy);
    atomicAdd(&a.reg_sxy[r], sxy);
    atomicMin(&a.reg_box[4 * r + 0], x0);
    atomicMax(&a.reg_box[4 * r + 1], x1);
    atomicMin(&a.reg_box[4 * r + 2], y0);
    atomicMax(&a.reg_box[4 * r + 3], y1);
  }
  if (l == (int)g) root[r] = l;
}

// Regions whose bounding box has at most SHORT_ROWS rows (nearly all of them:
// event regions are a few cell diameters tall) are decided by a kernel whose
// per-row tables fit in 1.5 KB of LDS, so many blocks share a CU; the others
// by one sized for the tallest frame (49 KB, three blocks per CU).
constexpr int SHORT_ROWS = 64;

__device__ __forceinline__ long long cross3(int ou, int ov, int au, int av, int bu, int bv) {
  return (long long)(au - ou) * (bv - ov) - (long long)(av - ov) * (bu - ou);
}

// One 64-thread block per region (grid-stride). Keep decision per Sec. III-D:
// area bounds, eccentricity of the pixel-centre covariance, solidity against
// the convex hull of the pixel-square corners. TALL selects the regions of
// more than SHORT_ROWS rows, else those of at most SHORT_ROWS; HULL_ROWS is
// the row capacity of the tables.
template <int HULL_ROWS, bool TALL>
__global__ __launch_bounds__(64) void k_region_decide(FinalizeArgs a, const int* __restrict__ root) {
  __shared__ int xl[HULL_ROWS], xr[HULL_ROWS];
  __shared__ int sl[2 * HULL_ROWS + 2], sr[2 * HULL_ROWS + 2];  // packed (u << 16) | v
  __shared__ int decide;
  const int nreg = a.counters[1];
  const int lane = threadIdx.x;
  for (int r = blockIdx.x; r < nreg; r += gridDim.x) {
    // the same for every lane, so the whole block skips the region
    if ((a.reg_box[4 * r + 3] - a.reg_box[4 * r + 2] + 1 > SHORT_ROWS) != TALL) continue;
    const long long n = a.reg_area[r];
    if (lane == 0) {
      int d = 0;
      if (n >= a.area_min && n <= a.area_max) {
        const long long sx = a.reg_sx[r], sy = a.reg_sy[r];
        const long long A_ = n * (long long)a.reg_sxx[r] - sx * sx;
        const long long B_ = n * (long long)a.reg_syy[r] - sy * sy;
        const long long C_ = n * (long long)a.reg_sxy[r] - sx * sy;
        const double p = (double)(A_ + B_);
        const double dab = (double)(A_ - B_);
        const double dc = (double)C_;
        const double t1 = dab * dab;
        const double t2 = 4.0 * dc;
        const double t3 = t2 * dc;
        const double s = sqrt(t1 + t3);
        const double ratio = (p + s > 0.0) ? (p - s) / (p + s) : 1.0;
        d = ratio >= a.ecc_thr ? 1 : 0;
      }
      decide = d;
    }
    __syncthreads();
    if (!decide) {
      __syncthreads();
      continue;
    }
    // per-row extremes of the region inside its bounding box: one lane per
    // row, eight label loads in flight at a time
    const int x0 = a.reg_box[4 * r + 0], x1 = a.reg_box[4 * r + 1];
    const int y0 = a.reg_box[4 * r + 2], y1 = a.reg_box[4 * r + 3];
    const int rt = root[r];
    const long long img = (long long)(rt / a.M) * a.M;
    for (int y = y0 + lane; y <= y1; y += 64) {
      const int* row = a.lab + img + (long long)y * a.W;
      int mn = 0x7fffffff, mx = -1;
      for (int x = x0; x <= x1; x += 8) {
        int v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = x + k <= x1 ? row[x + k] : -1;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (v[k] == rt) {
            mn = min(mn, x + k);
            mx = max(mx, x + k);
          }
      }
      xl[y - y0] = mn;
      xr[y - y0] = mx + 1;
    }
    __syncthreads();
    if (lane == 0) {
      const int rows = y1 - y0 + 1;
      // lower chain over the left corner points, upper chain over the right
      // ones, both in (u = y, v = x) coordinates sorted by (u, v)
      int nl = 0, nu = 0;
      auto push_l = [&](int u, int v) {
        while (nl >= 2 && cross3(sl[nl - 2] >> 16, sl[nl - 2] & 0xffff, sl[nl - 1] >> 16,
                                 sl[nl - 1] & 0xffff, u, v) <= 0)
          --nl;
        sl[nl++] = (u << 16) | v;
      };
      push_l(y0, xl[0]);
      for (int k = 1; k < rows; ++k) {
        const int lo = min(xl[k - 1], xl[k]), hi = max(xl[k - 1], xl[k]);
        push_l(y0 + k, lo);
        push_l(y0 + k, hi);
      }
      push_l(y1 + 1, xl[rows - 1]);
      // upper chain: traverse the right points in reverse (u, v) order
      auto push_u = [&](int u, int v) {
        while (nu >= 2 && cross3(sr[nu - 2] >> 16, sr[nu - 2] & 0xffff, sr[nu - 1] >> 16,
                                 sr[nu - 1] & 0xffff, u, v) <= 0)
          --nu;
        sr[nu++] = (u << 16) | v;
      };
      push_u(y1 + 1, xr[rows - 1]);
      for (int k = rows - 1; k >= 1; --k) {
        const int lo = min(xr[k - 1], xr[k]), hi = max(xr[k - 1], xr[k]);
        push_u(y0 + k, hi);
        push_u(y0 + k, lo);
      }
      push_u(y0, xr[0]);
      long long a2 = 0;
      const int nt = nl + nu;
      for (int k = 0; k < nt; ++k) {
        const int k2 = k + 1 == nt ? 0 : k + 1;
        const int pk = k < nl ? sl[k] : sr[k - nl];
        const int pm = k2 < nl ? sl[k2] : sr[k2 - nl];
        const int ku = pk >> 16, kv = pk & 0xffff, mu = pm >> 16, mv = pm & 0xffff;
        a2 += (long long)ku * mv - (long long)mu * kv;
      }
      if (a2 < 0) a2 = -a2;
      const double sol = a2 ? 2.0 * (double)n / (double)a2 : 1.0;
      a.reg_keep[r] = sol >= a.solidity_min ? 1 : 0;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- aggregation

__global__ void k_kept(FinalizeArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.M) return;
  int nb = 0, i0, i1;
  seg_chunk(a.K, i0, i1);
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    const long long g = (long long)i * a.M + x;
    const int l = a.lab[g];
    const int b = l >= 0 ? a.reg_keep[a.rid[l]] : 0;
    a.bmask[g] = (uint8_t)b;
    nb += b;
  }
  if (nb) atomicAdd(&a.nb[x], nb);
}

// the aggregate mask b = [n_b >= c_min] as union-find seeds
__global__ void k_aggregate(FinalizeArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.M) return;
  a.blab[x] = a.nb[x] >= a.min_event_segs ? x : -1;
  if (x < a.Ccap) {   // per-component pixel counts and bounding boxes start empty
    a.coff[x] = 0;
    reinterpret_cast<int4*>(a.cbox)[x] = make_int4(INT_MAX, -1, INT_MAX, -1);
  }
}

__global__ void k_component_labels(FinalizeArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.M) return;
  const int l = a.blab[x];
  a.comp[x] = l >= 0 ? a.rid[l] + 1 : 0;
}

// Pixel count and bounding box of each component, one update per horizontal
// run of its pixels (by the run's first pixel): atomics on one address
// serialise, and a component has far fewer runs than pixels.
__global__ void k_comp_stats(FinalizeArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.M) return;
  const int c = a.comp[x];
  if (c == 0) return;
  const int yy = x / a.W, xx = x - yy * a.W;
  if (xx > 0 && a.comp[x - 1] == c) return;
  int e = xx;
  while (e + 1 < a.W && a.comp[x + (e + 1 - xx)] == c) ++e;
  int* b = a.cbox + 4 * (c - 1);
  atomicAdd(&a.coff[c - 1], e - xx + 1);
  atomicMin(b + 0, xx);
  atomicMax(b + 1, e);
  atomicMin(b + 2, yy);
  atomicMax(b + 3, yy);
}

// Component offsets: exclusive scan of the pixel counts of the counters[0]
// components, in place; coff[ncomp] = number of component pixels.
__global__ __launch_bounds__(SCAN_NT) void k_comp_offsets(FinalizeArgs a) {
  __shared__ int sh[SCAN_NT / 64];
  const int n = a.counters[0];
  int carry = 0;
  for (int base = 0; base < n; base += SCAN_NT) {
    const int i = base + threadIdx.x;
    const int v = i < n ? a.coff[i] : 0;
    int tot;
    const int ex = block_exclusive_scan<SCAN_NT>(v, sh, &tot);
    if (i < n) a.coff[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) a.coff[n] = carry;
}

// Pixel list of each component in raster order: a workgroup walks the
// component's bounding box row by row, 4,096 pixels at a time (four adjacent
// ones per thread, loaded at once), and places the component's pixels by an
// exclusive scan of the per-thread counts, so the lists do not depend on
// scheduling.
constexpr int PIX_NT = 1024, PIX_PER = 4;
__global__ __launch_bounds__(PIX_NT) void k_comp_pixels(FinalizeArgs a) {
  __shared__ int sh[PIX_NT / 64];
  const int n = a.counters[0];
  for (int c = blockIdx.x; c < n; c += gridDim.x) {
    const int4 b = reinterpret_cast<const int4*>(a.cbox)[c];
    const int bw = b.y - b.x + 1, area = bw * (b.w - b.z + 1);
    int run = a.coff[c];
    for (int base = 0; base < area; base += PIX_NT * PIX_PER) {
      int px[PIX_PER];
      unsigned f = 0;
#pragma unroll
      for (int k = 0; k < PIX_PER; ++k) {
        const int idx = base + (int)threadIdx.x * PIX_PER + k;
        px[k] = -1;
        if (idx < area) {
          const int r = idx / bw;
          px[k] = (b.z + r) * a.W + b.x + (idx - r * bw);
        }
      }
#pragma unroll
      for (int k = 0; k < PIX_PER; ++k)
        if (px[k] >= 0 && a.comp[px[k]] == c + 1) f |= 1u << k;
      int tot;
      int off = run + block_exclusive_scan<PIX_NT>(__popc(f), sh, &tot);
#pragma unroll
      for (int k = 0; k < PIX_PER; ++k)
        if (f >> k & 1u) a.pix[off++] = px[k];
      run += tot;
    }
  }
}

__global__ void k_u8_to_f32(const uint8_t* __restrict__ in, float* __restrict__ out, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = (float)in[g];
}

inline unsigned blocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t compact_roots(const int* lab, long long n, int* sums, int scan_cap, int* total,
                         int* id, hipStream_t st) {
  const long long nb = (n + CHUNK - 1) / CHUNK;
  if (nb > scan_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_count_roots, dim3((unsigned)nb), dim3(BS), 0, st, lab, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_NT), 0, st, sums, (int)nb, total);
  hipLaunchKernelGGL(k_assign_ids, dim3((unsigned)nb), dim3(BS), 0, st, lab, n, sums, id);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_finalize_maps(const FinalizeArgs& a, hipStream_t st) {
  double* C = a.C;
  int* root = a.root;
  const long long KM = (long long)a.K * a.M;
  hipLaunchKernelGGL(k_moments, dim3(blocks(a.M, BS)), dim3(BS), 0, st, a, C);
  hipLaunchKernelGGL(k_pointwise, dim3(blocks(a.M, BS)), dim3(BS), 0, st, a, (const double*)C);
  hipLaunchKernelGGL(k_events, dim3(blocks(a.M, BS), KCH), dim3(BS), 0, st, a);
  hipLaunchKernelGGL(k_ccl_merge, dim3(blocks(KM, BS)), dim3(BS), 0, st, a.lab, a.H, a.W, KM);
  hipLaunchKernelGGL(k_ccl_flatten, dim3(blocks((KM + CCL_PER - 1) / CCL_PER, BS)), dim3(BS), 0, st, a.lab, KM);
  hipError_t e = compact_roots(a.lab, KM, a.scan, a.scan_cap, &a.counters[1], a.rid, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_region_zero, dim3(1024), dim3(BS), 0, st, a, root);
  hipLaunchKernelGGL(k_region_accum, dim3(blocks(KM, BS)), dim3(BS), 0, st, a, KM, root);
  hipLaunchKernelGGL((k_region_decide<SHORT_ROWS, false>), dim3(8192), dim3(64), 0, st, a, (const int*)root);
  hipLaunchKernelGGL((k_region_decide<kMaxDim, true>), dim3(768), dim3(64), 0, st, a, (const int*)root);
  hipLaunchKernelGGL(k_kept, dim3(blocks(a.M, BS), KCH), dim3(BS), 0, st, a);
  hipLaunchKernelGGL(k_aggregate, dim3(blocks(a.M, BS)), dim3(BS), 0, st, a);
  hipLaunchKernelGGL(k_ccl_merge, dim3(blocks(a.M, BS)), dim3(BS), 0, st, a.blab, a.H, a.W, (long long)a.M);
  hipLaunchKernelGGL(k_ccl_flatten, dim3(blocks((a.M + CCL_PER - 1) / CCL_PER, BS)), dim3(BS), 0, st, a.blab,
                     (long long)a.M);
  // component ids reuse the rid array (the per-segment ids are no longer needed)
  e = compact_roots(a.blab, a.M, a.scan, a.scan_cap, &a.counters[0], a.rid, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_component_labels, dim3(blocks(a.M, BS)), dim3(BS), 0, st, a);
  hipLaunchKernelGGL(k_comp_stats, dim3(blocks(a.M, BS)), dim3(BS), 0, st, a);
  hipLaunchKernelGGL(k_comp_offsets, dim3(1), dim3(SCAN_NT), 0, st, a);
  hipLaunchKernelGGL(k_comp_pixels, dim3(256), dim3(PIX_NT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_u8_to_f32(const uint8_t* in, float* out, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_u8_to_f32, dim3(blocks(n, BS)), dim3(BS), 0, st, in, out, n);
  return hipGetLastError();
}

}  // namespace seg
