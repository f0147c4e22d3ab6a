// Declarations shared by the kernel files and the host library: limits,
// kernel argument structures and launchers. Host-only state (workspace
// layout, session) is declared in seg_internal.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include "seg.h"

namespace seg {

constexpr int kSegLen = 50;       // L, Sec. III-B
constexpr int kMaxRadius = 12;    // smoothing taps |k| <= 12
constexpr int kMaxRank = 8;       // NMF rank cap per component
constexpr int kMaxDim = 2048;     // frame height / width limit
constexpr int kMaxSegments = 4096;
constexpr int kMaxBatch = 64;     // sessions per batched launch
constexpr int kUnetGroup = 8;     // segments whose summary patches share network calls

// ---- kernel launchers (defined in the .hip files) ----

struct StreamLaunch {
  const uint16_t* src0;  // first n0 frames come from here (the tail buffer)
  const uint16_t* src1;  // then from here (the caller's frames)
  long long n0;
  int H, W;
  int seg0;       // index of the first segment written
  int nseg;       // segments in this launch
  float *T, *S, *D, *U, *P;
  long long plane;  // Kmax * M, stride between the five P planes
  const double* w;  // 2 * kMaxRadius + 1 taps (zero beyond the radius)
};
hipError_t launch_block_stats(const StreamLaunch& a, hipStream_t st);
// serving: slot table for one persistent launch over several recordings
size_t batch_table_bytes();
int fill_batch_table(void* host_table, const StreamLaunch* launches, int count);
hipError_t launch_block_stats_batch(const void* dev_table, int grid, hipStream_t st);

struct FinalizeArgs {
  int H, W, M, K, Kmax;
  const float *T, *S, *D, *U, *P;
  long long plane;
  double* sigma;
  float* corr;
  float* mean;
  int* count;
  float* p;
  int* lab;
  int* rid;
  uint8_t* bmask;
  uint32_t *reg_area, *reg_sx, *reg_sy;
  unsigned long long *reg_sxx, *reg_syy, *reg_sxy;
  int* reg_box;
  uint8_t* reg_keep;
  int* nb;
  int* blab;
  int* comp;
  int* pix;        // i32 [M] component pixel lists, raster order within each
  int* coff;       // i32 [Ccap + 1] component offsets into pix
  int* cbox;       // i32 [Ccap][4] component bounding boxes (x0, x1, y0, y1)
  int Ccap;        // component capacity
  int* scan;
  int* counters;
  long long Rcap;
  int scan_cap;
  double* C;       // f64 [5][M] pooled co-moments
  int* root;       // i32 [Rcap] root pixel of each region
  double theta, sigma_floor, solidity_min, ecc_thr;
  int area_min, area_max, min_event_segs;
  bool have_moments;
  bool prob_mode;  // surrogate: p holds probabilities, events are p >= theta
};
// pointwise images, events, per-segment regions, kept masks, aggregate,
// canonical components and their pixel lists; writes the component count to
// counters[0], the offsets to coff and the lists to pix
hipError_t launch_finalize_maps(const FinalizeArgs& a, hipStream_t st);
hipError_t launch_u8_to_f32(const uint8_t* in, float* out, long long n, hipStream_t st);

struct NmfArgs {
  int M, K, Kmax, ncomp;
  const float* p;
  const int* pix;
  const int* coff;
  double *P, *PT, *R, *F, *A, *G, *Wk;
  int* N;
  int max_rank, sweeps;
  double delta;
  int Q;                 // pixel partitions of the column sums
  bool lds_A, lds_F;     // A (and the partial sums) / F held in LDS
  size_t lds_bytes;      // dynamic LDS per workgroup
};
// LDS plan for the NMF given the largest component and the segment count
void plan_nmf(NmfArgs& a, int max_mc);
hipError_t launch_nmf(const NmfArgs& a, hipStream_t st);

// NMF with every component split over co-resident workgroups (k_nmf_split)
struct NmfSplit {
  int G;                 // workgroups of one cooperative launch (all of them in the plan)
  int mw;                // pixels (rows of P_c) per workgroup
  int Kp;                // LDS row stride of the P_c rows (odd)
  int scr;               // doubles of LDS scratch
  int XS;                // doubles per exchange slot
  size_t lds_bytes;      // dynamic LDS per workgroup
  long long limit;       // wall-clock ticks a meeting may wait
  const int* wg_comp;    // [G] component of each workgroup of the launch
  const int* wg_rank;    // [G] its number within the component (its slice and slots)
  const int* wg_base;    // [ncomp] first slot index of each component within its launch
  const int* wg_n;       // [ncomp] workgroups of each component
  unsigned long long* xbuf;  // [G][2][2 XS] exchange slots: tagged high, then low words
  unsigned* sync;        // [ncomp + 1] abandon flags, error flag
};
// Host copies of the workgroup tables and the launches (first workgroup in
// `comp`, workgroup count) of a split plan.
struct NmfSplitTables {
  std::vector<int> comp, rank, base, n;
  std::vector<std::pair<int, int>> groups;
};
// Chooses the slice width (fewest launches of at most one workgroup per
// compute unit that fit LDS and xbuf_bytes) and packs the components into
// launches; false when the split path does not apply.
bool plan_nmf_split(NmfSplit& s, const NmfArgs& a, const std::vector<int>& coff, size_t xbuf_bytes,
                    NmfSplitTables& tab);
// One launch of the plan (s.G and s.wg_comp select it): clears its exchange
// slots first; `first` also clears the abandon and error flags.
hipError_t launch_nmf_split(const NmfArgs& a, const NmfSplit& s, bool first, hipStream_t st);

}  // namespace seg
