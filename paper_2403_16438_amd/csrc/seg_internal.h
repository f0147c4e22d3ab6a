// Host-side declarations of the library: workspace layout, footprints and
// the session; the kernel interfaces come from seg_kernels.h.
#pragma once

#include <vector>

#include "seg_kernels.h"

namespace seg {

// Offsets (bytes) of every array inside the caller's workspace.
struct Layout {
  size_t tail;      // u16 [L-1][M]   frames carried to the next push
  size_t T, S, D, U;  // f32 [Kmax][M] per-segment summaries
  size_t P;         // f32 [5][Kmax][M] per-segment co-moment sums
  size_t sigma;     // f64 [M]
  size_t corr;      // f32 [M]
  size_t mean;      // f32 [M]
  size_t count;     // i32 [M] events per pixel
  size_t p;         // f32 [Kmax][M] detection maps
  size_t lab;       // i32 [Kmax][M] per-segment event labels (union-find)
  size_t rid;       // i32 [Kmax][M] region id at each root pixel
  size_t bmask;     // u8  [Kmax][M] kept-region masks b_i
  size_t reg_area;  // u32 [Rcap]
  size_t reg_sx, reg_sy;          // u32 [Rcap]
  size_t reg_sxx, reg_syy, reg_sxy;  // u64 [Rcap]
  size_t reg_box;   // i32 [Rcap][4] xmin, xmax, ymin, ymax
  size_t reg_keep;  // u8  [Rcap]
  size_t nb;        // i32 [M]
  size_t blab;      // i32 [M] union-find labels of the aggregate mask
  size_t comp;      // i32 [M] canonical component labels
  size_t scan;      // i32 [scan_cap] block sums for compaction scans
  size_t counters;  // i32 [16]
  size_t pix;       // i32 [M] component pixel lists (raster order)
  size_t coff;      // i32 [M + 1] component offsets
  size_t cbox;      // i32 [Ccap][4] component bounding boxes
  size_t nmf_P;     // f64 [M][Kmax] gathered P_c (pixel-major)
  size_t nmf_PT;    // f64 [Kmax][M] gathered P_c (segment-major)
  size_t nmf_R;     // f64 [M][Kmax] SPA residual
  size_t nmf_F;     // f64 [M][kMaxRank]
  size_t nmf_A;     // f64 [Ccap][kMaxRank][Kmax]
  size_t nmf_N;     // i32 [Ccap] rank per component
  size_t nmf_G;     // f64 [M][kMaxRank] P A^T and SPA direction
  size_t nmf_W;     // f64 [Ccap][2][Kmax] SPA column flags and projections
  size_t cmom;      // f64 [5][M] pooled co-moments
  size_t reg_root;  // i32 [Rcap]
  size_t stage;     // u16 [50][M] one segment's frames for the surrogate (else 0 bytes)
  size_t total;
  size_t Rcap;      // region capacity
  size_t Ccap;      // component capacity
  size_t scan_cap;
};

Layout make_layout(const seg_config& c);

// A footprint is kept sparse: its weights on the pixels of its component
// (raster order, the session's component pixel lists); seg_get_footprints
// expands it to dense frames.
struct Footprint {
  int component;               // 1-based
  int peak;                    // raster index of the largest weight
  std::vector<float> w;        // [M_c] weights of the component's pixels
  std::vector<uint8_t> on;     // [M_c] mask: FP64 weight >= the footprint level
  std::vector<float> activity; // [K]
};

enum class State { Open, Finalized, Failed };

}  // namespace seg

struct seg_session {
  seg_config cfg;
  seg::Layout lay;
  char* ws;            // device workspace base
  size_t ws_bytes;
  int device;
  uint32_t M;
  uint32_t Kmax;
  uint64_t frames;     // frames accepted so far
  uint32_t K;          // complete segments
  uint32_t tail_n;     // frames held in the tail buffer
  seg::State state;
  int error;           // sticky error
  double w[2 * seg::kMaxRadius + 1];
  struct seg_nn* net; // surrogate network (SEG_DET_SURROGATE)
  // results (host copies after finalize)
  uint32_t n_comp;
  std::vector<seg::Footprint> fps;
  std::vector<int> comp_pix, comp_off;   // component pixel lists (CSR, raster order)
  // trace extraction tables (built at finalize, uploaded by the first
  // seg_extract_traces into the NMF factor region, unused after finalize)
  std::vector<int> tr_pix;          // masked pixels of every component, raster order
  std::vector<uint8_t> tr_bits;     // bit r: in the mask of the component's footprint r
  std::vector<int> tr_comp;         // [4 per component] entry begin, end, first footprint, footprints
  std::vector<uint32_t> tr_count;   // [N] mask sizes
  bool tr_ready;
  size_t tr_at[4];                  // workspace offsets of the four tables
  hipEvent_t ev[4];    // finalize timing: maps start/end, NMF start/end
  bool have_ev;
  seg_profile prof;
};
