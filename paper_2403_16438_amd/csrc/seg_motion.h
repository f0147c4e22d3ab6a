// Kernel interface of the motion correction (k_motion.hip), shared with the
// host library (mc_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace seg {

constexpr int kPatch = 21;                 // tile side (Sec. II)
constexpr int kPatchPix = kPatch * kPatch; // 441
constexpr int kPatchK = 444;               // 441 padded to the MFMA depth 4
constexpr int kMcFrames = 16;              // frames per workgroup (the MFMA's N)
constexpr int kMcMaxRadius = 10;           // |dy|, |dx| <= R
constexpr int kMcChunk = 2048;             // frames per scoring launch
constexpr int kMcSlices = 8;               // patch slices per frame group

// Geometry of one motion corrector: tile grid and candidate vectors.
struct McGeom {
  int H, W, R;
  int TW;          // template window side 21 + 2R
  int ny, nx;      // tiles per column / row
  int oy, ox;      // origin of the first tile
  int P;           // tiles, ny * nx
  int V;           // vectors (2R + 1)^2, ordered by dy then dx
  int Vp;          // V rounded up to 16 (the MFMA's M)
  int S;           // patch slices
  int pps;         // patches per slice
};

struct McScoreArgs {
  McGeom g;
  const uint16_t* frames;   // [n][H][W]
  int n;                    // frames of this launch, <= chunk
  const uint16_t* tmpl;     // [H][W]
  const double* sT;         // [P][Vp] template window sums
  const double* vT;         // [P][Vp] 1 / sqrt(441 sum T^2 - (sum T)^2), 0 if that is 0
  double* part;             // [S][chunk][Vp] per-slice ZNCC sums
  int chunk;                // frame stride of `part`, >= n
};

// template = per-pixel sum of n frames, rounded half up after division by n
hipError_t launch_mc_template(const uint16_t* frames, int n, long long M, uint16_t* tmpl, hipStream_t st);
// integral images of T and T^2 ([H+1][W+1] each, uint64) and the window
// tables: sum T and the reciprocal root of 441 sum T^2 - (sum T)^2
hipError_t launch_mc_tables(const McGeom& g, const uint16_t* tmpl, unsigned long long* ii,
                            double* sT, double* vT, hipStream_t st);
hipError_t launch_mc_scores(const McScoreArgs& a, hipStream_t st);
// per frame: slice sums in order, argmax (first maximum), motion = -d;
// scores (may be null) [n][V]; `part` as in McScoreArgs with frame stride chunk
hipError_t launch_mc_pick(const McGeom& g, const double* part, int chunk, int n, int32_t* motion,
                          double* scores, hipStream_t st);

// Fixed device array for the partial sums of callers that cannot allocate:
// kMcStaticFrames frames of the largest geometry (8 slices, 448 padded
// vectors at radius 10), 7 MiB per GPU, alive until the process ends.
constexpr int kMcStaticFrames = 256;
constexpr int kMaxMcDevices = 64;
constexpr size_t kMcStaticDoubles = (size_t)kMcSlices * kMcStaticFrames * 448;
// Device address of that array on the current device, resolved once per
// device (hipGetSymbolAddress) and cached. Returns the HIP status.
hipError_t mc_static_scratch(double** ptr);
// out(y, x) = in(y + my, x + mx) inside the frame, else tmpl(y, x)
hipError_t launch_mc_apply(const uint16_t* in, long long n, int H, int W, const int32_t* motion,
                           const uint16_t* tmpl, uint16_t* out, hipStream_t st);

}  // namespace seg
