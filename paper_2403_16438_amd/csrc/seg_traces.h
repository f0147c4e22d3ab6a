// Kernel interface of the trace extraction (k_traces.hip), shared with the
// host library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace seg {

// Per component, the pixels that lie in at least one of its footprints'
// masks, with one mask bit per footprint of the component.
struct TraceArgs {
  const uint16_t* frames;  // [n_frames][M]
  long long n_frames;
  int M;
  int ncomp;               // entries of comp
  int max_fp;              // largest footprint count of a component (<= kMaxRank)
  const int* pix;          // [entries] raster index of each masked pixel
  const uint8_t* bits;     // [entries] bit r: in the mask of footprint z + r
  const int4* comp;        // [ncomp] {entry begin, entry end, first footprint z, footprints}
  const uint32_t* count;   // [footprints] mask sizes
  float* out;              // [footprints][ld] traces, column t = frame t
  long long ld;
};
hipError_t launch_traces(const TraceArgs& a, hipStream_t st);

}  // namespace seg
