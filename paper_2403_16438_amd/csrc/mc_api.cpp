// Host side of the motion-correction C ABI declared in include/seg_mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "seg_mc.h"
#include "seg_motion.h"

struct seg_mc {
  seg_mc_config cfg;
  seg::McGeom g;
  char* ws;
  size_t at_tmpl, at_ii, at_sT, at_vT, at_part, total;
  int device;
  double* scratch;   // this device's copy of the static partial-sum array (or null)
  bool have_template;
  bool failed;
};

namespace {

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

bool make_geom(const seg_mc_config* c, seg::McGeom& g) {
  if (!c || c->radius < 1 || c->radius > (uint32_t)seg::kMcMaxRadius) return false;
  if (c->height > 2048 || c->width > 2048) return false;
  const int R = (int)c->radius, H = (int)c->height, W = (int)c->width;
  if (H < seg::kPatch + 2 * R || W < seg::kPatch + 2 * R) return false;
  g.H = H;
  g.W = W;
  g.R = R;
  g.TW = seg::kPatch + 2 * R;
  g.ny = (H - 2 * R) / seg::kPatch;
  g.nx = (W - 2 * R) / seg::kPatch;
  g.oy = R + ((H - 2 * R) - seg::kPatch * g.ny) / 2;
  g.ox = R + ((W - 2 * R) - seg::kPatch * g.nx) / 2;
  g.P = g.ny * g.nx;
  g.V = (2 * R + 1) * (2 * R + 1);
  g.Vp = (g.V + 15) / 16 * 16;
  g.S = std::min(seg::kMcSlices, g.P);
  g.pps = (g.P + g.S - 1) / g.S;
  g.S = (g.P + g.pps - 1) / g.pps;
  return true;
}

size_t layout(const seg::McGeom& g, seg_mc* m) {
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = up256(o + b);
    return at;
  };
  const size_t M = (size_t)g.H * g.W;
  const size_t a0 = take(M * 2);
  const size_t a1 = take((size_t)(g.H + 1) * (g.W + 1) * 8 * 2);
  const size_t a2 = take((size_t)g.P * g.Vp * 8);
  const size_t a3 = take((size_t)g.P * g.Vp * 8);
  const size_t a4 = take((size_t)g.S * seg::kMcChunk * g.Vp * 8);
  if (m) {
    m->at_tmpl = a0;
    m->at_ii = a1;
    m->at_sT = a2;
    m->at_vT = a3;
    m->at_part = a4;
    m->total = o;
  }
  return o;
}

int fail(seg_mc* m, hipError_t e) {
  if (e == hipSuccess) return SEG_OK;
  m->failed = true;
  return SEG_E_DEVICE;
}

int enter(seg_mc* m) {
  if (!m) return SEG_E_INVAL;
  if (m->failed) return SEG_E_DEVICE;
  if (hipSetDevice(m->device) != hipSuccess) return fail(m, hipErrorInvalidDevice);
  return SEG_OK;
}

template <typename T>
T* at(seg_mc* m, size_t off) {
  return reinterpret_cast<T*>(m->ws + off);
}

}  // namespace

extern "C" {

int seg_mc_default_config(uint32_t height, uint32_t width, seg_mc_config* out) {
  if (!out || height == 0 || width == 0) return SEG_E_INVAL;
  out->height = height;
  out->width = width;
  out->radius = 8;
  return SEG_OK;
}

int seg_mc_workspace_bytes(const seg_mc_config* cfg, size_t* bytes) {
  seg::McGeom g;
  if (!bytes || !make_geom(cfg, g)) return SEG_E_INVAL;
  *bytes = layout(g, nullptr);
  return SEG_OK;
}

int seg_mc_create(const seg_mc_config* cfg, void* dev_workspace, size_t bytes, seg_mc** out) {
  if (!out || !dev_workspace) return SEG_E_INVAL;
  *out = nullptr;
  seg::McGeom g;
  if (!make_geom(cfg, g)) return SEG_E_INVAL;
  if (reinterpret_cast<uintptr_t>(dev_workspace) & 255) return SEG_E_INVAL;
  seg_mc* m = new (std::nothrow) seg_mc();
  if (!m) return SEG_E_INVAL;
  m->cfg = *cfg;
  m->g = g;
  layout(g, m);
  if (bytes < m->total) {
    delete m;
    return SEG_E_CAPACITY;
  }
  m->ws = static_cast<char*>(dev_workspace);
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return SEG_E_DEVICE;
  }
  // the static partial-sum array's address on this device, for
  // seg_mc_estimate_static (which fails with SEG_E_DEVICE if it is missing)
  if (seg::mc_static_scratch(&m->scratch) != hipSuccess) {
    (void)hipGetLastError();
    m->scratch = nullptr;
  }
  *out = m;
  return SEG_OK;
}

int seg_mc_layout(const seg_mc* mc, uint32_t* n_patches, uint32_t* n_vectors) {
  if (!mc) return SEG_E_INVAL;
  if (n_patches) *n_patches = (uint32_t)mc->g.P;
  if (n_vectors) *n_vectors = (uint32_t)mc->g.V;
  return SEG_OK;
}

int seg_mc_set_template(seg_mc* mc, const uint16_t* dev_frames, uint32_t n_frames, void* stream) {
  int e = enter(mc);
  if (e) return e;
  if (!dev_frames || n_frames == 0 || n_frames > 65536) return SEG_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const seg::McGeom& g = mc->g;
  uint16_t* t = at<uint16_t>(mc, mc->at_tmpl);
  if ((e = fail(mc, seg::launch_mc_template(dev_frames, (int)n_frames, (long long)g.H * g.W, t, st)))) return e;
  if ((e = fail(mc, seg::launch_mc_tables(g, t, at<unsigned long long>(mc, mc->at_ii), at<double>(mc, mc->at_sT),
                                          at<double>(mc, mc->at_vT), st))))
    return e;
  mc->have_template = true;
  return SEG_OK;
}

int seg_mc_get_template(seg_mc* mc, uint16_t* host_out) {
  int e = enter(mc);
  if (e) return e;
  if (!host_out) return SEG_E_INVAL;
  if (!mc->have_template) return SEG_E_STATE;
  if ((e = fail(mc, hipDeviceSynchronize()))) return e;
  return fail(mc, hipMemcpy(host_out, mc->ws + mc->at_tmpl, (size_t)mc->g.H * mc->g.W * 2, hipMemcpyDeviceToHost));
}

int seg_mc_estimate(seg_mc* mc, const uint16_t* dev_frames, uint64_t n_frames, int32_t* dev_motion,
                    double* dev_scores, void* stream) {
  int e = enter(mc);
  if (e) return e;
  if (!mc->have_template) return SEG_E_STATE;
  if (n_frames == 0) return SEG_OK;
  if (!dev_frames || !dev_motion) return SEG_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const seg::McGeom& g = mc->g;
  const size_t M = (size_t)g.H * g.W;
  for (uint64_t f0 = 0; f0 < n_frames; f0 += seg::kMcChunk) {
    const int n = (int)std::min<uint64_t>(seg::kMcChunk, n_frames - f0);
    seg::McScoreArgs a{};
    a.g = g;
    a.frames = dev_frames + f0 * M;
    a.n = n;
    a.tmpl = at<uint16_t>(mc, mc->at_tmpl);
    a.sT = at<double>(mc, mc->at_sT);
    a.vT = at<double>(mc, mc->at_vT);
    a.part = at<double>(mc, mc->at_part);
    a.chunk = seg::kMcChunk;
    if ((e = fail(mc, seg::launch_mc_scores(a, st)))) return e;
    if ((e = fail(mc, seg::launch_mc_pick(g, a.part, a.chunk, n, dev_motion + 2 * f0,
                                          dev_scores ? dev_scores + f0 * g.V : nullptr, st))))
      return e;
  }
  return SEG_OK;
}

int seg_mc_estimate_static(seg_mc* mc, const uint16_t* dev_frames, uint64_t n_frames, int32_t* dev_motion,
                           double* dev_scores, void* stream) {
  int e = enter(mc);
  if (e) return e;
  if (!mc->have_template) return SEG_E_STATE;
  if (n_frames > (uint64_t)seg::kMcStaticFrames) return SEG_E_CAPACITY;
  if (n_frames == 0) return SEG_OK;
  if (!dev_frames || !dev_motion) return SEG_E_INVAL;
  const seg::McGeom& g = mc->g;
  if ((size_t)g.S * seg::kMcStaticFrames * g.Vp > seg::kMcStaticDoubles) return SEG_E_CAPACITY;
  if (!mc->scratch) return fail(mc, hipErrorInvalidSymbol);
  hipStream_t st = static_cast<hipStream_t>(stream);
  seg::McScoreArgs a{};
  a.g = g;
  a.frames = dev_frames;
  a.n = (int)n_frames;
  a.tmpl = at<uint16_t>(mc, mc->at_tmpl);
  a.sT = at<double>(mc, mc->at_sT);
  a.vT = at<double>(mc, mc->at_vT);
  a.part = mc->scratch;          // every entry the pick reads is written first
  a.chunk = seg::kMcStaticFrames;
  if ((e = fail(mc, seg::launch_mc_scores(a, st)))) return e;
  return fail(mc, seg::launch_mc_pick(g, a.part, a.chunk, a.n, dev_motion, dev_scores, st));
}

int seg_mc_apply(seg_mc* mc, const uint16_t* dev_frames, uint64_t n_frames, const int32_t* dev_motion,
                 uint16_t* dev_out, void* stream) {
  int e = enter(mc);
  if (e) return e;
  if (!mc->have_template) return SEG_E_STATE;
  if (n_frames == 0) return SEG_OK;
  if (!dev_frames || !dev_motion || !dev_out) return SEG_E_INVAL;
  const size_t bytes = n_frames * (size_t)mc->g.H * mc->g.W * 2;
  const char *a = reinterpret_cast<const char*>(dev_frames), *b = reinterpret_cast<const char*>(dev_out);
  if (a < b + bytes && b < a + bytes) return SEG_E_INVAL;
  return fail(mc, seg::launch_mc_apply(dev_frames, (long long)n_frames, mc->g.H, mc->g.W, dev_motion,
                                       at<uint16_t>(mc, mc->at_tmpl), dev_out, static_cast<hipStream_t>(stream)));
}

int seg_mc_destroy(seg_mc* mc) {
  delete mc;
  return SEG_OK;
}

}  // extern "C"
