// Host side of the C ABI declared in include/seg.h: configuration checks,
// workspace layout, the frame-to-segment bookkeeping of the streaming push,
// and the orchestration of the finalize kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "seg_internal.h"
#include "seg_traces.h"
#include "seg_nn.h"
#include "nn_internal.h"

using seg::Layout;
using seg::State;

namespace seg {
namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int check_config(const seg_config* c) {
  if (!c) return SEG_E_INVAL;
  if (c->height < 1 || c->width < 1 || c->height > (uint32_t)kMaxDim || c->width > (uint32_t)kMaxDim)
    return SEG_E_INVAL;
  if (c->seg_len != (uint32_t)kSegLen) return SEG_E_INVAL;
  if (c->max_frames < (uint32_t)kSegLen || c->max_frames / kSegLen > (uint32_t)kMaxSegments)
    return SEG_E_INVAL;
  const long long M = (long long)c->height * c->width;
  if ((long long)(c->max_frames / kSegLen) * M >= (1LL << 31)) return SEG_E_INVAL;
  if (!(c->gauss_sigma > 0.f) || c->gauss_radius < 1 || c->gauss_radius > (uint32_t)kMaxRadius)
    return SEG_E_INVAL;
  if (!(c->event_z >= 0.f) || c->min_event_segs < 1) return SEG_E_INVAL;
  if (c->area_min > c->area_max || c->area_max > 65536) return SEG_E_INVAL;
  if (!(c->solidity_min >= 0.f && c->solidity_min <= 1.f)) return SEG_E_INVAL;
  if (!(c->ecc_max >= 0.f && c->ecc_max <= 1.f)) return SEG_E_INVAL;
  if (c->nmf_max_rank < 1 || c->nmf_max_rank > (uint32_t)kMaxRank) return SEG_E_INVAL;
  if (!(c->spa_delta >= 0.f) || !(c->footprint_level > 0.f && c->footprint_level <= 1.f))
    return SEG_E_INVAL;
  if (!(c->sigma_floor >= 0.f)) return SEG_E_INVAL;
  if (c->detector != SEG_DET_PLAIN && c->detector != SEG_DET_SURROGATE && c->detector != SEG_DET_UNET)
    return SEG_E_INVAL;
  if (c->detector == SEG_DET_SURROGATE && (c->height % 4 || c->width % 4)) return SEG_E_INVAL;
  if (c->detector == SEG_DET_UNET && (c->height < 64 || c->width < 64)) return SEG_E_INVAL;
  if (c->nmf_path > SEG_NMF_SPLIT) return SEG_E_INVAL;
  return SEG_OK;
}

}  // namespace

Layout make_layout(const seg_config& c) {
  Layout l{};
  const size_t M = (size_t)c.height * c.width;
  const size_t K = c.max_frames / kSegLen;
  const size_t half = (size_t)((c.height + 1) / 2) * ((c.width + 1) / 2);
  l.Rcap = K * half;
  l.Ccap = half;
  l.scan_cap = (K * M + 1023) / 1024 + 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  l.tail = take((size_t)(kSegLen - 1) * M * 2);
  l.T = take(K * M * 4);
  l.S = take(K * M * 4);
  l.D = take(K * M * 4);
  l.U = take(K * M * 4);
  l.P = take(5 * K * M * 4);
  l.sigma = take(M * 8);
  l.corr = take(M * 4);
  l.mean = take(M * 4);
  l.count = take(M * 4);
  l.p = take(K * M * 4);
  l.lab = take(K * M * 4);
  l.rid = take(K * M * 4);
  l.bmask = take(K * M);
  l.reg_area = take(l.Rcap * 4);
  l.reg_sx = take(l.Rcap * 4);
  l.reg_sy = take(l.Rcap * 4);
  l.reg_sxx = take(l.Rcap * 8);
  l.reg_syy = take(l.Rcap * 8);
  l.reg_sxy = take(l.Rcap * 8);
  l.reg_box = take(l.Rcap * 16);
  l.reg_keep = take(l.Rcap);
  l.reg_root = take(l.Rcap * 4);
  l.nb = take(M * 4);
  l.blab = take(M * 4);
  l.comp = take(M * 4);
  l.scan = take(l.scan_cap * 4);
  l.counters = take(16 * 4);
  l.coff = take((M + 1) * 4);   // right after the counters: both come back in one copy
  l.pix = take(M * 4);
  l.cbox = take(l.Ccap * 16);
  l.nmf_P = take(M * K * 8);
  l.nmf_PT = take(M * K * 8);
  l.nmf_R = take(M * K * 8);
  l.nmf_F = take(M * kMaxRank * 8);
  l.nmf_G = take(M * kMaxRank * 8);
  l.nmf_A = take(l.Ccap * kMaxRank * K * 8);
  l.nmf_W = take(l.Ccap * 2 * K * 8);
  l.nmf_N = take(l.Ccap * 4);
  l.cmom = take(5 * M * 8);
  size_t stage = 0;
  if (c.detector == SEG_DET_SURROGATE) stage = (size_t)kSegLen * M * 2;
  if (c.detector == SEG_DET_UNET) {
    uint32_t np = 0;
    seg_nn_st_patch_count(c.height, c.width, &np);
    // patches (S, T) and their probabilities of kUnetGroup segments
    stage = (size_t)kUnetGroup * np * 3 * 4096 * 4;
  }
  l.stage = take(stage);
  l.total = o;
  return l;
}

}  // namespace seg

namespace {

template <class T>
T* at(seg_session* s, size_t off) {
  return reinterpret_cast<T*>(s->ws + off);
}

int fail(seg_session* s, hipError_t e);

// Surrogate detector: for each segment completed by this push, write the
// network's probability map into p[K + j]. A segment that straddles the
// carried tail and the caller's buffer is staged contiguously first; the
// others are read where they are, as many per network call as its batch.
int surrogate_maps(seg_session* s, const uint16_t* dev_frames, uint32_t nseg, hipStream_t st) {
  const size_t M = s->M;
  uint16_t* tail = at<uint16_t>(s, s->lay.tail);
  uint16_t* stage = at<uint16_t>(s, s->lay.stage);
  float* p = at<float>(s, s->lay.p);
  uint32_t B = 1;
  if (seg_nn_shape(s->net, &B, nullptr, nullptr) || B < 1) return fail(s, hipErrorUnknown);
  for (uint32_t j = 0; j < nseg;) {
    const long long f0 = (long long)j * seg::kSegLen;   // first frame, counted from the tail start
    const long long in_tail = std::max(0LL, std::min<long long>(seg::kSegLen, (long long)s->tail_n - f0));
    if (in_tail > 0) {
      // a segment that starts in the tail: staged contiguously, alone
      hipError_t he =
          hipMemcpyAsync(stage, tail + (size_t)f0 * M, (size_t)in_tail * M * 2, hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess && in_tail < seg::kSegLen) {
        const long long from = f0 + in_tail - (long long)s->tail_n;
        he = hipMemcpyAsync(stage + (size_t)in_tail * M, dev_frames + (size_t)from * M,
                            (size_t)(seg::kSegLen - in_tail) * M * 2, hipMemcpyDeviceToDevice, st);
      }
      if (fail(s, he)) return SEG_E_DEVICE;
      if (seg_nn_forward(s->net, stage, 1, p + (size_t)(s->K + j) * M, st)) return fail(s, hipErrorUnknown);
      ++j;
      continue;
    }
    // segments wholly in this push's frames lie back to back: up to the
    // network's batch of them in one call, read in place
    const uint32_t b = std::min(B, nseg - j);
    const uint16_t* src = dev_frames + (size_t)(f0 - (long long)s->tail_n) * M;
    if (seg_nn_forward(s->net, src, b, p + (size_t)(s->K + j) * M, st)) return fail(s, hipErrorUnknown);
    j += b;
  }
  return SEG_OK;
}

// Summary-image U-Net: for segments first .. first + nseg - 1 (whose S and T
// are written), cut the patches of up to kUnetGroup segments at a time, run
// the network over all of them in batches of its size (so the small
// low-resolution layers see more patches per launch), and merge each
// segment's patch probabilities into p[k].
int unet_maps(seg_session* s, uint32_t first, uint32_t nseg, hipStream_t st) {
  const size_t M = s->M;
  const uint32_t H = s->cfg.height, W = s->cfg.width;
  uint32_t np = 0, B = 0;
  if (seg_nn_st_patch_count(H, W, &np) || seg_nn_shape(s->net, &B, nullptr, nullptr)) return fail(s, hipErrorUnknown);
  float* in = at<float>(s, s->lay.stage);
  float* prob = in + (size_t)seg::kUnetGroup * np * 2 * 4096;
  for (uint32_t j0 = 0; j0 < nseg; j0 += seg::kUnetGroup) {
    const uint32_t g = std::min<uint32_t>(seg::kUnetGroup, nseg - j0);
    // the group's patches, and below its maps, in one launch each
    seg::nn::st_patches_n(at<float>(s, s->lay.S) + (first + j0) * M, at<float>(s, s->lay.T) + (first + j0) * M,
                          (int)H, (int)W, (int)g, in, st);
    const uint32_t total = g * np;
    for (uint32_t a = 0; a < total; a += B) {
      const uint32_t b = std::min(B, total - a);
      if (seg_nn_st_forward(s->net, in + (size_t)a * 2 * 4096, b, prob + (size_t)a * 4096, st))
        return fail(s, hipErrorUnknown);
    }
    seg::nn::st_merge_n(prob, (int)H, (int)W, (int)g, at<float>(s, s->lay.p) + (first + j0) * M, st);
    if (hipGetLastError() != hipSuccess) return fail(s, hipErrorUnknown);
  }
  return SEG_OK;
}

int fail(seg_session* s, hipError_t e) {
  if (e == hipSuccess) return SEG_OK;
  s->error = SEG_E_DEVICE;
  s->state = State::Failed;
  return SEG_E_DEVICE;
}

int enter(seg_session* s) {
  if (!s) return SEG_E_INVAL;
  if (s->state == State::Failed) return SEG_E_DEVICE;
  if (hipSetDevice(s->device) != hipSuccess) return fail(s, hipErrorInvalidDevice);
  return SEG_OK;
}

}  // namespace

extern "C" {

int seg_default_config(uint32_t height, uint32_t width, uint32_t max_frames, seg_config* out) {
  if (!out || height == 0 || width == 0) return SEG_E_INVAL;
  seg_config c{};
  c.height = height;
  c.width = width;
  c.seg_len = seg::kSegLen;
  c.max_frames = max_frames;
  c.gauss_sigma = 3.0f;
  c.gauss_radius = 12;
  c.event_z = 5.0f;
  c.min_event_segs = 2;
  c.area_min = 16;
  c.area_max = 1600;
  c.solidity_min = 0.75f;
  c.ecc_max = 0.95f;
  c.nmf_max_rank = 6;
  c.nmf_sweeps = 200;
  c.spa_delta = 0.3f;
  c.footprint_level = 0.25f;
  c.sigma_floor = 1e-3f;
  c.detector = SEG_DET_PLAIN;
  c.nmf_path = SEG_NMF_AUTO;
  *out = c;
  return SEG_OK;
}

int seg_workspace_bytes(const seg_config* cfg, size_t* bytes) {
  if (!bytes) return SEG_E_INVAL;
  const int e = seg::check_config(cfg);
  if (e) return e;
  *bytes = seg::make_layout(*cfg).total;
  return SEG_OK;
}

int seg_create(const seg_config* cfg, void* dev_workspace, size_t bytes, seg_session** out) {
  if (!out || !dev_workspace) return SEG_E_INVAL;
  *out = nullptr;
  const int e = seg::check_config(cfg);
  if (e) return e;
  if (reinterpret_cast<uintptr_t>(dev_workspace) & 255) return SEG_E_INVAL;
  Layout lay = seg::make_layout(*cfg);
  if (bytes < lay.total) return SEG_E_CAPACITY;
  seg_session* s = new (std::nothrow) seg_session();
  if (!s) return SEG_E_INVAL;
  s->cfg = *cfg;
  s->lay = lay;
  s->ws = static_cast<char*>(dev_workspace);
  s->ws_bytes = bytes;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return SEG_E_DEVICE;
  }
  s->M = cfg->height * cfg->width;
  s->Kmax = cfg->max_frames / seg::kSegLen;
  s->frames = 0;
  s->K = 0;
  s->tail_n = 0;
  s->state = State::Open;
  s->error = SEG_OK;
  s->n_comp = 0;
  s->net = nullptr;
  // smoothing taps: exp(-k^2 / (2 sigma^2)) normalised over |k| <= radius
  const int r = (int)cfg->gauss_radius;
  const double sg = (double)cfg->gauss_sigma;
  double sum = 0.0;
  for (int k = -r; k <= r; ++k) sum += std::exp(-(double)(k * k) / (2.0 * sg * sg));
  for (int k = -seg::kMaxRadius; k <= seg::kMaxRadius; ++k)
    s->w[k + seg::kMaxRadius] =
        (k >= -r && k <= r) ? std::exp(-(double)(k * k) / (2.0 * sg * sg)) / sum : 0.0;
  s->have_ev = true;
  for (int k = 0; k < 4; ++k)
    if (hipEventCreate(&s->ev[k]) != hipSuccess) {
      for (int j = 0; j < k; ++j) (void)hipEventDestroy(s->ev[j]);
      delete s;
      return SEG_E_DEVICE;
    }
  s->prof = seg_profile{};
  *out = s;
  return SEG_OK;
}

int seg_push_frames(seg_session* s, const uint16_t* dev_frames, uint32_t n, void* stream) {
  int e = enter(s);
  if (e) return e;
  if (s->state != State::Open) return SEG_E_STATE;
  if (n == 0) return SEG_OK;
  if (!dev_frames) return SEG_E_INVAL;
  if (s->cfg.detector != SEG_DET_PLAIN && !s->net) return SEG_E_NOMODEL;
  if (s->frames + n > s->cfg.max_frames) return SEG_E_CAPACITY;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long M = s->M;
  const uint32_t total = s->tail_n + n;
  const uint32_t nseg = total / seg::kSegLen;
  const uint32_t rem = total - nseg * seg::kSegLen;
  uint16_t* tail = at<uint16_t>(s, s->lay.tail);
  if (nseg > 0) {
    seg::StreamLaunch a{};
    a.src0 = tail;
    a.src1 = dev_frames;
    a.n0 = s->tail_n;
    a.H = (int)s->cfg.height;
    a.W = (int)s->cfg.width;
    a.seg0 = (int)s->K;
    a.nseg = (int)nseg;
    a.T = at<float>(s, s->lay.T);
    a.S = at<float>(s, s->lay.S);
    a.D = at<float>(s, s->lay.D);
    a.U = at<float>(s, s->lay.U);
    a.P = at<float>(s, s->lay.P);
    a.plane = (long long)s->Kmax * M;
    a.w = s->w;
    if ((e = fail(s, seg::launch_block_stats(a, st)))) return e;
    if (s->cfg.detector == SEG_DET_SURROGATE && (e = surrogate_maps(s, dev_frames, nseg, st))) return e;
    if (s->cfg.detector == SEG_DET_UNET && (e = unet_maps(s, s->K, nseg, st))) return e;
    if (rem) {
      const uint16_t* from = dev_frames + (size_t)(n - rem) * M;
      if ((e = fail(s, hipMemcpyAsync(tail, from, (size_t)rem * M * 2, hipMemcpyDeviceToDevice, st))))
        return e;
    }
  } else {
    if ((e = fail(s, hipMemcpyAsync(tail + (size_t)s->tail_n * M, dev_frames, (size_t)n * M * 2,
                                    hipMemcpyDeviceToDevice, st))))
      return e;
  }
  s->K += nseg;
  s->tail_n = rem;
  s->frames += n;
  return SEG_OK;
}

int seg_load_summaries(seg_session* s, uint32_t k, const float* T, const float* S, const float* D,
                       const float* U, const float* P) {
  int e = enter(s);
  if (e) return e;
  if (s->state != State::Open || s->frames != 0 || s->K != 0) return SEG_E_STATE;
  if (!T || !S || !D || k == 0) return SEG_E_INVAL;
  if (k > s->Kmax) return SEG_E_CAPACITY;
  if (s->cfg.detector == SEG_DET_SURROGATE) return SEG_E_STATE;   // its maps need the frames
  if (s->cfg.detector == SEG_DET_UNET && !s->net) return SEG_E_NOMODEL;
  const size_t n = (size_t)k * s->M * 4;
  if ((e = fail(s, hipMemcpy(at<float>(s, s->lay.T), T, n, hipMemcpyHostToDevice)))) return e;
  if ((e = fail(s, hipMemcpy(at<float>(s, s->lay.S), S, n, hipMemcpyHostToDevice)))) return e;
  if ((e = fail(s, hipMemcpy(at<float>(s, s->lay.D), D, n, hipMemcpyHostToDevice)))) return e;
  const bool mom = U && P;
  if (mom) {
    if ((e = fail(s, hipMemcpy(at<float>(s, s->lay.U), U, n, hipMemcpyHostToDevice)))) return e;
    for (int o = 0; o < 5; ++o) {
      float* dst = at<float>(s, s->lay.P) + (size_t)o * s->Kmax * s->M;
      if ((e = fail(s, hipMemcpy(dst, P + (size_t)o * k * s->M, n, hipMemcpyHostToDevice)))) return e;
    }
  } else {
    // no co-moments: zero sums give a zero correlation image
    if ((e = fail(s, hipMemset(at<float>(s, s->lay.U), 0, n)))) return e;
    for (int o = 0; o < 5; ++o)
      if ((e = fail(s, hipMemset(at<float>(s, s->lay.P) + (size_t)o * s->Kmax * s->M, 0, n)))) return e;
  }
  if (s->cfg.detector == SEG_DET_UNET) {
    if ((e = unet_maps(s, 0, k, nullptr))) return e;
    if ((e = fail(s, hipStreamSynchronize(nullptr)))) return e;
  }
  s->K = k;
  s->frames = (uint64_t)k * seg::kSegLen;
  return SEG_OK;
}

int seg_num_segments(const seg_session* s, uint32_t* k) {
  if (!s || !k) return SEG_E_INVAL;
  *k = s->K;
  return SEG_OK;
}

int seg_finalize(seg_session* s, void* stream) {
  int e = enter(s);
  if (e) return e;
  if (s->state != State::Open || s->K == 0) return SEG_E_STATE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout& l = s->lay;
  const seg_config& c = s->cfg;
  seg::FinalizeArgs a{};
  a.H = (int)c.height;
  a.W = (int)c.width;
  a.M = (int)s->M;
  a.K = (int)s->K;
  a.Kmax = (int)s->Kmax;
  a.T = at<float>(s, l.T);
  a.S = at<float>(s, l.S);
  a.D = at<float>(s, l.D);
  a.U = at<float>(s, l.U);
  a.P = at<float>(s, l.P);
  a.plane = (long long)s->Kmax * s->M;
  a.sigma = at<double>(s, l.sigma);
  a.corr = at<float>(s, l.corr);
  a.mean = at<float>(s, l.mean);
  a.count = at<int>(s, l.count);
  a.p = at<float>(s, l.p);
  a.lab = at<int>(s, l.lab);
  a.rid = at<int>(s, l.rid);
  a.bmask = at<uint8_t>(s, l.bmask);
  a.reg_area = at<uint32_t>(s, l.reg_area);
  a.reg_sx = at<uint32_t>(s, l.reg_sx);
  a.reg_sy = at<uint32_t>(s, l.reg_sy);
  a.reg_sxx = at<unsigned long long>(s, l.reg_sxx);
  a.reg_syy = at<unsigned long long>(s, l.reg_syy);
  a.reg_sxy = at<unsigned long long>(s, l.reg_sxy);
  a.reg_box = at<int>(s, l.reg_box);
  a.reg_keep = at<uint8_t>(s, l.reg_keep);
  a.nb = at<int>(s, l.nb);
  a.blab = at<int>(s, l.blab);
  a.comp = at<int>(s, l.comp);
  a.pix = at<int>(s, l.pix);
  a.coff = at<int>(s, l.coff);
  a.cbox = at<int>(s, l.cbox);
  a.Ccap = (int)l.Ccap;
  a.scan = at<int>(s, l.scan);
  a.counters = at<int>(s, l.counters);
  a.Rcap = (long long)l.Rcap;
  a.scan_cap = (int)l.scan_cap;
  a.C = at<double>(s, l.cmom);
  a.root = at<int>(s, l.reg_root);
  a.theta = (double)c.event_z;
  a.sigma_floor = (double)c.sigma_floor;
  a.solidity_min = (double)c.solidity_min;
  a.ecc_thr = 1.0 - (double)c.ecc_max * (double)c.ecc_max;
  a.area_min = (int)c.area_min;
  a.area_max = (int)c.area_max;
  a.min_event_segs = (int)c.min_event_segs;
  a.have_moments = true;
  a.prob_mode = c.detector != SEG_DET_PLAIN;
  s->prof = seg_profile{};
  bool nmf_timed = false;
  if ((e = fail(s, hipEventRecord(s->ev[0], st)))) return e;
  if ((e = fail(s, seg::launch_finalize_maps(a, st)))) return e;
  if ((e = fail(s, hipEventRecord(s->ev[1], st)))) return e;
  // component count and offsets (the pixel lists stay on the device for the
  // NMF): the counters and the first few thousand offsets, which follow them
  // in the workspace, in one copy
  int ncomp = 0;
  std::vector<int> coff(std::min<size_t>(s->M + 1, 4097));
  {
    const size_t gap = l.coff - l.counters, bytes = gap + coff.size() * 4;
    std::vector<int> head((bytes + 3) / 4);
    if ((e = fail(s, hipMemcpyAsync(head.data(), a.counters, bytes, hipMemcpyDeviceToHost, st)))) return e;
    if ((e = fail(s, hipStreamSynchronize(st)))) return e;
    ncomp = head[0];
    std::memcpy(coff.data(), head.data() + gap / 4, coff.size() * 4);
  }
  if ((size_t)ncomp + 1 > coff.size()) {
    coff.resize((size_t)ncomp + 1);
    if ((e = fail(s, hipMemcpyAsync(coff.data(), a.coff, coff.size() * 4, hipMemcpyDeviceToHost, st)))) return e;
    if ((e = fail(s, hipStreamSynchronize(st)))) return e;
  }
  coff.resize((size_t)ncomp + 1);
  std::vector<int> pix(coff[ncomp]);
  s->n_comp = (uint32_t)ncomp;
  s->fps.clear();
  if (ncomp > 0) {
    int* dpix = a.pix;
    int* dcoff = a.coff;
    seg::NmfArgs na{};
    na.M = (int)s->M;
    na.K = (int)s->K;
    na.Kmax = (int)s->Kmax;
    na.ncomp = ncomp;
    na.p = a.p;
    na.pix = dpix;
    na.coff = dcoff;
    na.P = at<double>(s, l.nmf_P);
    na.PT = at<double>(s, l.nmf_PT);
    na.R = at<double>(s, l.nmf_R);
    na.F = at<double>(s, l.nmf_F);
    na.A = at<double>(s, l.nmf_A);
    na.G = at<double>(s, l.nmf_G);
    na.Wk = at<double>(s, l.nmf_W);
    na.N = at<int>(s, l.nmf_N);
    na.max_rank = (int)c.nmf_max_rank;
    na.sweeps = (int)c.nmf_sweeps;
    na.delta = (double)c.spa_delta;
    // split path: the exchange slots reuse the pixel-major P_c area, the
    // workgroup tables the SPA-direction area and the abandon and error flags the
    // SPA-flag area (all three belong to the single-workgroup kernel)
    seg::NmfSplit sp{};
    seg::NmfSplitTables tabs;
    bool split = c.nmf_path != SEG_NMF_SINGLE &&
                 seg::plan_nmf_split(sp, na, coff, (size_t)s->M * s->Kmax * 8, tabs);
    if (!split && c.nmf_path == SEG_NMF_SPLIT) return SEG_E_CAPACITY;
    // cooperative grids of concurrent finalizes could each hold part of the
    // device while waiting for the rest: one split NMF at a time per process
    static std::mutex split_mutex;
    std::unique_lock<std::mutex> hold(split_mutex, std::defer_lock);
    std::vector<int> up;   // host tables of the split launch (kept until the stream is synchronised)
    if (split) {
      int* tab = at<int>(s, l.nmf_G);
      const size_t G = tabs.comp.size();
      // the four tables in one upload: comp [G], base [ncomp], n [ncomp], rank [G]
      up.reserve(2 * G + 2 * (size_t)ncomp);
      up.insert(up.end(), tabs.comp.begin(), tabs.comp.end());
      up.insert(up.end(), tabs.base.begin(), tabs.base.end());
      up.insert(up.end(), tabs.n.begin(), tabs.n.end());
      up.insert(up.end(), tabs.rank.begin(), tabs.rank.end());
      if ((e = fail(s, hipMemcpyAsync(tab, up.data(), up.size() * 4, hipMemcpyHostToDevice, st)))) return e;
      int* rank = tab + G + 2 * (size_t)ncomp;
      sp.wg_base = tab + G;
      sp.wg_n = tab + G + ncomp;
      sp.xbuf = reinterpret_cast<unsigned long long*>(na.P);
      sp.sync = reinterpret_cast<unsigned*>(na.Wk);
      hold.lock();
      if ((e = fail(s, hipEventRecord(s->ev[2], st)))) return e;
      // launches in order on the stream; each reuses the slots and counters
      hipError_t le = hipSuccess;
      for (size_t gi = 0; gi < tabs.groups.size(); ++gi) {
        seg::NmfSplit one = sp;
        one.G = tabs.groups[gi].second;
        one.wg_comp = tab + tabs.groups[gi].first;
        one.wg_rank = rank + tabs.groups[gi].first;
        le = seg::launch_nmf_split(na, one, gi == 0, st);
        if (le != hipSuccess) break;
      }
      if (le != hipSuccess) {
        (void)hipGetLastError();
        hold.unlock();
        if (c.nmf_path == SEG_NMF_SPLIT || le != hipErrorCooperativeLaunchTooLarge) return fail(s, le);
        split = false;  // the device is shared: one workgroup per component
      }
    }
    if (!split) {
      int max_mc = 0;
      for (int k = 0; k < ncomp; ++k) max_mc = std::max(max_mc, coff[k + 1] - coff[k]);
      seg::plan_nmf(na, max_mc);
      if ((e = fail(s, hipEventRecord(s->ev[2], st)))) return e;
      if ((e = fail(s, seg::launch_nmf(na, st)))) return e;
    }
    if ((e = fail(s, hipEventRecord(s->ev[3], st)))) return e;
    nmf_timed = true;
    const size_t npx = pix.size();
    std::vector<int> N(ncomp);
    std::vector<double> F(npx * seg::kMaxRank), A((size_t)ncomp * seg::kMaxRank * s->Kmax);
    unsigned split_error = 0;
    // The results (error flag, ranks, pixel lists, F, A) are packed by
    // device-to-device copies into the P_c area, free after the NMF, and come
    // back in one copy: each copy into pageable host memory waits for the
    // device, so five of them cost five round trips.
    const size_t o_err = 0, o_n = 8, o_pix = seg::align_up(o_n + (size_t)ncomp * 4),
                 o_f = seg::align_up(o_pix + npx * 4), o_a = o_f + F.size() * 8, packed = o_a + A.size() * 8;
    if (packed <= (size_t)s->M * s->Kmax * 8) {
      char* dst = reinterpret_cast<char*>(na.P);
      hipError_t he = hipSuccess;
      if (split) he = hipMemcpyAsync(dst + o_err, sp.sync + ncomp, 4, hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(dst + o_n, na.N, (size_t)ncomp * 4, hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(dst + o_pix, dpix, npx * 4, hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(dst + o_f, na.F, F.size() * 8, hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(dst + o_a, na.A, A.size() * 8, hipMemcpyDeviceToDevice, st);
      std::vector<double> host((packed + 7) / 8);
      if (he == hipSuccess) he = hipMemcpyAsync(host.data(), dst, packed, hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if ((e = fail(s, he))) return e;
      const char* h = reinterpret_cast<const char*>(host.data());
      if (split) std::memcpy(&split_error, h + o_err, 4);
      std::memcpy(N.data(), h + o_n, (size_t)ncomp * 4);
      std::memcpy(pix.data(), h + o_pix, npx * 4);
      std::memcpy(F.data(), h + o_f, F.size() * 8);
      std::memcpy(A.data(), h + o_a, A.size() * 8);
    } else {
      if ((e = fail(s, hipMemcpyAsync(N.data(), na.N, ncomp * 4, hipMemcpyDeviceToHost, st)))) return e;
      if ((e = fail(s, hipMemcpyAsync(pix.data(), dpix, pix.size() * 4, hipMemcpyDeviceToHost, st)))) return e;
      if ((e = fail(s, hipMemcpyAsync(F.data(), na.F, F.size() * 8, hipMemcpyDeviceToHost, st)))) return e;
      if ((e = fail(s, hipMemcpyAsync(A.data(), na.A, A.size() * 8, hipMemcpyDeviceToHost, st)))) return e;
      if (split && (e = fail(s, hipMemcpyAsync(&split_error, sp.sync + ncomp, 4, hipMemcpyDeviceToHost, st))))
        return e;
      if ((e = fail(s, hipStreamSynchronize(st)))) return e;
    }
    if (hold.owns_lock()) hold.unlock();
    if (split_error) return fail(s, hipErrorLaunchTimeOut);  // a wait for a slot was abandoned
    // algorithmic work of the NMF (seg_profile)
    {
      const double Kd = (double)s->K, S = (double)c.nmf_sweeps;
      double fl = 0.0;
      uint32_t rmax = 0;
      for (int k = 0; k < ncomp; ++k) {
        const double Mc = (double)(coff[k + 1] - coff[k]), Nn = (double)N[k];
        rmax = std::max(rmax, (uint32_t)N[k]);
        fl += (6.0 * Nn + 2.0) * Mc * Kd;                                   // SPA
        if (N[k] == 0) continue;
        fl += (S + 1.0) * (2.0 * Mc * Kd * Nn + Mc * Nn * (Nn + 1.0) + 2.0 * Kd * Nn * Nn);  // A updates
        fl += S * (2.0 * Mc * Kd * Nn + Kd * Nn * (Nn + 1.0) + 2.0 * Mc * Nn * Nn);          // F updates
      }
      s->prof.nmf_flops = fl;
      s->prof.max_rank = rmax;
      s->prof.nmf_path = split ? SEG_NMF_SPLIT : SEG_NMF_SINGLE;
      s->prof.nmf_workgroups = split ? (uint32_t)sp.G : (uint32_t)ncomp;
    }
    const double level = (double)c.footprint_level;
    for (int k = 0; k < ncomp; ++k) {
      const int off = coff[k], Mc = coff[k + 1] - coff[k];
      std::vector<seg::Footprint> items;
      for (int n = 0; n < N[k]; ++n) {
        double mx = 0.0;
        int arg = 0;
        for (int m = 0; m < Mc; ++m) {
          const double v = F[(size_t)(off + m) * seg::kMaxRank + n];
          if (v > mx) {
            mx = v;
            arg = m;
          }
        }
        if (mx <= 0.0) continue;
        uint32_t area = 0;
        for (int m = 0; m < Mc; ++m) area += F[(size_t)(off + m) * seg::kMaxRank + n] >= level;
        if (area < c.area_min) continue;
        seg::Footprint fp;
        fp.component = k + 1;
        fp.peak = pix[off + arg];
        fp.w.resize(Mc);
        fp.on.resize(Mc);
        for (int m = 0; m < Mc; ++m) {
          const double v = F[(size_t)(off + m) * seg::kMaxRank + n];
          fp.w[m] = (float)v;
          fp.on[m] = v >= level;
        }
        fp.activity.resize(s->K);
        for (uint32_t i = 0; i < s->K; ++i)
          fp.activity[i] = (float)A[((size_t)k * seg::kMaxRank + n) * s->Kmax + i];
        items.push_back(std::move(fp));
      }
      std::stable_sort(items.begin(), items.end(),
                       [](const seg::Footprint& x, const seg::Footprint& y) { return x.peak < y.peak; });
      for (auto& it : items) s->fps.push_back(std::move(it));
    }
    // trace tables: per component with footprints, the pixels in at least
    // one mask and their mask bits (footprints of a component are adjacent)
    for (size_t j = 0; j < s->fps.size();) {
      const int k = s->fps[j].component - 1, off = coff[k], Mc = coff[k + 1] - coff[k];
      size_t e = j;
      while (e < s->fps.size() && s->fps[e].component == k + 1) ++e;
      const int begin = (int)s->tr_pix.size();
      for (int m = 0; m < Mc; ++m) {
        uint32_t b = 0;
        for (size_t q = j; q < e; ++q) b |= (uint32_t)s->fps[q].on[m] << (q - j);
        if (!b) continue;
        s->tr_pix.push_back(pix[off + m]);
        s->tr_bits.push_back((uint8_t)b);
      }
      s->tr_comp.insert(s->tr_comp.end(), {begin, (int)s->tr_pix.size(), (int)j, (int)(e - j)});
      for (size_t q = j; q < e; ++q) {
        uint32_t area = 0;
        for (uint8_t o : s->fps[q].on) area += o;
        s->tr_count.push_back(area);
      }
      j = e;
    }
    s->comp_pix = std::move(pix);
    s->comp_off = std::move(coff);
  }
  s->prof.components = (uint32_t)ncomp;
  {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev[0], s->ev[1]) == hipSuccess) s->prof.maps_ms = ms;
    if (nmf_timed && hipEventElapsedTime(&ms, s->ev[2], s->ev[3]) == hipSuccess) s->prof.nmf_ms = ms;
  }
  s->state = State::Finalized;
  return SEG_OK;
}

int seg_get_footprints(seg_session* s, uint32_t capacity, uint32_t* n_out, float* weights, uint8_t* masks,
                       float* activity, int32_t* component) {
  if (!s) return SEG_E_INVAL;
  if (s->state == State::Failed) return SEG_E_DEVICE;
  if (s->state != State::Finalized) return SEG_E_STATE;
  if (n_out) *n_out = (uint32_t)s->fps.size();
  const uint32_t n = std::min<uint32_t>(capacity, (uint32_t)s->fps.size());
  for (uint32_t j = 0; j < n; ++j) {
    const seg::Footprint& f = s->fps[j];
    const int off = s->comp_off[f.component - 1];
    const int* px = s->comp_pix.data() + off;
    const size_t Mc = f.w.size();
    if (weights) {
      float* wj = weights + (size_t)j * s->M;
      std::memset(wj, 0, (size_t)s->M * 4);
      for (size_t m = 0; m < Mc; ++m) wj[px[m]] = f.w[m];
    }
    if (masks) {
      uint8_t* mj = masks + (size_t)j * s->M;
      std::memset(mj, 0, s->M);
      for (size_t m = 0; m < Mc; ++m) mj[px[m]] = f.on[m];
    }
    if (activity) std::memcpy(activity + (size_t)j * s->K, f.activity.data(), (size_t)s->K * 4);
    if (component) component[j] = f.component;
  }
  return SEG_OK;
}

int seg_extract_traces(seg_session* s, const uint16_t* dev_frames, uint64_t n_frames, float* dev_out,
                       uint64_t ld, void* stream) {
  int e = enter(s);
  if (e) return e;
  if (s->state != State::Finalized) return SEG_E_STATE;
  if (ld < n_frames || n_frames > (uint64_t)INT64_MAX / 2) return SEG_E_INVAL;
  if (n_frames == 0 || s->fps.empty()) return SEG_OK;
  if (!dev_frames || !dev_out) return SEG_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!s->tr_ready) {
    // the NMF factor region is free once the footprints are on the host
    const size_t n = s->tr_pix.size(), nc = s->tr_comp.size() / 4, base = s->lay.nmf_F;
    s->tr_at[0] = base;
    s->tr_at[1] = s->tr_at[0] + seg::align_up(n * 4);
    s->tr_at[2] = s->tr_at[1] + seg::align_up(n);
    s->tr_at[3] = s->tr_at[2] + seg::align_up(nc * 16);
    if (s->tr_at[3] + s->tr_count.size() * 4 > base + (size_t)s->M * seg::kMaxRank * 8) return SEG_E_CAPACITY;
    const void* src[4] = {s->tr_pix.data(), s->tr_bits.data(), s->tr_comp.data(), s->tr_count.data()};
    const size_t len[4] = {n * 4, n, nc * 16, s->tr_count.size() * 4};
    for (int i = 0; i < 4; ++i)
      if (len[i] && (e = fail(s, hipMemcpyAsync(s->ws + s->tr_at[i], src[i], len[i], hipMemcpyHostToDevice, st))))
        return e;
    if ((e = fail(s, hipStreamSynchronize(st)))) return e;
    s->tr_ready = true;
  }
  seg::TraceArgs a{};
  a.frames = dev_frames;
  a.n_frames = (long long)n_frames;
  a.M = (int)s->M;
  a.ncomp = (int)(s->tr_comp.size() / 4);
  a.max_fp = 1;
  for (int k = 0; k < a.ncomp; ++k) a.max_fp = std::max(a.max_fp, s->tr_comp[4 * k + 3]);
  a.pix = at<int>(s, s->tr_at[0]);
  a.bits = at<uint8_t>(s, s->tr_at[1]);
  a.comp = at<int4>(s, s->tr_at[2]);
  a.count = at<uint32_t>(s, s->tr_at[3]);
  a.out = dev_out;
  a.ld = (long long)ld;
  return fail(s, seg::launch_traces(a, st));
}

int seg_get_image(seg_session* s, int kind, void* host_out) {
  int e = enter(s);
  if (e) return e;
  if (!host_out) return SEG_E_INVAL;
  if (s->state != State::Finalized) return SEG_E_STATE;
  const Layout& l = s->lay;
  const size_t M = s->M;
  switch (kind) {
    case SEG_IMG_MEAN:
      return fail(s, hipMemcpy(host_out, s->ws + l.mean, M * 4, hipMemcpyDeviceToHost));
    case SEG_IMG_CORR:
      return fail(s, hipMemcpy(host_out, s->ws + l.corr, M * 4, hipMemcpyDeviceToHost));
    case SEG_IMG_NOISE: {
      std::vector<double> tmp(M);
      if ((e = fail(s, hipMemcpy(tmp.data(), s->ws + l.sigma, M * 8, hipMemcpyDeviceToHost)))) return e;
      float* o = static_cast<float*>(host_out);
      for (size_t x = 0; x < M; ++x) o[x] = (float)tmp[x];
      return SEG_OK;
    }
    case SEG_IMG_EVENT_COUNT:
      return fail(s, hipMemcpy(host_out, s->ws + l.count, M * 4, hipMemcpyDeviceToHost));
    case SEG_IMG_MASK_COUNT:
      return fail(s, hipMemcpy(host_out, s->ws + l.nb, M * 4, hipMemcpyDeviceToHost));
    case SEG_IMG_LABELS:
      return fail(s, hipMemcpy(host_out, s->ws + l.comp, M * 4, hipMemcpyDeviceToHost));
    default:
      return SEG_E_INVAL;
  }
}

int seg_get_segment_maps(seg_session* s, int kind, uint32_t first, uint32_t count, float* dev_out,
                         void* stream) {
  int e = enter(s);
  if (e) return e;
  if (!dev_out) return SEG_E_INVAL;
  if ((uint64_t)first + count > s->K) return SEG_E_INVAL;
  const Layout& l = s->lay;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t M = s->M;
  size_t base;
  switch (kind) {
    case SEG_MAP_S: base = l.S; break;
    case SEG_MAP_T: base = l.T; break;
    case SEG_MAP_D: base = l.D; break;
    case SEG_MAP_P:
      if (s->state != State::Finalized) return SEG_E_STATE;
      base = l.p;
      break;
    case SEG_MAP_B:
      if (s->state != State::Finalized) return SEG_E_STATE;
      return fail(s, seg::launch_u8_to_f32(at<uint8_t>(s, l.bmask) + (size_t)first * M, dev_out,
                                           (long long)count * M, st));
    default:
      return SEG_E_INVAL;
  }
  return fail(s, hipMemcpyAsync(dev_out, s->ws + base + (size_t)first * M * 4, (size_t)count * M * 4,
                                hipMemcpyDeviceToDevice, st));
}

int seg_destroy(seg_session* s) {
  if (s && s->have_ev)
    for (int k = 0; k < 4; ++k) (void)hipEventDestroy(s->ev[k]);
  delete s;
  return SEG_OK;
}

// ---- checkpoint / resume: header, carried frames, per-segment planes
namespace {

struct StateHeader {
  char magic[8];
  uint32_t version;
  uint32_t planes;        // FP32 [K][M] planes that follow the carried frames
  uint64_t frames;
  uint32_t K, tail_n;
  seg_config cfg;
};
constexpr char kStateMagic[8] = {'S', 'E', 'G', 'S', 'T', 'A', 'T', 'E'};

// T, S, D, U, the five co-moment planes, and the probability maps of the
// surrogate detector
uint32_t state_planes(const seg_session* s) { return s->cfg.detector != SEG_DET_PLAIN ? 10u : 9u; }

float* state_plane(seg_session* s, uint32_t j) {
  const Layout& l = s->lay;
  const size_t KM = (size_t)s->Kmax * s->M;
  switch (j) {
    case 0: return at<float>(s, l.T);
    case 1: return at<float>(s, l.S);
    case 2: return at<float>(s, l.D);
    case 3: return at<float>(s, l.U);
    case 9: return at<float>(s, l.p);
    default: return at<float>(s, l.P) + (size_t)(j - 4) * KM;   // co-moment planes 0..4
  }
}

size_t state_size(const seg_session* s) {
  return sizeof(StateHeader) + (size_t)s->tail_n * s->M * 2 +
         (size_t)state_planes(s) * s->K * s->M * 4;
}

}  // namespace

int seg_state_bytes(const seg_session* s, size_t* bytes) {
  if (!s || !bytes) return SEG_E_INVAL;
  *bytes = state_size(s);
  return SEG_OK;
}

int seg_export_state(seg_session* s, void* host, size_t bytes, void* stream) {
  int e = enter(s);
  if (e) return e;
  if (!host) return SEG_E_INVAL;
  if (s->state != State::Open) return SEG_E_STATE;
  if (bytes < state_size(s)) return SEG_E_CAPACITY;
  hipStream_t st = static_cast<hipStream_t>(stream);
  StateHeader h{};
  std::memcpy(h.magic, kStateMagic, 8);
  h.version = 1;
  h.planes = state_planes(s);
  h.frames = s->frames;
  h.K = s->K;
  h.tail_n = s->tail_n;
  h.cfg = s->cfg;
  char* out = static_cast<char*>(host);
  std::memcpy(out, &h, sizeof h);
  out += sizeof h;
  const size_t tb = (size_t)s->tail_n * s->M * 2;
  if (tb && (e = fail(s, hipMemcpyAsync(out, s->ws + s->lay.tail, tb, hipMemcpyDeviceToHost, st)))) return e;
  out += tb;
  const size_t pb = (size_t)s->K * s->M * 4;
  for (uint32_t j = 0; j < h.planes && pb; ++j, out += pb)
    if ((e = fail(s, hipMemcpyAsync(out, state_plane(s, j), pb, hipMemcpyDeviceToHost, st)))) return e;
  return fail(s, hipStreamSynchronize(st));
}

int seg_import_state(seg_session* s, const void* host, size_t bytes, void* stream) {
  int e = enter(s);
  if (e) return e;
  if (!host || bytes < sizeof(StateHeader)) return host ? SEG_E_CAPACITY : SEG_E_INVAL;
  if (s->state != State::Open || s->frames != 0 || s->K != 0 || s->tail_n != 0) return SEG_E_STATE;
  StateHeader h;
  std::memcpy(&h, host, sizeof h);
  if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.version != 1) return SEG_E_INVAL;
  if (std::memcmp(&h.cfg, &s->cfg, sizeof(seg_config)) != 0 || h.planes != state_planes(s)) return SEG_E_INVAL;
  if (h.K > s->Kmax || h.tail_n >= (uint32_t)seg::kSegLen ||
      h.frames != (uint64_t)h.K * seg::kSegLen + h.tail_n)
    return SEG_E_INVAL;
  const size_t need = sizeof h + (size_t)h.tail_n * s->M * 2 + (size_t)h.planes * h.K * s->M * 4;
  if (bytes < need) return SEG_E_CAPACITY;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const char* in = static_cast<const char*>(host) + sizeof h;
  const size_t tb = (size_t)h.tail_n * s->M * 2;
  if (tb && (e = fail(s, hipMemcpyAsync(s->ws + s->lay.tail, in, tb, hipMemcpyHostToDevice, st)))) return e;
  in += tb;
  const size_t pb = (size_t)h.K * s->M * 4;
  for (uint32_t j = 0; j < h.planes && pb; ++j, in += pb)
    if ((e = fail(s, hipMemcpyAsync(state_plane(s, j), in, pb, hipMemcpyHostToDevice, st)))) return e;
  if ((e = fail(s, hipStreamSynchronize(st)))) return e;
  s->frames = h.frames;
  s->K = h.K;
  s->tail_n = h.tail_n;
  return SEG_OK;
}

int seg_get_profile(const seg_session* s, seg_profile* out) {
  if (!s || !out) return SEG_E_INVAL;
  if (s->state != State::Finalized) return SEG_E_STATE;
  *out = s->prof;
  return SEG_OK;
}

int seg_set_model(seg_session* s, struct seg_nn* net) {
  if (!s || !net || s->cfg.detector == SEG_DET_PLAIN) return SEG_E_INVAL;
  if (s->state != State::Open || s->frames != 0 || s->K != 0) return SEG_E_STATE;
  uint32_t b = 0, h = 0, w = 0, input = 0;
  if (seg_nn_shape(net, &b, &h, &w) != SEG_OK || seg_nn_input(net, &input) != SEG_OK) return SEG_E_INVAL;
  if (s->cfg.detector == SEG_DET_SURROGATE &&
      (input != SEG_NN_INPUT_FRAMES || h != s->cfg.height || w != s->cfg.width))
    return SEG_E_SHAPE;
  if (s->cfg.detector == SEG_DET_UNET && (input != SEG_NN_INPUT_SUMMARIES || h != 64 || w != 64))
    return SEG_E_SHAPE;
  s->net = net;
  return SEG_OK;
}

}  // extern "C"

struct seg_batch {
  uint32_t max_slots;
  void* dev_table;
  void* host_table;      // pinned
  int device;
  int grid;              // persistent grid of the captured launch
  hipStream_t capture;   // private stream used for the capture
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipEvent_t copied;     // the last table upload has completed
  hipEvent_t replayed;   // the last replay (which reads the device table) has completed
  bool have_copy;
};

extern "C" {

int seg_batch_bytes(uint32_t max_slots, size_t* bytes) {
  if (!bytes || max_slots < 1 || max_slots > (uint32_t)seg::kMaxBatch) return SEG_E_INVAL;
  *bytes = (seg::batch_table_bytes() + 255) & ~size_t(255);
  return SEG_OK;
}

int seg_batch_create(uint32_t max_slots, void* dev_table, size_t bytes, seg_batch** out) {
  if (!out || !dev_table) return SEG_E_INVAL;
  *out = nullptr;
  size_t need = 0;
  int e = seg_batch_bytes(max_slots, &need);
  if (e) return e;
  if (bytes < need) return SEG_E_CAPACITY;
  if (reinterpret_cast<uintptr_t>(dev_table) & 255) return SEG_E_INVAL;
  seg_batch* b = new (std::nothrow) seg_batch();
  if (!b) return SEG_E_INVAL;
  b->max_slots = max_slots;
  b->dev_table = dev_table;
  b->have_copy = false;
  int cus = 256;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess ||
      hipHostMalloc(&b->host_table, seg::batch_table_bytes(), hipHostMallocDefault) != hipSuccess) {
    delete b;
    return SEG_E_DEVICE;
  }
  std::memset(b->host_table, 0, seg::batch_table_bytes());
  b->grid = 2 * cus;  // two resident workgroups per CU
  bool ok = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->replayed, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const hipError_t le = seg::launch_block_stats_batch(b->dev_table, b->grid, b->capture);
    const hipError_t ce = hipStreamEndCapture(b->capture, &b->graph);
    ok = le == hipSuccess && ce == hipSuccess;
  }
  ok = ok && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
  if (!ok) {
    (void)hipHostFree(b->host_table);
    delete b;
    return SEG_E_DEVICE;
  }
  *out = b;
  return SEG_OK;
}

int seg_push_batch(seg_batch* b, seg_session* const* sessions, const uint16_t* const* dev_frames,
                   const uint32_t* n_frames, uint32_t count, void* stream) {
  if (!b || (count && (!sessions || !dev_frames || !n_frames)) || count > b->max_slots) return SEG_E_INVAL;
  // validate everything first: on error nothing is pushed
  for (uint32_t k = 0; k < count; ++k) {
    seg_session* s = sessions[k];
    if (!s) return SEG_E_INVAL;
    if (s->state == State::Failed) return SEG_E_DEVICE;
    if (s->state != State::Open) return SEG_E_STATE;
    if (s->device != b->device || s->cfg.detector != SEG_DET_PLAIN) return SEG_E_INVAL;
    if (n_frames[k] && !dev_frames[k]) return SEG_E_INVAL;
    if (s->frames + n_frames[k] > s->cfg.max_frames) return SEG_E_CAPACITY;
    for (uint32_t j = 0; j < k; ++j)
      if (sessions[j] == s) return SEG_E_INVAL;
  }
  if (hipSetDevice(b->device) != hipSuccess) return SEG_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<seg::StreamLaunch> ls(count);
  for (uint32_t k = 0; k < count; ++k) {
    seg_session* s = sessions[k];
    const uint32_t total = s->tail_n + n_frames[k];
    seg::StreamLaunch& a = ls[k];
    a = seg::StreamLaunch{};
    a.src0 = at<uint16_t>(s, s->lay.tail);
    a.src1 = dev_frames[k];
    a.n0 = s->tail_n;
    a.H = (int)s->cfg.height;
    a.W = (int)s->cfg.width;
    a.seg0 = (int)s->K;
    a.nseg = (int)(total / seg::kSegLen);
    a.T = at<float>(s, s->lay.T);
    a.S = at<float>(s, s->lay.S);
    a.D = at<float>(s, s->lay.D);
    a.U = at<float>(s, s->lay.U);
    a.P = at<float>(s, s->lay.P);
    a.plane = (long long)s->Kmax * s->M;
    a.w = s->w;
  }
  // the previous upload must have left the pinned table before it is rewritten
  if (b->have_copy && hipEventSynchronize(b->copied) != hipSuccess) return SEG_E_DEVICE;
  const int items = seg::fill_batch_table(b->host_table, ls.data(), (int)count);
  if (items > 0) {
    // the previous replay reads the device table for its whole run: a push
    // on another stream must not overwrite it before that replay ends
    if (b->have_copy && hipStreamWaitEvent(st, b->replayed, 0) != hipSuccess) return SEG_E_DEVICE;
    if (hipMemcpyAsync(b->dev_table, b->host_table, seg::batch_table_bytes(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipEventRecord(b->copied, st) != hipSuccess)
      return SEG_E_DEVICE;
    b->have_copy = true;
    if (hipGraphLaunch(b->exec, st) != hipSuccess || hipEventRecord(b->replayed, st) != hipSuccess)
      return SEG_E_DEVICE;
  }
  // tails and counters, as in seg_push_frames
  for (uint32_t k = 0; k < count; ++k) {
    seg_session* s = sessions[k];
    const uint32_t n = n_frames[k];
    if (n == 0) continue;
    const long long M = s->M;
    const uint32_t total = s->tail_n + n;
    const uint32_t nseg = total / seg::kSegLen;
    const uint32_t rem = total - nseg * seg::kSegLen;
    uint16_t* tail = at<uint16_t>(s, s->lay.tail);
    hipError_t he = hipSuccess;
    if (nseg > 0) {
      if (rem)
        he = hipMemcpyAsync(tail, dev_frames[k] + (size_t)(n - rem) * M, (size_t)rem * M * 2,
                            hipMemcpyDeviceToDevice, st);
    } else {
      he = hipMemcpyAsync(tail + (size_t)s->tail_n * M, dev_frames[k], (size_t)n * M * 2,
                          hipMemcpyDeviceToDevice, st);
    }
    if (fail(s, he)) return SEG_E_DEVICE;
    s->K += nseg;
    s->tail_n = rem;
    s->frames += n;
  }
  return SEG_OK;
}

int seg_batch_destroy(seg_batch* b) {
  if (!b) return SEG_OK;
  (void)hipSetDevice(b->device);
  if (b->have_copy) (void)hipEventSynchronize(b->replayed);
  (void)hipGraphExecDestroy(b->exec);
  (void)hipGraphDestroy(b->graph);
  (void)hipEventDestroy(b->copied);
  (void)hipEventDestroy(b->replayed);
  (void)hipStreamDestroy(b->capture);
  (void)hipHostFree(b->host_table);
  delete b;
  return SEG_OK;
}

const char* seg_strerror(int code) {
  switch (code) {
    case SEG_OK: return "ok";
    case SEG_E_INVAL: return "invalid argument or configuration";
    case SEG_E_SHAPE: return "shape mismatch";
    case SEG_E_STATE: return "call not allowed in the session's state";
    case SEG_E_CAPACITY: return "capacity exceeded";
    case SEG_E_DEVICE: return "HIP device error";
    case SEG_E_NOMODEL: return "no model loaded";
    default: return "unknown status";
  }
}

int seg_last_error(const seg_session* s) {
  if (!s) return SEG_E_INVAL;
  return s->error;
}

}  // extern "C"
