// C ABI of the learned warm start: network training and inference, input
// features, probe rendering and the forward-model training-set generator.
// Every computation runs in the kernels of learned_kernels.hip; this file
// validates arguments, owns device memory and orders launches on one stream.

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/ptycho_ws.h"
#include "learned.hpp"

using namespace ws;

namespace {

thread_local std::string g_ws_error;

int32_t ws_fail(int32_t code, const std::string& msg) {
  g_ws_error = msg;
  return code;
}

int32_t hip_check(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ws_fail(PTYCHO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PTYCHO_OK;
}

template <typename T>
bool dalloc(std::vector<void*>& owned, T*& p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess) return false;
  owned.push_back(q);
  p = static_cast<T*>(q);
  return true;
}

void free_all(std::vector<void*>& owned) {
  for (void* q : owned) (void)hipFree(q);
  owned.clear();
}

constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kAdamEps = 1e-8f;

}  // namespace

struct ptycho_ws {
  hipStream_t stream = nullptr;
  int max_batch = 0;
  std::vector<void*> owned;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  __bf16 *w1b = nullptr, *wf = nullptr, *wb = nullptr, *hwb = nullptr;
  __bf16* act[kLayers] = {};
  __bf16* gact[kLayers] = {};
  float *y = nullptr, *loss_part = nullptr, *head_part = nullptr, *wpart = nullptr, *loss = nullptr;
  Norm norm{};
  int step = 0;
};

struct ptycho_fm {
  ptycho_fm_config cfg{};
  hipStream_t stream = nullptr;
  int max_chunk = 0, n_pos = 0;
  std::vector<void*> owned;
  float* sp = nullptr;
  int* pos = nullptr;
  float2* obj = nullptr;
  float* pat = nullptr;
  float* tot = nullptr;
};

namespace {

int32_t run_forward(ptycho_ws* w, const float* x, const int32_t* idx, int nb, const float* target, float* y) {
  launch_conv1_fwd(x, idx, nb, w->w1b, w->theta + kTaps * kC, w->act[0], w->stream);
  for (int l = 1; l < kLayers; ++l)
    launch_conv_fwd(l, w->act[l - 1], nb, w->wf + (size_t)(l - 1) * kConvW, w->theta + conv_offset(l) + kConvW,
                    w->act[l], w->stream);
  launch_head(w->act[kLayers - 1], nb, w->hwb, w->theta + kHeadB, target, idx, w->norm, y, w->loss_part,
              w->head_part, w->gact[kLayers - 1], w->stream);
  return hip_check("network forward");
}

int32_t run_backward(ptycho_ws* w, const float* x, const int32_t* idx, int nb) {
  launch_reduce(w->head_part, nb, kHeadCols, RED_HEAD, kHeadW, 1.f, w->grad, w->stream);
  launch_reduce(w->loss_part, nb, 1, RED_LOSS, 0, 1.f / (float)(nb * kOut), w->loss, w->stream);
  for (int l = kLayers - 1; l >= 1; --l) {
    const int rows = launch_conv_bwd_weight(l, w->gact[l], w->act[l - 1], nb, w->wpart, w->stream);
    launch_reduce(w->wpart, rows, kConvStride, RED_CONV, conv_offset(l), 1.f, w->grad, w->stream);
    launch_conv_bwd_data(l, w->gact[l], nb, w->wb + (size_t)(l - 1) * kConvW, w->act[l - 1], w->gact[l - 1],
                         w->stream);
  }
  const int rows = launch_conv1_bwd_weight(w->gact[0], x, idx, nb, w->wpart, w->stream);
  launch_reduce(w->wpart, rows, kL1, RED_CONV1, 0, 1.f, w->grad, w->stream);
  return hip_check("network backward");
}

int32_t check_batch(const ptycho_ws* w, const float* x, int nb) {
  if (!w) return ws_fail(PTYCHO_E_INVALID, "null network");
  if (!x) return ws_fail(PTYCHO_E_INVALID, "null input");
  if (nb < 1 || nb > w->max_batch)
    return ws_fail(PTYCHO_E_SHAPE, "batch " + std::to_string(nb) + " outside [1, " + std::to_string(w->max_batch) + "]");
  return PTYCHO_OK;
}

bool finite(float v) { return std::isfinite(v); }

}  // namespace

extern "C" {

int32_t ptycho_ws_param_count(void) { return kParams; }

const char* ptycho_ws_last_error(void) { return g_ws_error.c_str(); }

int32_t ptycho_ws_create(int32_t max_batch, void* stream, ptycho_ws** out) {
  if (!out) return ws_fail(PTYCHO_E_INVALID, "null output handle");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 4096) return ws_fail(PTYCHO_E_INVALID, "max_batch outside [1, 4096]");
  auto* w = new ptycho_ws();
  w->stream = static_cast<hipStream_t>(stream);
  w->max_batch = max_batch;
  bool ok = dalloc(w->owned, w->theta, kParams) && dalloc(w->owned, w->grad, kParams) &&
            dalloc(w->owned, w->m, kParams) && dalloc(w->owned, w->v, kParams) &&
            dalloc(w->owned, w->w1b, kTaps * kC) && dalloc(w->owned, w->wf, (size_t)(kLayers - 1) * kConvW) &&
            dalloc(w->owned, w->wb, (size_t)(kLayers - 1) * kConvW) && dalloc(w->owned, w->hwb, kOut * kC) &&
            dalloc(w->owned, w->y, (size_t)max_batch * kOut) && dalloc(w->owned, w->loss_part, max_batch) &&
            dalloc(w->owned, w->head_part, (size_t)max_batch * kHeadCols) &&
            dalloc(w->owned, w->wpart, (size_t)max_weight_partials()) && dalloc(w->owned, w->loss, 1);
  for (int l = 0; ok && l < kLayers; ++l) {
    const size_t elems = (size_t)max_batch * side_out(l) * side_out(l) * kC;
    ok = dalloc(w->owned, w->act[l], elems) && dalloc(w->owned, w->gact[l], elems);
  }
  if (!ok) {
    free_all(w->owned);
    delete w;
    return ws_fail(PTYCHO_E_OOM, "device allocation failed");
  }
  for (int i = 0; i < kOut; ++i) {
    w->norm.off[i] = 0.f;
    w->norm.scale[i] = 1.f;
  }
  const size_t pbytes = kParams * sizeof(float);
  hipError_t e = hipMemsetAsync(w->theta, 0, pbytes, w->stream);
  if (e == hipSuccess) e = hipMemsetAsync(w->m, 0, pbytes, w->stream);
  if (e == hipSuccess) e = hipMemsetAsync(w->v, 0, pbytes, w->stream);
  if (e == hipSuccess) e = hipMemsetAsync(w->grad, 0, pbytes, w->stream);
  if (e != hipSuccess) {
    free_all(w->owned);
    delete w;
    return ws_fail(PTYCHO_E_HIP, std::string("memset: ") + hipGetErrorString(e));
  }
  launch_adam_pack(w->theta, w->grad, w->m, w->v, false, 0.f, kBeta1, kBeta2, kAdamEps, 1.f, 1.f, w->w1b, w->wf,
                   w->wb, w->hwb, w->stream);
  if (hip_check("pack") != PTYCHO_OK || hipStreamSynchronize(w->stream) != hipSuccess) {
    free_all(w->owned);
    delete w;
    return ws_fail(PTYCHO_E_HIP, "network initialisation failed");
  }
  *out = w;
  return PTYCHO_OK;
}

int32_t ptycho_ws_set_params(ptycho_ws* w, const float* theta, int32_t mem_kind) {
  if (!w || !theta) return ws_fail(PTYCHO_E_INVALID, "null argument");
  if (mem_kind != PTYCHO_MEM_HOST && mem_kind != PTYCHO_MEM_DEVICE) return ws_fail(PTYCHO_E_INVALID, "bad mem_kind");
  if (mem_kind == PTYCHO_MEM_HOST)
    for (int i = 0; i < kParams; ++i)
      if (!finite(theta[i])) return ws_fail(PTYCHO_E_INVALID, "non-finite parameter " + std::to_string(i));
  const hipMemcpyKind kind = mem_kind == PTYCHO_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  if (hipMemcpyAsync(w->theta, theta, kParams * sizeof(float), kind, w->stream) != hipSuccess)
    return ws_fail(PTYCHO_E_HIP, "parameter copy failed");
  launch_adam_pack(w->theta, w->grad, w->m, w->v, false, 0.f, kBeta1, kBeta2, kAdamEps, 1.f, 1.f, w->w1b, w->wf,
                   w->wb, w->hwb, w->stream);
  if (hipStreamSynchronize(w->stream) != hipSuccess) return ws_fail(PTYCHO_E_HIP, "synchronise failed");
  return hip_check("pack");
}

int32_t ptycho_ws_get_params(ptycho_ws* w, float* theta, int32_t mem_kind) {
  if (!w || !theta) return ws_fail(PTYCHO_E_INVALID, "null argument");
  if (mem_kind != PTYCHO_MEM_HOST && mem_kind != PTYCHO_MEM_DEVICE) return ws_fail(PTYCHO_E_INVALID, "bad mem_kind");
  const hipMemcpyKind kind = mem_kind == PTYCHO_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (hipMemcpyAsync(theta, w->theta, kParams * sizeof(float), kind, w->stream) != hipSuccess ||
      hipStreamSynchronize(w->stream) != hipSuccess)
    return ws_fail(PTYCHO_E_HIP, "parameter copy failed");
  return PTYCHO_OK;
}

int32_t ptycho_ws_set_target_scaling(ptycho_ws* w, const float* off, const float* scale) {
  if (!w || !off || !scale) return ws_fail(PTYCHO_E_INVALID, "null argument");
  for (int i = 0; i < kOut; ++i)
    if (!finite(off[i]) || !finite(scale[i]) || !(scale[i] > 0.f))
      return ws_fail(PTYCHO_E_INVALID, "target scaling must be finite with scale > 0");
  for (int i = 0; i < kOut; ++i) {
    w->norm.off[i] = off[i];
    w->norm.scale[i] = scale[i];
  }
  return PTYCHO_OK;
}

int32_t ptycho_ws_forward(ptycho_ws* w, const float* x, const int32_t* idx, int32_t nb, float* y) {
  int32_t rc = check_batch(w, x, nb);
  if (rc != PTYCHO_OK) return rc;
  if (!y) return ws_fail(PTYCHO_E_INVALID, "null output");
  return run_forward(w, x, idx, nb, nullptr, y);
}

int32_t ptycho_ws_loss_grad(ptycho_ws* w, const float* x, const int32_t* idx, const float* target, int32_t nb,
                            float* loss_host, float* grad, int32_t mem_kind) {
  int32_t rc = check_batch(w, x, nb);
  if (rc != PTYCHO_OK) return rc;
  if (!target) return ws_fail(PTYCHO_E_INVALID, "null target");
  if (grad && mem_kind != PTYCHO_MEM_HOST && mem_kind != PTYCHO_MEM_DEVICE)
    return ws_fail(PTYCHO_E_INVALID, "bad mem_kind");
  if ((rc = run_forward(w, x, idx, nb, target, w->y)) != PTYCHO_OK) return rc;
  if ((rc = run_backward(w, x, idx, nb)) != PTYCHO_OK) return rc;
  if (grad) {
    const hipMemcpyKind kind = mem_kind == PTYCHO_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(grad, w->grad, kParams * sizeof(float), kind, w->stream) != hipSuccess)
      return ws_fail(PTYCHO_E_HIP, "gradient copy failed");
  }
  if (loss_host) {
    if (hipMemcpyAsync(loss_host, w->loss, sizeof(float), hipMemcpyDeviceToHost, w->stream) != hipSuccess)
      return ws_fail(PTYCHO_E_HIP, "loss copy failed");
  }
  if ((grad && mem_kind == PTYCHO_MEM_HOST) || loss_host)
    if (hipStreamSynchronize(w->stream) != hipSuccess) return ws_fail(PTYCHO_E_HIP, "synchronise failed");
  return PTYCHO_OK;
}

int32_t ptycho_ws_train_step(ptycho_ws* w, const float* x, const int32_t* idx, const float* target, int32_t nb,
                             float lr, float* loss_host) {
  int32_t rc = check_batch(w, x, nb);
  if (rc != PTYCHO_OK) return rc;
  if (!target) return ws_fail(PTYCHO_E_INVALID, "null target");
  if (!finite(lr) || !(lr > 0.f)) return ws_fail(PTYCHO_E_INVALID, "learning rate must be finite and > 0");
  if ((rc = run_forward(w, x, idx, nb, target, w->y)) != PTYCHO_OK) return rc;
  if ((rc = run_backward(w, x, idx, nb)) != PTYCHO_OK) return rc;
  w->step += 1;
  const float c1 = 1.f - std::pow(kBeta1, (float)w->step), c2 = 1.f - std::pow(kBeta2, (float)w->step);
  launch_adam_pack(w->theta, w->grad, w->m, w->v, true, lr, kBeta1, kBeta2, kAdamEps, c1, c2, w->w1b, w->wf, w->wb,
                   w->hwb, w->stream);
  if ((rc = hip_check("adam")) != PTYCHO_OK) return rc;
  if (loss_host) {
    if (hipMemcpyAsync(loss_host, w->loss, sizeof(float), hipMemcpyDeviceToHost, w->stream) != hipSuccess ||
        hipStreamSynchronize(w->stream) != hipSuccess)
      return ws_fail(PTYCHO_E_HIP, "loss copy failed");
  }
  return PTYCHO_OK;
}

int32_t ptycho_ws_reset_optimizer(ptycho_ws* w) {
  if (!w) return ws_fail(PTYCHO_E_INVALID, "null network");
  w->step = 0;
  if (hipMemsetAsync(w->m, 0, kParams * sizeof(float), w->stream) != hipSuccess ||
      hipMemsetAsync(w->v, 0, kParams * sizeof(float), w->stream) != hipSuccess)
    return ws_fail(PTYCHO_E_HIP, "memset failed");
  return PTYCHO_OK;
}

void ptycho_ws_destroy(ptycho_ws* w) {
  if (!w) return;
  (void)hipStreamSynchronize(w->stream);
  free_all(w->owned);
  delete w;
}

int32_t ptycho_ws_features(const float* intensities, int32_t n_pat, int32_t n, float* out, void* stream) {
  if (!intensities || !out) return ws_fail(PTYCHO_E_INVALID, "null argument");
  if (n < 2 || n > kSide || (n & 1)) return ws_fail(PTYCHO_E_SHAPE, "frame side must be even and <= 128");
  if (n_pat < 1) return ws_fail(PTYCHO_E_SHAPE, "need at least one pattern");
  launch_features(intensities, n_pat, n, kSide, out, static_cast<hipStream_t>(stream));
  return hip_check("features");
}

int32_t ptycho_ws_render_probe(int32_t n, int32_t n_modes, float radius, float defocus, float total_power,
                               float* probe, void* stream) {
  if (!probe) return ws_fail(PTYCHO_E_INVALID, "null output");
  if (n < 8 || n > 1024) return ws_fail(PTYCHO_E_SHAPE, "n outside [8, 1024]");
  if (n_modes < 1 || n_modes > 4) return ws_fail(PTYCHO_E_INVALID, "n_modes outside [1, 4]");
  if (!finite(radius) || !(radius > 0.f) || !(radius < 0.5f * (float)n))
    return ws_fail(PTYCHO_E_INVALID, "radius outside (0, n/2)");
  if (!finite(defocus) || !finite(total_power) || !(total_power > 0.f))
    return ws_fail(PTYCHO_E_INVALID, "defocus and total_power must be finite, total_power > 0");
  launch_render_probe(n, n_modes, radius, defocus, total_power, reinterpret_cast<float2*>(probe),
                      static_cast<hipStream_t>(stream));
  return hip_check("render probe");
}

void ptycho_fm_default_config(ptycho_fm_config* c) {
  if (!c) return;
  c->obj_side = 144;
  c->n_scan = 10;
  c->step = 8;
  c->jitter = 1;
  c->n_wl = 5;
  c->counts = 1e5f;
  c->sigma_lo = 0.5f;
  c->sigma_hi = 3.f;
  c->bw_lo = 0.f;
  c->bw_hi = 0.05f;
  c->r_lo = 12.f;
  c->r_hi = 20.f;
  c->c_lo = 0.5f;
  c->c_hi = 2.f;
}

int32_t ptycho_fm_create(const ptycho_fm_config* cfg, int32_t max_chunk, void* stream, ptycho_fm** out) {
  if (!cfg || !out) return ws_fail(PTYCHO_E_INVALID, "null argument");
  *out = nullptr;
  const ptycho_fm_config& c = *cfg;
  if (c.obj_side < kFmN || c.obj_side > kFmMaxSide) return ws_fail(PTYCHO_E_SHAPE, "obj_side outside [64, 160]");
  if (c.n_scan < 1 || c.n_scan * c.n_scan > 1024 || c.step < 0 || c.jitter < 0)
    return ws_fail(PTYCHO_E_SHAPE, "bad raster");
  if ((c.n_scan - 1) * c.step + kFmN + 2 * c.jitter > c.obj_side)
    return ws_fail(PTYCHO_E_SHAPE, "scan extent exceeds the object");
  if (c.n_wl < 1 || c.n_wl > 16) return ws_fail(PTYCHO_E_INVALID, "n_wl outside [1, 16]");
  const float v[] = {c.counts, c.sigma_lo, c.sigma_hi, c.bw_lo, c.bw_hi, c.r_lo, c.r_hi, c.c_lo, c.c_hi};
  for (float x : v)
    if (!finite(x)) return ws_fail(PTYCHO_E_INVALID, "non-finite configuration value");
  if (!(c.counts > 0.f) || c.sigma_lo < 0.f || c.sigma_hi < c.sigma_lo || c.bw_lo < 0.f || c.bw_hi < c.bw_lo ||
      c.bw_hi >= 0.5f || !(c.r_lo > 0.f) || c.r_hi < c.r_lo || c.r_hi >= 0.5f * kFmN || c.c_hi < c.c_lo)
    return ws_fail(PTYCHO_E_INVALID, "bad sampling ranges");
  if (max_chunk < 1 || max_chunk > 65535) return ws_fail(PTYCHO_E_INVALID, "max_chunk outside [1, 65535]");
  auto* f = new ptycho_fm();
  f->cfg = c;
  f->stream = static_cast<hipStream_t>(stream);
  f->max_chunk = max_chunk;
  f->n_pos = c.n_scan * c.n_scan;
  const size_t mc = (size_t)max_chunk;
  const bool ok = dalloc(f->owned, f->sp, mc * 4) && dalloc(f->owned, f->pos, mc * f->n_pos * 2) &&
                  dalloc(f->owned, f->obj, mc * c.obj_side * c.obj_side) &&
                  dalloc(f->owned, f->pat, mc * f->n_pos * kFmN * kFmN) && dalloc(f->owned, f->tot, mc * f->n_pos);
  if (!ok) {
    free_all(f->owned);
    delete f;
    return ws_fail(PTYCHO_E_OOM, "device allocation failed");
  }
  *out = f;
  return PTYCHO_OK;
}

int32_t ptycho_fm_objects(ptycho_fm* f, uint64_t seed, int64_t first, int32_t count, float* log_amp_phase) {
  if (!f || !log_amp_phase) return ws_fail(PTYCHO_E_INVALID, "null argument");
  if (count < 1 || count > f->max_chunk || first < 0) return ws_fail(PTYCHO_E_SHAPE, "count outside [1, max_chunk]");
  launch_fm_object(seed, (long)first, count, f->cfg.obj_side, reinterpret_cast<float2*>(log_amp_phase), f->stream);
  return hip_check("fm objects");
}

int32_t ptycho_fm_generate(ptycho_fm* f, uint64_t seed, int64_t first, int32_t count, float* feat, float* targets) {
  if (!f || !feat || !targets) return ws_fail(PTYCHO_E_INVALID, "null argument");
  if (count < 1 || count > f->max_chunk || first < 0) return ws_fail(PTYCHO_E_SHAPE, "count outside [1, max_chunk]");
  const ptycho_fm_config& c = f->cfg;
  const FmRanges rg{c.sigma_lo, c.sigma_hi, c.bw_lo, c.bw_hi, c.r_lo, c.r_hi, c.c_lo, c.c_hi};
  launch_fm_setup(seed, (long)first, count, rg, c.obj_side, c.n_scan, c.step, c.jitter, f->sp, f->pos, f->stream);
  launch_fm_object(seed, (long)first, count, c.obj_side, f->obj, f->stream);
  launch_fm_patterns(f->obj, c.obj_side, f->sp, f->pos, f->n_pos, count, c.n_wl, f->pat, f->tot, f->stream);
  launch_fm_features(f->pat, f->tot, f->sp, seed, (long)first, count, f->n_pos, c.counts, feat, targets, f->stream);
  return hip_check("fm generate");
}

int32_t ptycho_fm_patterns(ptycho_fm* f, const float* log_amp_phase, const int32_t* positions, int32_t n_pos,
                           float sigma, float bandwidth, float radius, float defocus, float* patterns) {
  if (!f || !log_amp_phase || !positions || !patterns) return ws_fail(PTYCHO_E_INVALID, "null argument");
  if (n_pos < 1 || n_pos > f->n_pos) return ws_fail(PTYCHO_E_SHAPE, "n_pos outside [1, n_scan^2]");
  if (!finite(sigma) || sigma < 0.f || !finite(bandwidth) || bandwidth < 0.f || bandwidth >= 0.5f ||
      !finite(radius) || !(radius > 0.f) || radius >= 0.5f * kFmN || !finite(defocus))
    return ws_fail(PTYCHO_E_INVALID, "bad sample values");
  const int side = f->cfg.obj_side;
  for (int i = 0; i < n_pos; ++i) {
    const int r = positions[2 * i], cc = positions[2 * i + 1];
    if (r < 0 || cc < 0 || r > side - kFmN || cc > side - kFmN)
      return ws_fail(PTYCHO_E_SHAPE, "position " + std::to_string(i) + " puts the frame outside the object");
  }
  const float h[4] = {sigma, bandwidth, radius, defocus};
  if (hipMemcpyAsync(f->sp, h, sizeof(h), hipMemcpyHostToDevice, f->stream) != hipSuccess ||
      hipMemcpyAsync(f->pos, positions, (size_t)n_pos * 2 * sizeof(int32_t), hipMemcpyHostToDevice, f->stream) !=
          hipSuccess ||
      hipStreamSynchronize(f->stream) != hipSuccess)
    return ws_fail(PTYCHO_E_HIP, "copy failed");
  launch_fm_patterns(reinterpret_cast<const float2*>(log_amp_phase), side, f->sp, f->pos, n_pos, 1,
                     f->cfg.n_wl, patterns, f->tot, f->stream);
  return hip_check("fm patterns");
}

void ptycho_fm_destroy(ptycho_fm* f) {
  if (!f) return;
  (void)hipStreamSynchronize(f->stream);
  free_all(f->owned);
  delete f;
}

}  // extern "C"
