// Host runtime of the pc-ePIE library: validation, device memory, the iteration
// schedule and the C ABI declared in include/ptycho.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ptycho.h"
#include "kernels.hpp"

using namespace pty;

namespace {

thread_local std::string g_thread_error = "";

struct Timing {
  uint32_t mask = 0;
  double total_ms[KC_COUNT] = {};
  int64_t launches[KC_COUNT] = {};
  std::vector<hipEvent_t> pool;  // pairs: start, stop
  std::vector<int> cls;          // class of each used pair
  size_t used = 0;
};

}  // namespace

struct ptycho_ctx {
  ptycho_params prm{};
  DevParams dp{};
  DevBufs db{};
  hipStream_t stream = nullptr;
  int device = 0;
  int t = 0;
  bool failed = false;
  std::string err;
  double inv_denom = 0.0;  // 1 / sum_n sum_q I_n
  // owned device allocations
  std::vector<void*> allocs;
  int* d_order = nullptr;   // [order_cap]
  size_t order_cap = 0;
  int* h_order = nullptr;   // pinned staging
  float* d_err = nullptr;   // [err_cap]
  size_t err_cap = 0;
  int bmax = 1;
  int n_err_part = 0;
  Timing tm;
};

namespace {

ptycho_status fail(ptycho_ctx* c, ptycho_status st, const std::string& msg) {
  if (c) c->err = msg;
  else g_thread_error = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((ctx), PTYCHO_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool finite_f(float v) { return std::isfinite(v); }

std::string validate(const ptycho_params* p) {
  if (!p) return "params is NULL";
  if (!supported_n(p->n)) return "n=" + std::to_string(p->n) + " unsupported (8,16,24,32,48,64,96,128,192,256,384,512,768,1024)";
  if (p->n_modes < 1 || p->n_modes > kMaxModes) return "n_modes must be in [1,16]";
  if (p->n_pos < 1) return "n_pos must be >= 1";
  if (p->obj_h < p->n || p->obj_w < p->n) return "object must be at least n x n";
  if (p->geometry != PTYCHO_FAR_FIELD && p->geometry != PTYCHO_NEAR_FIELD) return "bad geometry";
  if (p->geometry == PTYCHO_NEAR_FIELD && !(std::isfinite(p->fresnel_px) && p->fresnel_px > 0))
    return "near field needs fresnel_px > 0";
  if (!(finite_f(p->sigma1) && p->sigma1 >= 0 && finite_f(p->sigma2) && p->sigma2 >= 0)) return "sigma must be >= 0";
  if (p->kernel_size < 1 || p->kernel_size > 2 * kMaxHalf + 1 || p->kernel_size % 2 == 0)
    return "kernel_size must be odd in [1,31]";
  if (p->kernel_size > p->n) return "kernel_size must not exceed n";
  if (p->blur_domain != PTYCHO_BLUR_AMPLITUDE && p->blur_domain != PTYCHO_BLUR_INTENSITY) return "bad blur_domain";
  if (!(finite_f(p->eps) && p->eps >= 0)) return "eps must be >= 0";
  if (!(p->alpha1 >= 0 && p->alpha1 <= 1 && p->alpha2 >= 0 && p->alpha2 <= 1)) return "alpha1, alpha2 must be in [0,1]";
  if (!(finite_f(p->cbar_min) && finite_f(p->cbar_max) && p->cbar_min > 0 && p->cbar_max >= p->cbar_min))
    return "need 0 < cbar_min <= cbar_max";
  if (p->cc_period < 0) return "cc_period must be >= 0";
  if (!(finite_f(p->obj_step) && p->obj_step >= 0 && finite_f(p->probe_step) && p->probe_step >= 0))
    return "steps must be finite and >= 0";
  if (!(p->gamma_obj > 0 && p->gamma_obj <= 1 && p->gamma_probe > 0 && p->gamma_probe <= 1))
    return "gamma_obj, gamma_probe must be in (0,1]";
  if (p->batch < 1 || p->batch > kMaxBatch) return "batch must be in [1,256]";
  if (p->orthogonalize != 0 && p->orthogonalize != 1) return "orthogonalize must be 0 or 1";
  return "";
}

bool in_window(const ptycho_params& p, int t) {
  if (p.cc_start < 1 || p.cc_end < p.cc_start) return false;
  int tt = t;
  if (p.cc_period > 0) tt = (t - 1) % p.cc_period + 1;
  return tt >= p.cc_start && tt <= p.cc_end;
}

void gaussian_taps(float sigma, int half, float* out) {
  double w[kMaxHalf + 1];
  double tot = 0.0;
  for (int d = 0; d <= half; ++d) {
    w[d] = (d == 0) ? 1.0 : (sigma > 0 ? std::exp(-(double)d * d / (2.0 * (double)sigma * sigma)) : 0.0);
    tot += (d == 0) ? w[d] : 2.0 * w[d];
  }
  for (int d = 0; d <= kMaxHalf; ++d) out[d] = (d <= half) ? (float)(w[d] / tot) : 0.f;
}

template <typename T>
ptycho_status dev_alloc(ptycho_ctx* c, T** ptr, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, PTYCHO_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  c->allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return PTYCHO_OK;
}

hipMemcpyKind kind_in(int32_t mem_kind) { return mem_kind == PTYCHO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kind_out(int32_t mem_kind) { return mem_kind == PTYCHO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

// Time one launch of class `cls` if selected.
struct Timed {
  ptycho_ctx* c;
  int cls;
  hipEvent_t stop = nullptr;
  Timed(ptycho_ctx* ctx, int k) : c(ctx), cls(k) {
    if (!(c->tm.mask & (1u << k))) return;
    if (c->tm.used * 2 + 2 > c->tm.pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->tm.pool.push_back(e);
      }
    }
    hipEvent_t start = c->tm.pool[c->tm.used * 2];
    stop = c->tm.pool[c->tm.used * 2 + 1];
    c->tm.cls.resize(c->tm.used + 1);
    c->tm.cls[c->tm.used] = k;
    c->tm.used++;
    (void)hipEventRecord(start, c->stream);
  }
  ~Timed() {
    if (stop) (void)hipEventRecord(stop, c->stream);
  }
};

void harvest_timing(ptycho_ctx* c) {
  for (size_t i = 0; i < c->tm.used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->tm.pool[2 * i], c->tm.pool[2 * i + 1]) == hipSuccess) {
      c->tm.total_ms[c->tm.cls[i]] += ms;
      c->tm.launches[c->tm.cls[i]] += 1;
    }
  }
  c->tm.used = 0;
}

#define LAUNCH(ctx, cls, expr)                                                            \
  do {                                                                                    \
    hipError_t e_;                                                                        \
    {                                                                                     \
      Timed tmd_((ctx), (cls));                                                           \
      e_ = (expr);                                                                        \
    }                                                                                     \
    if (e_ != hipSuccess)                                                                 \
      return fail((ctx), PTYCHO_E_HIP, std::string(kKernelNames[cls]) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One batch update: the body of Fig. 1 over slots[0..ns).
ptycho_status run_batch(ptycho_ctx* c, const int* d_slots, int ns, int t, const DebugPtrs& dbg) {
  const DevParams& p = c->dp;
  const DevBufs& d = c->db;
  const bool near = c->prm.geometry == PTYCHO_NEAR_FIELD;
  hipStream_t s = c->stream;
  const int bm = ns;  // grid sized to the batch
  const bool cc = in_window(c->prm, t);
  const bool probe = t >= c->prm.probe_update_start;
  LAUNCH(c, KC_FWD_ROWS, launch_fwd_rows(p.n, near, p, d, d_slots, ns, probe, s));
  LAUNCH(c, KC_FWD_COLS, launch_fwd_cols(p.n, near, p, d, ns, bm, s));
  LAUNCH(c, KC_INV_COLS, launch_inv_cols(p.n, near, p, d, d_slots, ns, bm, dbg, s));
  LAUNCH(c, KC_INV_ROWS, launch_inv_rows(p.n, near, p, d, d_slots, ns, bm, dbg, s));
  LAUNCH(c, KC_OBJ_UPDATE, launch_obj_update(p, d, d_slots, ns, cc, dbg, s));
  if (probe || cc) LAUNCH(c, KC_POST, launch_post(p, d, d_slots, ns, probe, cc, s));
  return PTYCHO_OK;
}

ptycho_status end_iteration(ptycho_ctx* c, float* d_err_slot) {
  const DevParams& p = c->dp;
  if (p.k > 1 && c->prm.orthogonalize) {
    LAUNCH(c, KC_GRAM, launch_gram(p, c->db, c->stream));
    LAUNCH(c, KC_EIG, launch_eig(p, c->db, c->stream));
    LAUNCH(c, KC_REMIX, launch_remix(p, c->db, c->stream));
  }
  LAUNCH(c, KC_ERR, launch_err_reduce(c->db.err_part, c->n_err_part, c->inv_denom, d_err_slot, c->stream));
  return PTYCHO_OK;
}

void splitmix_perm(uint64_t seed, int32_t t, int32_t n, int32_t* out) {
  for (int i = 0; i < n; ++i) out[i] = i;
  uint64_t s = seed ^ (uint64_t)(int64_t)t;
  for (int i = n - 1; i >= 1; --i) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int j = (int)(z % (uint64_t)(i + 1));
    std::swap(out[i], out[j]);
  }
}

ptycho_status ensure_order_capacity(ptycho_ctx* c, size_t count) {
  if (count <= c->order_cap) return PTYCHO_OK;
  if (c->d_order) {
    (void)hipFree(c->d_order);
    c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void*)c->d_order));
    c->d_order = nullptr;
  }
  if (c->h_order) {
    (void)hipHostFree(c->h_order);
    c->h_order = nullptr;
  }
  ptycho_status st = dev_alloc(c, &c->d_order, count);
  if (st != PTYCHO_OK) return st;
  hipError_t e = hipHostMalloc((void**)&c->h_order, count * sizeof(int), hipHostMallocDefault);
  if (e != hipSuccess) return fail(c, PTYCHO_E_OOM, "pinned host allocation failed");
  c->order_cap = count;
  return PTYCHO_OK;
}

ptycho_status ensure_err_capacity(ptycho_ctx* c, size_t count) {
  if (count <= c->err_cap) return PTYCHO_OK;
  if (c->d_err) {
    (void)hipFree(c->d_err);
    c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void*)c->d_err));
    c->d_err = nullptr;
  }
  ptycho_status st = dev_alloc(c, &c->d_err, count);
  if (st != PTYCHO_OK) return st;
  c->err_cap = count;
  return PTYCHO_OK;
}

ptycho_status check_probe_power(ptycho_ctx* c, const float* probe_host, size_t count) {
  double s = 0.0;
  for (size_t i = 0; i < count; ++i) {
    if (!std::isfinite(probe_host[i])) return fail(c, PTYCHO_E_INVALID, "probe has a non-finite value");
    s += (double)probe_host[i] * probe_host[i];
  }
  if (!(s > 0.0)) return fail(c, PTYCHO_E_INVALID, "probe has zero power");
  return PTYCHO_OK;
}

ptycho_status fetch_host(ptycho_ctx* c, const float* src, size_t count, int32_t mem_kind, std::vector<float>& out) {
  out.resize(count);
  if (mem_kind == PTYCHO_MEM_DEVICE) {
    HIP_TRY(c, hipMemcpy(out.data(), src, count * sizeof(float), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(out.data(), src, count * sizeof(float));
  }
  return PTYCHO_OK;
}

}  // namespace

extern "C" {

void ptycho_default_params(ptycho_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n = 64;
  p->n_modes = 1;
  p->geometry = PTYCHO_FAR_FIELD;
  p->fresnel_px = 0.0;
  p->sigma1 = p->sigma2 = 1.0f;
  p->kernel_size = 11;
  p->blur_domain = PTYCHO_BLUR_AMPLITUDE;
  p->eps = 1e-6f;
  p->alpha1 = 1.0f;
  p->alpha2 = 0.0f;
  p->cbar_min = 0.01f;
  p->cbar_max = 10.0f;
  p->cc_start = 0;
  p->cc_end = -1;
  p->cc_period = 0;
  p->obj_step = p->probe_step = 1.0f;
  p->gamma_obj = p->gamma_probe = 1.0f;
  p->probe_update_start = 1;
  p->batch = 1;
  p->orthogonalize = 1;
  p->seed = 0;
}

ptycho_status ptycho_permutation(uint64_t seed, int32_t t, int32_t n_pos, int32_t* out) {
  if (n_pos < 0 || (n_pos > 0 && !out)) return fail(nullptr, PTYCHO_E_INVALID, "bad permutation arguments");
  splitmix_perm(seed, t, n_pos, out);
  return PTYCHO_OK;
}

ptycho_status ptycho_init(const ptycho_params* params, const float* intensities, const int32_t* positions,
                          const float* probe0, const float* object0, int32_t mem_kind, void* hip_stream,
                          ptycho_ctx** out) {
  if (out) *out = nullptr;
  if (!out) return fail(nullptr, PTYCHO_E_INVALID, "out is NULL");
  std::string v = validate(params);
  if (!v.empty()) return fail(nullptr, PTYCHO_E_INVALID, v);
  if (!intensities || !positions || !probe0 || !object0) return fail(nullptr, PTYCHO_E_INVALID, "NULL input array");
  if (mem_kind != PTYCHO_MEM_HOST && mem_kind != PTYCHO_MEM_DEVICE) return fail(nullptr, PTYCHO_E_INVALID, "bad mem_kind");
  const ptycho_params& p = *params;
  const int n = p.n, K = p.n_modes;
  const size_t nn = (size_t)n * n;

  // Host-side checks that need no device: positions and (for host inputs) values.
  std::vector<int32_t> hpos(2 * (size_t)p.n_pos);
  if (mem_kind == PTYCHO_MEM_HOST) {
    std::memcpy(hpos.data(), positions, hpos.size() * sizeof(int32_t));
  } else {
    hipError_t e = hipMemcpy(hpos.data(), positions, hpos.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(nullptr, PTYCHO_E_HIP, std::string("reading positions: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < p.n_pos; ++i) {
    const int r = hpos[2 * i], cc = hpos[2 * i + 1];
    if (r < 0 || cc < 0 || r > p.obj_h - n || cc > p.obj_w - n)
      return fail(nullptr, PTYCHO_E_SHAPE, "position " + std::to_string(i) + " puts the box outside the object");
  }
  if (mem_kind == PTYCHO_MEM_HOST) {
    const size_t ni = (size_t)p.n_pos * nn;
    for (size_t i = 0; i < ni; ++i)
      if (!std::isfinite(intensities[i])) return fail(nullptr, PTYCHO_E_INVALID, "intensities contain a non-finite value");
    const size_t no = 2 * (size_t)p.obj_h * p.obj_w;
    for (size_t i = 0; i < no; ++i)
      if (!std::isfinite(object0[i])) return fail(nullptr, PTYCHO_E_INVALID, "object contains a non-finite value");
    ptycho_status st = check_probe_power(nullptr, probe0, 2 * K * nn);
    if (st != PTYCHO_OK) return st;
  }

  ptycho_ctx* c = new ptycho_ctx();
  c->prm = p;
  c->stream = (hipStream_t)hip_stream;
  auto bail = [&](ptycho_status st) {
    g_thread_error = c->err;
    ptycho_destroy(c);
    return st;
  };
  if (hipGetDevice(&c->device) != hipSuccess) {
    c->err = "no HIP device";
    return bail(PTYCHO_E_HIP);
  }
  if (mem_kind == PTYCHO_MEM_DEVICE) {
    std::vector<float> hp;
    ptycho_status st = fetch_host(c, probe0, 2 * K * nn, mem_kind, hp);
    if (st == PTYCHO_OK) st = check_probe_power(c, hp.data(), hp.size());
    if (st != PTYCHO_OK) return bail(st);
    std::vector<float> ho;
    st = fetch_host(c, object0, 2 * (size_t)p.obj_h * p.obj_w, mem_kind, ho);
    if (st != PTYCHO_OK) return bail(st);
    for (float x : ho)
      if (!std::isfinite(x)) {
        c->err = "object contains a non-finite value";
        return bail(PTYCHO_E_INVALID);
      }
  }

  DevParams& dp = c->dp;
  dp.n = n;
  dp.k = K;
  dp.h_obj = p.obj_h;
  dp.w_obj = p.obj_w;
  dp.n_pos = p.n_pos;
  dp.near_field = p.geometry == PTYCHO_NEAR_FIELD;
  dp.blur_intensity = p.blur_domain == PTYCHO_BLUR_INTENSITY;
  dp.ks_half = (p.kernel_size - 1) / 2;
  dp.eps = p.eps;
  dp.alpha1 = p.alpha1;
  dp.alpha2 = p.alpha2;
  dp.cbar_min = p.cbar_min;
  dp.cbar_max = p.cbar_max;
  dp.obj_step = p.obj_step;
  dp.probe_step = p.probe_step;
  dp.gamma_obj = p.gamma_obj;
  dp.gamma_probe = p.gamma_probe;
  gaussian_taps(p.sigma1, dp.ks_half, dp.gx);
  gaussian_taps(p.sigma2, dp.ks_half, dp.gy);

  const int B = p.batch;
  c->bmax = B;
  DevBufs& d = c->db;
  float2 *obj, *probe, *tw, *hn, *X, *dO, *nP, *vmix;
  float *pw, *amp, *q, *V, *maxv, *maxw;
  int2* pos;
  double *errp, *eig;
  double2 *ccp, *gramp;
  const int nobjt = n_obj_tiles(dp);
  const int nbt = n_err_slots(n);
  ptycho_status st = PTYCHO_OK;
  if ((st = dev_alloc(c, &obj, (size_t)p.obj_h * p.obj_w)) || (st = dev_alloc(c, &probe, K * nn)) ||
      (st = dev_alloc(c, &pw, nn)) || (st = dev_alloc(c, &amp, (size_t)p.n_pos * nn)) ||
      (st = dev_alloc(c, &pos, (size_t)p.n_pos)) || (st = dev_alloc(c, &tw, (size_t)n)) ||
      (st = dev_alloc(c, &hn, (size_t)n)) || (st = dev_alloc(c, &X, (size_t)B * K * nn)) ||
      (st = dev_alloc(c, &q, (size_t)B * nn)) ||
      (st = dev_alloc(c, &dO, (size_t)B * nn)) || (st = dev_alloc(c, &nP, K * nn)) || (st = dev_alloc(c, &V, nn)) ||
      (st = dev_alloc(c, &maxv, (size_t)n_probe_blocks(n))) || (st = dev_alloc(c, &maxw, (size_t)nobjt)) ||
      (st = dev_alloc(c, &errp, (size_t)p.n_pos * nbt)) || (st = dev_alloc(c, &ccp, (size_t)nobjt)) ||
      (st = dev_alloc(c, &gramp, (size_t)(K * (K + 1) / 2) * kGramBlocks)) || (st = dev_alloc(c, &vmix, (size_t)K * K)) ||
      (st = dev_alloc(c, &eig, (size_t)K)))
    return bail(st);
  d.obj = obj;
  d.probe = probe;
  d.pw = pw;
  d.amp = amp;
  d.pos = pos;
  d.tw = tw;
  d.hnear = hn;
  d.X = X;
  d.q = q;
  d.dO = dO;
  d.nP = nP;
  d.V = V;
  d.maxv_part = maxv;
  d.maxw_part = maxw;
  d.err_part = errp;
  d.cc_part = ccp;
  d.gram_part = gramp;
  d.vmix = vmix;
  d.eig = eig;
  c->n_err_part = p.n_pos * nbt;

  // tables (double precision on the host)
  std::vector<float2> htw(n), hh(n);
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * pi * m / n;
    htw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    const double u = (m < n / 2) ? m : m - n;  // signed index (n even)
    const double ph = dp.near_field ? -pi * u * u / ((double)n * n * p.fresnel_px) : 0.0;
    hh[m] = make_float2((float)std::cos(ph), (float)std::sin(ph));
  }
  std::vector<int2> hp2(p.n_pos);
  for (int i = 0; i < p.n_pos; ++i) hp2[i] = make_int2(hpos[2 * i], hpos[2 * i + 1]);
  hipStream_t s = c->stream;
#define INIT_TRY(expr)                                                                                   \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess) {                                                                              \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                                        \
      return bail(PTYCHO_E_HIP);                                                                         \
    }                                                                                                    \
  } while (0)
  INIT_TRY(hipMemcpyAsync(tw, htw.data(), n * sizeof(float2), hipMemcpyHostToDevice, s));
  INIT_TRY(hipMemcpyAsync(hn, hh.data(), n * sizeof(float2), hipMemcpyHostToDevice, s));
  INIT_TRY(hipMemcpyAsync(pos, hp2.data(), p.n_pos * sizeof(int2), hipMemcpyHostToDevice, s));
  INIT_TRY(hipMemcpyAsync(obj, object0, (size_t)p.obj_h * p.obj_w * sizeof(float2), kind_in(mem_kind), s));
  INIT_TRY(hipMemcpyAsync(probe, probe0, K * nn * sizeof(float2), kind_in(mem_kind), s));
  INIT_TRY(hipMemsetAsync(errp, 0, (size_t)p.n_pos * nbt * sizeof(double), s));
  // measured amplitudes: raw intensities staged in a temporary device buffer
  float* raw = nullptr;
  if (mem_kind == PTYCHO_MEM_HOST) {
    st = dev_alloc(c, &raw, (size_t)p.n_pos * nn);
    if (st != PTYCHO_OK) return bail(st);
    INIT_TRY(hipMemcpyAsync(raw, intensities, (size_t)p.n_pos * nn * sizeof(float), hipMemcpyHostToDevice, s));
  } else {
    raw = const_cast<float*>(intensities);
  }
  int* d_bad = nullptr;
  double* d_sum = nullptr;
  const int gx = 8;
  if ((st = dev_alloc(c, &d_bad, (size_t)p.n_pos * gx)) || (st = dev_alloc(c, &d_sum, (size_t)p.n_pos * gx)))
    return bail(st);
  INIT_TRY(launch_prepare_amp(raw, amp, n, p.n_pos, p.geometry == PTYCHO_FAR_FIELD, d_bad, d_sum, s));
  INIT_TRY(launch_pw(dp, d, s));
  std::vector<int> hb((size_t)p.n_pos * gx);
  std::vector<double> hs((size_t)p.n_pos * gx);
  INIT_TRY(hipMemcpyAsync(hb.data(), d_bad, hb.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  INIT_TRY(hipMemcpyAsync(hs.data(), d_sum, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  INIT_TRY(hipStreamSynchronize(s));
  // free the init temporaries
  auto drop = [&](void* ptr) {
    if (!ptr) return;
    (void)hipFree(ptr);
    c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), ptr));
  };
  if (mem_kind == PTYCHO_MEM_HOST) drop(raw);
  drop(d_bad);
  drop(d_sum);
  long long nbad = 0;
  double denom = 0.0;
  for (size_t i = 0; i < hb.size(); ++i) {
    nbad += hb[i];
    denom += hs[i];
  }
  if (nbad) {
    c->err = "intensities contain " + std::to_string(nbad) + " non-finite values";
    return bail(PTYCHO_E_INVALID);
  }
  c->inv_denom = denom > 0 ? 1.0 / denom : 0.0;
  *out = c;
  return PTYCHO_OK;
}

ptycho_status ptycho_iterate(ptycho_ctx* c, int32_t n_iter, const int32_t* order, float* err_out) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (c->failed) return fail(c, PTYCHO_E_STATE, "context failed earlier: " + c->err);
  if (n_iter < 0) return fail(c, PTYCHO_E_INVALID, "n_iter must be >= 0");
  if (n_iter == 0) return PTYCHO_OK;
  const int np = c->prm.n_pos;
  ptycho_status st = ensure_order_capacity(c, (size_t)n_iter * np);
  if (st != PTYCHO_OK) return st;
  if ((st = ensure_err_capacity(c, (size_t)n_iter)) != PTYCHO_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // the pinned staging buffer may be in use
  std::vector<char> seen(np);
  for (int it = 0; it < n_iter; ++it) {
    int32_t* row = c->h_order + (size_t)it * np;
    if (order) {
      std::memcpy(row, order + (size_t)it * np, np * sizeof(int32_t));
      std::fill(seen.begin(), seen.end(), 0);
      for (int i = 0; i < np; ++i) {
        if (row[i] < 0 || row[i] >= np || seen[row[i]])
          return fail(c, PTYCHO_E_INVALID, "order row " + std::to_string(it) + " is not a permutation of 0..n_pos-1");
        seen[row[i]] = 1;
      }
    } else {
      splitmix_perm(c->prm.seed, c->t + 1 + it, np, row);
    }
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_order, c->h_order, (size_t)n_iter * np * sizeof(int32_t), hipMemcpyHostToDevice,
                            c->stream));
  const int B = c->prm.batch;
  DebugPtrs none{nullptr, nullptr, nullptr, nullptr};
  for (int it = 0; it < n_iter; ++it) {
    const int t = c->t + 1 + it;
    const int* ord = c->d_order + (size_t)it * np;
    for (int s0 = 0; s0 < np; s0 += B) {
      st = run_batch(c, ord + s0, std::min(B, np - s0), t, none);
      if (st != PTYCHO_OK) return st;
    }
    if ((st = end_iteration(c, c->d_err + it)) != PTYCHO_OK) return st;
  }
  std::vector<float> herr(n_iter);
  HIP_TRY(c, hipMemcpyAsync(herr.data(), c->d_err, n_iter * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->tm.used) harvest_timing(c);
  c->t += n_iter;
  if (err_out) std::memcpy(err_out, herr.data(), n_iter * sizeof(float));
  for (int i = 0; i < n_iter; ++i)
    if (!std::isfinite(herr[i])) {
      c->failed = true;
      return fail(c, PTYCHO_E_NUMERIC, "non-finite data error at iteration " + std::to_string(c->t - n_iter + 1 + i));
    }
  return PTYCHO_OK;
}

ptycho_status ptycho_get_object(ptycho_ctx* c, float* out, int32_t mem_kind) {
  if (!c || !out) return fail(c, PTYCHO_E_INVALID, "NULL argument");
  HIP_TRY(c, hipMemcpyAsync(out, c->db.obj, (size_t)c->prm.obj_h * c->prm.obj_w * sizeof(float2), kind_out(mem_kind),
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PTYCHO_OK;
}

ptycho_status ptycho_get_probe(ptycho_ctx* c, float* out, int32_t mem_kind) {
  if (!c || !out) return fail(c, PTYCHO_E_INVALID, "NULL argument");
  const size_t nn = (size_t)c->prm.n * c->prm.n;
  HIP_TRY(c, hipMemcpyAsync(out, c->db.probe, c->prm.n_modes * nn * sizeof(float2), kind_out(mem_kind), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PTYCHO_OK;
}

ptycho_status ptycho_set_state(ptycho_ctx* c, const float* object, const float* probe, int32_t iter,
                               int32_t mem_kind) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (iter < 0) return fail(c, PTYCHO_E_INVALID, "iter must be >= 0");
  const size_t nn = (size_t)c->prm.n * c->prm.n;
  if (probe) {
    std::vector<float> hp;
    ptycho_status st = fetch_host(c, probe, 2 * c->prm.n_modes * nn, mem_kind, hp);
    if (st == PTYCHO_OK) st = check_probe_power(c, hp.data(), hp.size());
    if (st != PTYCHO_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(c->db.probe, probe, c->prm.n_modes * nn * sizeof(float2), kind_in(mem_kind), c->stream));
    HIP_TRY(c, launch_pw(c->dp, c->db, c->stream));
  }
  if (object)
    HIP_TRY(c, hipMemcpyAsync(c->db.obj, object, (size_t)c->prm.obj_h * c->prm.obj_w * sizeof(float2),
                              kind_in(mem_kind), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->t = iter;
  c->failed = false;
  return PTYCHO_OK;
}

int32_t ptycho_iteration(const ptycho_ctx* c) { return c ? c->t : -1; }

ptycho_status ptycho_debug_step(ptycho_ctx* c, const int32_t* idx, int32_t B, int32_t t, float* psi,
                                float* psi_new, float* factor, float* n_obj, float* w_obj, float* n_probe,
                                float* v_probe, int32_t mem_kind) {
  if (!c || !idx) return fail(c, PTYCHO_E_INVALID, "NULL argument");
  if (c->failed) return fail(c, PTYCHO_E_STATE, "context failed earlier: " + c->err);
  if (B < 1 || B > c->prm.batch) return fail(c, PTYCHO_E_INVALID, "B must be in [1, batch]");
  if (t < 1) return fail(c, PTYCHO_E_INVALID, "t must be >= 1");
  if ((n_obj == nullptr) != (w_obj == nullptr)) return fail(c, PTYCHO_E_INVALID, "n_obj and w_obj go together");
  for (int i = 0; i < B; ++i)
    if (idx[i] < 0 || idx[i] >= c->prm.n_pos) return fail(c, PTYCHO_E_INVALID, "index out of range");
  ptycho_status st = ensure_order_capacity(c, (size_t)std::max(B, c->prm.n_pos));
  if (st != PTYCHO_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(c->h_order, idx, B * sizeof(int32_t));
  HIP_TRY(c, hipMemcpyAsync(c->d_order, c->h_order, B * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  const int n = c->prm.n, K = c->prm.n_modes;
  const size_t nn = (size_t)n * n, no = (size_t)c->prm.obj_h * c->prm.obj_w;
  // device staging for the captures
  float2 *d_psi = nullptr, *d_psin = nullptr, *d_nobj = nullptr;
  float* d_wobj = nullptr;
  std::vector<void*> tmp;
  auto alloc_tmp = [&](size_t bytes, void** p) -> bool {
    if (hipMalloc(p, bytes) != hipSuccess) return false;
    tmp.push_back(*p);
    return true;
  };
  auto cleanup = [&]() {
    for (void* p : tmp) (void)hipFree(p);
  };
  bool ok = true;
  if (psi) ok = ok && alloc_tmp((size_t)B * K * nn * sizeof(float2), (void**)&d_psi);
  if (psi_new) ok = ok && alloc_tmp((size_t)B * K * nn * sizeof(float2), (void**)&d_psin);
  if (n_obj) ok = ok && alloc_tmp(no * sizeof(float2), (void**)&d_nobj) && alloc_tmp(no * sizeof(float), (void**)&d_wobj);
  if (!ok) {
    cleanup();
    return fail(c, PTYCHO_E_OOM, "debug staging allocation failed");
  }
  if (d_nobj) {
    (void)hipMemsetAsync(d_nobj, 0, no * sizeof(float2), c->stream);
    (void)hipMemsetAsync(d_wobj, 0, no * sizeof(float), c->stream);
  }
  if (n_probe) (void)hipMemsetAsync(c->db.nP, 0, K * nn * sizeof(float2), c->stream);
  if (v_probe) (void)hipMemsetAsync(c->db.V, 0, nn * sizeof(float), c->stream);
  if (d_psi) {
    hipError_t e = launch_exit_waves(c->dp, c->db, c->d_order, B, d_psi, c->stream);
    if (e != hipSuccess) {
      cleanup();
      return fail(c, PTYCHO_E_HIP, std::string("exit waves: ") + hipGetErrorString(e));
    }
  }
  float* d_fac = nullptr;
  if (factor && !alloc_tmp((size_t)B * nn * sizeof(float), (void**)&d_fac)) {
    cleanup();
    return fail(c, PTYCHO_E_OOM, "debug staging allocation failed");
  }
  DebugPtrs dbg{d_psin, d_nobj, d_wobj, d_fac};
  st = run_batch(c, c->d_order, B, t, dbg);
  auto copy = [&](float* dst, const void* src, size_t bytes) -> hipError_t {
    return dst ? hipMemcpyAsync(dst, src, bytes, kind_out(mem_kind), c->stream) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  if (st == PTYCHO_OK) {
    if (e == hipSuccess) e = copy(psi, d_psi, (size_t)B * K * nn * sizeof(float2));
    if (e == hipSuccess) e = copy(psi_new, d_psin, (size_t)B * K * nn * sizeof(float2));
    if (e == hipSuccess) e = copy(factor, d_fac, (size_t)B * nn * sizeof(float));
    if (e == hipSuccess) e = copy(n_obj, d_nobj, no * sizeof(float2));
    if (e == hipSuccess) e = copy(w_obj, d_wobj, no * sizeof(float));
    if (e == hipSuccess) e = copy(n_probe, c->db.nP, K * nn * sizeof(float2));
    if (e == hipSuccess) e = copy(v_probe, c->db.V, nn * sizeof(float));
    hipError_t e2 = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = e2;
  } else {
    (void)hipStreamSynchronize(c->stream);
  }
  if (c->tm.used) harvest_timing(c);
  cleanup();
  if (st != PTYCHO_OK) return st;
  if (e != hipSuccess) return fail(c, PTYCHO_E_HIP, std::string("debug copies: ") + hipGetErrorString(e));
  return PTYCHO_OK;
}

ptycho_status ptycho_set_timing(ptycho_ctx* c, uint32_t mask) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  c->tm.mask = mask;
  return PTYCHO_OK;
}

ptycho_status ptycho_kernel_time(ptycho_ctx* c, int32_t cls, double* total_ms, int64_t* launches, int32_t reset) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (cls < 0 || cls >= KC_COUNT) return fail(c, PTYCHO_E_INVALID, "kernel class out of range");
  if (total_ms) *total_ms = c->tm.total_ms[cls];
  if (launches) *launches = c->tm.launches[cls];
  if (reset) {
    c->tm.total_ms[cls] = 0.0;
    c->tm.launches[cls] = 0;
  }
  return PTYCHO_OK;
}

const char* ptycho_kernel_name(int32_t cls) { return (cls >= 0 && cls < KC_COUNT) ? kKernelNames[cls] : nullptr; }
int32_t ptycho_kernel_class_count(void) { return KC_COUNT; }

void ptycho_destroy(ptycho_ctx* c) {
  if (!c) return;
  if (c->stream || true) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->tm.pool) (void)hipEventDestroy(e);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->h_order) (void)hipHostFree(c->h_order);
  delete c;
}

const char* ptycho_last_error(const ptycho_ctx* c) { return c ? c->err.c_str() : g_thread_error.c_str(); }

}  // extern "C"
