// Host runtime of the pc-ePIE library: validation, device memory, the iteration
// schedule (eager or replayed from a captured HIP graph), groups of
// independent reconstructions, the column-tile autotuner, and the C ABI
// declared in include/ptycho.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
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

// Device and pinned host buffers of one call's schedule (orders, flags, errors).
struct CallBufs {
  int* d_order = nullptr;
  int* h_order = nullptr;
  size_t order_cap = 0;
  int* d_flags = nullptr;
  int* h_flags = nullptr;
  float* d_err = nullptr;
  float* h_err = nullptr;
  size_t iter_cap = 0;
};

}  // namespace

struct ptycho_ctx {
  ptycho_params prm{};
  DevParams dp{};
  DevBufs db{};
  hipStream_t stream = nullptr;
  int device = 0;
  int t = 0;
  int pw_par = 0;          // copy of db.pw that holds sum_k |P_k|^2 of the current probe
  int pw_par_next = 0;     // the same after the staged call has run
  bool failed = false;
  std::string err;
  double inv_denom = 0.0;  // 1 / sum_n sum_q I_n
  std::vector<void*> allocs;
  CallBufs call;
  int* d_iter = nullptr;           // device iteration counter of the current call
  CaseDesc* h_case = nullptr;      // pinned staging of the case table (one entry)
  CaseDesc* d_case = nullptr;
  CaseDesc* d_case_dbg = nullptr;  // table used by ptycho_debug_step
  int* d_dbg_order = nullptr;      // [batch]
  int* d_dbg_flags = nullptr;      // [1]
  int* d_dbg_iter = nullptr;
  float* d_dbg_err = nullptr;
  int col_variant = 1;
  bool seq = false;          // whole iterations in the sequential kernel (batch 1, small far-field frames)
  void* d_planes = nullptr;  // bf16 DFT table planes (dft_bf16 path)
  // graph replay of one iteration
  bool use_graph = false;
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  Timing tm;
};

struct ptycho_mono {
  int n = 0, max_pat = 0;
  MonoWork w{};
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  float *d_in = nullptr, *d_out = nullptr;  // staging of host patterns
  float* d_res = nullptr;                   // residual history
  size_t res_cap = 0;
};

struct ptycho_group {
  std::vector<ptycho_ctx*> ctx;
  struct Table {
    TableShape shape{};
    std::vector<int> members;  // indices into ctx
    bool seq = false;          // members run whole iterations in the sequential kernel
    CaseDesc* d_cases = nullptr;
    CaseDesc* h_cases = nullptr;  // pinned
    int max_nb = 0;               // batches per iteration of its member with the most
  };
  std::vector<Table> tables;
  // tables run concurrently, table i on side[i % side.size()], forked from and joined
  // back into the calling stream each iteration (no side streams for one table)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_done;
  hipEvent_t fork = nullptr;
  hipStream_t stream = nullptr;
  CallBufs call;
  int* d_iter = nullptr;
  std::vector<void*> allocs;
  std::string err;
  // iteration replay from a captured graph
  bool use_graph = false;
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace {

ptycho_status fail(ptycho_ctx* c, ptycho_status st, const std::string& msg) {
  if (c) c->err = msg;
  else g_thread_error = msg;
  return st;
}
ptycho_status gfail(ptycho_group* g, ptycho_status st, const std::string& msg) {
  if (g) g->err = msg;
  else g_thread_error = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((ctx), PTYCHO_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define HIP_GTRY(g, expr)                                                                \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return gfail((g), PTYCHO_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
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
  if (p->dft_bf16 != 0 && p->dft_bf16 != 1) return "dft_bf16 must be 0 or 1";
  if (p->dft_bf16 && (p->geometry != PTYCHO_FAR_FIELD || !dft_supported(p->n)))
    return "dft_bf16 needs the far field and n in {64, 128, 192, 256}";
  if (p->engine != PTYCHO_ENGINE_EPIE && p->engine != PTYCHO_ENGINE_DM && p->engine != PTYCHO_ENGINE_LSQML)
    return "bad engine";
  if (p->engine == PTYCHO_ENGINE_LSQML && !(finite_f(p->lsq_damping) && p->lsq_damping >= 0))
    return "lsq_damping must be finite and >= 0";
  if (p->engine == PTYCHO_ENGINE_DM) {
    if (!(finite_f(p->dm_reg) && p->dm_reg > 0)) return "dm_reg must be finite and > 0";
    if (p->dft_bf16) return "the pc-DM engine runs the FP32 transforms (dft_bf16 must be 0)";
  }
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


template <typename T>
void drop_alloc(std::vector<void*>& allocs, T*& ptr) {
  if (!ptr) return;
  (void)hipFree(ptr);
  auto it = std::find(allocs.begin(), allocs.end(), (void*)ptr);
  if (it != allocs.end()) allocs.erase(it);
  ptr = nullptr;
}

// Grow the schedule buffers to orders for `n_order` ints and `n_iter` iterations.
template <class Owner>
bool grow_call(Owner* o, std::vector<void*>& allocs, CallBufs& cb, size_t n_order, size_t n_iter) {
  if (n_order > cb.order_cap) {
    drop_alloc(allocs, cb.d_order);
    if (cb.h_order) (void)hipHostFree(cb.h_order);
    cb.h_order = nullptr;
    cb.order_cap = 0;
    void* p = nullptr;
    if (hipMalloc(&p, n_order * sizeof(int)) != hipSuccess) return false;
    allocs.push_back(p);
    cb.d_order = (int*)p;
    if (hipHostMalloc((void**)&cb.h_order, n_order * sizeof(int), hipHostMallocDefault) != hipSuccess) return false;
    cb.order_cap = n_order;
  }
  if (n_iter > cb.iter_cap) {
    drop_alloc(allocs, cb.d_flags);
    drop_alloc(allocs, cb.d_err);
    if (cb.h_flags) (void)hipHostFree(cb.h_flags);
    if (cb.h_err) (void)hipHostFree(cb.h_err);
    cb.h_flags = nullptr;
    cb.h_err = nullptr;
    cb.iter_cap = 0;
    void* p = nullptr;
    if (hipMalloc(&p, n_iter * sizeof(int)) != hipSuccess) return false;
    allocs.push_back(p);
    cb.d_flags = (int*)p;
    if (hipMalloc(&p, n_iter * sizeof(float)) != hipSuccess) return false;
    allocs.push_back(p);
    cb.d_err = (float*)p;
    if (hipHostMalloc((void**)&cb.h_flags, n_iter * sizeof(int), hipHostMallocDefault) != hipSuccess) return false;
    if (hipHostMalloc((void**)&cb.h_err, n_iter * sizeof(float), hipHostMallocDefault) != hipSuccess) return false;
    cb.iter_cap = n_iter;
  }
  (void)o;
  return true;
}

void free_call(CallBufs& cb) {
  if (cb.h_order) (void)hipHostFree(cb.h_order);
  if (cb.h_flags) (void)hipHostFree(cb.h_flags);
  if (cb.h_err) (void)hipHostFree(cb.h_err);
  cb = CallBufs{};
}

// Time one launch of class `cls` if selected.
struct Timed {
  ptycho_ctx* c;
  hipStream_t s;
  hipEvent_t stop = nullptr;
  Timed(ptycho_ctx* ctx, int k, hipStream_t st) : c(ctx), s(st) {
    if (!c || !(c->tm.mask & (1u << k))) return;
    if (c->tm.used * 2 + 2 > c->tm.pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        // timing only (read after a stream synchronisation): no system-scope fence, which
        // would add a cache write-back and invalidation to every timed launch
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return;
        c->tm.pool.push_back(e);
      }
    }
    hipEvent_t start = c->tm.pool[c->tm.used * 2];
    stop = c->tm.pool[c->tm.used * 2 + 1];
    c->tm.cls.resize(c->tm.used + 1);
    c->tm.cls[c->tm.used] = k;
    c->tm.used++;
    // recorded by the launched kernels themselves (LaunchEvents)
    launch_events() = LaunchEvents{start, stop};
  }
  ~Timed() {
    if (!stop) return;
    LaunchEvents& ev = launch_events();
    if (ev.start) {  // nothing was launched: an empty interval
      (void)hipEventRecord(ev.start, s);
      (void)hipEventRecord(stop, s);
    }
    ev = LaunchEvents{};
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

// Launch `expr`; on failure return the HIP error text.  `tc` (may be null) times it.
#define LAUNCH(tc, cls, s, expr)                                                           \
  do {                                                                                     \
    hipError_t e_;                                                                         \
    {                                                                                      \
      Timed tmd_((tc), (cls), (s));                                                        \
      e_ = (expr);                                                                         \
    }                                                                                      \
    if (e_ != hipSuccess) return std::string(kKernelNames[cls]) + ": " + hipGetErrorString(e_); \
  } while (0)

// The seven launches of batch `beta` for every case of a table (five when the
// fused middle pass replaces fwd_cols, modulus_factor and inv_cols).
// The column passes of batch `beta`: forward columns, mode sum, blur, modulus
// factor, inverse columns (or the fused middle pass).
std::string launch_middle(ptycho_ctx* tc, const CaseDesc* cases, const TableShape& sh, int beta, const int* it,
                          hipStream_t s) {
  if (fused_active(sh.n, sh.col_variant, sh.max_half)) {
    LAUNCH(tc, KC_COLS_FUSED, s, launch_cols_fused(cases, sh, beta, it, s));
  } else {
    LAUNCH(tc, KC_FWD_COLS, s, launch_fwd_cols(cases, sh, beta, it, s));
    LAUNCH(tc, KC_FACTOR, s, launch_factor(cases, sh, beta, it, s));
    LAUNCH(tc, KC_INV_COLS, s, launch_inv_cols(cases, sh, beta, it, s));
  }
  return "";
}

// The updates of batch `beta` once the per-slot numerators are in place: the
// pc-ePIE / pc-rPIE update, or pc-LSQML's directions, step sums, step solve and
// update along the directions; then the complex constraint.
std::string launch_updates(ptycho_ctx* tc, const CaseDesc* cases, const TableShape& sh, int beta, const int* it,
                           hipStream_t s, bool lsq) {
  if (lsq) {
    LAUNCH(tc, KC_LSQ_DIR, s, launch_lsq_dir(cases, sh, beta, it, s));
    LAUNCH(tc, KC_LSQ_STEP, s, launch_lsq_sums(cases, sh, beta, it, s));
    LAUNCH(tc, KC_LSQ_STEP, s, launch_lsq_solve(cases, sh, beta, it, s));
    LAUNCH(tc, KC_LSQ_APPLY, s, launch_lsq_apply(cases, sh, beta, it, s));
  } else {
    LAUNCH(tc, KC_OBJ_UPDATE, s, launch_obj_update(cases, sh, beta, it, s));
  }
  LAUNCH(tc, KC_CONSTRAINT, s, launch_constraint(cases, sh, beta, it, s));
  return "";
}

std::string launch_batch(ptycho_ctx* tc, const CaseDesc* cases, const TableShape& sh, int beta, const int* it,
                         hipStream_t s, bool lsq = false) {
  LAUNCH(tc, KC_FWD_ROWS, s, launch_fwd_rows(cases, sh, beta, it, s));
  std::string e = launch_middle(tc, cases, sh, beta, it, s);
  if (!e.empty()) return e;
  LAUNCH(tc, KC_INV_ROWS, s, launch_inv_rows(cases, sh, beta, it, s));
  return launch_updates(tc, cases, sh, beta, it, s, lsq);
}

// Mode orthogonalisation (cases flagged) and the data error of every case.
std::string launch_end(ptycho_ctx* tc, const CaseDesc* cases, const TableShape& sh, const int* it, hipStream_t s) {
  if (sh.max_k > 1) {
    LAUNCH(tc, KC_GRAM, s, launch_gram(cases, sh, it, s));
    LAUNCH(tc, KC_EIG, s, launch_eig(cases, sh, it, s));
    LAUNCH(tc, KC_REMIX, s, launch_remix(cases, sh, it, s));
  }
  LAUNCH(tc, KC_ERR, s, launch_err_reduce(cases, sh, it, s));
  return "";
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


int case_flags(const ptycho_params& p, int t) {
  int f = 0;
  if (t >= p.probe_update_start) f |= FLAG_PROBE;
  if (in_window(p, t)) f |= FLAG_CC;
  if (p.n_modes > 1 && p.orthogonalize) f |= FLAG_ORTHO;
  return f;
}

int n_batches_of(const ptycho_params& p) { return (p.n_pos + p.batch - 1) / p.batch; }

// The sequential kernel runs ePIE iterations of batch size 1 on small far-field frames.
bool seq_eligible(const ptycho_params& p) {
  return p.batch == 1 && !p.dft_bf16 && p.engine == PTYCHO_ENGINE_EPIE &&
         seq_supported(p.n, p.geometry == PTYCHO_NEAR_FIELD);
}
// Launch variant index of the sequential kernel (after the batch-pass variants).
constexpr int kSeqVariant = kColVariants;
// Side streams of a group (one frame-size class each; within the box's hardware queues).
constexpr size_t kGroupStreams = 4;

// Fill the per-case fields of a table entry for the current call.
void fill_case(const ptycho_ctx* c, CaseDesc& cd, const int* order, const int* flags, float* err) {
  cd.p = c->dp;
  cd.d = c->db;
  cd.dbg = DebugPtrs{nullptr, nullptr, nullptr, nullptr};
  cd.order = order;
  cd.flags = flags;
  cd.err_out = err;
  cd.inv_denom = c->inv_denom;
  cd.n_pos = c->prm.n_pos;
  cd.batch = c->prm.batch;
  cd.n_batches = n_batches_of(c->prm);
  cd.n_err_part = c->prm.n_pos * (c->prm.dft_bf16 ? dft_err_slots(c->prm.n) : n_err_slots(c->prm.n, c->col_variant, c->dp.ks_half));
}

TableShape single_shape(const ptycho_ctx* c, int max_batch) {
  TableShape sh{};
  sh.n = c->prm.n;
  sh.near_field = c->prm.geometry == PTYCHO_NEAR_FIELD;
  sh.n_cases = 1;
  sh.max_batch = max_batch;
  sh.max_tiles = n_obj_tiles(c->dp);
  sh.max_k = c->prm.n_modes;
  sh.max_side_jobs = sh.max_tiles + n_probe_blocks(c->prm.n);
  sh.col_variant = c->col_variant;
  sh.max_half = c->dp.ks_half;
  sh.max_dm_segments = c->prm.engine == PTYCHO_ENGINE_DM ? dm_segments(c->prm.n_pos, c->dp.dm_seg_len) : 0;
  // pc-LSQML's step sums read every slot's own probe contributions, and the dft_bf16
  // path writes them per slot
  sh.x_pairs = c->prm.engine == PTYCHO_ENGINE_EPIE && !c->prm.dft_bf16 && max_batch >= 2 && inv_rows_paired(sh.n);
  return sh;
}

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_val(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Host-built split planes (re_hi, re_lo, im_hi, im_lo) of
// F[u][x] = exp(-2 pi i u x / n) / sqrt(n), evaluated in double, each stored in
// MFMA fragment order: [u / 16][x / 32][lane = 16 ((x % 32) / 8) + u % 16][x % 8],
// so that the 16 x 32 fragment a wave needs is one contiguous 1 KB read.
static size_t dft_frag_index(int n, int plane, int u, int x) {
  const int lane = 16 * ((x % 32) / 8) + u % 16;
  return ((((size_t)plane * (n / 16) + u / 16) * (n / 32) + x / 32) * 64 + lane) * 8 + x % 8;
}
std::vector<uint16_t> dft_planes(int n) {
  std::vector<uint16_t> pl((size_t)4 * n * n);
  const double pi = 3.14159265358979323846, sc = 1.0 / std::sqrt((double)n);
  for (int u = 0; u < n; ++u)
    for (int x = 0; x < n; ++x) {
      const double a = -2.0 * pi * (double)(((long long)u * x) % n) / n;
      const double v[2] = {std::cos(a) * sc, std::sin(a) * sc};
      for (int c = 0; c < 2; ++c) {
        const uint16_t hi = bf16_rne((float)v[c]);
        const uint16_t lo = bf16_rne((float)(v[c] - (double)bf16_val(hi)));
        pl[dft_frag_index(n, 2 * c, u, x)] = hi;
        pl[dft_frag_index(n, 2 * c + 1, u, x)] = lo;
      }
    }
  return pl;
}

// The batch of the dft_bf16 path: the same updates as launch_batch, with the
// two FFT passes per direction replaced by BF16 matrix-core DFT GEMMs.
std::string launch_batch_dft(ptycho_ctx* tc, const ptycho_ctx* c, const CaseDesc* cases, float2* X,
                             const TableShape& sh, int beta, int ns, const int* it, hipStream_t s) {
  const int frames = ns * c->prm.n_modes;
  LAUNCH(tc, KC_DFT_OTHER, s, launch_dft_side(cases, sh, beta, it, s));
  LAUNCH(tc, KC_DFT_GEMM, s, launch_dft2_exit(X, c->d_planes, cases, beta, it, sh.n, frames, s));
  LAUNCH(tc, KC_DFT_OTHER, s, launch_dft_modsum(cases, sh, beta, it, s));
  LAUNCH(tc, KC_DFT_OTHER, s, launch_dft_blur_apply(cases, sh, beta, it, s));
  LAUNCH(tc, KC_DFT_GEMM, s, launch_dft2(X, c->d_planes, sh.n, frames, true, s));
  LAUNCH(tc, KC_DFT_OTHER, s, launch_dft_delta(cases, sh, beta, it, s));
  return launch_updates(tc, cases, sh, beta, it, s, c->prm.engine == PTYCHO_ENGINE_LSQML);
}

// One batch of a single context (either propagation path); X is the work-frame
// buffer the case table `cases` points at.
std::string launch_one(ptycho_ctx* tc, const ptycho_ctx* c, const CaseDesc* cases, float2* X, const TableShape& sh,
                       int beta, int ns, const int* it, hipStream_t s) {
  if (c->prm.dft_bf16) return launch_batch_dft(tc, c, cases, X, sh, beta, ns, it, s);
  return launch_batch(tc, cases, sh, beta, it, s, c->prm.engine == PTYCHO_ENGINE_LSQML);
}

// One iteration of a single context on stream s from the case table `cases`
// (work buffers X) and the device iteration counter `it`.
std::string enqueue_iteration_on(ptycho_ctx* c, const CaseDesc* cases, float2* X, int* it, hipStream_t s,
                                 bool timed) {
  const TableShape sh = single_shape(c, c->prm.batch);
  ptycho_ctx* tc = timed ? c : nullptr;
  const int nb = n_batches_of(c->prm);
  if (c->prm.engine == PTYCHO_ENGINE_DM) {
    // pc-DM: overlap projection over every position, then the Fourier step batch by batch
    LAUNCH(tc, KC_DM_OVERLAP, s, launch_dm_overlap(cases, sh, it, s));
    for (int beta = 0; beta < nb; ++beta) {
      LAUNCH(tc, KC_DM_ROWS, s, launch_dm_rows_fwd(cases, sh, beta, it, s));
      std::string e = launch_middle(tc, cases, sh, beta, it, s);
      if (!e.empty()) return e;
      LAUNCH(tc, KC_DM_ROWS, s, launch_dm_rows_inv(cases, sh, beta, it, s));
    }
    LAUNCH(tc, KC_ERR, s, launch_err_reduce(cases, sh, it, s));
    hipError_t he = launch_iter_advance(it, s);
    if (he != hipSuccess) return std::string("iter_advance: ") + hipGetErrorString(he);
    return "";
  }
  if (c->seq) {
    LAUNCH(tc, KC_SEQ, s, launch_seq_iter(cases, sh, it, s));
  } else {
    for (int beta = 0; beta < nb; ++beta) {
      const int ns = std::min(c->prm.batch, c->prm.n_pos - beta * c->prm.batch);
      std::string e = launch_one(tc, c, cases, X, sh, beta, ns, it, s);
      if (!e.empty()) return e;
    }
  }
  std::string e = launch_end(tc, cases, sh, it, s);
  if (!e.empty()) return e;
  hipError_t he = launch_iter_advance(it, s);
  if (he != hipSuccess) return std::string("iter_advance: ") + hipGetErrorString(he);
  return "";
}

// One iteration of a single context on its own buffers (eager or under capture).
std::string enqueue_iteration(ptycho_ctx* c, hipStream_t s, bool timed) {
  return enqueue_iteration_on(c, c->d_case, c->db.X, c->d_iter, s, timed);
}

void drop_graph(ptycho_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
}

ptycho_status build_graph(ptycho_ctx* c) {
  if (c->gexec) return PTYCHO_OK;
  if (!c->gstream) HIP_TRY(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
  if (!c->ev_in) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  if (!c->ev_out) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  HIP_TRY(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
  std::string e = enqueue_iteration(c, c->gstream, false);
  hipGraph_t graph = nullptr;
  hipError_t he = hipStreamEndCapture(c->gstream, &graph);
  if (!e.empty()) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(c, PTYCHO_E_HIP, "capturing the iteration: " + e);
  }
  if (he != hipSuccess) return fail(c, PTYCHO_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
  he = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (he != hipSuccess) {
    c->gexec = nullptr;
    return fail(c, PTYCHO_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
  }
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


// ---------------------------------------------------------------------------
// Column-tile autotuner: times each valid column-block width on the first
// batch of a context, keeps the fastest; results are cached per
// (n, K, batch, geometry) for the process, and in the file named by the
// environment variable PTYCHO_TUNE_CACHE if it is set.
// ---------------------------------------------------------------------------

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("PTYCHO_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  int n, k, b, g, v;
  while (f >> n >> k >> b >> g >> v)
    if (v >= 0 && v < kColVariants) g_tune[std::make_tuple(n, k, b, g)] = v;
}

void tune_store_locked(const std::tuple<int, int, int, int>& key, int v) {
  g_tune[key] = v;
  const char* path = std::getenv("PTYCHO_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << std::get<0>(key) << ' ' << std::get<1>(key) << ' ' << std::get<2>(key) << ' ' << std::get<3>(key) << ' ' << v
    << '\n';
}

// ---------------------------------------------------------------------------
// Static scratch of ptycho_iterate_static.  The work frames, partial sums,
// schedule and case table of its iterations live in this file-scope device
// array, so the call allocates nothing.  In host code `scratch` names only a
// host-side handle: kernels are given the device address that
// hipGetSymbolAddress returns for the current device (each device holds its
// own copy of the array), resolved once per device and kept in g_static_ptr.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kDmSegLen = 64;  // pc-DM: positions per probe-numerator partial sum
constexpr size_t kStaticOrderInts = (size_t)1 << 18;  // schedule entries staged per chunk of iterations
constexpr int kStaticMaxChunk = 1024;                 // iterations per chunk
constexpr int kStaticMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Grid-stride zero fill of `words` 8-byte words (a kernel rather than a memset,
// so the clearing is an ordinary kernel node should a caller capture the stream).
__global__ void k_static_zero(unsigned long long* __restrict__ p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

namespace {

std::mutex g_static_ptr_mu;
void* g_static_ptr[kStaticMaxDevices] = {};
// host staging of one chunk's schedule (guarded by g_static_mu; calls are serialised)
std::mutex g_static_mu;
int32_t g_static_order[kStaticOrderInts];
int g_static_flags[kStaticMaxChunk];
float g_static_err[kStaticMaxChunk];
char g_static_seen[kStaticOrderInts];

// Device address of `scratch` on device `dev`, which must be current; resolved
// by hipGetSymbolAddress on the first request per device.
hipError_t static_scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_static_ptr_mu);
  if (dev < 0 || dev >= kStaticMaxDevices) return hipErrorInvalidDevice;
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return hipSuccess;
}

// Byte offsets of the buffers of one context inside the static scratch.
struct StaticLayout {
  size_t cases, order, flags, err, iter, X, q, dO, nP, V, maxv, maxw, errp, ccp, covm, gramp, vmix, eig, total;
  int chunk;  // iterations per staged chunk
};

StaticLayout static_layout(const ptycho_ctx* c, int n_iter) {
  const ptycho_params& p = c->prm;
  const size_t nn = (size_t)p.n * p.n, B = p.batch, K = p.n_modes;
  const int nobjt = n_obj_tiles(c->dp);
  const int nbt = std::max(max_err_slots(p.n), p.dft_bf16 ? dft_err_slots(p.n) : 0);
  StaticLayout L{};
  L.chunk = (int)std::min<size_t>({(size_t)std::max(n_iter, 1), (size_t)kStaticMaxChunk,
                                   kStaticOrderInts / (size_t)std::max(p.n_pos, 1)});
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  L.cases = take(sizeof(CaseDesc));
  L.order = take(sizeof(int32_t) * (size_t)L.chunk * p.n_pos);
  L.flags = take(sizeof(int) * (size_t)L.chunk);
  L.err = take(sizeof(float) * (size_t)L.chunk);
  L.iter = take(sizeof(int));
  L.X = take(sizeof(float2) * B * K * nn);
  L.q = take(sizeof(float) * B * nn);
  L.dO = take(sizeof(float2) * B * nn);
  L.nP = take(sizeof(float2) * K * nn);
  L.V = take(sizeof(float) * nn);
  L.maxv = take(sizeof(float) * (size_t)n_probe_blocks(p.n));
  L.maxw = take(sizeof(float) * (size_t)nobjt);
  L.errp = take(sizeof(double) * (size_t)p.n_pos * nbt);
  L.ccp = take(sizeof(double2) * (size_t)nobjt);
  L.covm = take(sizeof(unsigned) * (size_t)nobjt * kObjTile);
  L.gramp = take(sizeof(double2) * (K * (K + 1) / 2) * kGramBlocks);
  L.vmix = take(sizeof(float2) * K * K);
  L.eig = take(sizeof(double) * K);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

void ptycho_default_params(ptycho_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n = 64;
  p->n_modes = 1;
  p->geometry = PTYCHO_FAR_FIELD;
  p->engine = PTYCHO_ENGINE_EPIE;
  p->dm_reg = 1e-3f;
  p->lsq_damping = 0.1f;
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
  if (hipError_t e = init_kernel_attributes(); e != hipSuccess) {
    c->err = std::string("kernel attributes: ") + hipGetErrorString(e);
    return bail(PTYCHO_E_HIP);
  }
  {
    // resolve the static scratch of ptycho_iterate_static for this device now, with
    // the device current; a failure is reported by that entry point, which retries
    void* unused = nullptr;
    (void)static_scratch_ptr(c->device, &unused);
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
  dp.lsq_damping = p.lsq_damping;
  gaussian_taps(p.sigma1, dp.ks_half, dp.gx);
  gaussian_taps(p.sigma2, dp.ks_half, dp.gy);

  const int B = p.batch;
  DevBufs& d = c->db;
  float2 *obj, *probe, *tw, *hn, *X, *dO, *nP, *vmix;
  float *pw, *amp, *q, *V, *maxv, *maxw;
  int2* pos;
  double *errp, *eig;
  double2 *ccp, *gramp;
  unsigned* covm;
  const int nobjt = n_obj_tiles(dp);
  const int nbt = std::max(max_err_slots(n), p.dft_bf16 ? dft_err_slots(n) : 0);
  ptycho_status st = PTYCHO_OK;
  if ((st = dev_alloc(c, &obj, (size_t)p.obj_h * p.obj_w)) || (st = dev_alloc(c, &probe, K * nn)) ||
      (st = dev_alloc(c, &pw, 2 * nn)) || (st = dev_alloc(c, &amp, (size_t)p.n_pos * nn)) ||
      (st = dev_alloc(c, &pos, (size_t)p.n_pos)) || (st = dev_alloc(c, &tw, (size_t)n)) ||
      (st = dev_alloc(c, &hn, (size_t)n)) || (st = dev_alloc(c, &X, (size_t)B * K * nn)) ||
      (st = dev_alloc(c, &q, (size_t)B * nn)) || (st = dev_alloc(c, &dO, (size_t)B * nn)) ||
      (st = dev_alloc(c, &nP, K * nn)) || (st = dev_alloc(c, &V, nn)) ||
      (st = dev_alloc(c, &maxv, (size_t)n_probe_blocks(n))) || (st = dev_alloc(c, &maxw, (size_t)nobjt)) ||
      (st = dev_alloc(c, &errp, (size_t)p.n_pos * nbt)) || (st = dev_alloc(c, &ccp, (size_t)nobjt)) ||
      (st = dev_alloc(c, &covm, (size_t)nobjt * kObjTile)) ||
      (st = dev_alloc(c, &gramp, (size_t)(K * (K + 1) / 2) * kGramBlocks)) ||
      (st = dev_alloc(c, &vmix, (size_t)K * K)) || (st = dev_alloc(c, &eig, (size_t)K)) ||
      (st = dev_alloc(c, &c->d_iter, 1)) || (st = dev_alloc(c, &c->d_case, 1)) ||
      (st = dev_alloc(c, &c->d_case_dbg, 1)) || (st = dev_alloc(c, &c->d_dbg_order, (size_t)B)) ||
      (st = dev_alloc(c, &c->d_dbg_flags, 1)) || (st = dev_alloc(c, &c->d_dbg_iter, 1)) ||
      (st = dev_alloc(c, &c->d_dbg_err, 1)))
    return bail(st);
  if (hipHostMalloc((void**)&c->h_case, sizeof(CaseDesc), hipHostMallocDefault) != hipSuccess) {
    c->h_case = nullptr;
    c->err = "pinned host allocation failed";
    return bail(PTYCHO_E_OOM);
  }
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
  d.cov_mask = covm;
  d.gram_part = gramp;
  d.vmix = vmix;
  d.eig = eig;

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
  std::vector<uint16_t> planes;
  if (p.dft_bf16) {
    planes = dft_planes(n);
    uint16_t* dpl = nullptr;
    if ((st = dev_alloc(c, &dpl, planes.size())) != PTYCHO_OK) return bail(st);
    c->d_planes = dpl;
    INIT_TRY(hipMemcpyAsync(dpl, planes.data(), planes.size() * sizeof(uint16_t), hipMemcpyHostToDevice, s));
  }
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
  INIT_TRY(launch_pw(dp, d, 0, s));
  if (p.engine == PTYCHO_ENGINE_DM) {
    // pc-DM: exit-wave state, probe partial sums, and per object tile the ascending
    // list of positions whose boxes intersect it
    dp.dm_reg = p.dm_reg;
    dp.dm_seg_len = kDmSegLen;
    const int segs = dm_segments(p.n_pos, kDmSegLen);
    const int tiles_x = (p.obj_w + kObjTile - 1) / kObjTile;
    std::vector<int> off((size_t)nobjt + 1, 0);
    auto for_tiles = [&](int i, auto&& fn) {
      const int r = hpos[2 * i], cc = hpos[2 * i + 1];
      for (int ty = r / kObjTile; ty <= (r + n - 1) / kObjTile; ++ty)
        for (int tx = cc / kObjTile; tx <= (cc + n - 1) / kObjTile; ++tx) fn(ty * tiles_x + tx);
    };
    for (int i = 0; i < p.n_pos; ++i) for_tiles(i, [&](int t) { ++off[(size_t)t + 1]; });
    for (int t = 0; t < nobjt; ++t) off[(size_t)t + 1] += off[t];
    std::vector<int> lst(std::max(off[nobjt], 1)), cur(off.begin(), off.end() - 1);
    for (int i = 0; i < p.n_pos; ++i) for_tiles(i, [&](int t) { lst[cur[t]++] = i; });
    int *d_off = nullptr, *d_lst = nullptr;
    float2 *psi = nullptr, *npp = nullptr;
    float* vpp = nullptr;
    if ((st = dev_alloc(c, &d_off, off.size())) || (st = dev_alloc(c, &d_lst, lst.size())) ||
        (st = dev_alloc(c, &psi, (size_t)p.n_pos * K * nn)) || (st = dev_alloc(c, &npp, (size_t)segs * K * nn)) ||
        (st = dev_alloc(c, &vpp, (size_t)segs * nn)))
      return bail(st);
    INIT_TRY(hipMemcpyAsync(d_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync(d_lst, lst.data(), lst.size() * sizeof(int), hipMemcpyHostToDevice, s));
    d.cov_off = d_off;
    d.cov_pos = d_lst;
    d.psi = psi;
    d.np_part = npp;
    d.v_part = vpp;
    INIT_TRY(launch_dm_init_psi(dp, d, s));
  }
  if (p.engine == PTYCHO_ENGINE_LSQML) {
    // pc-LSQML: directions, step partial sums and the steps
    float2 *ldo = nullptr, *ldp = nullptr, *lpdp = nullptr;
    float *ldp2 = nullptr, *lab = nullptr, *lst = nullptr;
    double* lpart = nullptr;
    if ((st = dev_alloc(c, &ldo, (size_t)p.obj_h * p.obj_w)) || (st = dev_alloc(c, &ldp, K * nn)) ||
        (st = dev_alloc(c, &lpdp, nn)) || (st = dev_alloc(c, &ldp2, nn)) ||
        (st = dev_alloc(c, &lpart, (size_t)B * lsq_chunks(n) * kLsqTerms)) || (st = dev_alloc(c, &lab, 2)) ||
        (st = dev_alloc(c, &lst, (size_t)2 * B)))
      return bail(st);
    INIT_TRY(hipMemsetAsync(ldo, 0, (size_t)p.obj_h * p.obj_w * sizeof(float2), s));
    INIT_TRY(hipMemsetAsync(lab, 0, 2 * sizeof(float), s));
    INIT_TRY(hipMemsetAsync(lst, 0, (size_t)2 * B * sizeof(float), s));
    d.lsq_do = ldo;
    d.lsq_dp = ldp;
    d.lsq_pdp = lpdp;
    d.lsq_dp2 = ldp2;
    d.lsq_part = lpart;
    d.lsq_ab = lab;
    d.lsq_steps = lst;
  }
  std::vector<int> hb((size_t)p.n_pos * gx);
  std::vector<double> hs((size_t)p.n_pos * gx);
  INIT_TRY(hipMemcpyAsync(hb.data(), d_bad, hb.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  INIT_TRY(hipMemcpyAsync(hs.data(), d_sum, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  INIT_TRY(hipStreamSynchronize(s));
  if (mem_kind == PTYCHO_MEM_HOST) drop_alloc(c->allocs, raw);
  drop_alloc(c->allocs, d_bad);
  drop_alloc(c->allocs, d_sum);
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
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(std::make_tuple(n, K, B, (int)p.geometry));
    if (it != g_tune.end() && col_variant_valid(n, it->second)) c->col_variant = it->second;
    c->seq = seq_eligible(p);
  }
  *out = c;
  return PTYCHO_OK;
}

// FLAG_PW_ODD for an iteration whose first batch reads probe-power copy `par`;
// advances `par` past the iteration (every batch with probe update flips it).
int with_pw_parity(int flags, int& par, int n_batches) {
  if (par) flags |= FLAG_PW_ODD;
  if (flags & FLAG_PROBE) par ^= n_batches & 1;
  return flags;
}

// Orders and flags of iterations first_it+1 .. first_it+n_iter (1-based, from the
// context's counter c->t) into host arrays h_order [n_iter][n_pos] and h_flags
// [n_iter]; `order` (may be NULL) holds the caller's rows for these iterations.
// `par` enters as the probe-power copy of the first iteration and leaves as the
// copy after the last.  `seen` is n_pos bytes of scratch for the permutation check.
static ptycho_status fill_schedule(ptycho_ctx* c, int32_t first_it, int32_t n_iter, const int32_t* order,
                                   int32_t* h_order, int* h_flags, int& par, char* seen) {
  const int np = c->prm.n_pos;
  const int nb = n_batches_of(c->prm);
  for (int it = 0; it < n_iter; ++it) {
    int32_t* row = h_order + (size_t)it * np;
    const int t = c->t + first_it + 1 + it;
    if (order) {
      std::memcpy(row, order + (size_t)it * np, np * sizeof(int32_t));
      std::memset(seen, 0, np);
      for (int i = 0; i < np; ++i) {
        if (row[i] < 0 || row[i] >= np || seen[row[i]])
          return fail(c, PTYCHO_E_INVALID,
                      "order row " + std::to_string(first_it + it) + " is not a permutation of 0..n_pos-1");
        seen[row[i]] = 1;
      }
    } else {
      splitmix_perm(c->prm.seed, t, np, row);
    }
    // pc-DM keeps the probe-power map in copy 0 and does not orthogonalise the modes
    h_flags[it] = c->prm.engine == PTYCHO_ENGINE_DM ? (case_flags(c->prm, t) & ~FLAG_ORTHO)
                                                    : with_pw_parity(case_flags(c->prm, t), par, nb);
  }
  return PTYCHO_OK;
}

// Fill the schedule of n_iter iterations of context c into its call buffers.
static ptycho_status stage_call(ptycho_ctx* c, int32_t n_iter, const int32_t* order) {
  const int np = c->prm.n_pos;
  if (!grow_call(c, c->allocs, c->call, (size_t)n_iter * np, (size_t)n_iter))
    return fail(c, PTYCHO_E_OOM, "schedule buffer allocation failed");
  std::vector<char> seen(np);
  int par = c->pw_par;
  ptycho_status st = fill_schedule(c, 0, n_iter, order, c->call.h_order, c->call.h_flags, par, seen.data());
  if (st != PTYCHO_OK) return st;
  c->pw_par_next = par;
  return PTYCHO_OK;
}

ptycho_status ptycho_iterate(ptycho_ctx* c, int32_t n_iter, const int32_t* order, float* err_out) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (c->failed) return fail(c, PTYCHO_E_STATE, "context failed earlier: " + c->err);
  if (n_iter < 0) return fail(c, PTYCHO_E_INVALID, "n_iter must be >= 0");
  if (n_iter == 0) return PTYCHO_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // the pinned staging buffers may still be in use
  ptycho_status st = stage_call(c, n_iter, order);
  if (st != PTYCHO_OK) return st;
  const int np = c->prm.n_pos;
  fill_case(c, *c->h_case, c->call.d_order, c->call.d_flags, c->call.d_err);
  hipStream_t s = c->stream;
  HIP_TRY(c, hipMemcpyAsync(c->call.d_order, c->call.h_order, (size_t)n_iter * np * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->call.d_flags, c->call.h_flags, n_iter * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->d_case, c->h_case, sizeof(CaseDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(c, launch_iter_set(c->d_iter, 0, s));
  const bool timed = c->tm.mask != 0;
  if (c->use_graph && !timed) {
    if ((st = build_graph(c)) != PTYCHO_OK) return st;
    HIP_TRY(c, hipEventRecord(c->ev_in, s));
    HIP_TRY(c, hipStreamWaitEvent(c->gstream, c->ev_in, 0));
    for (int it = 0; it < n_iter; ++it) HIP_TRY(c, hipGraphLaunch(c->gexec, c->gstream));
    HIP_TRY(c, hipEventRecord(c->ev_out, c->gstream));
    HIP_TRY(c, hipStreamWaitEvent(s, c->ev_out, 0));
  } else {
    for (int it = 0; it < n_iter; ++it) {
      std::string e = enqueue_iteration(c, s, timed);
      if (!e.empty()) return fail(c, PTYCHO_E_HIP, e);
    }
  }
  HIP_TRY(c, hipMemcpyAsync(c->call.h_err, c->call.d_err, n_iter * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (c->tm.used) harvest_timing(c);
  c->t += n_iter;
  c->pw_par = c->pw_par_next;
  if (err_out) std::memcpy(err_out, c->call.h_err, n_iter * sizeof(float));
  for (int i = 0; i < n_iter; ++i)
    if (!std::isfinite(c->call.h_err[i])) {
      c->failed = true;
      return fail(c, PTYCHO_E_NUMERIC,
                  "non-finite data error at iteration " + std::to_string(c->t - n_iter + 1 + i));
    }
  return PTYCHO_OK;
}

ptycho_status ptycho_iterate_static(ptycho_ctx* c, int32_t n_iter, const int32_t* order, float* err_out) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (c->prm.engine != PTYCHO_ENGINE_EPIE) return fail(c, PTYCHO_E_STATE, "ptycho_iterate_static runs the ePIE engine");
  if (c->failed) return fail(c, PTYCHO_E_STATE, "context failed earlier: " + c->err);
  if (n_iter < 0) return fail(c, PTYCHO_E_INVALID, "n_iter must be >= 0");
  if (n_iter == 0) return PTYCHO_OK;
  const int np = c->prm.n_pos;
  if ((size_t)np > kStaticOrderInts)
    return fail(c, PTYCHO_E_SHAPE, "ptycho_iterate_static takes at most " + std::to_string(kStaticOrderInts) +
                                       " positions; use ptycho_iterate");
  const StaticLayout L = static_layout(c, n_iter);
  if (L.total > kStaticScratchBytes)
    return fail(c, PTYCHO_E_SHAPE, "this reconstruction needs " + std::to_string(L.total) +
                                       " bytes of scratch; ptycho_iterate_static holds at most " +
                                       std::to_string(kStaticScratchBytes) + " (use ptycho_iterate)");
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev != c->device) return fail(c, PTYCHO_E_STATE, "the current device is not the context's device");
  void* base = nullptr;
  {
    const hipError_t e = static_scratch_ptr(dev, &base);
    if (e != hipSuccess)
      return fail(c, PTYCHO_E_HIP, std::string("resolving the static scratch: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_static_mu);
  // every order row is checked before anything runs
  if (order) {
    for (int it = 0; it < n_iter; ++it) {
      const int32_t* row = order + (size_t)it * np;
      std::memset(g_static_seen, 0, np);
      for (int i = 0; i < np; ++i) {
        if (row[i] < 0 || row[i] >= np || g_static_seen[row[i]])
          return fail(c, PTYCHO_E_INVALID, "order row " + std::to_string(it) + " is not a permutation of 0..n_pos-1");
        g_static_seen[row[i]] = 1;
      }
    }
  }
  char* b = static_cast<char*>(base);
  hipStream_t s = c->stream;
  // the array keeps the previous call's contents: the data-error partials start at zero
  {
    const size_t words = (sizeof(double) * (size_t)np * std::max(max_err_slots(c->prm.n),
                                                                 c->prm.dft_bf16 ? dft_err_slots(c->prm.n) : 0)) / 8;
    const int blocks = (int)std::min<size_t>((words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_static_zero, dim3(std::max(blocks, 1)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(b + L.errp), words);
    HIP_TRY(c, hipGetLastError());
  }
  CaseDesc cd;
  for (int done = 0; done < n_iter; done += L.chunk) {
    const int m = std::min(L.chunk, n_iter - done);
    int par = c->pw_par;
    ptycho_status st = fill_schedule(c, 0, m, order ? order + (size_t)done * np : nullptr, g_static_order,
                                     g_static_flags, par, g_static_seen);
    if (st != PTYCHO_OK) return st;
    fill_case(c, cd, reinterpret_cast<int*>(b + L.order), reinterpret_cast<int*>(b + L.flags),
              reinterpret_cast<float*>(b + L.err));
    cd.d.X = reinterpret_cast<float2*>(b + L.X);
    cd.d.q = reinterpret_cast<float*>(b + L.q);
    cd.d.dO = reinterpret_cast<float2*>(b + L.dO);
    cd.d.nP = reinterpret_cast<float2*>(b + L.nP);
    cd.d.V = reinterpret_cast<float*>(b + L.V);
    cd.d.maxv_part = reinterpret_cast<float*>(b + L.maxv);
    cd.d.maxw_part = reinterpret_cast<float*>(b + L.maxw);
    cd.d.err_part = reinterpret_cast<double*>(b + L.errp);
    cd.d.cc_part = reinterpret_cast<double2*>(b + L.ccp);
    cd.d.cov_mask = reinterpret_cast<unsigned*>(b + L.covm);
    cd.d.gram_part = reinterpret_cast<double2*>(b + L.gramp);
    cd.d.vmix = reinterpret_cast<float2*>(b + L.vmix);
    cd.d.eig = reinterpret_cast<double*>(b + L.eig);
    HIP_TRY(c, hipMemcpyAsync(b + L.cases, &cd, sizeof(CaseDesc), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(b + L.order, g_static_order, (size_t)m * np * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(b + L.flags, g_static_flags, (size_t)m * sizeof(int), hipMemcpyHostToDevice, s));
    int* d_it = reinterpret_cast<int*>(b + L.iter);
    HIP_TRY(c, launch_iter_set(d_it, 0, s));
    for (int it = 0; it < m; ++it) {
      std::string e = enqueue_iteration_on(c, reinterpret_cast<const CaseDesc*>(b + L.cases),
                                           reinterpret_cast<float2*>(b + L.X), d_it, s, false);
      if (!e.empty()) return fail(c, PTYCHO_E_HIP, e);
    }
    HIP_TRY(c, hipMemcpyAsync(g_static_err, b + L.err, (size_t)m * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->t += m;
    c->pw_par = par;
    if (err_out) std::memcpy(err_out + done, g_static_err, (size_t)m * sizeof(float));
    for (int i = 0; i < m; ++i)
      if (!std::isfinite(g_static_err[i])) {
        c->failed = true;
        return fail(c, PTYCHO_E_NUMERIC, "non-finite data error at iteration " + std::to_string(c->t - m + 1 + i));
      }
  }
  return PTYCHO_OK;
}

int32_t ptycho_variant_count(void) { return kColVariants + 1; }

ptycho_status ptycho_set_variant(ptycho_ctx* c, int32_t variant) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (variant == kSeqVariant) {
    if (!seq_eligible(c->prm))
      return fail(c, PTYCHO_E_INVALID, "the sequential kernel runs batch 1 on far-field frames of side 16, 32, 48 or 64");
    if (!c->seq) drop_graph(c);
    c->seq = true;
    return PTYCHO_OK;
  }
  if (c->seq) drop_graph(c);
  c->seq = false;
  if (!col_variant_valid(c->prm.n, variant))
    return fail(c, PTYCHO_E_INVALID, "launch variant " + std::to_string(variant) + " does not exist for n = " +
                                         std::to_string(c->prm.n));
  if (variant != c->col_variant) drop_graph(c);
  c->col_variant = variant;
  return PTYCHO_OK;
}

ptycho_status ptycho_set_graph(ptycho_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  c->use_graph = enable != 0;
  if (!c->use_graph) drop_graph(c);
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
    HIP_TRY(c, launch_pw(c->dp, c->db, c->pw_par, c->stream));
  }
  if (object)
    HIP_TRY(c, hipMemcpyAsync(c->db.obj, object, (size_t)c->prm.obj_h * c->prm.obj_w * sizeof(float2),
                              kind_in(mem_kind), c->stream));
  if (c->prm.engine == PTYCHO_ENGINE_DM && (object || probe)) HIP_TRY(c, launch_dm_init_psi(c->dp, c->db, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->t = iter;
  c->failed = false;
  return PTYCHO_OK;
}

ptycho_status ptycho_get_exit_waves(ptycho_ctx* c, float* out, int32_t mem_kind) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (c->prm.engine != PTYCHO_ENGINE_DM) return fail(c, PTYCHO_E_STATE, "exit waves are state of the pc-DM engine only");
  if (!out) return fail(c, PTYCHO_E_INVALID, "out is NULL");
  const size_t count = (size_t)c->prm.n_pos * c->prm.n_modes * c->prm.n * c->prm.n;
  HIP_TRY(c, hipMemcpyAsync(out, c->db.psi, count * sizeof(float2), kind_out(mem_kind), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PTYCHO_OK;
}

ptycho_status ptycho_get_lsq_steps(ptycho_ctx* c, float* steps, float* mean) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (c->prm.engine != PTYCHO_ENGINE_LSQML)
    return fail(c, PTYCHO_E_STATE, "step lengths are state of the pc-LSQML engine only");
  if (steps)
    HIP_TRY(c, hipMemcpyAsync(steps, c->db.lsq_steps, (size_t)2 * c->prm.batch * sizeof(float),
                              hipMemcpyDeviceToHost, c->stream));
  if (mean) HIP_TRY(c, hipMemcpyAsync(mean, c->db.lsq_ab, 2 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PTYCHO_OK;
}

ptycho_status ptycho_set_exit_waves(ptycho_ctx* c, const float* in, int32_t mem_kind) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (c->prm.engine != PTYCHO_ENGINE_DM) return fail(c, PTYCHO_E_STATE, "exit waves are state of the pc-DM engine only");
  if (!in) return fail(c, PTYCHO_E_INVALID, "in is NULL");
  const size_t count = (size_t)c->prm.n_pos * c->prm.n_modes * c->prm.n * c->prm.n;
  std::vector<float> h;
  ptycho_status st = fetch_host(c, in, 2 * count, mem_kind, h);
  if (st != PTYCHO_OK) return st;
  for (float x : h)
    if (!std::isfinite(x)) return fail(c, PTYCHO_E_INVALID, "exit waves contain a non-finite value");
  HIP_TRY(c, hipMemcpyAsync(c->db.psi, h.data(), count * sizeof(float2), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PTYCHO_OK;
}

int32_t ptycho_iteration(const ptycho_ctx* c) { return c ? c->t : -1; }

ptycho_status ptycho_debug_step(ptycho_ctx* c, const int32_t* idx, int32_t B, int32_t t, float* psi,
                                float* psi_new, float* factor, float* n_obj, float* w_obj, float* n_probe,
                                float* v_probe, int32_t mem_kind) {
  if (!c || !idx) return fail(c, PTYCHO_E_INVALID, "NULL argument");
  if (c->prm.engine != PTYCHO_ENGINE_EPIE) return fail(c, PTYCHO_E_STATE, "debug_step captures a batch of the ePIE engine");
  if (c->failed) return fail(c, PTYCHO_E_STATE, "context failed earlier: " + c->err);
  if (B < 1 || B > c->prm.batch) return fail(c, PTYCHO_E_INVALID, "B must be in [1, batch]");
  if (t < 1) return fail(c, PTYCHO_E_INVALID, "t must be >= 1");
  if ((n_obj == nullptr) != (w_obj == nullptr)) return fail(c, PTYCHO_E_INVALID, "n_obj and w_obj go together");
  for (int i = 0; i < B; ++i)
    if (idx[i] < 0 || idx[i] >= c->prm.n_pos) return fail(c, PTYCHO_E_INVALID, "index out of range");
  hipStream_t s = c->stream;
  HIP_TRY(c, hipStreamSynchronize(s));
  const int n = c->prm.n, K = c->prm.n_modes;
  const size_t nn = (size_t)n * n, no = (size_t)c->prm.obj_h * c->prm.obj_w;
  std::vector<void*> tmp;
  auto alloc_tmp = [&](size_t bytes, void** p) -> bool {
    if (hipMalloc(p, bytes) != hipSuccess) return false;
    tmp.push_back(*p);
    return true;
  };
  auto cleanup = [&]() {
    for (void* p : tmp) (void)hipFree(p);
  };
  float2 *d_psi = nullptr, *d_psin = nullptr, *d_nobj = nullptr;
  float *d_wobj = nullptr, *d_fac = nullptr;
  bool ok = true;
  if (psi) ok = ok && alloc_tmp((size_t)B * K * nn * sizeof(float2), (void**)&d_psi);
  if (psi_new) ok = ok && alloc_tmp((size_t)B * K * nn * sizeof(float2), (void**)&d_psin);
  if (n_obj) ok = ok && alloc_tmp(no * sizeof(float2), (void**)&d_nobj) && alloc_tmp(no * sizeof(float), (void**)&d_wobj);
  if (factor) ok = ok && alloc_tmp((size_t)B * nn * sizeof(float), (void**)&d_fac);
  if (!ok) {
    cleanup();
    return fail(c, PTYCHO_E_OOM, "debug staging allocation failed");
  }
  // schedule of the one batch: order = idx, flags of iteration t
  std::vector<int> hidx(idx, idx + B);
  int pw_par = c->pw_par;
  const int flags = with_pw_parity(case_flags(c->prm, t) & ~FLAG_ORTHO, pw_par, 1);
  CaseDesc cd;
  fill_case(c, cd, c->d_dbg_order, c->d_dbg_flags, c->d_dbg_err);
  cd.dbg = DebugPtrs{d_psin, d_nobj, d_wobj, d_fac};
  cd.n_pos = B;
  cd.batch = B;
  cd.n_batches = 1;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chk(hipMemcpyAsync(c->d_dbg_order, hidx.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(c->d_dbg_flags, &flags, sizeof(int), hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(c->d_case_dbg, &cd, sizeof(CaseDesc), hipMemcpyHostToDevice, s));
  chk(launch_iter_set(c->d_dbg_iter, 0, s));
  if (d_nobj) {
    chk(hipMemsetAsync(d_nobj, 0, no * sizeof(float2), s));
    chk(hipMemsetAsync(d_wobj, 0, no * sizeof(float), s));
  }
  if (n_probe) chk(hipMemsetAsync(c->db.nP, 0, K * nn * sizeof(float2), s));
  if (v_probe) chk(hipMemsetAsync(c->db.V, 0, nn * sizeof(float), s));
  if (d_psi) chk(launch_exit_waves(c->dp, c->db, c->d_dbg_order, B, d_psi, s));
  std::string le;
  if (e == hipSuccess)
    le = launch_one(c->tm.mask ? c : nullptr, c, c->d_case_dbg, c->db.X, single_shape(c, B), 0, B, c->d_dbg_iter, s);
  auto copy = [&](float* dst, const void* src, size_t bytes) {
    if (dst) chk(hipMemcpyAsync(dst, src, bytes, kind_out(mem_kind), s));
  };
  if (e == hipSuccess && le.empty()) {
    copy(psi, d_psi, (size_t)B * K * nn * sizeof(float2));
    copy(psi_new, d_psin, (size_t)B * K * nn * sizeof(float2));
    copy(factor, d_fac, (size_t)B * nn * sizeof(float));
    copy(n_obj, d_nobj, no * sizeof(float2));
    copy(w_obj, d_wobj, no * sizeof(float));
    copy(n_probe, c->db.nP, K * nn * sizeof(float2));
    copy(v_probe, c->db.V, nn * sizeof(float));
  }
  hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  if (c->tm.used) harvest_timing(c);
  cleanup();
  if (!le.empty()) return fail(c, PTYCHO_E_HIP, le);
  if (e != hipSuccess) return fail(c, PTYCHO_E_HIP, std::string("debug step: ") + hipGetErrorString(e));
  c->pw_par = pw_par;
  return PTYCHO_OK;
}

ptycho_status ptycho_autotune(ptycho_ctx* c, int32_t trials, int32_t force, int32_t* chosen) {
  if (!c) return fail(nullptr, PTYCHO_E_INVALID, "ctx is NULL");
  if (c->prm.engine != PTYCHO_ENGINE_EPIE) return fail(c, PTYCHO_E_STATE, "the autotuner times the ePIE batch passes");
  if (c->seq) {  // one launch per iteration: nothing to tune
    if (chosen) *chosen = kSeqVariant;
    return PTYCHO_OK;
  }
  if (c->failed) return fail(c, PTYCHO_E_STATE, "context failed earlier: " + c->err);
  if (trials < 1) trials = 1;
  const int n = c->prm.n;
  if (c->prm.dft_bf16) {  // the column passes are not used by this path
    if (chosen) *chosen = c->col_variant;
    return PTYCHO_OK;
  }
  const auto key = std::make_tuple(n, c->prm.n_modes, c->prm.batch, (int)c->prm.geometry);
  if (!force) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end() && col_variant_valid(n, it->second)) {
      if (c->col_variant != it->second) drop_graph(c);
      c->col_variant = it->second;
      if (chosen) *chosen = c->col_variant;
      return PTYCHO_OK;
    }
  }
  hipStream_t s = c->stream;
  HIP_TRY(c, hipStreamSynchronize(s));
  // back up the state the timing runs modify
  const size_t no = (size_t)c->prm.obj_h * c->prm.obj_w, npr = (size_t)c->prm.n_modes * n * n;
  float2 *bo = nullptr, *bp = nullptr;
  if (hipMalloc((void**)&bo, no * sizeof(float2)) != hipSuccess) return fail(c, PTYCHO_E_OOM, "autotune backup");
  if (hipMalloc((void**)&bp, npr * sizeof(float2)) != hipSuccess) {
    (void)hipFree(bo);
    return fail(c, PTYCHO_E_OOM, "autotune backup");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  std::string err;
  int best = c->col_variant;
  float best_ms = 1e30f;
  hipError_t he = hipMemcpyAsync(bo, c->db.obj, no * sizeof(float2), hipMemcpyDeviceToDevice, s);
  if (he == hipSuccess) he = hipMemcpyAsync(bp, c->db.probe, npr * sizeof(float2), hipMemcpyDeviceToDevice, s);
  const int saved_variant = c->col_variant;
  ptycho_status st = (he == hipSuccess) ? stage_call(c, 1, nullptr) : PTYCHO_E_HIP;
  if (st == PTYCHO_OK) {
    int par = c->pw_par;  // every trial runs the first batch from the same state
    c->call.h_flags[0] = with_pw_parity(FLAG_PROBE | FLAG_CC, par, n_batches_of(c->prm));
    for (int v = 0; v < kColVariants && err.empty(); ++v) {
      if (!col_variant_valid(n, v)) continue;
      c->col_variant = v;
      fill_case(c, *c->h_case, c->call.d_order, c->call.d_flags, c->call.d_err);
      he = hipMemcpyAsync(c->call.d_order, c->call.h_order, c->prm.n_pos * sizeof(int), hipMemcpyHostToDevice, s);
      if (he == hipSuccess) he = hipMemcpyAsync(c->call.d_flags, c->call.h_flags, sizeof(int), hipMemcpyHostToDevice, s);
      if (he == hipSuccess) he = hipMemcpyAsync(c->d_case, c->h_case, sizeof(CaseDesc), hipMemcpyHostToDevice, s);
      if (he == hipSuccess) he = launch_iter_set(c->d_iter, 0, s);
      if (he != hipSuccess) {
        err = hipGetErrorString(he);
        break;
      }
      const TableShape sh = single_shape(c, c->prm.batch);
      err = launch_batch(nullptr, c->d_case, sh, 0, c->d_iter, s);  // warm-up
      if (!err.empty()) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < trials && err.empty(); ++r) err = launch_batch(nullptr, c->d_case, sh, 0, c->d_iter, s);
      (void)hipEventRecord(e1, s);
      (void)hipStreamSynchronize(s);
      float ms = 0.f;
      if (err.empty() && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
  }
  // restore the state
  (void)hipMemcpyAsync(c->db.obj, bo, no * sizeof(float2), hipMemcpyDeviceToDevice, s);
  (void)hipMemcpyAsync(c->db.probe, bp, npr * sizeof(float2), hipMemcpyDeviceToDevice, s);
  (void)launch_pw(c->dp, c->db, c->pw_par, s);
  hipError_t fin = hipStreamSynchronize(s);
  (void)hipFree(bo);
  (void)hipFree(bp);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PTYCHO_OK) {
    c->col_variant = saved_variant;
    return st;
  }
  if (!err.empty() || fin != hipSuccess) {
    c->col_variant = saved_variant;
    return fail(c, PTYCHO_E_HIP, "autotune: " + (err.empty() ? std::string(hipGetErrorString(fin)) : err));
  }
  if (best != saved_variant) drop_graph(c);
  c->col_variant = best;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_store_locked(key, best);
  }
  if (chosen) *chosen = best;
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
  (void)hipStreamSynchronize(c->stream);
  if (c->gstream) (void)hipStreamSynchronize(c->gstream);
  drop_graph(c);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  for (hipEvent_t e : c->tm.pool) (void)hipEventDestroy(e);
  for (void* p : c->allocs) (void)hipFree(p);
  free_call(c->call);
  if (c->h_case) (void)hipHostFree(c->h_case);
  delete c;
}

const char* ptycho_last_error(const ptycho_ctx* c) { return c ? c->err.c_str() : g_thread_error.c_str(); }

// ---------------------------------------------------------------------------
// Groups of independent reconstructions
// ---------------------------------------------------------------------------

ptycho_status ptycho_group_create(ptycho_ctx* const* ctxs, int32_t n, ptycho_group** out) {
  if (out) *out = nullptr;
  if (!out || !ctxs || n < 1) return gfail(nullptr, PTYCHO_E_INVALID, "need out and n >= 1 contexts");
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return gfail(nullptr, PTYCHO_E_INVALID, "NULL context in group");
    if (ctxs[i]->failed) return gfail(nullptr, PTYCHO_E_STATE, "a context in the group has failed");
    if (ctxs[i]->prm.dft_bf16) return gfail(nullptr, PTYCHO_E_INVALID, "groups run the FFT path only (dft_bf16 = 0)");
    if (ctxs[i]->prm.engine != PTYCHO_ENGINE_EPIE)
      return gfail(nullptr, PTYCHO_E_INVALID, "groups run the ePIE engine (one pc-DM context runs alone)");
    if (ctxs[i]->device != ctxs[0]->device || ctxs[i]->stream != ctxs[0]->stream)
      return gfail(nullptr, PTYCHO_E_INVALID, "group contexts must share one device and stream");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return gfail(nullptr, PTYCHO_E_INVALID, "a context appears twice in the group");
  }
  ptycho_group* g = new ptycho_group();
  g->ctx.assign(ctxs, ctxs + n);
  g->stream = ctxs[0]->stream;
  // one table per (frame size, geometry)
  std::map<std::tuple<int, int, int>, int> idx;
  for (int i = 0; i < n; ++i) {
    const ptycho_ctx* c = ctxs[i];
    const auto key = std::make_tuple(c->prm.n, (int)c->prm.geometry, c->seq ? 1 : 0);
    if (!idx.count(key)) {
      idx[key] = (int)g->tables.size();
      g->tables.emplace_back();
      g->tables.back().seq = c->seq;
      TableShape& sh = g->tables.back().shape;
      sh.n = c->prm.n;
      sh.near_field = c->prm.geometry == PTYCHO_NEAR_FIELD;
      sh.col_variant = c->col_variant;
    }
    ptycho_group::Table& tb = g->tables[idx[key]];
    tb.members.push_back(i);
    TableShape& sh = tb.shape;
    sh.n_cases = (int)tb.members.size();
    sh.max_batch = std::max(sh.max_batch, c->prm.batch);
    sh.x_pairs = sh.max_batch >= 2 && inv_rows_paired(sh.n);  // groups run the ePIE engine on the FFT path
    sh.max_tiles = std::max(sh.max_tiles, n_obj_tiles(c->dp));
    sh.max_k = std::max(sh.max_k, c->prm.n_modes);
    sh.max_side_jobs = std::max(sh.max_side_jobs, n_obj_tiles(c->dp) + n_probe_blocks(c->prm.n));
    sh.max_half = std::max(sh.max_half, c->dp.ks_half);
    tb.max_nb = std::max(tb.max_nb, n_batches_of(c->prm));
  }
  if (g->tables.size() > 1) {
    const size_t ns = std::min<size_t>(g->tables.size(), kGroupStreams);
    g->side.assign(ns, nullptr);
    g->side_done.assign(ns, nullptr);
    bool ok = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess;
    for (size_t i = 0; ok && i < ns; ++i)
      ok = hipStreamCreateWithFlags(&g->side[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&g->side_done[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      ptycho_group_destroy(g);
      return gfail(nullptr, PTYCHO_E_HIP, "group stream creation failed");
    }
  }
  for (auto& tb : g->tables) {
    void* p = nullptr;
    if (hipMalloc(&p, tb.members.size() * sizeof(CaseDesc)) != hipSuccess) {
      ptycho_group_destroy(g);
      return gfail(nullptr, PTYCHO_E_OOM, "group table allocation failed");
    }
    g->allocs.push_back(p);
    tb.d_cases = (CaseDesc*)p;
    if (hipHostMalloc((void**)&tb.h_cases, tb.members.size() * sizeof(CaseDesc), hipHostMallocDefault) != hipSuccess) {
      tb.h_cases = nullptr;
      ptycho_group_destroy(g);
      return gfail(nullptr, PTYCHO_E_OOM, "pinned host allocation failed");
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(int)) != hipSuccess) {
    ptycho_group_destroy(g);
    return gfail(nullptr, PTYCHO_E_OOM, "group counter allocation failed");
  }
  g->allocs.push_back(p);
  g->d_iter = (int*)p;
  *out = g;
  return PTYCHO_OK;
}

}  // extern "C"

namespace {

// One iteration of one table on stream s: the sequential kernel (one workgroup per
// case) or the batches in order, then the end-of-iteration work.
std::string enqueue_table_iteration(ptycho_group* g, ptycho_group::Table& tb, hipStream_t s) {
  if (tb.seq) {
    const hipError_t he = launch_seq_iter(tb.d_cases, tb.shape, g->d_iter, s);
    if (he != hipSuccess) return std::string("seq_iteration: ") + hipGetErrorString(he);
  } else {
    for (int beta = 0; beta < tb.max_nb; ++beta) {
      std::string e = launch_batch(nullptr, tb.d_cases, tb.shape, beta, g->d_iter, s);
      if (!e.empty()) return e;
    }
  }
  return launch_end(nullptr, tb.d_cases, tb.shape, g->d_iter, s);
}

// One iteration of every member: the tables (independent cases, each with its own
// buffers) on their side streams at once, joined before the iteration counter
// advances.  Each table's kernels run in the same order as alone, so results do not
// depend on the overlap.
std::string enqueue_group_iteration(ptycho_group* g, hipStream_t s) {
  const size_t ns = g->side.size();
  if (ns == 0) {
    std::string e = enqueue_table_iteration(g, g->tables[0], s);
    if (!e.empty()) return e;
  } else {
    hipError_t he = hipEventRecord(g->fork, s);
    for (size_t i = 0; he == hipSuccess && i < ns; ++i) he = hipStreamWaitEvent(g->side[i], g->fork, 0);
    if (he != hipSuccess) return std::string("group fork: ") + hipGetErrorString(he);
    for (size_t i = 0; i < g->tables.size(); ++i) {
      std::string e = enqueue_table_iteration(g, g->tables[i], g->side[i % ns]);
      if (!e.empty()) return e;
    }
    for (size_t i = 0; he == hipSuccess && i < ns; ++i) {
      he = hipEventRecord(g->side_done[i], g->side[i]);
      if (he == hipSuccess) he = hipStreamWaitEvent(s, g->side_done[i], 0);
    }
    if (he != hipSuccess) return std::string("group join: ") + hipGetErrorString(he);
  }
  const hipError_t he = launch_iter_advance(g->d_iter, s);
  return he == hipSuccess ? std::string() : std::string("iteration counter: ") + hipGetErrorString(he);
}

// The captured iteration reads its schedule (orders, flags, case tables) from
// device buffers that every call refills, so one capture serves all calls as
// long as those buffers stay where they are.
ptycho_status build_group_graph(ptycho_group* g) {
  if (g->gexec) return PTYCHO_OK;
  if (!g->gstream) HIP_GTRY(g, hipStreamCreateWithFlags(&g->gstream, hipStreamNonBlocking));
  if (!g->ev_in) HIP_GTRY(g, hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming));
  if (!g->ev_out) HIP_GTRY(g, hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming));
  HIP_GTRY(g, hipStreamBeginCapture(g->gstream, hipStreamCaptureModeThreadLocal));
  std::string e = enqueue_group_iteration(g, g->gstream);
  hipGraph_t graph = nullptr;
  hipError_t he = hipStreamEndCapture(g->gstream, &graph);
  if (!e.empty()) {
    if (graph) (void)hipGraphDestroy(graph);
    return gfail(g, PTYCHO_E_HIP, "capturing the group iteration: " + e);
  }
  if (he != hipSuccess) return gfail(g, PTYCHO_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
  he = hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (he != hipSuccess) {
    g->gexec = nullptr;
    return gfail(g, PTYCHO_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
  }
  return PTYCHO_OK;
}

void drop_group_graph(ptycho_group* g) {
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  g->gexec = nullptr;
}

}  // namespace

extern "C" {

ptycho_status ptycho_group_set_graph(ptycho_group* g, int32_t enable) {
  if (!g) return gfail(nullptr, PTYCHO_E_INVALID, "group is NULL");
  g->use_graph = enable != 0;
  if (!g->use_graph) drop_group_graph(g);
  return PTYCHO_OK;
}

ptycho_status ptycho_group_iterate(ptycho_group* g, int32_t n_iter, float* err_out) {
  if (!g) return gfail(nullptr, PTYCHO_E_INVALID, "group is NULL");
  if (n_iter < 0) return gfail(g, PTYCHO_E_INVALID, "n_iter must be >= 0");
  if (n_iter == 0) return PTYCHO_OK;
  const int nc = (int)g->ctx.size();
  for (ptycho_ctx* c : g->ctx)
    if (c->failed) return gfail(g, PTYCHO_E_STATE, "a context in the group has failed: " + c->err);
  hipStream_t s = g->stream;
  HIP_GTRY(g, hipStreamSynchronize(s));
  // schedules of every case, concatenated
  std::vector<size_t> off(nc + 1, 0);
  for (int i = 0; i < nc; ++i) off[i + 1] = off[i] + (size_t)n_iter * g->ctx[i]->prm.n_pos;
  if (!grow_call(g, g->allocs, g->call, off[nc], (size_t)n_iter * nc))
    return gfail(g, PTYCHO_E_OOM, "schedule buffer allocation failed");
  for (int i = 0; i < nc; ++i) {
    ptycho_ctx* c = g->ctx[i];
    const int np = c->prm.n_pos;
    for (int it = 0; it < n_iter; ++it) {
      splitmix_perm(c->prm.seed, c->t + 1 + it, np, g->call.h_order + off[i] + (size_t)it * np);
      g->call.h_flags[(size_t)i * n_iter + it] = case_flags(c->prm, c->t + 1 + it);
    }
    int par = c->pw_par;
    const int nb = n_batches_of(c->prm);
    for (int it = 0; it < n_iter; ++it) {
      int& f = g->call.h_flags[(size_t)i * n_iter + it];
      f = with_pw_parity(f, par, nb);
    }
    c->pw_par_next = par;
  }
  for (auto& tb : g->tables)
    for (size_t m = 0; m < tb.members.size(); ++m) {
      const int i = tb.members[m];
      fill_case(g->ctx[i], tb.h_cases[m], g->call.d_order + off[i], g->call.d_flags + (size_t)i * n_iter,
                g->call.d_err + (size_t)i * n_iter);
      tb.h_cases[m].n_err_part = g->ctx[i]->prm.n_pos * n_err_slots(tb.shape.n, tb.shape.col_variant, tb.shape.max_half);
    }
  HIP_GTRY(g, hipMemcpyAsync(g->call.d_order, g->call.h_order, off[nc] * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_GTRY(g, hipMemcpyAsync(g->call.d_flags, g->call.h_flags, (size_t)n_iter * nc * sizeof(int),
                             hipMemcpyHostToDevice, s));
  for (auto& tb : g->tables)
    HIP_GTRY(g, hipMemcpyAsync(tb.d_cases, tb.h_cases, tb.members.size() * sizeof(CaseDesc), hipMemcpyHostToDevice, s));
  HIP_GTRY(g, launch_iter_set(g->d_iter, 0, s));
  if (g->use_graph) {
    ptycho_status gs = build_group_graph(g);
    if (gs != PTYCHO_OK) return gs;
    HIP_GTRY(g, hipEventRecord(g->ev_in, s));
    HIP_GTRY(g, hipStreamWaitEvent(g->gstream, g->ev_in, 0));
    for (int it = 0; it < n_iter; ++it) HIP_GTRY(g, hipGraphLaunch(g->gexec, g->gstream));
    HIP_GTRY(g, hipEventRecord(g->ev_out, g->gstream));
    HIP_GTRY(g, hipStreamWaitEvent(s, g->ev_out, 0));
  } else {
    for (int it = 0; it < n_iter; ++it) {
      std::string e = enqueue_group_iteration(g, s);
      if (!e.empty()) return gfail(g, PTYCHO_E_HIP, e);
    }
  }
  HIP_GTRY(g, hipMemcpyAsync(g->call.h_err, g->call.d_err, (size_t)n_iter * nc * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_GTRY(g, hipStreamSynchronize(s));
  ptycho_status st = PTYCHO_OK;
  for (int i = 0; i < nc; ++i) {
    ptycho_ctx* c = g->ctx[i];
    c->t += n_iter;
    c->pw_par = c->pw_par_next;
    for (int it = 0; it < n_iter; ++it)
      if (!std::isfinite(g->call.h_err[(size_t)i * n_iter + it]) && !c->failed) {
        c->failed = true;
        c->err = "non-finite data error at iteration " + std::to_string(c->t - n_iter + 1 + it);
        st = gfail(g, PTYCHO_E_NUMERIC, "case " + std::to_string(i) + ": " + c->err);
      }
  }
  if (err_out) std::memcpy(err_out, g->call.h_err, (size_t)n_iter * nc * sizeof(float));
  return st;
}

void ptycho_group_destroy(ptycho_group* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  if (g->gstream) (void)hipStreamSynchronize(g->gstream);
  for (hipStream_t st : g->side)
    if (st) (void)hipStreamSynchronize(st);
  drop_group_graph(g);
  if (g->gstream) (void)hipStreamDestroy(g->gstream);
  for (hipStream_t st : g->side)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : g->side_done)
    if (ev) (void)hipEventDestroy(ev);
  if (g->fork) (void)hipEventDestroy(g->fork);
  if (g->ev_in) (void)hipEventDestroy(g->ev_in);
  if (g->ev_out) (void)hipEventDestroy(g->ev_out);
  for (auto& tb : g->tables)
    if (tb.h_cases) (void)hipHostFree(tb.h_cases);
  for (void* p : g->allocs) (void)hipFree(p);
  free_call(g->call);
  delete g;
}

ptycho_status ptycho_dft2_bf16(float* frames_inout, int32_t n, int32_t frames, int32_t inverse, void* hip_stream) {
  if (!frames_inout || frames < 0 || !dft_supported(n))
    return fail(nullptr, PTYCHO_E_INVALID, "need device frames and n in {64, 128, 192, 256}");
  if (frames == 0) return PTYCHO_OK;
  static std::mutex mu;
  static std::map<std::pair<int, int>, void*> cache;  // (device, n) -> planes; kept for the process
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, PTYCHO_E_HIP, "no HIP device");
  void* planes = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({dev, n});
    if (it == cache.end()) {
      std::vector<uint16_t> pl = dft_planes(n);
      if (hipMalloc(&planes, pl.size() * sizeof(uint16_t)) != hipSuccess)
        return fail(nullptr, PTYCHO_E_OOM, "DFT table allocation failed");
      if (hipMemcpy(planes, pl.data(), pl.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(planes);
        return fail(nullptr, PTYCHO_E_HIP, "DFT table upload failed");
      }
      cache[{dev, n}] = planes;
    } else {
      planes = it->second;
    }
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = launch_dft2(reinterpret_cast<float2*>(frames_inout), planes, n, frames, inverse != 0, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(nullptr, PTYCHO_E_HIP, std::string("dft2_bf16: ") + hipGetErrorString(e));
  return PTYCHO_OK;
}

// ---------------------------------------------------------------------------
// Numerical monochromatisation by CGLS (Sec. 4.2)
// ---------------------------------------------------------------------------

ptycho_status ptycho_mono_create(int32_t n, int32_t max_patterns, const float* scales, const float* weights,
                                 int32_t n_lambda, void* hip_stream, ptycho_mono** out) {
  if (out) *out = nullptr;
  if (!out || !scales || !weights) return fail(nullptr, PTYCHO_E_INVALID, "NULL argument");
  if (n < 2 || n > 4096 || (n & 1)) return fail(nullptr, PTYCHO_E_SHAPE, "n must be even and in [2, 4096]");
  if (max_patterns < 1 || max_patterns > 65535) return fail(nullptr, PTYCHO_E_SHAPE, "max_patterns must be in [1, 65535]");
  if (n_lambda < 1 || n_lambda > kMonoMaxLambda) return fail(nullptr, PTYCHO_E_INVALID, "n_lambda must be in [1, 16]");
  double wsum = 0.0;
  for (int j = 0; j < n_lambda; ++j) {
    if (!(std::isfinite(scales[j]) && scales[j] >= kMonoMinScale && scales[j] <= kMonoMaxScale))
      return fail(nullptr, PTYCHO_E_INVALID, "scales must be in [1/16, 16]");
    if (!(std::isfinite(weights[j]) && weights[j] >= 0.f)) return fail(nullptr, PTYCHO_E_INVALID, "weights must be >= 0");
    wsum += weights[j];
  }
  if (!(wsum > 0.0)) return fail(nullptr, PTYCHO_E_INVALID, "the weights must not all be zero");
  ptycho_mono* m = new ptycho_mono();
  m->n = n;
  m->max_pat = max_patterns;
  m->stream = (hipStream_t)hip_stream;
  m->w.spec.count = n_lambda;
  for (int j = 0; j < n_lambda; ++j) {
    m->w.spec.scale[j] = scales[j];
    m->w.spec.coef[j] = (float)(weights[j] / wsum * (double)scales[j] * (double)scales[j]);
  }
  const size_t nn = (size_t)n * n, tot = nn * max_patterns;
  const size_t blocks = (size_t)mono_part_count(n);
  auto alloc = [&](void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) return false;
    m->allocs.push_back(*p);
    return true;
  };
  if (!alloc((void**)&m->w.r, tot * 4) || !alloc((void**)&m->w.s, tot * 4) || !alloc((void**)&m->w.p, tot * 4) ||
      !alloc((void**)&m->w.q, tot * 4) || !alloc((void**)&m->w.part, blocks * max_patterns * 8) ||
      !alloc((void**)&m->w.part2, blocks * max_patterns * 8) || !alloc((void**)&m->w.gamma, max_patterns * 8) ||
      !alloc((void**)&m->w.coef, max_patterns * 8) || !alloc((void**)&m->d_in, tot * 4) ||
      !alloc((void**)&m->d_out, tot * 4)) {
    ptycho_mono_destroy(m);
    return fail(nullptr, PTYCHO_E_OOM, "device allocation failed");
  }
  MonoTables& tb = m->w.tab;
  tb.adj_stride = mono_adj_stride(m->w.spec);
  const size_t tn = (size_t)n_lambda * n;
  if (!alloc((void**)&tb.i0, tn * 4) || !alloc((void**)&tb.t, tn * 4) || !alloc((void**)&tb.adj_first, tn * 4) ||
      !alloc((void**)&tb.adj_cnt, tn * 4) ||
      !alloc((void**)&tb.adj_w, tn * tb.adj_stride * 4)) {
    ptycho_mono_destroy(m);
    return fail(nullptr, PTYCHO_E_OOM, "device allocation failed");
  }
  hipError_t e = launch_mono_tables(m->w, n, m->stream);
  std::vector<int> hcnt(tn);
  if (e == hipSuccess) e = hipMemcpyAsync(hcnt.data(), tb.adj_cnt, tn * sizeof(int), hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  tb.adj_max = 0;
  for (int c : hcnt) tb.adj_max = std::max(tb.adj_max, c);
  if (e != hipSuccess) {
    ptycho_mono_destroy(m);
    return fail(nullptr, PTYCHO_E_HIP, std::string("monochromatisation tables: ") + hipGetErrorString(e));
  }
  *out = m;
  return PTYCHO_OK;
}

ptycho_status ptycho_mono_run(ptycho_mono* m, const float* broadband, float* mono_out, int32_t n_patterns,
                              int32_t k_iters, float* residuals, int32_t mem_kind) {
  if (!m || !broadband || !mono_out) return fail(nullptr, PTYCHO_E_INVALID, "NULL argument");
  if (n_patterns < 1 || n_patterns > m->max_pat) return fail(nullptr, PTYCHO_E_SHAPE, "n_patterns must be in [1, max_patterns]");
  if (k_iters < 0 || k_iters > 100000) return fail(nullptr, PTYCHO_E_INVALID, "k_iters must be in [0, 100000]");
  if (mem_kind != PTYCHO_MEM_HOST && mem_kind != PTYCHO_MEM_DEVICE) return fail(nullptr, PTYCHO_E_INVALID, "bad mem_kind");
  const size_t bytes = (size_t)m->n * m->n * n_patterns * sizeof(float);
  hipStream_t s = m->stream;
  const float* b = broadband;
  float* x = mono_out;
  if (mem_kind == PTYCHO_MEM_HOST) {
    if (hipMemcpyAsync(m->d_in, broadband, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(nullptr, PTYCHO_E_HIP, "upload failed");
    b = m->d_in;
    x = m->d_out;
  }
  const size_t nres = (size_t)n_patterns * (k_iters + 1);
  if (residuals && nres > m->res_cap) {
    if (m->d_res) (void)hipFree(m->d_res);
    m->d_res = nullptr;
    m->res_cap = 0;
    if (hipMalloc((void**)&m->d_res, nres * sizeof(float)) != hipSuccess) return fail(nullptr, PTYCHO_E_OOM, "residual buffer");
    m->res_cap = nres;
  }
  hipError_t e = launch_mono_cgls(b, x, m->w, m->n, n_patterns, k_iters, residuals ? m->d_res : nullptr, s);
  if (e == hipSuccess && mem_kind == PTYCHO_MEM_HOST) e = hipMemcpyAsync(mono_out, x, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && residuals) e = hipMemcpyAsync(residuals, m->d_res, nres * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(nullptr, PTYCHO_E_HIP, std::string("monochromatisation: ") + hipGetErrorString(e));
  return PTYCHO_OK;
}

void ptycho_mono_destroy(ptycho_mono* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  for (void* p : m->allocs) (void)hipFree(p);
  if (m->d_res) (void)hipFree(m->d_res);
  delete m;
}

const char* ptycho_group_last_error(const ptycho_group* g) { return g ? g->err.c_str() : g_thread_error.c_str(); }

}  // extern "C"
