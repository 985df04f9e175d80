// HIP kernels (gfx950) of one pc-ePIE batch update and its per-iteration bookkeeping.
//
// One batch of B scan positions, each with K incoherent probe modes, moves
// through seven launches (frames live in X[b][k][N][N], complex64):
//   fwd_rows        psi = o_b P_k (box gather fused), 1D transform along x      (Eq. 1);
//                   side blocks: per-tile max of W = sum_b |P(r - r_b)|^2 and
//                   V = sum_b |o_b|^2, both from the pre-update state
//   fwd_cols        1D transform along y; I_mod = sum_k |Psi_k|^2 (mode sum); vertical
//                   half of the Gaussian blur of sqrt(I_mod) (or I_mod)        (Eq. 6-7, box 1)
//   modulus_factor  horizontal half of the blur over whole rows, modulus factor, data error
//   inv_cols        Psi_k again (recomputed in the far field), Psi' = factor Psi,
//                   inverse 1D transform along y
//   inv_rows        inverse along x -> psi'; dpsi = psi' - o_b P_k; per-slot object
//                   numerator sum_k conj(P_k) dpsi_k; X <- conj(o_b) dpsi_k
//   obj_update      probe blocks: N_P,k = sum_b X[b][k], P_k update, sum_k |P_k|^2 into
//                   the probe-power copy the next batch reads; tile blocks: N_O gathered
//                   per object tile in slot order, O update and, in constraint windows,
//                   the C-bar sums of Eq. (11)
//   constraint      the complex constraint, Eq. (9)-(10)                      (box 2)
// The launch variant cols_fused does fwd_cols, modulus_factor and inv_cols in one launch.
// Near-field frames use the separable paraxial transfer function: each 1D
// pass is forward FFT, multiply by h, inverse FFT.  Every reduction runs in a
// fixed order (no atomics), so results are bitwise reproducible.
#include "kernels.hpp"

#include <cmath>
#include <type_traits>

#include "fft_lds.hpp"
#include "kernels_dev.hpp"

#include <hip/hip_ext.h>

namespace pty {

const char* const kKernelNames[KC_COUNT] = {
    "fwd_rows", "fwd_cols", "inv_cols", "inv_rows_update", "obj_probe_update", "complex_constraint",
    "gram", "eig", "mode_remix", "err_reduce", "dft_bf16_gemm", "dft_pointwise", "modulus_factor", "cols_fused",
    "dm_rows", "dm_overlap", "seq_iteration", "lsq_direction", "lsq_step", "lsq_apply"};

LaunchEvents& launch_events() {
  thread_local LaunchEvents ev;
  return ev;
}

struct SideScratch;
__device__ void side_job(const DevParams& p, const DevBufsG& d, int pwc, const int* slots, int ns, int job,
                         bool with_v, SideScratch& sc);

// Row pass 1: psi = o_b P_k and the 1D transform along x.  Serial launches walk
// the K modes in one workgroup (blocks past the case's slots do the batch's side
// work); MP launches take one mode each, the side blocks following the
// `main_blocks` mode-parallel ones.
template <int N, bool NEAR, bool MP>
__global__ __launch_bounds__(kThreads) void k_fwd_rows(const CaseDesc* __restrict__ cases, int beta, const int* __restrict__ it,
                                                       int km, int main_blocks) {
  constexpr int L = Cfg<N>::ROWS;
  constexpr int LS = RegShape<N, L>::LOAD_SLOTS;
  constexpr int GX = N / L;
  extern __shared__ float2 sm[];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  int b, bx, k0 = 0;
  if (MP) {
    if ((int)blockIdx.x >= main_blocks) {
      side_job(p, d, pw_copy(bt.flags, beta), bt.slots, bt.ns,
               (int)blockIdx.x - main_blocks, (bt.flags & FLAG_PROBE) != 0, *reinterpret_cast<SideScratch*>(sm));
      return;
    }
    int tile;
    mp_decode(blockIdx.x, km, tile, k0);
    b = tile / GX;
    bx = tile % GX;
    if (b >= bt.ns || k0 >= p.k) return;
  } else {
    b = blockIdx.x / GX;
    bx = blockIdx.x % GX;
    if (b >= bt.ns) {
      side_job(p, d, pw_copy(bt.flags, beta), bt.slots, bt.ns, (b - bt.ns) * GX + bx,
               (bt.flags & FLAG_PROBE) != 0, *reinterpret_cast<SideScratch*>(sm));
      return;
    }
  }
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N;
  const int y0 = bx * L;
  const int2 rc = d.pos[bt.slots[b]];
  for (int i = threadIdx.x; i < N; i += kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  const int K = p.k, W = p.w_obj;
  float2 o[LS];
  const float2* orow = d.obj + (size_t)(rc.x + y0) * W + rc.y;
  for_load_slots<N, L, false>([&](int s, int line, int pos) { o[s] = orow[line * W + pos]; });
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  const float2* p0 = d.probe + ((size_t)k0 * N + y0) * N;
  float2* x0 = d.X + (((size_t)b * K + k0) * N + y0) * N;
  auto gather = [&](int k, float2* v) {
    const float2* pk = p0 + (size_t)k * N * N;
    auto load = [&](int s, int line, int pos) { return cmul(o[s], pk[line * N + pos]); };
    fft_gather<N, L, false>(v, load);
  };
  auto store_for = [&](int k) {
    float2* out = x0 + (size_t)k * N * N;
    return [=](int s, int line, int pos, float2 v) { out[line * N + pos] = cscale(v, scale); };
  };
  mode_loop<N, L, false, false, NEAR, false>(MP ? 1 : K, buf, tw, hn, gather, store_for);
}

// Epilogue of the inverse row pass: psi' -> dpsi = psi' - o P_k; the object
// numerator sum_k conj(P_k) dpsi_k accumulates in acc; the frame becomes
// conj(o) dpsi_k (the probe numerator's contribution).  P_k and o are fetched
// (P_k by pre(), the box once per workgroup) for every output slot before the transform.
template <int N, int SS>
struct InvRowsStore {
  float2* fr;
  const float2* pk;
  const float2* ov;  // the box values of the thread's output slots (registers)
  float2* dbgp;
  float2* acc;
  float scale;
  float2 pv[SS];
  __device__ __forceinline__ void pre(int s, int line, int pos) { pv[s] = pk[line * N + pos]; }
  __device__ __forceinline__ void operator()(int s, int line, int pos, float2 v) {
    const float2 psi_new = cscale(v, scale);
    const float2 dpsi = csub(psi_new, cmul(ov[s], pv[s]));
    acc[s] = cadd(acc[s], cmulc(dpsi, pv[s]));  // conj(P) dpsi
    fr[line * N + pos] = cmulc(dpsi, ov[s]);    // conj(o) dpsi
    if (dbgp) dbgp[line * N + pos] = psi_new;
  }
};

template <int N, bool NEAR>
__global__ __launch_bounds__(kThreads) void k_inv_rows(const CaseDesc* __restrict__ cases, int beta, const int* __restrict__ it) {
  constexpr int L = Cfg<N>::ROWS;
  constexpr int SS = RegShape<N, L>::STORE_SLOTS;
  constexpr int GX = N / L;
  extern __shared__ float2 sm[];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const int b = blockIdx.x / GX, bx = blockIdx.x % GX;
  if (b >= bt.ns) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const DebugPtrsG dbg = global_dbg(bt.cs->dbg);
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N;
  const int y0 = bx * L;
  const int2 rc = d.pos[bt.slots[b]];
  for (int i = threadIdx.x; i < N; i += kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  const int K = p.k, W = p.w_obj;
  float2 acc[SS];
  const float2* orow = d.obj + (size_t)(rc.x + y0) * W + rc.y;
#pragma unroll
  for (int i = 0; i < SS; ++i) acc[i] = make_float2(0.f, 0.f);
  float2 ob[SS];
  for_store_slots<N, L, false>([&](int s, int line, int pos) { ob[s] = orow[line * W + pos]; });
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  float2* x0 = d.X + ((size_t)b * K * N + y0) * N;
  const float2* p0 = d.probe + (size_t)y0 * N;
  float2* dbg0 = dbg.psi_new ? dbg.psi_new + ((size_t)b * K * N + y0) * N : nullptr;
  auto gather = [&](int k, float2* v) {
    const float2* fr = x0 + (size_t)k * N * N;
    auto load = [&](int s, int line, int pos) { return fr[line * N + pos]; };
    fft_gather<N, L, false>(v, load);
  };
  auto store_for = [&](int k) {
    InvRowsStore<N, SS> st;
    st.fr = x0 + (size_t)k * N * N;
    st.pk = p0 + (size_t)k * N * N;
    st.ov = ob;
    st.dbgp = dbg0 ? dbg0 + (size_t)k * N * N : nullptr;
    st.acc = acc;
    st.scale = scale;
    return st;
  };
  mode_loop<N, L, false, true, NEAR, true>(K, buf, tw, hn, gather, store_for);
  float2* dO = d.dO + ((size_t)b * N + y0) * N;
  for_store_slots<N, L, false>([&](int s, int line, int pos) { dO[line * N + pos] = acc[s]; });
}

// The inverse row pass over two slots per workgroup of 512 threads, one slot per
// 256-thread half (LDS: a transform buffer per half and one exchange buffer).
// Same transforms and epilogue as k_inv_rows, except that the probe numerator
// contributions of the pair are added on chip: frame k of slot 2m receives
// conj(o_2m) dpsi_2m,k + conj(o_2m+1) dpsi_2m+1,k (the second half hands its values
// over through LDS) and the frames of slot 2m + 1 are left as they are, which
// halves the contribution frames this pass writes and the probe update reads.
// Without a slot 2m + 1 (the last pair of an odd batch) the second half
// transforms slot 2m again and discards the result, so that both halves pass the
// same synchronisations.
template <int N, int NL, int SS>
struct InvRowsPairStore {
  float2* fr;
  const float2* pk;
  const float2* ov;
  float2* dbgp;
  float2* acc;
  float2* xch;  // [SS][256]
  float scale;
  bool second, has_second;
  float2 pv[SS];
  float2 xv[SS];
  __device__ __forceinline__ void pre(int s, int line, int pos) { pv[s] = pk[line * N + pos]; }
  __device__ __forceinline__ void operator()(int s, int line, int pos, float2 v) {
    const float2 psi_new = cscale(v, scale);
    const float2 dpsi = csub(psi_new, cmul(ov[s], pv[s]));
    acc[s] = cadd(acc[s], cmulc(dpsi, pv[s]));  // conj(P) dpsi
    xv[s] = cmulc(dpsi, ov[s]);                 // conj(o) dpsi
    if (dbgp) dbgp[line * N + pos] = psi_new;
  }
  __device__ __forceinline__ void post() {
    const int t = fft_tid();
    if (second) for_store_slots<N, NL, false>([&](int s, int, int) { xch[s * 256 + t] = xv[s]; });
    __syncthreads();
    if (!second)
      for_store_slots<N, NL, false>([&](int s, int line, int pos) {
        fr[line * N + pos] = has_second ? cadd(xv[s], xch[s * 256 + t]) : xv[s];
      });
  }
};

// Frame sizes with a paired inverse row pass: the power-of-two sizes up to 512,
// whose pair kernels fit 256 registers per thread without spilling (the
// radix-3 plans and N = 1024 keep one slot per workgroup).
template <int N>
struct PairRows {
  static constexpr bool value = (N & (N - 1)) == 0 && N <= 512;
};

template <int N>
constexpr size_t inv_rows_pair_lds() {
  return sizeof(float2) *
         (2 * N + 2 * Frame<N, Cfg<N>::ROWS, false>::ELEMS + RegShape<N, Cfg<N>::ROWS>::STORE_SLOTS * 256);
}

template <int N, bool NEAR>
__global__ __launch_bounds__(2 * kThreads) void k_inv_rows_pair(const CaseDesc* __restrict__ cases, int beta,
                                                                const int* __restrict__ it) {
  constexpr int L = Cfg<N>::ROWS;
  constexpr int SS = RegShape<N, L>::STORE_SLOTS;
  constexpr int GX = N / L;
  constexpr int EL = Frame<N, L, false>::ELEMS;
  extern __shared__ float2 sm[];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const int b0 = 2 * (blockIdx.x / GX), bx = blockIdx.x % GX;
  if (b0 >= bt.ns) return;
  const bool second = threadIdx.x >= kThreads;
  const bool has_second = b0 + 1 < bt.ns;
  const bool real = !second || has_second;
  const int b = (second && has_second) ? b0 + 1 : b0;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const DebugPtrsG dbg = global_dbg(bt.cs->dbg);
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N + (second ? EL : 0);
  float2* xch = sm + 2 * N + 2 * EL;
  const int y0 = bx * L;
  const int2 rc = d.pos[bt.slots[b]];
  for (int i = threadIdx.x; i < N; i += 2 * kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  const int K = p.k, W = p.w_obj;
  float2 acc[SS];
  const float2* orow = d.obj + (size_t)(rc.x + y0) * W + rc.y;
#pragma unroll
  for (int i = 0; i < SS; ++i) acc[i] = make_float2(0.f, 0.f);
  float2 ob[SS];
  for_store_slots<N, L, false>([&](int s, int line, int pos) { ob[s] = orow[line * W + pos]; });
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  float2* x0 = d.X + ((size_t)b * K * N + y0) * N;
  const float2* p0 = d.probe + (size_t)y0 * N;
  float2* dbg0 = (dbg.psi_new && real) ? dbg.psi_new + ((size_t)b * K * N + y0) * N : nullptr;
  auto gather = [&](int k, float2* v) {
    const float2* fr = x0 + (size_t)k * N * N;
    auto load = [&](int s, int line, int pos) { return fr[line * N + pos]; };
    fft_gather<N, L, false>(v, load);
  };
  auto store_for = [&](int k) {
    InvRowsPairStore<N, L, SS> st;
    st.fr = x0 + (size_t)k * N * N;  // written by the first half only (slot 2m)
    st.pk = p0 + (size_t)k * N * N;
    st.ov = ob;
    st.dbgp = dbg0 ? dbg0 + (size_t)k * N * N : nullptr;
    st.acc = acc;
    st.xch = xch;
    st.scale = scale;
    st.second = second;
    st.has_second = has_second;
    return st;
  };
  mode_loop<N, L, false, true, NEAR, true>(K, buf, tw, hn, gather, store_for);
  if (!real) return;
  float2* dO = d.dO + ((size_t)b * N + y0) * N;
  for_store_slots<N, L, false>([&](int s, int line, int pos) { dO[line * N + pos] = acc[s]; });
}

// ---------------------------------------------------------------------------
// Column passes (lines along y; Frame<N, C, true>: adjacent threads take
// adjacent columns, so every global access is a coalesced row segment)
// ---------------------------------------------------------------------------

// Forward column transform of every mode, the incoherent mode sum, and the
// vertical (sigma2) half of the separable Gaussian blur of Eq. (6) (or of the
// intensity, Eq. 2): q = g_y (x) sqrt(sum_k |Psi_k|^2).  Only q leaves the
// workgroup in the far field (the inverse column pass recomputes Psi_k, which
// costs less than a write and a read of K frames); near-field Psi_k are stored.
template <int N, bool NEAR, int C>
__global__ __launch_bounds__(kThreads) void k_fwd_cols(const CaseDesc* __restrict__ cases, int beta, const int* __restrict__ it) {
  constexpr int SS = RegShape<N, C>::STORE_SLOTS;
  constexpr int GX = N / C;
  extern __shared__ float2 sm[];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const int pt = paired_tile(blockIdx.x);
  const int b = pt / GX, bx = pt % GX;
  if (b >= bt.ns) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N;
  const int x0 = bx * C;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  const int K = p.k;
  float acc[SS];
#pragma unroll
  for (int i = 0; i < SS; ++i) acc[i] = 0.f;
  // blur taps in LDS: read in the store loop below without reloads behind its global stores
  __shared__ float sgy[kMaxHalf + 1];
  if (threadIdx.x <= kMaxHalf) sgy[threadIdx.x] = p.gy[threadIdx.x];
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  float2* f0 = d.X + (size_t)b * K * N * N + x0;
  auto gather = [&](int k, float2* v) {
    const float2* fr = f0 + (size_t)k * N * N;
    auto load = [&](int s, int c, int y) { return fr[y * N + c]; };
    fft_gather<N, C, true>(v, load);
  };
  // the far-field inverse column pass recomputes this transform, so only the
  // near-field frames are written back
  auto store_for = [&](int k) {
    float2* fr = f0 + (size_t)k * N * N;
    return [&, fr](int s, int c, int y, float2 v) {
      v = cscale(v, scale);
      if (NEAR) fr[y * N + c] = v;
      acc[s] += v.x * v.x + v.y * v.y;
    };
  };
  mode_loop<N, C, true, false, NEAR, false>(K, buf, tw, hn, gather, store_for);
  // vertical blur of the modelled amplitude (or intensity) over whole columns
  float* tile = reinterpret_cast<float*>(buf);
  constexpr int TS = C + 1;
  const bool inten = p.blur_intensity != 0;
  float* q = d.q + (size_t)b * N * N + x0;
  const int h = p.ks_half;
  const float* gy = sgy;
  // taps outermost for independent per-element chains (each element still adds
  // its taps in the order 0, 1, ..., h)
  float gv[SS];
  constexpr int H = kMaxHalf;
  if constexpr (N >= 2 * H) {
    // the column tile with kMaxHalf rows of periodic padding above and below (it fits
    // the transform buffer from N = 2 kMaxHalf): every tap reads at a fixed offset
    // from the element's row, no index wrap
    for_store_slots<N, C, true>([&](int s, int c, int y) {
      const float v = inten ? acc[s] : sqrtf(acc[s]);
      tile[(y + H) * TS + c] = v;
      if (y < H) tile[(y + N + H) * TS + c] = v;
      if (y >= N - H) tile[(y - N + H) * TS + c] = v;
    });
    __syncthreads();
    for_store_slots<N, C, true>([&](int s, int c, int y) { gv[s] = gy[0] * tile[(y + H) * TS + c]; });
#pragma unroll
    for (int dy = 1; dy <= H; ++dy) {
      if (dy <= h) {  // uniform: the taps beyond the kernel's half-width are skipped
        const float gd = gy[dy];
        for_store_slots<N, C, true>([&](int s, int c, int y) {
          gv[s] += gd * (tile[(y + H - dy) * TS + c] + tile[(y + H + dy) * TS + c]);
        });
      }
    }
  } else {
    for_store_slots<N, C, true>([&](int s, int c, int y) { tile[y * TS + c] = inten ? acc[s] : sqrtf(acc[s]); });
    __syncthreads();
    for_store_slots<N, C, true>([&](int s, int c, int y) { gv[s] = gy[0] * tile[y * TS + c]; });
    for (int dy = 1; dy <= h; ++dy) {
      const float gd = gy[dy];
      for_store_slots<N, C, true>([&](int s, int c, int y) {
        gv[s] += gd * (tile[wrap(y - dy, N) * TS + c] + tile[wrap(y + dy, N) * TS + c]);
      });
    }
  }
  for_store_slots<N, C, true>([&](int s, int c, int y) { q[y * N + c] = gv[s]; });
}

// Horizontal (sigma1) half of the blur over whole rows, the modulus factor of
// box 1 and the data error: f = sqrt(I_meas) / (g_x (x) q + eps) (Eq. 6-7), or
// sqrt(I_meas / (g_x (x) q + eps^2)) for the intensity blur (Eq. 2), written over
// q in place; one data-error partial per row block.
template <int N>
__global__ __launch_bounds__(kThreads) void k_factor(const CaseDesc* __restrict__ cases, int beta, const int* __restrict__ it) {
  constexpr int L = FactorRows<N>::R;
  constexpr int GX = N / L;
  constexpr int E = (L * N + kThreads - 1) / kThreads;
  __shared__ float tile[L * N];
  __shared__ float gx[kMaxHalf + 1];
  __shared__ double red[kThreads / 64];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const int b = blockIdx.x / GX, by = blockIdx.x % GX;
  if (b >= bt.ns) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const int pat = bt.slots[b];
  float* qb = d.q + ((size_t)b * N + by * L) * N;
  const float* amp = d.amp + ((size_t)pat * N + by * L) * N;
  // every input is loaded before the first store (the stores go over q)
  float av[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = threadIdx.x + j * kThreads;
    if ((L * N) % kThreads == 0 || e < L * N) {
      tile[e] = qb[e];
      av[j] = amp[e];
    }
  }
  if (threadIdx.x <= kMaxHalf) gx[threadIdx.x] = p.gx[threadIdx.x];
  __syncthreads();
  const DebugPtrsG dbg = global_dbg(bt.cs->dbg);
  float* dbgf = dbg.factor ? dbg.factor + ((size_t)b * N + by * L) * N : nullptr;
  const bool inten = p.blur_intensity != 0;
  const float eps = p.eps;
  const int h = p.ks_half;
  double err = 0.0;
  // taps outermost: the E elements' sums are independent chains (ILP); each
  // element still adds its taps in the order 0, 1, ..., h
  float gv[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = threadIdx.x + j * kThreads;
    gv[j] = ((L * N) % kThreads != 0 && e >= L * N) ? 0.f : gx[0] * tile[e];
  }
  for (int dx = 1; dx <= h; ++dx) {
    const float gd = gx[dx];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = threadIdx.x + j * kThreads;
      if ((L * N) % kThreads != 0 && e >= L * N) continue;
      const int c = e % N;
      const float* row = tile + (e - c);
      gv[j] += gd * (row[wrap(c - dx, N)] + row[wrap(c + dx, N)]);
    }
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = threadIdx.x + j * kThreads;
    if ((L * N) % kThreads != 0 && e >= L * N) continue;
    const float g = gv[j];
    const float a = av[j];
    float ag, f;
    if (inten) {
      ag = sqrtf(g);
      f = a / sqrtf(g + eps * eps);
    } else {
      ag = g;
      f = a / (g + eps);
    }
    qb[e] = f;
    if (dbgf) dbgf[e] = f;
    const double dd = (double)a - (double)ag;
    err += dd * dd;
  }
  const double tot = block_sum_d(err, red);
  if (threadIdx.x == 0) d.err_part[(size_t)pat * GX + by] = tot;
}

// Psi' = factor Psi and the inverse column transform, Psi_k recomputed from the
// row-transformed frame in the far field (mode_loop_refwd) and read back in the
// near field.  MP launches take one mode per workgroup (see mp_decode).
template <int N, bool NEAR, int C, bool MP>
__global__ __launch_bounds__(kThreads) void k_inv_cols(const CaseDesc* __restrict__ cases, int beta, const int* __restrict__ it,
                                                       int km) {
  constexpr int LS = RegShape<N, C>::LOAD_SLOTS;
  constexpr int GX = N / C;
  extern __shared__ float2 sm[];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  int b, bx, k0 = 0;
  if (MP) {
    int tile;
    mp_decode(blockIdx.x, km, tile, k0);
    b = tile / GX;
    bx = tile % GX;
    if (b >= bt.ns || k0 >= p.k) return;
  } else {
    const int pt = paired_tile(blockIdx.x);
    b = pt / GX;
    bx = pt % GX;
    if (b >= bt.ns) return;
  }
  const DevBufsG d = global_bufs(bt.cs->d);
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N;
  const int x0 = bx * C;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  float f[LS];
  const float* fq = d.q + (size_t)b * N * N + x0;
  for_load_slots<N, C, true>([&](int s, int c, int y) { f[s] = fq[y * N + c]; });
  const int K = p.k;
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  float2* f0 = d.X + ((size_t)b * K + k0) * N * N + x0;
  // Psi' = f Psi: a rounded product of its own, never fused into the first
  // butterflies, so serial and mode-parallel launches give bitwise the same frames
  auto times_f = [&](int s, float2 x) {
#pragma clang fp contract(off)
    return make_float2(x.x * f[s], x.y * f[s]);
  };
  auto store_for = [&](int k) {
    float2* fr = f0 + (size_t)k * N * N;
    return [=](int s, int c, int y, float2 v) { fr[y * N + c] = cscale(v, scale); };
  };
  if constexpr (NEAR) {
    // near field: Psi_k as the forward column pass stored it
    auto gather = [&](int k, float2* v) {
      const float2* fr = f0 + (size_t)k * N * N;
      auto load = [&](int s, int c, int y) { return times_f(s, fr[y * N + c]); };
      fft_gather<N, C, true>(v, load);
    };
    mode_loop<N, C, true, true, NEAR, true>(MP ? 1 : K, buf, tw, hn, gather, store_for);
  } else {
    // far field: Psi_k recomputed from the row-transformed frame
    auto gather = [&](int k, float2* v) {
      const float2* fr = f0 + (size_t)k * N * N;
      auto load = [&](int s, int c, int y) { return fr[y * N + c]; };
      fft_gather<N, C, true>(v, load);
    };
    mode_loop_refwd<N, C>(MP ? 1 : K, buf, tw, scale, gather, times_f, store_for);
  }
}

// The three middle passes in one workgroup per (slot, column tile): the forward
// column transform of C + 2 kFusedHalo columns (the tile and a halo on each side,
// wrapping at the frame edge) for every mode, the mode sum and the vertical
// half of the blur in LDS, the horizontal half and the modulus factor for the
// tile's C columns (the halo supplies the horizontal neighbours), then
// Psi' = factor Psi and the inverse column transform of the tile.  The forward
// results of the tile's columns go through X (re-read by the same workgroup),
// so no separate blurred-amplitude or factor arrays exist.  Valid while the
// kernel half-width is at most kFusedHalo.  Same arithmetic, element by
// element, as fwd_cols + modulus_factor + inv_cols; the data-error partials
// are per column tile.
template <int N, bool NEAR, int C>
__global__ __launch_bounds__(kThreads) void k_cols_fused(const CaseDesc* __restrict__ cases, int beta, const int* __restrict__ it) {
  constexpr int H = kFusedHalo;
  constexpr int NL = C + 2 * H;
  constexpr int SS = RegShape<N, NL>::STORE_SLOTS;
  constexpr int LS = RegShape<N, C>::LOAD_SLOTS;
  constexpr int GX = N / C;
  constexpr int TS = NL + 1;  // float tile row pitch
  extern __shared__ float2 sm[];
  __shared__ double red[kThreads / 64];
  __shared__ float sgx[kMaxHalf + 1], sgy[kMaxHalf + 1];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const int pt = paired_tile(blockIdx.x);
  const int b = pt / GX, bx = pt % GX;
  if (b >= bt.ns) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const DebugPtrsG dbg = global_dbg(bt.cs->dbg);
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N;
  const int x0 = bx * C;
  const int pat = bt.slots[b];
  for (int i = threadIdx.x; i < N; i += kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  if (threadIdx.x <= kMaxHalf) {
    sgx[threadIdx.x] = p.gx[threadIdx.x];
    sgy[threadIdx.x] = p.gy[threadIdx.x];
  }
  const int K = p.k;
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  float2* f0 = d.X + (size_t)b * K * N * N;
  // forward: all NL columns, the tile's columns written to X, |Psi|^2 summed over modes
  float acc[SS];
#pragma unroll
  for (int i = 0; i < SS; ++i) acc[i] = 0.f;
  auto gather = [&](int k, float2* v) {
    const float2* fr = f0 + (size_t)k * N * N;
    auto load = [&](int s, int l, int y) { return fr[y * N + wrap(x0 - H + l, N)]; };
    fft_gather<N, NL, true>(v, load);
  };
  auto store_for = [&](int k) {
    float2* fr = f0 + (size_t)k * N * N + x0 - H;
    return [&, fr](int s, int l, int y, float2 v) {
      v = cscale(v, scale);
      if (l >= H && l < H + C) fr[y * N + l] = v;
      acc[s] += v.x * v.x + v.y * v.y;
    };
  };
  mode_loop<N, NL, true, false, NEAR, false>(K, buf, tw, hn, gather, store_for);
  // mode sum -> tile A; vertical blur -> tile B (both in the transform buffer)
  float* ta = reinterpret_cast<float*>(buf);
  float* tb = ta + N * TS;
  const bool inten = p.blur_intensity != 0;
  for_store_slots<N, NL, true>([&](int s, int l, int y) { ta[y * TS + l] = inten ? acc[s] : sqrtf(acc[s]); });
  __syncthreads();
  const int h = p.ks_half;
  {
    float gv[SS];
    for_store_slots<N, NL, true>([&](int s, int l, int y) { gv[s] = sgy[0] * ta[y * TS + l]; });
    for (int dy = 1; dy <= h; ++dy) {
      const float gd = sgy[dy];
      for_store_slots<N, NL, true>([&](int s, int l, int y) {
        gv[s] += gd * (ta[wrap(y - dy, N) * TS + l] + ta[wrap(y + dy, N) * TS + l]);
      });
    }
    for_store_slots<N, NL, true>([&](int s, int l, int y) { tb[y * TS + l] = gv[s]; });
  }
  __syncthreads();
  // horizontal blur and the modulus factor for the tile's columns, in the inverse pass's slots
  const float* amp = d.amp + (size_t)pat * N * N + x0;
  float* dbgf = dbg.factor ? dbg.factor + (size_t)b * N * N + x0 : nullptr;
  const float eps = p.eps;
  float f[LS];
  double err = 0.0;
  {
    float av[LS], g[LS];
    for_load_slots<N, C, true>([&](int s, int c, int y) {
      av[s] = amp[y * N + c];
      g[s] = sgx[0] * tb[y * TS + H + c];
    });
    for (int dx = 1; dx <= h; ++dx) {
      const float gd = sgx[dx];
      for_load_slots<N, C, true>([&](int s, int c, int y) {
        g[s] += gd * (tb[y * TS + H + c - dx] + tb[y * TS + H + c + dx]);
      });
    }
    for_load_slots<N, C, true>([&](int s, int c, int y) {
      const float a = av[s];
      float ag;
      if (inten) {
        ag = sqrtf(g[s]);
        f[s] = a / sqrtf(g[s] + eps * eps);
      } else {
        ag = g[s];
        f[s] = a / (g[s] + eps);
      }
      if (dbgf) dbgf[y * N + c] = f[s];
      const double dd = (double)a - (double)ag;
      err += dd * dd;
    });
  }
  const double tot = block_sum_d(err, red);  // also: every tile read is done before the transforms reuse buf
  if (threadIdx.x == 0) d.err_part[(size_t)pat * GX + bx] = tot;
  // inverse: the tile's columns
  float2* c0 = f0 + x0;
  auto igather = [&](int k, float2* v) {
    const float2* fr = c0 + (size_t)k * N * N;
    auto load = [&](int s, int c, int y) {
      const float2 x = fr[y * N + c];
      return make_float2(x.x * f[s], x.y * f[s]);
    };
    fft_gather<N, C, true>(v, load);
  };
  auto istore_for = [&](int k) {
    float2* fr = c0 + (size_t)k * N * N;
    return [=](int s, int c, int y, float2 v) { fr[y * N + c] = cscale(v, scale); };
  };
  mode_loop<N, C, true, true, NEAR, true>(K, buf, tw, hn, igather, istore_for);
}

// ---------------------------------------------------------------------------
// Probe numerator / weight, object gather and updates
// ---------------------------------------------------------------------------

// Ascending list of the slots whose boxes intersect the object tile
// [r0, r0+T) x [c0, c0+T); returns the list length (uniform).  ns <= 256.
struct TileList {
  int2 pos[kMaxBatch];
  int slot[kMaxBatch];
  int cnt[kThreads / 64];
};

__device__ __forceinline__ int tile_list(const DevBufsG& d, const int* slots, int ns, int n, int r0, int c0,
                                         TileList& tl) {
  const int b = threadIdx.x;
  int2 rc = make_int2(0, 0);
  bool hit = false;
  if (b < ns) {
    rc = d.pos[slots[b]];
    hit = rc.x < r0 + kObjTile && rc.x + n > r0 && rc.y < c0 + kObjTile && rc.y + n > c0;
  }
  const unsigned long long m = __ballot(hit);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) tl.cnt[w] = __popcll(m);
  __syncthreads();
  int off = 0;
  for (int i = 0; i < w; ++i) off += tl.cnt[i];
  if (hit) {
    const int at = off + __popcll(m & ((1ull << lane) - 1ull));
    tl.slot[at] = b;
    tl.pos[at] = rc;
  }
  int total = 0;
  for (int i = 0; i < kThreads / 64; ++i) total += tl.cnt[i];
  __syncthreads();
  return total;
}

struct SideScratch {
  TileList tl;
  float red[kThreads / 64];
  int2 bp[kMaxBatch];
};

// Side work of the first pass of a batch (runs in extra blocks of k_fwd_rows,
// before any update of the batch): job < tiles: the maximum over one object
// tile of W(r) = sum_b sum_k |P_k(r - r_b)|^2; next jobs (probe update only):
// V(pix) = sum_b |o_b(pix)|^2 over one block of probe pixels and its maximum.
__device__ void side_job(const DevParams& p, const DevBufsG& d, int pwc, const int* slots, int ns, int job,
                         bool with_v, SideScratch& sc) {
  const int n = p.n;
  const int tiles_x = tiles_x_of(p);
  const int tiles = tiles_of(p);
  if (job < tiles) {
    const int r0 = (job / tiles_x) * kObjTile, c0 = (job % tiles_x) * kObjTile;
    const int cnt = tile_list(d, slots, ns, n, r0, c0, sc.tl);
    if (cnt == 0) {
      if (threadIdx.x == 0) d.maxw_part[job] = 0.f;
      return;
    }
    const int ty = threadIdx.x / kObjTile, tx = threadIdx.x % kObjTile;
    float w[kTilePix];
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) w[q] = 0.f;
    const float* pw = d.pw + (size_t)pwc * n * n;
    for (int i0 = 0; i0 < cnt; i0 += 4) {  // four slots' loads in flight, summed in slot order
      float wv[4][kTilePix];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = i0 + j;
        const int2 rc = i < cnt ? sc.tl.pos[i] : make_int2(-(1 << 20), -(1 << 20));
        const int xx = c0 + tx - rc.y;
#pragma unroll
        for (int q = 0; q < kTilePix; ++q) {
          const int yy = r0 + ty + q * kTileRowsPerPass - rc.x;
          wv[j][q] = ((unsigned)yy < (unsigned)n && (unsigned)xx < (unsigned)n) ? pw[yy * n + xx] : -1.f;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < kTilePix; ++q)
          if (wv[j][q] >= 0.f) w[q] += wv[j][q];
    }
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) m = fmaxf(m, w[q]);
    m = block_max_f(m, sc.red);
    if (threadIdx.x == 0) d.maxw_part[job] = m;
    return;
  }
  const int vb = job - tiles;
  if (!with_v || vb >= n_probe_blocks_dev(n)) return;
  for (int b = threadIdx.x; b < ns; b += kThreads) sc.bp[b] = d.pos[slots[b]];
  __syncthreads();
  const int pix = vb * kThreads + threadIdx.x;
  float vmax = 0.f;
  if (pix < n * n) {
    const int y = pix / n, x = pix - y * n;
    float v0 = 0.f, v1 = 0.f;
    int b = 0;
    const float2* ob = d.obj;
    for (; b + 8 <= ns; b += 8) {  // eight boxes' loads in flight; v0 sums even, v1 odd slots in order
      float2 o[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) o[u] = ob[(size_t)(sc.bp[b + u].x + y) * p.w_obj + sc.bp[b + u].y + x];
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        v0 += o[u].x * o[u].x + o[u].y * o[u].y;
        v1 += o[u + 1].x * o[u + 1].x + o[u + 1].y * o[u + 1].y;
      }
    }
    for (; b + 2 <= ns; b += 2) {
      const float2 o0 = d.obj[(size_t)(sc.bp[b].x + y) * p.w_obj + sc.bp[b].y + x];
      const float2 o1 = d.obj[(size_t)(sc.bp[b + 1].x + y) * p.w_obj + sc.bp[b + 1].y + x];
      v0 += o0.x * o0.x + o0.y * o0.y;
      v1 += o1.x * o1.x + o1.y * o1.y;
    }
    if (b < ns) {
      const float2 o0 = d.obj[(size_t)(sc.bp[b].x + y) * p.w_obj + sc.bp[b].y + x];
      v0 += o0.x * o0.x + o0.y * o0.y;
    }
    const float v = v0 + v1;
    d.V[pix] = v;
    vmax = v;
  }
  const float m = block_max_f(vmax, sc.red);
  if (threadIdx.x == 0) d.maxv_part[vb] = m;
}

__host__ __device__ __forceinline__ int pow2_at_least(int k) {
  int kp = 1;
  while (kp < k) kp <<= 1;
  return kp;
}
// Probe blocks: KP threads per pixel pair (KP = K rounded up to a power of 2);
// a thread takes two adjacent pixels of one mode (one 16-byte load per slot) and
// keeps four partial sums over the slots (slot b goes to sum b mod 4).
constexpr int kPostPx = 2;
constexpr int kPostUnroll = 4;
__host__ __device__ __forceinline__ int post_probe_blocks(int n, int k) {
  const int px_per = kThreads / pow2_at_least(k);
  const int groups = (n * n + kPostPx - 1) / kPostPx;
  return (groups + px_per - 1) / px_per;
}

// What k_obj_update does with the batch's sums: the pc-ePIE / pc-rPIE update, or
// for pc-LSQML the directions dO, dP_k (no state change) and, once the steps are
// known, the update along them.
constexpr int kObjEpie = 0, kObjLsqDir = 1, kObjLsqApply = 2;

// Probe side of one block of probe pixels.  kObjEpie and kObjLsqDir: numerator
// N_P,k = sum of the contribution frames X[b][k] over b = 0, xstep, 2 xstep, ... < ns
// (xstep 1: one frame per slot; 2: the paired inverse row pass left the sums of
// slots b and b + 1 in frame b), in a fixed order: four interleaved partial sums
// over the frames, combined pairwise; over the denominator (1-g) V + g max V; kObjEpie adds
// probe_step times it to P_k, kObjLsqDir stores it as dP_k with sum_k conj(P_k) dP_k
// and sum_k |dP_k|^2 per pixel.  kObjLsqApply: P_k += probe_step b dP_k.  The
// updating modes write sum_k |P_k|^2 into the probe-power copy that the next batch
// reads.
template <int MODE>
__device__ __forceinline__ void probe_update_block(const DevParams& p, const DevBufsG& d, const Batch& bt, int beta,
                                                   int xstep, float* pk2, float* red) {
  const int n = p.n, K = p.k, nf = (bt.ns + xstep - 1) / xstep;
  const size_t nn = (size_t)n * n;
  float* pw_next = d.pw + (size_t)(pw_copy(bt.flags, beta) ^ 1) * nn;
  const int px_per = kThreads / pow2_at_least(K);
  const int k = threadIdx.x / px_per, px = threadIdx.x % px_per;
  const int pix = (blockIdx.x * px_per + px) * kPostPx;
  const bool act = k < K && pix < n * n;
  // every load is issued before the first wait: the V-maximum partials, V and
  // P_k at the thread's pixels, then the slots of the numerator sum
  float mv = 0.f;
  if (MODE != kObjLsqApply)
    for (int i = threadIdx.x; i < n_probe_blocks_dev(n); i += kThreads) mv = fmaxf(mv, d.maxv_part[i]);
  float2 s[kPostUnroll][kPostPx], pv[kPostPx];
  float vv[kPostPx];
#pragma unroll
  for (int j = 0; j < kPostPx; ++j) {
    vv[j] = (act && MODE != kObjLsqApply) ? d.V[pix + j] : 0.f;
    pv[j] = act ? d.probe[(size_t)k * nn + pix + j] : make_float2(0.f, 0.f);
#pragma unroll
    for (int u = 0; u < kPostUnroll; ++u) s[u][j] = make_float2(0.f, 0.f);
  }
  if (act && MODE != kObjLsqApply) {
    // n is even, so a pixel pair never straddles the frame end and is 16-byte aligned
    const float4* x = reinterpret_cast<const float4*>(d.X + (size_t)k * nn + pix);
    const size_t st = (size_t)xstep * K * nn / kPostPx;
    auto add = [&](float2* acc, const float4& w) {
      acc[0] = cadd(acc[0], make_float2(w.x, w.y));
      acc[1] = cadd(acc[1], make_float2(w.z, w.w));
    };
    int b = 0;
    for (; b + kPostUnroll <= nf; b += kPostUnroll) {
      float4 w[kPostUnroll];
#pragma unroll
      for (int u = 0; u < kPostUnroll; ++u) w[u] = x[(size_t)(b + u) * st];
#pragma unroll
      for (int u = 0; u < kPostUnroll; ++u) add(s[u], w[u]);
    }
    for (; b < nf; ++b) add(s[0], x[(size_t)b * st]);
  }
  const float maxv = (MODE != kObjLsqApply) ? block_max_f(mv, red) : 0.f;
  const float bstep = (MODE == kObjLsqApply) ? p.probe_step * d.lsq_ab[1] : 0.f;
  float mag2[kPostPx], cr[kPostPx], ci[kPostPx];
#pragma unroll
  for (int j = 0; j < kPostPx; ++j) {
    mag2[j] = cr[j] = ci[j] = 0.f;
    if (!act) continue;
    const size_t q = (size_t)k * nn + pix + j;
    float2 v = pv[j];
    if (MODE == kObjLsqApply) {
      const float2 dp = d.lsq_dp[q];
      v.x += bstep * dp.x;
      v.y += bstep * dp.y;
      d.probe[q] = v;
      mag2[j] = v.x * v.x + v.y * v.y;
      continue;
    }
    // partial sums combined pairwise: (s0 + s2) + (s1 + s3)
    const float2 np = cadd(cadd(s[0][j], s[2][j]), cadd(s[1][j], s[3][j]));
    d.nP[q] = np;
    const float den = (1.0f - p.gamma_probe) * vv[j] + p.gamma_probe * maxv;
    if (MODE == kObjLsqDir) {
      const float2 dp = den > 0.f ? cscale(np, 1.0f / den) : make_float2(0.f, 0.f);
      d.lsq_dp[q] = dp;
      const float2 c = cmulc(dp, v);  // conj(P_k) dP_k
      cr[j] = c.x;
      ci[j] = c.y;
      mag2[j] = dp.x * dp.x + dp.y * dp.y;
      continue;
    }
    if (den > 0.f) {
      const float sc = p.probe_step / den;
      v.x += sc * np.x;
      v.y += sc * np.y;
      d.probe[q] = v;
    }
    mag2[j] = v.x * v.x + v.y * v.y;
  }
  constexpr int kPlanes = MODE == kObjLsqDir ? 3 : 1;
#pragma unroll
  for (int j = 0; j < kPostPx; ++j) {
    pk2[j * kThreads + threadIdx.x] = mag2[j];
    if (kPlanes == 3) {
      pk2[(kPostPx + j) * kThreads + threadIdx.x] = cr[j];
      pk2[(2 * kPostPx + j) * kThreads + threadIdx.x] = ci[j];
    }
  }
  __syncthreads();
  if (k == 0 && pix < n * n) {
#pragma unroll
    for (int j = 0; j < kPostPx; ++j) {
      float pw = 0.f, sr = 0.f, si = 0.f;
      for (int kk = 0; kk < K; ++kk) {
        pw += pk2[j * kThreads + kk * px_per + px];
        if (kPlanes == 3) {
          sr += pk2[(kPostPx + j) * kThreads + kk * px_per + px];
          si += pk2[(2 * kPostPx + j) * kThreads + kk * px_per + px];
        }
      }
      if (MODE == kObjLsqDir) {
        d.lsq_dp2[pix + j] = pw;
        d.lsq_pdp[pix + j] = make_float2(sr, si);
      } else {
        pw_next[pix + j] = pw;
      }
    }
  }
}

// Object and probe update of a batch in one launch (both read only the state
// before the batch): blocks [0, probe blocks) run probe_update_block (only in
// iterations with probe update); the next blocks, one per object tile, gather the
// object numerator and weight over the covering slots in ascending order.
// kObjEpie: O += obj_step N_O / ((1-g) W + g max W); kObjLsqDir: that quotient
// without the step is stored as dO and O is left; kObjLsqApply: no gather (each
// pixel's box count only), O += obj_step a dO.  Inside a constraint window the
// updating modes also write the tile's share of the C-bar sums of Eq. (11), each
// pixel counted once per box that covers it, and the tile's coverage bitmasks.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_obj_update(const CaseDesc* __restrict__ cases, int beta, const int* __restrict__ it,
                                                         int xstep) {
  __shared__ TileList tl;
  __shared__ float red[kThreads / 64];
  __shared__ double2 redd[kThreads / 64];
  __shared__ float pk2[(MODE == kObjLsqDir ? 3 : 1) * kPostPx * kThreads];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const DebugPtrsG dbg = global_dbg(bt.cs->dbg);
  const int pb = (bt.flags & FLAG_PROBE) ? post_probe_blocks(p.n, p.k) : 0;
  if ((int)blockIdx.x < pb) {
    probe_update_block<MODE>(p, d, bt, beta, xstep, pk2, red);
    return;
  }
  const int tiles = tiles_of(p), tiles_x = tiles_x_of(p);
  const int tile = blockIdx.x - pb;
  if (tile >= tiles) return;
  const bool cc_sums = MODE != kObjLsqDir && (bt.flags & FLAG_CC) != 0;
  const int n = p.n;
  const int r0 = (tile / tiles_x) * kObjTile, c0 = (tile % tiles_x) * kObjTile;
  const int cnt = tile_list(d, bt.slots, bt.ns, n, r0, c0, tl);
  if (cnt == 0) {
    if (cc_sums && threadIdx.x == 0) d.cc_part[tile] = make_double2(0.0, 0.0);
    if (cc_sums && threadIdx.x < kObjTile) d.cov_mask[(size_t)tile * kObjTile + threadIdx.x] = 0u;
    return;
  }
  const size_t nn = (size_t)n * n;
  const int ty = threadIdx.x / kObjTile, tx = threadIdx.x % kObjTile;
  const int c = c0 + tx;
  // loads that do not depend on the gathers are issued with them: the W-maximum
  // partials and the tile's object values (or directions)
  float mw = 0.f;
  if (MODE != kObjLsqApply)
    for (int i = threadIdx.x; i < tiles; i += kThreads) mw = fmaxf(mw, d.maxw_part[i]);
  float2 ov[kTilePix], dv[kTilePix];
#pragma unroll
  for (int q = 0; q < kTilePix; ++q) {
    const int r = r0 + ty + q * kTileRowsPerPass;
    const bool inside = r < p.h_obj && c < p.w_obj;
    const size_t oi = (size_t)r * p.w_obj + c;
    ov[q] = (inside && MODE != kObjLsqDir) ? d.obj[oi] : make_float2(0.f, 0.f);
    dv[q] = (inside && MODE == kObjLsqApply) ? d.lsq_do[oi] : make_float2(0.f, 0.f);
  }
  float w[kTilePix];
  float2 num[kTilePix];
  int mult[kTilePix];
#pragma unroll
  for (int q = 0; q < kTilePix; ++q) {
    w[q] = 0.f;
    num[q] = make_float2(0.f, 0.f);
    mult[q] = 0;
  }
  if (MODE == kObjLsqApply) {
    const int xx0 = c0 + tx;
    for (int i = 0; i < cnt; ++i) {
      const int2 rc = tl.pos[i];
      const bool col_in = (unsigned)(xx0 - rc.y) < (unsigned)n;
#pragma unroll
      for (int q = 0; q < kTilePix; ++q)
        mult[q] += (col_in && (unsigned)(r0 + ty + q * kTileRowsPerPass - rc.x) < (unsigned)n) ? 1 : 0;
    }
  } else {
    // slots are visited in ascending order; the loads of kGather slots are issued
    // together before their (in-order) accumulation
    constexpr int kGather = 4;
    const float* pw = d.pw + (size_t)pw_copy(bt.flags, beta) * nn;
    for (int i0 = 0; i0 < cnt; i0 += kGather) {
      float wv[kGather][kTilePix];
      float2 nv[kGather][kTilePix];
      bool in[kGather][kTilePix];
#pragma unroll
      for (int j = 0; j < kGather; ++j) {
        const int i = i0 + j;
        const int2 rc = i < cnt ? tl.pos[i] : make_int2(-(1 << 20), -(1 << 20));
        const float2* dOb = d.dO + (size_t)(i < cnt ? tl.slot[i] : 0) * nn;
        const int xx = c0 + tx - rc.y;
#pragma unroll
        for (int q = 0; q < kTilePix; ++q) {
          const int yy = r0 + ty + q * kTileRowsPerPass - rc.x;
          in[j][q] = (unsigned)yy < (unsigned)n && (unsigned)xx < (unsigned)n;
          wv[j][q] = in[j][q] ? pw[yy * n + xx] : 0.f;
          nv[j][q] = in[j][q] ? dOb[yy * n + xx] : make_float2(0.f, 0.f);
        }
      }
#pragma unroll
      for (int j = 0; j < kGather; ++j)
#pragma unroll
        for (int q = 0; q < kTilePix; ++q)
          if (in[j][q]) {
            w[q] += wv[j][q];
            num[q] = cadd(num[q], nv[j][q]);
            ++mult[q];
          }
    }
  }
  const float maxw = (MODE != kObjLsqApply) ? block_max_f(mw, red) : 0.f;
  const float gam = p.gamma_obj, step = p.obj_step;
  const float astep = (MODE == kObjLsqApply) ? p.obj_step * d.lsq_ab[0] : 0.f;
  float sa = 0.f, sp = 0.f;
#pragma unroll
  for (int q = 0; q < kTilePix; ++q) {
    const int r = r0 + ty + q * kTileRowsPerPass;
    if (!mult[q] || r >= p.h_obj || c >= p.w_obj) continue;
    const size_t oi = (size_t)r * p.w_obj + c;
    if (MODE != kObjLsqApply && dbg.n_obj) {
      dbg.n_obj[oi] = num[q];
      dbg.w_obj[oi] = w[q];
    }
    float2 o = ov[q];
    if (MODE == kObjLsqApply) {
      o.x += astep * dv[q].x;
      o.y += astep * dv[q].y;
      d.obj[oi] = o;
    } else {
      const float den = (1.0f - gam) * w[q] + gam * maxw;
      if (MODE == kObjLsqDir) {
        d.lsq_do[oi] = den > 0.f ? cscale(num[q], 1.0f / den) : make_float2(0.f, 0.f);
        continue;
      }
      if (den > 0.f) {
        const float s = step / den;
        o.x += s * num[q].x;
        o.y += s * num[q].y;
        d.obj[oi] = o;
      }
    }
    if (cc_sums) {
      sa += mult[q] * fabsf(cc_ln_amp(o));
      sp += mult[q] * fabsf(cc_phase(o));
    }
  }
  if (cc_sums) {
    // coverage bitmasks of the tile's rows for the constraint pass: a wave holds rows
    // ty = 2w and 2w + 1 (lanes 0-31 and 32-63) of each group of eight
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) {
      const int r = r0 + ty + q * kTileRowsPerPass;
      const unsigned long long m = __ballot(mult[q] > 0 && r < p.h_obj && c < p.w_obj);
      if (lane == 0) {
        unsigned* mk = d.cov_mask + (size_t)tile * kObjTile + 2 * w + q * kTileRowsPerPass;
        mk[0] = (unsigned)m;
        mk[1] = (unsigned)(m >> 32);
      }
    }
    const double2 t = block_sum_d2((double)sa, (double)sp, redd);
    if (threadIdx.x == 0) d.cc_part[tile] = t;
  }
}

// The complex constraint, Eq. (9)-(10), on kCcTiles object tiles per block: on
// the tiles' pixels that lie in the union of the batch boxes (the coverage
// bitmasks the object update wrote), with C-bar of Eq. (11) from the partial
// sums the object update wrote (reduced once per block).  A block whose tiles
// hold no covered pixel (most of the object, for one batch) leaves after reading
// the bitmasks; the others fetch their covered pixels and the partial sums
// before the C-bar reduction.  One tile per block: the transcendentals want
// every wave the machine can hold (four tiles per block was measured slower).
constexpr int kCcTiles = 1;
__global__ __launch_bounds__(kThreads) void k_constraint(const CaseDesc* __restrict__ cases, int beta,
                                                         const int* __restrict__ it) {
  __shared__ double2 redd[kThreads / 64];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const int tiles = tiles_of(p);
  const int tile0 = blockIdx.x * kCcTiles;
  if (!(bt.flags & FLAG_CC) || tile0 >= tiles) return;
  const int tiles_x = tiles_x_of(p);
  const int ty = threadIdx.x / kObjTile, tx = threadIdx.x % kObjTile;
  constexpr int PX = kCcTiles * kTilePix;
  unsigned rowm[PX];
  float2 ov[PX];
  int any = 0;
#pragma unroll
  for (int u = 0; u < kCcTiles; ++u) {
    const int tile = tile0 + u;
    const bool tv = tile < tiles;
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) {
      const int rr = ty + q * kTileRowsPerPass;
      rowm[u * kTilePix + q] = tv ? d.cov_mask[(size_t)tile * kObjTile + rr] : 0u;
      any |= (int)((rowm[u * kTilePix + q] >> tx) & 1u);
    }
  }
  if (!__syncthreads_or(any)) return;
  // a covered pixel lies inside the object (the bitmasks mark no other)
#pragma unroll
  for (int u = 0; u < kCcTiles; ++u) {
    const int tile = tile0 + u;
    const int r0 = (tile / tiles_x) * kObjTile, c = (tile % tiles_x) * kObjTile + tx;
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) {
      const int e = u * kTilePix + q;
      const int r = r0 + ty + q * kTileRowsPerPass;
      ov[e] = ((rowm[e] >> tx) & 1u) ? d.obj[(size_t)r * p.w_obj + c] : make_float2(0.f, 0.f);
    }
  }
  double sa = 0.0, sp = 0.0;
  for (int i = threadIdx.x; i < tiles; i += kThreads) {
    const double2 v = d.cc_part[i];
    sa += v.x;
    sp += v.y;
  }
  const double2 tot = block_sum_d2(sa, sp, redd);
  if (!(tot.y > 0.0)) return;
  float cbar = (float)(tot.x / tot.y);
  cbar = fminf(fmaxf(cbar, p.cbar_min), p.cbar_max);
  const float inv_c = 1.0f / cbar;
  const float a1 = p.alpha1, a2 = p.alpha2;
#pragma unroll
  for (int u = 0; u < kCcTiles; ++u) {
    const int tile = tile0 + u;
    const int r0 = (tile / tiles_x) * kObjTile, c = (tile % tiles_x) * kObjTile + tx;
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) {
      const int e = u * kTilePix + q;
      if (!((rowm[e] >> tx) & 1u)) continue;  // outside the union of the boxes (or the object)
      const int r = r0 + ty + q * kTileRowsPerPass;
      d.obj[(size_t)r * p.w_obj + c] = cc_apply(ov[e], cbar, inv_c, a1, a2);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_pw(DevParams p, DevBufs d, int copy) {
  const int n = p.n;
  const size_t nn = (size_t)n * n;
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  if (pix >= n * n) return;
  float pw = 0.f;
  for (int k = 0; k < p.k; ++k) {
    const float2 v = d.probe[(size_t)k * nn + pix];
    pw += v.x * v.x + v.y * v.y;
  }
  d.pw[copy * nn + pix] = pw;
}

// ---------------------------------------------------------------------------
// Mode orthogonalisation (K > 1) and the data error, per case
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_gram(const CaseDesc* __restrict__ cases, const int* __restrict__ it_ptr) {
  __shared__ double red[kThreads / 64];
  const CaseDesc* cs = cases + blockIdx.y;
  if (!(cs->flags[*it_ptr] & FLAG_ORTHO)) return;
  const DevParams& p = cs->p;
  const DevBufsG d = global_bufs(cs->d);
  const int K = p.k;
  // blockIdx.x = pair (i <= j) * kGramBlocks + pixel chunk
  int pair = blockIdx.x / kGramBlocks;
  const int chunk_id = blockIdx.x % kGramBlocks;
  if (pair >= K * (K + 1) / 2) return;
  const int pair_id = pair;
  int i = 0;
  while (pair >= K - i) {
    pair -= K - i;
    ++i;
  }
  const int j = i + pair;
  const int nn = p.n * p.n;
  const int chunk = (nn + kGramBlocks - 1) / kGramBlocks;
  const int lo = chunk_id * chunk, hi = min(nn, lo + chunk);
  const float2* pi = d.probe + (size_t)i * nn;
  const float2* pj = d.probe + (size_t)j * nn;
  double re = 0.0, im = 0.0;
  for (int e = lo + threadIdx.x; e < hi; e += kThreads) {
    const float2 a = pi[e], bq = pj[e];
    // conj(P_i) P_j
    re += (double)a.x * bq.x + (double)a.y * bq.y;
    im += (double)a.x * bq.y - (double)a.y * bq.x;
  }
  re = block_sum_d(re, red);
  im = block_sum_d(im, red);
  if (threadIdx.x == 0) d.gram_part[(size_t)pair_id * kGramBlocks + chunk_id] = make_double2(re, im);
}

// Hermitian eigendecomposition by cyclic complex Jacobi rotations (double),
// K <= 16.  One wave: the matrices live in LDS; every lane derives the same
// rotation from the same LDS values, then lane m updates entry m of the two
// rotated columns (A and the eigenvectors), and after a barrier entry m of the
// two rotated rows -- element by element the serial sequence.
__global__ __launch_bounds__(64) void k_eig(const CaseDesc* __restrict__ cases, const int* __restrict__ it_ptr) {
  __shared__ double ar[kMaxModes][kMaxModes], ai[kMaxModes][kMaxModes];
  __shared__ double vr[kMaxModes][kMaxModes], vi[kMaxModes][kMaxModes];
  __shared__ int stop;
  if (blockIdx.x != 0) return;
  const CaseDesc* cs = cases + blockIdx.y;
  if (!(cs->flags[*it_ptr] & FLAG_ORTHO)) return;
  const DevBufsG d = global_bufs(cs->d);
  const int K = cs->p.k;
  const int m = threadIdx.x;
  if (m == 0) {
    int pair = 0;
    for (int i = 0; i < K; ++i)
      for (int j = i; j < K; ++j, ++pair) {
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < kGramBlocks; ++c) {
          sr += d.gram_part[(size_t)pair * kGramBlocks + c].x;
          si += d.gram_part[(size_t)pair * kGramBlocks + c].y;
        }
        ar[i][j] = sr;
        ai[i][j] = si;
        ar[j][i] = sr;
        ai[j][i] = -si;
      }
    for (int i = 0; i < K; ++i) {
      ai[i][i] = 0.0;
      for (int j = 0; j < K; ++j) {
        vr[i][j] = (i == j) ? 1.0 : 0.0;
        vi[i][j] = 0.0;
      }
    }
  }
  __syncthreads();
  double scale = 0.0;
  for (int i = 0; i < K; ++i) scale += fabs(ar[i][i]);
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (m == 0) {
      double off = 0.0;
      for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j) off += ar[i][j] * ar[i][j] + ai[i][j] * ai[i][j];
      stop = off <= 1e-30 * scale * scale;
    }
    __syncthreads();
    const int done = stop;
    __syncthreads();  // every lane has read the flag before lane 0 can rewrite it
    if (done) break;
    for (int pp = 0; pp < K; ++pp)
      for (int qq = pp + 1; qq < K; ++qq) {
        const double gr = ar[pp][qq], gi = ai[pp][qq];
        const double mag = sqrt(gr * gr + gi * gi);
        if (mag == 0.0) continue;  // uniform: every lane read the same value
        // A_pq = mag e^{i th}; rotate with a real Jacobi angle on the phase-removed pair
        const double er = gr / mag, ei = gi / mag;  // e^{i th}
        const double app = ar[pp][pp], aqq = ar[qq][qq];
        const double tau = (aqq - app) / (2.0 * mag);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        __syncthreads();  // every lane has read the pivot before it changes
        // unitary J: columns p,q of the identity replaced by
        //   J_pp = c, J_pq = s e^{i th}, J_qp = -s e^{-i th}, J_qq = c ; A <- J^H A J
        if (m < K) {  // A <- A J (columns p, q), V <- V J
          const double xr = ar[m][pp], xi = ai[m][pp], yr = ar[m][qq], yi = ai[m][qq];
          // new col p = c x - s e^{-i th} y ; new col q = s e^{i th} x + c y
          ar[m][pp] = c * xr - s * (er * yr + ei * yi);
          ai[m][pp] = c * xi - s * (er * yi - ei * yr);
          ar[m][qq] = s * (er * xr - ei * xi) + c * yr;
          ai[m][qq] = s * (er * xi + ei * xr) + c * yi;
          const double ur = vr[m][pp], ui = vi[m][pp], wr = vr[m][qq], wi = vi[m][qq];
          vr[m][pp] = c * ur - s * (er * wr + ei * wi);
          vi[m][pp] = c * ui - s * (er * wi - ei * wr);
          vr[m][qq] = s * (er * ur - ei * ui) + c * wr;
          vi[m][qq] = s * (er * ui + ei * ur) + c * wi;
        }
        __syncthreads();
        if (m < K) {  // A <- J^H A (rows p, q)
          const double xr = ar[pp][m], xi = ai[pp][m], yr = ar[qq][m], yi = ai[qq][m];
          // new row p = c x - s e^{i th} y ; new row q = s e^{-i th} x + c y
          ar[pp][m] = c * xr - s * (er * yr - ei * yi);
          ai[pp][m] = c * xi - s * (er * yi + ei * yr);
          ar[qq][m] = s * (er * xr + ei * xi) + c * yr;
          ai[qq][m] = s * (er * xi - ei * xr) + c * yi;
        }
        __syncthreads();
        if (m == 0) {
          ar[pp][qq] = ai[pp][qq] = ar[qq][pp] = ai[qq][pp] = 0.0;
          ai[pp][pp] = ai[qq][qq] = 0.0;
        }
        __syncthreads();
      }
  }
  if (m != 0) return;
  // sort by eigenvalue, descending (stable selection)
  int ord[kMaxModes];
  bool used[kMaxModes];
  for (int i = 0; i < K; ++i) used[i] = false;
  for (int r = 0; r < K; ++r) {
    int best = -1;
    for (int i = 0; i < K; ++i)
      if (!used[i] && (best < 0 || ar[i][i] > ar[best][best])) best = i;
    used[best] = true;
    ord[r] = best;
  }
  for (int r = 0; r < K; ++r) {
    const int col = ord[r];
    // phase: largest-magnitude entry (first on ties) made real positive
    int im = 0;
    double mbest = -1.0;
    for (int i = 0; i < K; ++i) {
      const double m2 = vr[i][col] * vr[i][col] + vi[i][col] * vi[i][col];
      if (m2 > mbest) {
        mbest = m2;
        im = i;
      }
    }
    const double mg = sqrt(mbest);
    const double pr = vr[im][col] / mg, pi = -vi[im][col] / mg;  // conj(phase)
    for (int i = 0; i < K; ++i) {
      const double xr = vr[i][col], xi = vi[i][col];
      d.vmix[i * K + r] = make_float2((float)(xr * pr - xi * pi), (float)(xr * pi + xi * pr));
    }
    d.eig[r] = ar[col][col];
  }
}

__global__ __launch_bounds__(kThreads) void k_remix(const CaseDesc* __restrict__ cases, const int* __restrict__ it_ptr) {
  const CaseDesc* cs = cases + blockIdx.y;
  if (!(cs->flags[*it_ptr] & FLAG_ORTHO)) return;
  const DevBufsG d = global_bufs(cs->d);
  const int n = cs->p.n, K = cs->p.k;
  const size_t nn = (size_t)n * n;
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  if (pix >= n * n) return;
  float2 in[kMaxModes];
  for (int i = 0; i < K; ++i) in[i] = d.probe[(size_t)i * nn + pix];
  float pw = 0.f;
  for (int j = 0; j < K; ++j) {
    float2 s = make_float2(0.f, 0.f);
    for (int i = 0; i < K; ++i) s = cadd(s, cmul(in[i], d.vmix[i * K + j]));
    d.probe[(size_t)j * nn + pix] = s;
    pw += s.x * s.x + s.y * s.y;
  }
  // both copies of the probe-power map: the next iteration's first batch reads one, and its probe
  // update (or, without one, nothing) writes the other before any batch reads it
  d.pw[pix] = pw;
  d.pw[nn + pix] = pw;
}

// One 1024-thread block per case (the partials of a whole iteration are few
// but one pass of 256 threads would wait on ~12 rounds of dependent loads).
constexpr int kErrThreads = 1024;
__global__ __launch_bounds__(kErrThreads) void k_err_reduce(const CaseDesc* __restrict__ cases, const int* __restrict__ it_ptr) {
  __shared__ double red[kErrThreads / 64];
  const CaseDesc* cs = cases + blockIdx.y;
  const double* part = global_bufs(cs->d).err_part;
  const int count = cs->n_err_part;
  // eight independent partial sums per thread (eight loads in flight), combined in a fixed order
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < count; i += 8 * kErrThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = i + u * kErrThreads;
      if (j < count) acc[u] += part[j];
    }
  }
  double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kErrThreads / 64; ++w) t += red[w];
    cs->err_out[*it_ptr] = (float)(t * cs->inv_denom);
  }
}

// ---------------------------------------------------------------------------
// Init-time and debug helpers
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_prepare_amp(const float* __restrict__ inten, float* amp, int n,
                                                          int shift, int* bad, double* sum_part) {
  __shared__ double red[kThreads / 64];
  const int pat = blockIdx.y;
  const size_t nn = (size_t)n * n;
  double s = 0.0;
  int nbad = 0;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n * n; e += kThreads * gridDim.x) {
    const int y = e / n, x = e - y * n;
    float v = inten[pat * nn + e];
    if (!isfinite(v)) {
      ++nbad;
      v = 0.f;
    }
    v = fmaxf(v, 0.f);
    // far field: move the zero frequency from (n/2, n/2) to (0, 0)
    const int yo = shift ? (y + n / 2) % n : y;
    const int xo = shift ? (x + n / 2) % n : x;
    amp[pat * nn + (size_t)yo * n + xo] = sqrtf(v);
    s += (double)v;
  }
  s = block_sum_d(s, red);
  const double tb = block_sum_d((double)nbad, red);
  if (threadIdx.x == 0) {
    sum_part[(size_t)pat * gridDim.x + blockIdx.x] = s;
    bad[(size_t)pat * gridDim.x + blockIdx.x] = (int)tb;
  }
}

__global__ __launch_bounds__(kThreads) void k_exit_waves(DevParams p, DevBufs d, const int* __restrict__ slots,
                                                         int ns, float2* out) {
  const int n = p.n;
  const size_t nn = (size_t)n * n;
  const int b = blockIdx.y;
  if (b >= ns) return;
  const int2 rc = d.pos[slots[b]];
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  if (pix >= n * n) return;
  const int y = pix / n, x = pix - y * n;
  const float2 o = d.obj[(size_t)(rc.x + y) * p.w_obj + rc.y + x];
  for (int k = 0; k < p.k; ++k) out[((size_t)b * p.k + k) * nn + pix] = cmul(o, d.probe[(size_t)k * nn + pix]);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

bool supported_n(int n) {
  switch (n) {
    case 8: case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 192: case 256: case 384:
    case 512: case 768: case 1024:
      return true;
    default:
      return false;
  }
}

// Column variants and mode-parallel launches are instantiated for the frame
// sizes the autotuner explores.
template <int N>
struct TunedCols {
  static constexpr bool value = N == 64 || N == 128 || N == 192 || N == 256 || N == 512;
};

// Launch variant v: column width index v % 3 (COLS/2, COLS, 2 COLS).  v < 12:
// the three middle passes as separate launches, the inverse column pass
// mode-parallel if (v / 3) & 1, the first row pass mode-parallel if (v / 6) & 1.
// v in [12, 18): the fused column pass, the first row pass mode-parallel if
// ((v - 12) / 3) & 1.
__host__ __device__ constexpr int var_width(int v) { return v % 3; }
__host__ __device__ constexpr bool var_fused(int v) { return v >= 12; }
__host__ __device__ constexpr bool var_mp_cols(int v) { return v < 12 && ((v / 3) & 1) != 0; }
__host__ __device__ constexpr bool var_mp_rows(int v) { return v < 12 ? ((v / 6) & 1) != 0 : (((v - 12) / 3) & 1) != 0; }

template <int N>
static int col_width_t(int v) {
  switch (var_width(v)) {
    case 0: return ColW<N, 0>::C;
    case 2: return ColW<N, 2>::C;
    default: return ColW<N, 1>::C;
  }
}
template <int N>
static bool col_valid_t(int v) {
  if (v < 0 || v >= kColVariants) return false;
  if (v >= 3 && !TunedCols<N>::value) return false;
  const int w = var_width(v);
  return w == 1 || (w == 0 && ColW<N, 0>::VALID) || (w == 2 && ColW<N, 2>::VALID);
}

int col_width(int n, int v) {
  switch (n) {
#define PTY_CASE(N) \
  case N:           \
    return col_width_t<N>(v);
    PTY_FOR_EACH_N(PTY_CASE)
#undef PTY_CASE
    default:
      return 1;
  }
}
bool col_variant_valid(int n, int v) {
  switch (n) {
#define PTY_CASE(N) \
  case N:           \
    return col_valid_t<N>(v);
    PTY_FOR_EACH_N(PTY_CASE)
#undef PTY_CASE
    default:
      return false;
  }
}
bool fused_active(int n, int v, int max_half) {
  return col_variant_valid(n, v) && var_fused(v) && max_half <= kFusedHalo;
}
int n_err_slots(int n, int v, int max_half) {
  if (fused_active(n, v, max_half)) return n / col_width(n, v);
  switch (n) {
#define PTY_CASE(N) \
  case N:           \
    return N / FactorRows<N>::R;
    PTY_FOR_EACH_N(PTY_CASE)
#undef PTY_CASE
    default:
      return 1;
  }
}
int max_err_slots(int n) {
  int m = 0;
  for (int v = 0; v < kColVariants; ++v)
    if (col_variant_valid(n, v)) m = std::max(m, n_err_slots(n, v, 0));
  return m;
}
int n_obj_tiles(const DevParams& p) { return tiles_of(p); }
int n_probe_blocks(int n) { return n_probe_blocks_dev(n); }

static int mp_blocks(int tiles, int km) { return paired_blocks(tiles) * km; }

template <int N, bool NEAR>
static hipError_t fwd_rows_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  constexpr int L = Cfg<N>::ROWS;
  size_t sh = sizeof(float2) * (2 * N + Frame<N, L, false>::ELEMS);
  if (sh < sizeof(SideScratch)) sh = sizeof(SideScratch);
  const int gx = N / L;
  if constexpr (TunedCols<N>::value) {
    if (var_mp_rows(t.col_variant)) {
      const int main = mp_blocks(gx * t.max_batch, t.max_k);
      pty_launch(k_fwd_rows<N, NEAR, true>, dim3(main + t.max_side_jobs, t.n_cases), dim3(kThreads), sh, s,
                         cases, beta, it, t.max_k, main);
      return hipGetLastError();
    }
  }
  const int side_rows = (t.max_side_jobs + gx - 1) / gx;
  pty_launch(k_fwd_rows<N, NEAR, false>, dim3(gx * (t.max_batch + side_rows), t.n_cases), dim3(kThreads),
                     sh, s, cases, beta, it, 1, 0);
  return hipGetLastError();
}
template <int N, bool NEAR>
static hipError_t inv_rows_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  constexpr int L = Cfg<N>::ROWS;
  if constexpr (PairRows<N>::value) {
    if (t.x_pairs) {
      pty_launch(k_inv_rows_pair<N, NEAR>, dim3((N / L) * ((t.max_batch + 1) / 2), t.n_cases), dim3(2 * kThreads),
                 inv_rows_pair_lds<N>(), s, cases, beta, it);
      return hipGetLastError();
    }
  }
  if (t.x_pairs) return hipErrorInvalidValue;  // a shape the runtime never builds
  const size_t sh = sizeof(float2) * (2 * N + Frame<N, L, false>::ELEMS);
  pty_launch(k_inv_rows<N, NEAR>, dim3((N / L) * t.max_batch, t.n_cases), dim3(kThreads), sh, s, cases,
                     beta, it);
  return hipGetLastError();
}
// The paired inverse row pass needs more than 64 KB of LDS per workgroup.
template <int N>
static hipError_t inv_rows_pair_attr() {
  if constexpr (PairRows<N>::value) {
    const int bytes = (int)inv_rows_pair_lds<N>();
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_inv_rows_pair<N, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_inv_rows_pair<N, true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  } else {
    return hipSuccess;
  }
}
bool inv_rows_paired(int n) {
  switch (n) {
#define PTY_CASE(N) \
  case N:           \
    return PairRows<N>::value;
    PTY_FOR_EACH_N(PTY_CASE)
#undef PTY_CASE
    default:
      return false;
  }
}
hipError_t init_kernel_attributes() {
  hipError_t e = hipSuccess;
#define PTY_CASE_ATTR(N) \
  if (e == hipSuccess) e = inv_rows_pair_attr<N>();
  PTY_FOR_EACH_N(PTY_CASE_ATTR)
#undef PTY_CASE_ATTR
  return e;
}
template <int N, bool NEAR, int V>
static hipError_t fwd_cols_v(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  constexpr int C = ColW<N, V>::C;
  const size_t sh = sizeof(float2) * (2 * N + Frame<N, C, true>::ELEMS);
  pty_launch(k_fwd_cols<N, NEAR, C>, dim3(paired_blocks((N / C) * t.max_batch), t.n_cases), dim3(kThreads), sh, s,
                     cases, beta, it);
  return hipGetLastError();
}
template <int N, bool NEAR, int V>
static hipError_t cols_fused_v(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  constexpr int C = ColW<N, V>::C;
  constexpr int NL = C + 2 * kFusedHalo;
  const size_t sh = sizeof(float2) * (2 * N + Frame<N, NL, true>::ELEMS);
  pty_launch(k_cols_fused<N, NEAR, C>, dim3(paired_blocks((N / C) * t.max_batch), t.n_cases), dim3(kThreads), sh, s, cases,
                     beta, it);
  return hipGetLastError();
}
template <int N, bool NEAR>
static hipError_t cols_fused_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  if constexpr (TunedCols<N>::value) {
    if (var_width(t.col_variant) == 0) return cols_fused_v<N, NEAR, 0>(cases, t, beta, it, s);
    if (var_width(t.col_variant) == 2) return cols_fused_v<N, NEAR, 2>(cases, t, beta, it, s);
    return cols_fused_v<N, NEAR, 1>(cases, t, beta, it, s);
  }
  return hipErrorInvalidValue;
}
template <int N>
static hipError_t factor_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  pty_launch(k_factor<N>, dim3((N / FactorRows<N>::R) * t.max_batch, t.n_cases), dim3(kThreads), 0, s, cases,
                     beta, it);
  return hipGetLastError();
}
template <int N, bool NEAR, int V>
static hipError_t inv_cols_v(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  constexpr int C = ColW<N, V>::C;
  const size_t sh = sizeof(float2) * (2 * N + Frame<N, C, true>::ELEMS);
  if constexpr (TunedCols<N>::value) {
    if (var_mp_cols(t.col_variant)) {
      pty_launch(k_inv_cols<N, NEAR, C, true>, dim3(mp_blocks((N / C) * t.max_batch, t.max_k), t.n_cases),
                         dim3(kThreads), sh, s, cases, beta, it, t.max_k);
      return hipGetLastError();
    }
  }
  pty_launch(k_inv_cols<N, NEAR, C, false>, dim3(paired_blocks((N / C) * t.max_batch), t.n_cases), dim3(kThreads), sh, s,
                     cases, beta, it, 1);
  return hipGetLastError();
}
template <int N, bool NEAR>
static hipError_t fwd_cols_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  if constexpr (TunedCols<N>::value) {
    if (var_width(t.col_variant) == 0) return fwd_cols_v<N, NEAR, 0>(cases, t, beta, it, s);
    if (var_width(t.col_variant) == 2) return fwd_cols_v<N, NEAR, 2>(cases, t, beta, it, s);
  }
  return fwd_cols_v<N, NEAR, 1>(cases, t, beta, it, s);
}
template <int N, bool NEAR>
static hipError_t inv_cols_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  if constexpr (TunedCols<N>::value) {
    if (var_width(t.col_variant) == 0) return inv_cols_v<N, NEAR, 0>(cases, t, beta, it, s);
    if (var_width(t.col_variant) == 2) return inv_cols_v<N, NEAR, 2>(cases, t, beta, it, s);
  }
  return inv_cols_v<N, NEAR, 1>(cases, t, beta, it, s);
}

#define PTY_DEFINE_LAUNCH(FN)                                                                                  \
  hipError_t launch_##FN(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {      \
    switch (t.n) {                                                                                           \
      PTY_FOR_EACH_N(PTY_CASE_##FN)                                                                          \
      default:                                                                                               \
        return hipErrorInvalidValue;                                                                         \
    }                                                                                                        \
  }
#define PTY_CASE_fwd_rows(N) \
  case N:                    \
    return t.near_field ? fwd_rows_t<N, true>(cases, t, beta, it, s) : fwd_rows_t<N, false>(cases, t, beta, it, s);
#define PTY_CASE_inv_rows(N) \
  case N:                    \
    return t.near_field ? inv_rows_t<N, true>(cases, t, beta, it, s) : inv_rows_t<N, false>(cases, t, beta, it, s);
#define PTY_CASE_fwd_cols(N) \
  case N:                    \
    return t.near_field ? fwd_cols_t<N, true>(cases, t, beta, it, s) : fwd_cols_t<N, false>(cases, t, beta, it, s);
#define PTY_CASE_inv_cols(N) \
  case N:                    \
    return t.near_field ? inv_cols_t<N, true>(cases, t, beta, it, s) : inv_cols_t<N, false>(cases, t, beta, it, s);
#define PTY_CASE_factor(N) \
  case N:                  \
    return factor_t<N>(cases, t, beta, it, s);
PTY_DEFINE_LAUNCH(factor)
#define PTY_CASE_cols_fused(N) \
  case N:                      \
    return t.near_field ? cols_fused_t<N, true>(cases, t, beta, it, s) : cols_fused_t<N, false>(cases, t, beta, it, s);
PTY_DEFINE_LAUNCH(cols_fused)
PTY_DEFINE_LAUNCH(fwd_rows)
PTY_DEFINE_LAUNCH(inv_rows)
PTY_DEFINE_LAUNCH(fwd_cols)
PTY_DEFINE_LAUNCH(inv_cols)

template <int MODE>
static hipError_t obj_update_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  const int pb = post_probe_blocks(t.n, t.max_k);
  pty_launch(k_obj_update<MODE>, dim3(pb + t.max_tiles, t.n_cases), dim3(kThreads), 0, s, cases, beta, it,
             (MODE == kObjEpie && t.x_pairs) ? 2 : 1);
  return hipGetLastError();
}
hipError_t launch_obj_update(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  return obj_update_t<kObjEpie>(cases, t, beta, it, s);
}
hipError_t launch_lsq_dir(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  return obj_update_t<kObjLsqDir>(cases, t, beta, it, s);
}
hipError_t launch_lsq_apply(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  return obj_update_t<kObjLsqApply>(cases, t, beta, it, s);
}
hipError_t launch_constraint(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  pty_launch(k_constraint, dim3((t.max_tiles + kCcTiles - 1) / kCcTiles, t.n_cases), dim3(kThreads), 0, s, cases,
             beta, it);
  return hipGetLastError();
}
hipError_t launch_gram(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s) {
  const int pairs = t.max_k * (t.max_k + 1) / 2;
  pty_launch(k_gram, dim3(kGramBlocks * pairs, t.n_cases), dim3(kThreads), 0, s, cases, it);
  return hipGetLastError();
}
hipError_t launch_eig(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s) {
  pty_launch(k_eig, dim3(1, t.n_cases), dim3(64), 0, s, cases, it);
  return hipGetLastError();
}
hipError_t launch_remix(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s) {
  pty_launch(k_remix, dim3(n_probe_blocks(t.n), t.n_cases), dim3(kThreads), 0, s, cases, it);
  return hipGetLastError();
}
hipError_t launch_err_reduce(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s) {
  pty_launch(k_err_reduce, dim3(1, t.n_cases), dim3(kErrThreads), 0, s, cases, it);
  return hipGetLastError();
}
hipError_t launch_pw(const DevParams& p, const DevBufs& d, int copy, hipStream_t s) {
  pty_launch(k_pw, dim3(n_probe_blocks(p.n)), dim3(kThreads), 0, s, p, d, copy);
  return hipGetLastError();
}
hipError_t launch_prepare_amp(const float* inten, float* amp, int n, int n_pos, bool shift, int* bad,
                              double* sum_part, hipStream_t s) {
  pty_launch(k_prepare_amp, dim3(8, n_pos), dim3(kThreads), 0, s, inten, amp, n, shift ? 1 : 0, bad,
                     sum_part);
  return hipGetLastError();
}
__global__ void k_iter_advance(int* it) {
  if (threadIdx.x == 0) *it = *it + 1;
}
__global__ void k_iter_set(int* it, int v) {
  if (threadIdx.x == 0) *it = v;
}
hipError_t launch_iter_advance(int* it, hipStream_t s) {
  pty_launch(k_iter_advance, dim3(1), dim3(64), 0, s, it);
  return hipGetLastError();
}
hipError_t launch_iter_set(int* it, int v, hipStream_t s) {
  pty_launch(k_iter_set, dim3(1), dim3(64), 0, s, it, v);
  return hipGetLastError();
}
hipError_t launch_exit_waves(const DevParams& p, const DevBufs& d, const int* slots, int ns, float2* out,
                             hipStream_t s) {
  pty_launch(k_exit_waves, dim3(n_probe_blocks(p.n), ns), dim3(kThreads), 0, s, p, d, slots, ns, out);
  return hipGetLastError();
}

}  // namespace pty

#include "dft_mfma.hip"
