// HIP kernels (gfx950) of the pc-DM engine: the difference map of ref. [26] with
// the blurred modulus projection (box 1 of Fig. 1) and the complex constraint
// (box 2), as Sec. 4.5 combines them (Fig. 11).
//
// The state is one exit wave psi_nk per scan position n and probe mode k
// (psi[n][k][N][N], complex64) besides the object and probe.  One iteration:
//   overlap projection  (launch_dm_overlap, once per iteration, every position)
//     dm_wmax          per object tile: max over the tile of W(r) = sum_n sum_k |P_k(r - r_n)|^2
//     dm_obj           per object tile: N_O = sum_n sum_k conj(P_k) psi_nk over the positions whose
//                      boxes cover the tile (ascending n), O = (N_O + d maxW O) / (W + d maxW), the
//                      C-bar partials of Eq. (11) and the coverage masks the constraint pass reads
//     (complex_constraint of the ePIE engine, inside windows, over the union of all boxes)
//     dm_probe_part    per segment of positions: sum conj(o_n) psi_nk and sum |o_n|^2 (ascending n)
//     dm_probe_sum     the segments summed in order: N_P,k and V; block maxima of V
//     dm_probe_apply   P_k = (N_P,k + d maxV P_k) / (V + d maxV); sum_k |P_k|^2
//   Fourier step, per batch of positions:
//     dm_rows_fwd      2 z_nk - psi_nk with z_nk = o_n P_k, transform along x
//     fwd_cols, modulus_factor, inv_cols (the ePIE engine's column passes: mode sum,
//                      blur, modulus factor, data error, inverse along y)
//     dm_rows_inv      inverse along x -> psi'_nk; psi_nk <- psi_nk + (psi'_nk - z_nk)
// Every reduction has a fixed order, so results are bitwise reproducible.
#include "kernels_dev.hpp"

namespace pty {

__host__ __device__ __forceinline__ int dm_segments_dev(int n_pos, int seg_len) {
  return (n_pos + seg_len - 1) / seg_len;
}
int dm_segments(int n_pos, int seg_len) { return dm_segments_dev(n_pos, seg_len); }

// Row pass of the Fourier step's input: 2 z_nk - psi_nk with z_nk = o_n P_k (the
// reflection through the overlap projection), transformed along x into X[b][k].
template <int N, bool NEAR>
__global__ __launch_bounds__(kThreads) void k_dm_rows_fwd(const CaseDesc* __restrict__ cases, int beta,
                                                          const int* __restrict__ it) {
  constexpr int L = Cfg<N>::ROWS;
  constexpr int LS = RegShape<N, L>::LOAD_SLOTS;
  constexpr int GX = N / L;
  extern __shared__ float2 sm[];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const int b = blockIdx.x / GX, bx = blockIdx.x % GX;
  if (b >= bt.ns) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N;
  const int y0 = bx * L;
  const int pn = bt.slots[b];
  const int2 rc = d.pos[pn];
  for (int i = threadIdx.x; i < N; i += kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  const int K = p.k, W = p.w_obj;
  float2 o[LS];
  const float2* orow = d.obj + (size_t)(rc.x + y0) * W + rc.y;
  for_load_slots<N, L, false>([&](int s, int line, int pos) { o[s] = orow[line * W + pos]; });
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  const float2* p0 = d.probe + (size_t)y0 * N;
  const float2* s0 = d.psi + ((size_t)pn * K * N + y0) * N;
  float2* x0 = d.X + ((size_t)b * K * N + y0) * N;
  auto gather = [&](int k, float2* v) {
    const float2* pk = p0 + (size_t)k * N * N;
    const float2* sk = s0 + (size_t)k * N * N;
    auto load = [&](int s, int line, int pos) {
      const float2 z = cmul(o[s], pk[line * N + pos]);
      const float2 ps = sk[line * N + pos];
      return make_float2(2.0f * z.x - ps.x, 2.0f * z.y - ps.y);
    };
    fft_gather<N, L, false>(v, load);
  };
  auto store_for = [&](int k) {
    float2* out = x0 + (size_t)k * N * N;
    return [=](int s, int line, int pos, float2 v) { out[line * N + pos] = cscale(v, scale); };
  };
  mode_loop<N, L, false, false, NEAR, false>(K, buf, tw, hn, gather, store_for);
}

// Epilogue of the Fourier step's inverse row pass: psi' -> psi_nk + (psi' - o_n P_k).
template <int N, int SS>
struct DmInvStore {
  float2* sk;          // psi_nk rows of the block
  const float2* pk;    // P_k rows of the block
  const float2* ov;    // box values of the thread's output slots
  float scale;
  float2 pv[SS], sv[SS];
  __device__ __forceinline__ void pre(int s, int line, int pos) {
    pv[s] = pk[line * N + pos];
    sv[s] = sk[line * N + pos];
  }
  __device__ __forceinline__ void operator()(int s, int line, int pos, float2 v) {
    const float2 psi_new = cscale(v, scale);
    const float2 dz = csub(psi_new, cmul(ov[s], pv[s]));
    sk[line * N + pos] = cadd(sv[s], dz);
  }
};

template <int N, bool NEAR>
__global__ __launch_bounds__(kThreads) void k_dm_rows_inv(const CaseDesc* __restrict__ cases, int beta,
                                                          const int* __restrict__ it) {
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
  float2* tw = sm;
  float2* hn = sm + N;
  float2* buf = sm + 2 * N;
  const int y0 = bx * L;
  const int pn = bt.slots[b];
  const int2 rc = d.pos[pn];
  for (int i = threadIdx.x; i < N; i += kThreads) {
    tw[i] = d.tw[i];
    if (NEAR) hn[i] = d.hnear[i];
  }
  const int K = p.k, W = p.w_obj;
  float2 ob[SS];
  const float2* orow = d.obj + (size_t)(rc.x + y0) * W + rc.y;
  for_store_slots<N, L, false>([&](int s, int line, int pos) { ob[s] = orow[line * W + pos]; });
  const float scale = NEAR ? 1.0f / N : rsqrtf((float)N);
  float2* x0 = d.X + ((size_t)b * K * N + y0) * N;
  const float2* p0 = d.probe + (size_t)y0 * N;
  float2* s0 = d.psi + ((size_t)pn * K * N + y0) * N;
  auto gather = [&](int k, float2* v) {
    const float2* fr = x0 + (size_t)k * N * N;
    auto load = [&](int s, int line, int pos) { return fr[line * N + pos]; };
    fft_gather<N, L, false>(v, load);
  };
  auto store_for = [&](int k) {
    DmInvStore<N, SS> st;
    st.sk = s0 + (size_t)k * N * N;
    st.pk = p0 + (size_t)k * N * N;
    st.ov = ob;
    st.scale = scale;
    return st;
  };
  mode_loop<N, L, false, true, NEAR, true>(K, buf, tw, hn, gather, store_for);
}

// Per object tile: the maximum over the tile of W(r) = sum_n sum_k |P_k(r - r_n)|^2
// (copy 0 of the probe-power map) over every position whose box covers it.
__global__ __launch_bounds__(kThreads) void k_dm_wmax(const CaseDesc* __restrict__ cases) {
  __shared__ float red[kThreads / 64];
  const CaseDesc* cs = cases + blockIdx.y;
  const DevParams& p = cs->p;
  const int tile = blockIdx.x;
  if (tile >= tiles_of(p)) return;
  const DevBufsG d = global_bufs(cs->d);
  const int n = p.n, tiles_x = tiles_x_of(p);
  const int r0 = (tile / tiles_x) * kObjTile, c0 = (tile % tiles_x) * kObjTile;
  const int ty = threadIdx.x / kObjTile, tx = threadIdx.x % kObjTile;
  const int lo = d.cov_off[tile], hi = d.cov_off[tile + 1];
  float w[kTilePix];
#pragma unroll
  for (int q = 0; q < kTilePix; ++q) w[q] = 0.f;
  for (int i = lo; i < hi; ++i) {
    const int2 rc = d.pos[d.cov_pos[i]];
    const int xx = c0 + tx - rc.y;
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) {
      const int yy = r0 + ty + q * kTileRowsPerPass - rc.x;
      if ((unsigned)yy < (unsigned)n && (unsigned)xx < (unsigned)n) w[q] += d.pw[yy * n + xx];
    }
  }
  float m = 0.f;
#pragma unroll
  for (int q = 0; q < kTilePix; ++q) m = fmaxf(m, w[q]);
  m = block_max_f(m, red);
  if (threadIdx.x == 0) d.maxw_part[tile] = m;
}

// Per object tile: the object of the overlap projection, O = (N_O + d maxW O) /
// (W + d maxW) with N_O = sum_n sum_k conj(P_k(r - r_n)) psi_nk(r - r_n) gathered
// over the covering positions in ascending order, on the pixels some box covers;
// inside a constraint window also the C-bar sums of Eq. (11) (every box counted)
// and the coverage masks the constraint pass reads.
__global__ __launch_bounds__(kThreads) void k_dm_obj(const CaseDesc* __restrict__ cases, const int* __restrict__ it) {
  __shared__ float red[kThreads / 64];
  __shared__ double2 redd[kThreads / 64];
  __shared__ int s_pn[kThreads];
  __shared__ int2 s_rc[kThreads];
  const CaseDesc* cs = cases + blockIdx.y;
  const DevParams& p = cs->p;
  const int tiles = tiles_of(p);
  const int tile = blockIdx.x;
  if (tile >= tiles) return;
  const DevBufsG d = global_bufs(cs->d);
  const bool cc_sums = (cs->flags[*it] & FLAG_CC) != 0;
  const int n = p.n, K = p.k, tiles_x = tiles_x_of(p);
  const size_t nn = (size_t)n * n;
  const int r0 = (tile / tiles_x) * kObjTile, c0 = (tile % tiles_x) * kObjTile;
  const int ty = threadIdx.x / kObjTile, tx = threadIdx.x % kObjTile;
  const int c = c0 + tx;
  const int lo = d.cov_off[tile], hi = d.cov_off[tile + 1];
  float mw = 0.f;
  for (int i = threadIdx.x; i < tiles; i += kThreads) mw = fmaxf(mw, d.maxw_part[i]);
  float2 ov[kTilePix];
#pragma unroll
  for (int q = 0; q < kTilePix; ++q) {
    const int r = r0 + ty + q * kTileRowsPerPass;
    ov[q] = (r < p.h_obj && c < p.w_obj) ? d.obj[(size_t)r * p.w_obj + c] : make_float2(0.f, 0.f);
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
  // the tile's covering positions (ascending), staged in LDS a chunk at a time so that
  // the gathers below wait on one load each; per pixel the terms are added in the
  // order position, then mode
  for (int c0i = lo; c0i < hi; c0i += kThreads) {
    const int cn = min(kThreads, hi - c0i);
    __syncthreads();  // the previous chunk is no longer read
    if ((int)threadIdx.x < cn) {
      const int pn = d.cov_pos[c0i + threadIdx.x];
      s_pn[threadIdx.x] = pn;
      s_rc[threadIdx.x] = d.pos[pn];
    }
    __syncthreads();
    for (int i = 0; i < cn; ++i) {
      const int pn = s_pn[i];
      const int2 rc = s_rc[i];
      const int xx = c0 + tx - rc.y;
      const float2* ps = d.psi + (size_t)pn * K * nn;
      bool in[kTilePix];
      size_t e[kTilePix];
#pragma unroll
      for (int q = 0; q < kTilePix; ++q) {
        const int yy = r0 + ty + q * kTileRowsPerPass - rc.x;
        in[q] = (unsigned)yy < (unsigned)n && (unsigned)xx < (unsigned)n;
        e[q] = in[q] ? (size_t)yy * n + xx : 0;
        if (in[q]) {
          w[q] += d.pw[e[q]];
          ++mult[q];
        }
      }
      int k = 0;
      for (; k + 2 <= K; k += 2) {  // two modes' loads in flight
        float2 a0[kTilePix], b0[kTilePix], a1[kTilePix], b1[kTilePix];
#pragma unroll
        for (int q = 0; q < kTilePix; ++q) {
          if (!in[q]) continue;
          a0[q] = ps[(size_t)k * nn + e[q]];
          b0[q] = d.probe[(size_t)k * nn + e[q]];
          a1[q] = ps[(size_t)(k + 1) * nn + e[q]];
          b1[q] = d.probe[(size_t)(k + 1) * nn + e[q]];
        }
#pragma unroll
        for (int q = 0; q < kTilePix; ++q)
          if (in[q]) num[q] = cadd(cadd(num[q], cmulc(a0[q], b0[q])), cmulc(a1[q], b1[q]));
      }
      if (k < K) {
#pragma unroll
        for (int q = 0; q < kTilePix; ++q)
          if (in[q]) num[q] = cadd(num[q], cmulc(ps[(size_t)k * nn + e[q]], d.probe[(size_t)k * nn + e[q]]));
      }
    }
  }
  const float maxw = block_max_f(mw, red);
  const float reg = p.dm_reg * maxw;
  float sa = 0.f, sp = 0.f;
#pragma unroll
  for (int q = 0; q < kTilePix; ++q) {
    const int r = r0 + ty + q * kTileRowsPerPass;
    if (!mult[q] || r >= p.h_obj || c >= p.w_obj) continue;
    float2 o = ov[q];
    const float den = w[q] + reg;
    if (den > 0.f) {
      o = make_float2((num[q].x + reg * o.x) / den, (num[q].y + reg * o.y) / den);
      d.obj[(size_t)r * p.w_obj + c] = o;
    }
    if (cc_sums) {
      sa += mult[q] * fabsf(cc_ln_amp(o));
      sp += mult[q] * fabsf(cc_phase(o));
    }
  }
  if (cc_sums) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kTilePix; ++q) {
      const int r = r0 + ty + q * kTileRowsPerPass;
      const unsigned long long m = __ballot(mult[q] > 0 && r < p.h_obj && c < p.w_obj);
      if (lane == 0) {
        unsigned* mk = d.cov_mask + (size_t)tile * kObjTile + 2 * wv + q * kTileRowsPerPass;
        mk[0] = (unsigned)m;
        mk[1] = (unsigned)(m >> 32);
      }
    }
    const double2 t = block_sum_d2((double)sa, (double)sp, redd);
    if (threadIdx.x == 0) d.cc_part[tile] = t;
  }
}

// Probe numerator and weight partial sums over one segment of the positions
// [s L, (s + 1) L) in ascending order, one probe pixel per thread (every mode).
__global__ __launch_bounds__(kThreads) void k_dm_probe_part(const CaseDesc* __restrict__ cases,
                                                            const int* __restrict__ it) {
  const CaseDesc* cs = cases + blockIdx.y;
  if (!(cs->flags[*it] & FLAG_PROBE)) return;
  const DevParams& p = cs->p;
  const int n = p.n, K = p.k;
  const size_t nn = (size_t)n * n;
  const int pblocks = n_probe_blocks_dev(n);
  const int seg = blockIdx.x / pblocks, pb = blockIdx.x % pblocks;
  const int n0 = seg * p.dm_seg_len;
  if (n0 >= p.n_pos) return;
  const int n1 = min(p.n_pos, n0 + p.dm_seg_len);
  const int pix = pb * kThreads + threadIdx.x;
  if (pix >= n * n) return;
  const DevBufsG d = global_bufs(cs->d);
  const int y = pix / n, x = pix - y * n;
  float v = 0.f;
  float2 acc[kMaxModes];
#pragma unroll
  for (int k = 0; k < kMaxModes; ++k) acc[k] = make_float2(0.f, 0.f);
  for (int pn = n0; pn < n1; ++pn) {
    const int2 rc = d.pos[pn];
    const float2 o = d.obj[(size_t)(rc.x + y) * p.w_obj + rc.y + x];
    v += o.x * o.x + o.y * o.y;
    const float2* ps = d.psi + (size_t)pn * K * nn + pix;
#pragma unroll
    for (int k = 0; k < kMaxModes; ++k)
      if (k < K) acc[k] = cadd(acc[k], cmulc(ps[(size_t)k * nn], o));
  }
  d.v_part[(size_t)seg * nn + pix] = v;
#pragma unroll
  for (int k = 0; k < kMaxModes; ++k)
    if (k < K) d.np_part[((size_t)seg * K + k) * nn + pix] = acc[k];
}

// N_P,k and V summed over the segments in ascending order; block maxima of V.
__global__ __launch_bounds__(kThreads) void k_dm_probe_sum(const CaseDesc* __restrict__ cases,
                                                           const int* __restrict__ it) {
  __shared__ float red[kThreads / 64];
  const CaseDesc* cs = cases + blockIdx.y;
  if (!(cs->flags[*it] & FLAG_PROBE)) return;
  const DevParams& p = cs->p;
  const int n = p.n, K = p.k;
  const size_t nn = (size_t)n * n;
  if ((int)blockIdx.x >= n_probe_blocks_dev(n)) return;
  const DevBufsG d = global_bufs(cs->d);
  const int segs = dm_segments_dev(p.n_pos, p.dm_seg_len);
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  float v = 0.f;
  if (pix < n * n) {
    for (int sgi = 0; sgi < segs; ++sgi) v += d.v_part[(size_t)sgi * nn + pix];
    d.V[pix] = v;
    for (int k = 0; k < K; ++k) {
      float2 np = make_float2(0.f, 0.f);
      for (int sgi = 0; sgi < segs; ++sgi) np = cadd(np, d.np_part[((size_t)sgi * K + k) * nn + pix]);
      d.nP[(size_t)k * nn + pix] = np;
    }
  }
  const float m = block_max_f(v, red);
  if (threadIdx.x == 0) d.maxv_part[blockIdx.x] = m;
}

// P_k = (N_P,k + d maxV P_k) / (V + d maxV) and sum_k |P_k|^2 into copy 0 of the
// probe-power map (the next overlap projection's W).
__global__ __launch_bounds__(kThreads) void k_dm_probe_apply(const CaseDesc* __restrict__ cases,
                                                             const int* __restrict__ it) {
  __shared__ float red[kThreads / 64];
  const CaseDesc* cs = cases + blockIdx.y;
  if (!(cs->flags[*it] & FLAG_PROBE)) return;
  const DevParams& p = cs->p;
  const int n = p.n, K = p.k;
  const size_t nn = (size_t)n * n;
  const int pblocks = n_probe_blocks_dev(n);
  if ((int)blockIdx.x >= pblocks) return;
  const DevBufsG d = global_bufs(cs->d);
  float mv = 0.f;
  for (int i = threadIdx.x; i < pblocks; i += kThreads) mv = fmaxf(mv, d.maxv_part[i]);
  const float maxv = block_max_f(mv, red);
  const float reg = p.dm_reg * maxv;
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  if (pix >= n * n) return;
  const float den = d.V[pix] + reg;
  float pw = 0.f;
  for (int k = 0; k < K; ++k) {
    const size_t e = (size_t)k * nn + pix;
    float2 v = d.probe[e];
    if (den > 0.f) {
      const float2 np = d.nP[e];
      v = make_float2((np.x + reg * v.x) / den, (np.y + reg * v.y) / den);
      d.probe[e] = v;
    }
    pw += v.x * v.x + v.y * v.y;
  }
  d.pw[pix] = pw;
}

// psi_nk = o_n P_k for every position (the state the iteration starts from).
__global__ __launch_bounds__(kThreads) void k_dm_init_psi(DevParams p, DevBufs d) {
  const int n = p.n;
  const size_t nn = (size_t)n * n;
  const int pn = blockIdx.y;
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  if (pix >= n * n) return;
  const int2 rc = d.pos[pn];
  const int y = pix / n, x = pix - y * n;
  const float2 o = d.obj[(size_t)(rc.x + y) * p.w_obj + rc.y + x];
  for (int k = 0; k < p.k; ++k)
    d.psi[((size_t)pn * p.k + k) * nn + pix] = cmul(o, d.probe[(size_t)k * nn + pix]);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

template <int N, bool NEAR>
static hipError_t dm_rows_fwd_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  constexpr int L = Cfg<N>::ROWS;
  const size_t sh = sizeof(float2) * (2 * N + Frame<N, L, false>::ELEMS);
  pty_launch(k_dm_rows_fwd<N, NEAR>, dim3((N / L) * t.max_batch, t.n_cases), dim3(kThreads), sh, s, cases, beta, it);
  return hipGetLastError();
}
template <int N, bool NEAR>
static hipError_t dm_rows_inv_t(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  constexpr int L = Cfg<N>::ROWS;
  const size_t sh = sizeof(float2) * (2 * N + Frame<N, L, false>::ELEMS);
  pty_launch(k_dm_rows_inv<N, NEAR>, dim3((N / L) * t.max_batch, t.n_cases), dim3(kThreads), sh, s, cases, beta, it);
  return hipGetLastError();
}

hipError_t launch_dm_rows_fwd(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  switch (t.n) {
#define PTY_CASE(N) \
  case N:           \
    return t.near_field ? dm_rows_fwd_t<N, true>(cases, t, beta, it, s) : dm_rows_fwd_t<N, false>(cases, t, beta, it, s);
    PTY_FOR_EACH_N(PTY_CASE)
#undef PTY_CASE
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_dm_rows_inv(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  switch (t.n) {
#define PTY_CASE(N) \
  case N:           \
    return t.near_field ? dm_rows_inv_t<N, true>(cases, t, beta, it, s) : dm_rows_inv_t<N, false>(cases, t, beta, it, s);
    PTY_FOR_EACH_N(PTY_CASE)
#undef PTY_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_dm_overlap(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s) {
  pty_launch(k_dm_wmax, dim3(t.max_tiles, t.n_cases), dim3(kThreads), 0, s, cases);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  pty_launch(k_dm_obj, dim3(t.max_tiles, t.n_cases), dim3(kThreads), 0, s, cases, it);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = launch_constraint(cases, t, 0, it, s);
  if (e != hipSuccess) return e;
  const int pblocks = n_probe_blocks_dev(t.n);
  pty_launch(k_dm_probe_part, dim3(pblocks * t.max_dm_segments, t.n_cases), dim3(kThreads), 0, s, cases, it);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  pty_launch(k_dm_probe_sum, dim3(pblocks, t.n_cases), dim3(kThreads), 0, s, cases, it);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  pty_launch(k_dm_probe_apply, dim3(pblocks, t.n_cases), dim3(kThreads), 0, s, cases, it);
  return hipGetLastError();
}

hipError_t launch_dm_init_psi(const DevParams& p, const DevBufs& d, hipStream_t s) {
  pty_launch(k_dm_init_psi, dim3(n_probe_blocks_dev(p.n), p.n_pos), dim3(kThreads), 0, s, p, d);
  return hipGetLastError();
}

}  // namespace pty
