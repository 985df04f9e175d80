// Device-side building blocks shared by the kernel sources of the library:
// the launch helper, tile shapes, fixed-order block reductions, global-pointer
// views of the case descriptor, batch lookup, the per-mode transform loops of
// the row and column passes, and the object-tile geometry.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "fft_lds.hpp"
#include "kernels.hpp"

#include <hip/hip_ext.h>

namespace pty {

// Every kernel of this library is launched through here (see LaunchEvents).
template <class... P, class... A>
static inline void pty_launch(void (*kernel)(P...), dim3 grid, dim3 block, size_t shmem, hipStream_t s, A... args) {
  LaunchEvents& ev = launch_events();
  if (ev.stop) {
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shmem, s, ev.start, ev.stop, 0u, static_cast<P>(args)...);
    ev.start = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, static_cast<P>(args)...);
  }
}

constexpr int kThreads = 256;

constexpr int largest_divisor_le(int n, int cap) {
  int best = 1;
  for (int d = 1; d <= n && d <= cap; ++d)
    if (n % d == 0) best = d;
  return best;
}

// Lines per block: ~4096 elements (16 per thread) for row blocks; column blocks
// take COLS columns (variant 1) or half / twice as many (variants 0 / 2, chosen
// by the autotuner when they divide N and stay within 64 columns).
template <int N>
struct Cfg {
  static constexpr int ROWS = largest_divisor_le(N, 4096 / N < 1 ? 1 : 4096 / N);
  static constexpr int CCAP = 4096 / N < 4 ? 4 : (4096 / N > 64 ? 64 : 4096 / N);
  static constexpr int COLS = largest_divisor_le(N, CCAP);
  static_assert(N % ROWS == 0 && N % COLS == 0, "tile must divide N");
};
// Rows per block of the modulus-factor pass: half a row-pass block, so that the
// pass (whole rows, a short blur and the factor per element) launches twice the
// workgroups and hides its latency with more waves.
template <int N>
struct FactorRows {
  static constexpr int R = Cfg<N>::ROWS >= 2 ? Cfg<N>::ROWS / 2 : 1;
  static_assert(N % R == 0, "row block must divide N");
};
template <int N, int V>
struct ColW {
  static constexpr int W0 = V == 0 ? Cfg<N>::COLS / 2 : (V == 2 ? Cfg<N>::COLS * 2 : Cfg<N>::COLS);
  static constexpr bool VALID = W0 >= 1 && W0 <= 64 && N % W0 == 0;
  static constexpr int C = VALID ? W0 : Cfg<N>::COLS;
};

// The complex constraint's per-pixel quantities (Eq. 9-11): the logarithm of the
// amplitude floored at 1e-20, the principal phase, and Eq. (9)-(10),
//   A^c = exp[(1 - a1) ln A + a1 C phi],  phi^c = (1 - a2) phi + a2 ln A / C,
// with the hardware base-2 logarithm, exponential, sine and cosine (v_log_f32,
// v_exp_f32, v_sin_f32, v_cos_f32: about 1e-6 relative on these arguments; the
// phase is reduced to [-pi, pi] first, inside the sine's valid range).
__device__ __forceinline__ float cc_ln_amp(float2 o) {
  return __logf(fmaxf(sqrtf(o.x * o.x + o.y * o.y), 1e-20f));
}
__device__ __forceinline__ float cc_phase(float2 o) { return atan2f(o.y, o.x); }
__device__ __forceinline__ float2 cc_apply_lp(float lna, float phi, float cbar, float inv_c, float a1, float a2) {
  const float ac = __expf((1.0f - a1) * lna + a1 * cbar * phi);
  float pc = (1.0f - a2) * phi + a2 * inv_c * lna;
  if (fabsf(pc) > 3.14159265f) pc -= 6.28318531f * rintf(pc * 0.159154943f);
  float sn, cs;
  __sincosf(pc, &sn, &cs);
  return make_float2(ac * cs, ac * sn);
}
__device__ __forceinline__ float2 cc_apply(float2 o, float cbar, float inv_c, float a1, float a2) {
  return cc_apply_lp(cc_ln_amp(o), cc_phase(o), cbar, inv_c, a1, a2);
}

// Block reductions in a fixed order: butterfly over the 64 lanes of each wave,
// then the 4 wave results in order.  `sh` holds kThreads / 64 entries.
__device__ __forceinline__ double block_sum_d(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Two sums at once, each in the order of block_sum_d (same results, half the barriers).
__device__ __forceinline__ double2 block_sum_d2(double a, double b, double2* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = make_double2(a, b);
  __syncthreads();
  return make_double2((sh[0].x + sh[1].x) + (sh[2].x + sh[3].x), (sh[0].y + sh[1].y) + (sh[2].y + sh[3].y));
}

__device__ __forceinline__ float block_max_f(float v, float* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

__host__ __device__ __forceinline__ int n_probe_blocks_dev(int n) { return (n * n + kThreads - 1) / kThreads; }

// Pointers read from the case descriptor are generic.  Held as address-space-1
// (global) pointers and converted back at each use, they let the compiler emit
// global rather than flat loads and stores, which carry no ordering against
// LDS traffic.
#define PTY_AS1 __attribute__((address_space(1)))
template <class T>
struct GPtr {
  PTY_AS1 T* p;
  __device__ __forceinline__ operator T*() const { return (T*)p; }
  __device__ __forceinline__ T* operator+(size_t i) const { return (T*)p + i; }
  __device__ __forceinline__ T& operator[](size_t i) const { return ((T*)p)[i]; }
};
template <class T>
__device__ __forceinline__ GPtr<T> as_global(T* ptr) {
  return GPtr<T>{(PTY_AS1 T*)ptr};
}
struct DevBufsG {
  GPtr<float2> obj, probe;
  GPtr<float> pw;
  GPtr<const float> amp;
  GPtr<const int2> pos;
  GPtr<const float2> tw, hnear;
  GPtr<float2> X;
  GPtr<float> q;
  GPtr<float2> dO, nP;
  GPtr<float> V, maxv_part, maxw_part;
  GPtr<double> err_part;
  GPtr<double2> cc_part, gram_part;
  GPtr<unsigned> cov_mask;
  GPtr<float2> psi;
  GPtr<const int> cov_off, cov_pos;
  GPtr<float2> np_part;
  GPtr<float> v_part;
  GPtr<float2> vmix;
  GPtr<double> eig;
  GPtr<float2> lsq_do, lsq_dp, lsq_pdp;
  GPtr<float> lsq_dp2;
  GPtr<double> lsq_part;
  GPtr<float> lsq_ab, lsq_steps;
};
__device__ __forceinline__ DevBufsG global_bufs(const DevBufs& in) {
  DevBufsG d;
  d.obj = as_global(in.obj);
  d.probe = as_global(in.probe);
  d.pw = as_global(in.pw);
  d.amp = as_global(in.amp);
  d.pos = as_global(in.pos);
  d.tw = as_global(in.tw);
  d.hnear = as_global(in.hnear);
  d.X = as_global(in.X);
  d.q = as_global(in.q);
  d.dO = as_global(in.dO);
  d.nP = as_global(in.nP);
  d.V = as_global(in.V);
  d.maxv_part = as_global(in.maxv_part);
  d.maxw_part = as_global(in.maxw_part);
  d.err_part = as_global(in.err_part);
  d.cc_part = as_global(in.cc_part);
  d.cov_mask = as_global(in.cov_mask);
  d.psi = as_global(in.psi);
  d.cov_off = as_global(in.cov_off);
  d.cov_pos = as_global(in.cov_pos);
  d.np_part = as_global(in.np_part);
  d.v_part = as_global(in.v_part);
  d.gram_part = as_global(in.gram_part);
  d.vmix = as_global(in.vmix);
  d.eig = as_global(in.eig);
  d.lsq_do = as_global(in.lsq_do);
  d.lsq_dp = as_global(in.lsq_dp);
  d.lsq_pdp = as_global(in.lsq_pdp);
  d.lsq_dp2 = as_global(in.lsq_dp2);
  d.lsq_part = as_global(in.lsq_part);
  d.lsq_ab = as_global(in.lsq_ab);
  d.lsq_steps = as_global(in.lsq_steps);
  return d;
}
struct DebugPtrsG {
  GPtr<float2> psi_new, n_obj;
  GPtr<float> w_obj, factor;
};
__device__ __forceinline__ DebugPtrsG global_dbg(const DebugPtrs& in) {
  DebugPtrsG g;
  g.psi_new = as_global(in.psi_new);
  g.n_obj = as_global(in.n_obj);
  g.w_obj = as_global(in.w_obj);
  g.factor = as_global(in.factor);
  return g;
}

// The batch a block works on: case blockIdx.y of the table, batch `beta` of
// iteration `it`.  False when the case has no such batch.
struct Batch {
  const CaseDesc* cs;
  const int* slots;
  int ns;
  int flags;
};

__device__ __forceinline__ bool open_batch(const CaseDesc* cases, int beta, const int* it_ptr, Batch& bt) {
  const int it = *it_ptr;
  bt.cs = cases + blockIdx.y;
  const int nb = bt.cs->n_batches;
  if (beta >= nb) return false;
  const int np = bt.cs->n_pos, B = bt.cs->batch;
  bt.slots = bt.cs->order + (size_t)it * np + (size_t)beta * B;
  bt.ns = min(B, np - beta * B);
  bt.flags = bt.cs->flags[it];
  return true;
}

// Copy of the probe-power map that batch `beta` reads: FLAG_PW_ODD gives the
// copy of the iteration's first batch; batches that update the probe alternate
// (each writes the copy the next one reads); without probe update all read one.
__device__ __forceinline__ int pw_copy(int flags, int beta) {
  return ((flags & FLAG_PW_ODD) ? 1 : 0) ^ ((flags & FLAG_PROBE) ? (beta & 1) : 0);
}

template <class T, class = void>
struct HasPre : std::false_type {};
template <class T>
struct HasPre<T, std::void_t<decltype(&T::pre)>> : std::true_type {};
template <class T, class = void>
struct HasPost : std::false_type {};
template <class T>
struct HasPost<T, std::void_t<decltype(&T::post)>> : std::true_type {};

// One 1D pass over the K modes of a block's lines, with the next mode's inputs
// gathered while the current mode is in its LDS stages.  gather(k, v) fills the
// first-stage registers of mode k; store_for(k) returns the Store functor of mode
// k.  NEAR: each pass is F^-1 h F (or F^-1 conj(h) F when CONJ), the transfer
// function applied between the two transforms in LDS.  A Store functor with a
// post() member has it called by every thread once the mode's outputs are all
// handed over (before the synchronisation that ends the mode).
template <int N, int NL, bool LF, bool INV, bool NEAR, bool CONJ, class Gather, class StoreFor>
__device__ __forceinline__ void mode_loop(int K, float2* buf, const float2* tw, const float2* hn, Gather& gather,
                                          StoreFor& store_for) {
  using F = Frame<N, NL, LF>;
  constexpr bool SINGLE = RegShape<N, NL>::SINGLE;
  float2 v[RegShape<N, NL>::LOAD_SLOTS];
  gather(0, v);
  for (int k = 0; k < K; ++k) {
    auto store = store_for(k);
    // stores whose epilogue reads other arrays fetch them here, all at once and
    // before the transform, instead of one load per output behind each store
    if constexpr (HasPre<decltype(store)>::value)
      for_store_slots<N, NL, LF>([&](int s, int line, int pos) { store.pre(s, line, pos); });
    if (!NEAR) {
      fft_first<N, NL, LF, INV>(v, buf);
      if (!SINGLE && k + 1 < K) gather(k + 1, v);
      fft_rest<N, NL, LF, INV>(v, buf, tw, store);
      if (SINGLE && k + 1 < K) gather(k + 1, v);
    } else {
      auto to_lds = [&](int s, int line, int pos, float2 x) {
        buf[F::lidx(line, pos)] = CONJ ? cmulc(x, hn[pos]) : cmul(x, hn[pos]);
      };
      auto from_lds = [&](int s, int line, int pos) { return buf[F::lidx(line, pos)]; };
      fft_first<N, NL, LF, false>(v, buf);
      if (!SINGLE && k + 1 < K) gather(k + 1, v);
      fft_rest<N, NL, LF, false, true>(v, buf, tw, to_lds);
      if (SINGLE && k + 1 < K) gather(k + 1, v);
      __syncthreads();
      fft_reg<N, NL, LF, true, true, false>(buf, tw, from_lds, store);
    }
    if constexpr (HasPost<decltype(store)>::value) store.post();
    __syncthreads();
  }
}

// Far-field inverse column pass that recomputes its input: per mode, the
// forward transform of the row-transformed frame (what the forward column pass
// computed, scaled by `fscale`) goes to LDS instead of global memory, and the
// inverse transform gathers it from there through `scale_in(slot, x)` (the
// modulus factor).  Same operations, in the same order, as storing the forward
// result to global memory and reading it back.
template <int N, int NL, class Gather, class ScaleIn, class StoreFor>
__device__ __forceinline__ void mode_loop_refwd(int K, float2* buf, const float2* tw, float fscale, Gather& gather,
                                                ScaleIn& scale_in, StoreFor& store_for) {
  using F = Frame<N, NL, true>;
  constexpr bool SINGLE = RegShape<N, NL>::SINGLE;
  float2 v[RegShape<N, NL>::LOAD_SLOTS];
  auto to_lds = [&](int s, int line, int pos, float2 x) { buf[F::lidx(line, pos)] = cscale(x, fscale); };
  auto from_lds = [&](int s, int line, int pos) { return scale_in(s, buf[F::lidx(line, pos)]); };
  gather(0, v);
  for (int k = 0; k < K; ++k) {
    auto store = store_for(k);
    fft_first<N, NL, true, false>(v, buf);
    if (!SINGLE && k + 1 < K) gather(k + 1, v);
    fft_rest<N, NL, true, false, true>(v, buf, tw, to_lds);
    if (SINGLE && k + 1 < K) gather(k + 1, v);
    __syncthreads();
    fft_reg<N, NL, true, true, true, false>(buf, tw, from_lds, store);
    __syncthreads();
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin (XCD = block index mod 8),
// each with its own L2.  Column tiles narrower than a 128-byte line (C < 16)
// share every line with their neighbour, so tiles 2m and 2m + 1 go to blocks that
// land on the same XCD in consecutive rounds: the second half of each line is an
// L2 hit instead of a second HBM fetch.  paired_tile is a permutation of each
// group of 16 block indices; launches round their grids up to 16 blocks.
__device__ __forceinline__ int paired_tile(int g) { return 2 * ((g >> 4) * 8 + (g & 7)) + ((g >> 3) & 1); }
static inline int paired_blocks(int tiles) { return (tiles + 15) / 16 * 16; }

// Mode-parallel launches (MP) give every (slot, line block, mode) its own
// workgroup.  The modes of one (slot, line block) are numbered g, g + 8,
// g + 16, ...: they land on the same XCD one after another and share its L2 for
// the inputs they have in common; the u-th tile an XCD receives is paired with
// its neighbour as in paired_tile.
__device__ __forceinline__ void mp_decode(int g, int km, int& tile, int& k0) {
  const int r = g >> 3;
  k0 = r % km;
  const int u = r / km;
  tile = 2 * ((u >> 1) * 8 + (g & 7)) + (u & 1);
}

__device__ __forceinline__ int wrap(int t, int n) {
  t += (t < 0) ? n : 0;
  return t - ((t >= n) ? n : 0);
}

__host__ __device__ __forceinline__ int tiles_x_of(const DevParams& p) { return (p.w_obj + kObjTile - 1) / kObjTile; }
__host__ __device__ __forceinline__ int tiles_of(const DevParams& p) {
  return tiles_x_of(p) * ((p.h_obj + kObjTile - 1) / kObjTile);
}

// Pixels of a 32 x 32 object tile handled by one thread: rows r0 + ty + 8q, column c0 + tx.
constexpr int kTileRowsPerPass = kThreads / kObjTile;
constexpr int kTilePix = kObjTile * kObjTile / kThreads;

// The frame sides the library is built for.
#define PTY_FOR_EACH_N(MACRO) \
  MACRO(8) MACRO(16) MACRO(24) MACRO(32) MACRO(48) MACRO(64) MACRO(96) MACRO(128) MACRO(192) MACRO(256) \
  MACRO(384) MACRO(512) MACRO(768) MACRO(1024)

}  // namespace pty
