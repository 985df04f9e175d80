// Workgroup-cooperative 1D FFTs of complex64 lines held in LDS (gfx950).
//
// A line of N = 2^a 3^b points is transformed by a sequence of mixed-radix
// Stockham autosort stages (radix 2, 3, 4 or 8).  Stage s with radix R and
// current sub-transform length NS performs N/R butterflies per line:
//   v[r] = src[j + r N/R] * w^(r (j mod NS)),  w = exp(-+2 pi i / (NS R))
//   v    = DFT_R(v)
//   dst[(j / NS) NS R + (j mod NS) + r NS] = v[r]
// The butterflies of all lines in a stage are spread over the 256 threads of
// the workgroup; a stage reads its inputs into registers, synchronises, and
// writes its outputs back in place, so one LDS buffer per line suffices.
// Twiddles come from an LDS table tw[m] = exp(-2 pi i m / N) built on the
// host in double precision.  Transforms are unnormalised; callers scale.
#pragma once

#include <hip/hip_runtime.h>

namespace pty {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 conjc(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    // X1 = v0 - (v1+v2)/2 -+ i (sqrt3/2)(v1-v2),  X2 = v0 - (v1+v2)/2 +- i (sqrt3/2)(v1-v2)
    const float s3 = 0.86602540378443864676f;
    float2 t1 = cadd(v[1], v[2]);
    float2 t2 = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    float2 r = mul_mi<INV>(cscale(t2, s3));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]);
    float2 t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]);
    float2 t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    // split into even/odd radix-4 DFTs, then combine with w8^k
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    const float h = 0.70710678118654752440f;
    // w8^1 = (1 -+ i)/sqrt2, w8^2 = -+i, w8^3 = (-1 -+ i)/sqrt2
    float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                    : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    float2 o2 = mul_mi<INV>(o[2]);
    float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                    : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// One in-place Stockham stage over NL lines: every thread first gathers the
// inputs of its butterflies into registers, the workgroup synchronises, then
// the outputs are written back into the same buffer.  blockDim.x must be 256.
template <int N, int NL, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_stage(float2* __restrict__ buf, int ld, const float2* __restrict__ tw) {
  constexpr int M = N / R;
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
  float2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      const int line = f / M;
      const int j = f - line * M;
      const float2* s = buf + line * ld;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = s[j + r * M];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      const int line = f / M;
      const int j = f - line * M;
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw[r * k * (N / (NS * R))];
          v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
        }
      }
      Dft<R, INV>::run(v[i]);
      float2* d = buf + line * ld;
      const int idx = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) d[idx + r * NS] = v[i][r];
    }
  }
  __syncthreads();
}

template <int N, int NL, bool INV, int NS, int R, int... Rest>
__device__ __forceinline__ void run_stages(float2* buf, int ld, const float2* tw) {
  stockham_stage<N, NL, R, NS, INV>(buf, ld, tw);
  if constexpr (sizeof...(Rest) > 0) run_stages<N, NL, INV, NS * R, Rest...>(buf, ld, tw);
}

// Transform NL lines of length N (line stride `ld` float2) in place in LDS.
// Must be called by all 256 threads of the workgroup with the data already
// visible (after a barrier); ends with a barrier.  Unnormalised.
template <int N, int NL, bool INV>
__device__ __forceinline__ void fft_lines(float2* buf, int ld, const float2* tw) {
  if constexpr (N == 8) run_stages<N, NL, INV, 1, 8>(buf, ld, tw);
  else if constexpr (N == 16) run_stages<N, NL, INV, 1, 4, 4>(buf, ld, tw);
  else if constexpr (N == 24) run_stages<N, NL, INV, 1, 3, 8>(buf, ld, tw);
  else if constexpr (N == 32) run_stages<N, NL, INV, 1, 8, 4>(buf, ld, tw);
  else if constexpr (N == 48) run_stages<N, NL, INV, 1, 3, 4, 4>(buf, ld, tw);
  else if constexpr (N == 64) run_stages<N, NL, INV, 1, 8, 8>(buf, ld, tw);
  else if constexpr (N == 96) run_stages<N, NL, INV, 1, 3, 8, 4>(buf, ld, tw);
  else if constexpr (N == 128) run_stages<N, NL, INV, 1, 8, 4, 4>(buf, ld, tw);
  else if constexpr (N == 192) run_stages<N, NL, INV, 1, 3, 8, 8>(buf, ld, tw);
  else if constexpr (N == 256) run_stages<N, NL, INV, 1, 4, 4, 4, 4>(buf, ld, tw);
  else if constexpr (N == 384) run_stages<N, NL, INV, 1, 3, 8, 4, 4>(buf, ld, tw);
  else if constexpr (N == 512) run_stages<N, NL, INV, 1, 8, 8, 8>(buf, ld, tw);
  else if constexpr (N == 768) run_stages<N, NL, INV, 1, 3, 4, 8, 8>(buf, ld, tw);
  else if constexpr (N == 1024) run_stages<N, NL, INV, 1, 4, 4, 8, 8>(buf, ld, tw);
  else static_assert(N == 8, "unsupported FFT length");
}

// ---------------------------------------------------------------------------
// Register-fed transforms: the first stage reads its inputs through a Load
// functor (global memory, with any elementwise prologue fused) and the last
// stage hands its outputs to a Store functor, so only the middle stages use
// LDS.  Lines are laid out in LDS by Frame<N, NL, LF>:
//   LF = false: line-major   (a row pass: thread butterflies run along a line)
//   LF = true : position-major (a column pass: consecutive threads take
//               consecutive lines, i.e. adjacent columns of the frame, so
//               global accesses are coalesced row segments)
// Load(slot, line, pos) -> float2 and Store(slot, line, pos, float2) receive a
// per-thread slot index (butterfly i, leg r) that is the same for every call
// of the same transform shape, so callers can keep per-element registers.
// ---------------------------------------------------------------------------

template <int N, int NL, bool LF>
struct Frame {
  static constexpr int LD = LF ? NL + 1 : N + 1;
  static constexpr int ELEMS = LF ? N * LD : NL * LD;
  __device__ __forceinline__ static int lidx(int line, int pos) { return LF ? pos * LD + line : line * LD + pos; }
  template <int M>
  __device__ __forceinline__ static void map(int f, int& line, int& j) {
    if (LF) {
      line = f % NL;
      j = f / NL;
    } else {
      line = f / M;
      j = f - line * M;
    }
  }
};

template <int N, int R>
struct StageShape {
  static constexpr int M = N / R;
};

template <int N, int NL, int R>
struct Slots {
  static constexpr int TOT = NL * (N / R);
  static constexpr int NB = (TOT + 255) / 256;
  static constexpr int COUNT = NB * R;
};

template <int N, int NL, bool LF, bool INV, int R, int NS>
__device__ __forceinline__ void mid_stage(float2* buf, const float2* __restrict__ tw) {
  using F = Frame<N, NL, LF>;
  constexpr int M = N / R;
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
  float2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      int line, j;
      F::template map<M>(f, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[F::lidx(line, j + r * M)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      int line, j;
      F::template map<M>(f, line, j);
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[r * k * (N / (NS * R))];
        v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
      }
      Dft<R, INV>::run(v[i]);
      const int idx = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[F::lidx(line, idx + r * NS)] = v[i][r];
    }
  }
  __syncthreads();
}

// Last stage: inputs from LDS, outputs to Store at positions j + r N/R.
// STORE_LDS: the store writes back into `buf`, so all reads finish first.
template <int N, int NL, bool LF, bool INV, bool STORE_LDS, int R, int NS, class Store>
__device__ __forceinline__ void last_stage(float2* buf, const float2* __restrict__ tw, Store& store) {
  using F = Frame<N, NL, LF>;
  constexpr int M = N / R;
  static_assert(NS == M, "last stage");
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
  float2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      int line, j;
      F::template map<M>(f, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[F::lidx(line, j + r * M)];
    }
  }
  if (STORE_LDS) __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      int line, j;
      F::template map<M>(f, line, j);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[r * j * (N / (NS * R))];
        v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
      }
      Dft<R, INV>::run(v[i]);
#pragma unroll
      for (int r = 0; r < R; ++r) store(i * R + r, line, j + r * M, v[i][r]);
    }
  }
}

template <int N, int NL, bool LF, bool INV, bool STORE_LDS, class Store, int NS, int R, int... Rest>
__device__ __forceinline__ void stages_from_lds(float2* buf, const float2* tw, Store& store) {
  if constexpr (sizeof...(Rest) == 0) {
    last_stage<N, NL, LF, INV, STORE_LDS, R, NS>(buf, tw, store);
  } else {
    mid_stage<N, NL, LF, INV, R, NS>(buf, tw);
    stages_from_lds<N, NL, LF, INV, STORE_LDS, Store, NS * R, Rest...>(buf, tw, store);
  }
}

// First stage (radix R0) fed by Load, remaining stages through LDS, last to Store.
// LOAD_LDS: the loads read `buf`, so they all finish before stage 0 writes it.
// On return the last stage's LDS reads are done but no barrier follows; a
// caller that rewrites `buf` afterwards must synchronise first.
template <int N, int NL, bool LF, bool INV, bool LOAD_LDS, bool STORE_LDS, class Load, class Store, int R0,
          int... Rs>
__device__ __forceinline__ void fft_reg_impl(float2* buf, const float2* __restrict__ tw, Load& load, Store& store) {
  using F = Frame<N, NL, LF>;
  constexpr int M = N / R0;
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
  float2 v[NB][R0];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      int line, j;
      F::template map<M>(f, line, j);
#pragma unroll
      for (int r = 0; r < R0; ++r) v[i][r] = load(i * R0 + r, line, j + r * M);
    }
  }
  if constexpr (sizeof...(Rs) == 0) {
    if (LOAD_LDS && STORE_LDS) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int f = threadIdx.x + i * 256;
      if (TOT % 256 == 0 || f < TOT) {
        int line, j;
        F::template map<M>(f, line, j);
        Dft<R0, INV>::run(v[i]);
#pragma unroll
        for (int r = 0; r < R0; ++r) store(i * R0 + r, line, j + r * M, v[i][r]);
      }
    }
  } else {
    if (LOAD_LDS) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int f = threadIdx.x + i * 256;
      if (TOT % 256 == 0 || f < TOT) {
        int line, j;
        F::template map<M>(f, line, j);
        Dft<R0, INV>::run(v[i]);
#pragma unroll
        for (int r = 0; r < R0; ++r) buf[F::lidx(line, j * R0 + r)] = v[i][r];
      }
    }
    __syncthreads();
    stages_from_lds<N, NL, LF, INV, STORE_LDS, Store, R0, Rs...>(buf, tw, store);
  }
}

// Radix plans (first radix, then the rest); the first and last radices set
// the Load and Store slot shapes: FirstR<N>, LastR<N>.
template <int N> struct Plan;
template <> struct Plan<8> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<8, NL, LF, INV, LL, SL, L, S, 8>(b, t, l, s); } static constexpr int FIRST = 8, LAST = 8; };
template <> struct Plan<16> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<16, NL, LF, INV, LL, SL, L, S, 4, 4>(b, t, l, s); } static constexpr int FIRST = 4, LAST = 4; };
template <> struct Plan<24> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<24, NL, LF, INV, LL, SL, L, S, 3, 8>(b, t, l, s); } static constexpr int FIRST = 3, LAST = 8; };
template <> struct Plan<32> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<32, NL, LF, INV, LL, SL, L, S, 8, 4>(b, t, l, s); } static constexpr int FIRST = 8, LAST = 4; };
template <> struct Plan<48> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<48, NL, LF, INV, LL, SL, L, S, 3, 4, 4>(b, t, l, s); } static constexpr int FIRST = 3, LAST = 4; };
template <> struct Plan<64> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<64, NL, LF, INV, LL, SL, L, S, 8, 8>(b, t, l, s); } static constexpr int FIRST = 8, LAST = 8; };
template <> struct Plan<96> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<96, NL, LF, INV, LL, SL, L, S, 3, 8, 4>(b, t, l, s); } static constexpr int FIRST = 3, LAST = 4; };
template <> struct Plan<128> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<128, NL, LF, INV, LL, SL, L, S, 8, 4, 4>(b, t, l, s); } static constexpr int FIRST = 8, LAST = 4; };
template <> struct Plan<192> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<192, NL, LF, INV, LL, SL, L, S, 3, 8, 8>(b, t, l, s); } static constexpr int FIRST = 3, LAST = 8; };
template <> struct Plan<256> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<256, NL, LF, INV, LL, SL, L, S, 4, 4, 4, 4>(b, t, l, s); } static constexpr int FIRST = 4, LAST = 4; };
template <> struct Plan<384> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<384, NL, LF, INV, LL, SL, L, S, 3, 8, 4, 4>(b, t, l, s); } static constexpr int FIRST = 3, LAST = 4; };
template <> struct Plan<512> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<512, NL, LF, INV, LL, SL, L, S, 8, 8, 8>(b, t, l, s); } static constexpr int FIRST = 8, LAST = 8; };
template <> struct Plan<768> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<768, NL, LF, INV, LL, SL, L, S, 3, 4, 8, 8>(b, t, l, s); } static constexpr int FIRST = 3, LAST = 8; };
template <> struct Plan<1024> { template <int NL, bool LF, bool INV, bool LL, bool SL, class L, class S> __device__ static void run(float2* b, const float2* t, L& l, S& s) { fft_reg_impl<1024, NL, LF, INV, LL, SL, L, S, 4, 4, 8, 8>(b, t, l, s); } static constexpr int FIRST = 4, LAST = 8; };

// Enumerate this thread's Load (first-stage) or Store (last-stage) slots:
// fn(slot, line, pos) for every element the transform will hand it.
template <int N, int NL, bool LF, int R, class Fn>
__device__ __forceinline__ void for_slots(Fn&& fn) {
  using F = Frame<N, NL, LF>;
  constexpr int M = N / R;
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = threadIdx.x + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      int line, j;
      F::template map<M>(f, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) fn(i * R + r, line, j + r * M);
    }
  }
}
template <int N, int NL, bool LF, class Fn>
__device__ __forceinline__ void for_load_slots(Fn&& fn) {
  for_slots<N, NL, LF, Plan<N>::FIRST>(fn);
}
template <int N, int NL, bool LF, class Fn>
__device__ __forceinline__ void for_store_slots(Fn&& fn) {
  for_slots<N, NL, LF, Plan<N>::LAST>(fn);
}

// Register-fed transform of NL lines of length N.  Load and Store see slots
// 0 .. LoadSlots-1 and 0 .. StoreSlots-1 respectively.
template <int N, int NL, bool LF, bool INV, bool LOAD_LDS = false, bool STORE_LDS = false, class Load, class Store>
__device__ __forceinline__ void fft_reg(float2* buf, const float2* tw, Load& load, Store& store) {
  Plan<N>::template run<NL, LF, INV, LOAD_LDS, STORE_LDS>(buf, tw, load, store);
}
template <int N, int NL>
struct RegShape {
  static constexpr int LOAD_SLOTS = Slots<N, NL, Plan<N>::FIRST>::COUNT;
  static constexpr int STORE_SLOTS = Slots<N, NL, Plan<N>::LAST>::COUNT;
};

}  // namespace pty
