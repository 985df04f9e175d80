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

#include <cmath>

// No implicit multiply-add fusion in any code that includes this header: the
// fused operations are the explicit fmaf calls below, so every instantiation
// of a kernel (tile widths, serial or mode-parallel launches, groups) rounds
// exactly alike and their results agree bitwise.
#pragma clang fp contract(off)

namespace pty {

__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
__host__ __device__ __forceinline__ float2 conjc(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// The thread's index within its 256-thread group: a workgroup of 512 threads runs
// two independent transforms, one per half, each on its own LDS buffer (every
// synchronisation is still workgroup-wide, so both halves take the same path).
__device__ __forceinline__ int fft_tid() { return threadIdx.x & 255; }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
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
  __host__ __device__ __forceinline__ static void run(float2* v) {
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
  __host__ __device__ __forceinline__ static void run(float2* v) {
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

template <bool INV>
struct Dft<16, INV> {
  // 16 = 4 x 4: radix-4 DFTs over n1 for each n2, internal twiddles w16^(n2 k1),
  // radix-4 DFTs over n2 for each k1; output index k1 + 4 k2.
  __host__ __device__ __forceinline__ static float2 w16(float2 a, int m) {
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
    const float sg = INV ? 1.0f : -1.0f;  // exp(sg * 2 pi i m / 16)
    switch (m) {
      case 1: return cmul(a, make_float2(c1, sg * s1));
      case 2: return make_float2(h * (a.x - sg * a.y), h * (a.y + sg * a.x));
      case 3: return cmul(a, make_float2(s1, sg * c1));
      case 4: return mul_mi<INV>(a);
      case 6: return make_float2(-h * (a.x + sg * a.y), h * (sg * a.x - a.y));
      case 9: return cmul(a, make_float2(-c1, -sg * s1));
      default: return a;
    }
  }
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = (n2 && k1) ? w16(t[k1], n2 * k1) : t[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// One in-place Stockham stage over NL lines: every thread first gathers the
// inputs of its butterflies into registers, the workgroup synchronises, then
// the outputs are written back into the same buffer.  256 threads per transform.
template <int N, int NL, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_stage(float2* __restrict__ buf, int ld, const float2* __restrict__ tw) {
  constexpr int M = N / R;
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
  float2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = fft_tid() + i * 256;
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
    const int f = fft_tid() + i * 256;
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
// Register-fed transforms: the first stage takes its inputs from registers
// that a Load functor filled (global memory, with any elementwise prologue
// fused) and the last stage hands its outputs to a Store functor, so only the
// middle exchanges use LDS.  Lines are laid out in LDS by Frame<N, NL, LF>:
//   LF = false: line-major (a row pass: a thread's butterflies run along a
//               line); every 16th position is followed by a pad slot so the
//               stride-R writes of the first stage spread over the banks
//   LF = true : position-major (a column pass: consecutive threads take
//               consecutive lines, i.e. adjacent columns of the frame, so
//               global accesses are coalesced row segments)
// Load(slot, line, pos) -> float2 and Store(slot, line, pos, float2) receive a
// per-thread slot index (butterfly i, leg r) that is the same for every call
// of the same transform shape, so callers can keep per-element registers.
// The gather of the next transform's inputs can be issued (fft_gather) while
// the current one is still in its LDS stages (fft_first / fft_rest).
// ---------------------------------------------------------------------------

template <int N, int NL, bool LF>
struct Frame {
  static constexpr int LD = LF ? NL + 1 : N + (N >> 4) + 1;
  static constexpr int ELEMS = LF ? N * LD : NL * LD;
  __device__ __forceinline__ static int lidx(int line, int pos) {
    return LF ? pos * LD + line : line * LD + pos + (pos >> 4);
  }
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
    const int f = fft_tid() + i * 256;
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
    const int f = fft_tid() + i * 256;
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
    const int f = fft_tid() + i * 256;
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
    const int f = fft_tid() + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      int line, j;
      F::template map<M>(f, line, j);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[r * j];
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

template <int... Rs>
struct Radices;
template <int R0, int... Rest>
struct Radices<R0, Rest...> {
  static constexpr int FIRST = R0;
  static constexpr int LAST = sizeof...(Rest) ? Radices<Rest...>::LAST : R0;
  static constexpr int COUNT = 1 + sizeof...(Rest);
};
template <int R0>
struct Radices<R0> {
  static constexpr int FIRST = R0;
  static constexpr int LAST = R0;
  static constexpr int COUNT = 1;
};

// Radix plans: N = product of the radices (first radix applied first).
template <int N> struct PlanOf;
template <> struct PlanOf<8> { using R = Radices<8>; };
template <> struct PlanOf<16> { using R = Radices<16>; };
template <> struct PlanOf<24> { using R = Radices<3, 8>; };
template <> struct PlanOf<32> { using R = Radices<8, 4>; };
template <> struct PlanOf<48> { using R = Radices<3, 16>; };
template <> struct PlanOf<64> { using R = Radices<8, 8>; };
template <> struct PlanOf<96> { using R = Radices<3, 8, 4>; };
template <> struct PlanOf<128> { using R = Radices<16, 8>; };
template <> struct PlanOf<192> { using R = Radices<3, 8, 8>; };
template <> struct PlanOf<256> { using R = Radices<16, 16>; };
template <> struct PlanOf<384> { using R = Radices<3, 8, 16>; };
template <> struct PlanOf<512> { using R = Radices<8, 8, 8>; };
template <> struct PlanOf<768> { using R = Radices<3, 16, 16>; };
template <> struct PlanOf<1024> { using R = Radices<16, 8, 8>; };

template <class Rads>
struct RestOf;
template <int R0, int... Rest>
struct RestOf<Radices<R0, Rest...>> {
  template <int N, int NL, bool LF, bool INV, bool STORE_LDS, class Store>
  __device__ __forceinline__ static void run(float2* buf, const float2* tw, Store& store) {
    stages_from_lds<N, NL, LF, INV, STORE_LDS, Store, R0, Rest...>(buf, tw, store);
  }
};

template <int N, int NL>
struct RegShape {
  using R = typename PlanOf<N>::R;
  static constexpr bool SINGLE = R::COUNT == 1;
  static constexpr int LOAD_SLOTS = Slots<N, NL, R::FIRST>::COUNT;
  static constexpr int STORE_SLOTS = Slots<N, NL, R::LAST>::COUNT;
};

// Enumerate this thread's first-stage (Load) or last-stage (Store) slots:
// fn(slot, line, pos) for every element the transform will hand it.
template <int N, int NL, bool LF, int R, class Fn>
__device__ __forceinline__ void for_slots(Fn&& fn) {
  using F = Frame<N, NL, LF>;
  constexpr int M = N / R;
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = fft_tid() + i * 256;
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
  for_slots<N, NL, LF, PlanOf<N>::R::FIRST>(fn);
}
template <int N, int NL, bool LF, class Fn>
__device__ __forceinline__ void for_store_slots(Fn&& fn) {
  for_slots<N, NL, LF, PlanOf<N>::R::LAST>(fn);
}

// Gather the first-stage inputs: v[slot] = load(slot, line, pos).
template <int N, int NL, bool LF, class Load>
__device__ __forceinline__ void fft_gather(float2* v, Load& load) {
  for_load_slots<N, NL, LF>([&](int s, int line, int pos) { v[s] = load(s, line, pos); });
}

// First stage from registers.  Multi-stage plans write the stage output to
// LDS and synchronise; single-stage plans transform in registers only.
// LOAD_LDS: the gathered values came from `buf`; all threads finish reading first.
template <int N, int NL, bool LF, bool INV, bool LOAD_LDS = false>
__device__ __forceinline__ void fft_first(float2* v, float2* buf) {
  using F = Frame<N, NL, LF>;
  constexpr int R0 = PlanOf<N>::R::FIRST;
  constexpr int M = N / R0;
  constexpr int TOT = NL * M;
  constexpr int NB = (TOT + 255) / 256;
  if (LOAD_LDS) __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int f = fft_tid() + i * 256;
    if (TOT % 256 == 0 || f < TOT) {
      Dft<R0, INV>::run(v + i * R0);
      if constexpr (!RegShape<N, NL>::SINGLE) {
        int line, j;
        F::template map<M>(f, line, j);
#pragma unroll
        for (int r = 0; r < R0; ++r) buf[F::lidx(line, j * R0 + r)] = v[i * R0 + r];
      }
    }
  }
  if constexpr (!RegShape<N, NL>::SINGLE) __syncthreads();
}

// Remaining stages; the last hands its outputs to Store.  For a single-stage
// plan this stores the registers transformed by fft_first.  On return the
// last stage's LDS reads are done but no barrier follows: a caller that
// rewrites `buf` afterwards must synchronise first.
template <int N, int NL, bool LF, bool INV, bool STORE_LDS = false, class Store>
__device__ __forceinline__ void fft_rest(const float2* v, float2* buf, const float2* tw, Store& store) {
  if constexpr (RegShape<N, NL>::SINGLE) {
    if (STORE_LDS) __syncthreads();
    for_load_slots<N, NL, LF>([&](int s, int line, int pos) { store(s, line, pos, v[s]); });
  } else {
    RestOf<typename PlanOf<N>::R>::template run<N, NL, LF, INV, STORE_LDS>(buf, tw, store);
  }
}

// Whole transform of NL lines: gather, first stage, remaining stages.
template <int N, int NL, bool LF, bool INV, bool LOAD_LDS = false, bool STORE_LDS = false, class Load, class Store>
__device__ __forceinline__ void fft_reg(float2* buf, const float2* tw, Load& load, Store& store) {
  float2 v[RegShape<N, NL>::LOAD_SLOTS];
  fft_gather<N, NL, LF>(v, load);
  fft_first<N, NL, LF, INV, LOAD_LDS>(v, buf);
  fft_rest<N, NL, LF, INV, STORE_LDS>(v, buf, tw, store);
}

}  // namespace pty
