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

}  // namespace pty
