// Kernels of the learned warm start (gfx950).
//
// Network: six 3 x 3 convolutions with 32 channels (zero padding 1, strides
// 2, 2, 2, 2, 2, 1, ReLU), a global average pool and a linear head with four
// outputs.  Activations and their gradients are stored NHWC in BF16 (one
// pixel's 32 channels are 64 contiguous bytes); weights are BF16 copies of
// FP32 master weights; every sum accumulates in FP32.
//
// Layers 2-6 run as implicit GEMMs on v_mfma_f32_16x16x32_bf16 (lane l of a
// wave64 holds A[row = l % 16][k = 8 (l / 16) + i], B[k = 8 (l / 16) + i][col = l % 16],
// and receives C[row = 4 (l / 16) + i][col = l % 16]):
//   forward      C[pixel][co]  += sum_{tap, ci} X[src(pixel, tap)][ci] Wf[tap][co][ci]   (K = 32 channels per tap)
//   input grad   C[pixel][ci]  += sum_{tap, co} G[dst(pixel, tap)][co] Wb[tap][ci][co]
//   weight grad  C[co][ci]     += sum_pixels   G[q][co] X[src(q, tap)][ci]              (K = 32 pixels, via LDS transposes)
// Layer 1 (one input channel) runs on the vector ALUs.  Reductions over
// blocks go through partial buffers summed in a fixed order, so gradients are
// bitwise reproducible.

#include "learned.hpp"

#include <math.h>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace ws {
namespace {

union Pack8 {
  uint4 u;
  bf16x8 v;
};

__device__ __forceinline__ bf16x8 load8(const __bf16* p) {
  Pack8 k;
  k.u = *reinterpret_cast<const uint4*>(p);
  return k.v;
}

__device__ __forceinline__ bf16x8 zero8() {
  Pack8 k;
  k.u = make_uint4(0u, 0u, 0u, 0u);
  return k.v;
}

__device__ __forceinline__ floatx4 mma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// fixed-order block sum / max for blockDim.x a multiple of 64 (<= 1024)
__device__ float block_sum(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float s = 0.f;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

__device__ float block_min(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_down(v, o, 64));
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float s = red[0];
  for (int i = 1; i < nw; ++i) s = fminf(s, red[i]);
  return s;
}

__device__ float block_max(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float s = red[0];
  for (int i = 1; i < nw; ++i) s = fmaxf(s, red[i]);
  return s;
}

// ---------------------------------------------------------------------------
// Layer 1: 128 x 128 x 1 (FP32 input) -> 64 x 64 x 32, stride 2, ReLU.
// One thread per output pixel, all 32 channels.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv1_fwd(const float* __restrict__ x, const int* __restrict__ idx, int nb,
                                                   const __bf16* __restrict__ w1, const float* __restrict__ b1,
                                                   __bf16* __restrict__ a1) {
  __shared__ float w[kTaps][kC];
  __shared__ float b[kC];
  for (int i = threadIdx.x; i < kTaps * kC; i += blockDim.x) w[i / kC][i % kC] = (float)w1[i];
  if (threadIdx.x < kC) b[threadIdx.x] = b1[threadIdx.x];
  __syncthreads();
  constexpr int HI = kSide, HO = kSide / 2;
  const long total = (long)nb * HO * HO;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < total; p += (long)gridDim.x * blockDim.x) {
    const int n = (int)(p / (HO * HO));
    const int rem = (int)(p - (long)n * HO * HO);
    const int ho = rem / HO, wo = rem - (rem / HO) * HO;
    const float* xs = x + (size_t)(idx ? idx[n] : n) * HI * HI;
    float in[kTaps];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int hi = 2 * ho + ky - 1, wi = 2 * wo + kx - 1;
        in[ky * 3 + kx] = (hi >= 0 && hi < HI && wi >= 0 && wi < HI) ? xs[hi * HI + wi] : 0.f;
      }
    Pack8 out[4];
#pragma unroll
    for (int co = 0; co < kC; ++co) {
      float acc = b[co];
#pragma unroll
      for (int t = 0; t < kTaps; ++t) acc += w[t][co] * in[t];
      out[co >> 3].v[co & 7] = (__bf16)fmaxf(acc, 0.f);
    }
    uint4* dst = reinterpret_cast<uint4*>(a1 + p * kC);
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = out[i].u;
  }
}

// ---------------------------------------------------------------------------
// Layers 2-6 forward: one wave computes 16 output pixels x 32 channels per task.
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(256) void k_conv_fwd(const __bf16* __restrict__ ain, int nb, int hin, int hout,
                                                  const __bf16* __restrict__ wf, const float* __restrict__ bias,
                                                  __bf16* __restrict__ aout) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  bf16x8 b[kTaps][2];
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int j = 0; j < 2; ++j) b[t][j] = load8(wf + ((t * kC + 16 * j + r) * kC + 8 * kq));
  const float bs0 = bias[r], bs1 = bias[16 + r];
  const int plane = hout * hout;
  const long tasks = (long)nb * plane / 16;
  const long nwaves = (long)gridDim.x * (blockDim.x >> 6);
  for (long tk = blockIdx.x * (long)(blockDim.x >> 6) + (threadIdx.x >> 6); tk < tasks; tk += nwaves) {
    const long p = tk * 16 + r;
    const int n = (int)(p / plane);
    const int rem = (int)(p - (long)n * plane);
    const int ho = rem / hout, wo = rem - (rem / hout) * hout;
    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int hi = ho * S + ky - 1, wi = wo * S + kx - 1;
        bf16x8 a = zero8();
        if (hi >= 0 && hi < hin && wi >= 0 && wi < hin)
          a = load8(ain + (((size_t)n * hin + hi) * hin + wi) * kC + 8 * kq);
        acc0 = mma(a, b[ky * 3 + kx][0], acc0);
        acc1 = mma(a, b[ky * 3 + kx][1], acc1);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const size_t q = (size_t)tk * 16 + 4 * kq + i;
      aout[q * kC + r] = (__bf16)fmaxf(acc0[i] + bs0, 0.f);
      aout[q * kC + 16 + r] = (__bf16)fmaxf(acc1[i] + bs1, 0.f);
    }
  }
}

// ---------------------------------------------------------------------------
// Head: global average pool over the last 4 x 4 map, linear layer, squared
// error against normalised targets, and the gradients it starts: per-sample
// head-weight partials and G6 = dL/d(pre-activation of layer 6).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_head(const __bf16* __restrict__ a6, int nb, int plane,
                                             const __bf16* __restrict__ hw, const float* __restrict__ hb,
                                             const float* __restrict__ target, const int* __restrict__ idx, Norm nm,
                                             float* __restrict__ y_out, float* __restrict__ loss_part,
                                             float* __restrict__ head_part, __bf16* __restrict__ g6) {
  const int n = blockIdx.x, t = threadIdx.x;
  __shared__ float feat[kC], dy[kOut], sq[kOut], dfeat[kC];
  const __bf16* a = a6 + (size_t)n * plane * kC;
  if (t < kC) {
    float s = 0.f;
    for (int p = 0; p < plane; ++p) s += (float)a[p * kC + t];
    feat[t] = s / (float)plane;
  }
  __syncthreads();
  if (t < kOut) {
    float y = hb[t];
    for (int c = 0; c < kC; ++c) y += (float)hw[t * kC + c] * feat[c];
    y_out[n * kOut + t] = y * nm.scale[t] + nm.off[t];
    if (target) {
      const float tn = (target[(size_t)(idx ? idx[n] : n) * kOut + t] - nm.off[t]) / nm.scale[t];
      const float d = y - tn;
      dy[t] = 2.f * d / (float)(nb * kOut);
      sq[t] = d * d;
    }
  }
  __syncthreads();
  if (!target) return;
  if (t == 0) loss_part[n] = ((sq[0] + sq[1]) + sq[2]) + sq[3];
  for (int e = t; e < kOut * kC; e += blockDim.x) head_part[(size_t)n * kHeadCols + e] = dy[e / kC] * feat[e % kC];
  if (t < kOut) head_part[(size_t)n * kHeadCols + kOut * kC + t] = dy[t];
  if (t < kC) {
    float s = 0.f;
    for (int o = 0; o < kOut; ++o) s += (float)hw[o * kC + t] * dy[o];
    dfeat[t] = s / (float)plane;
  }
  __syncthreads();
  for (int e = t; e < plane * kC; e += blockDim.x)
    g6[(size_t)n * plane * kC + e] = ((float)a[e] > 0.f) ? (__bf16)dfeat[e & (kC - 1)] : (__bf16)0.f;
}

// ---------------------------------------------------------------------------
// Input gradient of layers 2-6 fused with the ReLU mask of the layer below:
// Gin[p][ci] = [Ain[p][ci] > 0] sum_{tap, co} Gout[q(p, tap)][co] W[co][ci][tap],
// where p = S q + tap - 1 (taps whose q is not an output pixel contribute 0).
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const __bf16* __restrict__ gout, int nb, int hin, int hout,
                                                       const __bf16* __restrict__ wb, const __bf16* __restrict__ ain,
                                                       __bf16* __restrict__ gin) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  bf16x8 b[kTaps][2];
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int j = 0; j < 2; ++j) b[t][j] = load8(wb + ((t * kC + 16 * j + r) * kC + 8 * kq));
  const int plane = hin * hin;
  const long tasks = (long)nb * plane / 16;
  const long nwaves = (long)gridDim.x * (blockDim.x >> 6);
  for (long tk = blockIdx.x * (long)(blockDim.x >> 6) + (threadIdx.x >> 6); tk < tasks; tk += nwaves) {
    const long p = tk * 16 + r;
    const int n = (int)(p / plane);
    const int rem = (int)(p - (long)n * plane);
    const int hi = rem / hin, wi = rem - (rem / hin) * hin;
    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int hn = hi + 1 - ky, wn = wi + 1 - kx;
        bool ok = hn >= 0 && wn >= 0;
        if (S == 2) ok = ok && ((hn & 1) == 0) && ((wn & 1) == 0);
        const int ho = hn / S, wo = wn / S;
        ok = ok && ho < hout && wo < hout;
        bf16x8 a = zero8();
        if (ok) a = load8(gout + (((size_t)n * hout + ho) * hout + wo) * kC + 8 * kq);
        acc0 = mma(a, b[ky * 3 + kx][0], acc0);
        acc1 = mma(a, b[ky * 3 + kx][1], acc1);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const size_t q = (size_t)tk * 16 + 4 * kq + i;
      gin[q * kC + r] = ((float)ain[q * kC + r] > 0.f) ? (__bf16)acc0[i] : (__bf16)0.f;
      gin[q * kC + 16 + r] = ((float)ain[q * kC + 16 + r] > 0.f) ? (__bf16)acc1[i] : (__bf16)0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient of layers 2-6.  A block owns a contiguous range of output
// pixels q and walks it 64 at a time: the gradient tile G[q][co] and, per tap,
// the gathered input tile X[src(q, tap)][ci] are staged transposed in LDS
// ([channel][q], row pitch 72 BF16 so that 8-element fragments are 16-byte
// aligned); wave w accumulates the (co tile w / 2, ci tile w % 2) 16 x 16 block
// of all nine taps.  Partials: part[block][tap][co][ci], then db[co].
// ---------------------------------------------------------------------------
constexpr int kWPart = kConvW + kC;

template <int S>
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const __bf16* __restrict__ gout,
                                                         const __bf16* __restrict__ ain, int nb, int hin, int hout,
                                                         int chunk, float* __restrict__ part) {
  constexpr int P = 72;
  __shared__ __align__(16) __bf16 gT[kC * P];
  __shared__ __align__(16) __bf16 xT[kC * P];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, kq = lane >> 4;
  const int mt = w >> 1, nt = w & 1;
  const long Q = (long)nb * hout * hout;
  const long q_begin = blockIdx.x * (long)chunk;
  const long q_end = (q_begin + chunk < Q) ? q_begin + chunk : Q;
  floatx4 acc[kTaps];
#pragma unroll
  for (int t = 0; t < kTaps; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  float db = 0.f;
  const int ql = tid >> 2, c8 = (tid & 3) * 8;
  const int plane = hout * hout;
  for (long q0 = q_begin; q0 < q_end; q0 += 64) {
    const long q = q0 + ql;
    const bool qv = q < q_end;
    int n = 0, ho = 0, wo = 0;
    if (qv) {
      n = (int)(q / plane);
      const int rem = (int)(q - (long)n * plane);
      ho = rem / hout;
      wo = rem - ho * hout;
    }
    Pack8 gv;
    gv.u = make_uint4(0u, 0u, 0u, 0u);
    if (qv) gv.v = load8(gout + q * kC + c8);
    __syncthreads();  // the previous tile's fragments have been read
#pragma unroll
    for (int i = 0; i < 8; ++i) gT[(c8 + i) * P + ql] = gv.v[i];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int t = ky * 3 + kx;
        const int hi = ho * S + ky - 1, wi = wo * S + kx - 1;
        Pack8 xv;
        xv.u = make_uint4(0u, 0u, 0u, 0u);
        if (qv && hi >= 0 && hi < hin && wi >= 0 && wi < hin)
          xv.v = load8(ain + (((size_t)n * hin + hi) * hin + wi) * kC + c8);
        if (t > 0) __syncthreads();  // every wave is done with the previous tap's tile
#pragma unroll
        for (int i = 0; i < 8; ++i) xT[(c8 + i) * P + ql] = xv.v[i];
        __syncthreads();
        if (t == 0 && tid < kC) {
          for (int k = 0; k < 64; ++k) db += (float)gT[tid * P + k];
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(&gT[(16 * mt + r) * P + 32 * ks + 8 * kq]);
          const bf16x8 bb = *reinterpret_cast<const bf16x8*>(&xT[(16 * nt + r) * P + 32 * ks + 8 * kq]);
          acc[t] = mma(a, bb, acc[t]);
        }
      }
  }
  float* pb = part + (size_t)blockIdx.x * kWPart;
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) pb[t * kC * kC + (16 * mt + 4 * kq + i) * kC + 16 * nt + r] = acc[t][i];
  if (tid < kC) pb[kConvW + tid] = db;
}

// Weight gradient of layer 1 (one input channel): thread (tap, co) for tid < 288,
// bias co for tid in [288, 320).  Partials: part[block][tap * 32 + co], then db.
constexpr int kW1Part = kTaps * kC + kC;

__global__ __launch_bounds__(320) void k_conv1_bwd_weight(const __bf16* __restrict__ g1,
                                                          const float* __restrict__ x, const int* __restrict__ idx,
                                                          int nb, int chunk, float* __restrict__ part) {
  __shared__ float gs[64][kC + 1];
  __shared__ float xs[64][kTaps];
  constexpr int HI = kSide, HO = kSide / 2;
  const int tid = threadIdx.x;
  const long Q = (long)nb * HO * HO;
  const long q_begin = blockIdx.x * (long)chunk;
  const long q_end = (q_begin + chunk < Q) ? q_begin + chunk : Q;
  const int tap = tid >> 5, co = tid & (kC - 1);
  float acc = 0.f;
  for (long q0 = q_begin; q0 < q_end; q0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * kC; e += blockDim.x) {
      const int ql = e >> 5, c = e & (kC - 1);
      const long q = q0 + ql;
      gs[ql][c] = (q < q_end) ? (float)g1[q * kC + c] : 0.f;
    }
    for (int e = tid; e < 64 * kTaps; e += blockDim.x) {
      const int ql = e / kTaps, t = e - (e / kTaps) * kTaps;
      const long q = q0 + ql;
      float v = 0.f;
      if (q < q_end) {
        const int n = (int)(q / (HO * HO));
        const int rem = (int)(q - (long)n * HO * HO);
        const int ho = rem / HO, wo = rem - (rem / HO) * HO;
        const int hi = 2 * ho + t / 3 - 1, wi = 2 * wo + t % 3 - 1;
        if (hi >= 0 && hi < HI && wi >= 0 && wi < HI) v = x[(size_t)(idx ? idx[n] : n) * HI * HI + hi * HI + wi];
      }
      xs[ql][t] = v;
    }
    __syncthreads();
    if (tid < kTaps * kC) {
      for (int k = 0; k < 64; ++k) acc += gs[k][co] * xs[k][tap];
    } else {
      for (int k = 0; k < 64; ++k) acc += gs[k][co];
    }
  }
  part[(size_t)blockIdx.x * kW1Part + tid] = acc;
}

// Column sums of a partial buffer in row order, scattered into the flat
// parameter order (or the loss).
__global__ void k_reduce(const float* __restrict__ part, int rows, int cols, int mode, int off, float scale,
                         float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += part[(size_t)r * cols + e];
  int dst = off + e;
  if (mode == RED_CONV1) {
    dst = (e < kTaps * kC) ? (e & (kC - 1)) * kTaps + (e >> 5) : kTaps * kC + (e - kTaps * kC);
  } else if (mode == RED_CONV) {
    if (e < kConvW) {
      const int t = e >> 10, co = (e >> 5) & (kC - 1), ci = e & (kC - 1);
      dst = off + co * kC * kTaps + ci * kTaps + t;
    }
  }
  out[dst] = s * scale;
}

// Adam on the FP32 master weights (optional), then the BF16 working copies:
// w1b[tap][co], wf[l][tap][co][ci], wb[l][tap][ci][co], hwb[t][c].
__global__ void k_adam_pack(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, int update, float lr, float b1, float b2, float eps, float c1,
                            float c2, __bf16* __restrict__ w1b, __bf16* __restrict__ wf, __bf16* __restrict__ wb,
                            __bf16* __restrict__ hwb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  float th = theta[i];
  if (update) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    th -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = th;
  }
  const __bf16 h = (__bf16)th;
  if (i < kTaps * kC) {
    w1b[(i % kTaps) * kC + i / kTaps] = h;
  } else if (i >= kL1 && i < kHeadW) {
    const int j = i - kL1, l = j / kConvStride, k = j - l * kConvStride;
    if (k < kConvW) {
      const int co = k / (kC * kTaps), ci = (k / kTaps) % kC, t = k % kTaps;
      wf[(size_t)l * kConvW + (t * kC + co) * kC + ci] = h;
      wb[(size_t)l * kConvW + (t * kC + ci) * kC + co] = h;
    }
  } else if (i >= kHeadW && i < kHeadB) {
    hwb[i - kHeadW] = h;
  }
}

// ---------------------------------------------------------------------------
// Network input from a scan: mean over patterns of log(1 + I), standardised
// over the frame (constant up to rounding -> 0), centred in a side x side zero
// image.  One block of 1024 threads; n <= 128.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_features(const float* __restrict__ ints, int n_pat, int n, int side,
                                                   float* __restrict__ out) {
  __shared__ float red[16];
  const int tid = threadIdx.x, npx = n * n;
  float m[16];
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int e = tid + 1024 * j;
    float acc = 0.f;
    if (e < npx)
      for (int p = 0; p < n_pat; ++p) acc += log1pf(ints[(size_t)p * npx + e]);
    m[j] = (e < npx) ? acc / (float)n_pat : 0.f;
    s += m[j];
  }
  const float mu = block_sum(s, red) / (float)npx;
  float q = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (tid + 1024 * j < npx) q += (m[j] - mu) * (m[j] - mu);
  const float sd = sqrtf(block_sum(q, red) / (float)npx);
  const bool flat = !(sd > 1e-6f * (1.f + fabsf(mu)));
  const int o = (side - n) / 2;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int e = tid + 1024 * j;
    if (e < npx) out[(e / n + o) * side + (e % n) + o] = flat ? 0.f : (m[j] - mu) / sd;
  }
  for (int e = tid; e < side * side; e += 1024) {
    const int y = e / side - o, xx = e % side - o;
    if (y < 0 || y >= n || xx < 0 || xx >= n) out[e] = 0.f;
  }
}

// Rendered warm-start probe: disc of radius R about (n/2, n/2) with phase
// 2 pi c r^2 / n^2, times {1, x^, y^, x^ y^} (x^ = (x - n/2) / (n/4)), each mode
// normalised, powers (1, 0.05, 0.05, 0.05) scaled to sum to `total`.
__global__ __launch_bounds__(1024) void k_render_probe(int n, int k, float radius, float defocus, float total,
                                                       float2* __restrict__ out) {
  __shared__ float red[16];
  __shared__ float norm2[4];
  const int npx = n * n;
  const float h = 0.5f * (float)n, q = 0.25f * (float)n;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int e = threadIdx.x; e < npx; e += blockDim.x) {
    const float x = (float)(e % n) - h, y = (float)(e / n) - h;
    if (x * x + y * y <= radius * radius) {
      const float xh = x / q, yh = y / q;
      acc[0] += 1.f;
      acc[1] += xh * xh;
      acc[2] += yh * yh;
      acc[3] += xh * xh * yh * yh;
    }
  }
  for (int j = 0; j < 4; ++j) {
    const float s = block_sum(acc[j], red);
    if (threadIdx.x == 0) norm2[j] = s;
  }
  __syncthreads();
  const float wsum = 1.f + 0.05f * (float)(k - 1);
  for (int mode = 0; mode < k; ++mode) {
    const float pw = (mode == 0 ? 1.f : 0.05f) / wsum * total;
    const float amp = norm2[mode] > 0.f ? sqrtf(pw / norm2[mode]) : 0.f;
    for (int e = threadIdx.x; e < npx; e += blockDim.x) {
      const float x = (float)(e % n) - h, y = (float)(e / n) - h;
      const float r2 = x * x + y * y;
      float2 v = make_float2(0.f, 0.f);
      if (r2 <= radius * radius) {
        const float xh = x / q, yh = y / q;
        const float mul = mode == 0 ? 1.f : mode == 1 ? xh : mode == 2 ? yh : xh * yh;
        float sn, cs;
        sincospif(2.f * defocus * r2 / (float)(n * n), &sn, &cs);
        v = make_float2(amp * mul * cs, amp * mul * sn);
      }
      out[(size_t)mode * npx + e] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Forward-model generator.  Counter-based random numbers: SplitMix64's output
// mix applied to key + mix(stream + golden * (counter + 1)).  Streams per
// sample s: 8 s (parameters), 8 s + 1 / + 2 (object amplitude / phase noise),
// 8 s + 3 (scan jitter), 8 s + 4 (Poisson counts).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t rng64(uint64_t key, uint64_t stream, uint64_t ctr) {
  return mix64(key + mix64(stream + 0x9E3779B97F4A7C15ULL * (ctr + 1)));
}
__device__ __forceinline__ float unif(uint64_t u) {  // (0, 1)
  return ((float)(u >> 40) + 0.5f) * (1.0f / 16777216.0f);
}
__device__ __forceinline__ float normal(uint64_t key, uint64_t stream, uint64_t ctr) {
  const float u1 = unif(rng64(key, stream, 2 * ctr)), u2 = unif(rng64(key, stream, 2 * ctr + 1));
  return sqrtf(-2.f * logf(u1)) * cospif(2.f * u2);
}

// per-sample draws (sigma, bandwidth, radius, defocus) and raster positions with
// integer jitter in [-jitter, jitter], centred in the side x side object
__global__ void k_fm_setup(uint64_t key, long first, FmRanges rg, int side, int n_scan, int step, int jitter,
                           float* __restrict__ sp, int* __restrict__ pos) {
  const int ls = blockIdx.x;
  const uint64_t s = (uint64_t)(first + ls);
  if (threadIdx.x == 0) {
    sp[ls * 4 + 0] = rg.sigma_lo + (rg.sigma_hi - rg.sigma_lo) * unif(rng64(key, 8 * s, 0));
    sp[ls * 4 + 1] = rg.bw_lo + (rg.bw_hi - rg.bw_lo) * unif(rng64(key, 8 * s, 1));
    sp[ls * 4 + 2] = rg.r_lo + (rg.r_hi - rg.r_lo) * unif(rng64(key, 8 * s, 2));
    sp[ls * 4 + 3] = rg.c_lo + (rg.c_hi - rg.c_lo) * unif(rng64(key, 8 * s, 3));
  }
  const int n_pos = n_scan * n_scan;
  const int extent = (n_scan - 1) * step + kFmN;
  const int r0 = (side - extent) / 2;
  for (int p = threadIdx.x; p < n_pos; p += blockDim.x) {
    const int i = p / n_scan, j = p % n_scan;
    const int span = 2 * jitter + 1;
    const int dr = (int)(unif(rng64(key, 8 * s + 3, 2 * p)) * span) - jitter;
    const int dc = (int)(unif(rng64(key, 8 * s + 3, 2 * p + 1)) * span) - jitter;
    pos[(ls * n_pos + p) * 2 + 0] = min(max(r0 + i * step + dr, 0), side - kFmN);
    pos[(ls * n_pos + p) * 2 + 1] = min(max(r0 + j * step + dc, 0), side - kFmN);
  }
}

// Object texture: N(0, 1) noise low-passed by a periodic Gaussian of 3 px
// (taps |d| <= 12), min-max mapped to amplitude [0.8, 1] (stored as ln A) or
// phase [-pi/2, pi/2].  Block (sample, field); the field lives in LDS.
__global__ __launch_bounds__(1024) void k_fm_object(uint64_t key, long first, int side, float2* __restrict__ obj) {
  __shared__ float z[kFmMaxSide * kFmMaxSide];
  __shared__ float red[16];
  const int ls = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
  const uint64_t s = (uint64_t)(first + ls);
  const int npx = side * side;
  constexpr int kPer = (kFmMaxSide * kFmMaxSide + 1023) / 1024;
  for (int e = tid; e < npx; e += 1024) z[e] = normal(key, 8 * s + 1 + f, (uint64_t)e);
  __syncthreads();
  float g[13];
#pragma unroll
  for (int d = 0; d <= 12; ++d) g[d] = expf(-(float)(d * d) / 18.f);
  float tmp[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int e = tid + 1024 * j;
    float a = 0.f;
    if (e < npx) {
      const int y = e / side, x = e % side;
      a = g[0] * z[y * side + x];
      for (int d = 1; d <= 12; ++d) a += g[d] * (z[y * side + (x + d) % side] + z[y * side + (x - d + side) % side]);
    }
    tmp[j] = a;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j)
    if (tid + 1024 * j < npx) z[tid + 1024 * j] = tmp[j];
  __syncthreads();
  float lo = 3.4e38f, hi = -3.4e38f;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int e = tid + 1024 * j;
    float a = 0.f;
    if (e < npx) {
      const int y = e / side, x = e % side;
      a = g[0] * z[y * side + x];
      for (int d = 1; d <= 12; ++d) a += g[d] * (z[((y + d) % side) * side + x] + z[((y - d + side) % side) * side + x]);
      lo = fminf(lo, a);
      hi = fmaxf(hi, a);
    }
    tmp[j] = a;
  }
  lo = block_min(lo, red);
  hi = block_max(hi, red);
  const float span = fmaxf(hi - lo, 1e-30f);
  float2* o = obj + (size_t)ls * npx;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int e = tid + 1024 * j;
    if (e >= npx) continue;
    const float u = (tmp[j] - lo) / span;
    if (f == 0)
      o[e].x = logf(0.8f + 0.2f * u);
    else
      o[e].y = -0.5f * (float)M_PI + (float)M_PI * u;
  }
}

// Noise-free broadband pattern of one scan position (block = (position,
// sample), 256 threads as 16 x 16, each owning outputs (ty + 16 a, tx + 16 b)):
// for each of n_wl wavelength scales s, psi = exp(s (lnA + i phi)) P and
// Psi = F_s psi F_s^T with F_s[u][x] = exp(-2 pi i s (u - 32)(x - 32) / 64) / 8
// (two dense complex products of the LDS-staged operands on FP32 matrix cores);
// the mean |Psi|^2 is blurred by the normalised periodic full-frame Gaussian
// (separable), written with its total.
__global__ __launch_bounds__(256) void k_fm_patterns(const float2* __restrict__ obj, int side,
                                                     const float* __restrict__ sp, const int* __restrict__ pos,
                                                     int n_pos, int n_wl, float* __restrict__ pat,
                                                     float* __restrict__ tot) {
  constexpr int N = kFmN;
  __shared__ float2 X[N * N];
  __shared__ float2 Ft[N * N];
  __shared__ float g[N];
  __shared__ float red[4];
  const int p = blockIdx.x, ls = blockIdx.y, tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const float sigma = sp[ls * 4 + 0], bw = sp[ls * 4 + 1], radius = sp[ls * 4 + 2], defocus = sp[ls * 4 + 3];
  const int row = pos[(ls * n_pos + p) * 2 + 0], col = pos[(ls * n_pos + p) * 2 + 1];
  const float2* o = obj + (size_t)ls * side * side;
  const float h = 0.5f * (float)N;
  float cnt = 0.f;
  for (int e = tid; e < N * N; e += 256) {
    const float x = (float)(e % N) - h, y = (float)(e / N) - h;
    cnt += (x * x + y * y <= radius * radius) ? 1.f : 0.f;
  }
  cnt = block_sum(cnt, red);
  const float pn = cnt > 0.f ? rsqrtf(cnt) : 0.f;
  float I[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) I[i] = 0.f;
  for (int j = 0; j < n_wl; ++j) {
    const float d = n_wl > 1 ? -0.5f * bw + bw * (float)j / (float)(n_wl - 1) : 0.f;
    const float s = 1.f / (1.f + d);
    __syncthreads();
    for (int e = tid; e < N * N; e += 256) {
      const int xr = e / N, u = e % N;  // Ft[x][u] = F[u][x]
      const float t = s * (float)((u - N / 2) * (xr - N / 2)) / (float)N;
      float sn, cs;
      sincospif(-2.f * t, &sn, &cs);
      Ft[e] = make_float2(cs * 0.125f, sn * 0.125f);
      const int y = e / N, x = e % N;
      const float xx = (float)x - h, yy = (float)y - h;
      const float r2 = xx * xx + yy * yy;
      float2 v = make_float2(0.f, 0.f);
      if (r2 <= radius * radius) {
        const float2 la = o[(size_t)(row + y) * side + col + x];
        const float amp = expf(s * la.x) * pn;
        float ps, pc;
        sincosf(2.f * (float)M_PI * defocus * r2 / (float)(N * N) + s * la.y, &ps, &pc);
        v = make_float2(amp * pc, amp * ps);
      }
      X[e] = v;
    }
    __syncthreads();
    // Y1 = X Ft, then Y2 = F Y1 (F = Ft^T), on v_mfma_f32_16x16x4_f32: wave w owns
    // output rows 16 w .. 16 w + 15 of each product, four 16-column tiles; per step
    // of 4 along k, lane l supplies A[row l % 16][k l / 16] and B[k l / 16][col l % 16]
    // and holds C[row 4 (l / 16) + r][col l % 16], r < 4.  A complex product is four
    // real ones (the imaginary part of A negated once per step for the real part).
    floatx4 cr[4], ci[4];
    auto cmac = [&](float2 av, const float2* bv) {
      const float nai = -av.y;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        cr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv[t].x, cr[t], 0, 0, 0);
        cr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai, bv[t].y, cr[t], 0, 0, 0);
        ci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv[t].y, ci[t], 0, 0, 0);
        ci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv[t].x, ci[t], 0, 0, 0);
      }
    };
    const int wv = tid >> 6, ln = tid & 63, lr = ln & 15, lk = ln >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) cr[t] = ci[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < N; k0 += 4) {
      const float2 av = X[(16 * wv + lr) * N + k0 + lk];
      float2 bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[t] = Ft[(k0 + lk) * N + 16 * t + lr];
      cmac(av, bv);
    }
    __syncthreads();  // every wave has read X before Y1 overwrites it
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) X[(16 * wv + 4 * lk + r) * N + 16 * t + lr] = make_float2(cr[t][r], ci[t][r]);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) cr[t] = ci[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < N; k0 += 4) {
      const float2 av = Ft[(k0 + lk) * N + 16 * wv + lr];  // F[row][k] = Ft[k][row]
      float2 bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[t] = X[(k0 + lk) * N + 16 * t + lr];
      cmac(av, bv);
    }
    const float wgt = 1.f / (float)n_wl;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) I[t * 4 + r] += wgt * (cr[t][r] * cr[t][r] + ci[t][r] * ci[t][r]);
  }
  // I[t * 4 + r] is output (16 wv + 4 lk + r, 16 t + lr); move it to the (ty + 16 a,
  // tx + 16 b) ownership of the blur and the store below
  {
    float* ib = reinterpret_cast<float*>(X);
    const int wv = tid >> 6, ln = tid & 63, lr = ln & 15, lk = ln >> 4;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) ib[(16 * wv + 4 * lk + r) * N + 16 * t + lr] = I[t * 4 + r];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) I[a * 4 + b] = ib[(ty + 16 * a) * N + tx + 16 * b];
  }
  if (sigma > 0.f) {
    float* ib = reinterpret_cast<float*>(X);
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) ib[(ty + 16 * a) * N + tx + 16 * b] = I[a * 4 + b];
    if (tid < N) {
      const float dd = (float)min(tid, N - tid);
      g[tid] = expf(-dd * dd / (2.f * sigma * sigma));
    }
    __syncthreads();
    float gs = 0.f;
    for (int d = 0; d < N; ++d) gs += g[d];
    float tmp[16];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int v = ty + 16 * a, u = tx + 16 * b;
        float s = 0.f;
#pragma unroll 4
        for (int d = 0; d < N; ++d) s += g[d] * ib[v * N + ((u - d) & (N - 1))];
        tmp[a * 4 + b] = s;
      }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) ib[(ty + 16 * a) * N + tx + 16 * b] = tmp[a * 4 + b];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int v = ty + 16 * a, u = tx + 16 * b;
        float s = 0.f;
#pragma unroll 4
        for (int d = 0; d < N; ++d) s += g[d] * ib[((v - d) & (N - 1)) * N + u];
        I[a * 4 + b] = s / (gs * gs);
      }
  }
  float* out = pat + ((size_t)ls * n_pos + p) * N * N;
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      out[(ty + 16 * a) * N + tx + 16 * b] = I[a * 4 + b];
      s += I[a * 4 + b];
    }
  s = block_sum(s, red);
  if (tid == 0) tot[ls * n_pos + p] = s;
}

// Poisson draw: inversion by sequential search below 12, else the rounded
// normal approximation lambda + sqrt(lambda) z (training data only).
__device__ float poisson_draw(float lam, uint64_t key, uint64_t stream, uint64_t ctr) {
  if (!(lam > 0.f)) return 0.f;
  if (lam < 12.f) {
    const float u = unif(rng64(key, stream, 2 * ctr));
    float p = expf(-lam), F = p;
    int k = 0;
    while (u > F && k < 64) {
      ++k;
      p *= lam / (float)k;
      F += p;
    }
    return (float)k;
  }
  const float z = normal(key, stream, ctr);
  return fmaxf(0.f, floorf(lam + sqrtf(lam) * z + 0.5f));
}

// Per sample: scale the patterns to `counts` mean total, Poisson counts, mean
// log(1 + counts) over positions, standardise, centre in the 128 x 128 input;
// targets = the sample's (sigma, bandwidth, radius, defocus).
__global__ __launch_bounds__(256) void k_fm_features(const float* __restrict__ pat, const float* __restrict__ tot,
                                                     const float* __restrict__ sp, uint64_t key, long first,
                                                     int n_pos, float counts, float* __restrict__ feat,
                                                     float* __restrict__ targets) {
  constexpr int N = kFmN, NPX = N * N;
  __shared__ float red[4];
  const int ls = blockIdx.x, tid = threadIdx.x;
  const uint64_t s = (uint64_t)(first + ls);
  float T = 0.f;
  for (int p = 0; p < n_pos; ++p) T += tot[ls * n_pos + p];
  const float scale = T > 0.f ? counts * (float)n_pos / T : 0.f;
  float m[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) m[j] = 0.f;
  for (int p = 0; p < n_pos; ++p) {
    const float* src = pat + ((size_t)ls * n_pos + p) * NPX;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = tid + 256 * j;
      m[j] += log1pf(poisson_draw(scale * src[e], key, 8 * s + 4, (uint64_t)p * NPX + e));
    }
  }
  float sum = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    m[j] /= (float)n_pos;
    sum += m[j];
  }
  const float mu = block_sum(sum, red) / (float)NPX;
  float q = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) q += (m[j] - mu) * (m[j] - mu);
  const float sd = sqrtf(block_sum(q, red) / (float)NPX);
  const bool flat = !(sd > 1e-6f * (1.f + fabsf(mu)));
  float* out = feat + (size_t)ls * kSide * kSide;
  constexpr int o = (kSide - N) / 2;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int e = tid + 256 * j;
    out[(e / N + o) * kSide + e % N + o] = flat ? 0.f : (m[j] - mu) / sd;
  }
  for (int e = tid; e < kSide * kSide; e += 256) {
    const int y = e / kSide - o, x = e % kSide - o;
    if (y < 0 || y >= N || x < 0 || x >= N) out[e] = 0.f;
  }
  if (tid < 4) targets[ls * 4 + tid] = sp[ls * 4 + tid];
}

long grid_for(long work, int per_block, long cap) {
  long g = (work + per_block - 1) / per_block;
  return g < 1 ? 1 : (g > cap ? cap : g);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_conv1_fwd(const float* x, const int* idx, int nb, const __bf16* w1, const float* b1, __bf16* a1,
                      hipStream_t st) {
  const long total = (long)nb * (kSide / 2) * (kSide / 2);
  k_conv1_fwd<<<(unsigned)grid_for(total, 256, 8192), 256, 0, st>>>(x, idx, nb, w1, b1, a1);
}

void launch_conv_fwd(int l, const __bf16* ain, int nb, const __bf16* wf, const float* bias, __bf16* aout,
                     hipStream_t st) {
  const int hin = side_in(l), hout = side_out(l);
  const long tasks = (long)nb * hout * hout / 16;
  const unsigned g = (unsigned)grid_for(tasks, 16, 2048);
  if (stride_of(l) == 2)
    k_conv_fwd<2><<<g, 256, 0, st>>>(ain, nb, hin, hout, wf, bias, aout);
  else
    k_conv_fwd<1><<<g, 256, 0, st>>>(ain, nb, hin, hout, wf, bias, aout);
}

void launch_head(const __bf16* a6, int nb, const __bf16* hw, const float* hb, const float* target, const int* idx,
                 const Norm& nm, float* y, float* loss_part, float* head_part, __bf16* g6, hipStream_t st) {
  const int plane = side_out(kLayers - 1) * side_out(kLayers - 1);
  k_head<<<nb, 64, 0, st>>>(a6, nb, plane, hw, hb, target, idx, nm, y, loss_part, head_part, g6);
}

void launch_conv_bwd_data(int l, const __bf16* gout, int nb, const __bf16* wb, const __bf16* ain, __bf16* gin,
                          hipStream_t st) {
  const int hin = side_in(l), hout = side_out(l);
  const long tasks = (long)nb * hin * hin / 16;
  const unsigned g = (unsigned)grid_for(tasks, 16, 2048);
  if (stride_of(l) == 2)
    k_conv_bwd_data<2><<<g, 256, 0, st>>>(gout, nb, hin, hout, wb, ain, gin);
  else
    k_conv_bwd_data<1><<<g, 256, 0, st>>>(gout, nb, hin, hout, wb, ain, gin);
}

namespace {
constexpr int kMaxPartRows = 256;
long chunk_for(long q) {
  long c = (q + kMaxPartRows - 1) / kMaxPartRows;
  c = ((c + 63) / 64) * 64;
  return c < 64 ? 64 : c;
}
}  // namespace

int max_weight_partials() { return kMaxPartRows * kWPart; }

int launch_conv_bwd_weight(int l, const __bf16* gout, const __bf16* ain, int nb, float* part, hipStream_t st) {
  const int hin = side_in(l), hout = side_out(l);
  const long q = (long)nb * hout * hout;
  const long chunk = chunk_for(q);
  const int rows = (int)((q + chunk - 1) / chunk);
  if (stride_of(l) == 2)
    k_conv_bwd_weight<2><<<rows, 256, 0, st>>>(gout, ain, nb, hin, hout, (int)chunk, part);
  else
    k_conv_bwd_weight<1><<<rows, 256, 0, st>>>(gout, ain, nb, hin, hout, (int)chunk, part);
  return rows;
}

int launch_conv1_bwd_weight(const __bf16* g1, const float* x, const int* idx, int nb, float* part, hipStream_t st) {
  const long q = (long)nb * (kSide / 2) * (kSide / 2);
  const long chunk = chunk_for(q);
  const int rows = (int)((q + chunk - 1) / chunk);
  k_conv1_bwd_weight<<<rows, kW1Part, 0, st>>>(g1, x, idx, nb, (int)chunk, part);
  return rows;
}

void launch_reduce(const float* part, int rows, int cols, ReduceMode mode, int off, float scale, float* out,
                   hipStream_t st) {
  k_reduce<<<(cols + 255) / 256, 256, 0, st>>>(part, rows, cols, (int)mode, off, scale, out);
}

void launch_adam_pack(float* theta, const float* grad, float* m, float* v, bool update, float lr, float b1, float b2,
                      float eps, float c1, float c2, __bf16* w1b, __bf16* wf, __bf16* wb, __bf16* hwb,
                      hipStream_t st) {
  k_adam_pack<<<(kParams + 255) / 256, 256, 0, st>>>(theta, grad, m, v, update ? 1 : 0, lr, b1, b2, eps, c1, c2, w1b,
                                                     wf, wb, hwb);
}

void launch_features(const float* ints, int n_pat, int n, int side, float* out, hipStream_t st) {
  k_features<<<1, 1024, 0, st>>>(ints, n_pat, n, side, out);
}

void launch_render_probe(int n, int k, float radius, float defocus, float total, float2* out, hipStream_t st) {
  k_render_probe<<<1, 1024, 0, st>>>(n, k, radius, defocus, total, out);
}

void launch_fm_setup(uint64_t key, long first, int count, const FmRanges& rg, int side, int n_scan, int step,
                     int jitter, float* sp, int* pos, hipStream_t st) {
  k_fm_setup<<<count, 128, 0, st>>>(key, first, rg, side, n_scan, step, jitter, sp, pos);
}

void launch_fm_object(uint64_t key, long first, int count, int side, float2* obj, hipStream_t st) {
  k_fm_object<<<dim3(count, 2), 1024, 0, st>>>(key, first, side, obj);
}

void launch_fm_patterns(const float2* obj, int side, const float* sp, const int* pos, int n_pos, int count, int n_wl,
                        float* pat, float* tot, hipStream_t st) {
  k_fm_patterns<<<dim3(n_pos, count), 256, 0, st>>>(obj, side, sp, pos, n_pos, n_wl, pat, tot);
}

void launch_fm_features(const float* pat, const float* tot, const float* sp, uint64_t key, long first, int count,
                        int n_pos, float counts, float* feat, float* targets, hipStream_t st) {
  k_fm_features<<<count, 256, 0, st>>>(pat, tot, sp, key, first, n_pos, counts, feat, targets);
}

}  // namespace ws
