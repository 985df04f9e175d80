// Numerical monochromatisation of broadband far-field patterns by CGLS (gfx950),
// Sec. 4.2, Eq. (12)-(13): b = C m with C fixed by the source spectrum; the
// k-th CGLS iterate is the least-squares solution of ||C x - b|| over the Krylov
// subspace span{C^T b, (C^T C) C^T b, ...}.
//
// C m (u) = sum_j w_j s_j^2 m(c + s_j (u - c)), c = N / 2, s_j = lambda_c / lambda_j,
// sampled bilinearly (zero outside the frame); C^T is its exact adjoint, gathered
// per output pixel over the detector pixels whose samples touch it with the same
// weights.  Patterns are independent: every kernel covers all of them
// (blockIdx.y = pattern).  Per iteration: q = C p (with partial |q|^2), alpha,
// x += alpha p and r -= alpha q (partial |r|^2), s = C^T r (partial |s|^2), beta,
// p = s + beta p.  Partial sums are per block in double and summed in a fixed
// order, so the result is bitwise reproducible.
#include "kernels_dev.hpp"

namespace pty {

__device__ __forceinline__ float mono_at(const float* m, int n, int y, int x) {
  return ((unsigned)y < (unsigned)n && (unsigned)x < (unsigned)n) ? m[y * n + x] : 0.f;
}

// Bilinear sample position of detector pixel u at scale s: node i0 = floor(p) and weight t of node i0 + 1.
__device__ __forceinline__ void mono_sample(int u, float c, float s, int& i0, float& t) {
  const float p = c + s * ((float)u - c);
  const float f = floorf(p);
  i0 = (int)f;
  t = p - f;
}

// Forward table: i0 and t of every detector pixel at every scale.
__global__ __launch_bounds__(kThreads) void k_mono_fwd_table(MonoSpectrum sp, MonoTables tb, int n) {
  const int j = blockIdx.y;
  const int u = blockIdx.x * kThreads + threadIdx.x;
  if (u >= n) return;
  int i0;
  float t;
  mono_sample(u, 0.5f * (float)n, sp.scale[j], i0, t);
  tb.i0[j * n + u] = i0;
  tb.t[j * n + u] = t;
}

// Adjoint table from the forward table: node v takes weight 1 - t from pixels with
// i0 = v and t from pixels with i0 = v - 1 (t > 0).  i0 is nondecreasing in u, so
// these pixels are consecutive; the run starts at the first of them and holds
// adj_stride weights (zero past the last).  Pixels sampling v lie where
// v - 1 <= c + s (u - c) < v + 1, a window of width 2 / s, searched widened by one.
__global__ __launch_bounds__(kThreads) void k_mono_adj_table(MonoSpectrum sp, MonoTables tb, int n) {
  const int j = blockIdx.y;
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  const float c = 0.5f * (float)n, s = sp.scale[j];
  const int lo = max((int)floorf(((float)v - 1.0f - c) / s + c) - 1, 0);
  const int hi = min((int)ceilf(((float)v + 1.0f - c) / s + c) + 1, n - 1);
  const int* i0 = tb.i0 + j * n;
  const float* tt = tb.t + j * n;
  auto weight = [&](int u) -> float {
    if (u < 0 || u >= n) return 0.f;
    if (i0[u] == v) return 1.0f - tt[u];
    if (i0[u] == v - 1 && tt[u] > 0.f) return tt[u];
    return 0.f;
  };
  int first = lo;
  while (first <= hi && weight(first) == 0.f) ++first;
  float* w = tb.adj_w + ((size_t)j * n + v) * tb.adj_stride;
  int cnt = 0;
  for (int k = 0; k < tb.adj_stride; ++k) {
    w[k] = (first <= hi) ? weight(first + k) : 0.f;
    if (w[k] != 0.f) cnt = k + 1;
  }
  tb.adj_first[j * n + v] = first;
  tb.adj_cnt[j * n + v] = cnt;
}

// Output tiles of kMonoTy x kMonoTx pixels per block (a wave per 64-pixel row
// segment, kMonoQ rows per thread).  A block first copies its tile's slice of the
// interpolation tables into LDS (for every wavelength: kMonoTx column entries, then
// kMonoTy row entries, zero past the frame), then the input region its samples
// touch, clamped to the frame (when it holds at most kMonoLds values; otherwise the
// inputs are read from global memory with the same arithmetic).
constexpr int kMonoTx = 64, kMonoTy = 16, kMonoLds = 4096;
constexpr int kMonoSl = kMonoTx + kMonoTy;         // slice entries per wavelength
constexpr int kMonoQ = kMonoTy / (kThreads / 64);  // output rows per thread
__host__ __device__ inline int mono_tiles(int n) {
  return ((n + kMonoTx - 1) / kMonoTx) * ((n + kMonoTy - 1) / kMonoTy);
}
// dst[i] = ld(i) for i < cnt over the block's threads, kB loads of a thread in
// flight before its LDS stores (instead of one global round trip per value).
template <int kB, class Ld>
__device__ __forceinline__ void lds_fill(float* dst, int cnt, Ld ld) {
  for (int i0 = threadIdx.x; i0 < cnt; i0 += kB * kThreads) {
    float v[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int i = i0 + j * kThreads;
      v[j] = i < cnt ? ld(i) : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int i = i0 + j * kThreads;
      if (i < cnt) dst[i] = v[j];
    }
  }
}

// Dynamic LDS of k_mono_apply: region, slice indices and samples (or counts), and
// for the adjoint with few taps the slice's weights.
__host__ __device__ inline size_t mono_lds_bytes(int count, int stride, bool adj_w) {
  return sizeof(float) * ((size_t)kMonoLds + 2 * (size_t)count * kMonoSl +
                          (adj_w ? (size_t)count * kMonoSl * stride : 0));
}

// Smallest and largest input index along one axis (slice entries k0 .. k0 + len - 1)
// that the outputs touch: forward, nodes i0 and i0 + 1 of each sample; adjoint, the
// runs of nonzero weights; over every wavelength.
template <bool ADJ>
__device__ __forceinline__ int2 mono_span(int count, const int* sa, const int* sc, int k0, int len, int* sh) {
  int lo = 1 << 30, hi = -(1 << 30);
  for (int i = threadIdx.x; i < count * len; i += kThreads) {
    const int e = (i / len) * kMonoSl + k0 + i % len;
    const int a = sa[e];
    if (!ADJ) {
      lo = min(lo, a);
      hi = max(hi, a + 1);
    } else if (sc[e] > 0) {
      lo = min(lo, a);
      hi = max(hi, a + sc[e] - 1);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o));
    hi = max(hi, __shfl_xor(hi, o));
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = lo;
    sh[4 + (threadIdx.x >> 6)] = hi;
  }
  __syncthreads();
  lo = min(min(sh[0], sh[1]), min(sh[2], sh[3]));
  hi = max(max(sh[4], sh[5]), max(sh[6], sh[7]));
  return make_int2(lo, hi);
}

// The outputs of one thread (a column, kMonoQ rows) and their sum of squares.
// STAGED: inputs from the LDS copy of the region starting at (ry, rx), rw wide.
// Slice: sa = i0 (forward) or first pixel (adjoint), st = t (forward), sc = tap
// count (adjoint), sw = weights (adjoint with TAPS > 0; else the global table).
template <bool ADJ, int TAPS, bool STAGED>
__device__ __forceinline__ float mono_outputs(const float* __restrict__ m, const float* reg, int ry, int rx, int rw,
                                              int n, const MonoSpectrum& sp, const MonoTables& tb, int x0, int y0,
                                              const int* sa, const float* stt, const int* sc, const float* sw,
                                              float* __restrict__ outp) {
  // value at input (y, x): the staged copy (every in-frame index a sample touches
  // lies in the region) or the frame itself; forward samples outside the frame read
  // zero (the adjoint's taps are detector pixels, always inside)
  auto at = [&](int y, int x) -> float {
    if (!ADJ && ((unsigned)y >= (unsigned)n || (unsigned)x >= (unsigned)n)) return 0.f;
    return STAGED ? reg[(y - ry) * rw + (x - rx)] : m[(size_t)y * n + x];
  };
  const int kx = threadIdx.x & 63;
  const int ux = x0 + kx;
  const bool col_ok = ux < n;
  const int wrow = threadIdx.x >> 6;
  const int st = tb.adj_stride;
  float val[kMonoQ];
#pragma unroll
  for (int q = 0; q < kMonoQ; ++q) val[q] = 0.f;
  for (int j = 0; j < sp.count; ++j) {
    const float cj = sp.coef[j];
    const int ej = j * kMonoSl;
    if (!ADJ) {
      const int ix = sa[ej + kx];
      const float tx = stt[ej + kx];
#pragma unroll
      for (int q = 0; q < kMonoQ; ++q) {
        const int ky = wrow + q * (kThreads / 64);
        const int iy = sa[ej + kMonoTx + ky];
        const float ty = stt[ej + kMonoTx + ky];
        const float r0 = (1.0f - tx) * at(iy, ix) + tx * at(iy, ix + 1);
        const float r1 = (1.0f - tx) * at(iy + 1, ix) + tx * at(iy + 1, ix + 1);
        val[q] += cj * ((1.0f - ty) * r0 + ty * r1);
      }
    } else {
      const int ax = sa[ej + kx], cx = sc[ej + kx];
      const float* wxg = tb.adj_w + ((size_t)j * n + ux) * st;
      float wx[TAPS > 0 ? TAPS : 1];
      if (TAPS > 0) {
#pragma unroll
        for (int b = 0; b < TAPS; ++b) wx[b] = b < cx ? sw[(ej + kx) * st + b] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < kMonoQ; ++q) {
        const int ky = wrow + q * (kThreads / 64);
        const int ay = sa[ej + kMonoTx + ky], cy = sc[ej + kMonoTx + ky];
        const float* wyl = sw + (ej + kMonoTx + ky) * st;
        const float* wyg = tb.adj_w + ((size_t)j * n + min(y0 + ky, n - 1)) * st;
        float acc = 0.f;
        for (int a = 0; a < cy; ++a) {
          const float wa = TAPS > 0 ? wyl[a] : wyg[a];
          if (wa == 0.f) continue;
          float row = 0.f;
          if (TAPS > 0) {
#pragma unroll
            for (int b = 0; b < TAPS; ++b)
              if (b < cx && wx[b] != 0.f) row += wx[b] * at(ay + a, ax + b);
          } else {
            for (int b = 0; b < cx; ++b) {
              const float wb = wxg[b];
              if (wb != 0.f) row += wb * at(ay + a, ax + b);
            }
          }
          acc += wa * row;
        }
        val[q] += cj * acc;
      }
    }
  }
  float ss = 0.f;
#pragma unroll
  for (int q = 0; q < kMonoQ; ++q) {
    const int uy = y0 + wrow + q * (kThreads / 64);
    if (uy >= n || !col_ok) continue;
    outp[(size_t)uy * n + ux] = val[q];
    ss += val[q] * val[q];
  }
  return ss;
}

// out = C in (ADJ false) or C^T in (ADJ true) for every pattern (blockIdx.y) and
// output tile (blockIdx.x); part[pattern][tile] = sum out^2.  TAPS > 0: the
// adjoint's runs hold at most TAPS nonzero weights (the plan's maximum), kept in the
// LDS slice and a thread's column weights in registers; TAPS = 0: weights from the
// global table.  The adjoint sums, for each wavelength, its row weights in
// ascending pixel order, each row's column weights in ascending order (zero weights
// skipped).
template <bool ADJ, int TAPS>
__global__ __launch_bounds__(kThreads) void k_mono_apply(const float* __restrict__ in, float* __restrict__ out,
                                                         MonoSpectrum sp, MonoTables tb, int n,
                                                         double* __restrict__ part) {
  extern __shared__ float dyn[];
  __shared__ int spans[8];
  __shared__ double red[kThreads / 64];
  float* reg = dyn;
  int* sa = reinterpret_cast<int*>(dyn + kMonoLds);
  float* stt = dyn + kMonoLds + sp.count * kMonoSl;  // forward t
  int* sc = reinterpret_cast<int*>(stt);              // adjoint counts (same words)
  float* sw = dyn + kMonoLds + 2 * sp.count * kMonoSl;
  const size_t nn = (size_t)n * n;
  const int pat = blockIdx.y;
  const int tiles_x = (n + kMonoTx - 1) / kMonoTx;
  const int y0 = (blockIdx.x / tiles_x) * kMonoTy, x0 = (blockIdx.x % tiles_x) * kMonoTx;
  const int lx = min(x0 + kMonoTx, n) - x0, ly = min(y0 + kMonoTy, n) - y0;
  const float* m = in + (size_t)pat * nn;
  const int st = tb.adj_stride;
  // the slice: entry (j, k) for column x0 + k (k < kMonoTx) or row y0 + k - kMonoTx
  for (int i = threadIdx.x; i < sp.count * kMonoSl; i += kThreads) {
    const int j = i / kMonoSl, k = i % kMonoSl;
    const bool ok = k < kMonoTx ? k < lx : k - kMonoTx < ly;
    const int u = k < kMonoTx ? x0 + k : y0 + k - kMonoTx;
    if (!ADJ) {
      sa[i] = ok ? tb.i0[j * n + u] : 0;
      stt[i] = ok ? tb.t[j * n + u] : 0.f;
    } else {
      sa[i] = ok ? tb.adj_first[j * n + u] : 0;
      sc[i] = ok ? tb.adj_cnt[j * n + u] : 0;
    }
  }
  if (ADJ && TAPS > 0) {
    lds_fill<8>(sw, sp.count * kMonoSl * st, [&](int i) {
      const int e = i / st, w = i % st;
      const int j = e / kMonoSl, k = e % kMonoSl;
      const bool ok = k < kMonoTx ? k < lx : k - kMonoTx < ly;
      const int u = k < kMonoTx ? x0 + k : y0 + k - kMonoTx;
      return ok ? tb.adj_w[((size_t)j * n + u) * st + w] : 0.f;
    });
  }
  __syncthreads();
  // the spans clamped to the frame: samples outside it read zero
  int2 sx = mono_span<ADJ>(sp.count, sa, sc, 0, lx, spans);
  int2 sy = mono_span<ADJ>(sp.count, sa, sc, kMonoTx, ly, spans);
  sy = make_int2(max(sy.x, 0), min(sy.y, n - 1));
  sx = make_int2(max(sx.x, 0), min(sx.y, n - 1));
  const int rh = sy.y - sy.x + 1, rw = sx.y - sx.x + 1;
  const bool staged = rh > 0 && rw > 0 && rh * rw <= kMonoLds;
  if (staged) lds_fill<8>(reg, rh * rw, [&](int i) { return m[(size_t)(sy.x + i / rw) * n + sx.x + i % rw]; });
  __syncthreads();
  float* op = out + (size_t)pat * nn;
  const float ss = staged ? mono_outputs<ADJ, TAPS, true>(m, reg, sy.x, sx.x, rw, n, sp, tb, x0, y0, sa, stt, sc, sw, op)
                          : mono_outputs<ADJ, TAPS, false>(m, reg, sy.x, sx.x, rw, n, sp, tb, x0, y0, sa, stt, sc, sw, op);
  const double tot = block_sum_d((double)ss, red);
  if (threadIdx.x == 0) part[(size_t)pat * gridDim.x + blockIdx.x] = tot;
}

// Per pattern: sum of the block partials in order (blocks1 of part, the operator's tiles;
// blocks2 of part2, the element-wise kernels' blocks).  mode 0: alpha = gamma / |q|^2.
// mode 1: gamma_new = |s|^2, beta = gamma_new / gamma (0 while gamma is 0, as at the
// start), gamma = gamma_new, and the residual norm sqrt(part2) into res[pattern][slot].
__global__ __launch_bounds__(64) void k_mono_scalar(const double* __restrict__ part, const double* __restrict__ part2,
                                                    int blocks1, int blocks2, int mode, double* __restrict__ gamma,
                                                    double* __restrict__ coefv, float* __restrict__ res, int slot,
                                                    int res_stride) {
  const int pat = blockIdx.x;
  const double* p1 = part + (size_t)pat * blocks1;
  const double* p2 = part2 ? part2 + (size_t)pat * blocks2 : nullptr;
  // lane l sums blocks l, l + 64, ... in order; the 64 lane sums combine in a fixed butterfly
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < blocks1; i += 64) a += p1[i];
  if (p2)
    for (int i = threadIdx.x; i < blocks2; i += 64) b += p2[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    coefv[pat] = (a > 0.0) ? gamma[pat] / a : 0.0;
  } else {
    const double g = gamma[pat];
    coefv[pat] = (g > 0.0) ? a / g : 0.0;
    gamma[pat] = a;
    if (res) res[(size_t)pat * res_stride + slot] = (float)sqrt(b);
  }
}

// x += alpha p, r -= alpha q; part[pattern][block] = sum r^2.
__global__ __launch_bounds__(kThreads) void k_mono_xr(float* __restrict__ x, float* __restrict__ r,
                                                      const float* __restrict__ p, const float* __restrict__ q,
                                                      const double* __restrict__ alpha, int nn,
                                                      double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const int pat = blockIdx.y;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  const float a = (float)alpha[pat];
  float rv = 0.f;
  if (e < nn) {
    const size_t i = (size_t)pat * nn + e;
    x[i] += a * p[i];
    rv = r[i] - a * q[i];
    r[i] = rv;
  }
  const double tot = block_sum_d((double)rv * (double)rv, red);
  if (threadIdx.x == 0) part[(size_t)pat * gridDim.x + blockIdx.x] = tot;
}

// p = s + beta p (beta = 0 at the start: p = s); at the start also x = 0, r = b and part = |b|^2.
__global__ __launch_bounds__(kThreads) void k_mono_p(float* __restrict__ p, const float* __restrict__ s,
                                                     const double* __restrict__ beta, int nn) {
  const int pat = blockIdx.y;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= nn) return;
  const size_t i = (size_t)pat * nn + e;
  p[i] = s[i] + (float)beta[pat] * p[i];
}
__global__ __launch_bounds__(kThreads) void k_mono_start(const float* __restrict__ b, float* __restrict__ x,
                                                         float* __restrict__ r, float* __restrict__ p, int nn,
                                                         double* __restrict__ part, double* __restrict__ gamma) {
  __shared__ double red[kThreads / 64];
  const int pat = blockIdx.y;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  float bv = 0.f;
  if (e < nn) {
    const size_t i = (size_t)pat * nn + e;
    bv = b[i];
    x[i] = 0.f;
    r[i] = bv;
    p[i] = 0.f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) gamma[pat] = 0.0;
  const double tot = block_sum_d((double)bv * (double)bv, red);
  if (threadIdx.x == 0) part[(size_t)pat * gridDim.x + blockIdx.x] = tot;
}

hipError_t launch_mono_cgls(const float* b, float* x, const MonoWork& w, int n, int n_pat, int k_iters, float* res,
                            hipStream_t s) {
  const int nn = n * n;
  const int blocks = (nn + kThreads - 1) / kThreads;
  const int tiles = mono_tiles(n);
  const dim3 grid(blocks, n_pat), tgrid(tiles, n_pat);
  const int rs = k_iters + 1;
  const int cnt = w.spec.count, st = w.tab.adj_stride, mt = w.tab.adj_max;
  // the adjoint with its column taps in registers when the slice fits (under the 64 KiB per block)
  const int taps = mono_lds_bytes(cnt, st, true) > 60 * 1024 ? 0 : mt <= 2 ? 2 : mt <= 3 ? 3 : mt <= 4 ? 4 : mt <= 8 ? 8 : 0;
  auto adj_kernel = taps == 2   ? k_mono_apply<true, 2>
                    : taps == 3 ? k_mono_apply<true, 3>
                    : taps == 4 ? k_mono_apply<true, 4>
                    : taps == 8 ? k_mono_apply<true, 8>
                                : k_mono_apply<true, 0>;
  const size_t adj_lds = mono_lds_bytes(cnt, st, taps > 0), fwd_lds = mono_lds_bytes(cnt, st, false);
  pty_launch(k_mono_start, grid, dim3(kThreads), 0, s, b, x, w.r, w.p, nn, w.part2, w.gamma);
  pty_launch(adj_kernel, tgrid, dim3(kThreads), adj_lds, s, (const float*)w.r, w.s, w.spec, w.tab, n, w.part);
  pty_launch(k_mono_scalar, dim3(n_pat), dim3(64), 0, s, (const double*)w.part, (const double*)w.part2, tiles, blocks,
             1, w.gamma, w.coef, res, 0, rs);
  // the start's beta is 0 (gamma was 0): p = s
  pty_launch(k_mono_p, grid, dim3(kThreads), 0, s, w.p, (const float*)w.s, (const double*)w.coef, nn);
  for (int k = 0; k < k_iters; ++k) {
    pty_launch(k_mono_apply<false, 0>, tgrid, dim3(kThreads), fwd_lds, s, (const float*)w.p, w.q, w.spec, w.tab, n, w.part);
    pty_launch(k_mono_scalar, dim3(n_pat), dim3(64), 0, s, (const double*)w.part, (const double*)nullptr, tiles,
               blocks, 0, w.gamma, w.coef, (float*)nullptr, 0, rs);
    pty_launch(k_mono_xr, grid, dim3(kThreads), 0, s, x, w.r, (const float*)w.p, (const float*)w.q,
               (const double*)w.coef, nn, w.part2);
    pty_launch(adj_kernel, tgrid, dim3(kThreads), adj_lds, s, (const float*)w.r, w.s, w.spec, w.tab, n, w.part);
    pty_launch(k_mono_scalar, dim3(n_pat), dim3(64), 0, s, (const double*)w.part, (const double*)w.part2, tiles,
               blocks, 1, w.gamma, w.coef, res, k + 1, rs);
    pty_launch(k_mono_p, grid, dim3(kThreads), 0, s, w.p, (const float*)w.s, (const double*)w.coef, nn);
  }
  return hipGetLastError();
}

int mono_part_count(int n) { return max(mono_tiles(n), (n * n + kThreads - 1) / kThreads); }

int mono_adj_stride(const MonoSpectrum& sp) {
  float smin = sp.scale[0];
  for (int j = 1; j < sp.count; ++j) smin = fminf(smin, sp.scale[j]);
  return (int)floorf(2.0f / smin) + 3;
}

hipError_t launch_mono_tables(const MonoWork& w, int n, hipStream_t s) {
  const dim3 grid((n + kThreads - 1) / kThreads, w.spec.count);
  pty_launch(k_mono_fwd_table, grid, dim3(kThreads), 0, s, w.spec, w.tab, n);
  pty_launch(k_mono_adj_table, grid, dim3(kThreads), 0, s, w.spec, w.tab, n);
  return hipGetLastError();
}

}  // namespace pty
