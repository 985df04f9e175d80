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

// out = C in (ADJ false) or C^T in (ADJ true) for every pattern; part[pattern][block] = sum out^2.
// The adjoint sums, for each wavelength, its row weights in ascending pixel order, each
// row's column weights in ascending order (zero weights skipped).
template <bool ADJ>
__global__ __launch_bounds__(kThreads) void k_mono_apply(const float* __restrict__ in, float* __restrict__ out,
                                                         MonoSpectrum sp, MonoTables tb, int n,
                                                         double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const size_t nn = (size_t)n * n;
  const int pat = blockIdx.y;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  const float* m = in + (size_t)pat * nn;
  float val = 0.f;
  if (e < n * n) {
    const int uy = e / n, ux = e - uy * n;
    for (int j = 0; j < sp.count; ++j) {
      float acc = 0.f;
      if (!ADJ) {
        const int iy = tb.i0[j * n + uy], ix = tb.i0[j * n + ux];
        const float ty = tb.t[j * n + uy], tx = tb.t[j * n + ux];
        const float r0 = (1.0f - tx) * mono_at(m, n, iy, ix) + tx * mono_at(m, n, iy, ix + 1);
        const float r1 = (1.0f - tx) * mono_at(m, n, iy + 1, ix) + tx * mono_at(m, n, iy + 1, ix + 1);
        acc = (1.0f - ty) * r0 + ty * r1;
      } else {
        const int st = tb.adj_stride;
        const int ay = tb.adj_first[j * n + uy], ax = tb.adj_first[j * n + ux];
        const int cy = tb.adj_cnt[j * n + uy], cx = tb.adj_cnt[j * n + ux];
        const float* wy = tb.adj_w + ((size_t)j * n + uy) * st;
        const float* wx = tb.adj_w + ((size_t)j * n + ux) * st;
        for (int a = 0; a < cy; ++a) {
          const float wa = wy[a];
          if (wa == 0.f) continue;
          const float* mr = m + (size_t)(ay + a) * n + ax;
          float row = 0.f;
          for (int b = 0; b < cx; ++b) {
            const float wb = wx[b];
            if (wb != 0.f) row += wb * mr[b];
          }
          acc += wa * row;
        }
      }
      val += sp.coef[j] * acc;
    }
    out[(size_t)pat * nn + e] = val;
  }
  const double tot = block_sum_d((double)val * (double)val, red);
  if (threadIdx.x == 0) part[(size_t)pat * gridDim.x + blockIdx.x] = tot;
}

// Per pattern: sum of the block partials in order.  mode 0: alpha = gamma / |q|^2.
// mode 1: gamma_new = |s|^2, beta = gamma_new / gamma (0 while gamma is 0, as at the
// start), gamma = gamma_new, and the residual norm sqrt(part2) into res[pattern][slot].
__global__ __launch_bounds__(64) void k_mono_scalar(const double* __restrict__ part, const double* __restrict__ part2,
                                                    int blocks, int mode, double* __restrict__ gamma,
                                                    double* __restrict__ coefv, float* __restrict__ res, int slot,
                                                    int res_stride) {
  const int pat = blockIdx.x;
  const double* p1 = part + (size_t)pat * blocks;
  const double* p2 = part2 ? part2 + (size_t)pat * blocks : nullptr;
  // lane l sums blocks l, l + 64, ... in order; the 64 lane sums combine in a fixed butterfly
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < blocks; i += 64) {
    a += p1[i];
    if (p2) b += p2[i];
  }
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
  const dim3 grid(blocks, n_pat);
  const int rs = k_iters + 1;
  pty_launch(k_mono_start, grid, dim3(kThreads), 0, s, b, x, w.r, w.p, nn, w.part2, w.gamma);
  pty_launch(k_mono_apply<true>, grid, dim3(kThreads), 0, s, (const float*)w.r, w.s, w.spec, w.tab, n, w.part);
  pty_launch(k_mono_scalar, dim3(n_pat), dim3(64), 0, s, (const double*)w.part, (const double*)w.part2, blocks, 1,
             w.gamma, w.coef, res, 0, rs);
  // the start's beta is 0 (gamma was 0): p = s
  pty_launch(k_mono_p, grid, dim3(kThreads), 0, s, w.p, (const float*)w.s, (const double*)w.coef, nn);
  for (int k = 0; k < k_iters; ++k) {
    pty_launch(k_mono_apply<false>, grid, dim3(kThreads), 0, s, (const float*)w.p, w.q, w.spec, w.tab, n, w.part);
    pty_launch(k_mono_scalar, dim3(n_pat), dim3(64), 0, s, (const double*)w.part, (const double*)nullptr, blocks,
               0, w.gamma, w.coef, (float*)nullptr, 0, rs);
    pty_launch(k_mono_xr, grid, dim3(kThreads), 0, s, x, w.r, (const float*)w.p, (const float*)w.q,
               (const double*)w.coef, nn, w.part2);
    pty_launch(k_mono_apply<true>, grid, dim3(kThreads), 0, s, (const float*)w.r, w.s, w.spec, w.tab, n, w.part);
    pty_launch(k_mono_scalar, dim3(n_pat), dim3(64), 0, s, (const double*)w.part, (const double*)w.part2, blocks,
               1, w.gamma, w.coef, res, k + 1, rs);
    pty_launch(k_mono_p, grid, dim3(kThreads), 0, s, w.p, (const float*)w.s, (const double*)w.coef, nn);
  }
  return hipGetLastError();
}

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
