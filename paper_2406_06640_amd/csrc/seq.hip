// Sequential pc-ePIE for small frames (gfx950): one workgroup runs a whole
// iteration of one reconstruction with batch size 1 -- the loop of Fig. 1 over
// the iteration's positions, each update applied before the next position
// starts -- so the per-position chain costs one launch's worth of work instead
// of seven launches.  A table of independent reconstructions runs one
// workgroup per case in the same launch.
//
// Per position (box o at r_n, K modes, frames of side N <= 64 kept in LDS):
//   exit waves o P_k, 2D transform (rows then columns, each 1D pass scaled by
//   N^-1/2: the unitary DFT of Eq. 1) of every mode, Psi_0 kept in LDS and
//   further modes parked in the work frames X[0][k]; the incoherent mode sum, the separable Gaussian blur of the
//   amplitude (Eq. 6) or the intensity (Eq. 2), vertical then horizontal, the
//   modulus factor and the position's data error (box 1); per mode
//   Psi' = f Psi_k, inverse transform, dpsi = psi' - o P_k, the object
//   numerator sum_k conj(P_k) dpsi_k and the probe update
//   P_k += beta conj(o) dpsi_k / ((1 - g) |o|^2 + g max |o|^2) from the
//   pre-update box; then O += alpha N_O / ((1 - g) W + g max W) over the box
//   with W = sum_k |P_k|^2 of the pre-update probe; inside a constraint window
//   the complex constraint of Eq. (9)-(11) over the box.  The same arithmetic
//   as a batch of one position on the batch passes, in one workgroup.
// Global memory written by one position (object, probe, parked frames) is read
// by the next only after a workgroup barrier, which orders it for the waves of
// the workgroup (they share one CU and its L1).
#include "kernels_dev.hpp"

namespace pty {

bool seq_supported(int n, bool near_field) {
  return !near_field && (n == 16 || n == 32 || n == 48 || n == 64);
}

constexpr int kSlideHalf = 5;  // blur half-width held in the sliding windows

template <int N>
struct SeqLds {
  using RowF = Frame<N, N, false>;
  using ColF = Frame<N, N, true>;
  static constexpr int ROW = RowF::ELEMS;  // float2, row-pass layout
  static constexpr int COL = ColF::ELEMS;  // float2, column-pass layout
  // tw [N] | row buffer | column buffer | box [N^2] float2 | mode-0 frame [N^2] float2 | factor [N][N + 1] float
  static constexpr size_t BYTES =
      sizeof(float2) * ((size_t)N + ROW + COL + 2 * (size_t)N * N) + sizeof(float) * (size_t)N * (N + 1);
};

template <int N>
__global__ __launch_bounds__(kThreads) void k_seq_iter(const CaseDesc* __restrict__ cases, const int* __restrict__ it_ptr) {
  using RowF = Frame<N, N, false>;
  using ColF = Frame<N, N, true>;
  constexpr int SR = RegShape<N, N>::STORE_SLOTS;
  constexpr int LR = RegShape<N, N>::LOAD_SLOTS;
  constexpr int NN = N * N;
  constexpr int EP = (NN + kThreads - 1) / kThreads;  // plain elements per thread
  // Blur by sliding windows when the frame splits into whole line segments: a thread
  // owns RL consecutive elements of one column (vertical pass) and then of one row
  // (horizontal pass), loads its window once and applies every tap from registers.
  // Windows hold kSlideHalf taps each side (the paper's 11 x 11 kernel); wider
  // kernels take the per-tap path.
  constexpr bool SLIDE = kThreads % N == 0 && NN % kThreads == 0;
  constexpr int RL = SLIDE ? NN / kThreads : 1;  // elements per thread along a line
  constexpr int WL = RL + 2 * kSlideHalf;        // window length
  constexpr int S1 = N + 1;                      // padded row stride (horizontal pass input, factor)
  extern __shared__ float2 sm[];
  __shared__ double red[kThreads / 64];
  __shared__ double2 redd[kThreads / 64];
  __shared__ float redf[kThreads / 64];
  __shared__ float sgx[kMaxHalf + 1], sgy[kMaxHalf + 1];
  const CaseDesc* cs = cases + blockIdx.y;
  const DevParams& p = cs->p;
  const DevBufsG d = global_bufs(cs->d);
  const int it = *it_ptr;
  const int flags = cs->flags[it];
  const int np = cs->n_pos;
  const int* order = cs->order + (size_t)it * np;
  float2* tw = sm;
  float2* rowbuf = sm + N;
  float2* colbuf = rowbuf + SeqLds<N>::ROW;
  float2* obox = colbuf + SeqLds<N>::COL;
  float2* psi0 = obox + NN;  // Psi of mode 0 stays on chip; further modes are parked in X
  float* fbuf = reinterpret_cast<float*>(psi0 + NN);
  float* t0 = reinterpret_cast<float*>(rowbuf);  // blur buffers, free between the transforms
  float* t1 = reinterpret_cast<float*>(colbuf);
  for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = d.tw[i];
  if (threadIdx.x <= kMaxHalf) {
    sgx[threadIdx.x] = p.gx[threadIdx.x];
    sgy[threadIdx.x] = p.gy[threadIdx.x];
  }
  const int K = p.k, W = p.w_obj, h = p.ks_half;
  const float scale = rsqrtf((float)N);
  const bool inten = p.blur_intensity != 0;
  const bool probe_upd = (flags & FLAG_PROBE) != 0;
  const int err_slots = cs->n_err_part / np;
  float2* X = d.X;
  __syncthreads();
  for (int step = 0; step < np; ++step) {
    const int pat = order[step];
    const int2 rc = d.pos[pat];
    // box into LDS (row-major) and its largest |o|^2; the measured amplitudes are
    // fetched with it (every load of the position's first round trip issued together)
    float vmax = 0.f;
    float av[EP];
    {
      const float* amp = d.amp + (size_t)pat * NN;
      float2 ob[EP];
#pragma unroll
      for (int j = 0; j < EP; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (NN % kThreads != 0 && e >= NN) continue;
        const int y = e / N, x = e - y * N;
        ob[j] = d.obj[(size_t)(rc.x + y) * W + rc.y + x];
        // sliding layout: row threadIdx.x % N, columns (threadIdx.x / N) RL + j
        av[j] = SLIDE ? amp[(threadIdx.x % N) * N + (threadIdx.x / N) * RL + j] : amp[e];
      }
#pragma unroll
      for (int j = 0; j < EP; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (NN % kThreads != 0 && e >= NN) continue;
        obox[e] = ob[j];
        vmax = fmaxf(vmax, ob[j].x * ob[j].x + ob[j].y * ob[j].y);
      }
    }
    // mode 0 of the probe at the forward pass's input slots and the inverse pass's output slots
    float2 pf0[LR], pi0[SR];
    for_load_slots<N, N, false>([&](int s, int y, int x) { pf0[s] = d.probe[y * N + x]; });
    for_store_slots<N, N, false>([&](int s, int y, int x) { pi0[s] = d.probe[y * N + x]; });
    vmax = block_max_f(vmax, redf);  // also: the box is visible to every thread
    // forward transforms of every mode; |Psi_k|^2 summed in the column pass's store slots
    float acc[SR];
#pragma unroll
    for (int i = 0; i < SR; ++i) acc[i] = 0.f;
    for (int k = 0; k < K; ++k) {
      const float2* pk = d.probe + (size_t)k * NN;
      float2* xk = X + (size_t)k * NN;
      float2 v[LR];
      auto load_row = [&](int s, int y, int x) {
        return cmul(obox[y * N + x], k == 0 ? pf0[s] : pk[y * N + x]);
      };
      fft_gather<N, N, false>(v, load_row);
      fft_first<N, N, false, false>(v, rowbuf);
      auto to_col = [&](int s, int y, int u, float2 z) { colbuf[ColF::lidx(u, y)] = cscale(z, scale); };
      fft_rest<N, N, false, false>(v, rowbuf, tw, to_col);
      __syncthreads();  // every row-pass output is in the column buffer
      auto from_col = [&](int s, int u, int y) { return colbuf[ColF::lidx(u, y)]; };
      auto park = [&](int s, int u, int y, float2 z) {
        z = cscale(z, scale);
        if (k == 0)
          psi0[y * N + u] = z;
        else
          xk[y * N + u] = z;
        acc[s] += z.x * z.x + z.y * z.y;
      };
      fft_reg<N, N, true, false, true>(colbuf, tw, from_col, park);
      __syncthreads();  // the column buffer is read before the next mode rewrites it
    }
    // box 1: mode sum -> blur (vertical, then horizontal) -> modulus factor; data error
    for_store_slots<N, N, true>([&](int s, int u, int y) { t0[y * N + u] = inten ? acc[s] : sqrtf(acc[s]); });
    __syncthreads();
    double err = 0.0;
    // modulus factor and data error of element (y, x) from its blurred value g
    auto factor_at = [&](int y, int x, float g, float a) {
      float ag, f;
      if (inten) {
        ag = sqrtf(g);
        f = a / sqrtf(g + p.eps * p.eps);
      } else {
        ag = g;
        f = a / (g + p.eps);
      }
      fbuf[y * S1 + x] = f;
      const double dd = (double)a - (double)ag;
      err += dd * dd;
    };
    if (SLIDE && h <= kSlideHalf) {
      float* t1p = t1;  // [N][S1]
      {
        const int x = threadIdx.x % N, y0 = (threadIdx.x / N) * RL;
        float win[WL];
#pragma unroll
        for (int i = 0; i < WL; ++i) {
          const int off = i - kSlideHalf;
          win[i] = (off >= -h && off < RL + h) ? t0[wrap(y0 + off, N) * N + x] : 0.f;
        }
        float gv[RL];
#pragma unroll
        for (int i = 0; i < RL; ++i) gv[i] = sgy[0] * win[i + kSlideHalf];
#pragma unroll
        for (int dy = 1; dy <= kSlideHalf; ++dy) {
          if (dy > h) break;
          const float gd = sgy[dy];
#pragma unroll
          for (int i = 0; i < RL; ++i) gv[i] += gd * (win[i + kSlideHalf - dy] + win[i + kSlideHalf + dy]);
        }
#pragma unroll
        for (int i = 0; i < RL; ++i) t1p[(y0 + i) * S1 + x] = gv[i];
      }
      __syncthreads();
      {
        const int y = threadIdx.x % N, x0 = (threadIdx.x / N) * RL;
        float win[WL];
#pragma unroll
        for (int i = 0; i < WL; ++i) {
          const int off = i - kSlideHalf;
          win[i] = (off >= -h && off < RL + h) ? t1p[y * S1 + wrap(x0 + off, N)] : 0.f;
        }
        float gv[RL];
#pragma unroll
        for (int i = 0; i < RL; ++i) gv[i] = sgx[0] * win[i + kSlideHalf];
#pragma unroll
        for (int dx = 1; dx <= kSlideHalf; ++dx) {
          if (dx > h) break;
          const float gd = sgx[dx];
#pragma unroll
          for (int i = 0; i < RL; ++i) gv[i] += gd * (win[i + kSlideHalf - dx] + win[i + kSlideHalf + dx]);
        }
#pragma unroll
        for (int i = 0; i < RL; ++i) factor_at(y, x0 + i, gv[i], av[i]);
      }
    } else {
      {
        float gv[EP];
#pragma unroll
        for (int j = 0; j < EP; ++j) {
          const int e = threadIdx.x + j * kThreads;
          gv[j] = (NN % kThreads != 0 && e >= NN) ? 0.f : sgy[0] * t0[e];
        }
        for (int dy = 1; dy <= h; ++dy) {
          const float gd = sgy[dy];
#pragma unroll
          for (int j = 0; j < EP; ++j) {
            const int e = threadIdx.x + j * kThreads;
            if (NN % kThreads != 0 && e >= NN) continue;
            const int y = e / N, x = e - y * N;
            gv[j] += gd * (t0[wrap(y - dy, N) * N + x] + t0[wrap(y + dy, N) * N + x]);
          }
        }
#pragma unroll
        for (int j = 0; j < EP; ++j) {
          const int e = threadIdx.x + j * kThreads;
          if (NN % kThreads == 0 || e < NN) t1[e] = gv[j];
        }
      }
      __syncthreads();
      {
        float gv[EP];
#pragma unroll
        for (int j = 0; j < EP; ++j) {
          const int e = threadIdx.x + j * kThreads;
          gv[j] = (NN % kThreads != 0 && e >= NN) ? 0.f : sgx[0] * t1[e];
        }
        for (int dx = 1; dx <= h; ++dx) {
          const float gd = sgx[dx];
#pragma unroll
          for (int j = 0; j < EP; ++j) {
            const int e = threadIdx.x + j * kThreads;
            if (NN % kThreads != 0 && e >= NN) continue;
            const int x = e % N;
            const float* row = t1 + (e - x);
            gv[j] += gd * (row[wrap(x - dx, N)] + row[wrap(x + dx, N)]);
          }
        }
#pragma unroll
        for (int j = 0; j < EP; ++j) {
          const int e = threadIdx.x + j * kThreads;
          if (NN % kThreads != 0 && e >= NN) continue;
          factor_at(e / N, e % N, gv[j], av[j]);
        }
      }
    }
    const double etot = block_sum_d(err, red);  // also: fbuf and the blur buffers are settled
    if (threadIdx.x < err_slots) d.err_part[(size_t)pat * err_slots + threadIdx.x] = threadIdx.x == 0 ? etot : 0.0;
    // inverse transforms; object numerator, probe update
    float2 num[SR];
    float pw[SR];
#pragma unroll
    for (int i = 0; i < SR; ++i) {
      num[i] = make_float2(0.f, 0.f);
      pw[i] = 0.f;
    }
    for (int k = 0; k < K; ++k) {
      float2* pk = d.probe + (size_t)k * NN;
      const float2* xk = X + (size_t)k * NN;
      // P_k at the row pass's output slots, fetched before the transforms
      float2 pvs[SR];
      for_store_slots<N, N, false>([&](int s, int y, int x) { pvs[s] = k == 0 ? pi0[s] : pk[y * N + x]; });
      auto load_icol = [&](int s, int u, int y) {
        const float2 z = k == 0 ? psi0[y * N + u] : xk[y * N + u];
        const float f = fbuf[y * S1 + u];
        return make_float2(z.x * f, z.y * f);  // no contraction anywhere in this file (fft_lds.hpp)
      };
      auto to_row = [&](int s, int u, int y, float2 z) { rowbuf[RowF::lidx(y, u)] = cscale(z, scale); };
      fft_reg<N, N, true, true>(colbuf, tw, load_icol, to_row);
      __syncthreads();  // every column-pass output is in the row buffer
      auto from_row = [&](int s, int y, int x) { return rowbuf[RowF::lidx(y, x)]; };
      auto update = [&](int s, int y, int x, float2 z) {
        const int e = y * N + x;
        const float2 psi_new = cscale(z, scale);
        const float2 o = obox[e];
        const float2 pv = pvs[s];
        const float2 dpsi = csub(psi_new, cmul(o, pv));
        num[s] = cadd(num[s], cmulc(dpsi, pv));
        pw[s] += pv.x * pv.x + pv.y * pv.y;
        if (probe_upd) {
          const float den = (1.0f - p.gamma_probe) * (o.x * o.x + o.y * o.y) + p.gamma_probe * vmax;
          if (den > 0.f) {
            const float sc = p.probe_step / den;
            const float2 c = cmulc(dpsi, o);
            pk[e] = make_float2(pv.x + sc * c.x, pv.y + sc * c.y);
          }
        }
      };
      fft_reg<N, N, false, true, true>(rowbuf, tw, from_row, update);
      __syncthreads();  // the row buffer is read before the next mode rewrites it
    }
    // object update over the box (denominators from the pre-update probe power)
    float wmax = 0.f;
#pragma unroll
    for (int i = 0; i < SR; ++i) wmax = fmaxf(wmax, pw[i]);
    wmax = block_max_f(wmax, redf);
    const bool cc = (flags & FLAG_CC) != 0;
    float sa = 0.f, sp = 0.f;
    float lna_s[SR], phi_s[SR];  // ln A and phi of the updated box, reused by Eq. (9)-(10)
    for_store_slots<N, N, false>([&](int s, int y, int x) {
      const int e = y * N + x;
      float2 o = obox[e];
      const float den = (1.0f - p.gamma_obj) * pw[s] + p.gamma_obj * wmax;
      if (den > 0.f) {
        const float sc = p.obj_step / den;
        o.x += sc * num[s].x;
        o.y += sc * num[s].y;
        d.obj[(size_t)(rc.x + y) * W + rc.y + x] = o;
      }
      if (cc) {
        lna_s[s] = cc_ln_amp(o);
        phi_s[s] = cc_phase(o);
        sa += fabsf(lna_s[s]);
        sp += fabsf(phi_s[s]);
      }
    });
    if (cc) {
      // box 2: C-bar of Eq. (11) over the box, then Eq. (9)-(10)
      const double2 tot = block_sum_d2((double)sa, (double)sp, redd);
      if (tot.y > 0.0) {
        float cbar = (float)(tot.x / tot.y);
        cbar = fminf(fmaxf(cbar, p.cbar_min), p.cbar_max);
        const float inv_c = 1.0f / cbar;
        const float a1 = p.alpha1, a2 = p.alpha2;
        for_store_slots<N, N, false>([&](int s, int y, int x) {
          d.obj[(size_t)(rc.x + y) * W + rc.y + x] = cc_apply_lp(lna_s[s], phi_s[s], cbar, inv_c, a1, a2);
        });
      }
    }
    __syncthreads();  // object, probe and LDS settled before the next position
  }
  // the probe-power map sum_k |P_k|^2 of the final probe, both copies (batch passes read it)
  for (int e = threadIdx.x; e < NN; e += kThreads) {
    float s2 = 0.f;
    for (int k = 0; k < K; ++k) {
      const float2 v = d.probe[(size_t)k * NN + e];
      s2 += v.x * v.x + v.y * v.y;
    }
    d.pw[e] = s2;
    d.pw[(size_t)NN + e] = s2;
  }
}

template <int N>
static hipError_t seq_t(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s) {
  // more than 64 KiB of dynamic LDS for N = 64: allowed once per instantiation
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(k_seq_iter<N>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)SeqLds<N>::BYTES);
  if (attr != hipSuccess) return attr;
  pty_launch(k_seq_iter<N>, dim3(1, t.n_cases), dim3(kThreads), SeqLds<N>::BYTES, s, cases, it);
  return hipGetLastError();
}

hipError_t launch_seq_iter(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s) {
  if (t.near_field) return hipErrorInvalidValue;
  switch (t.n) {
    case 16: return seq_t<16>(cases, t, it, s);
    case 32: return seq_t<32>(cases, t, it, s);
    case 48: return seq_t<48>(cases, t, it, s);
    case 64: return seq_t<64>(cases, t, it, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pty
