// Far-field propagation as dense complex GEMMs on BF16 matrix cores (gfx950).
//
// The unitary 2D DFT of a frame X is F X F with F[u][x] = exp(-2 pi i u x / N) / sqrt(N)
// (F is symmetric); the inverse uses conj(F).  Each frame is transformed by a
// "right" GEMM (every row times F) and a "left" GEMM (F times every column).
// Operands are split into two BF16 parts, x = x_hi + x_lo, f = f_hi + f_lo,
// and each real product is x_hi f_hi + x_hi f_lo + x_lo f_hi (the x_lo f_lo
// term, ~2^-18 relative, is dropped), accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16.  A complex product is four real products.
// The modulus constraint, the step normalisation and the probe update stay
// in FP32 (the same kernels as the FFT path).
//
// MFMA 16x16x32 operand layout (lane l of a wave64): A[row = l % 16][k = 8 (l / 16) + i],
// B[k = 8 (l / 16) + i][col = l % 16], i = 0..7; result C[row = 4 (l / 16) + i][col = l % 16], i = 0..3.
//
// This file is included by kernels.hip (it shares its device helpers).

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace pty {

__device__ __forceinline__ floatx4 mma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void split8(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const __bf16 h = (__bf16)v[i];
    hi[i] = h;
    lo[i] = (__bf16)(v[i] - (float)h);
  }
}

__device__ __forceinline__ bf16x8 neg8(bf16x8 a) {
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = -a[i];
  return a;
}

// acc += (a_hi + a_lo)(b_hi + b_lo) without the lo*lo term
__device__ __forceinline__ floatx4 mma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, floatx4 c) {
  c = mma(ah, bh, c);
  c = mma(ah, bl, c);
  c = mma(al, bh, c);
  return c;
}

// DFT table planes (re_hi, re_lo, im_hi, im_lo) of F in MFMA fragment order:
// F[u][x] at [plane][u / 16][x / 32][16 ((x % 32) / 8) + u % 16][x % 8].  frag()
// returns lane `lane`'s 8 values of the 16 x 32 fragment rows 16 rt.., columns 32 kc..
// (row 16 rt + lane % 16, columns 32 kc + 8 (lane / 16) + 0..7): a wave reads 1 KB in a row.
struct DftPlanes {
  const __bf16* p;
  __device__ __forceinline__ bf16x8 frag(int plane, int n, int rt, int kc, int lane) const {
    return *reinterpret_cast<const bf16x8*>(p + ((((size_t)plane * (n / 16) + rt) * (n / 32) + kc) * 64 + lane) * 8);
  }
};

// Complex product of one 16 x 32 A fragment (split re/im) with one 32 x 16 B fragment,
// conj_b: use conj(B); with the negated pair of A given, na = -(a.ih, a.il) (conj_b
// false) or -(a.rh, a.rl) (conj_b true), so that no operand is negated per product:
// (ar + i ai)(br + i bi) = ar br - ai bi + i (ar bi + ai br);  conj(b): bi -> -bi.
struct CFrag {
  bf16x8 rh, rl, ih, il;
};
__device__ __forceinline__ void cmma_n(const CFrag& a, bf16x8 nah, bf16x8 nal, const CFrag& b, bool conj_b,
                                       floatx4& cr, floatx4& ci) {
  cr = mma3(a.rh, a.rl, b.rh, b.rl, cr);
  if (!conj_b) {
    cr = mma3(nah, nal, b.ih, b.il, cr);
    ci = mma3(a.rh, a.rl, b.ih, b.il, ci);
  } else {
    cr = mma3(a.ih, a.il, b.ih, b.il, cr);
    ci = mma3(nah, nal, b.ih, b.il, ci);
  }
  ci = mma3(a.ih, a.il, b.rh, b.rl, ci);
}
// A (F or conj F: conj_a) times B with the negated pair of B given, nb = -(b.ih, b.il)
// (conj_a false) or -(b.rh, b.rl) (conj_a true).  The BF16 products are exact in FP32,
// so a sign may sit on either operand of a product.
__device__ __forceinline__ void cmma_bn(const CFrag& a, const CFrag& b, bf16x8 nbh, bf16x8 nbl, bool conj_a,
                                        floatx4& cr, floatx4& ci) {
  cr = mma3(a.rh, a.rl, b.rh, b.rl, cr);
  if (!conj_a) {
    cr = mma3(a.ih, a.il, nbh, nbl, cr);
    ci = mma3(a.rh, a.rl, b.ih, b.il, ci);
    ci = mma3(a.ih, a.il, b.rh, b.rl, ci);
  } else {
    cr = mma3(a.ih, a.il, b.ih, b.il, cr);
    ci = mma3(a.rh, a.rl, b.ih, b.il, ci);
    ci = mma3(a.ih, a.il, nbh, nbl, ci);
  }
}

// Row or column groups of 16 per workgroup: every table fragment a wave loads
// serves kDftGroups groups (kDftGroups x 12 MFMAs per fragment load).  The frame
// operand is shared by the W waves of the workgroup: for each 32-wide k-chunk, wave
// w < kDftGroups loads and splits group w's slice once and stages it in LDS
// (double-buffered), loading the next chunk's slice while the current chunk's MFMAs
// run; the table fragments run two tiles ahead of the MFMAs.  W = 8 where N/16 splits
// into 8 equal shares of output tiles (two waves per SIMD, 64 accumulator registers
// each), 12 at N = 192 (one tile per wave), else 4.
constexpr int kDftGroups = 4;

// LDS stage of one chunk: [group][plane rh, rl, ih, il][lane] fragments.  The negated
// pair the complex product needs (-ih, -il or -rh, -rl) is formed in registers once
// per group and chunk by every reading wave.
struct DftStage {
  bf16x8 f[kDftGroups][4][64];
};
__device__ __forceinline__ void dft_stage_put(DftStage& st, int g, int lane, const float2* v) {
  float re[8], im[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    re[i] = v[i].x;
    im[i] = v[i].y;
  }
  bf16x8 rh, rl, ih, il;
  split8(re, rh, rl);
  split8(im, ih, il);
  st.f[g][0][lane] = rh;
  st.f[g][1][lane] = rl;
  st.f[g][2][lane] = ih;
  st.f[g][3][lane] = il;
}
__device__ __forceinline__ CFrag dft_stage_get(const DftStage& st, int g, int lane) {
  return CFrag{st.f[g][0][lane], st.f[g][1][lane], st.f[g][2][lane], st.f[g][3][lane]};
}

// Rows of every frame times F (or conj F): X[r][:] <- X[r][:] F, in place.
// Block = kDftGroups x 16 rows; wave w produces output columns [w N/W, (w+1) N/W)
// of every row group.  EXIT: the frames are the exit waves of batch `beta` (frame
// f = b K + k holds o_b P_k), formed while staging instead of read from X (which
// receives the transformed rows); the workgroup's 64 rows lie in one frame.
template <int N, bool INV, int W, bool EXIT>
__global__ __launch_bounds__(64 * W) void k_dft_right(float2* __restrict__ X, DftPlanes F, int rows,
                                                      const CaseDesc* __restrict__ cases, int beta,
                                                      const int* __restrict__ it) {
  constexpr int TPW = N / (16 * W);  // 16-column tiles per wave
  static_assert(W >= kDftGroups && TPW * 16 * W == N, "wave count");
  constexpr int G = kDftGroups;
  __shared__ DftStage stage[2];
  const int r0 = blockIdx.x * 16 * G;
  if (r0 >= rows) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, kq = lane >> 4;
  floatx4 cr[G][TPW], ci[G][TPW];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      cr[g][t] = floatx4{0.f, 0.f, 0.f, 0.f};
      ci[g][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  // A[row][k] = X[r0 + 16 g + row][k] per row group g; B[k][col] = F[col][k] for the
  // wave's columns w N/W + 16 t + lr, chunk kb
  auto load_b = [&](int kb, int t) {
    const int rt = w * TPW + t;
    return CFrag{F.frag(0, N, rt, kb, lane), F.frag(1, N, rt, kb, lane), F.frag(2, N, rt, kb, lane),
                 F.frag(3, N, rt, kb, lane)};
  };
  const bool stager = W == G || w < G;  // waves 0..G-1 stage one row group each
  // table fragments run two tiles ahead: b (this tile), b1 (the next), loads for the one after
  auto tile_at = [&](int kb, int t, CFrag& dst) {
    while (t >= TPW) {  // TPW may be 1: two tiles ahead can be two chunks ahead
      t -= TPW;
      ++kb;
    }
    if (kb * 32 < N) dst = load_b(kb, t);
  };
  CFrag b = load_b(0, 0), b1 = b;
  tile_at(0, 1, b1);
  const int srow = r0 + (stager ? w : 0) * 16 + lr;  // the row this lane stages
  const float2* xrow = X + (size_t)srow * N + kq * 8;
  // EXIT: this lane's row of o_b and of P_k (b, k from the frame of row srow)
  const float2* orow = nullptr;
  const float2* prow = nullptr;
  if constexpr (EXIT) {
    Batch bt;
    if (!open_batch(cases, beta, it, bt)) return;  // uniform: every thread leaves
    const DevParams& p = bt.cs->p;
    const DevBufsG d = global_bufs(bt.cs->d);
    const int f = srow / N, y = srow % N;
    const int b = f / p.k, k = f % p.k;
    const int2 rc = d.pos[bt.slots[b]];
    orow = d.obj + (size_t)(rc.x + y) * p.w_obj + rc.y + kq * 8;
    prow = d.probe + ((size_t)k * N + y) * N + kq * 8;
  }
  auto load_chunk = [&](int kc, float2* v) {
    if constexpr (EXIT) {
      float2 ov[8], pv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        ov[i] = orow[kc + i];
        pv[i] = prow[kc + i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = cmul(ov[i], pv[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = xrow[kc + i];
    }
  };
  float2 nx[8];
  if (stager) {
    load_chunk(0, nx);
    dft_stage_put(stage[0], w, lane, nx);
  }
  __syncthreads();
  for (int kc = 0, it = 0; kc < N; kc += 32, ++it) {
    const int cur = it & 1;
    const bool more = kc + 32 < N;
    if (more && stager) load_chunk(kc + 32, nx);
    CFrag a[G];
    bf16x8 na_h[G], na_l[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      a[g] = dft_stage_get(stage[cur], g, lane);
      na_h[g] = neg8(INV ? a[g].rh : a[g].ih);
      na_l[g] = neg8(INV ? a[g].rl : a[g].il);
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      // the table fragment two tiles ahead loads during this tile's MFMAs
      CFrag b2 = b1;
      tile_at(kc / 32, t + 2, b2);
#pragma unroll
      for (int g = 0; g < G; ++g) cmma_n(a[g], na_h[g], na_l[g], b, INV, cr[g][t], ci[g][t]);
      b = b1;
      b1 = b2;
    }
    if (more && stager) dft_stage_put(stage[cur ^ 1], w, lane, nx);
    // the next chunk is staged, and (after the last chunk) every wave has read the
    // block's rows before any is overwritten
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int col = (w * TPW + t) * 16 + lr;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        X[(size_t)(r0 + g * 16 + kq * 4 + i) * N + col] = make_float2(cr[g][t][i], ci[g][t][i]);
    }
}

// F (or conj F) times every column of each frame: X_f <- F X_f, in place.
// Block = kDftGroups x 16 columns of one frame (blockIdx.y); wave w produces rows
// [w N/W, (w+1) N/W) of every column group.
template <int N, bool INV, int W>
__global__ __launch_bounds__(64 * W) void k_dft_left(float2* __restrict__ X, DftPlanes F, int frames) {
  constexpr int TPW = N / (16 * W);
  static_assert(W >= kDftGroups && TPW * 16 * W == N, "wave count");
  constexpr int G = kDftGroups;
  __shared__ DftStage stage[2];
  const int f = blockIdx.y;
  if (f >= frames) return;
  const int c0 = blockIdx.x * 16 * G;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lc = lane & 15, kq = lane >> 4;
  float2* fr = X + (size_t)f * N * N;
  floatx4 cr[G][TPW], ci[G][TPW];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      cr[g][t] = floatx4{0.f, 0.f, 0.f, 0.f};
      ci[g][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  // B[k][col] = X[k][c0 + 16 g + col] per column group g; A[row][k] = F[row][k] for the
  // wave's rows w N/W + 16 t + lc, chunk kb
  auto load_a = [&](int kb, int t) {
    const int rt = w * TPW + t;
    return CFrag{F.frag(0, N, rt, kb, lane), F.frag(1, N, rt, kb, lane), F.frag(2, N, rt, kb, lane),
                 F.frag(3, N, rt, kb, lane)};
  };
  // table fragments run two tiles ahead: a (this tile), a1 (the next), loads for the one after
  auto tile_at = [&](int kb, int t, CFrag& dst) {
    while (t >= TPW) {  // TPW may be 1: two tiles ahead can be two chunks ahead
      t -= TPW;
      ++kb;
    }
    if (kb * 32 < N) dst = load_a(kb, t);
  };
  CFrag a = load_a(0, 0), a1 = a;
  tile_at(0, 1, a1);
  const bool stager = W == G || w < G;  // waves 0..G-1 stage one column group each
  const float2* xcol = fr + (size_t)(kq * 8) * N + c0 + (stager ? w : 0) * 16 + lc;
  float2 nx[8];
  if (stager) {
#pragma unroll
    for (int i = 0; i < 8; ++i) nx[i] = xcol[(size_t)i * N];
    dft_stage_put(stage[0], w, lane, nx);
  }
  __syncthreads();
  for (int kc = 0, it = 0; kc < N; kc += 32, ++it) {
    const int cur = it & 1;
    const bool more = kc + 32 < N;
    if (more && stager) {
#pragma unroll
      for (int i = 0; i < 8; ++i) nx[i] = xcol[(size_t)(kc + 32 + i) * N];
    }
    CFrag b[G];
    bf16x8 nb_h[G], nb_l[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      b[g] = dft_stage_get(stage[cur], g, lane);
      nb_h[g] = neg8(INV ? b[g].rh : b[g].ih);
      nb_l[g] = neg8(INV ? b[g].rl : b[g].il);
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      // the table fragment two tiles ahead loads during this tile's MFMAs
      CFrag a2 = a1;
      tile_at(kc / 32, t + 2, a2);
#pragma unroll
      for (int g = 0; g < G; ++g) cmma_bn(a, b[g], nb_h[g], nb_l[g], INV, cr[g][t], ci[g][t]);
      a = a1;
      a1 = a2;
    }
    if (more && stager) dft_stage_put(stage[cur ^ 1], w, lane, nx);
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int row0 = (w * TPW + t) * 16 + kq * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        fr[(size_t)(row0 + i) * N + c0 + g * 16 + lc] = make_float2(cr[g][t][i], ci[g][t][i]);
    }
}

// Side work of the batch (see side_job) as its own launch.
__global__ __launch_bounds__(kThreads) void k_dft_side(const CaseDesc* __restrict__ cases, int beta,
                                                       const int* __restrict__ it) {
  __shared__ SideScratch sc;
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  side_job(bt.cs->p, global_bufs(bt.cs->d), pw_copy(bt.flags, beta), bt.slots, bt.ns, blockIdx.x,
           (bt.flags & FLAG_PROBE) != 0, sc);
}

// q[b] = sum_k |Psi_k|^2 (intensity blur) or its square root (amplitude blur).
__global__ __launch_bounds__(kThreads) void k_dft_modsum(const CaseDesc* __restrict__ cases, int beta,
                                                         const int* __restrict__ it) {
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const int n = p.n, K = p.k;
  const size_t nn = (size_t)n * n;
  const int per = (n * n + kThreads - 1) / kThreads;
  const int b = blockIdx.x / per, pix = (blockIdx.x % per) * kThreads + threadIdx.x;
  if (b >= bt.ns || pix >= n * n) return;
  float s = 0.f;
  for (int k = 0; k < K; ++k) {
    const float2 v = d.X[((size_t)b * K + k) * nn + pix];
    s += v.x * v.x + v.y * v.y;
  }
  d.q[(size_t)b * nn + pix] = p.blur_intensity ? s : sqrtf(s);
}

// Separable periodic blur of q over a 32 x 32 tile (halo in LDS), the modulus
// factor of box 1, the data error, and Psi_k *= factor for every mode.
constexpr int kDftTile = 32;
__global__ __launch_bounds__(kThreads) void k_dft_blur_apply(const CaseDesc* __restrict__ cases, int beta,
                                                             const int* __restrict__ it) {
  constexpr int S = kDftTile + 2 * kMaxHalf;
  __shared__ float qs[S][S + 1];
  __shared__ float hs[S][kDftTile + 1];
  __shared__ double red[kThreads / 64];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const int n = p.n, K = p.k;
  const int tpr = n / kDftTile, tiles = tpr * tpr;
  const int b = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  if (b >= bt.ns) return;
  const int ty0 = (tile / tpr) * kDftTile, tx0 = (tile % tpr) * kDftTile;
  const int h = p.ks_half, s = kDftTile + 2 * h;
  const size_t nn = (size_t)n * n;
  const float* q = d.q + (size_t)b * nn;
  for (int e = threadIdx.x; e < s * s; e += kThreads) {
    const int yy = e / s, xx = e - yy * s;
    qs[yy][xx] = q[(size_t)wrap(ty0 - h + yy, n) * n + wrap(tx0 - h + xx, n)];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * kDftTile; e += kThreads) {
    const int yy = e / kDftTile, x = e - yy * kDftTile;
    float acc = p.gx[0] * qs[yy][x + h];
    for (int dx = 1; dx <= h; ++dx) acc += p.gx[dx] * (qs[yy][x + h - dx] + qs[yy][x + h + dx]);
    hs[yy][x] = acc;
  }
  __syncthreads();
  const int pat = bt.slots[b];
  const float* amp = d.amp + (size_t)pat * nn;
  float* dbgf = bt.cs->dbg.factor ? bt.cs->dbg.factor + (size_t)b * nn : nullptr;
  double err = 0.0;
  // the thread's kPx pixels: factors first, then per mode the loads of all of them,
  // with the next mode's loads issued before this mode's stores
  constexpr int kPx = kDftTile * kDftTile / kThreads;
  static_assert(kPx * kThreads == kDftTile * kDftTile, "whole pixels per thread");
  size_t idx[kPx];
  float f[kPx];
#pragma unroll
  for (int j = 0; j < kPx; ++j) {
    const int e = threadIdx.x + j * kThreads;
    const int y = e / kDftTile, x = e - y * kDftTile;
    float g = p.gy[0] * hs[y + h][x];
    for (int dy = 1; dy <= h; ++dy) g += p.gy[dy] * (hs[y + h - dy][x] + hs[y + h + dy][x]);
    idx[j] = (size_t)(ty0 + y) * n + tx0 + x;
    const float a = amp[idx[j]];
    float ag;
    if (p.blur_intensity) {
      ag = sqrtf(g);
      f[j] = a / sqrtf(g + p.eps * p.eps);
    } else {
      ag = g;
      f[j] = a / (g + p.eps);
    }
    if (dbgf) dbgf[idx[j]] = f[j];
    const double dd = (double)a - (double)ag;
    err += dd * dd;
  }
  float2* xb = d.X + (size_t)b * K * nn;
  float2 cur[kPx];
#pragma unroll
  for (int j = 0; j < kPx; ++j) cur[j] = xb[idx[j]];
  for (int k = 0; k < K; ++k) {
    float2 nxt[kPx];
#pragma unroll
    for (int j = 0; j < kPx; ++j) nxt[j] = k + 1 < K ? xb[(size_t)(k + 1) * nn + idx[j]] : cur[j];
#pragma unroll
    for (int j = 0; j < kPx; ++j) xb[(size_t)k * nn + idx[j]] = cscale(cur[j], f[j]);
#pragma unroll
    for (int j = 0; j < kPx; ++j) cur[j] = nxt[j];
  }
  const double tot = block_sum_d(err, red);
  if (threadIdx.x == 0) d.err_part[(size_t)pat * tiles + tile] = tot;
}

// psi' is in X: dpsi = psi' - o_b P_k; per-slot object numerator sum_k conj(P_k) dpsi_k;
// X <- conj(o_b) dpsi_k (the probe contributions).
__global__ __launch_bounds__(kThreads) void k_dft_delta(const CaseDesc* __restrict__ cases, int beta,
                                                        const int* __restrict__ it) {
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const int n = p.n, K = p.k;
  const size_t nn = (size_t)n * n;
  const int per = (n * n + kThreads - 1) / kThreads;
  const int b = blockIdx.x / per, pix = (blockIdx.x % per) * kThreads + threadIdx.x;
  if (b >= bt.ns || pix >= n * n) return;
  const int2 rc = d.pos[bt.slots[b]];
  const int y = pix / n, x = pix - y * n;
  const float2 o = d.obj[(size_t)(rc.x + y) * p.w_obj + rc.y + x];
  float2* dbgp = bt.cs->dbg.psi_new;
  float2 acc = make_float2(0.f, 0.f);
  // mode k + 1's inputs are loaded before mode k's stores
  float2* xb = d.X + (size_t)b * K * nn + pix;
  float2 psi_new = xb[0], pv = d.probe[pix];
  for (int k = 0; k < K; ++k) {
    const bool more = k + 1 < K;
    const float2 psi_n = more ? xb[(size_t)(k + 1) * nn] : psi_new;
    const float2 pv_n = more ? d.probe[(size_t)(k + 1) * nn + pix] : pv;
    if (dbgp) dbgp[((size_t)b * K + k) * nn + pix] = psi_new;
    const float2 dpsi = csub(psi_new, cmul(o, pv));
    acc = cadd(acc, cmulc(dpsi, pv));
    xb[(size_t)k * nn] = cmulc(dpsi, o);
    psi_new = psi_n;
    pv = pv_n;
  }
  d.dO[(size_t)b * nn + pix] = acc;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

bool dft_supported(int n) { return n == 64 || n == 128 || n == 192 || n == 256; }
int dft_err_slots(int n) { return (n / kDftTile) * (n / kDftTile); }

template <int N>
static hipError_t dft2_t(float2* X, const __bf16* planes, int frames, bool inverse, hipStream_t s,
                         const CaseDesc* exit_cases = nullptr, int beta = 0, const int* it = nullptr) {
  static_assert(N % (16 * kDftGroups) == 0, "whole row / column groups per block");
  // two waves per SIMD where the tiles divide into eight shares, three at N = 192 (twelve
  // waves of one 16-column tile each)
  constexpr int W = N == 192 ? 12 : (N % 128 == 0) ? 8 : 4;
  DftPlanes F{planes};
  const int rows = frames * N;
  const dim3 rgrid(rows / (16 * kDftGroups)), lgrid(N / (16 * kDftGroups), frames);
  if (!inverse) {
    if (exit_cases)
      pty_launch(k_dft_right<N, false, W, true>, rgrid, dim3(64 * W), 0, s, X, F, rows, exit_cases, beta, it);
    else
      pty_launch(k_dft_right<N, false, W, false>, rgrid, dim3(64 * W), 0, s, X, F, rows, (const CaseDesc*)nullptr,
                 0, (const int*)nullptr);
    pty_launch(k_dft_left<N, false, W>, lgrid, dim3(64 * W), 0, s, X, F, frames);
  } else {
    pty_launch(k_dft_left<N, true, W>, lgrid, dim3(64 * W), 0, s, X, F, frames);
    pty_launch(k_dft_right<N, true, W, false>, rgrid, dim3(64 * W), 0, s, X, F, rows, (const CaseDesc*)nullptr, 0,
               (const int*)nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_dft2_exit(float2* X, const void* planes, const CaseDesc* cases, int beta, const int* it, int n,
                           int frames, hipStream_t s) {
  const __bf16* pl = static_cast<const __bf16*>(planes);
  switch (n) {
    case 64: return dft2_t<64>(X, pl, frames, false, s, cases, beta, it);
    case 128: return dft2_t<128>(X, pl, frames, false, s, cases, beta, it);
    case 192: return dft2_t<192>(X, pl, frames, false, s, cases, beta, it);
    case 256: return dft2_t<256>(X, pl, frames, false, s, cases, beta, it);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_dft2(float2* X, const void* planes, int n, int frames, bool inverse, hipStream_t s) {
  const __bf16* pl = static_cast<const __bf16*>(planes);
  switch (n) {
    case 64: return dft2_t<64>(X, pl, frames, inverse, s);
    case 128: return dft2_t<128>(X, pl, frames, inverse, s);
    case 192: return dft2_t<192>(X, pl, frames, inverse, s);  // 3 tiles of 16 per wave, 6 k-chunks of 32
    case 256: return dft2_t<256>(X, pl, frames, inverse, s);
    default: return hipErrorInvalidValue;
  }
}

static int pix_blocks(int n) { return (n * n + kThreads - 1) / kThreads; }

hipError_t launch_dft_side(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  pty_launch(k_dft_side, dim3(t.max_side_jobs, t.n_cases), dim3(kThreads), 0, s, cases, beta, it);
  return hipGetLastError();
}
hipError_t launch_dft_modsum(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  pty_launch(k_dft_modsum, dim3(pix_blocks(t.n) * t.max_batch, t.n_cases), dim3(kThreads), 0, s, cases, beta,
                     it);
  return hipGetLastError();
}
hipError_t launch_dft_blur_apply(const CaseDesc* cases, const TableShape& t, int beta, const int* it,
                                 hipStream_t s) {
  pty_launch(k_dft_blur_apply, dim3(dft_err_slots(t.n) * t.max_batch, t.n_cases), dim3(kThreads), 0, s,
                     cases, beta, it);
  return hipGetLastError();
}
hipError_t launch_dft_delta(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  pty_launch(k_dft_delta, dim3(pix_blocks(t.n) * t.max_batch, t.n_cases), dim3(kThreads), 0, s, cases, beta,
                     it);
  return hipGetLastError();
}

}  // namespace pty
