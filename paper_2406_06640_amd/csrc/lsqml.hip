// pc-LSQML step lengths (gfx950): the least-squares engine of the paper's ref. [27]
// with the blurred modulus constraint (box 1) and the complex constraint (box 2),
// Sec. 3.2 and 4.1.  After the batch passes have left, per slot j, the object
// numerator dO_j = sum_k conj(P_k) chi_jk and the probe contributions
// X_jk = conj(o_j) chi_jk, and k_obj_update in direction mode has written the
// directions dO (object) and dP_k (probe) with sum_k conj(P_k) dP_k and
// sum_k |dP_k|^2, the real step pair (a_j, b_j) minimising
//   sum_k || chi_jk - a dO_j P_k - b o_j dP_k ||^2
// solves the 2x2 normal equations
//   M11 = sum |dO_j|^2 sum_k |P_k|^2          M12 = Re sum conj(dO_j) o_j sum_k conj(P_k) dP_k
//   M22 = sum |o_j|^2 sum_k |dP_k|^2          r1  = Re sum conj(dO_j) dO_j-numerator
//   r2  = Re sum_k sum conj(dP_k) X_jk
// (sums over the frame pixels), with the diagonal scaled by (1 + damping).
// k_lsq_sums writes per-block partial sums in double; k_lsq_solve adds them in a
// fixed order, solves every slot and averages the steps over the batch.
#include "kernels_dev.hpp"

namespace pty {

// One block per (slot, chunk of kLsqChunk frame pixels); part[slot][chunk][5].
__global__ __launch_bounds__(kThreads) void k_lsq_sums(const CaseDesc* __restrict__ cases, int beta,
                                                       const int* __restrict__ it) {
  __shared__ double2 red2[kThreads / 64];
  __shared__ double red[kThreads / 64];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const int n = p.n, K = p.k;
  const int chunks = lsq_chunks(n);
  const int b = blockIdx.x / chunks, chunk = blockIdx.x % chunks;
  if (b >= bt.ns) return;
  const size_t nn = (size_t)n * n;
  const bool probe = (bt.flags & FLAG_PROBE) != 0;
  const int2 rc = d.pos[bt.slots[b]];
  const float* pw = d.pw + (size_t)pw_copy(bt.flags, beta) * nn;
  const float2* gj = d.dO + (size_t)b * nn;
  const float2* xj = d.X + (size_t)b * K * nn;
  float m11 = 0.f, m12 = 0.f, m22 = 0.f, r1 = 0.f, r2 = 0.f;
  // kPx pixels per thread, each thread's loads issued before their sums
  constexpr int kPx = kLsqChunk / kThreads;
  int pixv[kPx];
  size_t oiv[kPx];
  bool ok[kPx];
  float2 dOv[kPx], gv[kPx], ov[kPx], pdpv[kPx];
  float pvv[kPx], dp2v[kPx];
#pragma unroll
  for (int j = 0; j < kPx; ++j) {
    pixv[j] = chunk * kLsqChunk + j * kThreads + threadIdx.x;
    ok[j] = pixv[j] < n * n;
    const int pix = ok[j] ? pixv[j] : 0;
    const int y = pix / n, x = pix - y * n;
    oiv[j] = (size_t)(rc.x + y) * p.w_obj + rc.y + x;
    dOv[j] = d.lsq_do[oiv[j]];
    gv[j] = gj[pix];
    pvv[j] = pw[pix];
    if (probe) {
      ov[j] = d.obj[oiv[j]];
      pdpv[j] = d.lsq_pdp[pix];
      dp2v[j] = d.lsq_dp2[pix];
    }
  }
#pragma unroll
  for (int j = 0; j < kPx; ++j) {
    if (!ok[j]) continue;
    const float2 dO = dOv[j], g = gv[j];
    m11 += (dO.x * dO.x + dO.y * dO.y) * pvv[j];
    r1 += dO.x * g.x + dO.y * g.y;
    if (probe) {
      const float2 o = ov[j], pdp = pdpv[j];
      const float2 u = cmulc(o, dO);  // conj(dO) o
      m12 += u.x * pdp.x - u.y * pdp.y;
      m22 += (o.x * o.x + o.y * o.y) * dp2v[j];
    }
  }
  if (probe) {
    // r2 = Re sum_k sum conj(dP_k) X_k: the modes' loads of all the thread's pixels at once
    for (int k = 0; k < K; ++k) {
      float2 xv[kPx], dpv[kPx];
#pragma unroll
      for (int j = 0; j < kPx; ++j) {
        const int pix = ok[j] ? pixv[j] : 0;
        xv[j] = xj[(size_t)k * nn + pix];
        dpv[j] = d.lsq_dp[(size_t)k * nn + pix];
      }
#pragma unroll
      for (int j = 0; j < kPx; ++j)
        if (ok[j]) r2 += dpv[j].x * xv[j].x + dpv[j].y * xv[j].y;
    }
  }
  const double2 s1 = block_sum_d2((double)m11, (double)m12, red2);
  const double2 s2 = block_sum_d2((double)m22, (double)r1, red2);
  const double s3 = block_sum_d((double)r2, red);
  if (threadIdx.x == 0) {
    double* out = d.lsq_part + ((size_t)b * chunks + chunk) * kLsqTerms;
    out[0] = s1.x;
    out[1] = s1.y;
    out[2] = s2.x;
    out[3] = s2.y;
    out[4] = s3;
  }
}

// One block per case: wave w takes slots w, w + 4, ...; its lanes sum a slot's chunk
// partials (lane l: chunks l, l + 64, ... in order, then a fixed butterfly) and lane 0
// solves the slot's damped 2x2 system (a zero-norm direction gets a zero step; without
// probe update, or when the damped matrix is singular, b = 0 and a = r1 / M11).  The
// steps' means over the batch go to lsq_ab, the steps to lsq_steps.
__global__ __launch_bounds__(kThreads) void k_lsq_solve(const CaseDesc* __restrict__ cases, int beta,
                                                        const int* __restrict__ it) {
  __shared__ double2 red2[kThreads / 64];
  __shared__ double sa[kMaxBatch], sb[kMaxBatch];
  Batch bt;
  if (!open_batch(cases, beta, it, bt)) return;
  const DevParams& p = bt.cs->p;
  const DevBufsG d = global_bufs(bt.cs->d);
  const int chunks = lsq_chunks(p.n);
  const bool probe = (bt.flags & FLAG_PROBE) != 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = w; j < bt.ns; j += kThreads / 64) {
    double s[kLsqTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = lane; c < chunks; c += 64)
#pragma unroll
      for (int i = 0; i < kLsqTerms; ++i) s[i] += d.lsq_part[((size_t)j * chunks + c) * kLsqTerms + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int i = 0; i < kLsqTerms; ++i) s[i] += __shfl_xor(s[i], o);
    if (lane == 0) {
      const double lam = (double)p.lsq_damping;
      const double m11 = s[0] * (1.0 + lam), m12 = s[1], m22 = s[2] * (1.0 + lam), r1 = s[3], r2 = s[4];
      const double det = m11 * m22 - m12 * m12;
      double a = 0.0, bb = 0.0;
      if (probe && m11 > 0.0 && m22 > 0.0 && det > 0.0) {
        a = (m22 * r1 - m12 * r2) / det;
        bb = (m11 * r2 - m12 * r1) / det;
      } else if (m11 > 0.0) {
        a = r1 / m11;
      } else if (probe && m22 > 0.0) {
        bb = r2 / m22;
      }
      sa[j] = a;
      sb[j] = bb;
      d.lsq_steps[2 * j] = (float)a;
      d.lsq_steps[2 * j + 1] = (float)bb;
    }
  }
  __syncthreads();
  const int j = threadIdx.x;
  const double2 tot = block_sum_d2(j < bt.ns ? sa[j] : 0.0, j < bt.ns ? sb[j] : 0.0, red2);
  if (threadIdx.x == 0) {
    d.lsq_ab[0] = (float)(tot.x / bt.ns);
    d.lsq_ab[1] = (float)(tot.y / bt.ns);
  }
}

hipError_t launch_lsq_sums(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  pty_launch(k_lsq_sums, dim3(t.max_batch * lsq_chunks(t.n), t.n_cases), dim3(kThreads), 0, s, cases, beta, it);
  return hipGetLastError();
}
hipError_t launch_lsq_solve(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s) {
  pty_launch(k_lsq_solve, dim3(1, t.n_cases), dim3(kThreads), 0, s, cases, beta, it);
  return hipGetLastError();
}

}  // namespace pty
