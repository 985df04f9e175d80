// Device-side parameter/buffer structs and host launchers of the pc-ePIE kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pty {

constexpr int kMaxHalf = 15;     // kernel_size <= 31
constexpr int kMaxModes = 16;
constexpr int kMaxBatch = 256;
constexpr int kObjTile = 32;     // object tile side for the gather/update kernels
constexpr int kGramBlocks = 16;  // pixel chunks of the Gram matrix reduction

struct DevParams {
  int n, k, h_obj, w_obj, n_pos;
  int near_field;
  int blur_intensity;
  int ks_half;
  float eps;
  float alpha1, alpha2, cbar_min, cbar_max;
  float obj_step, probe_step, gamma_obj, gamma_probe;
  float gx[kMaxHalf + 1];  // normalised taps for |dx| = 0..ks_half (x = columns, sigma1)
  float gy[kMaxHalf + 1];  // normalised taps for |dy| = 0..ks_half (y = rows, sigma2)
};

struct DevBufs {
  float2* obj;        // [H][W]
  float2* probe;      // [K][N][N]
  float* pw;          // [N][N] sum_k |P_k|^2
  const float* amp;   // [n_pos][N][N] sqrt(max(I,0)) in detector pixel order
  const int2* pos;    // [n_pos] (row, col)
  const float2* tw;   // [N] exp(-2 pi i m / N)
  const float2* hnear;// [N] near-field 1D transfer function, exp(-i pi u~^2/(N^2 F_px))
  float2* X;          // [B][K][N][N] batch work frames
  float* q;           // [B][N][N] vertically blurred sqrt(sum_k |Psi_k|^2) (or of the intensity)
  float2* dO;         // [B][N][N] per-slot object numerator sum_k conj(P_k) dpsi_k
  float2* nP;         // [K][N][N] probe numerator
  float* V;           // [N][N] probe weight sum_b |o_b|^2
  float* maxv_part;   // per-block max of V (one per 256 probe pixels)
  float* maxw_part;   // per-object-tile max of W
  double* err_part;   // [n_pos][column blocks per frame] data-error partial sums
  double2* cc_part;   // [object tiles] (sum |ln A|, sum |phi|) weighted by box multiplicity
  double2* gram_part; // [pairs][kGramBlocks]
  float2* vmix;       // [K][K] eigenvectors (column j = mode j), float
  double* eig;        // [K] eigenvalues
};

struct DebugPtrs {
  float2* psi_new;  // [B][K][N][N] or null
  float2* n_obj;    // [H][W] or null
  float* w_obj;     // [H][W] or null
  float* factor;    // [B][N][N] or null
};

// Kernel classes (for timing).
enum KernelClass {
  KC_FWD_ROWS = 0, KC_FWD_COLS, KC_INV_COLS, KC_INV_ROWS, KC_OBJ_UPDATE, KC_POST, KC_GRAM, KC_EIG, KC_REMIX,
  KC_ERR, KC_COUNT
};
extern const char* const kKernelNames[KC_COUNT];

// Launchers.  Each returns the hipGetLastError() after the launch.
hipError_t launch_fwd_rows(int n, bool near, const DevParams& p, const DevBufs& d, const int* slots, int ns,
                           bool with_v, hipStream_t s);
hipError_t launch_fwd_cols(int n, bool near, const DevParams& p, const DevBufs& d, int ns, int bmax, hipStream_t s);
hipError_t launch_inv_cols(int n, bool near, const DevParams& p, const DevBufs& d, const int* slots, int ns, int bmax,
                           const DebugPtrs& dbg, hipStream_t s);
hipError_t launch_inv_rows(int n, bool near, const DevParams& p, const DevBufs& d, const int* slots, int ns,
                           int bmax, const DebugPtrs& dbg, hipStream_t s);
hipError_t launch_obj_update(const DevParams& p, const DevBufs& d, const int* slots, int ns, bool cc_sums,
                             const DebugPtrs& dbg, hipStream_t s);
hipError_t launch_post(const DevParams& p, const DevBufs& d, const int* slots, int ns, bool probe, bool cc,
                       hipStream_t s);
hipError_t launch_gram(const DevParams& p, const DevBufs& d, hipStream_t s);
hipError_t launch_eig(const DevParams& p, const DevBufs& d, hipStream_t s);
hipError_t launch_remix(const DevParams& p, const DevBufs& d, hipStream_t s);
hipError_t launch_err_reduce(const double* part, int count, double inv_denom, float* out, hipStream_t s);
// init-time helpers
hipError_t launch_prepare_amp(const float* inten, float* amp, int n, int n_pos, bool shift, int* bad_count,
                              double* sum_part, hipStream_t s);
hipError_t launch_pw(const DevParams& p, const DevBufs& d, hipStream_t s);
hipError_t launch_exit_waves(const DevParams& p, const DevBufs& d, const int* slots, int ns, float2* out,
                             hipStream_t s);

int n_obj_tiles(const DevParams& p);
int n_err_slots(int n);  // data-error partials per position (one per column block)
int n_probe_blocks(int n);
bool supported_n(int n);

}  // namespace pty
