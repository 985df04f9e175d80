// Device-side descriptors and host launchers of the pc-ePIE kernels.
//
// Every batch kernel reads its reconstruction ("case") from a device table of
// CaseDesc: blockIdx.y selects the case, blockIdx.x the block within that
// case's grid.  A single reconstruction is a table of one; a group of
// independent reconstructions with the same frame size and geometry shares
// each launch (cases whose batch index is past their last batch, or whose
// grid is smaller, return at once).  A case's arithmetic does not depend on
// the other cases in the table, so grouped and single runs agree bitwise.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pty {

constexpr int kMaxHalf = 15;     // kernel_size <= 31
constexpr int kMaxModes = 16;
constexpr int kMaxBatch = 256;
constexpr int kObjTile = 32;     // object tile side for the gather/update kernels
constexpr int kGramBlocks = 16;  // pixel chunks of the Gram matrix reduction
// launch variants tried by the autotuner: column-tile width COLS/2, COLS or 2 COLS (v % 3);
// v < 12: separate middle passes, mode-parallel inverse column pass ((v / 3) & 1), mode-parallel
// first row pass ((v / 6) & 1); v in [12, 18): fused middle pass, mode-parallel first row pass
// (((v - 12) / 3) & 1)
constexpr int kColVariants = 18;
constexpr int kFusedHalo = 5;  // halo columns of the fused middle pass (kernel sizes up to 11)

// Per-iteration flags of a case.
// FLAG_PW_ODD: the iteration's first batch reads copy 1 of the probe-power map (see DevBufs::pw).
enum : int { FLAG_PROBE = 1, FLAG_CC = 2, FLAG_ORTHO = 4, FLAG_PW_ODD = 8 };

struct DevParams {
  int n, k, h_obj, w_obj, n_pos;
  int near_field;
  int blur_intensity;
  int ks_half;
  float eps;
  float alpha1, alpha2, cbar_min, cbar_max;
  float obj_step, probe_step, gamma_obj, gamma_probe;
  float dm_reg;            // pc-DM: Tikhonov weight delta of the overlap projection (relative to max W, max V)
  int dm_seg_len;          // pc-DM: scan positions per segment of the probe-numerator partial sums
  float lsq_damping;       // pc-LSQML: diagonal damping of the per-position 2x2 step solve
  float gx[kMaxHalf + 1];  // normalised taps for |dx| = 0..ks_half (x = columns, sigma1)
  float gy[kMaxHalf + 1];  // normalised taps for |dy| = 0..ks_half (y = rows, sigma2)
};

struct DevBufs {
  float2* obj;         // [H][W]
  float2* probe;       // [K][N][N]
  float* pw;           // [2][N][N] sum_k |P_k|^2, two copies: a batch reads one (pw_copy) while its
                       // probe update writes the other, so both updates share one launch
  const float* amp;    // [n_pos][N][N] sqrt(max(I,0)) in detector pixel order
  const int2* pos;     // [n_pos] (row, col)
  const float2* tw;    // [N] exp(-2 pi i m / N)
  const float2* hnear; // [N] near-field 1D transfer function, exp(-i pi u~^2/(N^2 F_px))
  float2* X;           // [B][K][N][N] batch work frames
  float* q;            // [B][N][N] vertically blurred sqrt(sum_k |Psi_k|^2) (or of the intensity)
  float2* dO;          // [B][N][N] per-slot object numerator sum_k conj(P_k) dpsi_k
  float2* nP;          // [K][N][N] probe numerator
  float* V;            // [N][N] probe weight sum_b |o_b|^2
  float* maxv_part;    // per-block max of V (one per 256 probe pixels)
  float* maxw_part;    // per-object-tile max of W
  double* err_part;    // [n_pos][column blocks per frame] data-error partial sums
  double2* cc_part;    // [object tiles] (sum |ln A|, sum |phi|) weighted by box multiplicity
  unsigned* cov_mask;  // [object tiles][32] row bitmasks of the tile pixels the batch's boxes cover
  // pc-DM engine only (null otherwise)
  float2* psi;         // [n_pos][K][N][N] exit waves of every scan position
  const int* cov_off;  // [object tiles + 1] offsets into cov_pos
  const int* cov_pos;  // scan positions whose boxes intersect each object tile, ascending
  float2* np_part;     // [segments][K][N][N] probe-numerator partial sums
  float* v_part;       // [segments][N][N] probe-weight partial sums
  double2* gram_part;  // [pairs][kGramBlocks]
  float2* vmix;        // [K][K] eigenvectors (column j = mode j), float
  double* eig;         // [K] eigenvalues
  // pc-LSQML engine only (null otherwise)
  float2* lsq_do;      // [H][W] object direction dO (valid on the batch's union)
  float2* lsq_dp;      // [K][N][N] probe direction dP_k
  float2* lsq_pdp;     // [N][N] sum_k conj(P_k) dP_k
  float* lsq_dp2;      // [N][N] sum_k |dP_k|^2
  double* lsq_part;    // [B][lsq chunks][5] per-slot partial sums of the step normal equations
  float* lsq_ab;       // [2] the batch's mean steps (a, b)
  float* lsq_steps;    // [B][2] the last batch's per-position steps (a_j, b_j)
};

struct DebugPtrs {
  float2* psi_new;  // [B][K][N][N] or null
  float2* n_obj;    // [H][W] or null
  float* w_obj;     // [H][W] or null
  float* factor;    // [B][N][N] or null
};

struct CaseDesc {
  DevParams p;
  DevBufs d;
  DebugPtrs dbg;
  const int* order;  // [iterations of the call][n_pos] visiting order
  const int* flags;  // [iterations of the call] FLAG_* bits
  float* err_out;    // [iterations of the call] data error E_t
  double inv_denom;  // 1 / sum_n sum_q I_n
  int n_pos, batch, n_batches, n_err_part;
};

// Host-side launch geometry of one table of cases (all with the same n and geometry).
struct TableShape {
  int n;
  bool near_field;
  int n_cases;
  int max_batch;       // max over cases of the batch size
  int max_tiles;       // max over cases of object tiles
  int max_k;           // max over cases of the number of modes
  int max_side_jobs;   // max over cases of object tiles + V blocks
  int col_variant;     // 0..kColVariants-1
  int max_half;        // max over cases of the blur half-width
  int max_dm_segments; // max over cases of the pc-DM probe-partial segments (0: no pc-DM case)
  bool x_pairs;        // the inverse row pass adds the probe contributions of slot pairs
};

// Kernel classes (for timing).
enum KernelClass {
  KC_FWD_ROWS = 0, KC_FWD_COLS, KC_INV_COLS, KC_INV_ROWS, KC_OBJ_UPDATE, KC_CONSTRAINT, KC_GRAM, KC_EIG, KC_REMIX,
  KC_ERR, KC_DFT_GEMM, KC_DFT_OTHER, KC_FACTOR, KC_COLS_FUSED, KC_DM_ROWS, KC_DM_OVERLAP, KC_SEQ, KC_LSQ_DIR,
  KC_LSQ_STEP, KC_LSQ_APPLY, KC_COUNT
};
extern const char* const kKernelNames[KC_COUNT];

// Per-kernel timing events for the launcher call in progress on this thread
// (set by the runtime's timing, empty otherwise): the first kernel the call
// launches records `start` when it starts, every kernel records `stop` when it
// ends, so the pair spans the call's kernels without separate event packets.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents& launch_events();

// Batch launches for batch index `beta` of the call's current iteration, which
// the kernels read from the device counter `it` (so that a captured iteration
// graph can be replayed unchanged).
hipError_t launch_fwd_rows(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_fwd_cols(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_factor(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_cols_fused(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_inv_cols(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_inv_rows(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
// Per-kernel launch attributes (LDS above 64 KB per workgroup); once per process
// before the first launch.
hipError_t init_kernel_attributes();
// Whether frame size n has the paired inverse row pass (TableShape::x_pairs).
bool inv_rows_paired(int n);
hipError_t launch_obj_update(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_constraint(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
// Per-iteration launches.
hipError_t launch_gram(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s);
hipError_t launch_eig(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s);
hipError_t launch_remix(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s);
hipError_t launch_err_reduce(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s);
// The iteration counter: advance by one / set.
hipError_t launch_iter_advance(int* it, hipStream_t s);
hipError_t launch_iter_set(int* it, int v, hipStream_t s);
// Init-time and debug helpers (one case, parameters by value).
hipError_t launch_prepare_amp(const float* inten, float* amp, int n, int n_pos, bool shift, int* bad_count,
                              double* sum_part, hipStream_t s);
// sum_k |P_k|^2 of the current probe into copy `copy` of d.pw
hipError_t launch_pw(const DevParams& p, const DevBufs& d, int copy, hipStream_t s);
hipError_t launch_exit_waves(const DevParams& p, const DevBufs& d, const int* slots, int ns, float2* out,
                             hipStream_t s);

// pc-DM engine: the overlap projection over every scan position (object, then
// probe), the two row passes of its Fourier step for batch `beta` of the
// positions (the column passes and the modulus factor are the ePIE engine's),
// and the initial exit waves P_k o_n of every position.
hipError_t launch_dm_overlap(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s);
hipError_t launch_dm_rows_fwd(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_dm_rows_inv(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_dm_init_psi(const DevParams& p, const DevBufs& d, hipStream_t s);
int dm_segments(int n_pos, int seg_len);

// pc-LSQML engine, batch `beta` after the inverse row pass (or the DFT path's delta
// pass) has left the per-slot numerators: the directions dO, dP_k (k_obj_update in
// direction mode), the per-slot partial sums of the step normal equations, the
// per-slot solves and their mean, and the update along the directions (k_obj_update
// in apply mode, which also writes the complex constraint's sums).
constexpr int kLsqChunk = 1024;  // frame pixels per block of the partial sums
constexpr int kLsqTerms = 5;     // M11, M12, M22, r1, r2
__host__ __device__ inline int lsq_chunks(int n) { return (n * n + kLsqChunk - 1) / kLsqChunk; }
hipError_t launch_lsq_dir(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_lsq_sums(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_lsq_solve(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_lsq_apply(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);

// Sequential pc-ePIE for batch size 1 and small far-field frames: one
// workgroup per case runs a whole iteration (every position in order).
bool seq_supported(int n, bool near_field);
hipError_t launch_seq_iter(const CaseDesc* cases, const TableShape& t, const int* it, hipStream_t s);

// Numerical monochromatisation by CGLS: spectrum (scales s_j = lambda_c / lambda_j
// and coefficients w_j s_j^2 with sum w_j = 1) and the work buffers of n_pat patterns.
constexpr int kMonoMaxLambda = 16;
constexpr float kMonoMinScale = 1.0f / 16.0f, kMonoMaxScale = 16.0f;
struct MonoSpectrum {
  int count;
  float scale[kMonoMaxLambda];
  float coef[kMonoMaxLambda];
};
// Per-wavelength interpolation tables, built once per plan by launch_mono_tables.
// Forward: detector pixel u samples nodes i0 and i0 + 1 with weights 1 - t and t.
// Adjoint: node v receives from the adj_cnt consecutive pixels starting at adj_first
// (weights adj_w, row stride adj_stride, zero where a pixel of the run does not touch v).
struct MonoTables {
  int* i0;        // [count][n]
  float* t;       // [count][n]
  int* adj_first; // [count][n]
  int* adj_cnt;   // [count][n] run length up to the last nonzero weight
  float* adj_w;   // [count][n][adj_stride]
  int adj_stride; // floor(2 / min scale) + 3
  int adj_max;    // largest adj_cnt (read back at plan creation)
};
int mono_adj_stride(const MonoSpectrum& sp);
// Partial sums per pattern that the CGLS kernels write (the larger of the operator's
// tiles and the element-wise kernels' blocks).
int mono_part_count(int n);
struct MonoWork {
  MonoSpectrum spec;
  MonoTables tab;
  float *r, *s, *p, *q;   // [n_pat][n][n] CGLS vectors
  double *part, *part2;   // [n_pat][blocks] partial sums
  double *gamma, *coef;   // [n_pat] |C^T r|^2 and alpha / beta
};
hipError_t launch_mono_tables(const MonoWork& w, int n, hipStream_t s);
// k_iters CGLS iterations from x = 0 for every pattern of b into x; res (device,
// [n_pat][k_iters + 1], may be null) receives |C x_i - b| for i = 0 .. k_iters.
hipError_t launch_mono_cgls(const float* b, float* x, const MonoWork& w, int n, int n_pat, int k_iters, float* res,
                            hipStream_t s);

// BF16 matrix-core DFT path (far field, n in {64, 128, 192, 256}); single table only.
// planes: [4][n][n] bf16 (re_hi, re_lo, im_hi, im_lo) of F[u][x] = exp(-2 pi i u x / n) / sqrt(n).
bool dft_supported(int n);
int dft_err_slots(int n);
hipError_t launch_dft2(float2* X, const void* planes, int n, int frames, bool inverse, hipStream_t s);
// The forward transform of batch beta's exit waves (frame b K + k = o_b P_k, formed
// while the first GEMM stages its operand) into X.
hipError_t launch_dft2_exit(float2* X, const void* planes, const CaseDesc* cases, int beta, const int* it, int n,
                           int frames, hipStream_t s);
hipError_t launch_dft_side(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_dft_modsum(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_dft_blur_apply(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);
hipError_t launch_dft_delta(const CaseDesc* cases, const TableShape& t, int beta, const int* it, hipStream_t s);

int n_obj_tiles(const DevParams& p);
// data-error partials per position for launch variant v: one per column tile of the fused
// middle pass when it runs (fused_active), else one per row block of the factor pass
bool fused_active(int n, int v, int max_half);
int n_err_slots(int n, int v, int max_half);
int max_err_slots(int n);  // over every variant
int n_probe_blocks(int n);
int col_width(int n, int col_variant);    // columns per column block
bool col_variant_valid(int n, int col_variant);
bool supported_n(int n);

}  // namespace pty
