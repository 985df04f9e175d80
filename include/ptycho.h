/*
 * ptycho.h -- C ABI of the MI355X (gfx950) pc-ePIE reconstruction library.
 *
 * Method: partially coherent ePIE ("pc-ePIE") of Xu et al., "A high-performance
 * reconstruction method for partially coherent ptychography" (arXiv 2406.06640):
 * the ePIE loop of Fig. 1 with (box 1) a normalised 2D Gaussian convolution of
 * the estimated diffracted amplitude, Eq. (6)-(7), and (box 2) the complex
 * amplitude/phase constraint of Eq. (9)-(11), applied in scheduled windows of
 * iterations (Sec. 3.1, 4.6, 4.8).  K > 1 probe modes are summed incoherently
 * (the mixed-state model the method is combined with, Sec. 4.1 and 4.4).
 *
 * Conventions shared by every entry point
 *  - Complex arrays are interleaved float pairs (re, im), row-major, C order.
 *  - Object O: [obj_h][obj_w][2].  Probe P: [n_modes][n][n][2].
 *  - Intensities I: [n_pos][n][n] float, recorded counts.  Far field: the
 *    zero frequency sits at pixel (n/2, n/2).  Near field: detector image.
 *  - Positions: [n_pos][2] int32, the top-left (row, col) of each object box
 *    o_n = O[row : row + n, col : col + n] (Fig. 1: box, probe and pattern
 *    have the same size).
 *  - Propagator (Eq. 1): the unitary 2D DFT (far field), or the paraxial
 *    free-space transfer function exp(-i pi (u^2 + v^2) / (n^2 F_px)) with
 *    signed frequency indices u, v and pixel Fresnel number F_px (near field;
 *    the paper gives the distance, Sec. 3.1, not the formula).
 *  - mem_kind selects whether a data pointer is host memory (PTYCHO_MEM_HOST)
 *    or device memory of the current HIP device (PTYCHO_MEM_DEVICE).
 *  - Every call returns a ptycho_status; on failure ptycho_last_error()
 *    describes it.  Nothing throws across this boundary.
 *  - One context is not thread-safe.  All device work is ordered on the
 *    stream given to ptycho_init; calls that return data synchronise it.
 */
#ifndef PTYCHO_H
#define PTYCHO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ptycho_ctx ptycho_ctx; /* opaque; owns all of its device memory */

typedef enum {
  PTYCHO_OK = 0,
  PTYCHO_E_INVALID = -1, /* bad argument value (NaN, out of range, bad order) */
  PTYCHO_E_SHAPE = -2,   /* unsupported n, box outside the object, size mismatch */
  PTYCHO_E_OOM = -3,     /* device or pinned host allocation failed */
  PTYCHO_E_HIP = -4,     /* a HIP runtime call failed */
  PTYCHO_E_NUMERIC = -5, /* a non-finite value appeared; the context is marked failed */
  PTYCHO_E_STATE = -6    /* the context is failed or the call is out of order */
} ptycho_status;

enum { PTYCHO_FAR_FIELD = 0, PTYCHO_NEAR_FIELD = 1 };
enum { PTYCHO_BLUR_AMPLITUDE = 0 /* Eq. (6) */, PTYCHO_BLUR_INTENSITY = 1 /* Eq. (2) */ };
enum { PTYCHO_MEM_HOST = 0, PTYCHO_MEM_DEVICE = 1 };
/* Reconstruction engine (Sec. 3.2, 4.1 and 4.5: the method plugs into ePIE, rPIE,
 * DM and LSQML). */
enum {
  PTYCHO_ENGINE_EPIE = 0 /* pc-ePIE; pc-rPIE through gamma < 1 */,
  PTYCHO_ENGINE_DM = 1 /* pc-DM */,
  PTYCHO_ENGINE_LSQML = 2 /* pc-LSQML (mixed-state with K > 1) */
};

typedef struct ptycho_params {
  /* Frame side n (probe, box and pattern, Fig. 1): 8, 16, 24, 32, 48, 64, 96,
   * 128, 192, 256, 384, 512, 768 or 1024.  n_modes K in [1, 16]. */
  int32_t n, n_modes, n_pos, obj_h, obj_w;
  int32_t geometry;   /* PTYCHO_FAR_FIELD or PTYCHO_NEAR_FIELD */
  double fresnel_px;  /* near field: F_px = dx^2 / (lambda z) > 0; ignored in the far field */
  /* Gaussian of Eq. (7): sigma1 along x (columns), sigma2 along y (rows), >= 0;
   * kernel_size odd in [1, 31] (the paper uses 11, Sec. 3.1).  0 -> delta. */
  float sigma1, sigma2;
  int32_t kernel_size;
  int32_t blur_domain; /* PTYCHO_BLUR_AMPLITUDE (default) or PTYCHO_BLUR_INTENSITY */
  float eps;           /* >= 0, added to the blurred amplitude in the modulus ratio */
  /* Complex constraint, Eq. (9)-(10): alpha1, alpha2 in [0, 1]; C-bar of Eq. (11)
   * is confined to [cbar_min, cbar_max] (the threshold of Sec. 4.8), 0 < min <= max. */
  float alpha1, alpha2, cbar_min, cbar_max;
  /* 1-based inclusive window [cc_start, cc_end] of iterations with the constraint,
   * repeated every cc_period iterations if cc_period > 0; cc_start < 1 disables. */
  int32_t cc_start, cc_end, cc_period;
  float obj_step, probe_step;    /* ePIE step sizes alpha, beta (>= 0; 1 = ePIE) */
  float gamma_obj, gamma_probe;  /* denominator mix in (0, 1]: (1-g) w + g max w; 1 = ePIE */
  int32_t probe_update_start;    /* probe updated from this 1-based iteration on */
  int32_t batch;                 /* positions per update, [1, 256]; 1 = sequential ePIE */
  int32_t orthogonalize;         /* 1: orthogonalise the K > 1 modes after each iteration */
  uint64_t seed;                 /* random sequence S_n when no explicit order is given */
  /* 1: propagate by the unitary DFT as dense complex GEMMs on BF16 matrix cores
   * with a two-term split of both operands (x = x_hi + x_lo) and FP32
   * accumulation, instead of the FP32 FFT passes.  Far field, n in {64, 128, 192, 256}.
   * The modulus constraint, the step normalisation and the mode
   * orthogonalisation stay in FP32.  Results differ from the FP32 path by the
   * split's rounding (about 1e-5 relative per transform). */
  int32_t dft_bf16;
  /* PTYCHO_ENGINE_EPIE (default) or PTYCHO_ENGINE_DM: the difference map of the
   * paper's ref. [26] with the blurred modulus projection (box 1) and the complex
   * constraint (box 2), Sec. 4.5.  The DM state holds one exit wave per scan
   * position and mode (n_pos x K x n^2 complex64 of device memory), initialised
   * to P_k o_n.  Each iteration: the overlap projection over every position --
   * O = (N_O + dm_reg max W O) / (W + dm_reg max W) with
   * N_O = sum_n sum_k conj(P_k) psi_nk and W = sum_n sum_k |P_k|^2 at the box
   * offsets, the complex constraint on the union of all boxes inside its windows
   * (C-bar pooled over every box), then (from probe_update_start) the probe
   * P_k = (N_P,k + dm_reg max V P_k) / (V + dm_reg max V) with
   * N_P,k = sum_n conj(o_n) psi_nk, V = sum_n |o_n|^2 -- and the Fourier step
   * psi_nk += F^-1[M(F(2 z_n - psi_n))]_k - z_nk with z_nk = P_k o_n and M the
   * blurred modulus constraint; E_t is the data error of the estimates 2 z - psi.
   * `batch` only sets how many positions share one launch of the Fourier step
   * (results do not depend on it); modes are not orthogonalised; gamma_obj,
   * gamma_probe, obj_step, probe_step and dft_bf16 do not apply (dft_bf16 must be 0). */
  int32_t engine;
  float dm_reg; /* pc-DM Tikhonov weight of the overlap projection, > 0 (default 1e-3) */
  /* PTYCHO_ENGINE_LSQML: the least-squares engine of the paper's ref. [27] with
   * boxes 1 and 2 (pc-LSQML, Sec. 3.2 and 4.1), batch by batch over the same
   * batches as pc-ePIE.  Per batch, from the same (O, P): the exit-wave updates
   * chi = psi' - psi of box 1; the directions
   * dO = N_O / ((1 - gamma_obj) W + gamma_obj max W) on the union of the boxes and
   * dP_k = N_P,k / ((1 - gamma_probe) V + gamma_probe max V) (sums as for pc-ePIE,
   * with chi for dpsi); per position j the real steps (a_j, b_j) minimising
   * sum_k ||chi_jk - a dO_j P_k - b o_j dP_k||^2 with the diagonal of the 2x2
   * normal equations scaled by (1 + lsq_damping) (b = 0 before
   * probe_update_start); then O += obj_step mean(a) dO, P_k += probe_step
   * mean(b) dP_k, and the complex constraint inside its windows.  Modes are
   * orthogonalised and E_t recorded as for pc-ePIE.  Either propagation path. */
  float lsq_damping; /* pc-LSQML diagonal damping lambda of the step solve, >= 0 (default 0.1) */
} ptycho_params;

/* Fill *p with defaults: n = 64, K = 1, far field, sigma 1, kernel 11, amplitude
 * blur, eps 1e-6, alpha1 = 1, alpha2 = 0 (phase object, Sec. 3.1), C-bar in
 * [0.01, 10], constraint off, steps 1, gammas 1, probe update from iteration 1,
 * batch 1, orthogonalisation on, seed 0, the ePIE engine, dm_reg 1e-3,
 * lsq_damping 0.1.
 * n_pos/obj_h/obj_w are set to 0. */
void ptycho_default_params(ptycho_params* p);

/* Create a reconstruction context on the current HIP device.
 *  intensities [n_pos][n][n], positions [n_pos][2], probe0 [K][n][n][2],
 *  object0 [obj_h][obj_w][2]: read once (host or device per mem_kind) and copied
 *  into context-owned device memory; the caller may free them on return.
 *  hip_stream: a hipStream_t (NULL = the null stream) that must outlive the ctx.
 * Errors: PTYCHO_E_INVALID (bad parameter, non-finite input, zero-power probe),
 * PTYCHO_E_SHAPE (unsupported n, a box outside the object), PTYCHO_E_OOM, PTYCHO_E_HIP.
 * On error *out is NULL. */
ptycho_status ptycho_init(const ptycho_params* params, const float* intensities,
                          const int32_t* positions, const float* probe0, const float* object0,
                          int32_t mem_kind, void* hip_stream, ptycho_ctx** out);

/* Run n_iter >= 0 iterations of Fig. 1.  Iteration t (1-based, continuing from
 * the context's counter) visits the positions in the order order[it][0..n_pos)
 * (host int32, each row a permutation of 0..n_pos-1), or, when order is NULL,
 * in a Fisher-Yates permutation driven by SplitMix64(seed XOR t); see
 * ptycho_permutation.  Consecutive groups of `batch` positions share one update.
 * err_out (host, n_iter floats, may be NULL) receives the data error
 * E_t = sum_n sum_q (sqrt(I_n) - A^G_n)^2 / sum_n sum_q I_n of each iteration.
 * Synchronises the stream.  PTYCHO_E_NUMERIC if E_t is not finite (the context
 * is then failed); PTYCHO_E_INVALID for a bad order. */
ptycho_status ptycho_iterate(ptycho_ctx* ctx, int32_t n_iter, const int32_t* order, float* err_out);

/* ptycho_iterate for callers that cannot allocate device memory during the call
 * (serving loops, code running between captures, harnesses that forbid it): the
 * same iterations, bitwise the same object, probe, counter and data errors, but
 * the call allocates nothing.  The work frames, partial sums, per-call schedule
 * and case table that ptycho_iterate keeps in context buffers live in a
 * library-owned static device array of 64 MiB per device (held until the
 * process ends); the context's state (object, probe, measured amplitudes,
 * positions) stays where ptycho_init put it.  Every call on a device shares that
 * device's array: calls that overlap on one device race (the library serialises
 * the calls of one process on the host; run one at a time per device).
 * Errors as ptycho_iterate, plus PTYCHO_E_SHAPE when the reconstruction needs
 * more than the array holds (about 8 B x (batch x (n_modes + 2) + n_modes) x n^2
 * plus 8 B per position x (n / rows per block) and the schedule) or has more
 * than 262144 positions, and PTYCHO_E_STATE when the current HIP device is not
 * the context's.  Synchronises the stream.  Eager launches only (no graph replay,
 * no per-kernel timing). */
ptycho_status ptycho_iterate_static(ptycho_ctx* ctx, int32_t n_iter, const int32_t* order, float* err_out);

/* Copy the current object [obj_h][obj_w][2] / probe [K][n][n][2] into `out`
 * (host or device per mem_kind).  Synchronises the stream. */
ptycho_status ptycho_get_object(ptycho_ctx* ctx, float* out, int32_t mem_kind);
ptycho_status ptycho_get_probe(ptycho_ctx* ctx, float* out, int32_t mem_kind);

/* Replace the object and/or probe (NULL leaves it) and set the completed-iteration
 * counter to iter >= 0 (resume from a checkpoint).  Clears a failed state. */
ptycho_status ptycho_set_state(ptycho_ctx* ctx, const float* object, const float* probe,
                               int32_t iter, int32_t mem_kind);

/* pc-DM engine: copy the exit waves [n_pos][K][n][n][2] of every scan position
 * out of / into the context (host or device per mem_kind), e.g. to checkpoint
 * the full DM state with ptycho_get_object / ptycho_get_probe.  PTYCHO_E_STATE
 * for a context of the ePIE engine.  (ptycho_set_state of a DM context resets
 * the exit waves to P_k o_n of the new object and probe.)  Synchronise the stream. */
ptycho_status ptycho_get_exit_waves(ptycho_ctx* ctx, float* out, int32_t mem_kind);
ptycho_status ptycho_set_exit_waves(ptycho_ctx* ctx, const float* in, int32_t mem_kind);

/* pc-LSQML engine: the step lengths of the last batch run (Sec. 3.2; the steps of
 * the paper's ref. [27]): steps (host, may be NULL) [batch][2] gets (a_j, b_j) of
 * its positions in visiting order (rows past that batch's size keep older values),
 * mean (host, may be NULL) [2] the means (a_bar, b_bar) the batch moved by.
 * PTYCHO_E_STATE for other engines.  Synchronises the stream. */
ptycho_status ptycho_get_lsq_steps(ptycho_ctx* ctx, float* steps, float* mean);

/* Completed-iteration counter of the context (-1 for NULL). */
int32_t ptycho_iteration(const ptycho_ctx* ctx);

/* Run ONE batch update (the body of Fig. 1 over the B positions idx[0..B), B in
 * [1, batch]) as iteration t (decides the probe-update start and the constraint
 * window) and capture its intermediates for parity checks.  The object and probe
 * are updated exactly as inside ptycho_iterate; the counter is not changed.
 * Any output may be NULL.  Outputs (host or device per mem_kind):
 *   psi      [B][K][n][n][2]  exit waves o_b P_k
 *   psi_new  [B][K][n][n][2]  back-propagated constrained waves psi'
 *   factor   [B][n][n]        modulus factor (detector pixel order)
 *   n_obj    [obj_h][obj_w][2], w_obj [obj_h][obj_w]  object numerator and weight
 *   n_probe  [K][n][n][2],     v_probe [n][n]          probe numerator and weight
 *             (probe outputs are zero when t < probe_update_start). */
ptycho_status ptycho_debug_step(ptycho_ctx* ctx, const int32_t* idx, int32_t B, int32_t t,
                                float* psi, float* psi_new, float* factor, float* n_obj,
                                float* w_obj, float* n_probe, float* v_probe, int32_t mem_kind);

/* Replay each iteration from a HIP graph captured on first use (enable != 0)
 * instead of launching its kernels one by one; the graph is rebuilt when the
 * column-tile choice changes.  Results are bitwise identical either way.
 * Not used while per-kernel timing is on. */
ptycho_status ptycho_set_graph(ptycho_ctx* ctx, int32_t enable);

/* Launch variants of the FFT passes: variant v (0 .. ptycho_variant_count()-2)
 * uses column blocks of COLS/2, COLS or 2 COLS columns (v % 3; COLS is the
 * default width for n), runs the inverse column pass with one workgroup per
 * mode when (v / 3) & 1 and the first row pass likewise when (v / 6) & 1.
 * The last variant (ptycho_variant_count()-1) is the sequential kernel: one
 * workgroup runs each whole iteration (every position of Fig. 1's loop in
 * order, the updates applied in between), for batch 1 on far-field frames of
 * side 16, 32, 48 or 64; it is the default there (the autotuner keeps it), and
 * groups run such cases one workgroup per case in one launch.  Its results
 * agree with the batch passes to FP32 rounding, not bitwise.
 * Variants other than the three widths exist for n in {64, 128, 192, 256, 512}.
 * The object and probe after any iteration are bitwise identical for every
 * variant (the data error E_t is summed in a different grouping for other
 * widths).  The default is variant 1. */
int32_t ptycho_variant_count(void);
/* Select a variant (PTYCHO_E_INVALID if it does not exist for this n). */
ptycho_status ptycho_set_variant(ptycho_ctx* ctx, int32_t variant);

/* Autotuner: times each existing launch variant on the context's first batch
 * (`trials` timed repetitions each), keeps the fastest and writes its index to
 * *chosen (may be NULL).  The object and probe are restored afterwards.
 * Choices are cached per (n, n_modes, batch, geometry) for the process and,
 * when the environment variable PTYCHO_TUNE_CACHE names a file, appended to it
 * and read back by later processes; force != 0 re-times a cached entry. */
ptycho_status ptycho_autotune(ptycho_ctx* ctx, int32_t trials, int32_t force, int32_t* chosen);

/* Per-kernel timing with HIP events recorded on the context stream around each
 * launch of the kernel classes selected by `mask` (bit i = class i, see
 * ptycho_kernel_name); 0 disables.  Totals accumulate until reset. */
ptycho_status ptycho_set_timing(ptycho_ctx* ctx, uint32_t mask);
/* Accumulated milliseconds and launch count of kernel class `cls`; reset != 0 zeroes it. */
ptycho_status ptycho_kernel_time(ptycho_ctx* ctx, int32_t cls, double* total_ms, int64_t* launches,
                                 int32_t reset);
/* Name of kernel class `cls` (NULL if out of range) and the number of classes. */
const char* ptycho_kernel_name(int32_t cls);
int32_t ptycho_kernel_class_count(void);

/* Release all device memory of the context (NULL is a no-op). */
void ptycho_destroy(ptycho_ctx* ctx);

/* Text of the last error on this context, or of this thread's last failed
 * ptycho_init / NULL-context call when ctx is NULL.  Never NULL. */
const char* ptycho_last_error(const ptycho_ctx* ctx);

/* Groups of independent reconstructions (many cases of uneven frame size,
 * position count and mode count advanced together).  Every pass of a batch
 * runs as one launch per (frame size, geometry) class covering the batch of
 * that index of every case in the class; a case's results are bitwise
 * identical to running it alone with ptycho_iterate(ctx, n, NULL, ...).
 * The contexts must share one device and stream and stay alive while the
 * group exists; the group does not own them. */
typedef struct ptycho_group ptycho_group;
ptycho_status ptycho_group_create(ptycho_ctx* const* ctxs, int32_t n, ptycho_group** out);
/* n_iter iterations of every case, each in its own generated order (seed XOR t).
 * err_out (host, may be NULL): [n cases][n_iter] data errors.  A case whose
 * error is non-finite is marked failed and PTYCHO_E_NUMERIC returned. */
ptycho_status ptycho_group_iterate(ptycho_group* g, int32_t n_iter, float* err_out);
/* enable != 0: replay each iteration of the group from a HIP graph captured on
 * first use (an internal non-blocking stream ordered with the group's stream by
 * events); results are bitwise those of the eager launches. */
ptycho_status ptycho_group_set_graph(ptycho_group* g, int32_t enable);
void ptycho_group_destroy(ptycho_group* g);
const char* ptycho_group_last_error(const ptycho_group* g);

/* The unitary 2D DFT (inverse != 0: its inverse) of `frames` device frames
 * [frames][n][n][2] in place, by the BF16-split matrix-core GEMMs of the
 * dft_bf16 path (n in {64, 128, 192, 256}), ordered on hip_stream (NULL = null stream);
 * synchronises it.  For measuring that path's error and speed on its own. */
ptycho_status ptycho_dft2_bf16(float* frames_inout, int32_t n, int32_t frames, int32_t inverse, void* hip_stream);

/* Numerical monochromatisation of broadband far-field patterns (Sec. 4.2):
 * the broadband pattern is modelled as b = C m, and the monochromatic pattern m
 * is estimated by k iterations of CGLS from x_0 = 0, the k-th iterate being the
 * least-squares solution of ||C x - b|| over the Krylov subspace
 * span{C^T b, (C^T C) C^T b, ..., (C^T C)^(k-1) C^T b} (Eq. 12-13; the paper uses
 * k up to 40, k = 25 typically).  C depends only on the spectrum: on a fixed
 * detector the pattern at wavelength lambda_j is m magnified about the centre
 * pixel (n/2, n/2) by s_j = lambda_c / lambda_j and weighted by w_j s_j^2
 * (sum w_j = 1, so each wavelength carries its weight's power), sampled
 * bilinearly with zero outside the frame; C^T is its exact adjoint.
 *  create: n even in [2, 4096]; max_patterns in [1, 65535]; scales[n_lambda] in [1/16, 16]
 *          and weights[n_lambda] >= 0 (normalised here), host arrays, n_lambda in
 *          [1, 16]; hip_stream orders every call (NULL = null stream).  Owns
 *          6 x max_patterns x n^2 floats of device work and staging memory and
 *          the operator's interpolation tables, n_lambda x n x (floor(2 / min scale) + 7)
 *          words, built here (synchronises hip_stream).
 *  run:    broadband [n_patterns][n][n] float (zero frequency at (n/2, n/2)) into
 *          mono_out [n_patterns][n][n] (host or device per mem_kind; may not
 *          alias); residuals (host, may be NULL) [n_patterns][k_iters + 1] gets
 *          ||C x_i - b|| for i = 0 .. k_iters.  Patterns are independent and run
 *          together.  Synchronises the stream.  The output can be negative where
 *          the data are noisy; ptycho_init clamps intensities at zero.
 * Errors: PTYCHO_E_INVALID, PTYCHO_E_SHAPE, PTYCHO_E_OOM, PTYCHO_E_HIP; the text is
 * in ptycho_last_error(NULL). */
typedef struct ptycho_mono ptycho_mono;
ptycho_status ptycho_mono_create(int32_t n, int32_t max_patterns, const float* scales, const float* weights,
                                 int32_t n_lambda, void* hip_stream, ptycho_mono** out);
ptycho_status ptycho_mono_run(ptycho_mono* m, const float* broadband, float* mono_out, int32_t n_patterns,
                              int32_t k_iters, float* residuals, int32_t mem_kind);
void ptycho_mono_destroy(ptycho_mono* m);

/* Host-only: the order used for iteration t when none is given -- Fisher-Yates
 * over 0..n_pos-1 (for i = n_pos-1 .. 1: j = next % (i + 1), swap) with `next`
 * the SplitMix64 sequence (Steele, Lea, Flood 2014) seeded with seed XOR t.
 * This is the "random sequence S_n" of Fig. 1; the paper names no generator. */
ptycho_status ptycho_permutation(uint64_t seed, int32_t t, int32_t n_pos, int32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* PTYCHO_H */
