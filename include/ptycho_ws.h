/*
 * ptycho_ws.h -- C ABI of the learned warm start of the pc-ePIE library.
 *
 * The reconstruction of Xu et al. (arXiv 2406.06640) needs the width sigma of
 * the Gaussian coherence kernel (Eq. 6-7) and an initial probe before its
 * first iteration; the paper sets sigma by hand (Sec. 4.2-4.4).  This part of
 * the library predicts them from the measured far-field patterns with a small
 * convolutional network trained only on data produced by its own GPU forward
 * model (Eq. 1-2 with an incoherent sum over wavelengths, Sec. 3.1).
 *
 * Network (all entry points agree on it): input a 128 x 128 image (the mean
 * over a scan's patterns of log(1 + I), standardised and zero-padded, see
 * ptycho_ws_features); six 3 x 3 convolutions with 32 channels, zero padding
 * 1, strides 2, 2, 2, 2, 2, 1, each followed by ReLU; global average pooling;
 * a linear head with 4 outputs (blur sigma in pixels, relative bandwidth,
 * aperture radius in pixels, defocus coefficient c of the phase 2 pi c r^2 / n^2).
 * Weights are used in BF16 (round-to-nearest-even copies of FP32 master
 * weights), biases in FP32, activations and activation gradients are stored
 * in BF16, and every sum accumulates in FP32.
 *
 * Parameter vector (float32, PTYCHO_WS_N_PARAMS entries): per convolution
 * W[co][ci][3][3] then b[co] (the first has ci = 1), then the head W[4][32] and
 * b[4].  The training loss is the mean over the batch and the 4 outputs of
 * (y - (t - off) / scale)^2, where y are the raw head outputs, t the targets in
 * natural units and (off, scale) the target normalisation; predictions are
 * returned in natural units, y * scale + off.
 *
 * All data pointers are device memory of the current HIP device unless a
 * mem_kind argument says otherwise; all work is ordered on the stream given at
 * creation (NULL = the default stream).  Calls return ptycho_status; the
 * message of the last failure is in ptycho_ws_last_error().  Nothing throws.
 */
#ifndef PTYCHO_WS_H
#define PTYCHO_WS_H

#include <stdint.h>

#include "ptycho.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { PTYCHO_WS_SIDE = 128, PTYCHO_WS_OUTPUTS = 4, PTYCHO_WS_CHANNELS = 32, PTYCHO_WS_N_PARAMS = 46692 };

typedef struct ptycho_ws ptycho_ws; /* opaque network with its optimiser state and work buffers */
typedef struct ptycho_fm ptycho_fm; /* opaque forward-model generator */

/* Number of parameters (PTYCHO_WS_N_PARAMS). */
int32_t ptycho_ws_param_count(void);

/* Create a network for batches of up to max_batch (1..4096) inputs.  The
 * parameters start at zero; set them with ptycho_ws_set_params.  Target
 * normalisation starts at off = 0, scale = 1.  Allocates device memory. */
int32_t ptycho_ws_create(int32_t max_batch, void* stream, ptycho_ws** out);

/* Copy the FP32 master parameters in (and refresh the BF16 copies) or out.
 * theta has PTYCHO_WS_N_PARAMS floats in host (PTYCHO_MEM_HOST) or device memory. */
int32_t ptycho_ws_set_params(ptycho_ws* ws, const float* theta, int32_t mem_kind);
int32_t ptycho_ws_get_params(ptycho_ws* ws, float* theta, int32_t mem_kind);

/* Target normalisation (host arrays of 4; every scale must be > 0). */
int32_t ptycho_ws_set_target_scaling(ptycho_ws* ws, const float* off, const float* scale);

/* Forward pass.  x: inputs [*][128][128] float; idx: optional int32 [nb] of
 * input indices (NULL: inputs 0..nb-1); y: [nb][4] predictions in natural units. */
int32_t ptycho_ws_forward(ptycho_ws* ws, const float* x, const int32_t* idx, int32_t nb, float* y);

/* Loss and gradient with respect to the parameters at the current point.
 * target: [*][4] float in natural units, indexed like x.  loss_host (optional)
 * receives the loss (synchronises the stream); grad (optional) receives the
 * PTYCHO_WS_N_PARAMS gradient entries in host or device memory per mem_kind. */
int32_t ptycho_ws_loss_grad(ptycho_ws* ws, const float* x, const int32_t* idx, const float* target, int32_t nb,
                            float* loss_host, float* grad, int32_t mem_kind);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the loss
 * of one batch.  loss_host (optional) receives the batch loss before the step. */
int32_t ptycho_ws_train_step(ptycho_ws* ws, const float* x, const int32_t* idx, const float* target, int32_t nb,
                             float lr, float* loss_host);

/* Zero the Adam moments and step count. */
int32_t ptycho_ws_reset_optimizer(ptycho_ws* ws);

void ptycho_ws_destroy(ptycho_ws* ws);
const char* ptycho_ws_last_error(void);

/* Network input from one scan: intensities [n_pat][n][n] float (far field,
 * zero frequency at (n/2, n/2)), n even and <= 128, n_pat >= 1.  out [128][128]
 * receives the mean over patterns of log(1 + I), standardised over the n x n
 * frame (mean 0, population standard deviation 1; a frame whose standard
 * deviation is at most 1e-6 (1 + |mean|) maps to zeros), centred in a zero image. */
int32_t ptycho_ws_features(const float* intensities, int32_t n_pat, int32_t n, float* out, void* stream);

/* Warm-start probe: n_modes (1..4) modes [n_modes][n][n] complex64 (interleaved
 * floats).  Mode 0 is the disc of the given radius about (n/2, n/2) with phase
 * 2 pi defocus r^2 / n^2; modes 1-3 are it times x^, y^ and x^ y^ (x^ = (x - n/2)/(n/4)),
 * orthogonal to it by symmetry; each is normalised and given the power share
 * (1, 0.05, 0.05, 0.05) / sum, the shares summing to total_power.  n in [8, 1024],
 * 0 < radius < n/2. */
int32_t ptycho_ws_render_probe(int32_t n, int32_t n_modes, float radius, float defocus, float total_power,
                               float* probe, void* stream);

/* Forward-model generator of training samples (far field, 64 x 64 frames).
 * One sample: an object of obj_side^2 pixels (amplitude in [0.8, 1] and phase
 * in [-pi/2, pi/2], each N(0,1) noise low-passed by a periodic Gaussian of
 * 3 px and min-max mapped), a probe (disc of radius R with phase 2 pi c r^2 / 64^2,
 * unit power), an n_scan x n_scan raster with the given step and integer
 * jitter centred in the object, patterns summed over n_wl wavelength scales
 * s_j = 1 / (1 + d_j) with d_j evenly spaced over [-bw/2, bw/2] (the object
 * becomes exp(s (ln A + i phi)) and the centred DFT's frequencies scale by s),
 * blurred by the normalised periodic Gaussian of width sigma on the full frame,
 * scaled to `counts` mean total per pattern and drawn as Poisson counts
 * (rounded normal approximation above a mean of 12).  sigma, bw, R and c are
 * uniform in the given ranges.  Sample k of a seed is the same whatever
 * chunk it is generated in. */
typedef struct ptycho_fm_config {
  int32_t obj_side;    /* <= 160, >= extent of the scan */
  int32_t n_scan;      /* raster side; n_scan^2 positions (<= 1024) */
  int32_t step, jitter;
  int32_t n_wl;        /* wavelengths, >= 1 */
  float counts;        /* mean total counts per pattern */
  float sigma_lo, sigma_hi, bw_lo, bw_hi, r_lo, r_hi, c_lo, c_hi;
} ptycho_fm_config;

/* Defaults: obj_side 144, 10 x 10 raster at 8 px with jitter 1, 5 wavelengths,
 * 1e5 counts, sigma in [0.5, 3], bw in [0, 0.05], R in [12, 20], c in [0.5, 2]. */
void ptycho_fm_default_config(ptycho_fm_config* cfg);

/* Create a generator that produces up to max_chunk samples per call. */
int32_t ptycho_fm_create(const ptycho_fm_config* cfg, int32_t max_chunk, void* stream, ptycho_fm** out);

/* Samples first .. first + count - 1 of seed: feat [count][128][128] network
 * inputs (as ptycho_ws_features of the noisy patterns) and targets [count][4]
 * (sigma, bw, R, c).  count <= max_chunk. */
int32_t ptycho_fm_generate(ptycho_fm* fm, uint64_t seed, int64_t first, int32_t count, float* feat, float* targets);

/* Noise-free patterns [n_pos][64][64] (before count scaling) of a given object:
 * log_amp_phase [obj_side][obj_side][2] float (ln A, phi, device), positions
 * [n_pos][2] int32 top-left corners in HOST memory (checked to keep every
 * frame inside the object), and the sample values (sigma, bw, R, c).
 * n_pos <= n_scan^2 of the configuration.  Synchronises the stream. */
int32_t ptycho_fm_patterns(ptycho_fm* fm, const float* log_amp_phase, const int32_t* positions, int32_t n_pos,
                           float sigma, float bandwidth, float radius, float defocus, float* patterns);

/* Objects [count][obj_side][obj_side][2] (ln A, phi) of samples first .. of seed. */
int32_t ptycho_fm_objects(ptycho_fm* fm, uint64_t seed, int64_t first, int32_t count, float* log_amp_phase);

void ptycho_fm_destroy(ptycho_fm* fm);

#ifdef __cplusplus
}
#endif

#endif /* PTYCHO_WS_H */
