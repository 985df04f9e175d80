// Device-side declarations of the learned warm start: the convolutional
// network (forward, backward, Adam), its input features, the rendered probe
// and the forward-model generator of its training set.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ws {

constexpr int kC = 32;      // channels of every hidden layer
constexpr int kLayers = 6;  // 3 x 3 convolutions
constexpr int kSide = 128;  // network input side
constexpr int kOut = 4;     // head outputs: blur sigma, bandwidth, aperture radius, defocus
constexpr int kTaps = 9;

// Flat parameter vector: per convolution W[co][ci][3][3] then b[co]; then the
// head W[T][C] and b[T].  The first convolution has one input channel.
constexpr int kConvW = kC * kC * kTaps;  // 9216
constexpr int kConvStride = kConvW + kC; // 9248
constexpr int kL1 = kC * kTaps + kC;     // 320 parameters in layer 1
constexpr int kHeadW = kL1 + (kLayers - 1) * kConvStride;
constexpr int kHeadB = kHeadW + kOut * kC;
constexpr int kParams = kHeadB + kOut;    // 46692
constexpr int kHeadCols = kOut * kC + kOut;

inline int conv_offset(int l) { return l == 0 ? 0 : kL1 + (l - 1) * kConvStride; }
// spatial side of layer l's input and output (strides 2, 2, 2, 2, 2, 1)
inline int side_in(int l) { return l < 5 ? (kSide >> l) : (kSide >> 5); }
inline int side_out(int l) { return l < 5 ? (kSide >> (l + 1)) : (kSide >> 5); }
inline int stride_of(int l) { return l < 5 ? 2 : 1; }

struct Norm {
  float off[kOut];
  float scale[kOut];
};

enum ReduceMode { RED_CONV1 = 0, RED_CONV = 1, RED_HEAD = 2, RED_LOSS = 3 };

// ---- network ----
void launch_conv1_fwd(const float* x, const int* idx, int nb, const __bf16* w1, const float* b1, __bf16* a1,
                      hipStream_t st);
void launch_conv_fwd(int l, const __bf16* ain, int nb, const __bf16* wf, const float* bias, __bf16* aout,
                     hipStream_t st);
void launch_head(const __bf16* a6, int nb, const __bf16* hw, const float* hb, const float* target, const int* idx,
                 const Norm& nm, float* y, float* loss_part, float* head_part, __bf16* g6, hipStream_t st);
void launch_conv_bwd_data(int l, const __bf16* gout, int nb, const __bf16* wb, const __bf16* ain, __bf16* gin,
                          hipStream_t st);
// returns the number of partial rows written to part
int launch_conv_bwd_weight(int l, const __bf16* gout, const __bf16* ain, int nb, float* part, hipStream_t st);
int launch_conv1_bwd_weight(const __bf16* g1, const float* x, const int* idx, int nb, float* part, hipStream_t st);
int max_weight_partials();
void launch_reduce(const float* part, int rows, int cols, ReduceMode mode, int off, float scale, float* out,
                   hipStream_t st);
void launch_adam_pack(float* theta, const float* grad, float* m, float* v, bool update, float lr, float b1, float b2,
                      float eps, float c1, float c2, __bf16* w1b, __bf16* wf, __bf16* wb, __bf16* hwb,
                      hipStream_t st);

// ---- features and probe ----
void launch_features(const float* ints, int n_pat, int n, int side, float* out, hipStream_t st);
void launch_render_probe(int n, int k, float radius, float defocus, float total, float2* out, hipStream_t st);

// ---- forward-model generator (far field, 64 x 64 frames) ----
constexpr int kFmN = 64;
constexpr int kFmMaxSide = 160;
struct FmRanges {
  float sigma_lo, sigma_hi, bw_lo, bw_hi, r_lo, r_hi, c_lo, c_hi;
};
void launch_fm_setup(uint64_t key, long first, int count, const FmRanges& rg, int side, int n_scan, int step,
                     int jitter, float* sp, int* pos, hipStream_t st);
void launch_fm_object(uint64_t key, long first, int count, int side, float2* obj, hipStream_t st);
void launch_fm_patterns(const float2* obj, int side, const float* sp, const int* pos, int n_pos, int count, int n_wl,
                        float* pat, float* tot, hipStream_t st);
void launch_fm_features(const float* pat, const float* tot, const float* sp, uint64_t key, long first, int count,
                        int n_pos, float counts, float* feat, float* targets, hipStream_t st);

}  // namespace ws
