// Proposal stage: STFT power map, 1-D CNN (inference and training), window
// scores and the proposal-to-segment mapping.  Launch interface used by
// cnn.hip.
//
// Rows are frames of a batch of equal-length blocks: row r is frame r mod F of
// block r / F.  Activations are row-major [rows][channels]; convolutions pad
// with zeros at each block's edges.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace acq {
namespace learned {

constexpr int kWin = 256;          // STFT length
constexpr int kHop = 128;          // STFT hop
constexpr int kSpan = 128;         // window-score length (frames)
constexpr int kCh = 64;            // channels of every conv layer
constexpr int kTaps = 5;
constexpr int kLayers = 4;
constexpr int kMaxTx = 32;         // transmissions per synthetic block
constexpr int kDilation[kLayers] = {1, 2, 4, 8};

inline int64_t num_frames(int64_t n) { return n < kWin ? 0 : (n - kWin) / kHop + 1; }

// FP32 parameter vector: per layer l, W_l[5][cin_l][64] then b_l[64]; then the
// head wh[64] and bh.  The bf16 copies hold, per layer, W_l in that layout
// ([tap][in][out], the B operand of the input-gradient product) and its
// transpose [tap][out][in] (the B operand of the forward product).
struct NetLayout {
    int cin[kLayers];
    int64_t w_off[kLayers], b_off[kLayers], wh_off, bh_off, total;
    int64_t bf_off[kLayers], bf_total;
};
NetLayout net_layout(int cin0);

// One transmission of a synthetic training block (sample-level model of the
// tag-bank workload: BPSK chips held spc samples, on-grid carrier offset,
// amplitude from the per-sample SNR, integer delay).
struct SynthTx {
    int64_t delay;              // first sample
    double cycles_per_sample;   // f / Fs
    float amp;                  // sqrt(SNR), noise power 1
    float phase0;               // carrier phase at sample 0, cycles
    uint32_t code;              // chip stream id
    uint32_t pad;
};

// Sample source of the STFT: a device block, or synthetic blocks generated on
// the fly (Philox4x32-10 noise and chips, Box-Muller normals).
struct BlockSource {
    const float2* x;            // device samples of block 0 (x[b * stride + n]) or nullptr
    int64_t stride;
    const SynthTx* tx;          // [block][kMaxTx] when x == nullptr
    const int32_t* ntx;         // [block]
    uint32_t seed_lo, seed_hi;  // generator key
    int64_t block0;             // stream id of block 0
    int32_t chip_len;           // samples per transmission L
    int32_t spc;
};

// Median state of one block for the radix selection over FP32 bit patterns.
struct MedianState {
    uint32_t prefix;
    uint32_t rank;
};

hipError_t launch_stft(const BlockSource& src, int nblocks, int64_t F, const float* hann, const float2* tw,
                       float* P, hipStream_t st);
hipError_t launch_median(const float* P, int nblocks, int64_t per_block, uint32_t* hist, MedianState* state,
                         float* med, hipStream_t st);
hipError_t launch_map(const float* P, int nblocks, int64_t F, const float* med, void* map, bool bf16,
                      hipStream_t st);
// Samples of synthetic block 0 of `src` (src.x == nullptr) into out[n].
hipError_t launch_synth(const BlockSource& src, int64_t n, float2* out, hipStream_t st);
hipError_t launch_labels(const SynthTx* tx, const int32_t* ntx, int nblocks, int64_t F, int L, float* labels,
                         hipStream_t st);

// Forward of one conv layer: out = relu(conv(in) + b).
hipError_t launch_conv_forward(const void* in, int cin, const void* wt, const float* bias, void* out,
                               int64_t rows, int64_t F, int d, bool bf16, hipStream_t st);
// Input gradient of layer l (cin = 64): dprev[r][c] = sum_i sum_o W[i][c][o] dA[r - d(i-2)][o],
// dA = dH * (H > 0).
hipError_t launch_conv_dinput(const float* dH, const void* H, const void* w, float* dprev, int64_t rows,
                              int64_t F, int d, bool bf16, hipStream_t st);
// Weight and bias gradients (accumulated): dW[i][c][o] += sum_r in[r + d(i-2)][c] dA[r][o],
// db[o] += sum_r dA[r][o].  The bf16 form sums row chunks into `part` (FP32, at least
// dweight_part_elems(cin) values; unused by the FP32 form) and adds the chunk sums
// to dW and db in a fixed order.
int64_t dweight_part_elems(int cin);
hipError_t launch_conv_dweight(const void* in, int cin, const float* dH, const void* H, float* dW, float* db,
                               float* part, int64_t part_elems, int64_t rows, int64_t F, int d, bool bf16,
                               hipStream_t st);
// Head logits y[r] = bh + h4[r] . wh; with labels also the loss terms and
// dH4 = dy wh^T, dwh += h4^T dy, dbh += sum dy, loss_sum += sum of losses.
hipError_t launch_head(const void* h4, const float* theta, int64_t wh_off, float* y, const float* labels,
                       float pos_weight, float inv_rows, float* dH4, float* grad, float* loss_sum, int64_t rows,
                       bool bf16, hipStream_t st);
hipError_t launch_adam(float* theta, float* grad, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, const NetLayout& lay, uint16_t* w_bf, uint16_t* wt_bf, hipStream_t st);
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t st);

// Window scores c[f] = sum_{i=-63}^{64} y[f+i] of one block.
hipError_t launch_window(const float* y, int64_t F, float* c, hipStream_t st);
// Frames at or above kappa, their lag ranges and the segment list of one block.
// out_info = {proposed frames, segments}.
hipError_t launch_propose(const float* c, int64_t F, float kappa, int64_t n, int64_t L, int64_t V,
                          int32_t max_segments, int32_t* segs, int32_t* out_info, hipStream_t st);

}  // namespace learned
}  // namespace acq
