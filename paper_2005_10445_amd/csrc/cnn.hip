// C ABI of the proposal network: lifecycle, parameters, forward, gradients,
// Adam, power maps, synthetic training batches; and the proposal step used by
// acq_detect_learned (cnn_internal.h).
//
// A network owns its FP32 master parameters, Adam moments and gradient, the
// bf16 weight copies in both operand layouts, activation buffers for
// max_rows frames, the STFT/median scratch and the transform tables.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "acq.h"
#include "cnn_internal.h"
#include "host_logic.h"
#include "learned.h"

using namespace acq::learned;

static_assert(sizeof(acq_synth_tx) == sizeof(SynthTx), "acq_synth_tx and SynthTx must share a layout");
static_assert(ACQ_SYNTH_MAX_TX == kMaxTx, "transmission capacity");

namespace {

constexpr int kMaxBatch = 256;   // blocks per training call

std::string hip_msg(const char* what, hipError_t e) { return std::string(what) + ": " + hipGetErrorString(e); }

#define CNN_HIP(call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return acq::fail(e_ == hipErrorOutOfMemory ? ACQ_ERR_OOM : ACQ_ERR_DEVICE, hip_msg(#call, e_)); \
    } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
}

}  // namespace

struct acq_cnn_s {
    acq_cnn_config cfg{};
    hipStream_t stream = nullptr;
    bool bf = true;
    NetLayout lay{};
    int step = 0;

    float* theta = nullptr;     // [np] FP32 master parameters
    float* grad = nullptr;      // [np]
    float* m = nullptr;         // [np]
    float* v = nullptr;         // [np]
    uint16_t* w_bf = nullptr;   // [bf_total] per layer [tap][in][out]
    uint16_t* wt_bf = nullptr;  // [bf_total] per layer [tap][out][in]

    void* act[kLayers + 1] = {};    // act[0]: map [rows][cin]; act[l]: layer l output [rows][64]
    float* dH[2] = {};              // [rows][64] FP32 gradients (ping-pong)
    float* dw_part = nullptr;       // [dw_part_elems] weight-gradient chunk sums
    int64_t dw_part_elems = 0;
    float* y = nullptr;             // [rows] logits
    float* labels = nullptr;        // [rows]
    float* P = nullptr;             // [rows][256] STFT powers
    uint32_t* hist = nullptr;       // [kMaxBatch][2048]
    MedianState* mstate = nullptr;  // [kMaxBatch]
    float* med = nullptr;           // [kMaxBatch]
    float* hann = nullptr;          // [256]
    float2* tw = nullptr;           // [256] exp(-j 2 pi m / 256)
    float* loss = nullptr;          // [1]
    SynthTx* d_tx = nullptr;        // [kMaxBatch][kMaxTx]
    int32_t* d_ntx = nullptr;       // [kMaxBatch]
    float* wscore = nullptr;        // [max frames of one block]
    int32_t* d_info = nullptr;      // [2]

    SynthTx* h_tx = nullptr;        // pinned staging
    int32_t* h_ntx = nullptr;
    int32_t* h_info = nullptr;      // pinned [2]
    float* h_scalar = nullptr;      // pinned [2]: loss, median

    bool floor_init = false;
    double floor = 0.0;
};

namespace {

void free_cnn(acq_cnn_s* c) {
    if (!c) return;
    void* dev[] = {c->theta, c->grad, c->m, c->v, c->w_bf, c->wt_bf, c->act[0], c->act[1], c->act[2], c->act[3],
                   c->act[4], c->dH[0], c->dH[1], c->dw_part, c->y, c->labels, c->P, c->hist, c->mstate, c->med,
                   c->hann, c->tw, c->loss, c->d_tx, c->d_ntx, c->wscore, c->d_info};
    for (void* d : dev)
        if (d) (void)hipFree(d);
    void* host[] = {c->h_tx, c->h_ntx, c->h_info, c->h_scalar};
    for (void* h : host)
        if (h) (void)hipHostFree(h);
    delete c;
}

int build_cnn(acq_cnn_s* c) {
    const size_t rows = size_t(c->cfg.max_rows), np = size_t(c->lay.total);
    const size_t es = c->bf ? 2 : 4;
    const size_t fmax = size_t(std::max<int64_t>(num_frames(c->cfg.max_block_len), 1));
    CNN_HIP(dalloc(&c->theta, np));
    CNN_HIP(dalloc(&c->grad, np));
    CNN_HIP(dalloc(&c->m, np));
    CNN_HIP(dalloc(&c->v, np));
    if (c->bf) {
        CNN_HIP(dalloc(&c->w_bf, size_t(c->lay.bf_total)));
        CNN_HIP(dalloc(&c->wt_bf, size_t(c->lay.bf_total)));
    }
    CNN_HIP(hipMalloc(&c->act[0], rows * size_t(c->cfg.in_channels) * es));
    for (int l = 1; l <= kLayers; ++l) CNN_HIP(hipMalloc(&c->act[l], rows * kCh * es));
    CNN_HIP(dalloc(&c->dH[0], rows * kCh));
    CNN_HIP(dalloc(&c->dH[1], rows * kCh));
    if (c->bf) {
        c->dw_part_elems = std::max(dweight_part_elems(c->cfg.in_channels), dweight_part_elems(kCh));
        CNN_HIP(dalloc(&c->dw_part, size_t(c->dw_part_elems)));
    }
    CNN_HIP(dalloc(&c->y, rows));
    CNN_HIP(dalloc(&c->labels, rows));
    CNN_HIP(dalloc(&c->P, rows * kWin));
    CNN_HIP(dalloc(&c->hist, size_t(kMaxBatch) * 2048));
    CNN_HIP(dalloc(&c->mstate, size_t(kMaxBatch)));
    CNN_HIP(dalloc(&c->med, size_t(kMaxBatch)));
    CNN_HIP(dalloc(&c->hann, size_t(kWin)));
    CNN_HIP(dalloc(&c->tw, size_t(kWin)));
    CNN_HIP(dalloc(&c->loss, 1));
    CNN_HIP(dalloc(&c->d_tx, size_t(kMaxBatch) * kMaxTx));
    CNN_HIP(dalloc(&c->d_ntx, size_t(kMaxBatch)));
    CNN_HIP(dalloc(&c->wscore, fmax));
    CNN_HIP(dalloc(&c->d_info, 2));
    CNN_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_tx), sizeof(SynthTx) * kMaxBatch * kMaxTx));
    CNN_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_ntx), sizeof(int32_t) * kMaxBatch));
    CNN_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_info), sizeof(int32_t) * 2));
    CNN_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_scalar), sizeof(float) * 2));

    // window and twiddles from FP64
    std::vector<float> hann(kWin);
    std::vector<float> tw(2 * kWin);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < kWin; ++i) {
        hann[size_t(i)] = float(0.5 * (1.0 - std::cos(2.0 * pi * i / kWin)));
        tw[2 * size_t(i)] = float(std::cos(2.0 * pi * i / kWin));
        tw[2 * size_t(i) + 1] = float(-std::sin(2.0 * pi * i / kWin));
    }
    hipStream_t st = c->stream;
    CNN_HIP(hipMemcpyAsync(c->hann, hann.data(), sizeof(float) * kWin, hipMemcpyHostToDevice, st));
    CNN_HIP(hipMemcpyAsync(c->tw, tw.data(), sizeof(float) * 2 * kWin, hipMemcpyHostToDevice, st));
    CNN_HIP(launch_fill_f32(c->theta, int64_t(np), st));
    CNN_HIP(launch_fill_f32(c->grad, int64_t(np), st));
    CNN_HIP(launch_fill_f32(c->m, int64_t(np), st));
    CNN_HIP(launch_fill_f32(c->v, int64_t(np), st));
    if (c->bf) CNN_HIP(launch_adam(c->theta, c->grad, c->m, c->v, int64_t(np), 0.f, 0.f, 0.f, 0.f, 0, c->lay,
                                   c->w_bf, c->wt_bf, st));
    CNN_HIP(hipStreamSynchronize(st));
    return ACQ_OK;
}

int check_rows(const acq_cnn_s* c, int32_t nblocks, int64_t frames) {
    if (nblocks < 1 || frames < 1) return acq::fail(ACQ_ERR_INVALID_ARG, "need at least one block and one frame");
    if (int64_t(nblocks) * frames > c->cfg.max_rows) return acq::fail(ACQ_ERR_INVALID_ARG, "more rows than max_rows");
    return ACQ_OK;
}

// layer-0 input `in`; logits to c->y
int run_forward(acq_cnn_s* c, const void* in, int32_t nblocks, int64_t F, hipStream_t st) {
    const int64_t rows = int64_t(nblocks) * F;
    const void* x = in;
    for (int l = 0; l < kLayers; ++l) {
        const void* w = c->bf ? static_cast<const void*>(c->wt_bf + c->lay.bf_off[l])
                              : static_cast<const void*>(c->theta + c->lay.w_off[l]);
        CNN_HIP(launch_conv_forward(x, c->lay.cin[l], w, c->theta + c->lay.b_off[l], c->act[l + 1], rows, F,
                                    kDilation[l], c->bf, st));
        x = c->act[l + 1];
    }
    CNN_HIP(launch_head(c->act[kLayers], c->theta, c->lay.wh_off, c->y, nullptr, 0.f, 0.f, nullptr, nullptr, nullptr,
                        rows, c->bf, st));
    return ACQ_OK;
}

// loss terms into c->loss and gradients added to c->grad (after run_forward on `in`)
int run_backward(acq_cnn_s* c, const void* in, int32_t nblocks, int64_t F, const float* labels, float pw,
                 hipStream_t st) {
    const int64_t rows = int64_t(nblocks) * F;
    CNN_HIP(launch_head(c->act[kLayers], c->theta, c->lay.wh_off, c->y, labels, pw, float(1.0 / double(rows)),
                        c->dH[0], c->grad, c->loss, rows, c->bf, st));
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const void* x = l == 0 ? in : c->act[l];
        CNN_HIP(launch_conv_dweight(x, c->lay.cin[l], c->dH[cur], c->act[l + 1], c->grad + c->lay.w_off[l],
                                    c->grad + c->lay.b_off[l], c->dw_part, c->dw_part_elems, rows, F,
                                    kDilation[l], c->bf, st));
        if (l > 0) {
            const void* w = c->bf ? static_cast<const void*>(c->w_bf + c->lay.bf_off[l])
                                  : static_cast<const void*>(c->theta + c->lay.w_off[l]);
            CNN_HIP(launch_conv_dinput(c->dH[cur], c->act[l + 1], w, c->dH[1 - cur], rows, F, kDilation[l], c->bf,
                                       st));
            cur = 1 - cur;
        }
    }
    return ACQ_OK;
}

int run_map(acq_cnn_s* c, const BlockSource& src, int32_t nblocks, int64_t F, void* map, hipStream_t st) {
    CNN_HIP(launch_stft(src, nblocks, F, c->hann, c->tw, c->P, st));
    CNN_HIP(launch_median(c->P, nblocks, F * kWin, c->hist, c->mstate, c->med, st));
    CNN_HIP(launch_map(c->P, nblocks, F, c->med, map, c->bf, st));
    return ACQ_OK;
}

int synth_source(acq_cnn_s* c, const acq_synth_batch* b, BlockSource* src) {
    if (!b || !b->tx || !b->ntx) return acq::fail(ACQ_ERR_INVALID_ARG, "null batch");
    if (b->nblocks < 1 || b->nblocks > kMaxBatch) return acq::fail(ACQ_ERR_INVALID_ARG, "nblocks outside [1, 256]");
    if (b->num_chips < 1 || b->samples_per_chip < 1 || b->block_len < kWin)
        return acq::fail(ACQ_ERR_INVALID_ARG, "bad synthetic block shape");
    for (int32_t i = 0; i < b->nblocks; ++i)
        if (b->ntx[i] < 0 || b->ntx[i] > kMaxTx) return acq::fail(ACQ_ERR_INVALID_ARG, "ntx outside [0, 32]");
    std::memcpy(c->h_tx, b->tx, sizeof(SynthTx) * size_t(b->nblocks) * kMaxTx);
    std::memcpy(c->h_ntx, b->ntx, sizeof(int32_t) * size_t(b->nblocks));
    CNN_HIP(hipMemcpyAsync(c->d_tx, c->h_tx, sizeof(SynthTx) * size_t(b->nblocks) * kMaxTx, hipMemcpyHostToDevice,
                           c->stream));
    CNN_HIP(hipMemcpyAsync(c->d_ntx, c->h_ntx, sizeof(int32_t) * size_t(b->nblocks), hipMemcpyHostToDevice,
                           c->stream));
    BlockSource s{};
    s.x = nullptr;
    s.tx = c->d_tx;
    s.ntx = c->d_ntx;
    s.seed_lo = uint32_t(b->seed);
    s.seed_hi = uint32_t(b->seed >> 32);
    s.block0 = b->first_block;
    s.chip_len = b->num_chips * b->samples_per_chip;
    s.spc = b->samples_per_chip;
    *src = s;
    return ACQ_OK;
}

}  // namespace

namespace acq {

int cnn_propose(acq_cnn_t c, const void* block, int64_t n, int64_t L, int64_t V, int32_t max_segments, float kappa,
                int32_t* d_segs, hipStream_t st, ProposalResult* out) {
    const int64_t F = num_frames(n);
    if (F < 1) return acq::fail(ACQ_ERR_INVALID_ARG, "block shorter than one frame");
    if (n > c->cfg.max_block_len || F > c->cfg.max_rows)
        return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "block longer than the network's max_block_len");
    BlockSource src{};
    src.x = static_cast<const float2*>(block);
    src.stride = n;
    int rc = run_map(c, src, 1, F, c->act[0], st);
    if (rc != ACQ_OK) return rc;
    rc = run_forward(c, c->act[0], 1, F, st);
    if (rc != ACQ_OK) return rc;
    CNN_HIP(launch_window(c->y, F, c->wscore, st));
    CNN_HIP(launch_propose(c->wscore, F, kappa, n, L, V, max_segments, d_segs, c->d_info, st));
    CNN_HIP(hipMemcpyAsync(c->h_info, c->d_info, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, st));
    CNN_HIP(hipMemcpyAsync(c->h_scalar + 1, c->med, sizeof(float), hipMemcpyDeviceToHost, st));
    CNN_HIP(hipStreamSynchronize(st));
    out->proposals = c->h_info[0];
    out->segments = c->h_info[1];
    out->median = c->h_scalar[1];
    return ACQ_OK;
}

bool cnn_floor(acq_cnn_t c, double* floor) {
    *floor = c->floor;
    return c->floor_init;
}

void cnn_update_floor(acq_cnn_t c, double median) {
    c->floor = c->floor_init ? 0.9 * c->floor + 0.1 * median : median;
    c->floor_init = true;
}

}  // namespace acq

extern "C" {

int64_t acq_cnn_num_params(int32_t in_channels) {
    if (in_channels < 1) return 0;
    return net_layout(in_channels).total;
}

int acq_cnn_create(const acq_cnn_config* cfg, void* stream, acq_cnn_t* out) {
    if (!cfg || !out) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (cfg->precision != ACQ_BF16 && cfg->precision != ACQ_FP32)
        return acq::fail(ACQ_ERR_UNSUPPORTED, "network precision must be ACQ_BF16 or ACQ_FP32");
    if (cfg->in_channels < 1 || (cfg->precision == ACQ_BF16 && cfg->in_channels % 64))
        return acq::fail(ACQ_ERR_INVALID_ARG, "in_channels must be positive (a multiple of 64 for ACQ_BF16)");
    if (cfg->max_rows < 1 || cfg->max_rows > (int64_t(1) << 26))
        return acq::fail(ACQ_ERR_INVALID_ARG, "max_rows outside [1, 2^26]");
    if (cfg->max_block_len < 0 || num_frames(cfg->max_block_len) > cfg->max_rows)
        return acq::fail(ACQ_ERR_INVALID_ARG, "max_block_len needs more frames than max_rows");
    acq_cnn_s* c = new (std::nothrow) acq_cnn_s();
    if (!c) return acq::fail(ACQ_ERR_OOM, "host allocation failed");
    c->cfg = *cfg;
    c->bf = cfg->precision == ACQ_BF16;
    c->lay = net_layout(cfg->in_channels);
    c->stream = static_cast<hipStream_t>(stream);
    const int rc = build_cnn(c);
    if (rc != ACQ_OK) {
        free_cnn(c);
        return rc;
    }
    *out = c;
    acq::clear_error();
    return ACQ_OK;
}

int acq_cnn_release(acq_cnn_t c) {
    if (!c) return ACQ_OK;
    (void)hipStreamSynchronize(c->stream);
    free_cnn(c);
    return ACQ_OK;
}

int acq_cnn_set_params(acq_cnn_t c, const float* params, int64_t n) {
    if (!c || !params) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (n != c->lay.total) return acq::fail(ACQ_ERR_INVALID_ARG, "parameter count mismatch");
    hipStream_t st = c->stream;
    CNN_HIP(hipMemcpyAsync(c->theta, params, sizeof(float) * size_t(n), hipMemcpyHostToDevice, st));
    CNN_HIP(launch_fill_f32(c->grad, n, st));
    CNN_HIP(launch_fill_f32(c->m, n, st));
    CNN_HIP(launch_fill_f32(c->v, n, st));
    if (c->bf) CNN_HIP(launch_adam(c->theta, c->grad, c->m, c->v, n, 0.f, 0.f, 0.f, 0.f, 0, c->lay, c->w_bf,
                                   c->wt_bf, st));
    CNN_HIP(hipStreamSynchronize(st));
    c->step = 0;
    acq::clear_error();
    return ACQ_OK;
}

int acq_cnn_get_params(acq_cnn_t c, float* params, int64_t n) {
    if (!c || !params) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (n != c->lay.total) return acq::fail(ACQ_ERR_INVALID_ARG, "parameter count mismatch");
    CNN_HIP(hipMemcpyAsync(params, c->theta, sizeof(float) * size_t(n), hipMemcpyDeviceToHost, c->stream));
    CNN_HIP(hipStreamSynchronize(c->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_cnn_forward(acq_cnn_t c, const void* input, int32_t nblocks, int64_t frames, float* logits) {
    if (!c || !input || !logits) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    int rc = check_rows(c, nblocks, frames);
    if (rc != ACQ_OK) return rc;
    rc = run_forward(c, input, nblocks, frames, c->stream);
    if (rc != ACQ_OK) return rc;
    CNN_HIP(hipMemcpyAsync(logits, c->y, sizeof(float) * size_t(nblocks) * size_t(frames), hipMemcpyDeviceToDevice,
                           c->stream));
    CNN_HIP(hipStreamSynchronize(c->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_cnn_gradients(acq_cnn_t c, const void* input, int32_t nblocks, int64_t frames, const float* labels,
                      float pos_weight, float* grad, float* loss) {
    if (!c || !input || !labels || !loss) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    int rc = check_rows(c, nblocks, frames);
    if (rc != ACQ_OK) return rc;
    hipStream_t st = c->stream;
    CNN_HIP(launch_fill_f32(c->grad, c->lay.total, st));
    CNN_HIP(launch_fill_f32(c->loss, 1, st));
    rc = run_forward(c, input, nblocks, frames, st);
    if (rc == ACQ_OK) rc = run_backward(c, input, nblocks, frames, labels, pos_weight, st);
    if (rc != ACQ_OK) return rc;
    if (grad)
        CNN_HIP(hipMemcpyAsync(grad, c->grad, sizeof(float) * size_t(c->lay.total), hipMemcpyDeviceToDevice, st));
    CNN_HIP(hipMemcpyAsync(c->h_scalar, c->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    CNN_HIP(hipStreamSynchronize(st));
    *loss = float(double(c->h_scalar[0]) / (double(nblocks) * double(frames)));
    acq::clear_error();
    return ACQ_OK;
}

int acq_cnn_adam_step(acq_cnn_t c, float lr) {
    if (!c) return acq::fail(ACQ_ERR_INVALID_ARG, "null network");
    c->step += 1;
    CNN_HIP(launch_adam(c->theta, c->grad, c->m, c->v, c->lay.total, lr, 0.9f, 0.999f, 1e-8f, c->step, c->lay,
                        c->bf ? c->w_bf : nullptr, c->bf ? c->wt_bf : nullptr, c->stream));
    CNN_HIP(hipStreamSynchronize(c->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_power_map(acq_cnn_t c, const void* block, int64_t n, void* map, float* median) {
    if (!c || !block || !map || !median) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    const int64_t F = num_frames(n);
    if (F < 1) return acq::fail(ACQ_ERR_INVALID_ARG, "block shorter than one frame");
    if (F > c->cfg.max_rows) return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "more frames than max_rows");
    if (reinterpret_cast<uintptr_t>(block) % 8) return acq::fail(ACQ_ERR_INVALID_ARG, "block must be 8-byte aligned");
    BlockSource src{};
    src.x = static_cast<const float2*>(block);
    src.stride = n;
    const int rc = run_map(c, src, 1, F, map, c->stream);
    if (rc != ACQ_OK) return rc;
    CNN_HIP(hipMemcpyAsync(c->h_scalar + 1, c->med, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    CNN_HIP(hipStreamSynchronize(c->stream));
    *median = c->h_scalar[1];
    acq::clear_error();
    return ACQ_OK;
}

int acq_synth_block(acq_cnn_t c, const acq_synth_batch* batch, void* out) {
    if (!c || !out) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    BlockSource src{};
    int rc = synth_source(c, batch, &src);
    if (rc != ACQ_OK) return rc;
    CNN_HIP(launch_synth(src, batch->block_len, static_cast<float2*>(out), c->stream));
    CNN_HIP(hipStreamSynchronize(c->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_synth_labels(acq_cnn_t c, const acq_synth_batch* batch, float* labels) {
    if (!c || !labels) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    BlockSource src{};
    int rc = synth_source(c, batch, &src);
    if (rc != ACQ_OK) return rc;
    CNN_HIP(launch_labels(c->d_tx, c->d_ntx, batch->nblocks, num_frames(batch->block_len), src.chip_len, labels,
                          c->stream));
    CNN_HIP(hipStreamSynchronize(c->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_cnn_train_synthetic(acq_cnn_t c, const acq_synth_batch* batch, float pos_weight, float lr, float* loss) {
    if (!c || !loss) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (c->cfg.in_channels != kWin) return acq::fail(ACQ_ERR_INVALID_ARG, "power-map training needs 256 inputs");
    BlockSource src{};
    int rc = synth_source(c, batch, &src);
    if (rc != ACQ_OK) return rc;
    const int32_t nb = batch->nblocks;
    const int64_t F = num_frames(batch->block_len);
    rc = check_rows(c, nb, F);
    if (rc != ACQ_OK) return rc;
    hipStream_t st = c->stream;
    rc = run_map(c, src, nb, F, c->act[0], st);
    if (rc != ACQ_OK) return rc;
    CNN_HIP(launch_labels(c->d_tx, c->d_ntx, nb, F, src.chip_len, c->labels, st));
    CNN_HIP(launch_fill_f32(c->grad, c->lay.total, st));
    CNN_HIP(launch_fill_f32(c->loss, 1, st));
    rc = run_forward(c, c->act[0], nb, F, st);
    if (rc == ACQ_OK) rc = run_backward(c, c->act[0], nb, F, c->labels, pos_weight, st);
    if (rc != ACQ_OK) return rc;
    c->step += 1;
    CNN_HIP(launch_adam(c->theta, c->grad, c->m, c->v, c->lay.total, lr, 0.9f, 0.999f, 1e-8f, c->step, c->lay,
                        c->bf ? c->w_bf : nullptr, c->bf ? c->wt_bf : nullptr, st));
    CNN_HIP(hipMemcpyAsync(c->h_scalar, c->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    CNN_HIP(hipStreamSynchronize(st));
    *loss = float(double(c->h_scalar[0]) / (double(nb) * double(F)));
    acq::clear_error();
    return ACQ_OK;
}

}  // extern "C"
