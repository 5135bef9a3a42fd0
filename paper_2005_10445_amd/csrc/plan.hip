// C ABI of the acquisition library: plan lifecycle and the per-block search.
//
// A plan owns everything that does not change from block to block (Section
// 4.2: allocate once, keep the transformed replicas and transform tables on the
// GPU for the plan's lifetime): the replica spectra, the rectangular-chip
// spectrum, the unit-root tables, the per-bin rotations, the segment spectra
// workspace and the small result buffers.  acq_detect then only launches
// kernels on the plan's stream and copies the detections back.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "acq.h"
#include "host_logic.h"
#include "kernels.h"

using acq::Geometry;

struct acq_plan_s {
    acq_config cfg{};
    Geometry g;
    hipStream_t stream = nullptr;
    int device = 0;

    float2* d_X = nullptr;              // [S][M] FP32 segment spectra
    void* d_Xh = nullptr;               // [S][M] 16-bit segment spectra (FP16/BF16 plans)
    void* d_bank = nullptr;             // [T][Msub] in the plan's storage format
    int bank_exp = 0;                   // power-of-two prescale of the stored bank
    float2* d_rect = nullptr;           // [M]
    float2* d_rootsM = nullptr;         // [M]
    float2* d_rootsSub = nullptr;       // [Msub]
    float2* d_b1tab = nullptr;          // 2^14-point engine table (or a 1-entry stub)
    int8_t* d_chips = nullptr;          // [T][C]
    int32_t* d_rot = nullptr;           // [K]
    int64_t* d_rot_signed = nullptr;    // [K]
    double* d_freqs = nullptr;          // [K]
    unsigned long long* d_keys = nullptr;   // [T]
    double* d_parts = nullptr;          // [kPowerParts]
    acq_detection* d_dets = nullptr;    // [T]
    acq_detection* d_out = nullptr;     // [T]
    int32_t* d_found = nullptr;         // [T]
    int32_t* d_count = nullptr;         // [1]
    acq_detection* h_out = nullptr;     // pinned [T]
    int32_t* h_count = nullptr;         // pinned [1]

    bool profiling = false;
    hipEvent_t ev[ACQ_NUM_KERNELS][2] = {};
    bool ev_used[ACQ_NUM_KERNELS] = {};
};

namespace {

std::string hip_msg(const char* what, hipError_t e) {
    return std::string(what) + ": " + hipGetErrorString(e);
}

#define ACQ_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            return acq::fail(e_ == hipErrorOutOfMemory ? ACQ_ERR_OOM : ACQ_ERR_DEVICE, \
                             hip_msg(#call, e_));                                \
        }                                                                        \
    } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
}

void free_plan(acq_plan_s* p) {
    if (!p) return;
    void* dev[] = {p->d_X, p->d_Xh, p->d_bank, p->d_rect, p->d_rootsM, p->d_rootsSub, p->d_b1tab, p->d_chips,
                   p->d_rot, p->d_rot_signed, p->d_freqs, p->d_keys, p->d_parts, p->d_dets,
                   p->d_out, p->d_found, p->d_count};
    for (void* d : dev)
        if (d) (void)hipFree(d);
    if (p->h_out) (void)hipHostFree(p->h_out);
    if (p->h_count) (void)hipHostFree(p->h_count);
    for (auto& pair : p->ev)
        for (hipEvent_t e : pair)
            if (e) (void)hipEventDestroy(e);
    delete p;
}

int build_plan(acq_plan_s* p) {
    const Geometry& g = p->g;
    const acq_config& c = p->cfg;
    const size_t T = size_t(c.num_tags), C = size_t(c.num_chips), K = size_t(c.num_bins);
    const size_t S = size_t(g.max_segments > 0 ? g.max_segments : 1);
    const bool half = c.precision != ACQ_FP32;
    ACQ_HIP(dalloc(&p->d_X, S * size_t(g.M)));
    if (half) ACQ_HIP(hipMalloc(&p->d_Xh, S * size_t(g.M) * 4));
    ACQ_HIP(hipMalloc(&p->d_bank, T * size_t(g.Msub) * (half ? 4 : 8)));
    // 16-bit banks are stored with rms magnitude near 1: 2^round(log2(M / sqrt(C)))
    p->bank_exp = half ? int(std::lrint(std::log2(double(g.M) / std::sqrt(double(C))))) : 0;
    ACQ_HIP(dalloc(&p->d_rect, size_t(g.M)));
    ACQ_HIP(dalloc(&p->d_rootsM, size_t(g.M)));
    ACQ_HIP(dalloc(&p->d_rootsSub, size_t(g.Msub)));
    const std::vector<float> b1 = g.log2_sub == 14 ? acq::fft14_b1_table() : std::vector<float>(2, 0.f);
    ACQ_HIP(dalloc(&p->d_b1tab, b1.size() / 2));
    ACQ_HIP(dalloc(&p->d_chips, T * C));
    ACQ_HIP(dalloc(&p->d_rot, K));
    ACQ_HIP(dalloc(&p->d_rot_signed, K));
    ACQ_HIP(dalloc(&p->d_freqs, K));
    ACQ_HIP(dalloc(&p->d_keys, T));
    ACQ_HIP(dalloc(&p->d_parts, size_t(acq::kPowerParts)));
    ACQ_HIP(dalloc(&p->d_dets, T));
    ACQ_HIP(dalloc(&p->d_out, T));
    ACQ_HIP(dalloc(&p->d_found, T));
    ACQ_HIP(dalloc(&p->d_count, 1));
    ACQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_out), sizeof(acq_detection) * T));
    ACQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_count), sizeof(int32_t)));

    const std::vector<float> rootsM = acq::unit_roots(g.M);
    const std::vector<float> rootsSub = acq::unit_roots(g.Msub);
    const std::vector<float> rect = acq::rect_spectrum_conj(g.M, c.samples_per_chip);
    hipStream_t st = p->stream;
    ACQ_HIP(hipMemcpyAsync(p->d_rootsM, rootsM.data(), rootsM.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rootsSub, rootsSub.data(), rootsSub.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rect, rect.data(), rect.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_b1tab, b1.data(), b1.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_chips, c.chips, T * C, hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rot, g.rot.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rot_signed, g.rot_signed.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_freqs, g.freqs_hz.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    ACQ_HIP(acq::launch_bank(p->d_chips, int(T), int(C), p->d_bank, p->d_rootsSub, p->d_b1tab, int(g.Msub),
                             int(g.M), p->bank_exp, g.log2_sub, c.precision, st));
    ACQ_HIP(hipStreamSynchronize(st));
    return ACQ_OK;
}

// Event pair around one kernel launch when profiling is on.
struct KernelTimer {
    acq_plan_s* p;
    int id;
    KernelTimer(acq_plan_s* plan, int kernel) : p(plan), id(kernel) {
        if (p->profiling) {
            (void)hipEventRecord(p->ev[id][0], p->stream);
            p->ev_used[id] = true;
        }
    }
    ~KernelTimer() {
        if (p->profiling) (void)hipEventRecord(p->ev[id][1], p->stream);
    }
};

void reset_timers(acq_plan_s* p) {
    for (bool& u : p->ev_used) u = false;
}

// Kernels shared by acq_detect and acq_correlate_power: block power, segment
// spectra, correlation (argmax keys, optional power dump).
int run_search(acq_plan_s* p, const float2* x, int64_t n, float* dump) {
    const Geometry& g = p->g;
    const acq_config& c = p->cfg;
    hipStream_t st = p->stream;
    const int64_t lags = n - g.L + 1;
    const int S = int((lags + g.V - 1) / g.V);
    reset_timers(p);
    {
        KernelTimer kt(p, ACQ_KERNEL_BLOCK_POWER);
        ACQ_HIP(acq::launch_block_power(x, n, p->d_parts, st));
    }
    ACQ_HIP(acq::launch_fill_u64(p->d_keys, c.num_tags, st));

    acq::FwdArgs fa{};
    fa.x = x;
    fa.X = p->d_X;
    fa.Xh = p->d_Xh;
    fa.parts = p->d_parts;
    fa.rootsM = p->d_rootsM;
    fa.rootsSub = p->d_rootsSub;
    fa.b1tab = p->d_b1tab;
    fa.n = n;
    fa.V = g.V;
    fa.S = S;
    fa.spc = c.samples_per_chip;
    fa.M = int(g.M);
    fa.Msub = int(g.Msub);
    {
        KernelTimer kt(p, ACQ_KERNEL_FORWARD);
        ACQ_HIP(acq::launch_forward(fa, g.log2_sub, c.precision, st));
    }

    acq::CorrArgs ca{};
    ca.X = c.precision == ACQ_FP32 ? static_cast<const void*>(p->d_X) : p->d_Xh;
    ca.bank = p->d_bank;
    ca.parts = p->d_parts;
    ca.bank_exp = p->bank_exp;
    ca.rect = p->d_rect;
    ca.rootsM = p->d_rootsM;
    ca.rootsSub = p->d_rootsSub;
    ca.b1tab = p->d_b1tab;
    ca.rot = p->d_rot;
    ca.keys = p->d_keys;
    ca.dump = dump;
    ca.n = n;
    ca.lags = lags;
    ca.V = g.V;
    ca.S = S;
    ca.K = c.num_bins;
    ca.spc = c.samples_per_chip;
    ca.M = int(g.M);
    ca.Msub = int(g.Msub);
    ca.T = c.num_tags;
    ca.tile = g.tag_tile;
    ca.ntiles = (c.num_tags + g.tag_tile - 1) / g.tag_tile;
    const int64_t nwork = int64_t(ca.ntiles) * S * c.num_bins * c.samples_per_chip;
    if (nwork >= (int64_t(1) << 31) - 8) return acq::fail(ACQ_ERR_UNSUPPORTED, "too many work items");
    ca.nwork = int(nwork);
    {
        KernelTimer kt(p, ACQ_KERNEL_CORRELATE);
        ACQ_HIP(acq::launch_correlate(ca, g.log2_sub, c.precision, st));
    }
    return ACQ_OK;
}

int check_block(acq_plan_s* p, const void* block, int64_t n) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (n < 0) return acq::fail(ACQ_ERR_INVALID_ARG, "negative block length");
    if (n > p->cfg.max_block_len) return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "block longer than max_block_len");
    if (n > 0 && !block) return acq::fail(ACQ_ERR_INVALID_ARG, "null block");
    if (reinterpret_cast<uintptr_t>(block) % 8 != 0)
        return acq::fail(ACQ_ERR_INVALID_ARG, "block must be 8-byte aligned");
    return ACQ_OK;
}

}  // namespace

extern "C" {

int acq_plan_geometry(const acq_config* cfg, acq_geometry* out) {
    if (!out) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    Geometry g;
    const int rc = acq::derive_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    out->template_len = g.L;
    out->min_fft_len = g.m_min;
    out->fft_len = g.M;
    out->sub_fft_len = g.Msub;
    out->valid_per_segment = g.V;
    out->max_segments = g.max_segments;
    out->freq_quantum_hz = g.q;
    out->bin_center_hz = double(g.centre_q) * g.q;
    out->bin_step_hz = double(g.step_q) * g.q;
    out->device_bytes = g.device_bytes;
    return ACQ_OK;
}

int acq_bin_frequencies(const acq_config* cfg, double* freqs_hz, int32_t n) {
    if (!freqs_hz) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    Geometry g;
    const int rc = acq::derive_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    if (n < cfg->num_bins) return acq::fail(ACQ_ERR_INVALID_ARG, "output shorter than num_bins");
    for (int32_t k = 0; k < cfg->num_bins; ++k) freqs_hz[k] = g.freqs_hz[size_t(k)];
    return ACQ_OK;
}

int acq_plan(const acq_config* cfg, void* stream, acq_plan_t* out) {
    if (!out) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    Geometry g;
    int rc = acq::derive_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    acq_plan_s* p = new (std::nothrow) acq_plan_s();
    if (!p) return acq::fail(ACQ_ERR_OOM, "host allocation failed");
    p->cfg = *cfg;                   // chips are read by build_plan only
    p->g = std::move(g);
    p->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return acq::fail(ACQ_ERR_DEVICE, "no HIP device");
    }
    rc = build_plan(p);
    p->cfg.chips = nullptr;          // copied to the device; the caller keeps its buffer
    if (rc != ACQ_OK) {
        free_plan(p);
        return rc;
    }
    *out = p;
    acq::clear_error();
    return ACQ_OK;
}

int acq_detect(acq_plan_t p, const void* block, int64_t n, acq_detection* out, int32_t capacity,
               int32_t* n_found) {
    int rc = check_block(p, block, n);
    if (rc != ACQ_OK) return rc;
    if (!n_found) return acq::fail(ACQ_ERR_INVALID_ARG, "null n_found");
    if (capacity < 0 || (capacity > 0 && !out)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad output buffer");
    *n_found = 0;
    const Geometry& g = p->g;
    if (n < g.L) {
        acq::clear_error();
        return ACQ_OK;
    }
    const float2* x = static_cast<const float2*>(block);
    rc = run_search(p, x, n, nullptr);
    if (rc != ACQ_OK) return rc;
    const acq_config& c = p->cfg;
    acq::RefineArgs ra{};
    ra.x = x;
    ra.chips = p->d_chips;
    ra.rot_signed = p->d_rot_signed;
    ra.freqs = p->d_freqs;
    ra.keys = p->d_keys;
    ra.parts = p->d_parts;
    ra.dets = p->d_dets;
    ra.found = p->d_found;
    ra.n = n;
    ra.L = g.L;
    ra.lags = n - g.L + 1;
    ra.theta = c.threshold > 0.0 ? c.threshold : acq::default_threshold(c.num_tags, c.num_bins, n, g.L);
    ra.T = c.num_tags;
    ra.C = c.num_chips;
    ra.K = c.num_bins;
    ra.spc = c.samples_per_chip;
    ra.M = int(g.M);
    ra.radius = c.refine_radius > 0 ? c.refine_radius : 1;
    hipStream_t st = p->stream;
    {
        KernelTimer kt(p, ACQ_KERNEL_REFINE);
        ACQ_HIP(acq::launch_refine(ra, st));
    }
    {
        KernelTimer kt(p, ACQ_KERNEL_COMPACT);
        ACQ_HIP(acq::launch_compact(p->d_dets, p->d_found, c.num_tags, p->d_out, p->d_count, st));
    }
    ACQ_HIP(hipMemcpyAsync(p->h_count, p->d_count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ACQ_HIP(hipMemcpyAsync(p->h_out, p->d_out, sizeof(acq_detection) * size_t(c.num_tags),
                           hipMemcpyDeviceToHost, st));
    ACQ_HIP(hipStreamSynchronize(st));
    const int32_t found = *p->h_count;
    *n_found = found;
    const int32_t ncopy = found < capacity ? found : capacity;
    if (ncopy > 0) std::memcpy(out, p->h_out, sizeof(acq_detection) * size_t(ncopy));
    if (found > capacity) return acq::fail(ACQ_ERR_TRUNCATED, "more detections than capacity");
    acq::clear_error();
    return ACQ_OK;
}

int acq_correlate_power(acq_plan_t p, const void* block, int64_t n, float* power) {
    int rc = check_block(p, block, n);
    if (rc != ACQ_OK) return rc;
    if (n < p->g.L) {
        acq::clear_error();
        return ACQ_OK;
    }
    if (!power) return acq::fail(ACQ_ERR_INVALID_ARG, "null power output");
    rc = run_search(p, static_cast<const float2*>(block), n, power);
    if (rc != ACQ_OK) return rc;
    ACQ_HIP(hipStreamSynchronize(p->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_set_profiling(acq_plan_t p, int on) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (on && !p->ev[0][0]) {
        for (auto& pair : p->ev)
            for (hipEvent_t& e : pair) ACQ_HIP(hipEventCreate(&e));
    }
    p->profiling = on != 0;
    reset_timers(p);
    return ACQ_OK;
}

int acq_last_kernel_times(acq_plan_t p, double* ms, int32_t n, int32_t* count) {
    if (!p || !count || (n > 0 && !ms)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad arguments");
    *count = ACQ_NUM_KERNELS;
    ACQ_HIP(hipStreamSynchronize(p->stream));
    for (int i = 0; i < n && i < ACQ_NUM_KERNELS; ++i) {
        float t = 0.f;
        if (p->profiling && p->ev_used[i]) ACQ_HIP(hipEventElapsedTime(&t, p->ev[i][0], p->ev[i][1]));
        ms[i] = double(t);
    }
    return ACQ_OK;
}

int acq_release(acq_plan_t p) {
    if (!p) return ACQ_OK;
    (void)hipStreamSynchronize(p->stream);
    free_plan(p);
    return ACQ_OK;
}

const char* acq_strerror(int status) {
    switch (status) {
        case ACQ_OK: return "ok";
        case ACQ_ERR_INVALID_ARG: return "invalid argument";
        case ACQ_ERR_OOM: return "out of memory";
        case ACQ_ERR_DEVICE: return "device error";
        case ACQ_ERR_TRUNCATED: return "output truncated";
        case ACQ_ERR_BLOCK_TOO_LONG: return "block too long";
        case ACQ_ERR_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* acq_last_error(void) { return acq::last_error(); }

}  // extern "C"
